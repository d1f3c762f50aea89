// CKKS plan shared by the per-call operations and the batch runtime.
#pragma once
#include <vector>

#include "context.h"

namespace cross {

// Device-resident constants of one BConv (source set -> target set).
struct BconvStatic {
  const BconvSrc* src = nullptr;
  const BconvDst* dst = nullptr;
  const int8_t* table = nullptr;
  int nsrc = 0, ndst = 0;
  int wide = 0;             // a prime >= 2^28: byte operands, signed digits, row corrections
};


struct CkksPlan {
  int log_n = 0, L = 0, K = 0, dnum = 0, alpha = 0, ndig = 0;
  bool wide = false;                      // a prime >= 2^28: 64-bit remainders in the VALU products
  std::vector<uint32_t> primes;
  std::vector<Plan*> plans;               // L + K
  std::vector<Plan*> plans2;              // the same primes in the two-factor form (batch runtime)
  const LimbMod* mods = nullptr;          // L + K, device
  const TailConst* tail = nullptr;        // L, device
  std::vector<BconvStatic> modup;         // per active digit: digit limbs -> all other limbs
  std::vector<std::vector<int>> targets;  // per active digit
  BconvStatic moddown;                    // P -> Q
  const uint64_t* copy_src = nullptr;     // per active digit limb list (ModUp copies)
  const uint64_t* copy_dst = nullptr;
};

// Order in which the fused ModUp NTT + inner product takes the L + K target limbs:
// the K special limbs (three transforms each, against two and a load for a Q limb)
// spread evenly among the Q limbs, so that each XCD's contiguous share of the blocks
// gets the same mix.  Q limb i sits at (2i + 1) / 2L, special limb k at (2k + 1) / 2K,
// Q limbs first on ties.
inline std::vector<int> ip_limb_order(int L, int K) {
  std::vector<int> ord;
  int i = 0, k = 0;
  while (i < L || k < K) {
    if (k >= K || (i < L && (int64_t)(2 * i + 1) * K <= (int64_t)(2 * k + 1) * L))
      ord.push_back(i++);
    else
      ord.push_back(L + k++);
  }
  return ord;
}

// Validated, cached plan for a parameter set (tables uploaded on first use).
cross_status get_ckks_plan(cross_ctx ctx, const cross_ckks_params* prm, CkksPlan** out);

// NTT-domain automorphism index table for Galois element g (cached on the device).
cross_status perm_table(cross_ctx ctx, int log_n, uint32_t g, const uint32_t** out);

}  // namespace cross
