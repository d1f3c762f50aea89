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

// Validated, cached plan for a parameter set (tables uploaded on first use).
cross_status get_ckks_plan(cross_ctx ctx, const cross_ckks_params* prm, CkksPlan** out);

// NTT-domain automorphism index table for Galois element g (cached on the device).
cross_status perm_table(cross_ctx ctx, int log_n, uint32_t g, const uint32_t** out);

}  // namespace cross
