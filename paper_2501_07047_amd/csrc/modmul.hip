// VecModMul with a pre-known operand under four modular reductions
// (arXiv 2501.07047, Sec. Evaluation "Impact of Modular Reduction Algorithm",
// Fig. diff_modred: Barrett, Montgomery, Shoup; App. "BAT for Modular
// Reduction": the lazy partial reduction as a low-precision matrix product).
//
// out[p][l][n] = a[p][l][n] * w[l][n] mod q_l: w is one pre-known vector per
// limb (a plaintext, a twiddle or key vector) shared by all npoly polynomials.
// Each method reads w in the form it needs, prepared once:
//   Barrett    : w;             product reduced by Alg. barrett (two conditional subtractions)
//   Montgomery : w 2^32 mod q;  REDC of the product (Alg. montgomery_reduction), [0, 2q) -> [0, q)
//   Shoup      : w and floor(w 2^32 / q) (planar);  a w - umulhi(a, w') q in [0, 2q) -> [0, q)
//   BAT-lazy   : w;  the product's four 7-bit chunks above bit 28 go through one
//                int8 MFMA against the chunk matrix of 2^(7 (4 + j)) mod q; the lazy
//                sum (< 2^38) is finished by the Barrett step.
// All four give the canonical residue, so results are bit-identical.
#include "kernels.h"

namespace cross {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t barrett64(uint64_t z, const ModLimb& m) {
  // z < 2^(2k), k = bitlen(q), bar_m = floor(2^(2k) / q): the quotient estimate
  // is low by at most 2
  const uint32_t zh = (uint32_t)(z >> (m.bar_k - 1));
  const uint32_t t = (uint32_t)(((uint64_t)zh * m.bar_m) >> (m.bar_k + 1));
  uint32_t r = (uint32_t)z - t * m.q;
  if (r >= m.q) r -= m.q;
  if (r >= m.q) r -= m.q;
  return r;
}

__device__ __forceinline__ uint32_t pack7(uint32_t x) {
  // four 7-bit chunks of x (< 2^28) in the four bytes of one word
  return (x & 0x7fu) | ((x << 1) & 0x7f00u) | ((x << 2) & 0x7f0000u) | ((x << 3) & 0x7f000000u);
}

template <int METHOD>
__global__ void __launch_bounds__(256)
vec_modmul_kernel(const v4u* a, const v4u* w, const v4u* ws, v4u* out, const ModLimb* limbs,
                  const v4i* lazy, int L, int log_n4, uint64_t total4) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (METHOD == kModredBatLazy) {
    // the MFMA needs the whole wave; waves never straddle a limb (N >= 256) and
    // total4 is a multiple of 64, so a wave is either entirely in range or out
    if ((i & ~63ull) >= total4) return;
  } else if (i >= total4) {
    return;
  }
  const uint64_t limb_all = i >> log_n4;
  const int limb = (int)(limb_all % (uint64_t)L);
  const uint64_t wi = ((uint64_t)limb << log_n4) + (i & ((1ull << log_n4) - 1));
  const ModLimb m = limbs[limb];
  const v4u x = a[i], y = w[wi];
  v4u r;
  if (METHOD == kModredBarrett) {
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = barrett64((uint64_t)x[k] * y[k], m);
  } else if (METHOD == kModredMontgomery) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t z = (uint64_t)x[k] * y[k];          // y = w 2^32 mod q
      uint32_t v = (uint32_t)(z >> 32) + m.q - __umulhi((uint32_t)z * m.qinv, m.q);
      r[k] = v >= m.q ? v - m.q : v;
    }
  } else if (METHOD == kModredShoup) {
    const v4u yp = ws[wi];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t v = x[k] * y[k] - __umulhi(x[k], yp[k]) * m.q;
      r[k] = v >= m.q ? v - m.q : v;
    }
  } else {
    // BAT lazy reduction.  Element t of this lane (t < 4) puts the chunks of its
    // product above bit 28 into K segment 4 h + t (h = lane / 32) of the B
    // operand (column lane % 32); the A operand (one 1 KB fragment per prime)
    // holds the 4 x 4 chunk matrix LC of that segment in row block 2 t + h, so
    // the lane gets T_k = sum_j c_(4+j) LC[j][k] of element t in accumulator
    // registers 4t .. 4t + 3 of its own column.
    uint32_t lo[4];
    v4i hb;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t z = (uint64_t)x[k] * y[k];          // < 2^56
      lo[k] = (uint32_t)z & 0x0fffffffu;
      hb[k] = (int)pack7((uint32_t)(z >> 28));
    }
    const v16i T = __builtin_amdgcn_mfma_i32_32x32x32_i8(lazy[limb * 64 + (threadIdx.x & 63)], hb, v16i{}, 0, 0, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // T_j <= 4 * 127^2: the first three shifted terms stay below 2^31
      const uint32_t t012 = (uint32_t)T[4 * k] + ((uint32_t)T[4 * k + 1] << 7) + ((uint32_t)T[4 * k + 2] << 14);
      const uint64_t z = (uint64_t)lo[k] + t012 + ((uint64_t)(uint32_t)T[4 * k + 3] << 21);   // < 2^38
      r[k] = barrett64(z, m);
    }
  }
  if (METHOD == kModredBatLazy && i >= total4) return;
  out[i] = r;
}

// Prepared forms of w: Montgomery w 2^32 mod q, Shoup quotients floor(w 2^32 / q).
__global__ void __launch_bounds__(256)
modmul_prepare_kernel(const uint32_t* w, uint32_t* w_prep, uint32_t* w_quot, const ModLimb* limbs, int log_n,
                      int method, uint64_t total) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const ModLimb m = limbs[i >> log_n];
  const uint32_t v = w[i];
  if (method == kModredMontgomery) {
    w_prep[i] = barrett64((uint64_t)v * m.r32, m);   // r32 = 2^32 mod q
  } else {
    w_prep[i] = v;
    if (method == kModredShoup) w_quot[i] = (uint32_t)(((uint64_t)v << 32) / m.q);
  }
}

inline unsigned blocks_for(uint64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

hipError_t launch_vec_modmul(const uint32_t* a, const uint32_t* w, const uint32_t* w_quot, uint32_t* out,
                             const ModLimb* limbs, const int8_t* lazy, int L, int log_n, int npoly, int method,
                             hipStream_t s) {
  const uint64_t total4 = ((uint64_t)npoly * L) << (log_n - 2);
  const dim3 grid(blocks_for(total4)), block(256);
  const v4u *va = (const v4u*)a, *vw = (const v4u*)w, *vq = (const v4u*)w_quot;
  v4u* vo = (v4u*)out;
  switch (method) {
    case kModredBarrett:
      launch_kernel(vec_modmul_kernel<kModredBarrett>, grid, block, 0, s, va, vw, vq, vo, limbs,
                         (const v4i*)lazy, L, log_n - 2, total4);
      break;
    case kModredMontgomery:
      launch_kernel(vec_modmul_kernel<kModredMontgomery>, grid, block, 0, s, va, vw, vq, vo, limbs,
                         (const v4i*)lazy, L, log_n - 2, total4);
      break;
    case kModredShoup:
      launch_kernel(vec_modmul_kernel<kModredShoup>, grid, block, 0, s, va, vw, vq, vo, limbs,
                         (const v4i*)lazy, L, log_n - 2, total4);
      break;
    case kModredBatLazy:
      if (log_n < 8) return hipErrorInvalidValue;
      launch_kernel(vec_modmul_kernel<kModredBatLazy>, grid, block, 0, s, va, vw, vq, vo, limbs,
                         (const v4i*)lazy, L, log_n - 2, total4);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_modmul_prepare(const uint32_t* w, uint32_t* w_prep, uint32_t* w_quot, const ModLimb* limbs,
                                 int L, int log_n, int method, hipStream_t s) {
  const uint64_t total = (uint64_t)L << log_n;
  launch_kernel(modmul_prepare_kernel, dim3(blocks_for(total)), dim3(256), 0, s, w, w_prep, w_quot, limbs,
                     log_n, method, total);
  return hipGetLastError();
}

}  // namespace cross
