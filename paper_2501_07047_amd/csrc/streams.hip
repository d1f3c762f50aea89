// Chunked forms of the two key-switching vector streams, measured against the
// plain VALU forms (arXiv 2501.07047, App. "Applying BAT to Preknown Parameters":
// evaluation keys through BAT on a fine-grained engine; App. "Fall-back Algorithm
// for unknown parameters", Fig. 1d_conv: a runtime x runtime product as a
// chunk-wise 1D convolution).
//
// Both run on the VALU's four-way byte dot product (v_dot4_u32_u8) with 8-bit
// chunks.  The evaluation-key reduction is only dnum x 4 bytes deep and every
// residue has its own 4 x 4 key block, so there is no operand a 32 x 32 MFMA
// tile could share; a dot4 per output chunk is the finest engine that fits.
//
// Evaluation-key BAT: word l of a residue's expanded key packs bytes
// E[l][0..3] with E[l][i] = byte l of (k 2^(32 + 8 i) mod p), so that
//   y_l = sum_j dot4(e_j, word l of key_j)       (e_j: the four bytes of digit j)
//   V = sum_l y_l 2^(8 l) == 2^32 sum_j k_j e_j  (mod p),  V < p 2^32,
// and one Montgomery reduction finishes.  The expanded key is 16 bytes per
// residue instead of 4.
#include "kernels.h"

namespace cross {

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t dot4(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_udot4(a, b, c, false);
}

// z < q^2 < 2^(2k), k = bit length of q: the quotient estimate is short by at most 2.
__device__ __forceinline__ uint32_t barrett64(uint64_t z, const StreamMod& m) {
  const uint32_t zh = (uint32_t)(z >> (m.bar_k - 1));
  const uint32_t t = (uint32_t)(((uint64_t)zh * m.bar_m) >> (m.bar_k + 1));
  uint32_t r = (uint32_t)z - t * m.q;
  if (r >= m.q) r -= m.q;
  if (r >= m.q) r -= m.q;
  return r;
}

// ChunkMerge of the four byte-position sums (each below 2^20) and Montgomery
// reduction: (V + t q) / 2^32 with t = V qneg mod 2^32; the low words cancel, with
// a carry exactly when V mod 2^32 is not zero.
__device__ __forceinline__ uint32_t merge_redc8(const uint32_t (&y)[4], const StreamMod& m) {
  const uint64_t v = (uint64_t)y[0] + ((uint64_t)y[1] << 8) + ((uint64_t)y[2] << 16) + ((uint64_t)y[3] << 24);
  const uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  const uint32_t t = lo * m.qneg;
  const uint32_t r = hi + __umulhi(t, m.q) + (lo != 0 ? 1u : 0u);
  return r >= m.q ? r - m.q : r;
}

// The exact 64-bit product of two residues from the seven partial sums of the
// byte convolution: with rb = b byte-reversed, dot4(a, rb >> 8 (3 - k)) for
// k <= 3 and dot4(a, rb << 8 (k - 3)) for k > 3 is psum_k = sum_(i+l=k) a_i b_l.
__device__ __forceinline__ uint64_t conv_product(uint32_t a, uint32_t b) {
  const uint32_t rb = __builtin_bswap32(b);
  const uint32_t p0 = dot4(a, rb >> 24, 0), p1 = dot4(a, rb >> 16, 0), p2 = dot4(a, rb >> 8, 0);
  const uint32_t p3 = dot4(a, rb, 0);
  const uint32_t p4 = dot4(a, rb << 8, 0), p5 = dot4(a, rb << 16, 0), p6 = dot4(a, rb << 24, 0);
  const uint64_t lo = (uint64_t)p0 + ((uint64_t)p1 << 8) + ((uint64_t)p2 << 16) + ((uint64_t)p3 << 24);
  const uint64_t hi = (uint64_t)p4 + ((uint64_t)p5 << 8) + ((uint64_t)p6 << 16);
  return lo + (hi << 32);
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t r = a + b;
  return r >= q ? r - q : r;
}

__global__ void __launch_bounds__(256)
evk_bat_prepare_kernel(const uint32_t* key, v4u* kb, const StreamMod* mods, int LK, int log_n, uint64_t total) {
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= total) return;
  const StreamMod m = mods[(int)((x >> log_n) % (uint64_t)LK)];
  const uint32_t k = key[x];
  uint32_t w[4] = {0, 0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t v = barrett64((uint64_t)k * m.pow2[i], m);     // k 2^(32 + 8 i) mod p
#pragma unroll
    for (int l = 0; l < 4; ++l) w[l] |= ((v >> (8 * l)) & 0xffu) << (8 * i);
  }
  kb[x] = v4u{w[0], w[1], w[2], w[3]};
}

// acc[b][s][t][n] = sum_j ext[b][j][t][n] key_j.s[t][n] mod p_t.  A thread takes
// one residue (t, n) of kIpBatch ciphertexts, so each expanded key residue (16
// bytes per digit and polynomial) is read once per kIpBatch ciphertexts.
constexpr int kIpBatch = 4;

__global__ void __launch_bounds__(256)
inner_product_bat_kernel(const uint32_t* ext, const v4u* kb, uint32_t* acc, const StreamMod* mods, int LK,
                         int dnum, int log_n, int B, uint64_t total) {
  const uint64_t x = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= total) return;
  const uint64_t n = x & ((1ull << log_n) - 1), gt = x >> log_n;
  const int t = (int)(gt % (uint64_t)LK);
  const int b0 = (int)(gt / (uint64_t)LK) * kIpBatch;
  const int nb = B - b0 < kIpBatch ? B - b0 : kIpBatch;
  const StreamMod m = mods[t];
  uint32_t y[kIpBatch][2][4] = {};
  for (int j = 0; j < dnum; ++j) {
    const v4u k0 = kb[(((uint64_t)(2 * j) * LK + t) << log_n) | n];
    const v4u k1 = kb[(((uint64_t)(2 * j + 1) * LK + t) << log_n) | n];
#pragma unroll
    for (int i = 0; i < kIpBatch; ++i) {
      if (i < nb) {
        const uint32_t e = ext[((((uint64_t)(b0 + i) * dnum + j) * LK + t) << log_n) | n];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          y[i][0][l] = dot4(e, k0[l], y[i][0][l]);
          y[i][1][l] = dot4(e, k1[l], y[i][1][l]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kIpBatch; ++i) {
    if (i < nb) {
      const uint64_t bb = (uint64_t)(b0 + i);
      acc[((bb * 2 * LK + t) << log_n) | n] = merge_redc8(y[i][0], m);
      acc[(((bb * 2 + 1) * LK + t) << log_n) | n] = merge_redc8(y[i][1], m);
    }
  }
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 limb-wise, every product by convolution.
__global__ void __launch_bounds__(256)
tensor_conv_kernel(const v4u* a, const v4u* b, v4u* out, v4u* d2, const StreamMod* mods, int L, int log_n4,
                   uint64_t total4) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= total4) return;
  const uint64_t per_limb = 1ull << log_n4;
  const uint64_t limb_all = i >> log_n4;
  const int limb = (int)(limb_all % (uint64_t)L);
  const uint64_t bb = limb_all / (uint64_t)L, w = i & (per_limb - 1);
  const uint64_t o0 = ((bb * 2) * L + limb) * per_limb + w, o1 = ((bb * 2 + 1) * L + limb) * per_limb + w;
  const StreamMod m = mods[limb];
  const v4u a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
  v4u r0, r1, r2;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r0[k] = barrett64(conv_product(a0[k], b0[k]), m);
    r1[k] = addmod(barrett64(conv_product(a0[k], b1[k]), m), barrett64(conv_product(a1[k], b0[k]), m), m.q);
    r2[k] = barrett64(conv_product(a1[k], b1[k]), m);
  }
  out[o0] = r0;
  out[o1] = r1;
  d2[(bb * L + limb) * per_limb + w] = r2;
}

inline unsigned blocks_for(uint64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

hipError_t launch_evk_bat_prepare(const uint32_t* key, uint32_t* key_bat, const StreamMod* mods, int LK, int dnum,
                                  int log_n, hipStream_t s) {
  const uint64_t total = ((uint64_t)dnum * 2 * LK) << log_n;
  launch_kernel(evk_bat_prepare_kernel, dim3(blocks_for(total)), dim3(256), 0, s, key, (v4u*)key_bat, mods,
                     LK, log_n, total);
  return hipGetLastError();
}

hipError_t launch_inner_product_bat(const uint32_t* ext, const uint32_t* key_bat, uint32_t* acc,
                                    const StreamMod* mods, int LK, int dnum, int log_n, int B, hipStream_t s) {
  const uint64_t groups = (uint64_t)(B + kIpBatch - 1) / kIpBatch;
  const uint64_t total = (groups * LK) << log_n;
  launch_kernel(inner_product_bat_kernel, dim3(blocks_for(total)), dim3(256), 0, s, ext, (const v4u*)key_bat,
                     acc, mods, LK, dnum, log_n, B, total);
  return hipGetLastError();
}

hipError_t launch_tensor_conv(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                              const StreamMod* mods, int L, int log_n, int B, hipStream_t s) {
  if (log_n < 2) return hipErrorInvalidValue;
  const uint64_t total4 = ((uint64_t)B * L) << (log_n - 2);
  launch_kernel(tensor_conv_kernel, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)a, (const v4u*)b,
                     (v4u*)out, (v4u*)d2, mods, L, log_n - 2, total4);
  return hipGetLastError();
}

}  // namespace cross
