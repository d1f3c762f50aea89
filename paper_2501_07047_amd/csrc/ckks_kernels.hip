// Vector-ALU streams and the BConv MFMA GEMM of CKKS key switching
// (arXiv 2501.07047: Tab. HE_operator_AI_operator -- VecModMul / VecModAdd;
// App. "Basis Conversion (BConv)" -- step 1 L x N VecModMul, step 2 (N, L, L')
// MatModMul, the latter on int8 MFMA through BAT; Sec. Evaluation -- HE-Mult and
// Rotate built from NTT, BConv, VecModMul and automorphism).
//
// The streams are HBM-bound: every kernel reads and writes each residue once,
// with 128-bit (4 x uint32) coalesced accesses per lane.
#include "kernels.h"

#include <algorithm>

namespace cross {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

namespace {

// Barrett multiplication for two runtime residues (Alg. barrett): with
// k = bitlen(q) and m = floor(2^(2k)/q), t = ((z >> (k-1)) * m) >> (k+1)
// underestimates floor(z/q) by at most 2, so two conditional subtractions finish.
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const LimbMod& md) {
  uint64_t z = (uint64_t)a * b;
  uint32_t zh = (uint32_t)(z >> (md.bar_k - 1));
  uint32_t t = (uint32_t)(((uint64_t)zh * md.bar_m) >> (md.bar_k + 1));
  uint32_t r = (uint32_t)z - t * md.q;
  if (r >= md.q) r -= md.q;
  if (r >= md.q) r -= md.q;
  return r;
}

// The same product for wide primes (2^28 <= q < 2^31): the remainder before the two
// subtractions is below 3q, which needs 33 bits, so it is kept in 64.
__device__ __forceinline__ uint32_t mulmod_wide(uint32_t a, uint32_t b, const LimbMod& md) {
  const uint64_t z = (uint64_t)a * b;
  const uint32_t zh = (uint32_t)(z >> (md.bar_k - 1));
  const uint32_t t = (uint32_t)(((uint64_t)zh * md.bar_m) >> (md.bar_k + 1));
  uint64_t r = z - (uint64_t)t * md.q;
  if (r >= md.q) r -= md.q;
  if (r >= md.q) r -= md.q;
  return (uint32_t)r;
}

template <bool WIDE>
__device__ __forceinline__ uint32_t mulmod_t(uint32_t a, uint32_t b, const LimbMod& md) {
  if constexpr (WIDE)
    return mulmod_wide(a, b, md);
  else
    return mulmod(a, b, md);
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) {
  uint32_t r = a + b;
  return r >= q ? r - q : r;
}

// Shoup multiplication by a pre-known w (w_shoup = floor(w 2^32 / q)): result in [0, q).
__device__ __forceinline__ uint32_t mulmod_shoup(uint32_t x, uint32_t w, uint32_t ws, uint32_t q) {
  uint32_t t = __umulhi(x, ws);
  uint32_t r = x * w - t * q;
  return r >= q ? r - q : r;
}

__device__ __forceinline__ uint32_t pack_chunks(uint32_t x) {
  return (x & 0x7fu) | ((x << 1) & 0x7f00u) | ((x << 2) & 0x7f0000u) | ((x << 3) & 0x7f000000u);
}

template <bool WIDE>
__global__ void __launch_bounds__(256)
tensor_kernel(const v4u* a, const v4u* b, v4u* out, v4u* d2, const LimbMod* mods, int L,
              int log_n4, uint64_t total4) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const uint64_t per_limb = 1ull << log_n4;            // vectors per limb
  const uint64_t limb_all = i >> log_n4;                // (b, limb)
  const int limb = (int)(limb_all % L);
  const uint64_t bb = limb_all / L;
  const uint64_t w = i & (per_limb - 1);
  const uint64_t o0 = ((bb * 2 + 0) * L + limb) * per_limb + w;
  const uint64_t o1 = ((bb * 2 + 1) * L + limb) * per_limb + w;
  const LimbMod md = mods[limb];
  v4u a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
  v4u r0, r1, r2;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r0[k] = mulmod_t<WIDE>(a0[k], b0[k], md);
    r1[k] = addmod(mulmod_t<WIDE>(a0[k], b1[k], md), mulmod_t<WIDE>(a1[k], b0[k], md), md.q);
    r2[k] = mulmod_t<WIDE>(a1[k], b1[k], md);
  }
  out[o0] = r0;
  out[o1] = r1;
  d2[(bb * L + limb) * per_limb + w] = r2;
}

// A thread takes four residues (t, 4w..4w+3) of kIpCts ciphertexts, so every key
// vector is read once per kIpCts ciphertexts rather than once per ciphertext.
constexpr int kIpCts = 4;

// With d (NTT-form ModUp input [B][L][N]), digit j's own limbs t in [j alpha,
// (j + 1) alpha) are read from d instead of ext (where they are not stored).
template <bool WIDE>
__global__ void __launch_bounds__(256)
inner_product_kernel(const v4u* ext, const v4u* key, v4u* acc, const LimbMod* mods, int LK,
                     int dnum, int ndig, int log_n4, int B, uint64_t total4, const v4u* d, int L, int alpha) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const uint64_t per_limb = 1ull << log_n4;
  const uint64_t limb_all = i >> log_n4;
  const int t = (int)(limb_all % LK);
  const int b0 = (int)(limb_all / LK) * kIpCts;
  const int nb = B - b0 < kIpCts ? B - b0 : kIpCts;
  const uint64_t w = i & (per_limb - 1);
  const LimbMod md = mods[t];
  v4u s0[kIpCts], s1[kIpCts];
#pragma unroll
  for (int c = 0; c < kIpCts; ++c) s0[c] = s1[c] = v4u{0, 0, 0, 0};
  for (int j = 0; j < ndig; ++j) {
    const v4u k0 = key[((uint64_t)(j * 2 + 0) * LK + t) * per_limb + w];
    const v4u k1 = key[((uint64_t)(j * 2 + 1) * LK + t) * per_limb + w];
    const bool own = d && t < L && t >= j * alpha && t < (j + 1) * alpha;
#pragma unroll
    for (int c = 0; c < kIpCts; ++c) {
      if (c < nb) {
        const v4u e = own ? d[((uint64_t)(b0 + c) * L + t) * per_limb + w]
                          : ext[(((uint64_t)(b0 + c) * dnum + j) * LK + t) * per_limb + w];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          s0[c][k] = addmod(s0[c][k], mulmod_t<WIDE>(e[k], k0[k], md), md.q);
          s1[c][k] = addmod(s1[c][k], mulmod_t<WIDE>(e[k], k1[k], md), md.q);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < kIpCts; ++c) {
    if (c < nb) {
      const uint64_t bb = (uint64_t)(b0 + c);
      acc[((bb * 2 + 0) * LK + t) * per_limb + w] = s0[c];
      acc[((bb * 2 + 1) * LK + t) * per_limb + w] = s1[c];
    }
  }
}

__global__ void __launch_bounds__(256)
moddown_tail_kernel(const v4u* acc, uint64_t acc_stride4, const v4u* z, const v4u* base, v4u* out,
                    uint64_t out_stride4, const TailConst* tc, int L, int log_n4, uint64_t total4,
                    bool base_only_even) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const uint64_t per_limb = 1ull << log_n4;
  const uint64_t limb_all = i >> log_n4;
  const int limb = (int)(limb_all % L);
  const uint64_t p = limb_all / L;
  const uint64_t w = i & (per_limb - 1);
  const TailConst c = tc[limb];
  v4u x = acc[p * acc_stride4 + limb * per_limb + w];
  v4u y = z[(p * L + limb) * per_limb + w];
  const uint64_t oo = p * out_stride4 + limb * per_limb + w;
  const bool use_base = base && (!base_only_even || (p & 1) == 0);
  v4u bs = use_base ? base[oo] : v4u{0, 0, 0, 0};
  v4u r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t d = x[k] + c.q - y[k];                       // in (0, 2q)
    r[k] = addmod(bs[k], mulmod_shoup(d, c.pinv, c.pinv_shoup, c.q), c.q);
  }
  out[oo] = r;
}

__global__ void __launch_bounds__(256)
automorphism_kernel(const uint32_t* in, uint64_t in_stride, uint32_t* out, uint64_t out_stride,
                    const uint32_t* perm, int log_n, int L, uint64_t total) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const uint64_t n = 1ull << log_n;
  const uint64_t limb_all = i >> log_n;
  const uint64_t p = limb_all / L;
  const uint64_t l = limb_all - p * L;
  const uint64_t x = i & (n - 1);
  out[p * out_stride + l * n + x] = in[p * in_stride + l * n + perm[x]];
}

__global__ void __launch_bounds__(256)
pointwise_kernel(const v4u* a, const v4u* b, v4u* out, const LimbMod* mods, int L, int log_n4,
                 uint64_t total4) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const int limb = (int)((i >> log_n4) % L);
  const LimbMod md = mods[limb];
  v4u x = a[i], y = b[i], r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = mulmod(x[k], y[k], md);
  out[i] = r;
}

// HE-Add (VecModAdd): out = a + b mod q_limb.
__global__ void __launch_bounds__(256)
pointwise_add_kernel(const v4u* a, const v4u* b, v4u* out, const LimbMod* mods, int L, int log_n4,
                     uint64_t total4) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const uint32_t q = mods[(int)((i >> log_n4) % L)].q;
  v4u x = a[i], y = b[i], r;
#pragma unroll
  for (int k = 0; k < 4; ++k) r[k] = addmod(x[k], y[k], q);
  out[i] = r;
}

__global__ void __launch_bounds__(256)
limb_copy_kernel(const v4u* src, uint64_t src_stride4, const uint64_t* src_off, v4u* dst,
                 uint64_t dst_stride4, const uint64_t* dst_off, int nl, int log_n4, uint64_t total4) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total4) return;
  const uint64_t per_limb = 1ull << log_n4;
  const uint64_t limb_all = i >> log_n4;
  const int l = (int)(limb_all % nl);
  const uint64_t p = limb_all / nl;
  const uint64_t w = i & (per_limb - 1);
  v4u v = src ? src[p * src_stride4 + src_off[l] / 4 + w] : v4u{0, 0, 0, 0};
  dst[p * dst_stride4 + dst_off[l] / 4 + w] = v;
}

// ---- BConv on MFMA -----------------------------------------------------------
// GEMM: out[(t, ii)][n] = sum_{(i, j)} A[(t, ii)][(i, j)] * chunk_j(b_i[n]), with
// A[(t, ii)][(i, j)] = chunk_ii(([qhat_i]_t * 2^32 * 2^(7j)) mod t) (BAT, Montgomery form).
// v_mfma_i32_32x32x32_i8: 8 targets x 8 sources x 32 coefficients per instruction.
// Lane l of a 32x32 output block holds rows 8(v/4) + 4(l/32) + v%4 (v < 16) of
// column l%32, so the four chunk rows of each target sit in four consecutive
// registers and the merge stays in-register.
//
// Each wave converts 128 consecutive coefficients of the flattened (polynomial,
// coefficient) range.  Lane l loads the four coefficients 4 (l % 32) .. +3 of each of
// its sources with one 16-byte load, and product k (k < 4) takes coefficient k of
// them as column l % 32: after the four products of a 32-target block each lane
// holds four consecutive outputs of each of its targets, stored as one 16-byte word.
// Source and target descriptors are wave-uniform loads (one per pair of lane halves).
//
// Wide primes (template flag WIDE): the B operand is the four bytes of each step-1
// residue, each as b - 128 (one XOR); the accumulators start at the table's int32 row
// corrections, so they hold the plain digit sums, which merge_redc_wide32 merges
// with weights 2^(8i) and reduces (contractions of at most 32 sources).
constexpr int BCONV_MAX_KB = 4;   // up to 32 source limbs
constexpr int BCONV_COLS = 128;   // coefficients per wave

template <int KB, bool WIDE = false>
__device__ __forceinline__ void bconv_wave(const BconvLaunch& g, uint64_t wave_global) {
  const int lane = threadIdx.x & 63, half = lane >> 5;
  const uint64_t total = (uint64_t)g.npoly << g.log_n;
  if (wave_global * BCONV_COLS >= total) return;
  const uint64_t f = wave_global * BCONV_COLS + (uint64_t)(lane & 31) * 4;
  const bool live = f < total;             // total is a multiple of 32: groups of four are whole
  const uint64_t poly = f >> g.log_n, n = f & ((1ull << g.log_n) - 1);
  const uint32_t* in = g.in + poly * g.in_stride + n;
  uint32_t* out = g.out + poly * g.out_stride + n;
  const int kblocks = (g.nsrc + 7) >> 3;
  const int mblocks = (g.ndst + 7) >> 3;

  // B operands: step 1 (x * qhat^-1 mod q) and chunking; bf[kb][k] holds the packed
  // sources kb * 8 + 4 half + e (e < 4) at coefficient 4 (l % 32) + k
  v4i bf[KB][4];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    v4u x[4];
    BconvSrc sd[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i0 = kb * 8 + e, i1 = i0 + 4;
      const BconvSrc s0 = g.src[i0 < g.nsrc ? i0 : 0], s1 = g.src[i1 < g.nsrc ? i1 : 0];
      sd[e] = half ? s1 : s0;
      const bool ok = live && (half ? i1 : i0) < g.nsrc;
      x[e] = ok ? *reinterpret_cast<const v4u*>(in + sd[e].off) : v4u{0, 0, 0, 0};
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t y = mulmod_shoup(x[e][k], sd[e].w, sd[e].w_shoup, sd[e].q);
        bf[kb][k][e] = WIDE ? (int)(y ^ 0x80808080u) : (int)pack_chunks(y);
      }
  }

  for (int mb = 0; mb < mblocks; ++mb) {
    v4i a[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
      a[kb] = kb < kblocks ? *reinterpret_cast<const v4i*>(g.table + ((size_t)(mb * kblocks + kb) * 1024) + lane * 16)
                           : v4i{0, 0, 0, 0};
    BconvDst d[4];
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4) {
      const int t0 = mb * 8 + 2 * g4, t1 = t0 + 1;
      const BconvDst d0 = g.dst[t0 < g.ndst ? t0 : 0], d1 = g.dst[t1 < g.ndst ? t1 : 0];
      d[g4] = half ? d1 : d0;
    }
    // product k, merged and reduced at once: r[g4][k] is target mb * 8 + 2 g4 + half
    // at coefficient 4 (l % 32) + k
    uint32_t r[4][4];
    // wide: lane l's register v of a 32-row block holds row 8 (v / 4) + 4 half + v % 4
    v16i acc0 = v16i{};
    if constexpr (WIDE) {
      const int* corr = reinterpret_cast<const int*>(g.table + (size_t)mblocks * kblocks * 1024) + mb * 32;
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        const v4i c = *reinterpret_cast<const v4i*>(corr + 8 * g4 + 4 * half);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc0[4 * g4 + i] = c[i];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v16i acc = acc0;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        if (kb < kblocks) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[kb], bf[kb][k], acc, 0, 0, 0);
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        if constexpr (WIDE) {
          r[g4][k] = merge_redc_wide32(acc[4 * g4], acc[4 * g4 + 1], acc[4 * g4 + 2], acc[4 * g4 + 3], d[g4].q,
                                       d[g4].qinv);
        } else {
          const uint64_t z = (uint64_t)(uint32_t)acc[4 * g4] + ((uint64_t)(uint32_t)acc[4 * g4 + 1] << 7) +
                             ((uint64_t)(uint32_t)acc[4 * g4 + 2] << 14) +
                             ((uint64_t)(uint32_t)acc[4 * g4 + 3] << 21);
          const uint32_t tq = (uint32_t)z * d[g4].qinv;
          const uint32_t v = (uint32_t)(z >> 32) + d[g4].q - __umulhi(tq, d[g4].q);
          r[g4][k] = v >= d[g4].q ? v - d[g4].q : v;
        }
      }
    }
#pragma unroll
    for (int g4 = 0; g4 < 4; ++g4)
      if (live && mb * 8 + 2 * g4 + half < g.ndst)
        *reinterpret_cast<v4u*>(out + d[g4].off) = v4u{r[g4][0], r[g4][1], r[g4][2], r[g4][3]};
  }
}

// Occupancy: four waves per SIMD for one K block (120 registers, no spills), fewer
// for deeper conversions (more live B operands).
template <int KB, bool WIDE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KB == 1 ? 4 : KB == 2 ? 3 : 2)))
bconv_kernel(BconvLaunch g) {
  bconv_wave<KB, WIDE>(g, ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

// Work-list form (batch runtime): one task per blockIdx.y, KB the largest K-block
// count of the list (tasks with fewer K blocks skip the rest).
template <int KB>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KB == 1 ? 4 : KB == 2 ? 3 : 2)))
bconv_list_kernel(const BconvLaunch* tasks) {
  const BconvLaunch g = tasks[blockIdx.y];
  bconv_wave<KB>(g, ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

// Up to kBconvMulti conversions in one launch, passed by value (one per blockIdx.y):
// the ModUp digits of one call, which alone fill the device only once each.
template <int KB, bool WIDE = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KB == 1 ? 4 : KB == 2 ? 3 : 2)))
bconv_multi_kernel(BconvMulti m) {
  bconv_wave<KB, WIDE>(m.g[blockIdx.y], ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
}

__global__ void __launch_bounds__(256)
tensor_list_kernel(const TensorTask* tasks) {
  const TensorTask t = tasks[blockIdx.y];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.count4) return;
  const int log_n4 = t.log_n - 2;
  const uint64_t per_limb = 1ull << log_n4;
  const int limb = (int)(i >> log_n4);
  const uint64_t w = i & (per_limb - 1);
  const LimbMod md = t.mods[limb];
  const v4u* a = (const v4u*)t.a;
  const v4u* b = (const v4u*)t.b;
  const uint64_t o0 = (uint64_t)limb * per_limb + w, o1 = ((uint64_t)t.L + limb) * per_limb + w;
  v4u a0 = a[o0], a1 = a[o1], b0 = b[o0], b1 = b[o1];
  v4u r0, r1, r2;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    r0[k] = mulmod(a0[k], b0[k], md);
    r1[k] = addmod(mulmod(a0[k], b1[k], md), mulmod(a1[k], b0[k], md), md.q);
    r2[k] = mulmod(a1[k], b1[k], md);
  }
  ((v4u*)t.out)[o0] = r0;
  ((v4u*)t.out)[o1] = r1;
  ((v4u*)t.d2)[o0] = r2;
}

__global__ void __launch_bounds__(256)
auto_list_kernel(const AutoTask* tasks) {
  const AutoTask t = tasks[blockIdx.y];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.count) return;
  const uint64_t n = 1ull << t.log_n;
  const uint64_t limb = i >> t.log_n;
  t.out[i] = t.in[limb * n + t.perm[i & (n - 1)]];
}

__global__ void __launch_bounds__(256)
copy_list_kernel(const CopyTask* tasks) {
  const CopyTask t = tasks[blockIdx.y];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.count4) return;
  ((v4u*)t.dst)[i] = t.src ? ((const v4u*)t.src)[i] : v4u{0, 0, 0, 0};
}

__global__ void __launch_bounds__(256)
inner_list_kernel(const InnerTask* tasks) {
  const InnerTask t = tasks[blockIdx.y];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.count4) return;
  const int log_n4 = t.log_n - 2;
  const uint64_t per_limb = 1ull << log_n4;
  const int limb = (int)(i >> log_n4);
  const uint64_t w = i & (per_limb - 1);
  const LimbMod md = t.mods[limb];
  const v4u* ext = (const v4u*)t.ext;
  const v4u* key = (const v4u*)t.key;
  v4u s0 = {0, 0, 0, 0}, s1 = {0, 0, 0, 0};
  for (int j = 0; j < t.ndig; ++j) {
    v4u e = ext[((uint64_t)j * t.LK + limb) * per_limb + w];
    v4u k0 = key[((uint64_t)(j * 2 + 0) * t.LK + limb) * per_limb + w];
    v4u k1 = key[((uint64_t)(j * 2 + 1) * t.LK + limb) * per_limb + w];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      s0[k] = addmod(s0[k], mulmod(e[k], k0[k], md), md.q);
      s1[k] = addmod(s1[k], mulmod(e[k], k1[k], md), md.q);
    }
  }
  ((v4u*)t.acc)[(uint64_t)limb * per_limb + w] = s0;
  ((v4u*)t.acc)[((uint64_t)t.LK + limb) * per_limb + w] = s1;
}

__global__ void __launch_bounds__(256)
tail_list_kernel(const TailTask* tasks) {
  const TailTask t = tasks[blockIdx.y];
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= t.count4) return;
  const int log_n4 = t.log_n - 2;
  const int limb = (int)(i >> log_n4);
  const TailConst c = t.tc[limb];
  v4u x = ((const v4u*)t.acc)[i];
  v4u y = ((const v4u*)t.z)[i];
  v4u bs = t.base ? ((const v4u*)t.base)[i] : v4u{0, 0, 0, 0};
  v4u r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t d = x[k] + c.q - y[k];
    r[k] = addmod(bs[k], mulmod_shoup(d, c.pinv, c.pinv_shoup, c.q), c.q);
  }
  ((v4u*)t.out)[i] = r;
}

inline unsigned blocks_for(uint64_t total, int per = 256) { return (unsigned)((total + per - 1) / per); }

}  // namespace

hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                         const LimbMod* mods, int L, int log_n, int B, hipStream_t s, bool wide) {
  const uint64_t total4 = ((uint64_t)B * L) << (log_n - 2);
  if (wide)
    launch_kernel(tensor_kernel<true>, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)a, (const v4u*)b,
                  (v4u*)out, (v4u*)d2, mods, L, log_n - 2, total4);
  else
    launch_kernel(tensor_kernel<false>, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)a, (const v4u*)b,
                  (v4u*)out, (v4u*)d2, mods, L, log_n - 2, total4);
  return hipGetLastError();
}

hipError_t launch_inner_product(const uint32_t* ext, const uint32_t* key, uint32_t* acc,
                                const LimbMod* mods, int LK, int dnum, int ndig, int log_n, int B,
                                hipStream_t s, const uint32_t* d, int L, int alpha, bool wide) {
  const uint64_t groups = (uint64_t)(B + kIpCts - 1) / kIpCts;
  const uint64_t total4 = (groups * LK) << (log_n - 2);
  if (wide)
    launch_kernel(inner_product_kernel<true>, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)ext,
                  (const v4u*)key, (v4u*)acc, mods, LK, dnum, ndig, log_n - 2, B, total4, (const v4u*)d, L, alpha);
  else
    launch_kernel(inner_product_kernel<false>, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)ext,
                  (const v4u*)key, (v4u*)acc, mods, LK, dnum, ndig, log_n - 2, B, total4, (const v4u*)d, L, alpha);
  return hipGetLastError();
}

hipError_t launch_moddown_tail(const uint32_t* acc, uint64_t acc_stride, const uint32_t* z,
                               const uint32_t* base, uint32_t* out, uint64_t out_stride,
                               const TailConst* tc, int L, int log_n, int npoly,
                               bool base_only_even, hipStream_t s) {
  const uint64_t total4 = ((uint64_t)npoly * L) << (log_n - 2);
  launch_kernel(moddown_tail_kernel, dim3(blocks_for(total4)), dim3(256), 0, s,
                     (const v4u*)acc, acc_stride / 4, (const v4u*)z, (const v4u*)base, (v4u*)out,
                     out_stride / 4, tc, L, log_n - 2, total4, base_only_even);
  return hipGetLastError();
}

hipError_t launch_automorphism(const uint32_t* in, uint64_t in_stride, uint32_t* out,
                               uint64_t out_stride, const uint32_t* perm, int log_n, int L,
                               int npoly, hipStream_t s) {
  const uint64_t total = ((uint64_t)npoly * L) << log_n;
  launch_kernel(automorphism_kernel, dim3(blocks_for(total)), dim3(256), 0, s, in, in_stride,
                     out, out_stride, perm, log_n, L, total);
  return hipGetLastError();
}

hipError_t launch_pointwise_mul(const uint32_t* a, const uint32_t* b, uint32_t* out,
                                const LimbMod* mods, int L, int log_n, int B, hipStream_t s) {
  const uint64_t total4 = ((uint64_t)B * L) << (log_n - 2);
  launch_kernel(pointwise_kernel, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)a,
                     (const v4u*)b, (v4u*)out, mods, L, log_n - 2, total4);
  return hipGetLastError();
}

hipError_t launch_pointwise_add(const uint32_t* a, const uint32_t* b, uint32_t* out,
                                const LimbMod* mods, int L, int log_n, int npoly, hipStream_t s) {
  const uint64_t total4 = ((uint64_t)npoly * L) << (log_n - 2);
  launch_kernel(pointwise_add_kernel, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)a,
                     (const v4u*)b, (v4u*)out, mods, L, log_n - 2, total4);
  return hipGetLastError();
}

hipError_t launch_limb_copy(const uint32_t* src, uint64_t src_stride, const uint64_t* src_off,
                            uint32_t* dst, uint64_t dst_stride, const uint64_t* dst_off, int nl,
                            int log_n, int npoly, hipStream_t s) {
  const uint64_t total4 = ((uint64_t)npoly * nl) << (log_n - 2);
  launch_kernel(limb_copy_kernel, dim3(blocks_for(total4)), dim3(256), 0, s, (const v4u*)src,
                     src_stride / 4, src_off, (v4u*)dst, dst_stride / 4, dst_off, nl, log_n - 2,
                     total4);
  return hipGetLastError();
}

hipError_t launch_tensor_list(const TensorTask* t, int n, uint64_t max4, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_kernel(tensor_list_kernel, dim3(blocks_for(max4), n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_auto_list(const AutoTask* t, int n, uint64_t max_count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_kernel(auto_list_kernel, dim3(blocks_for(max_count), n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_copy_list(const CopyTask* t, int n, uint64_t max4, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_kernel(copy_list_kernel, dim3(blocks_for(max4), n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_inner_list(const InnerTask* t, int n, uint64_t max4, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_kernel(inner_list_kernel, dim3(blocks_for(max4), n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_tail_list(const TailTask* t, int n, uint64_t max4, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  launch_kernel(tail_list_kernel, dim3(blocks_for(max4), n), dim3(256), 0, s, t);
  return hipGetLastError();
}
hipError_t launch_bconv_list(const BconvLaunch* t, int n, uint64_t max_cols, int max_nsrc, hipStream_t s) {
  if (n <= 0 || max_cols == 0) return hipSuccess;
  if (max_nsrc < 1 || max_nsrc > 8 * BCONV_MAX_KB) return hipErrorInvalidValue;   // (narrow primes only)
  const dim3 grid(blocks_for((max_cols + BCONV_COLS - 1) / BCONV_COLS * 64), n);
  switch ((max_nsrc + 7) >> 3) {
    case 1: launch_kernel(bconv_list_kernel<1>, grid, dim3(256), 0, s, t); break;
    case 2: launch_kernel(bconv_list_kernel<2>, grid, dim3(256), 0, s, t); break;
    case 3: launch_kernel(bconv_list_kernel<3>, grid, dim3(256), 0, s, t); break;
    default: launch_kernel(bconv_list_kernel<4>, grid, dim3(256), 0, s, t); break;
  }
  return hipGetLastError();
}

hipError_t launch_bconv_multi(const BconvLaunch* gs, int n, hipStream_t s) {
  for (int base = 0; base < n; base += kBconvMulti) {
    BconvMulti m{};
    const int cnt = n - base < kBconvMulti ? n - base : kBconvMulti;
    uint64_t cols = 0;
    int nsrc = 1;
    for (int i = 0; i < cnt; ++i) {
      const BconvLaunch& b = gs[base + i];
      if (b.nsrc < 1 || b.nsrc > 8 * BCONV_MAX_KB || b.ndst < 1 || b.log_n < 5 || b.npoly < 0 ||
          b.wide != gs[base].wide)
        return hipErrorInvalidValue;      // one launch takes one form
      m.g[i] = b;
      cols = std::max(cols, (uint64_t)b.npoly << b.log_n);
      nsrc = std::max(nsrc, b.nsrc);
    }
    if (cols == 0) continue;
    const dim3 grid(blocks_for((cols + BCONV_COLS - 1) / BCONV_COLS * 64), cnt);
    const int kb = (nsrc + 7) >> 3;
    if (gs[base].wide) {
      switch (kb) {
        case 1: launch_kernel(bconv_multi_kernel<1, true>, grid, dim3(256), 0, s, m); break;
        case 2: launch_kernel(bconv_multi_kernel<2, true>, grid, dim3(256), 0, s, m); break;
        case 3: launch_kernel(bconv_multi_kernel<3, true>, grid, dim3(256), 0, s, m); break;
        default: launch_kernel(bconv_multi_kernel<4, true>, grid, dim3(256), 0, s, m); break;
      }
    } else {
      switch (kb) {
        case 1: launch_kernel(bconv_multi_kernel<1>, grid, dim3(256), 0, s, m); break;
        case 2: launch_kernel(bconv_multi_kernel<2>, grid, dim3(256), 0, s, m); break;
        case 3: launch_kernel(bconv_multi_kernel<3>, grid, dim3(256), 0, s, m); break;
        default: launch_kernel(bconv_multi_kernel<4>, grid, dim3(256), 0, s, m); break;
      }
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_bconv(const BconvLaunch& b, hipStream_t s) {
  if (b.nsrc < 1 || b.nsrc > 8 * BCONV_MAX_KB || b.ndst < 1 || b.log_n < 5) return hipErrorInvalidValue;
  if (b.npoly <= 0) return hipSuccess;
  const uint64_t waves = (((uint64_t)b.npoly << b.log_n) + BCONV_COLS - 1) / BCONV_COLS;
  const dim3 grid(blocks_for(waves * 64));
  if (b.wide) {
    switch ((b.nsrc + 7) >> 3) {
      case 1: launch_kernel(bconv_kernel<1, true>, grid, dim3(256), 0, s, b); break;
      case 2: launch_kernel(bconv_kernel<2, true>, grid, dim3(256), 0, s, b); break;
      case 3: launch_kernel(bconv_kernel<3, true>, grid, dim3(256), 0, s, b); break;
      default: launch_kernel(bconv_kernel<4, true>, grid, dim3(256), 0, s, b); break;
    }
    return hipGetLastError();
  }
  switch ((b.nsrc + 7) >> 3) {
    case 1: launch_kernel(bconv_kernel<1>, grid, dim3(256), 0, s, b); break;
    case 2: launch_kernel(bconv_kernel<2>, grid, dim3(256), 0, s, b); break;
    case 3: launch_kernel(bconv_kernel<3>, grid, dim3(256), 0, s, b); break;
    default: launch_kernel(bconv_kernel<4>, grid, dim3(256), 0, s, b); break;
  }
  return hipGetLastError();
}

}  // namespace cross
