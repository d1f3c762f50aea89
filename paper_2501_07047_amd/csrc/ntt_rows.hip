// Three-factor layout-invariant NTT: the C-point row transform of step 3 (and
// the first step of the inverse) with each row split as C1 x C2 (MAT applied to
// a third dimension, arXiv 2501.07047 Sec. MAT; reading G18).
//
// A row of C = C1 * C2 residues is a C1 x C2 matrix in place (c = c1 * C2 + c2).
// Forward, per row:  Z = (TB @ Y) (.) T3   (C1-point transform over c1, twiddle)
//                    X = Z @ TC            (C2-point transform over c2)
// Inverse, per row:  Z = (X @ ITC) (.) IT3;  Y = (ITB @ Z) (.) IT2  (IT2: the inverse
//                    step-2 twiddle of the outer R x C split, applied here)
// Both sub-steps are BAT int8 GEMMs on v_mfma_i32_32x32x32_i8 with the same
// epilogue as the step GEMMs (ChunkMerge, REDC with the Montgomery factor folded
// into the tables, Shoup twiddle, one conditional subtraction, 7-bit packing).
//
// One workgroup (kRowsWaves waves) takes kRowsWaves * 1024 / C rows of one
// polynomial and prime: the input rows are read once from HBM, the intermediate
// Z lives in LDS, and the output rows are staged in LDS (over Z) and written
// back as 16-byte row segments.  Each wave owns whole 32-column blocks of a
// sub-step (all of its M rows), so a B fragment is loaded once.  The two
// tables (16 C1^2 and 16 C2^2 bytes in fragment order) and the first
// epilogue's twiddle pairs are copied into LDS once per workgroup with 16-byte
// loads, so the per-wave memory instructions are the data rows alone (plus the
// inverse step-2 twiddles); only at C1 = C2 = 64, where the tables do not fit
// beside the Z tile, are table fragments read from global memory (L1 / L2).
//
// Wide primes (2^28 <= q < 2^31, template flag WIDE): the data operand is the
// four bytes of a residue, each fed as b - 128 (one XOR instead of the 7-bit
// packing); the tables hold balanced signed 8-bit digits followed by one int32
// row correction 128 * (row sum) per row, staged with them and used as the
// accumulators' start; the epilogue merges with weights 2^(8i) in 64 bits and
// reduces with a signed Montgomery step (Montgomery epilogue only).
#include "kernels.h"

#include <algorithm>
#include <type_traits>

namespace cross {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

constexpr int kRowsWaves = 8;          // waves per workgroup
constexpr int kLdsBytes = 160 * 1024;  // LDS per CU

// Buffer descriptor of a workgroup-uniform range (base and size are read from
// the first lane, so the descriptor always lives in SGPRs).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const void* base, uint64_t bytes) {
  const uint64_t v = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  const uint32_t n = __builtin_amdgcn_readfirstlane(bytes > 0xfffffff0ull ? 0xfffffff0u : (uint32_t)bytes);
  void* p = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, (int)n, 0x00020000);
}

__device__ __forceinline__ uint32_t pack7(uint32_t x) {
  // (x & 0x7f) | (x & 0x3f80) << 1 | (x & 0x1fc000) << 2 | (x & 0xfe00000) << 3, as
  // x plus each chunk times 2^i - 1
  return x + (x & ~0x7fu) + ((x & ~0x3fffu) << 1) + ((x & ~0x1fffffu) << 2);
}

// Data operand of a residue: four 7-bit chunks, or (wide primes) its four bytes
// each biased to b - 128.
template <bool WIDE>
__device__ __forceinline__ uint32_t operand(uint32_t x) {
  if constexpr (WIDE)
    return x ^ 0x80808080u;
  else
    return pack7(x);
}

// ChunkMerge of register group j (the four chunk sums of one output) and REDC:
// (0, 2q).  Contractions here are at most 256 chunks deep, so both half-merges
// fit 32 bits.
__device__ __forceinline__ uint32_t merge_redc(const v16i& a, int j, uint32_t q, uint32_t qinv) {
  const uint32_t x = (uint32_t)a[4 * j] + ((uint32_t)a[4 * j + 1] << 7);
  const uint32_t w = (uint32_t)a[4 * j + 2] + ((uint32_t)a[4 * j + 3] << 7);
  const uint32_t wl = w << 14;
  const uint32_t lo = x + wl;
  const uint32_t hi = (w >> 18) + (lo < wl ? 1u : 0u);
  return hi + q - __umulhi(lo * qinv, q);
}

// ChunkMerge and Barrett reduction (Alg. barrett) for plain tables: with k = bit
// length of q, z = x + w 2^14 < 2^44 <= 2^(2k), the quotient estimate
// ((z >> (k - 1)) * floor(2^(2k) / q)) >> (k + 1) is short by at most 2: [0, q).
__device__ __forceinline__ uint32_t merge_barrett(const v16i& a, int j, uint32_t q, uint32_t bar_m, uint32_t bar_k) {
  const uint32_t x = (uint32_t)a[4 * j] + ((uint32_t)a[4 * j + 1] << 7);
  const uint32_t w = (uint32_t)a[4 * j + 2] + ((uint32_t)a[4 * j + 3] << 7);
  const uint32_t wl = w << 14;
  const uint32_t lo = x + wl;
  const uint32_t hi = (w >> 18) + (lo < wl ? 1u : 0u);
  const uint32_t zh = (hi << (33 - bar_k)) | (lo >> (bar_k - 1));
  const uint32_t t = (uint32_t)(((uint64_t)zh * bar_m) >> (bar_k + 1));
  uint32_t r = lo - t * q;
  r = r >= q ? r - q : r;
  return r >= q ? r - q : r;
}

// Wide primes: merge of the four signed digit sums and signed Montgomery
// reduction (contractions here are at most 64 inputs deep).
__device__ __forceinline__ uint32_t merge_redc_wide(const v16i& a, int j, uint32_t q, uint32_t qinv) {
  return merge_redc_wide32(a[4 * j], a[4 * j + 1], a[4 * j + 2], a[4 * j + 3], q, qinv);
}

// Epilogue reduction of register group j: RED = 0 Montgomery (0, 2q), 1 Barrett
// [0, q); wide primes (Montgomery only) [0, q).
template <int RED, bool WIDE>
__device__ __forceinline__ uint32_t merge_reduce(const v16i& a, int j, const RowsJob& jb) {
  if constexpr (WIDE)
    return merge_redc_wide(a, j, jb.q, jb.qinv);
  else if constexpr (RED == 0)
    return merge_redc(a, j, jb.q, jb.qinv);
  else
    return merge_barrett(a, j, jb.q, jb.bar_m, jb.bar_k);
}

__device__ __forceinline__ uint32_t shoup_tw(uint32_t r, v2u tw, uint32_t q) {
  const uint32_t v = r * tw.x - __umulhi(r, tw.y) * q;      // [0, 2q)
  return v >= q ? v - q : v;
}

// Table fragment sources: LDS (staged once per workgroup) or global memory.
struct LdsTab {
  const int8_t* p;
  __device__ __forceinline__ v4i operator()(int off) const { return *reinterpret_cast<const v4i*>(p + off); }
};
struct GlobalTab {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ v4i operator()(int off) const {
    return (v4i)__builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  }
};

template <bool IN_LDS>
__device__ __forceinline__ auto table(const int8_t* lds, const int8_t* global, int bytes) {
  if constexpr (IN_LDS)
    return LdsTab{lds};
  else
    return GlobalTab{rows_rsrc(global, (uint64_t)bytes)};
}

// acc[mb] = sum over KS K-steps of table fragment (mb, ks) x B fragment bfrag(ks):
// the M x K table (M = 32 MB) is in fragment order, fragment (mb, ks) at byte
// ((ks / 2) * MB + mb) * 2048 + (ks % 2) * 1024, 16 bytes per lane.
//
// Wide primes: the M int32 row corrections follow the table (at byte M * K) and
// start the accumulators; lane l starts register v of block mb at the correction
// of row mb * 32 + 8 (v / 4) + 4 (l / 32) + v % 4.
template <int MB, int KS, bool WIDE, class TAB, class BF>
__device__ __forceinline__ void block_gemm(v16i (&acc)[MB], const TAB& tab, int lane, BF bfrag) {
  if constexpr (WIDE) {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const v4i c = tab(MB * KS * 1024 + (mb * 32 + 8 * j + 4 * (lane >> 5)) * 4);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[mb][4 * j + i] = c[i];
      }
    // the K-step groups below pair table reads with products; the correction
    // reads stay out of them
    __builtin_amdgcn_sched_barrier(0);
  } else {
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) acc[mb] = v16i{};
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const v4i b = bfrag(ks);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const v4i a = tab(((ks >> 1) * MB + mb) * 2048 + (ks & 1) * 1024 + lane * 16);
      acc[mb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[mb], 0, 0, 0);
    }
    // keep each K-step's table reads next to its products (bounds the registers
    // held by fragments read ahead)
    __builtin_amdgcn_sched_group_barrier(0x100, MB, 0);
    __builtin_amdgcn_sched_group_barrier(0x008, MB, 0);
  }
}

template <int C1, int C2, bool WIDE = false>
struct RowsShape {
  static constexpr int C = C1 * C2;
  static constexpr int NW = kRowsWaves, NT = 64 * kRowsWaves;
  static constexpr int BR = NW * 1024 / C;      // rows per workgroup
  static constexpr int ZP1 = C2 + 4;            // forward Z line [row][m][.] (words, 16-byte rows)
  static constexpr int ZP2 = C1 + 4;            // inverse Z line [row][c2][.]
  static constexpr int XP = C2 + 1;             // output staging line [row][c1 or m][.]
  static constexpr int ZA = BR * C1 * ZP1, ZB = BR * C2 * ZP2, XW = BR * C1 * XP;
  // Z tile, reused for the output staging once every wave has read it
  static constexpr int ZWORDS = (ZA > ZB ? ZA : ZB) > XW ? (ZA > ZB ? ZA : ZB) : XW;
  // two workgroups per CU (4 waves per SIMD, at most 128 registers) where the
  // accumulators allow; the 64-wide splits keep more registers at one
  static constexpr int OCC = (C1 <= 32 && C2 <= 32) ? 4 : 2;
  // table bytes (wide primes: with their row corrections)
  static constexpr int TB1 = 16 * C1 * C1 + (WIDE ? 16 * C1 : 0), TB2 = 16 * C2 * C2 + (WIDE ? 16 * C2 : 0);
  // C1 = C2: the two sub-step tables are one matrix (TB[m][c1] = psi^(2R C2 c1 brv(m))
  // and TC[c2][c2'] = psi^(2R C1 c2 brv(c2')) coincide, as do ITC and ITB), so a
  // single copy is staged
  static constexpr bool SHARED = C1 == C2;
  // the tables in LDS where they fit beside the Z tile and the twiddles
  static constexpr bool TAB_LDS = (SHARED ? TB1 : TB1 + TB2) + 8 * C + 4 * ZWORDS <= kLdsBytes;
  static constexpr int T1 = TAB_LDS ? TB1 : 16, T2 = (TAB_LDS && !SHARED) ? TB2 : 16;
  static_assert(C1 >= 16 && C2 >= 16 && BR >= 1 && (NW * 1024) % C == 0, "row split");
};

// Locate the workgroup's rows: block = (job, poly, row block).
struct RowsPos {
  RowsJob job;
  uint64_t base;    // element offset of the first row
  int row0;         // first row index within the polynomial's R rows
};

template <int BR, int C>
__device__ __forceinline__ RowsPos rows_pos(const RowsJob* jobs, uint64_t stride, int npoly, int log_r) {
  // R / BR row blocks per polynomial (both powers of two); the quotient is made
  // explicitly wave-uniform so that the row buffers' descriptors stay in SGPRs
  constexpr int kLogBr = __builtin_ctz(BR);
  const int lpp = log_r - kLogBr;
  const int b = blockIdx.x;
  const int rb = b & ((1 << lpp) - 1);
  const int pj = b >> lpp;
  const int jb = __builtin_amdgcn_readfirstlane(pj / npoly);
  const int poly = pj - jb * npoly;
  RowsPos p;
  p.job = jobs[jb];
  p.row0 = rb * BR;
  p.base = p.job.off + (uint64_t)poly * stride + (uint64_t)p.row0 * C;
  return p;
}

// Copy `bytes` (a multiple of 16) from global memory to LDS with 16-byte loads.
template <int NT>
__device__ __forceinline__ void stage(void* lds, const void* src, int bytes) {
  const __amdgpu_buffer_rsrc_t r = rows_rsrc(src, (uint64_t)bytes);
  for (int o = threadIdx.x * 16; o < bytes; o += NT * 16)
    *reinterpret_cast<v4u*>(static_cast<char*>(lds) + o) = __builtin_amdgcn_raw_buffer_load_b128(r, o, 0, 0);
}

// Write the staged output rows [row][line][.] (line = c1 or m, XP words) back to
// global memory as 16-byte row segments.
template <int C1, int C2>
__device__ __forceinline__ void write_rows(const uint32_t* xs, __amdgpu_buffer_rsrc_t rout) {
  using S = RowsShape<C1, C2>;
#pragma unroll
  for (int it = 0; it < S::BR * S::C / 4 / S::NT; ++it) {
    const int e = (threadIdx.x + it * S::NT) * 4;       // element of the workgroup's rows
    const int row = e / S::C, rem = e % S::C;
    const int line = rem / C2, c = rem % C2;
    const uint32_t* src = xs + (row * C1 + line) * S::XP + c;
    const v4u v = v4u{src[0], src[1], src[2], src[3]};
    __builtin_amdgcn_raw_buffer_store_b128(v, rout, e * 4, 0, 0);
  }
}

template <int C1, int C2, int RED, bool WIDE>
__global__ void __launch_bounds__(64 * kRowsWaves, (RowsShape<C1, C2>::OCC))
ntt_rows_fwd_kernel(const RowsJob* jobs, const uint32_t* in, uint32_t* out, uint64_t stride, int npoly, int log_r) {
  using S = RowsShape<C1, C2, WIDE>;
  constexpr int C = S::C, BR = S::BR;
  constexpr int MB1 = C1 / 8, MB2 = C2 / 8;                 // 32-row blocks (M = 4 C1, 4 C2)
  constexpr int NB1 = BR * C2 / 32, NB2 = BR * C1 / 32;     // 32-column blocks of the two sub-steps
  constexpr int NBW2 = (NB2 + S::NW - 1) / S::NW;           // sub-step 2 blocks per wave
  __shared__ __attribute__((aligned(16))) int8_t tab1s[S::T1];
  __shared__ __attribute__((aligned(16))) int8_t tab2s[S::T2];
  __shared__ __attribute__((aligned(16))) uint32_t tws[2 * C];
  __shared__ __attribute__((aligned(16))) uint32_t zs[S::ZWORDS];
  const RowsPos P = rows_pos<BR, C>(jobs, stride, npoly, log_r);
  const __amdgpu_buffer_rsrc_t rin = rows_rsrc(in + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t rout = rows_rsrc(out + P.base, (uint64_t)BR * C * 4);
  const auto tab1 = table<S::TAB_LDS>(tab1s, P.job.tab1, S::TB1);
  const auto tab2 = table<S::TAB_LDS>(S::SHARED ? tab1s : tab2s, S::SHARED ? P.job.tab1 : P.job.tab2, S::TB2);
  if constexpr (S::TAB_LDS) {
    stage<S::NT>(tab1s, P.job.tab1, S::TB1);
    if constexpr (!S::SHARED) stage<S::NT>(tab2s, P.job.tab2, S::TB2);
  }
  stage<S::NT>(tws, P.job.tw1, 8 * C);
  const uint32_t q = P.job.q;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __syncthreads();

  // sub-step 1: columns (row, c2), contraction over c1 (packed input, 4 words C2 apart)
  for (int cb = wave; cb < NB1; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C2, c2 = col % C2;
    v16i acc[MB1];
    block_gemm<MB1, MB1, WIDE>(acc, tab1, lane, [&](int ks) {
      const uint32_t o = (uint32_t)(row * C + (8 * ks + 4 * h) * C2 + c2) * 4;
      return v4i{(int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 0, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, C2 * 4, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 2 * C2 * 4, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 3 * C2 * 4, 0)};
    });
    // output m = mb * 8 + 2 j + h: lane bases plus compile-time offsets
    const uint32_t* twl = &tws[(h * C2 + c2) * 2];
    uint32_t* zl = &zs[(row * C1 + h) * S::ZP1 + c2];
#pragma unroll
    for (int mb = 0; mb < MB1; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m0 = mb * 8 + 2 * j;
        const v2u w = *reinterpret_cast<const v2u*>(&twl[m0 * C2 * 2]);
        zl[m0 * S::ZP1] = operand<WIDE>(shoup_tw(merge_reduce<RED, WIDE>(acc[mb], j, P.job), w, q));
      }
  }
  __syncthreads();
  // sub-step 2: columns (row, m), contraction over c2 (16 contiguous bytes of a Z line);
  // every block of the wave is multiplied before the Z tile is overwritten
  v16i acc2[NBW2][MB2];
#pragma unroll
  for (int i = 0; i < NBW2; ++i) {
    const int cb = wave + i * S::NW;
    if (cb < NB2) {
      const int col = cb * 32 + (lane & 31);
      const int row = col / C1, m = col % C1;
      block_gemm<MB2, MB2, WIDE>(acc2[i], tab2, lane, [&](int ks) {
        return *reinterpret_cast<const v4i*>(&zs[(row * C1 + m) * S::ZP1 + 8 * ks + 4 * h]);
      });
    }
  }
  __syncthreads();
  uint32_t* xs = zs;
#pragma unroll
  for (int i = 0; i < NBW2; ++i) {
    const int cb = wave + i * S::NW;
    if (cb < NB2) {
      const int col = cb * 32 + (lane & 31);
      const int row = col / C1, m = col % C1;
      uint32_t* xl = &xs[(row * C1 + m) * S::XP + h];     // output c2' = mb * 8 + 2 j + h
#pragma unroll
      for (int mb = 0; mb < MB2; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t r = merge_reduce<RED, WIDE>(acc2[i][mb], j, P.job);
          xl[mb * 8 + 2 * j] = r >= q ? r - q : r;
        }
    }
  }
  __syncthreads();
  write_rows<C1, C2>(xs, rout);
}

template <int C1, int C2, int RED, bool WIDE>
__global__ void __launch_bounds__(64 * kRowsWaves, (RowsShape<C1, C2>::OCC))
ntt_rows_inv_kernel(const RowsJob* jobs, const uint32_t* in, uint32_t* out, uint64_t stride, int npoly, int log_r) {
  using S = RowsShape<C1, C2, WIDE>;
  constexpr int C = S::C, BR = S::BR;
  constexpr int MB1 = C2 / 8, MB2 = C1 / 8;                 // sub-step 1 over c2', sub-step 2 over m
  constexpr int NB1 = BR * C1 / 32, NB2 = BR * C2 / 32;
  constexpr int NBW2 = (NB2 + S::NW - 1) / S::NW;
  __shared__ __attribute__((aligned(16))) int8_t tab1s[S::SHARED ? S::T1 : S::T2];
  __shared__ __attribute__((aligned(16))) int8_t tab2s[S::SHARED ? S::T2 : S::T1];
  __shared__ __attribute__((aligned(16))) uint32_t tws[2 * C];
  __shared__ __attribute__((aligned(16))) uint32_t zs[S::ZWORDS];
  const RowsPos P = rows_pos<BR, C>(jobs, stride, npoly, log_r);
  const __amdgpu_buffer_rsrc_t rin = rows_rsrc(in + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t rout = rows_rsrc(out + P.base, (uint64_t)BR * C * 4);
  // inverse step-2 twiddles of this workgroup's rows: pairs [row][c]
  const __amdgpu_buffer_rsrc_t tw2 = rows_rsrc(P.job.tw2 + (uint64_t)P.row0 * C * 2, (uint64_t)8 * BR * C);
  const auto tab1 = table<S::TAB_LDS>(tab1s, P.job.tab1, S::TB2);
  const auto tab2 = table<S::TAB_LDS>(S::SHARED ? tab1s : tab2s, S::SHARED ? P.job.tab1 : P.job.tab2, S::TB1);
  if constexpr (S::TAB_LDS) {
    stage<S::NT>(tab1s, P.job.tab1, S::TB2);
    if constexpr (!S::SHARED) stage<S::NT>(tab2s, P.job.tab2, S::TB1);
  }
  stage<S::NT>(tws, P.job.tw1, 8 * C);
  const uint32_t q = P.job.q;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  __syncthreads();

  // sub-step 1: columns (row, m), contraction over c2' (plain input, 16 contiguous bytes)
  for (int cb = wave; cb < NB1; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C1, m = col % C1;
    v16i acc[MB1];
    block_gemm<MB1, MB1, WIDE>(acc, tab1, lane, [&](int ks) {
      const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rin, (uint32_t)(row * C + m * C2 + 8 * ks + 4 * h) * 4, 0, 0);
      return v4i{(int)operand<WIDE>(x.x), (int)operand<WIDE>(x.y), (int)operand<WIDE>(x.z), (int)operand<WIDE>(x.w)};
    });
    // output c2 = mb * 8 + 2 j + h: lane bases plus compile-time offsets (IT3 pairs [c2][m])
    const uint32_t* twl = &tws[(h * C1 + m) * 2];
    uint32_t* zl = &zs[(row * C2 + h) * S::ZP2 + m];
#pragma unroll
    for (int mb = 0; mb < MB1; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c0 = mb * 8 + 2 * j;
        const v2u w = *reinterpret_cast<const v2u*>(&twl[c0 * C1 * 2]);
        zl[c0 * S::ZP2] = operand<WIDE>(shoup_tw(merge_reduce<RED, WIDE>(acc[mb], j, P.job), w, q));
      }
  }
  __syncthreads();
  // sub-step 2: columns (row, c2), contraction over m (16 contiguous bytes of a Z line)
  v16i acc2[NBW2][MB2];
#pragma unroll
  for (int i = 0; i < NBW2; ++i) {
    const int cb = wave + i * S::NW;
    if (cb < NB2) {
      const int col = cb * 32 + (lane & 31);
      const int row = col / C2, c2 = col % C2;
      block_gemm<MB2, MB2, WIDE>(acc2[i], tab2, lane, [&](int ks) {
        return *reinterpret_cast<const v4i*>(&zs[(row * C2 + c2) * S::ZP2 + 8 * ks + 4 * h]);
      });
    }
  }
  __syncthreads();
  uint32_t* xs = zs;
#pragma unroll
  for (int i = 0; i < NBW2; ++i) {
    const int cb = wave + i * S::NW;
    if (cb < NB2) {
      const int col = cb * 32 + (lane & 31);
      const int row = col / C2, c2 = col % C2;
      // output c1 = mb * 8 + 2 j + h: lane bases plus compile-time offsets
      const uint32_t twl = (uint32_t)(row * C + h * C2 + c2) * 8;
      uint32_t* xl = &xs[(row * C1 + h) * S::XP + c2];
#pragma unroll
      for (int mb = 0; mb < MB2; ++mb)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c0 = mb * 8 + 2 * j;
          const v2u w = __builtin_amdgcn_raw_buffer_load_b64(tw2, twl, c0 * C2 * 8, 0);
          xl[c0 * S::XP] = operand<WIDE>(shoup_tw(merge_reduce<RED, WIDE>(acc2[i][mb], j, P.job), w, q));
        }
    }
  }
  __syncthreads();
  write_rows<C1, C2>(xs, rout);
}

template <int C1, int C2, int RED, bool WIDE = false>
hipError_t rows_cfg(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                    int npoly, int log_r, bool inverse, hipStream_t s) {
  using S = RowsShape<C1, C2, WIDE>;
  if ((1 << log_r) % S::BR) return hipErrorInvalidValue;
  const int grid = njobs * npoly * ((1 << log_r) / S::BR);
  if (inverse)
    launch_kernel((ntt_rows_inv_kernel<C1, C2, RED, WIDE>), dim3(grid), dim3(S::NT), 0, s, jobs, in, out, stride, npoly,
                       log_r);
  else
    launch_kernel((ntt_rows_fwd_kernel<C1, C2, RED, WIDE>), dim3(grid), dim3(S::NT), 0, s, jobs, in, out, stride, npoly,
                       log_r);
  return hipGetLastError();
}

// Compute units of the current device (cached per device).
int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    cached[dev] = (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
                      ? n : 256;
  }
  return cached[dev];
}

// ---- persistent row kernels for C1 = C2 = 32 ---------------------------------
// With C = 1024 and eight waves per block of eight rows, wave w owns row w of the
// block in both sub-steps (its 32 columns are (row w, c2) in the first and (row w,
// m) in the second), so the sub-steps exchange data only inside a wave: each wave
// keeps its row's Z lines and output staging in a private LDS slice and needs no
// workgroup barrier.  Each workgroup walks a contiguous range of blocks; when the
// range enters a new prime it stages that prime's 16 KB sub-step table (one matrix
// for both sub-steps, C1 = C2) and first twiddles into LDS and copies the table
// into 64 registers per lane, so the products read no LDS.  Each sub-step runs one
// 32-row block at a time (16 live accumulators), which leaves room for the table in
// registers at four waves per SIMD.  Narrow primes, Montgomery epilogue; other
// splits and forms use the kernels above.  (Measured alternatives, all bit-exact
// and slower or level: the table read from LDS per product, the next row's operands
// loaded a block ahead, all four 32-row blocks of a sub-step at once, three waves
// per SIMD with 4-wave workgroups, two waves per SIMD.)
constexpr int kP32Waves = 8;                     // waves (= rows) per block
constexpr int kP32Zp = 36;                       // Z line pitch (words): 16-byte aligned rows
constexpr int kP32Xp = 33;                       // output staging pitch (words)
constexpr int kP32SliceWords = 32 * kP32Zp;      // per-wave LDS slice

__device__ __forceinline__ void wave_lds_sync() {
  // LDS written by other lanes of this wave becomes visible to its later reads
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);            // lgkmcnt(0)
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Where wave `wave`'s row of block b lives, and its prime's tables.
struct RowLoc {
  const int8_t* tab;        // 128 x 128 sub-step table (fragment order)
  const uint32_t* tw1;      // first-epilogue twiddle pairs (T3 [m][c2] or IT3 [c2][m])
  const uint32_t* tw2;      // inverse: step-2 twiddle pairs of this row, [C][2]
  const uint32_t* in;       // the row (1024 residues)
  uint32_t* out;
  uint32_t q, qinv;
};

// One launch of the uniform form: njobs limbs (one prime each) at offsets from
// common bases, npoly polynomials `stride` apart, R / 8 blocks per polynomial;
// block b is (job, row block, polynomial) with the polynomial fastest.
struct P32Uniform {
  static constexpr bool kTail = false, kList = false;
  const RowsJob* jobs;
  const uint32_t* in;
  uint32_t* out;
  uint64_t stride;
  int npoly, rb_log;
  __device__ __forceinline__ RowLoc locate(int b, int wave) {
    const int per_job = npoly << rb_log;
    const int j = __builtin_amdgcn_readfirstlane(b / per_job);
    const int rem = b - j * per_job;
    const int rb = __builtin_amdgcn_readfirstlane(rem / npoly);
    const int poly = rem - rb * npoly, row = rb * kP32Waves + wave;
    const RowsJob& jb = jobs[j];
    const uint64_t off = jb.off + (uint64_t)poly * stride + (uint64_t)row * 1024;
    return RowLoc{jb.tab1, jb.tw1, jb.tw2 ? jb.tw2 + (uint64_t)row * 2048 : nullptr, in + off, out + off,
                  jb.q, jb.qinv};
  }
};

// The batch runtime's form: a task list (each task one limb with its own buffers,
// polynomial count and R), block b in the task whose first_block is the last one
// not above b (within a task: row block, then polynomial, the polynomial fastest).
// Blocks of a workgroup are contiguous, so the task index only moves forward.
struct P32List {
  static constexpr bool kTail = false, kList = true;
  const RowsTask* tasks;
  int ntasks;
  int t = 0;                // current task (wave-uniform)
  __device__ __forceinline__ void seek(int b) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].first_block <= b) lo = mid;
      else hi = mid - 1;
    }
    t = __builtin_amdgcn_readfirstlane(lo);
  }
  __device__ __forceinline__ RowLoc locate(int b, int wave) {
    while (t + 1 < ntasks && tasks[t + 1].first_block <= b) ++t;
    t = __builtin_amdgcn_readfirstlane(t);
    const RowsTask& k = tasks[t];
    const int local = b - k.first_block;
    const int rb = __builtin_amdgcn_readfirstlane(local / k.npoly);
    const int poly = __builtin_amdgcn_readfirstlane(local - rb * k.npoly), row = rb * kP32Waves + wave;
    const uint64_t off = (uint64_t)poly * k.stride + (uint64_t)row * 1024;
    return RowLoc{k.tab, k.tw1, k.tw2 ? k.tw2 + (uint64_t)row * 2048 : nullptr, k.in + off, k.out + off, k.q, k.qinv};
  }
};

// The 16 fragments (K step ks, 32-row block mb; 1 KB each) of the sub-step table in
// registers; fragment order ((ks / 2) * 4 + mb) * 2 + ks % 2.
struct P32Tab {
  v4i f[16];
  __device__ __forceinline__ void load(const int8_t* lds, int lane) {
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = *reinterpret_cast<const v4i*>(lds + i * 1024 + lane * 16);
  }
  __device__ __forceinline__ v4i get(int ks, int mb) const { return f[((ks >> 1) * 4 + mb) * 2 + (ks & 1)]; }
};

// The same fragments read from the LDS copy at each product (frees the 64 registers).
struct P32LdsTab {
  const int8_t* lds;
  int lane;
  __device__ __forceinline__ v4i get(int ks, int mb) const {
    return *reinterpret_cast<const v4i*>(lds + (((ks >> 1) * 4 + mb) * 2 + (ks & 1)) * 1024 + lane * 16);
  }
};

// One 32-row block mb of a sub-step: the four K steps of the wave's 32 columns.
template <class TAB>
__device__ __forceinline__ v16i p32_block_mb(const TAB& tab, const v4i (&b)[4], int mb) {
  v16i acc = v16i{};
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(tab.get(ks, mb), b[ks], acc, 0, 0, 0);
  return acc;
}

// Stage a prime's table and first twiddles when the block's prime changes
// (workgroup-uniform: every wave of a block has the same prime).
__device__ __forceinline__ void p32_stage(const RowLoc& L, const int8_t*& cur_tab, int8_t* tabs, uint32_t* tws,
                                          P32Tab& tab, int lane) {
  if (L.tab == cur_tab) return;
  __syncthreads();
  stage<64 * kP32Waves>(tabs, L.tab, 16 * 32 * 32);
  stage<64 * kP32Waves>(tws, L.tw1, 8 * 1024);
  __syncthreads();
  tab.load(tabs, lane);
  cur_tab = L.tab;
}

// Write the staged output lines of a row (element e = line * 32 + c) with 16-byte stores.
__device__ __forceinline__ void p32_write_row(const uint32_t* zw, uint32_t* out, int lane) {
  const __amdgpu_buffer_rsrc_t ro = rows_rsrc(out, 1024 * 4);
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int e = (lane + it * 64) * 4;
    const uint32_t* src = &zw[(e >> 5) * kP32Xp + (e & 31)];
    __builtin_amdgcn_raw_buffer_store_b128(v4u{src[0], src[1], src[2], src[3]}, ro, e * 4, 0, 0);
  }
}

// Tail write of one staged output row y: out = base + (acc - y) * Pinv (base may be
// null), 16-byte loads and stores of the row.
__device__ __forceinline__ void p32_tail_row(const uint32_t* zw, const uint32_t* acc, const uint32_t* base,
                                             uint32_t* out, const TailConst c, int lane) {
  const __amdgpu_buffer_rsrc_t ra = rows_rsrc(acc, 1024 * 4);
  const __amdgpu_buffer_rsrc_t ro = rows_rsrc(out, 1024 * 4);
  // without a base the descriptor holds no records: its loads read zero
  const __amdgpu_buffer_rsrc_t rbase = rows_rsrc(base ? base : out, base ? 1024 * 4 : 0);
  v4u a[4], bs[4];
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const uint32_t e = (uint32_t)(lane + it * 64) * 16;
    a[it] = __builtin_amdgcn_raw_buffer_load_b128(ra, e, 0, 0);
    bs[it] = __builtin_amdgcn_raw_buffer_load_b128(rbase, e, 0, 0);
  }
#pragma unroll
  for (int it = 0; it < 4; ++it) {
    const int e = (lane + it * 64) * 4;
    const uint32_t* y = &zw[(e >> 5) * kP32Xp + (e & 31)];
    v4u r;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint32_t d = a[it][k] + c.q - y[k];                       // (0, 2q)
      const uint32_t m = d * c.pinv - __umulhi(d, c.pinv_shoup) * c.q; // [0, 2q)
      const uint32_t v = (m >= c.q ? m - c.q : m) + bs[it][k];
      r[k] = v >= c.q ? v - c.q : v;
    }
    __builtin_amdgcn_raw_buffer_store_b128(r, ro, (uint32_t)e * 4, 0, 0);
  }
}

// The uniform form with the ModDown / rescale tail fused into the forward kernel's
// write: out = base + (acc - y) * Pinv for the staged output row y.
struct P32UniformTail : P32Uniform {
  static constexpr bool kTail = true;
  RowsTail t;
  __device__ __forceinline__ void write_tail(int b, int wave, const uint32_t* zw, uint32_t q, int lane) const {
    const int per_job = npoly << rb_log;
    const int j = __builtin_amdgcn_readfirstlane(b / per_job);
    const int rem = b - j * per_job;
    const int rb = __builtin_amdgcn_readfirstlane(rem / npoly);
    const int poly = rem - rb * npoly, row = rb * kP32Waves + wave;
    const uint64_t o = jobs[j].off + (uint64_t)row * 1024;
    const bool use_base = t.base != nullptr && (!t.base_only_even || (poly & 1) == 0);
    p32_tail_row(zw, t.acc + poly * t.acc_stride + o, use_base ? t.base + poly * t.out_stride + o : nullptr,
                 t.out + poly * t.out_stride + o, t.tc[j], lane);
  }
};

// The task-list form of the fused tail (batch runtime): each task is one limb of
// the NTT of z with its own tail buffers.
struct P32ListTail {
  static constexpr bool kTail = true, kList = true;
  const RowsTailTask* tasks;
  int ntasks;
  int t = 0;
  __device__ __forceinline__ void seek(int b) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].r.first_block <= b) lo = mid;
      else hi = mid - 1;
    }
    t = __builtin_amdgcn_readfirstlane(lo);
  }
  __device__ __forceinline__ RowLoc locate(int b, int wave) {
    while (t + 1 < ntasks && tasks[t + 1].r.first_block <= b) ++t;
    t = __builtin_amdgcn_readfirstlane(t);
    const RowsTask& k = tasks[t].r;
    const int local = b - k.first_block;
    const int rb = __builtin_amdgcn_readfirstlane(local / k.npoly);
    const int poly = __builtin_amdgcn_readfirstlane(local - rb * k.npoly), row = rb * kP32Waves + wave;
    const uint64_t off = (uint64_t)poly * k.stride + (uint64_t)row * 1024;
    return RowLoc{k.tab, k.tw1, nullptr, k.in + off, nullptr, k.q, k.qinv};
  }
  __device__ __forceinline__ void write_tail(int b, int wave, const uint32_t* zw, uint32_t q, int lane) const {
    const RowsTailTask& k = tasks[t];
    const int local = b - k.r.first_block;
    const int rb = __builtin_amdgcn_readfirstlane(local / k.r.npoly);
    const int poly = __builtin_amdgcn_readfirstlane(local - rb * k.r.npoly), row = rb * kP32Waves + wave;
    const uint64_t o = (uint64_t)row * 1024;
    const bool use_base = k.base != nullptr && (!k.base_only_even || (poly & 1) == 0);
    p32_tail_row(zw, k.acc + poly * k.acc_stride + o, use_base ? k.base + poly * k.out_stride + o : nullptr,
                 k.out + poly * k.out_stride + o, TailConst{k.r.q, k.pinv, k.pinv_shoup, 0}, lane);
  }
};

__device__ __forceinline__ void p32_range(int nblocks, int& b0, int& b1) {
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
  const int lo = (int)((int64_t)nblocks * xcd / 8), hi = (int)((int64_t)nblocks * (xcd + 1) / 8);
  b0 = lo + (int)((int64_t)(hi - lo) * local / per_xcd);
  b1 = lo + (int)((int64_t)(hi - lo) * (local + 1) / per_xcd);
}

// Forward transform of one row (the wave's): sub-step 1 (TB over c1, columns (row, c2))
// reads the chunk-packed row-side output at `in`, applies T3 and packs Z lines [m][c2];
// sub-step 2 (TC over c2, columns (row, m)) finishes the row in natural residues, staged
// in the wave's LDS slice (element e at zw[(e >> 5) * kP32Xp + (e & 31)]).
template <class TAB>
__device__ __forceinline__ void p32_fwd_row(const uint32_t* in, const TAB& tab, const uint32_t* tws, uint32_t* zw,
                                            uint32_t q, uint32_t qinv, int lane) {
  const int h = lane >> 5, c2 = lane & 31;
  // operands: chunk-packed words of c1 = 8 ks + 4 h + i at column c2
  v4i cur[4];
  {
    const __amdgpu_buffer_rsrc_t r = rows_rsrc(in, 1024 * 4);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const uint32_t o = (uint32_t)((8 * ks + 4 * h) * 32 + c2) * 4;
      cur[ks] = v4i{(int)__builtin_amdgcn_raw_buffer_load_b32(r, o, 0, 0),
                    (int)__builtin_amdgcn_raw_buffer_load_b32(r, o, 128, 0),
                    (int)__builtin_amdgcn_raw_buffer_load_b32(r, o, 256, 0),
                    (int)__builtin_amdgcn_raw_buffer_load_b32(r, o, 384, 0)};
    }
  }
  // sub-step 1: out m = mb * 8 + 2 j + h at column c2, T3 twiddle, packed into Z
  {
    const uint32_t* twl = &tws[(h * 32 + c2) * 2];
    uint32_t* zl = &zw[h * kP32Zp + c2];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const v16i acc = p32_block_mb(tab, cur, mb);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int m0 = mb * 8 + 2 * jj;
        const v2u w = *reinterpret_cast<const v2u*>(&twl[m0 * 64]);
        zl[m0 * kP32Zp] = pack7(shoup_tw(merge_redc(acc, jj, q, qinv), w, q));
      }
    }
  }
  wave_lds_sync();
  // sub-step 2: column m = lane % 32 reads its Z line (16 contiguous bytes per K step)
  v4i zb[4];
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) zb[ks] = *reinterpret_cast<const v4i*>(&zw[c2 * kP32Zp + 8 * ks + 4 * h]);
  wave_lds_sync();
  {
    uint32_t* xl = &zw[c2 * kP32Xp + h];          // output c2' = mb * 8 + 2 j + h of line m = c2
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const v16i acc = p32_block_mb(tab, zb, mb);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const uint32_t r = merge_redc(acc, jj, q, qinv);
        xl[mb * 8 + 2 * jj] = r >= q ? r - q : r;
      }
    }
  }
  wave_lds_sync();
}

template <class SRC>
__global__ void __launch_bounds__(64 * kP32Waves, 4) ntt_rows32_fwd_kernel(SRC src, int nblocks) {
  __shared__ __attribute__((aligned(16))) int8_t tabs[16 * 32 * 32];
  __shared__ __attribute__((aligned(16))) uint32_t tws[2 * 1024];
  __shared__ __attribute__((aligned(16))) uint32_t zs[kP32Waves * kP32SliceWords];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int b0, b1;
  p32_range(nblocks, b0, b1);
  if constexpr (SRC::kList) src.seek(b0);
  uint32_t* zw = zs + wave * kP32SliceWords;
  P32Tab tab;
  const int8_t* cur_tab = nullptr;
  for (int b = b0; b < b1; ++b) {
    const RowLoc L = src.locate(b, wave);
    p32_stage(L, cur_tab, tabs, tws, tab, lane);
    p32_fwd_row(L.in, tab, tws, zw, L.q, L.qinv, lane);
    if constexpr (SRC::kTail)
      src.write_tail(b, wave, zw, L.q, lane);
    else
      p32_write_row(zw, L.out, lane);
    wave_lds_sync();       // staging reads done before the next block's Z writes
  }
}

// Montgomery product x' k 2^-32 mod q of a Montgomery-form residue x' = x 2^32 mod q and a
// plain one: x k in (0, 2q) (x' k < q 2^32, so one REDC step).
__device__ __forceinline__ uint32_t ip_mont(uint32_t xm, uint32_t k, const IpLimb& md) {
  const uint32_t lo = xm * k, hi = __umulhi(xm, k);
  return hi + md.q - __umulhi(lo * md.qinv, md.q);
}

// Barrett product of two runtime residues (Alg. barrett): k = bit length of q,
// m = floor(2^(2k) / q); the quotient estimate ((z >> (k - 1)) m) >> (k + 1) is short
// by at most 2, so two conditional subtractions finish.
__device__ __forceinline__ uint32_t ip_mulmod(uint32_t a, uint32_t b, const IpLimb& md) {
  const uint64_t z = (uint64_t)a * b;
  const uint32_t zh = (uint32_t)(z >> (md.bar_k - 1));
  const uint32_t t = (uint32_t)(((uint64_t)zh * md.bar_m) >> (md.bar_k + 1));
  uint32_t r = (uint32_t)z - t * md.q;
  if (r >= md.q) r -= md.q;
  if (r >= md.q) r -= md.q;
  return r;
}

// ModUp NTT fused with the key-switch inner product: the (row, ciphertext) pairs of a
// target limb t, the ciphertext fastest, are dealt eight to a block, one per wave, so
// with eight or more ciphertexts the waves of a block read the same key rows together
// (one fetch from HBM; a block per ciphertext re-fetched them about four times, once
// the other workgroups' streams had pushed them out of L2).  Each wave, for every active
// digit j, either transforms its row of limb (j, t) of the packed row-side output (t
// outside digit j) or reads that row of the NTT-form input (t in digit j), and
// accumulates its products with the two key rows of (j, t) in registers; the two
// accumulator rows are written once.  The blocks take the target limbs in the order of
// the limb list, which spreads the special limbs (three transforms each, against two and
// a load for a Q limb) evenly, so that each XCD's contiguous eighth of the blocks holds
// the same mix of work.  The transforms run with T3 * 2^32 as their first
// twiddle, so their outputs come out times 2^32 and each key product is one REDC step
// (four multiplies) instead of a Barrett product (five, and two 64-bit shifts); the key
// products are most of this kernel's vector work.  Every transform of a block uses t's
// prime, so the row tables are staged once per run of blocks with the same t.
// Block sources of the fused kernel: one RowsIp, or a task list of them (batch
// runtime; blocks of a task contiguous, tasks in first_block order).
struct IpUniform {
  RowsIp p;
  __device__ __forceinline__ void seek(int) {}
  __device__ __forceinline__ const RowsIp& at(int b, int& local) {
    local = b;
    return p;
  }
};
struct IpList {
  const IpTask* tasks;
  int ntasks;
  int t = 0;
  __device__ __forceinline__ void seek(int b) {
    int lo = 0, hi = ntasks - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (tasks[mid].first_block <= b) lo = mid;
      else hi = mid - 1;
    }
    t = __builtin_amdgcn_readfirstlane(lo);
  }
  __device__ __forceinline__ const RowsIp& at(int b, int& local) {
    while (t + 1 < ntasks && tasks[t + 1].first_block <= b) ++t;
    t = __builtin_amdgcn_readfirstlane(t);
    local = b - tasks[t].first_block;
    return tasks[t].p;
  }
};

template <class SRC>
__global__ void __launch_bounds__(64 * kP32Waves, 4) ntt_rows32_ip_kernel(SRC src, int nblocks) {
  __shared__ __attribute__((aligned(16))) int8_t tabs[16 * 32 * 32];
  __shared__ __attribute__((aligned(16))) uint32_t tws[2 * 1024];
  __shared__ __attribute__((aligned(16))) uint32_t zs[kP32Waves * kP32SliceWords];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int b0, b1;
  p32_range(nblocks, b0, b1);
  if (b0 < b1) src.seek(b0);
  uint32_t* zw = zs + wave * kP32SliceWords;
  const P32LdsTab tab{tabs, lane};
  const int8_t* cur_tab = nullptr;
  for (int b = b0; b < b1; ++b) {
    int local;
    const RowsIp& p = src.at(b, local);
    const uint64_t N = 1024ull << p.rb_log << 3;
    const int per_t = p.B << p.rb_log;
    const int tp = __builtin_amdgcn_readfirstlane(local / per_t);    // position in the limb list
    // the wave's (row, ciphertext) pair, the ciphertext fastest
    const int pair = (local - tp * per_t) * kP32Waves + wave;
    const int row = __builtin_amdgcn_readfirstlane(pair / p.B);
    const int ct = __builtin_amdgcn_readfirstlane(pair - row * p.B);
    const IpLimb md = p.limbs[tp];
    // the limb index and its digit drive the row addresses and branches: wave-uniform
    const int t = __builtin_amdgcn_readfirstlane(md.limb), own = __builtin_amdgcn_readfirstlane(md.own);
    if (md.tab != cur_tab) {
      // t's table and first twiddles into LDS (workgroup-uniform: a block has one t)
      __syncthreads();
      stage<64 * kP32Waves>(tabs, md.tab, 16 * 32 * 32);
      stage<64 * kP32Waves>(tws, md.tw1, 8 * 1024);
      __syncthreads();
      cur_tab = md.tab;
    }
    const uint64_t roff = (uint64_t)t * N + (uint64_t)row * 1024;
    v4u s0[4], s1[4];
#pragma unroll
    for (int it = 0; it < 4; ++it) s0[it] = s1[it] = v4u{0, 0, 0, 0};
    for (int j = 0; j < p.ndig; ++j) {
      v4u v[4];
      if (j == own) {
        const __amdgpu_buffer_rsrc_t rd = rows_rsrc(p.d + (uint64_t)ct * p.L * N + roff, 1024 * 4);
#pragma unroll
        for (int it = 0; it < 4; ++it) v[it] = __builtin_amdgcn_raw_buffer_load_b128(rd, (lane + it * 64) * 16, 0, 0);
      } else {
        p32_fwd_row(p.tmp + (uint64_t)ct * p.ext_stride + (uint64_t)j * p.LK * N + roff, tab, tws, zw, md.q, md.qinv,
                    lane);
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          const int e = (lane + it * 64) * 4;
          const uint32_t* y = &zw[(e >> 5) * kP32Xp + (e & 31)];
          v[it] = v4u{y[0], y[1], y[2], y[3]};
        }
        wave_lds_sync();   // staging reads done before the next transform's Z writes
      }
      const uint32_t* k0 = p.key + (uint64_t)(j * 2) * p.LK * N + roff;
      const __amdgpu_buffer_rsrc_t rk0 = rows_rsrc(k0, 1024 * 4);
      const __amdgpu_buffer_rsrc_t rk1 = rows_rsrc(k0 + (uint64_t)p.LK * N, 1024 * 4);
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const uint32_t e = (uint32_t)(lane + it * 64) * 16;
        const v4u a0 = __builtin_amdgcn_raw_buffer_load_b128(rk0, e, 0, 0);
        const v4u a1 = __builtin_amdgcn_raw_buffer_load_b128(rk1, e, 0, 0);
        // accumulators in [0, 2q): the own digit's plain residues take a Barrett product
        // ([0, q)), the transforms' Montgomery-form ones a REDC step ((0, 2q))
        if (j == own) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            uint32_t x = s0[it][k] + ip_mulmod(v[it][k], a0[k], md);
            s0[it][k] = x >= 2 * md.q ? x - 2 * md.q : x;
            x = s1[it][k] + ip_mulmod(v[it][k], a1[k], md);
            s1[it][k] = x >= 2 * md.q ? x - 2 * md.q : x;
          }
        } else {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            uint32_t x = s0[it][k] + ip_mont(v[it][k], a0[k], md);
            s0[it][k] = x >= 2 * md.q ? x - 2 * md.q : x;
            x = s1[it][k] + ip_mont(v[it][k], a1[k], md);
            s1[it][k] = x >= 2 * md.q ? x - 2 * md.q : x;
          }
        }
      }
    }
    uint32_t* o0 = p.acc + (uint64_t)ct * 2 * p.LK * N + roff;
    const __amdgpu_buffer_rsrc_t ro0 = rows_rsrc(o0, 1024 * 4);
    const __amdgpu_buffer_rsrc_t ro1 = rows_rsrc(o0 + (uint64_t)p.LK * N, 1024 * 4);
#pragma unroll
    for (int it = 0; it < 4; ++it) {
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s0[it][k] = s0[it][k] >= md.q ? s0[it][k] - md.q : s0[it][k];
        s1[it][k] = s1[it][k] >= md.q ? s1[it][k] - md.q : s1[it][k];
      }
      __builtin_amdgcn_raw_buffer_store_b128(s0[it], ro0, (lane + it * 64) * 16, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b128(s1[it], ro1, (lane + it * 64) * 16, 0, 0);
    }
  }
}

// Inverse: sub-step 1 (ITC over c2', columns (row, m)) reads plain residues, applies
// IT3 and packs Z lines [c2][m]; sub-step 2 (ITB over m, columns (row, c2)) applies the
// inverse step-2 twiddle of the outer split, read per 32-row block before its products,
// and stages packed output lines c1.
template <class SRC>
__global__ void __launch_bounds__(64 * kP32Waves, 4) ntt_rows32_inv_kernel(SRC src, int nblocks) {
  __shared__ __attribute__((aligned(16))) int8_t tabs[16 * 32 * 32];
  __shared__ __attribute__((aligned(16))) uint32_t tws[2 * 1024];
  __shared__ __attribute__((aligned(16))) uint32_t zs[kP32Waves * kP32SliceWords];
  const int lane = threadIdx.x & 63, h = lane >> 5, cl = lane & 31;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int b0, b1;
  p32_range(nblocks, b0, b1);
  if constexpr (SRC::kList) src.seek(b0);
  uint32_t* zw = zs + wave * kP32SliceWords;
  P32Tab tab;
  const int8_t* cur_tab = nullptr;
  for (int b = b0; b < b1; ++b) {
    const RowLoc L = src.locate(b, wave);
    p32_stage(L, cur_tab, tabs, tws, tab, lane);
    const uint32_t q = L.q, qinv = L.qinv;
    const __amdgpu_buffer_rsrc_t tw2 = rows_rsrc(L.tw2, 8 * 1024);
    // operands: residues c2' = 8 ks + 4 h + i of line m = cl, packed
    v4i cur[4];
    {
      const __amdgpu_buffer_rsrc_t r = rows_rsrc(L.in, 1024 * 4);
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const v4u x = __builtin_amdgcn_raw_buffer_load_b128(r, (uint32_t)(cl * 32 + 8 * ks + 4 * h) * 4, 0, 0);
        cur[ks] = v4i{(int)pack7(x.x), (int)pack7(x.y), (int)pack7(x.z), (int)pack7(x.w)};
      }
    }
    // sub-step 1: out c2 = mb * 8 + 2 j + h at column m = cl, IT3 pairs [c2][m], Z lines [c2][m]
    {
      const uint32_t* twl = &tws[(h * 32 + cl) * 2];
      uint32_t* zl = &zw[h * kP32Zp + cl];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const v16i acc = p32_block_mb(tab, cur, mb);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int c0 = mb * 8 + 2 * jj;
          const v2u w = *reinterpret_cast<const v2u*>(&twl[c0 * 64]);
          zl[c0 * kP32Zp] = pack7(shoup_tw(merge_redc(acc, jj, q, qinv), w, q));
        }
      }
    }
    wave_lds_sync();
    // sub-step 2: column c2 = cl reads its Z line
    v4i zb[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) zb[ks] = *reinterpret_cast<const v4i*>(&zw[cl * kP32Zp + 8 * ks + 4 * h]);
    wave_lds_sync();
    {
      uint32_t* xl = &zw[h * kP32Xp + cl];          // output c1 = mb * 8 + 2 j + h at position c2 = cl
      const uint32_t tw_lane = (uint32_t)(h * 32 + cl) * 8;
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        v2u w2[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          w2[jj] = __builtin_amdgcn_raw_buffer_load_b64(tw2, tw_lane, (mb * 8 + 2 * jj) * 32 * 8, 0);
        const v16i acc = p32_block_mb(tab, zb, mb);
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int c0 = mb * 8 + 2 * jj;
          xl[c0 * kP32Xp] = pack7(shoup_tw(merge_redc(acc, jj, q, qinv), w2[jj], q));
        }
      }
    }
    wave_lds_sync();
    p32_write_row(zw, L.out, lane);
    wave_lds_sync();
  }
}

// Workgroups that fit the device at four waves per SIMD (two per CU), at most one
// per block, rounded to a multiple of 8 (p32_range; surplus workgroups get no block).
int p32_grid(int64_t nblocks) {
  const int64_t fit = std::max<int64_t>(8, 2 * (int64_t)cu_count() / 8 * 8);
  return (int)std::min<int64_t>((nblocks + 7) / 8 * 8, fit);
}

template <class SRC>
hipError_t p32_launch(const SRC& src, int64_t nblocks, bool inverse, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const int grid = p32_grid(nblocks);
  if (inverse)
    launch_kernel((ntt_rows32_inv_kernel<SRC>), dim3(grid), dim3(64 * kP32Waves), 0, s, src, (int)nblocks);
  else
    launch_kernel((ntt_rows32_fwd_kernel<SRC>), dim3(grid), dim3(64 * kP32Waves), 0, s, src, (int)nblocks);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt_rows(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                           int npoly, int log_r, int log_c1, int log_c2, bool inverse, int red, bool wide,
                           hipStream_t s) {
  if (red != 0 && red != 1) return hipErrorInvalidValue;
  if (wide && red != 0) return hipErrorInvalidValue;   // the wide form has a Montgomery epilogue only
  if (njobs <= 0 || npoly <= 0) return hipSuccess;
  // per-lane offsets are 32-bit within a workgroup's 32 KB of rows
  if (stride >= (1ull << 40)) return hipErrorInvalidValue;
  if (log_c1 == 5 && log_c2 == 5 && red == 0 && !wide && log_r >= 3) {
    // persistent form: workgroups walk contiguous ranges of 8-row blocks
    const P32Uniform src{jobs, in, out, stride, npoly, log_r - 3};
    return p32_launch(src, (int64_t)njobs * npoly << (log_r - 3), inverse, s);
  }
#define CROSS_ROWS(a, b)                                                                                    \
  if (log_c1 == a && log_c2 == b)                                                                         \
    return red    ? rows_cfg<(1 << a), (1 << b), 1>(jobs, njobs, in, out, stride, npoly, log_r, inverse, s)      \
           : wide ? rows_cfg<(1 << a), (1 << b), 0, true>(jobs, njobs, in, out, stride, npoly, log_r, inverse, s) \
                  : rows_cfg<(1 << a), (1 << b), 0>(jobs, njobs, in, out, stride, npoly, log_r, inverse, s);
  CROSS_ROWS(4, 4)
  CROSS_ROWS(4, 5)
  CROSS_ROWS(5, 4)
  CROSS_ROWS(5, 5)
  CROSS_ROWS(5, 6)
  CROSS_ROWS(6, 5)
  CROSS_ROWS(6, 6)
  CROSS_ROWS(4, 6)
  CROSS_ROWS(6, 4)
#undef CROSS_ROWS
  return hipErrorInvalidValue;
}

hipError_t launch_ntt_rows_tail(const RowsJob* jobs, int njobs, const uint32_t* in, uint64_t stride, int npoly,
                                int log_r, const RowsTail& tail, hipStream_t s) {
  if (njobs <= 0 || npoly <= 0) return hipSuccess;
  if (log_r < 3 || stride >= (1ull << 40) || !tail.acc || !tail.out || !tail.tc) return hipErrorInvalidValue;
  P32UniformTail src;
  src.jobs = jobs;
  src.in = in;
  src.out = tail.out;       // unused: the tail writes every row
  src.stride = stride;
  src.npoly = npoly;
  src.rb_log = log_r - 3;
  src.t = tail;
  const int64_t nblocks = (int64_t)njobs * npoly << (log_r - 3);
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  launch_kernel((ntt_rows32_fwd_kernel<P32UniformTail>), dim3(p32_grid(nblocks)), dim3(64 * kP32Waves), 0, s, src,
                (int)nblocks);
  return hipGetLastError();
}

hipError_t launch_ntt_rows_ip(const RowsIp& p, hipStream_t s) {
  if (p.B <= 0 || p.LK <= 0 || p.ndig <= 0) return hipSuccess;
  if (p.rb_log < 0 || !p.limbs || !p.tmp || !p.d || !p.key || !p.acc) return hipErrorInvalidValue;
  const int64_t nblocks = (int64_t)p.LK * p.B << p.rb_log;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const IpUniform src{p};
  launch_kernel((ntt_rows32_ip_kernel<IpUniform>), dim3(p32_grid(nblocks)), dim3(64 * kP32Waves), 0, s, src,
                (int)nblocks);
  return hipGetLastError();
}

hipError_t launch_ntt_rows_ip_list(const IpTask* tasks, int ntasks, int64_t nblocks, hipStream_t s) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const IpList src{tasks, ntasks, 0};
  launch_kernel((ntt_rows32_ip_kernel<IpList>), dim3(p32_grid(nblocks)), dim3(64 * kP32Waves), 0, s, src,
                (int)nblocks);
  return hipGetLastError();
}

hipError_t launch_ntt_rows_tail_list(const RowsTailTask* tasks, int ntasks, int64_t nblocks, hipStream_t s) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const P32ListTail src{tasks, ntasks, 0};
  launch_kernel((ntt_rows32_fwd_kernel<P32ListTail>), dim3(p32_grid(nblocks)), dim3(64 * kP32Waves), 0, s, src,
                (int)nblocks);
  return hipGetLastError();
}

bool rows_tail_supported(int log_n, int log_r, int log_c1) {
  return log_c1 == 5 && log_n - log_r - log_c1 == 5 && log_r >= 3;
}

hipError_t launch_ntt_rows_list(const RowsTask* tasks, int ntasks, int64_t nblocks, bool inverse, hipStream_t s) {
  if (ntasks <= 0 || nblocks <= 0) return hipSuccess;
  const P32List src{tasks, ntasks, 0};
  return p32_launch(src, nblocks, inverse, s);
}

int rows_list_rows_per_block() { return kP32Waves; }

bool rows_split_supported(int log_n, int log_r, int log_c1) {
  const int log_c2 = log_n - log_r - log_c1;
  if (log_c1 < 4 || log_c1 > 6 || log_c2 < 4 || log_c2 > 6) return false;
  int log_w = 0;
  while ((1 << log_w) < kRowsWaves) ++log_w;
  const int log_br = log_w + 10 - (log_c1 + log_c2);   // rows per workgroup: kRowsWaves * 1024 / C
  return log_br >= 0 && log_r >= log_br && log_r >= 4;
}

}  // namespace cross
