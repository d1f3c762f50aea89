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

}  // namespace

hipError_t launch_ntt_rows(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                           int npoly, int log_r, int log_c1, int log_c2, bool inverse, int red, bool wide,
                           hipStream_t s) {
  if (red != 0 && red != 1) return hipErrorInvalidValue;
  if (wide && red != 0) return hipErrorInvalidValue;   // the wide form has a Montgomery epilogue only
  if (njobs <= 0 || npoly <= 0) return hipSuccess;
  // per-lane offsets are 32-bit within a workgroup's 32 KB of rows
  if (stride >= (1ull << 40)) return hipErrorInvalidValue;
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

bool rows_split_supported(int log_n, int log_r, int log_c1) {
  const int log_c2 = log_n - log_r - log_c1;
  if (log_c1 < 4 || log_c1 > 6 || log_c2 < 4 || log_c2 > 6) return false;
  int log_w = 0;
  while ((1 << log_w) < kRowsWaves) ++log_w;
  const int log_br = log_w + 10 - (log_c1 + log_c2);   // rows per workgroup: kRowsWaves * 1024 / C
  return log_br >= 0 && log_r >= log_br && log_r >= 4;
}

}  // namespace cross
