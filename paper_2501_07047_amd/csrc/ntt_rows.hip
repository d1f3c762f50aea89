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
// One workgroup (8 waves) takes BR = 8192 / C rows of one polynomial and prime:
// the input rows are read once from HBM, the intermediate Z lives in LDS, and
// the output rows are staged in LDS and written back as 16-byte row segments.
// Each wave owns whole 32-column blocks of a sub-step (all of its M rows), so a
// B fragment is loaded once; table fragments (16 KB per table at C1 = 32) are
// read from global memory in fragment order and stay in L1 / L2.
#include "kernels.h"

namespace cross {

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rows_rsrc(const void* base, uint64_t bytes) {
  const uint32_t n = bytes > 0xfffffff0ull ? 0xfffffff0u : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)n, 0x00020000);
}

__device__ __forceinline__ uint32_t pack7(uint32_t x) {
  return (x & 0x7fu) | ((x << 1) & 0x7f00u) | ((x << 2) & 0x7f0000u) | ((x << 3) & 0x7f000000u);
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

__device__ __forceinline__ uint32_t shoup_tw(uint32_t r, v2u tw, uint32_t q) {
  const uint32_t v = r * tw.x - __umulhi(r, tw.y) * q;      // [0, 2q)
  return v >= q ? v - q : v;
}

// acc[mb] = sum over KS K-steps of table fragment (mb, ks) x B fragment bfrag(ks):
// the M x K table (M = 32 MB) is in fragment order, fragment (mb, ks) at
// ((ks / 2) * MB + mb) * 2048 + (ks % 2) * 1024, 16 bytes per lane.
template <int MB, int KS, class BF>
__device__ __forceinline__ void block_gemm(v16i (&acc)[MB], __amdgpu_buffer_rsrc_t tab, int lane, BF bfrag) {
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = v16i{};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const v4i b = bfrag(ks);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const v4i a = (v4i)__builtin_amdgcn_raw_buffer_load_b128(
          tab, (((ks >> 1) * MB + mb) * 2048 + (ks & 1) * 1024 + lane * 16), 0, 0);
      acc[mb] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b, acc[mb], 0, 0, 0);
    }
  }
}

template <int C1, int C2>
struct RowsShape {
  static constexpr int C = C1 * C2;
  static constexpr int BR = 8192 / C;           // rows per workgroup (32 KB of residues)
  static constexpr int NT = 512, NW = 8;
  static constexpr int ZP1 = C2 + 4;            // forward Z line [row][m][.] (words, 16-byte rows)
  static constexpr int ZP2 = C1 + 4;            // inverse Z line [row][c2][.]
  static constexpr int XP = C2 + 1;             // output staging line [row][c1 or m][.]
  static constexpr int ZWORDS = BR * (C1 * ZP1 > C2 * ZP2 ? C1 * ZP1 : C2 * ZP2);
  static constexpr int XWORDS = BR * C1 * XP;
  // two workgroups per CU (4 waves per SIMD, at most 128 registers) where the
  // accumulators allow; the 64-wide splits keep more registers at one
  static constexpr int OCC = (C1 <= 32 && C2 <= 32) ? 4 : 2;
  static_assert(C1 >= 16 && C2 >= 16 && BR >= 1 && 8192 % C == 0, "row split");
};

// Locate the workgroup's rows: block = (job, poly, row block).
struct RowsPos {
  RowsJob job;
  uint64_t base;    // element offset of the first row
  int row0;         // first row index within the polynomial's R rows
};

template <int BR, int C>
__device__ __forceinline__ RowsPos rows_pos(const RowsJob* jobs, uint64_t stride, int npoly, int log_r) {
  const int per_poly = (1 << log_r) / BR;
  int b = blockIdx.x;
  const int rb = b % per_poly;
  b /= per_poly;
  const int poly = b % npoly;
  RowsPos p;
  p.job = jobs[b / npoly];
  p.row0 = rb * BR;
  p.base = p.job.off + (uint64_t)poly * stride + (uint64_t)p.row0 * C;
  return p;
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

template <int C1, int C2>
__global__ void __launch_bounds__(512, (RowsShape<C1, C2>::OCC))
ntt_rows_fwd_kernel(const RowsJob* jobs, const uint32_t* in, uint32_t* out, uint64_t stride, int npoly, int log_r) {
  using S = RowsShape<C1, C2>;
  constexpr int C = S::C, BR = S::BR;
  constexpr int MB1 = C1 / 8, MB2 = C2 / 8;                 // 32-row blocks (M = 4 C1, 4 C2)
  constexpr int NB1 = BR * C2 / 32, NB2 = BR * C1 / 32;     // 32-column blocks of the two sub-steps
  __shared__ __attribute__((aligned(16))) uint32_t zs[S::ZWORDS];
  __shared__ __attribute__((aligned(16))) uint32_t xs[S::XWORDS];
  const RowsPos P = rows_pos<BR, C>(jobs, stride, npoly, log_r);
  const __amdgpu_buffer_rsrc_t rin = rows_rsrc(in + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t rout = rows_rsrc(out + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t t1 = rows_rsrc(P.job.tab1, (uint64_t)16 * C1 * C1);
  const __amdgpu_buffer_rsrc_t t2 = rows_rsrc(P.job.tab2, (uint64_t)16 * C2 * C2);
  const __amdgpu_buffer_rsrc_t tw = rows_rsrc(P.job.tw1, (uint64_t)8 * C);
  const uint32_t q = P.job.q, qinv = P.job.qinv;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // sub-step 1: columns (row, c2), contraction over c1 (packed input, 4 words C2 apart)
  for (int cb = wave; cb < NB1; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C2, c2 = col % C2;
    v16i acc[MB1];
    block_gemm<MB1, MB1>(acc, t1, lane, [&](int ks) {
      const uint32_t o = (uint32_t)(row * C + (8 * ks + 4 * h) * C2 + c2) * 4;
      return v4i{(int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 0, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, C2 * 4, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 2 * C2 * 4, 0),
                 (int)__builtin_amdgcn_raw_buffer_load_b32(rin, o, 3 * C2 * 4, 0)};
    });
#pragma unroll
    for (int mb = 0; mb < MB1; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = mb * 8 + 2 * j + h;
        const v2u w = __builtin_amdgcn_raw_buffer_load_b64(tw, (uint32_t)(m * C2 + c2) * 8, 0, 0);
        zs[(row * C1 + m) * S::ZP1 + c2] = pack7(shoup_tw(merge_redc(acc[mb], j, q, qinv), w, q));
      }
  }
  __syncthreads();
  // sub-step 2: columns (row, m), contraction over c2 (16 contiguous bytes of a Z line)
  for (int cb = wave; cb < NB2; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C1, m = col % C1;
    v16i acc[MB2];
    block_gemm<MB2, MB2>(acc, t2, lane, [&](int ks) {
      return *reinterpret_cast<const v4i*>(&zs[(row * C1 + m) * S::ZP1 + 8 * ks + 4 * h]);
    });
#pragma unroll
    for (int mb = 0; mb < MB2; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c2p = mb * 8 + 2 * j + h;
        const uint32_t r = merge_redc(acc[mb], j, q, qinv);
        xs[(row * C1 + m) * S::XP + c2p] = r >= q ? r - q : r;
      }
  }
  __syncthreads();
  write_rows<C1, C2>(xs, rout);
}

template <int C1, int C2>
__global__ void __launch_bounds__(512, (RowsShape<C1, C2>::OCC))
ntt_rows_inv_kernel(const RowsJob* jobs, const uint32_t* in, uint32_t* out, uint64_t stride, int npoly, int log_r) {
  using S = RowsShape<C1, C2>;
  constexpr int C = S::C, BR = S::BR;
  constexpr int MB1 = C2 / 8, MB2 = C1 / 8;                 // sub-step 1 over c2', sub-step 2 over m
  constexpr int NB1 = BR * C1 / 32, NB2 = BR * C2 / 32;
  __shared__ __attribute__((aligned(16))) uint32_t zs[S::ZWORDS];
  __shared__ __attribute__((aligned(16))) uint32_t xs[S::XWORDS];
  const RowsPos P = rows_pos<BR, C>(jobs, stride, npoly, log_r);
  const __amdgpu_buffer_rsrc_t rin = rows_rsrc(in + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t rout = rows_rsrc(out + P.base, (uint64_t)BR * C * 4);
  const __amdgpu_buffer_rsrc_t t1 = rows_rsrc(P.job.tab1, (uint64_t)16 * C2 * C2);
  const __amdgpu_buffer_rsrc_t t2 = rows_rsrc(P.job.tab2, (uint64_t)16 * C1 * C1);
  const __amdgpu_buffer_rsrc_t tw = rows_rsrc(P.job.tw1, (uint64_t)8 * C);
  // inverse step-2 twiddles of this workgroup's rows: pairs [row][c]
  const __amdgpu_buffer_rsrc_t tw2 = rows_rsrc(P.job.tw2 + (uint64_t)P.row0 * C * 2, (uint64_t)8 * BR * C);
  const uint32_t q = P.job.q, qinv = P.job.qinv;
  const int lane = threadIdx.x & 63, h = lane >> 5;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // sub-step 1: columns (row, m), contraction over c2' (plain input, 16 contiguous bytes)
  for (int cb = wave; cb < NB1; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C1, m = col % C1;
    v16i acc[MB1];
    block_gemm<MB1, MB1>(acc, t1, lane, [&](int ks) {
      const v4u x = __builtin_amdgcn_raw_buffer_load_b128(rin, (uint32_t)(row * C + m * C2 + 8 * ks + 4 * h) * 4, 0, 0);
      return v4i{(int)pack7(x.x), (int)pack7(x.y), (int)pack7(x.z), (int)pack7(x.w)};
    });
#pragma unroll
    for (int mb = 0; mb < MB1; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c2 = mb * 8 + 2 * j + h;
        const v2u w = __builtin_amdgcn_raw_buffer_load_b64(tw, (uint32_t)(m * C2 + c2) * 8, 0, 0);
        zs[(row * C2 + c2) * S::ZP2 + m] = pack7(shoup_tw(merge_redc(acc[mb], j, q, qinv), w, q));
      }
  }
  __syncthreads();
  // sub-step 2: columns (row, c2), contraction over m (16 contiguous bytes of a Z line)
  for (int cb = wave; cb < NB2; cb += S::NW) {
    const int col = cb * 32 + (lane & 31);
    const int row = col / C2, c2 = col % C2;
    v16i acc[MB2];
    block_gemm<MB2, MB2>(acc, t2, lane, [&](int ks) {
      return *reinterpret_cast<const v4i*>(&zs[(row * C2 + c2) * S::ZP2 + 8 * ks + 4 * h]);
    });
#pragma unroll
    for (int mb = 0; mb < MB2; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c1 = mb * 8 + 2 * j + h;
        const v2u w = __builtin_amdgcn_raw_buffer_load_b64(tw2, (uint32_t)(row * C + c1 * C2 + c2) * 8, 0, 0);
        xs[(row * C1 + c1) * S::XP + c2] = pack7(shoup_tw(merge_redc(acc[mb], j, q, qinv), w, q));
      }
  }
  __syncthreads();
  write_rows<C1, C2>(xs, rout);
}

template <int C1, int C2>
hipError_t rows_cfg(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                    int npoly, int log_r, bool inverse, hipStream_t s) {
  using S = RowsShape<C1, C2>;
  if ((1 << log_r) % S::BR) return hipErrorInvalidValue;
  const int grid = njobs * npoly * ((1 << log_r) / S::BR);
  if (inverse)
    hipLaunchKernelGGL((ntt_rows_inv_kernel<C1, C2>), dim3(grid), dim3(S::NT), 0, s, jobs, in, out, stride, npoly,
                       log_r);
  else
    hipLaunchKernelGGL((ntt_rows_fwd_kernel<C1, C2>), dim3(grid), dim3(S::NT), 0, s, jobs, in, out, stride, npoly,
                       log_r);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ntt_rows(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                           int npoly, int log_r, int log_c1, int log_c2, bool inverse, hipStream_t s) {
  if (njobs <= 0 || npoly <= 0) return hipSuccess;
  // per-lane offsets are 32-bit within a workgroup's 32 KB of rows
  if (stride >= (1ull << 40)) return hipErrorInvalidValue;
#define CROSS_ROWS(a, b) \
  if (log_c1 == a && log_c2 == b) return rows_cfg<(1 << a), (1 << b)>(jobs, njobs, in, out, stride, npoly, log_r, inverse, s);
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
  const int log_br = 13 - (log_c1 + log_c2);      // rows per workgroup: 8192 / C
  return log_br >= 0 && log_r >= log_br && log_r >= 4;
}

}  // namespace cross
