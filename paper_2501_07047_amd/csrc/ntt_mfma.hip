// BAT int8-MFMA steps of the layout-invariant 3-step negacyclic NTT
// (arXiv 2501.07047, Sec. BAT "Accelerating core HE kernels", Alg. bat_deployment;
// Sec. MAT "Applying MAT to 4-step NTT").
//
// One launch runs one step for many limbs.  Each step is a modular matrix
// product with a pre-known twiddle matrix, carried out as an exact int8 GEMM:
// residues (< 2^28) are split into four 7-bit chunks (RuntimeCompileRight), the
// pre-known matrix was expanded on the host into 4x4 chunk blocks
// (OfflineCompileLeft / DirectScalarBAT, with the Montgomery factor 2^32 folded
// in), so every int32 partial sum is exact.  The epilogue merges the four
// chunk partial sums of one output (ChunkMerge), reduces with Montgomery REDC
// (Alg. montgomery_reduction, result in [0, 2q)), optionally multiplies by the
// step-2 twiddle, and finishes with one conditional subtraction (the final
// reduction the paper assigns to Barrett; one subtraction suffices here).
//
// GEMM view (M x K times K x Ncols):
//   A[m][k]: pre-known, m = 4*u + i (output u, output chunk i), k = 4*x + j (input x, chunk j)
//   B[k][n]: chunk j of data element x of column n;  n = poly * V + v
// MFMA v_mfma_i32_16x16x64_i8: lane l holds rows 4*(l/16) .. +3 of column l%16 of
// its 16x16 output block, i.e. all four chunk rows of one output: the merge is
// entirely in-register.
//
// Rows of the output block order chunks fastest (m = 4u + i) for exactly that reason.
#include "kernels.h"

namespace cross {

typedef int v4i __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 64;            // K per MFMA step

__device__ __forceinline__ uint32_t pack_chunks(uint32_t x) {
  // four 7-bit chunks of x (< 2^28) in the four bytes of one word
  return (x & 0x7fu) | ((x << 1) & 0x7f00u) | ((x << 2) & 0x7f0000u) | ((x << 3) & 0x7f000000u);
}

__device__ __forceinline__ uint32_t redc(uint64_t z, uint32_t q, uint32_t qinv) {
  // z < q * 2^32  ->  z * 2^-32 mod q in (0, 2q)
  uint32_t t = (uint32_t)z * qinv;
  uint32_t u = __umulhi(t, q);
  return (uint32_t)(z >> 32) + q - u;
}

// One BM x BN output tile of one step (all of K).  Shared by the uniform
// launch (one limb list of one shape) and the work-list launch (mixed shapes).
struct TileArgs {
  const int8_t* table;
  const uint32_t* tw;
  const uint32_t* src;
  uint32_t* dst;
  uint64_t src_stride, dst_stride;
  uint32_t q, qinv;
  int npoly, log_r, log_c;
  int m0, n0;
};

// LDS holds two stages of the A tile (BM/16 fragments) and the B tile (BN/16
// fragments).  A fragment is the 1 KB operand of one 16x16x64 MFMA in lane
// order (lane l: row l%16, K bytes 16*(l/16) .. +15).  The tables are stored in
// the same order in global memory, so staging is contiguous 16-byte copies and
// every LDS access -- staging writes and MFMA operand reads -- is a lane-linear
// 16-byte access, free of bank conflicts.
//
// Pipeline over 64-deep K steps with one barrier per step: step k+1 is written
// to the idle LDS stage from registers while step k is multiplied and step
// k+2 is loaded from global memory.  Plain residues are cut into 7-bit chunks
// on the way into LDS; packed data (the intermediate) is copied as is.
template <int WM, int WN, int MB, int NB, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW>
__device__ __forceinline__ void gemm_tile(const TileArgs& t, int8_t* lds_a, int8_t* lds_b) {
  constexpr int NW = WM * WN;
  constexpr int NT = NW * 64;
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  constexpr int FA = BM / 16, FB = BN / 16;          // fragments per stage
  constexpr int STAGE_A = FA * 1024, STAGE_B = FB * 1024;
  constexpr int A_PIECES = FA * 64 / NT;             // 16-byte table pieces per thread
  constexpr int B_PIECES = FB * 64 / NT;             // 16-byte data pieces per thread (4 inputs x 1 column)
  static_assert(A_PIECES >= 1 && FA * 64 % NT == 0 && B_PIECES >= 1 && FB * 64 % NT == 0, "tile split");

  const int R = 1 << t.log_r, C = 1 << t.log_c;
  const int U = RIGHT ? C : R;          // outputs per column (and inputs per column)
  const int V = RIGHT ? R : C;          // columns per polynomial
  const int log_v = RIGHT ? t.log_r : t.log_c;   // V is a power of two: shifts, not divisions
  const int M = 4 * U, K = 4 * U;
  const int ncols = t.npoly * V;
  const int m0 = t.m0, n0 = t.n0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  v4i acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  // Element (input x, column v) of one polynomial:
  //   plain, row side   : x*C + v        plain, column side  : v*C + x
  //   packed, row side  : v*R + x (the inverse intermediate is stored transposed)
  //   packed, col side  : v*C + x
  // Piece p of a stage is lane p%64 of fragment p/64: column n0 + 16*(p/64) + p%16,
  // inputs 4*((p%64)/16) .. +3 of the K step.  Columns past the end read column 0;
  // their outputs are never stored.
  const uint32_t* colbase[B_PIECES];
#pragma unroll
  for (int i = 0; i < B_PIECES; ++i) {
    const int piece = tid + i * NT;
    int n = n0 + (piece >> 6) * 16 + (piece & 15);
    if (n >= ncols) n = 0;
    const int gp = ((piece & 63) >> 4) * 4;
    const int poly = n >> log_v, v = n & (V - 1);
    size_t off;
    if (IN_PACKED) off = (size_t)v * (RIGHT ? C : R) + gp;
    else off = RIGHT ? (size_t)v * C + gp : (size_t)gp * C + v;
    colbase[i] = t.src + (size_t)poly * t.src_stride + off;
  }
  const int8_t* tab = t.table + (size_t)(m0 / 16) * 1024;

  v4i ra[A_PIECES], rb[B_PIECES];
  auto load = [&](int ks) {
    const int8_t* g = tab + (size_t)ks * ((size_t)(M / 16) * 1024);
#pragma unroll
    for (int i = 0; i < A_PIECES; ++i) ra[i] = *reinterpret_cast<const v4i*>(g + (tid + i * NT) * 16);
#pragma unroll
    for (int i = 0; i < B_PIECES; ++i) {
      if (IN_PACKED || RIGHT) {
        rb[i] = *reinterpret_cast<const v4i*>(colbase[i] + ks * 16);
      } else {
        const uint32_t* p = colbase[i] + (size_t)(ks * 16) * C;
        rb[i] = v4i{(int)p[0], (int)p[C], (int)p[2 * C], (int)p[3 * C]};
      }
    }
  };
  auto store_lds = [&](int st) {
#pragma unroll
    for (int i = 0; i < A_PIECES; ++i)
      *reinterpret_cast<v4i*>(lds_a + st * STAGE_A + (tid + i * NT) * 16) = ra[i];
#pragma unroll
    for (int i = 0; i < B_PIECES; ++i) {
      v4i w = rb[i];
      if (!IN_PACKED) {
        w.x = pack_chunks(w.x);
        w.y = pack_chunks(w.y);
        w.z = pack_chunks(w.z);
        w.w = pack_chunks(w.w);
      }
      *reinterpret_cast<v4i*>(lds_b + st * STAGE_B + (tid + i * NT) * 16) = w;
    }
  };
  auto compute = [&](int st) {
    v4i fa[MB], fb[NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
      fa[a] = *reinterpret_cast<const v4i*>(lds_a + st * STAGE_A + (wm * MB + a) * 1024 + lane * 16);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      fb[b] = *reinterpret_cast<const v4i*>(lds_b + st * STAGE_B + (wn * NB + b) * 1024 + lane * 16);
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
  };

  const int nk = K / BK;
  load(0);
  store_lds(0);
  if (nk > 1) load(1);
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    if (ks + 1 < nk) store_lds((ks + 1) & 1);
    if (ks + 2 < nk) load(ks + 2);
    compute(ks & 1);
    __syncthreads();
  }

  // ---- epilogue: ChunkMerge + REDC (+ twiddle) + final subtraction ----------
  const uint32_t q = t.q, qinv = t.qinv;
  uint32_t* dst = t.dst;
  // Column side with plain output: the tile's outputs run down columns of the
  // R x C result, so they are staged in LDS (free after the last K step) as
  // [column v][row u] and written back row by row, 16 bytes per lane.
  constexpr bool STAGE_OUT = RIGHT && !OUT_PACKED;
  constexpr int BU = BM / 4;              // outputs per tile column
  constexpr int SROW = BU + 4;            // padded LDS row (words)
  uint32_t* so = reinterpret_cast<uint32_t*>(lds_a);   // lds_a spans the whole workgroup allocation
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    const int u = (m0 + wm * MB * 16 + a * 16) / 4 + (lane >> 4);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int nl = wn * NB * 16 + b * 16 + (lane & 15);
      const int n = n0 + nl;
      if (!STAGE_OUT && n >= ncols) continue;
      const int poly = n >> log_v, v = n & (V - 1);
      v4i s = acc[a][b];
      uint64_t z = (uint64_t)(uint32_t)s.x + ((uint64_t)(uint32_t)s.y << 7) +
                   ((uint64_t)(uint32_t)s.z << 14) + ((uint64_t)(uint32_t)s.w << 21);
      uint32_t r = redc(z, q, qinv);
      if (TW) {
        uint32_t w = t.tw[(size_t)u * V + v];
        r = redc((uint64_t)r * w, q, qinv);
      }
      if (r >= q) r -= q;
      if (OUT_PACKED) r = pack_chunks(r);
      if (STAGE_OUT) {
        so[nl * SROW + (u - m0 / 4)] = r;
      } else {
        // column side with packed output = the inverse intermediate, stored transposed
        size_t off = RIGHT ? (size_t)u * R + v : (size_t)u * C + v;
        dst[(size_t)poly * t.dst_stride + off] = r;
      }
    }
  }
  if (STAGE_OUT) {
    __syncthreads();
    constexpr int VEC_PER_ROW = BU / 4;
#pragma unroll
    for (int i = 0; i < BN * VEC_PER_ROW / NT; ++i) {
      const int idx = tid + i * NT;
      const int nl = idx / VEC_PER_ROW, uq = idx % VEC_PER_ROW;
      const int n = n0 + nl;
      if (n < ncols) {
        const int poly = n >> log_v, v = n & (V - 1);
        const v4i w = *reinterpret_cast<const v4i*>(so + nl * SROW + uq * 4);
        *reinterpret_cast<v4i*>(dst + (size_t)poly * t.dst_stride + (size_t)v * C + m0 / 4 + uq * 4) = w;
      }
    }
    __syncthreads();   // LDS is reused by the next tile of a work list
  }
  (void)M;
}

// LDS bytes of one workgroup: two operand stages, or the output staging tile if larger.
template <int WM, int WN, int MB, int NB, bool RIGHT, bool OUT_PACKED>
constexpr int gemm_lds_bytes() {
  constexpr int BM = WM * MB * 16, BN = WN * NB * 16;
  constexpr int ops = 2 * (BM + BN) * 64;
  constexpr int out = (RIGHT && !OUT_PACKED) ? BN * (BM / 4 + 4) * 4 : 0;
  return ops > out ? ops : out;
}

template <int WM, int WN, int MB, int NB, int OCC, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW>
__global__ void __launch_bounds__(WM * WN * 64, OCC)
bat_gemm_kernel(GemmLaunch g, int tiles_m, int tiles_n) {
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  // two LDS stages of operand fragments (A stages then B stages), reused for output staging
  __shared__ __attribute__((aligned(1024))) int8_t lds[gemm_lds_bytes<WM, WN, MB, NB, RIGHT, OUT_PACKED>()];
  int8_t* lds_a = lds;
  int8_t* lds_b = lds + 2 * BM * 64;
  // XCD-aware tile order: consecutive logical tiles land on the same XCD so a
  // job's table and columns stay in one L2.
  const int total = g.njobs * tiles_m * tiles_n;
  const int bid = blockIdx.x;
  int logical = bid;
  if ((total & 7) == 0) logical = (bid & 7) * (total >> 3) + (bid >> 3);
  const int per_job = tiles_m * tiles_n;
  const int job_id = logical / per_job;
  const int rem = logical - job_id * per_job;
  const int tn = rem / tiles_m;          // m fastest: tiles sharing columns run together
  const int tm = rem - tn * tiles_m;
  const GemmJob job = g.jobs[job_id];
  TileArgs t{job.table, job.tw, g.src + job.src_off, g.dst + job.dst_off, g.src_stride, g.dst_stride,
             job.q, job.qinv, g.npoly, g.log_r, g.log_c, tm * BM, tn * BN};
  gemm_tile<WM, WN, MB, NB, RIGHT, IN_PACKED, OUT_PACKED, TW>(t, lds_a, lds_b);
}

// Work-list form: tiles of many tasks (mixed N, R x C, primes, buffers) in one
// persistent launch.  The grid is a multiple of 8; XCD x (= blockIdx % 8) walks
// the x-th eighth of the tile list so each task's tiles share one L2.
template <int WM, int WN, int MB, int NB, int OCC, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW>
__global__ void __launch_bounds__(WM * WN * 64, OCC)
bat_gemm_list_kernel(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles) {
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  __shared__ __attribute__((aligned(1024))) int8_t lds[gemm_lds_bytes<WM, WN, MB, NB, RIGHT, OUT_PACKED>()];
  int8_t* lds_a = lds;
  int8_t* lds_b = lds + 2 * BM * 64;
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
  const int lo = (int)((long)ntiles * xcd / 8), hi = (int)((long)ntiles * (xcd + 1) / 8);
  for (int i = lo + local; i < hi; i += per_xcd) {
    const GemmTileRef r = tiles[i];
    const GemmTask k = tasks[r.task];
    TileArgs t{k.table, k.tw, k.src, k.dst, k.src_stride, k.dst_stride, k.q, k.qinv, k.npoly,
               k.log_r, k.log_c, (int)r.tm * BM, (int)r.tn * BN};
    gemm_tile<WM, WN, MB, NB, RIGHT, IN_PACKED, OUT_PACKED, TW>(t, lds_a, lds_b);
  }
}

template <int WM, int WN, int MB, int NB, int OCC, bool RIGHT, bool INP, bool OUTP, bool TW>
hipError_t launch_cfg(const GemmLaunch& g, hipStream_t s) {
  constexpr int BM = WM * MB * 16, BN = WN * NB * 16;
  const int U = RIGHT ? (1 << g.log_c) : (1 << g.log_r);
  const int V = RIGHT ? (1 << g.log_r) : (1 << g.log_c);
  const int M = 4 * U;
  if (M % BM) return hipErrorInvalidValue;
  const int tiles_m = M / BM;
  const int ncols = g.npoly * V;
  const int tiles_n = (ncols + BN - 1) / BN;
  const int grid = g.njobs * tiles_m * tiles_n;
  hipLaunchKernelGGL((bat_gemm_kernel<WM, WN, MB, NB, OCC, RIGHT, INP, OUTP, TW>), dim3(grid),
                     dim3(WM * WN * 64), 0, s, g, tiles_m, tiles_n);
  return hipGetLastError();
}

template <int WM, int WN, int MB, int NB, int OCC>
hipError_t dispatch_flags(const GemmLaunch& g, hipStream_t s) {
  // forward: LEFT(plain in, packed out, twiddle) then RIGHT(packed in, plain out)
  // inverse: RIGHT(plain in, packed out, twiddle) then LEFT(packed in, plain out)
  const bool right = g.kind == kRight;
  if (!right && !g.in_packed && g.out_packed && g.twiddle)
    return launch_cfg<WM, WN, MB, NB, OCC, false, false, true, true>(g, s);
  if (right && g.in_packed && !g.out_packed && !g.twiddle)
    return launch_cfg<WM, WN, MB, NB, OCC, true, true, false, false>(g, s);
  if (right && !g.in_packed && g.out_packed && g.twiddle)
    return launch_cfg<WM, WN, MB, NB, OCC, true, false, true, true>(g, s);
  if (!right && g.in_packed && !g.out_packed && !g.twiddle)
    return launch_cfg<WM, WN, MB, NB, OCC, false, true, false, false>(g, s);
  return hipErrorInvalidValue;
}

}  // namespace

template <bool RIGHT, bool INP, bool OUTP, bool TW>
hipError_t launch_list_cfg(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, int grid,
                           hipStream_t s) {
  // 256 x 128 tiles, 8 waves of 64 x 64, two workgroups per CU
  hipLaunchKernelGGL((bat_gemm_list_kernel<4, 2, 4, 4, 4, RIGHT, INP, OUTP, TW>), dim3(grid), dim3(512), 0, s,
                     tasks, tiles, ntiles);
  return hipGetLastError();
}

int gemm_list_tile_rows() { return 256; }
int gemm_list_tile_cols() { return 128; }

hipError_t launch_bat_gemm_list(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, int grid,
                                int kind, bool in_packed, bool out_packed, bool twiddle, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (grid <= 0 || (grid & 7)) return hipErrorInvalidValue;
  const bool right = kind == kRight;
  if (!right && !in_packed && out_packed && twiddle) return launch_list_cfg<false, false, true, true>(tasks, tiles, ntiles, grid, s);
  if (right && in_packed && !out_packed && !twiddle) return launch_list_cfg<true, true, false, false>(tasks, tiles, ntiles, grid, s);
  if (right && !in_packed && out_packed && twiddle) return launch_list_cfg<true, false, true, true>(tasks, tiles, ntiles, grid, s);
  if (!right && in_packed && !out_packed && !twiddle) return launch_list_cfg<false, true, false, false>(tasks, tiles, ntiles, grid, s);
  return hipErrorInvalidValue;
}

int resolve_gemm_tile(const GemmLaunch& g) {
  const int U = (g.kind == kRight) ? (1 << g.log_c) : (1 << g.log_r);
  const int V = (g.kind == kRight) ? (1 << g.log_r) : (1 << g.log_c);
  const int M = 4 * U;
  const long ncols = (long)g.npoly * V;
  int t = g.tile;
  if ((t == kTile256x256 || t == kTile256x128w8 || t == kTile256x256w16) && M < 256) t = kTileAuto;
  if (t == kTile256x128 && M < 256) t = kTileAuto;
  if (t == kTile128x64 && M < 128) t = kTileAuto;
  if (t != kTileAuto) return t;
  if (M >= 256) {
    // 8 waves of 64x64 (4 waves per SIMD) when the grid still covers every CU
    long grid = (long)g.njobs * (M / 256) * ((ncols + 127) / 128);
    if (grid >= 256) return kTile256x128w8;
    return kTile128x64;
  }
  if (M >= 128) return kTile128x64;
  return kTile64x64;
}

hipError_t launch_bat_gemm(const GemmLaunch& g, hipStream_t s) {
  const int U = (g.kind == kRight) ? (1 << g.log_c) : (1 << g.log_r);
  if (4 * U < 64) return hipErrorInvalidValue;
  switch (resolve_gemm_tile(g)) {
    case kTile256x256: return dispatch_flags<2, 4, 8, 4, 2>(g, s);   // 8 waves, one workgroup per CU
    case kTile256x128: return dispatch_flags<2, 2, 8, 4, 2>(g, s);   // 4 waves, two workgroups per CU
    case kTile128x64: return dispatch_flags<2, 2, 4, 2, 2>(g, s);
    case kTile256x128w8: return dispatch_flags<4, 2, 4, 4, 4>(g, s);   // 8 waves of 64x64
    case kTile256x256w16: return dispatch_flags<4, 4, 4, 4, 4>(g, s);  // 16 waves of 64x64
    default: return dispatch_flags<2, 2, 2, 2, 2>(g, s);
  }
}

}  // namespace cross
