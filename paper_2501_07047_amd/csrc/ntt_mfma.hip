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
constexpr int LDS_ROW = BK + 16;  // padded LDS row (bytes): 16 lanes x 16 B hit 64 distinct banks

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

template <int WM, int WN, int MB, int NB, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW>
__device__ __forceinline__ void gemm_tile(const TileArgs& t, int8_t* lds_a, int8_t* lds_b) {
  constexpr int NT = WM * WN * 64;
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  const int R = 1 << t.log_r, C = 1 << t.log_c;
  const int U = RIGHT ? C : R;          // outputs per column (and inputs per column)
  const int V = RIGHT ? R : C;          // columns per polynomial
  const int M = 4 * U, K = 4 * U;
  const int ncols = t.npoly * V;
  const int m0 = t.m0, n0 = t.n0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  const uint32_t* src = t.src;
  const int8_t* tab = t.table;

  v4i acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = v4i{0, 0, 0, 0};

  // ---- global -> register staging ------------------------------------------
  constexpr int A_VEC = BM * BK / 16 / NT;     // 16-byte table pieces per thread
  static_assert(A_VEC >= 1, "tile too small");
  // B staging: each thread owns BN*16 words / NT words (16 = inputs per K step)
  constexpr int B_WORDS = BN * 16 / NT;
  static_assert(B_WORDS >= 4 && (B_WORDS % 4) == 0, "B staging");
  constexpr int TPC_R = 16 / B_WORDS;           // RIGHT: threads per column
  v4i ra[A_VEC];
  uint32_t rb[B_WORDS];

  // this thread's B column and first input of a K step
  const int b_n = RIGHT ? tid / TPC_R : tid % BN;
  const int b_xs = RIGHT ? (tid % TPC_R) * B_WORDS : (tid / BN) * B_WORDS;
  const bool b_ok = (n0 + b_n) < ncols;
  const uint32_t* b_base;
  {
    const int n = b_ok ? n0 + b_n : 0;
    const int poly = n / V, v = n - poly * V;
    b_base = src + (size_t)poly * t.src_stride + (RIGHT ? (size_t)v * C + b_xs : (size_t)b_xs * C + v);
  }

  auto load = [&](int ks) {
    const int8_t* base = tab + (size_t)ks * ((size_t)M * BK) + (size_t)m0 * BK;
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) ra[i] = *reinterpret_cast<const v4i*>(base + (tid + i * NT) * 16);
    // B element (input x, column n) lives at src + poly * stride + x * sx + v * sv
    const int x0 = ks * 16;
    if (!RIGHT) {
      const uint32_t* p = b_base + (size_t)x0 * C;
#pragma unroll
      for (int w = 0; w < B_WORDS; ++w) rb[w] = b_ok ? p[(size_t)w * C] : 0u;
    } else {
      const uint32_t* p = b_base + x0;
#pragma unroll
      for (int w = 0; w < B_WORDS; w += 4) {
        v4i t = b_ok ? *reinterpret_cast<const v4i*>(p + w) : v4i{0, 0, 0, 0};
        rb[w] = t.x; rb[w + 1] = t.y; rb[w + 2] = t.z; rb[w + 3] = t.w;
      }
    }
  };

  auto store_lds = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_VEC; ++i) {
      int piece = tid + i * NT;
      *reinterpret_cast<v4i*>(&lds_a[buf * (BM * LDS_ROW) + (piece >> 2) * LDS_ROW + (piece & 3) * 16]) = ra[i];
    }
#pragma unroll
    for (int w = 0; w < B_WORDS; w += 4) {
      v4i t;
      t.x = IN_PACKED ? rb[w] : pack_chunks(rb[w]);
      t.y = IN_PACKED ? rb[w + 1] : pack_chunks(rb[w + 1]);
      t.z = IN_PACKED ? rb[w + 2] : pack_chunks(rb[w + 2]);
      t.w = IN_PACKED ? rb[w + 3] : pack_chunks(rb[w + 3]);
      *reinterpret_cast<v4i*>(&lds_b[buf * (BN * LDS_ROW) + b_n * LDS_ROW + (b_xs + w) * 4]) = t;
    }
  };

  auto compute = [&](int buf) {
    const int koff = (lane >> 4) * 16;
    v4i fa[MB], fb[NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
      fa[a] = *reinterpret_cast<const v4i*>(&lds_a[buf * (BM * LDS_ROW) + (wm * MB * 16 + a * 16 + (lane & 15)) * LDS_ROW + koff]);
#pragma unroll
    for (int b = 0; b < NB; ++b)
      fb[b] = *reinterpret_cast<const v4i*>(&lds_b[buf * (BN * LDS_ROW) + (wn * NB * 16 + b * 16 + (lane & 15)) * LDS_ROW + koff]);
    __builtin_amdgcn_s_setprio(1);   // keep the matrix pipe fed ahead of the staging waves
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
    __builtin_amdgcn_s_setprio(0);
  };

  // Software pipeline over K steps: LDS stage ks&1 is multiplied while stage
  // (ks+1)&1 is written from registers and step ks+2 is in flight from global
  // memory.  One barrier per step.
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
#pragma unroll
  for (int a = 0; a < MB; ++a) {
    const int u = (m0 + wm * MB * 16 + a * 16) / 4 + (lane >> 4);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int n = n0 + wn * NB * 16 + b * 16 + (lane & 15);
      if (n >= ncols) continue;
      const int poly = n / V, v = n - poly * V;
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
      size_t off = RIGHT ? (size_t)v * C + u : (size_t)u * C + v;
      dst[(size_t)poly * t.dst_stride + off] = r;
    }
  }
  (void)M;
}

template <int WM, int WN, int MB, int NB, int OCC, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW>
__global__ void __launch_bounds__(WM * WN * 64, OCC)
bat_gemm_kernel(GemmLaunch g, int tiles_m, int tiles_n) {
  constexpr int BM = WM * MB * 16;
  constexpr int BN = WN * NB * 16;
  // two LDS stages: the next K step is written while the current one is multiplied
  __shared__ __attribute__((aligned(16))) int8_t lds_a[2 * BM * LDS_ROW];
  __shared__ __attribute__((aligned(16))) int8_t lds_b[2 * BN * LDS_ROW];
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
  __shared__ __attribute__((aligned(16))) int8_t lds_a[2 * BM * LDS_ROW];
  __shared__ __attribute__((aligned(16))) int8_t lds_b[2 * BN * LDS_ROW];
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
  hipLaunchKernelGGL((bat_gemm_list_kernel<2, 2, 8, 4, 2, RIGHT, INP, OUTP, TW>), dim3(grid), dim3(256), 0, s,
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
  if (t == kTile256x256 && M < 256) t = kTileAuto;
  if (t == kTile256x128 && M < 256) t = kTileAuto;
  if (t == kTile128x64 && M < 128) t = kTileAuto;
  if (t != kTileAuto) return t;
  if (M >= 256) {
    // prefer the large tile when it still gives every CU two workgroups
    long grid = (long)g.njobs * (M / 256) * ((ncols + 127) / 128);
    if (grid >= 512) return kTile256x128;
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
    default: return dispatch_flags<2, 2, 2, 2, 2>(g, s);
  }
}

}  // namespace cross
