// Internal interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <cstdint>

namespace cross {

// Profiling events of the innermost enabled ProfScope of this thread (null when
// profiling is off).  The scope's first launch stamps `start`, every launch
// stamps `stop`, both from the dispatch itself (hipExtLaunchKernel), so timing
// adds no packets to the queue.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  int stamped = 0;          // launches that stamped the events
};
LaunchEvents& launch_events();

template <typename F, typename... Args>
inline void launch_kernel(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
  LaunchEvents& ev = launch_events();
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (ev.stop && hipStreamIsCapturing(s, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone) {
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, ev.start, ev.stop, 0u, args...);
    ev.start = nullptr;
    ++ev.stamped;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
  }
}

// Wide primes (2^28 <= q < 2^31): merge of the four signed digit sums s_i
// (weights 2^(8i)) and signed Montgomery reduction to [0, q), for contractions of
// at most 64 inputs, where |s_i| <= 64 * 4 * 128 * 255 < 2^23.  Then A = s0 + 2^8 s1
// and B = s2 + 2^8 s3 fit int32; z = A + 2^16 B has low word lo = A + (B << 16) mod
// 2^32 and high word (B >> 16) + carry + (A >> 31) (the sign of A borrows one).
// |z| < 64 * 1020 * 2^31.01 < 2^48, so |hi| <= 2^16 and w = (z - m q) / 2^32 + q =
// (hi + q) - umulhi(m, q) lies in (-2^16, q + 2^16]: computed mod 2^32 a negative w
// reads as at least 2^32 - 2^16, and one conditional addition or subtraction of q
// brings it to [0, q).
__device__ __forceinline__ uint32_t merge_redc_wide32(int32_t s0, int32_t s1, int32_t s2, int32_t s3, uint32_t q,
                                                      uint32_t qinv) {
  const int32_t A = s0 + (int32_t)((uint32_t)s1 << 8);
  const int32_t B = s2 + (int32_t)((uint32_t)s3 << 8);
  const uint32_t U = (uint32_t)B << 16;
  const uint32_t lo = (uint32_t)A + U;
  const int32_t hi = (B >> 16) + (lo < U ? 1 : 0) + (A >> 31);
  const uint32_t m = lo * qinv;
  uint32_t w = ((uint32_t)hi + q) - __umulhi(m, q);
  if (w >= 0xffff0000u)
    w += q;
  else if (w >= q)
    w -= q;
  return w;
}

// One limb of one BAT NTT step: all `npoly` polynomials of the limb share the
// prime and therefore the table.  Offsets are in uint32 elements from the
// launch's base pointers, so a job list can be reused for any buffer.
struct GemmJob {
  const int8_t* table;     // tile-major BAT-expanded matrix (params.h, bat_expand)
  const uint32_t* tw;      // step-2 twiddles (Montgomery form) or nullptr
  uint64_t src_off, dst_off;
  uint32_t q, qinv;        // prime and q^-1 mod 2^32
  uint32_t bar_m, bar_k;   // Barrett epilogue (plain table): floor(2^(2k) / q), k = bit length of q
};

// Step kinds of the layout-invariant 3-step NTT.
//  LEFT : out[u][v] = sum_r T[r][u] X[r][v]   (pre-known matrix on the left; step 1)
//  RIGHT: out[v][u] = sum_c X[v][c] T[c][u]   (pre-known matrix on the right; step 3)
// For LEFT, u runs over rows (R of them) and v over columns (C); for RIGHT,
// u runs over columns (C) and v over rows (R).
enum StepKind { kLeft = 0, kRight = 1 };

struct GemmLaunch {
  const GemmJob* jobs;     // device array
  int njobs;
  const uint32_t* src;
  uint32_t* dst;
  uint64_t src_stride, dst_stride;   // elements between successive polynomials of a job
  int npoly;
  int log_r, log_c;
  int kind;                // StepKind
  bool in_packed, out_packed, twiddle;
  int tile;                // GemmTile; kTileAuto picks by shape and grid size
  bool in_rows;            // row side, packed input stored row-major (three-factor inverse)
  bool wide;               // wide primes (2^28 <= q < 2^31): byte operands, signed-digit tables
  int red;                 // epilogue reduction: 0 Montgomery REDC, 1 Barrett (plain tables, q >= 2^21)
};

// Workgroup tile shapes of the BAT GEMM (rows x columns of the int8 product).
enum GemmTile { kTileAuto = 0, kTile256x256 = 1, kTile256x128 = 2, kTile128x64 = 3, kTile64x64 = 4,
                kTile256x128w8 = 5, kTile256x256w16 = 6, kTile256x256w16k2 = 7, kTileDirect256x128 = 8,
                kTileDirect256x128n = 9, kTileCount = 10 };
// Tile that launch_bat_gemm would use for g (resolves kTileAuto).
int resolve_gemm_tile(const GemmLaunch& g);

hipError_t launch_bat_gemm(const GemmLaunch& g, hipStream_t s);

// Three-factor NTT: the row transform with C-point rows split as C1 x C2, for
// every row of every polynomial of every job (ntt_rows.hip).  Forward: in =
// packed step-1 output, out = plain result; inverse: in = plain, out = packed
// rows with the inverse step-2 twiddle applied.  in / out: same layout as the
// polynomials (job offset + poly * stride + row * C).
struct RowsJob {
  const int8_t* tab1;       // first sub-step table (fragment order)
  const int8_t* tab2;       // second sub-step table
  const uint32_t* tw1;      // (w, w') pairs [C1][C2] after the first sub-step
  const uint32_t* tw2;      // inverse only: (w, w') pairs [R][C] after the second sub-step
  uint64_t off;             // element offset of the job's limb
  uint32_t q, qinv;
  uint32_t bar_m, bar_k;    // Barrett epilogue: floor(2^(2k) / q), k = bit length of q
};
// red: epilogue reduction of both sub-steps, 0 = Montgomery REDC (tables carry 2^32),
// 1 = Barrett (plain tables).  wide: primes 2^28 <= q < 2^31 (byte operands,
// signed-digit tables with row corrections; red must be 0).
hipError_t launch_ntt_rows(const RowsJob* jobs, int njobs, const uint32_t* in, uint32_t* out, uint64_t stride,
                           int npoly, int log_r, int log_c1, int log_c2, bool inverse, int red, bool wide,
                           hipStream_t s);
// Work-list form of the row transform (batch runtime), split C1 = C2 = 32 only: each
// task is one limb of one job (its prime's tables, its own buffers, npoly
// polynomials `stride` apart, R = 2^log_r rows of 1024) and owns npoly * R / 8
// blocks of eight rows (row block major, polynomial minor), blocks [first_block,
// first_block of the next task); tasks are
// in first_block order and nblocks is the total.  Forward: in = packed row-side
// output, out = plain; inverse: in = plain, out = packed rows with the inverse step-2
// twiddle applied (tw2 = its [R][C][2] pairs).
struct RowsTask {
  const int8_t* tab;        // 128 x 128 sub-step table (C1 = C2: one matrix for both sub-steps)
  const uint32_t* tw1;      // first-epilogue twiddle pairs
  const uint32_t* tw2;      // inverse only: step-2 twiddle pairs
  const uint32_t* in;
  uint32_t* out;
  uint64_t stride;
  uint32_t q, qinv;
  int32_t npoly, log_r;
  int32_t first_block, pad;
};
hipError_t launch_ntt_rows_list(const RowsTask* tasks, int ntasks, int64_t nblocks, bool inverse, hipStream_t s);
int rows_list_rows_per_block();
// Whether (log_r, log_c1, log_n - log_r - log_c1) is a split the row kernels implement.
bool rows_split_supported(int log_n, int log_r, int log_c1);

// Work-list GEMM step (batch runtime): each task is one limb list of one
// transform with its own shape and buffers; each tile ref names (task, tm, tn)
// of one list tile (gemm_list_tile_dims).  All tasks of one launch share the step
// kind, the packed/twiddle/row-major flags and the tile.
struct GemmTask {
  const int8_t* table;
  const uint32_t* tw;
  const uint32_t* src;
  uint32_t* dst;
  uint64_t src_stride, dst_stride;
  uint32_t q, qinv;
  int32_t npoly;
  int16_t log_r, log_c;
};
struct GemmTileRef {
  uint32_t task;
  uint16_t tm, tn;
};
// List tiles (rows x columns of the int8 product per workgroup tile).
enum GemmListTile { kListTile256x128 = 0, kListTile128x64 = 1, kListTile64x64 = 2, kListTileCount = 3 };
bool gemm_list_tile_dims(int tile, int* rows, int* cols);
// in_rows: row side with packed input stored row-major (the three-factor inverse's
// row-side step).  The grid is chosen here (resident workgroups of the tile).
hipError_t launch_bat_gemm_list(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, int kind, bool in_packed,
                                bool out_packed, bool twiddle, bool in_rows, int tile, hipStream_t s);

struct ButterflyJob {
  const uint32_t* tw;      // psi^brv(i) (or its inverse), Montgomery form, N entries
  uint64_t off;            // element offset of the limb in the launch's buffer
  uint32_t q, qinv, ninv;  // ninv: N^-1 * 2^32 mod q (inverse only)
};
hipError_t launch_butterfly(const ButterflyJob* jobs, int njobs, uint32_t* data, uint64_t stride,
                            int npoly, int log_n, bool inverse, hipStream_t s);

}  // namespace cross

namespace cross {

// Per-limb modulus constants for the vector-ALU streams.
struct LimbMod {
  uint32_t q;
  uint32_t bar_m;     // floor(2^(2k) / q), k = bit length of q (Barrett, Alg. barrett)
  uint32_t bar_k;     // k
  uint32_t pad;
};

// Tensor product of two ciphertext batches in NTT form (HE-Mult step 1):
// out0 = a0 b0, out1 = a0 b1 + a1 b0, d2 = a1 b1, limb-wise mod q_i.
// a, b, out: [B][2][L][N]; d2: [B][L][N].
hipError_t launch_tensor(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                         const LimbMod* mods, int L, int log_n, int B, hipStream_t s, bool wide = false);

// Key-switch inner product: acc[b][s][t] = sum_j ext[b][j][t] * key[j][s][t] mod p_t,
// j < ndig (active digits), s in {0, 1}.  ext: [B][dnum][LK][N], key: [dnum][2][LK][N],
// acc: [B][2][LK][N].  With d ([B][L][N]), digit j's own limbs t in [j alpha,
// min((j + 1) alpha, L)) are read from d[b][t] instead of ext[b][j][t].
hipError_t launch_inner_product(const uint32_t* ext, const uint32_t* key, uint32_t* acc,
                                const LimbMod* mods, int LK, int dnum, int ndig, int log_n, int B,
                                hipStream_t s, const uint32_t* d = nullptr, int L = 0, int alpha = 0,
                                bool wide = false);

// Per-limb constants of the chunked stream forms (streams.hip).
struct StreamMod {
  uint32_t q;
  uint32_t qneg;      // -q^-1 mod 2^32 (Montgomery reduction)
  uint32_t bar_m;     // floor(2^(2k) / q), k = bit length of q (Barrett, Alg. barrett)
  uint32_t bar_k;     // k
  uint32_t pow2[4];   // 2^(32 + 8 i) mod q: the evaluation-key BAT expansion
};

// Evaluation-key BAT expansion: key [dnum][2][LK][N] -> key_bat [dnum][2][LK][N][4 words].
hipError_t launch_evk_bat_prepare(const uint32_t* key, uint32_t* key_bat, const StreamMod* mods, int LK, int dnum,
                                  int log_n, hipStream_t s);
// Key-switch inner product from the expanded key (same result as launch_inner_product
// with ndig = dnum).
hipError_t launch_inner_product_bat(const uint32_t* ext, const uint32_t* key_bat, uint32_t* acc,
                                    const StreamMod* mods, int LK, int dnum, int log_n, int B, hipStream_t s);
// Tensor product with every product taken as a chunk-wise convolution (same result
// as launch_tensor).
hipError_t launch_tensor_conv(const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                              const StreamMod* mods, int L, int log_n, int B, hipStream_t s);

// ModDown tail: out[p][i] = (base[p][i] + (acc[p][i] - z[p][i]) * Pinv_i) mod q_i for the
// first L limbs of every polynomial p < npoly.  base may be null (treated as 0) or alias out.
// acc stride: acc_stride elements per poly; z and out/base: L*N per poly.
struct TailConst {
  uint32_t q, pinv, pinv_shoup, pad;
};
hipError_t launch_moddown_tail(const uint32_t* acc, uint64_t acc_stride, const uint32_t* z,
                               const uint32_t* base, uint32_t* out, uint64_t out_stride,
                               const TailConst* tc, int L, int log_n, int npoly,
                               bool base_only_even, hipStream_t s);

// The same tail fused into the forward row kernel of the NTT of z (three factors
// with the 32 x 32 row split): the kernel's output row y of job j (limb offset
// jobs[j].off), polynomial p, row r is not stored; instead, at o = jobs[j].off + r * 1024,
// out[p * out_stride + o ..] = base[p * out_stride + o ..] + (acc[p * acc_stride + o ..] - y) * Pinv_j
// mod q_j (tc[j] per job).  base may be null (treated as 0), alias out, or, with
// base_only_even, be added for even p only.
struct RowsTail {
  const uint32_t* acc;
  uint64_t acc_stride;
  const uint32_t* base;
  uint32_t* out;
  uint64_t out_stride;
  const TailConst* tc;
  int base_only_even;
};
// in: the packed row-side output (layout of z: job offset + p * stride + r * 1024).
hipError_t launch_ntt_rows_tail(const RowsJob* jobs, int njobs, const uint32_t* in, uint64_t stride, int npoly,
                                int log_r, const RowsTail& tail, hipStream_t s);
// Whether the fused form exists for this split (the persistent 32 x 32 row kernel).
bool rows_tail_supported(int log_n, int log_r, int log_c1);

// ModUp NTT fused with the key-switch inner product (three factors R x 32 x 32): for
// every ciphertext b < B and limb t < LK,
//   acc[b][s][t] = sum_{j < ndig} E_j[b][t] * key[j][s][t] mod p_t,
// where E_j[b][t] = d[b][t] for t in digit j (own == j in t's limb entry) and otherwise
// the forward row transform of tmp + b * ext_stride + (j * LK + t) * N (the packed
// row-side step output of the converted limb, ext layout).  limbs: LK entries, one per
// limb, in the order the blocks take them (each carries its limb index).
// d: [B][L][N]; key: [dnum][2][LK][N]; acc: [B][2][LK][N]; N = 2^(rb_log + 13).
struct IpLimb {
  const int8_t* tab;        // forward 32-point sub-step table of t's prime (fragment order)
  const uint32_t* tw1;      // its first-epilogue twiddle pairs times 2^32 (T3 * 2^32 mod q): the
                            // transforms come out times 2^32, ready for a Montgomery product
  uint32_t q, qinv;         // prime, q^-1 mod 2^32
  uint32_t bar_m, bar_k;    // Barrett constants of the key products with t's own digit
  int32_t own;              // digit holding t (-1 for special primes)
  int32_t limb;             // t itself: the list runs in the order the blocks take the
                            // limbs, which need not be 0 .. LK - 1
};
struct RowsIp {
  const IpLimb* limbs;
  const uint32_t* tmp;
  const uint32_t* d;
  const uint32_t* key;
  uint32_t* acc;
  uint64_t ext_stride;
  int LK, L, B, ndig, rb_log;
};
hipError_t launch_ntt_rows_ip(const RowsIp& p, hipStream_t s);
// Task-list form (batch runtime): task k covers blocks [first_block, next task's
// first_block), LK * B * R / 8 of them, in first_block order; nblocks is the total.
struct IpTask {
  RowsIp p;
  int32_t first_block, pad;
};
hipError_t launch_ntt_rows_ip_list(const IpTask* tasks, int ntasks, int64_t nblocks, hipStream_t s);
// Task-list form of the forward row kernel with the fused tail (batch runtime): each
// task one limb (r, in = its packed row-side output, npoly polynomials) and its tail:
// out[p * out_stride + r * 1024 ..] = base[same] + (acc[p * acc_stride + r * 1024 ..] - y) * Pinv,
// base null (0) or, with base_only_even, added for even p only.
struct RowsTailTask {
  RowsTask r;
  const uint32_t* acc;
  uint64_t acc_stride;
  const uint32_t* base;
  uint32_t* out;
  uint64_t out_stride;
  uint32_t pinv, pinv_shoup;
  int32_t base_only_even, pad;
};
hipError_t launch_ntt_rows_tail_list(const RowsTailTask* tasks, int ntasks, int64_t nblocks, hipStream_t s);

// NTT-domain automorphism: out[p][l][x] = in[p][l][perm[x]] for L limbs of npoly polynomials.
hipError_t launch_automorphism(const uint32_t* in, uint64_t in_stride, uint32_t* out,
                               uint64_t out_stride, const uint32_t* perm, int log_n, int L,
                               int npoly, hipStream_t s);

// Pointwise product (VecModMul): out = a * b mod q_limb, all [B][L][N].
hipError_t launch_pointwise_mul(const uint32_t* a, const uint32_t* b, uint32_t* out,
                                const LimbMod* mods, int L, int log_n, int B, hipStream_t s);

// HE-Add (VecModAdd): out = a + b mod q_limb, all [npoly][L][N]; out may alias a or b.
hipError_t launch_pointwise_add(const uint32_t* a, const uint32_t* b, uint32_t* out,
                                const LimbMod* mods, int L, int log_n, int npoly, hipStream_t s);

// VecModMul with a pre-known operand under a chosen modular reduction
// (out[p][l] = a[p][l] * w[l] mod q_l, all limbs [N]; out may alias a).
enum Modred { kModredBarrett = 0, kModredMontgomery = 1, kModredShoup = 2, kModredBatLazy = 3 };
struct ModLimb {
  uint32_t q, qinv;      // q^-1 mod 2^32 (Montgomery REDC)
  uint32_t bar_m, bar_k; // Barrett: k = bitlen(q), m = floor(2^(2k) / q)
  uint32_t r32, pad[3];  // 2^32 mod q
};
// w: [L][N] prepared values; w_quot: [L][N] Shoup quotients (Shoup only);
// lazy: L fragments of 1 KB, the BAT chunk matrix per prime (BAT-lazy only, log_n >= 8).
hipError_t launch_vec_modmul(const uint32_t* a, const uint32_t* w, const uint32_t* w_quot, uint32_t* out,
                             const ModLimb* limbs, const int8_t* lazy, int L, int log_n, int npoly, int method,
                             hipStream_t s);
hipError_t launch_modmul_prepare(const uint32_t* w, uint32_t* w_prep, uint32_t* w_quot, const ModLimb* limbs,
                                 int L, int log_n, int method, hipStream_t s);

// Strided limb copy / zero: for each poly p < npoly and limb l < nl:
// dst[p*dst_stride + dst_off[l] ..+N] = src ? src[p*src_stride + src_off[l] ..] : 0.
hipError_t launch_limb_copy(const uint32_t* src, uint64_t src_stride, const uint64_t* src_off,
                            uint32_t* dst, uint64_t dst_stride, const uint64_t* dst_off, int nl,
                            int log_n, int npoly, hipStream_t s);

// Fast basis conversion (App. BConv) as an int8 MFMA GEMM.
// Step 1 (fused prologue): b_i = x_i * qhat_i^-1 mod q_i (Shoup constants per source).
// Step 2: out_t = sum_i b_i [qhat_i]_t mod t via the BAT-expanded table (32x32x32 MFMA).
struct BconvSrc {
  uint64_t off;        // element offset of source limb i within a polynomial
  uint32_t q, w, w_shoup, pad;   // w = qhat_i^-1 mod q_i
};
struct BconvDst {
  uint64_t off;        // element offset of target limb t within a polynomial
  uint32_t q, qinv;    // target prime, q^-1 mod 2^32
};
struct BconvLaunch {
  const BconvSrc* src;    // nsrc entries (device)
  const BconvDst* dst;    // ndst entries (device)
  const int8_t* table;    // fragment-ordered BAT table, mblocks x kblocks x 1 KB
  int nsrc, ndst;
  const uint32_t* in;
  uint32_t* out;
  uint64_t in_stride, out_stride;   // elements per polynomial
  int npoly, log_n;
  // 1 when a source or target prime is wide (2^28 <= q < 2^31): the operand is
  // the four bytes of each step-1 residue fed as b - 128, the table holds balanced
  // signed 8-bit digits followed by one int32 row correction 128 * (row sum) per
  // output row (mblocks x 32), and the epilogue merges with weights 2^(8i)
  int wide;
};
hipError_t launch_bconv(const BconvLaunch& b, hipStream_t s);
// Several conversions in one launch (by value, kBconvMulti per launch; more are
// split over launches), e.g. the digits of one ModUp; all of one form (narrow or wide).
constexpr int kBconvMulti = 8;
struct BconvMulti {
  BconvLaunch g[kBconvMulti];
};
hipError_t launch_bconv_multi(const BconvLaunch* gs, int n, hipStream_t s);

}  // namespace cross

namespace cross {

// ---- work-list forms of the vector streams (batch runtime) ------------------
// One task per blockIdx.y; each task covers `count4` 16-byte vectors.
struct TensorTask {            // one ciphertext pair: a, b, out [2][L][N], d2 [L][N]
  const uint32_t* a;
  const uint32_t* b;
  uint32_t* out;
  uint32_t* d2;
  const LimbMod* mods;
  int L, log_n;
  uint64_t count4;
};
struct CopyTask {              // dst[0 .. 4*count4) = src ? src[...] : 0
  const uint32_t* src;
  uint32_t* dst;
  uint64_t count4;
};
struct InnerTask {             // one ciphertext: ext [dnum][LK][N], key [dnum][2][LK][N], acc [2][LK][N]
  const uint32_t* ext;
  const uint32_t* key;
  uint32_t* acc;
  const LimbMod* mods;
  int LK, dnum, ndig, log_n;
  uint64_t count4;
};
struct TailTask {              // one polynomial: out[i] = base[i] + (acc[i] - z[i]) * Pinv_i, i < L
  const uint32_t* acc;
  const uint32_t* z;
  const uint32_t* base;
  uint32_t* out;
  const TailConst* tc;
  int L, log_n;
  uint64_t count4;
};
hipError_t launch_tensor_list(const TensorTask* t, int n, uint64_t max4, hipStream_t s);
hipError_t launch_copy_list(const CopyTask* t, int n, uint64_t max4, hipStream_t s);
hipError_t launch_inner_list(const InnerTask* t, int n, uint64_t max4, hipStream_t s);
hipError_t launch_tail_list(const TailTask* t, int n, uint64_t max4, hipStream_t s);
// BConv over many independent conversions (one BconvLaunch per task, pointers absolute):
// max_cols the largest npoly << log_n and max_nsrc the largest nsrc of the tasks.
hipError_t launch_bconv_list(const BconvLaunch* t, int n, uint64_t max_cols, int max_nsrc, hipStream_t s);

}  // namespace cross

namespace cross {
// Debug mode: record in *first the lowest position (p * nl + l) * N + n with
// base[p * stride + limbs[l].off + n] >= limbs[l].q (*first untouched if none).
struct CheckLimb {
  uint64_t off;
  uint32_t q, pad;
};
hipError_t launch_residue_check(const uint32_t* base, uint64_t stride, int npoly, const CheckLimb* limbs, int nl,
                                int log_n, unsigned long long* first, hipStream_t s);

struct AutoTask {              // out[l][x] = in[l][perm[x]] for L limbs of one polynomial
  const uint32_t* in;
  uint32_t* out;
  const uint32_t* perm;
  int log_n;
  uint64_t count;              // L * N
};
hipError_t launch_auto_list(const AutoTask* t, int n, uint64_t max_count, hipStream_t s);
}  // namespace cross
