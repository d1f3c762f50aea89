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
// Wide primes (2^28 <= q < 2^31, template flag WIDE): residues are cut into
// their four bytes instead, each entering the signed MFMA as b - 128 (one XOR
// per word); the table holds balanced signed 8-bit digits and, after its bytes,
// one int32 correction 128 * (row sum) per row, which starts the accumulator;
// the epilogue merges the four signed sums with weights 2^(8i) in 64 bits and
// reduces with a signed Montgomery step.  Intermediates ("packed") are then
// the biased bytes.
//
// GEMM view (M x K times K x Ncols):
//   A[m][k]: pre-known, m = 4*u + i (output u, output chunk i), k = 4*x + j (input x, chunk j)
//   B[k][n]: chunk j of data element x of column n;  n = poly * V + v
// Rows order chunks fastest (m = 4u + i) so that the four chunk partial sums of
// one output land in four consecutive accumulator registers of one lane.
//
// All global accesses go through buffer resources: a wave-uniform base (the
// tile's first polynomial, the table, the twiddles) in scalar registers, a
// 32-bit per-lane byte offset, and the per-slab or per-row step in the scalar
// offset.  Addresses cost no 64-bit vector arithmetic, and a column past the
// end of the launch falls outside the resource's range: its loads read zero
// and its stores are dropped by the hardware.
#include "kernels.h"

#include <type_traits>

namespace cross {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef unsigned int v2u __attribute__((ext_vector_type(2)));

namespace {

constexpr int BK = 64;            // K per MFMA step

__device__ __forceinline__ uint32_t pack_chunks(uint32_t x) {
  // four 7-bit chunks of x (< 2^28) in the four bytes of one word
  return (x & 0x7fu) | ((x << 1) & 0x7f00u) | ((x << 2) & 0x7f0000u) | ((x << 3) & 0x7f000000u);
}

// Wide form: the four bytes of x, each biased to b - 128.
__device__ __forceinline__ uint32_t bias_bytes(uint32_t x) { return x ^ 0x80808080u; }

// Data operand of a residue in either form.
template <bool WIDE>
__device__ __forceinline__ uint32_t to_operand(uint32_t x) {
  if constexpr (WIDE)
    return bias_bytes(x);
  else
    return pack_chunks(x);
}

// Raw buffer resource over [base, base + bytes): range-checked per access.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint64_t bytes) {
  const uint32_t n = bytes > 0xfffffff0ull ? 0xfffffff0u : (uint32_t)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)n, 0x00020000);
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
  uint32_t bar_m, bar_k;   // Barrett epilogue constants (plain tables)
};

// MFMA v_mfma_i32_32x32x32_i8 (the int8 instruction that reaches the chip's
// dense int8 rate; the 16x16x64 form runs at half of it).  Lane l of a 32x32
// output block holds rows 8*(v/4) + 4*(l/32) + v%4 (v < 16) of column l%32:
// with rows ordered output-major, chunk-minor (m = 4u + i), registers 4g..4g+3
// are the four chunk partial sums of output u = 2g + l/32 -- the ChunkMerge is
// entirely in-register.
//
// Operand fragments are 1 KB: 32 rows (A) or columns (B) x 32 K bytes, lane l
// holding row/column l%32 and K bytes 16*(l/32) .. +15.  A 64-deep K slab of a
// 32-row block is two fragments (K halves).  The tables are stored in global
// memory in exactly this order, so staging is contiguous 16-byte copies and
// every LDS access (staging writes and MFMA operand reads) is lane-linear.

// Shape of one step as seen by a tile.
struct StepShape {
  int R, C, U, V, log_v, M, K, poly0;
};

template <bool RIGHT>
__device__ __forceinline__ StepShape step_shape(const TileArgs& t) {
  StepShape g;
  g.R = 1 << t.log_r;
  g.C = 1 << t.log_c;
  g.U = RIGHT ? g.C : g.R;              // outputs per column (and inputs per column)
  g.V = RIGHT ? g.R : g.C;              // columns per polynomial
  g.log_v = RIGHT ? t.log_r : t.log_c;  // V is a power of two: shifts, not divisions
  g.M = 4 * g.U;
  g.K = 4 * g.U;
  g.poly0 = t.n0 >> g.log_v;            // first polynomial of the tile's columns
  return g;
}

// Data buffers of a tile start at its first polynomial.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t data_rsrc(const uint32_t* base, uint64_t stride, int npoly,
                                                            int poly0) {
  return make_rsrc(base + (size_t)poly0 * stride, (uint64_t)(npoly - poly0) * stride * 4);
}

// Byte offset (from the tile's first polynomial) of the first of the four
// inputs held by B piece p of a 64-deep slab.  Piece p is lane p%64 of
// fragment f = p/64 = (32-column block f/2, K half f%2): column n0 + 32*(f/2) +
// p%32, inputs 8*(f%2) + 4*((p%64)/32) .. +3.  Element (input x, column v) of one
// polynomial lies at
//   plain, row side   : x*C + v        plain, column side  : v*C + x
//   packed, row side  : v*R + x (the inverse intermediate is stored transposed)
//   packed, col side  : v*C + x
template <bool RIGHT, bool IN_PACKED>
__device__ __forceinline__ uint32_t b_piece_offset(const TileArgs& t, const StepShape& g, int piece) {
  const int f = piece >> 6;
  const int n = t.n0 + (f >> 1) * 32 + (piece & 31);
  const int gp = (f & 1) * 8 + ((piece & 63) >> 5) * 4;
  const uint32_t dpoly = (uint32_t)((n >> g.log_v) - g.poly0), v = n & (g.V - 1);
  uint32_t off;
  if (IN_PACKED) off = v * (RIGHT ? g.C : g.R) + gp;
  else off = RIGHT ? v * g.C + gp : gp * g.C + v;
  return (dpoly * (uint32_t)t.src_stride + off) * 4;
}

// The four inputs of one B piece of slab k64, cut into 7-bit chunks if plain.
template <bool RIGHT, bool IN_PACKED>
__device__ __forceinline__ v4i load_b_piece(__amdgpu_buffer_rsrc_t rs, uint32_t off, int k64, int C) {
  v4i w;
  if (IN_PACKED || RIGHT) {
    w = (v4i)__builtin_amdgcn_raw_buffer_load_b128(rs, off, k64 * 64, 0);
  } else {
    // four inputs of one column lie C words apart
    const int row = k64 * 16 * C * 4;
    w = v4i{(int)__builtin_amdgcn_raw_buffer_load_b32(rs, off, row, 0),
            (int)__builtin_amdgcn_raw_buffer_load_b32(rs, off, row + C * 4, 0),
            (int)__builtin_amdgcn_raw_buffer_load_b32(rs, off, row + 2 * C * 4, 0),
            (int)__builtin_amdgcn_raw_buffer_load_b32(rs, off, row + 3 * C * 4, 0)};
  }
  return w;
}

template <bool WIDE>
__device__ __forceinline__ v4i pack4(v4i w) {
  return v4i{(int)to_operand<WIDE>(w.x), (int)to_operand<WIDE>(w.y), (int)to_operand<WIDE>(w.z),
             (int)to_operand<WIDE>(w.w)};
}

// Wide form: accumulator start of NA 32-row blocks from table row row0 on, the
// row corrections (int32, after the M x K table bytes) of the rows lane `lane`
// holds, 8 (v / 4) + 4 (lane / 32) + v % 4 of each block.
template <int NA>
__device__ __forceinline__ void corr_init(v16i (&init)[NA], const int8_t* table, int M, int K, int row0, int lane) {
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(table + (size_t)M * K, (uint64_t)M * 4);
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const v4i c = (v4i)__builtin_amdgcn_raw_buffer_load_b128(
          rs, (uint32_t)(row0 + a * 32 + 8 * j + 4 * (lane >> 5)) * 4, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) init[a][4 * j + i] = c[i];
    }
}

// Wide form: merge of the four signed digit sums (weights 2^(8i)) and signed
// Montgomery reduction to [0, q).  |z| < U * 1020 * 2^31.01 < 2^53 for U <= 4096,
// so (z - m q) / 2^32 = (z >> 32) - umulhi(m, q) lies in (-q - 2^21, 2^21], and
// two conditional additions of q (q > 2^21) bring it to [0, q).
__device__ __forceinline__ uint32_t merge_redc_wide(int s0, int s1, int s2, int s3, uint32_t q, uint32_t qinv) {
  const int64_t z = (int64_t)s0 + ((int64_t)s1 << 8) + ((int64_t)s2 << 16) + ((int64_t)s3 << 24);
  const uint32_t m = (uint32_t)z * qinv;
  int64_t r = (z >> 32) - (int64_t)__umulhi(m, q);
  if (r < 0) r += q;
  if (r < 0) r += q;
  return (uint32_t)r;
}

// ---- epilogue: ChunkMerge + REDC (+ twiddle) + final subtraction ------------
// Wave (wm, wn) holds MB x NB accumulator blocks of 32 x 32.  Column side with
// plain output: the tile's outputs run down columns of the R x C result, so
// they are staged in LDS (free after the last K stage; `so` must hold
// BN x (BM/4 + 4) words) as [column v][row u] and written back row by row, 16
// bytes per lane.
template <int NT, int BM, int BN, int MB, int NB, bool RIGHT, bool OUT_PACKED, bool TW, bool NARROW_ONLY = false,
          bool WIDE = false, int RED = 0>
__device__ __forceinline__ void gemm_epilogue(const v16i (&acc)[MB][NB], const TileArgs& t, const StepShape& g,
                                              int wm, int wn, uint32_t* so) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int m0 = t.m0, n0 = t.n0;
  const uint32_t q = t.q, qinv = t.qinv;
  const int V = g.V, log_v = g.log_v, poly0 = g.poly0;
  const __amdgpu_buffer_rsrc_t rs_dst = data_rsrc(t.dst, t.dst_stride, t.npoly, poly0);
  const __amdgpu_buffer_rsrc_t rs_tw = make_rsrc(t.tw, TW ? (uint64_t)g.U * V * 8 : 0);
  constexpr bool STAGE_OUT = RIGHT && !OUT_PACKED;
  constexpr int BU = BM / 4;              // outputs per tile column
  constexpr int SROW = BU + 4;            // padded LDS row (words)
  const uint32_t row_words = RIGHT ? g.R : g.C;         // output row length (transposed when RIGHT)

  // All twiddle pairs of this lane are loaded before the first store: issued next
  // to their use, each load would wait behind the stores before it (the compiler
  // cannot tell the twiddle table from the output), one round trip per output.
  v2u twv[TW ? MB : 1][TW ? NB : 1][4];
  if constexpr (TW) {
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      const int u0 = (m0 + (wm * MB + a) * 32) / 4 + (lane >> 5);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int n = n0 + (wn * NB + b) * 32 + (lane & 31);
        const uint32_t tw_off = ((uint32_t)u0 * V + (n & (V - 1))) * 8;
#pragma unroll
        for (int j = 0; j < 4; ++j) twv[a][b][j] = __builtin_amdgcn_raw_buffer_load_b64(rs_tw, tw_off, j * 2 * V * 8, 0);
      }
    }
  }

  auto body = [&](auto wide_tag) {
    constexpr bool WIDE_MERGE = decltype(wide_tag)::value;   // 64-bit ChunkMerge (narrow primes, U > 512)
#pragma unroll
    for (int a = 0; a < MB; ++a) {
      const int u0 = (m0 + (wm * MB + a) * 32) / 4 + (lane >> 5);   // output of register group 0
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int nl = (wn * NB + b) * 32 + (lane & 31);
        const int n = n0 + nl;
        const uint32_t dpoly = (uint32_t)((n >> log_v) - poly0), v = n & (V - 1);
        // register group j holds output u0 + 2j: consecutive groups are 2 rows apart
        const uint32_t out_off = (dpoly * (uint32_t)t.dst_stride + (uint32_t)u0 * row_words + v) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const v16i& sv = acc[a][b];
          const uint32_t s0 = (uint32_t)sv[4 * j], s1 = (uint32_t)sv[4 * j + 1];
          const uint32_t s2 = (uint32_t)sv[4 * j + 2], s3 = (uint32_t)sv[4 * j + 3];
          uint32_t r;
          if constexpr (WIDE) {
            // [0, q); the 32-bit merge where the contraction is at most 64 inputs deep
            r = g.U <= 64 ? merge_redc_wide32(sv[4 * j], sv[4 * j + 1], sv[4 * j + 2], sv[4 * j + 3], q, qinv)
                          : merge_redc_wide(sv[4 * j], sv[4 * j + 1], sv[4 * j + 2], sv[4 * j + 3], q, qinv);
          } else {
          uint32_t zlo, zhi;
          if (!WIDE_MERGE) {
            // z = x + w * 2^14 with x = s0 + s1 * 2^7 and w = s2 + s3 * 2^7 (both < 2^32)
            const uint32_t x = s0 + (s1 << 7), w = s2 + (s3 << 7);
            const uint32_t wl = w << 14;
            zlo = x + wl;
            zhi = (w >> 18) + (zlo < wl ? 1u : 0u);
          } else {
            const uint64_t z = (uint64_t)s0 + ((uint64_t)s1 << 7) + ((uint64_t)s2 << 14) + ((uint64_t)s3 << 21);
            zlo = (uint32_t)z;
            zhi = (uint32_t)(z >> 32);
          }
          if constexpr (RED == 1) {
            // Barrett (Alg. barrett) for plain tables: with k = bit length of q, z below
            // U * q * 4 * 127 < 2^21 q <= 2^(2k) (q >= 2^21), the quotient estimate
            // ((z >> (k - 1)) * floor(2^(2k) / q)) >> (k + 1) is short by at most 2: [0, q)
            const uint32_t kb = t.bar_k;
            const uint32_t zh = (zhi << (33 - kb)) | (zlo >> (kb - 1));
            const uint32_t tq = (uint32_t)(((uint64_t)zh * t.bar_m) >> (kb + 1));
            r = zlo - tq * q;
            r = r >= q ? r - q : r;
            r = r >= q ? r - q : r;
          } else {
            // Montgomery REDC of z (the 2^32 factor was folded into the table): (0, 2q)
            r = zhi + q - __umulhi(zlo * qinv, q);
          }
          }
          if (TW) {
            // Shoup multiplication by the pre-known twiddle (w, floor(w 2^32 / q)): [0, 2q)
            const v2u tw = twv[TW ? a : 0][TW ? b : 0][j];
            r = r * tw.x - __umulhi(r, tw.y) * q;
          }
          r = r >= q ? r - q : r;
          if (OUT_PACKED) r = to_operand<WIDE>(r);
          if (STAGE_OUT) {
            so[nl * SROW + (u0 + 2 * j - m0 / 4)] = r;
          } else {
            // column side with packed output = the inverse intermediate, stored transposed;
            // columns past the launch fall outside rs_dst and are dropped
            __builtin_amdgcn_raw_buffer_store_b32(r, rs_dst, out_off, j * 2 * row_words * 4, 0);
          }
        }
      }
    }
  };
  // Chunk partial sums are below K * 127 * 127 = 4U * 127^2; for U <= 512 the
  // two half-merges x and w fit 32 bits, larger U merges in 64 bits.
  if (NARROW_ONLY || WIDE || g.U <= 512) body(std::false_type{});
  else body(std::true_type{});

  if (STAGE_OUT) {
    __syncthreads();
    constexpr int VEC_PER_ROW = BU / 4;
#pragma unroll
    for (int i = 0; i < BN * VEC_PER_ROW / NT; ++i) {
      const int idx = tid + i * NT;
      const int nl = idx / VEC_PER_ROW, uq = idx % VEC_PER_ROW;
      const int n = n0 + nl;
      const uint32_t dpoly = (uint32_t)((n >> log_v) - poly0), v = n & (V - 1);
      const v4u w = *reinterpret_cast<const v4u*>(so + nl * SROW + uq * 4);
      const uint32_t off = (dpoly * (uint32_t)t.dst_stride + v * g.C + m0 / 4 + uq * 4) * 4;
      __builtin_amdgcn_raw_buffer_store_b128(w, rs_dst, off, 0, 0);
    }
    __syncthreads();   // LDS is reused by the next tile of a work list
  }
}

// LDS-staged form: both operands go through LDS.  Pipeline over K stages (KS
// slabs of 64 each) with one barrier per stage: the MFMAs of stage k are issued
// first, then stage k+1 (loaded one stage earlier) is written from registers
// to the idle LDS buffer and stage k+2 is loaded from global memory.  Plain
// residues are cut into 7-bit chunks on the way into LDS; packed data is
// copied as is.
template <int WM, int WN, int MB, int NB, int KS, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW,
          bool PROWS = false, bool WIDE = false, int RED = 0>
__device__ __forceinline__ void gemm_tile(const TileArgs& t, int8_t* lds_a, int8_t* lds_b) {
  constexpr int NW = WM * WN;
  constexpr int NT = NW * 64;
  constexpr int BM = WM * MB * 32;                   // MB, NB count 32 x 32 blocks per wave
  constexpr int BN = WN * NB * 32;
  constexpr int FA = 2 * BM / 32, FB = 2 * BN / 32;  // fragments per 64-deep slab
  constexpr int SLAB_A = FA * 1024, SLAB_B = FB * 1024;
  constexpr int STAGE_A = KS * SLAB_A, STAGE_B = KS * SLAB_B;
  constexpr int A_PIECES = FA * 64 / NT;             // 16-byte table pieces per thread per slab
  constexpr int B_PIECES = FB * 64 / NT;             // 16-byte data pieces (4 inputs x 1 column)
  static_assert(A_PIECES >= 1 && FA * 64 % NT == 0 && B_PIECES >= 1 && FB * 64 % NT == 0, "tile split");

  const StepShape g = step_shape<RIGHT>(t);
  const int M = g.M, K = g.K, C = g.C;
  const int m0 = t.m0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WN, wn = wave % WN;

  v16i acc[MB][NB];
#pragma unroll
  for (int a = 0; a < MB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = v16i{};

  const __amdgpu_buffer_rsrc_t rs_src = data_rsrc(t.src, t.src_stride, t.npoly, g.poly0);
  const __amdgpu_buffer_rsrc_t rs_tab =
      make_rsrc(t.table + (size_t)(m0 / 32) * 2048, (uint64_t)M * K - (uint64_t)(m0 / 32) * 2048);
  const uint32_t slab_bytes = (uint32_t)(M / 32) * 2048;   // one 64-deep K slab of the whole table
  uint32_t coloff[B_PIECES];
#pragma unroll
  for (int i = 0; i < B_PIECES; ++i) coloff[i] = b_piece_offset<RIGHT, IN_PACKED && !PROWS>(t, g, tid + i * NT);

  v4i ra[KS][A_PIECES], rb[KS][B_PIECES];
  auto load = [&](int ks) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
      const int k64 = ks * KS + sl;
#pragma unroll
      for (int i = 0; i < A_PIECES; ++i)
        ra[sl][i] = (v4i)__builtin_amdgcn_raw_buffer_load_b128(rs_tab, (tid + i * NT) * 16, k64 * slab_bytes, 0);
#pragma unroll
      for (int i = 0; i < B_PIECES; ++i) rb[sl][i] = load_b_piece<RIGHT, IN_PACKED && !PROWS>(rs_src, coloff[i], k64, C);
    }
  };
  auto store_lds = [&](int st) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
#pragma unroll
      for (int i = 0; i < A_PIECES; ++i)
        *reinterpret_cast<v4i*>(lds_a + st * STAGE_A + sl * SLAB_A + (tid + i * NT) * 16) = ra[sl][i];
#pragma unroll
      for (int i = 0; i < B_PIECES; ++i)
        *reinterpret_cast<v4i*>(lds_b + st * STAGE_B + sl * SLAB_B + (tid + i * NT) * 16) =
            IN_PACKED ? rb[sl][i] : pack4<WIDE>(rb[sl][i]);
    }
  };
  auto compute = [&](int st) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {          // K halves of the 64-deep slab
        v4i fa[MB], fb[NB];
#pragma unroll
        for (int a = 0; a < MB; ++a)
          fa[a] = *reinterpret_cast<const v4i*>(lds_a + st * STAGE_A + sl * SLAB_A +
                                                ((wm * MB + a) * 2 + h) * 1024 + lane * 16);
#pragma unroll
        for (int b = 0; b < NB; ++b)
          fb[b] = *reinterpret_cast<const v4i*>(lds_b + st * STAGE_B + sl * SLAB_B +
                                                ((wn * NB + b) * 2 + h) * 1024 + lane * 16);
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
      }
    }
  };

  const int nk = K / (BK * KS);
  load(0);
  store_lds(0);
  if (nk > 1) load(1);
  if constexpr (WIDE) {
    // accumulators start at the row corrections (loaded after the first stages,
    // so they do not add to the prologue's live registers)
    v16i init[MB];
    corr_init<MB>(init, t.table, M, K, m0 + wm * MB * 32, lane);
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = init[a];
  }
  __syncthreads();
  for (int ks = 0; ks < nk; ++ks) {
    compute(ks & 1);
    if (ks + 1 < nk) store_lds((ks + 1) & 1);
    if (ks + 2 < nk) load(ks + 2);
    __syncthreads();
  }
  gemm_epilogue<NT, BM, BN, MB, NB, RIGHT, OUT_PACKED, TW, false, WIDE, RED>(acc, t, g, wm, wn,
                                                                        reinterpret_cast<uint32_t*>(lds_a));
}

// Direct-table form (contractions of at most 512 inputs, so the ChunkMerge is
// 32-bit): WA x WN waves, each a (32 MA) x (32 NBD) block of the output.  Only
// the data operand goes through LDS (shared by the WA waves of a column
// group); each wave reads its own rows of the pre-known table straight from
// global memory (L2) into registers, in fragment order, one stage ahead.  The
// staged form moves 1 KB through LDS per MFMA with 64 x 64 waves, more than the
// LDS delivers at the MFMA rate; here half of that goes through the vector
// memory path instead, and the LDS writes shrink to the data operand.
template <int WA, int WN, int MA, int NBD, int KS, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW,
          bool PROWS = false>
__device__ __forceinline__ void gemm_tile_direct(const TileArgs& t, int8_t* lds) {
  constexpr int NT = WA * WN * 64;
  constexpr int BM = WA * MA * 32;
  constexpr int BN = WN * NBD * 32;
  constexpr int FB = 2 * BN / 32;                    // data fragments per 64-deep slab
  constexpr int SLAB_B = FB * 1024, STAGE_B = KS * SLAB_B;
  constexpr int B_PIECES = FB * 64 / NT;
  static_assert(B_PIECES >= 1 && FB * 64 % NT == 0, "tile split");

  const StepShape g = step_shape<RIGHT>(t);
  const int M = g.M, K = g.K, C = g.C;
  const int m0 = t.m0;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: the table resource is scalar
  const int wm = wave / WN, wn = wave % WN;

  v16i acc[MA][NBD];
#pragma unroll
  for (int a = 0; a < MA; ++a)
#pragma unroll
    for (int b = 0; b < NBD; ++b) acc[a][b] = v16i{};

  const __amdgpu_buffer_rsrc_t rs_src = data_rsrc(t.src, t.src_stride, t.npoly, g.poly0);
  // this wave's rows of the table: fragment (32-row block, slab, half) at
  // ((slab * M/32 + block) * 2 + half) * 1024
  const int blk0 = m0 / 32 + wm * MA;
  const __amdgpu_buffer_rsrc_t rs_tab =
      make_rsrc(t.table + (size_t)blk0 * 2048, (uint64_t)M * K - (uint64_t)blk0 * 2048);
  const uint32_t slab_bytes = (uint32_t)(M / 32) * 2048;
  uint32_t coloff[B_PIECES];
#pragma unroll
  for (int i = 0; i < B_PIECES; ++i) coloff[i] = b_piece_offset<RIGHT, IN_PACKED && !PROWS>(t, g, tid + i * NT);

  v4i fa[2][KS][2][MA];                  // table fragments of two stages
  v4i rb[KS][B_PIECES];
  auto load_a = [&](int ks, v4i (&dst)[KS][2][MA]) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int a = 0; a < MA; ++a)
          dst[sl][h][a] = (v4i)__builtin_amdgcn_raw_buffer_load_b128(
              rs_tab, (a * 2 + h) * 1024 + lane * 16, (ks * KS + sl) * slab_bytes, 0);
  };
  auto load_b = [&](int ks) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl)
#pragma unroll
      for (int i = 0; i < B_PIECES; ++i) rb[sl][i] = load_b_piece<RIGHT, IN_PACKED && !PROWS>(rs_src, coloff[i], ks * KS + sl, C);
  };
  auto store_b = [&](int st) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl)
#pragma unroll
      for (int i = 0; i < B_PIECES; ++i)
        *reinterpret_cast<v4i*>(lds + st * STAGE_B + sl * SLAB_B + (tid + i * NT) * 16) =
            IN_PACKED ? rb[sl][i] : pack4<false>(rb[sl][i]);
  };
  auto compute = [&](int st, const v4i (&a_frag)[KS][2][MA]) {
#pragma unroll
    for (int sl = 0; sl < KS; ++sl) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v4i fb[NBD];
#pragma unroll
        for (int b = 0; b < NBD; ++b)
          fb[b] = *reinterpret_cast<const v4i*>(lds + st * STAGE_B + sl * SLAB_B + ((wn * NBD + b) * 2 + h) * 1024 +
                                                lane * 16);
#pragma unroll
        for (int a = 0; a < MA; ++a)
#pragma unroll
          for (int b = 0; b < NBD; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a_frag[sl][h][a], fb[b], acc[a][b], 0, 0, 0);
      }
    }
  };
  const int nk = K / (BK * KS);          // even: K is a multiple of 2 * BK * KS
  // one stage: MFMAs of stage ks, then stage ks+1 of the data into the idle
  // LDS buffer, then the loads of stage ks+2 (table fragments into the
  // registers just consumed).  Every step issues the same loads (the last two
  // re-read the final stage, unused) so the number of loads in flight is the
  // same on every path and the waits stay one stage behind.
  auto step = [&](int ks, v4i (&cur)[KS][2][MA]) {
    compute(ks & 1, cur);
    if (ks + 1 < nk) store_b((ks + 1) & 1);
    const int kn = ks + 2 < nk ? ks + 2 : nk - 1;
    load_b(kn);
    load_a(kn, cur);
    // keep the loads here: left to itself the compiler sinks them to their
    // first use, a stage later, which leaves their latency exposed
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
  };

  load_a(0, fa[0]);
  load_b(0);
  store_b(0);
  load_b(1);            // nk >= 2
  load_a(1, fa[1]);
  __syncthreads();
  for (int ks = 0; ks < nk; ks += 2) {
    step(ks, fa[0]);
    step(ks + 1, fa[1]);
  }
  gemm_epilogue<NT, BM, BN, MA, NBD, RIGHT, OUT_PACKED, TW, true>(acc, t, g, wm, wn,
                                                                  reinterpret_cast<uint32_t*>(lds));
}

// LDS bytes of one workgroup: two operand stages, or the output staging tile if larger.
template <int WM, int WN, int MB, int NB, int KS, bool RIGHT, bool OUT_PACKED>
constexpr int gemm_lds_bytes() {
  constexpr int BM = WM * MB * 32, BN = WN * NB * 32;
  constexpr int ops = 2 * (BM + BN) * 64 * KS;
  constexpr int out = (RIGHT && !OUT_PACKED) ? BN * (BM / 4 + 4) * 4 : 0;
  return ops > out ? ops : out;
}

// Tile (job, tm, tn) of block b of a uniform launch.  XCD-aware order:
// consecutive logical tiles land on the same XCD so a job's table and columns
// stay in one L2; within a job m runs fastest so tiles sharing columns run
// together.
template <int BM, int BN>
__device__ __forceinline__ TileArgs uniform_tile(const GemmLaunch& g, int tiles_m, int tiles_n) {
  const int total = g.njobs * tiles_m * tiles_n;
  const int bid = blockIdx.x;
  int logical = bid;
  if ((total & 7) == 0) logical = (bid & 7) * (total >> 3) + (bid >> 3);
  const int per_job = tiles_m * tiles_n;
  const int job_id = logical / per_job;
  const int rem = logical - job_id * per_job;
  const int tn = rem / tiles_m;
  const int tm = rem - tn * tiles_m;
  const GemmJob job = g.jobs[job_id];
  return TileArgs{job.table, job.tw, g.src + job.src_off, g.dst + job.dst_off, g.src_stride, g.dst_stride,
                  job.q, job.qinv, g.npoly, g.log_r, g.log_c, tm * BM, tn * BN, job.bar_m, job.bar_k};
}

template <int WM, int WN, int MB, int NB, int OCC, int KS, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW,
          bool PROWS, bool WIDE, int RED>
__global__ void __launch_bounds__(WM * WN * 64, OCC)
bat_gemm_kernel(GemmLaunch g, int tiles_m, int tiles_n) {
  constexpr int BM = WM * MB * 32;
  constexpr int BN = WN * NB * 32;
  // two LDS stages of operand fragments (A stages then B stages), reused for output staging
  __shared__ __attribute__((aligned(1024))) int8_t lds[gemm_lds_bytes<WM, WN, MB, NB, KS, RIGHT, OUT_PACKED>()];
  const TileArgs t = uniform_tile<BM, BN>(g, tiles_m, tiles_n);
  gemm_tile<WM, WN, MB, NB, KS, RIGHT, IN_PACKED, OUT_PACKED, TW, PROWS, WIDE, RED>(t, lds, lds + 2 * BM * 64 * KS);
}

// LDS bytes of the direct-table form: two stages of data fragments, or the
// output staging tile if larger.
template <int WA, int WN, int MA, int NBD, int KS, bool RIGHT, bool OUT_PACKED>
constexpr int direct_lds_bytes() {
  constexpr int BM = WA * MA * 32, BN = WN * NBD * 32;
  constexpr int ops = 2 * KS * BN * 64;
  constexpr int out = (RIGHT && !OUT_PACKED) ? BN * (BM / 4 + 4) * 4 : 0;
  return ops > out ? ops : out;
}

template <int WA, int WN, int MA, int NBD, int OCC, int KS, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW,
          bool PROWS>
__global__ void __launch_bounds__(WA * WN * 64, OCC)
bat_gemm_direct_kernel(GemmLaunch g, int tiles_m, int tiles_n) {
  constexpr int BM = WA * MA * 32;
  constexpr int BN = WN * NBD * 32;
  __shared__ __attribute__((aligned(1024))) int8_t lds[direct_lds_bytes<WA, WN, MA, NBD, KS, RIGHT, OUT_PACKED>()];
  const TileArgs t = uniform_tile<BM, BN>(g, tiles_m, tiles_n);
  gemm_tile_direct<WA, WN, MA, NBD, KS, RIGHT, IN_PACKED, OUT_PACKED, TW, PROWS>(t, lds);
}

// Work-list form: tiles of many tasks (mixed N, R x C, primes, buffers) in one
// persistent launch.  The grid is a multiple of 8; XCD x (= blockIdx % 8) walks
// the x-th eighth of the tile list so each task's tiles share one L2.
template <int WM, int WN, int MB, int NB, int OCC, int KS, bool RIGHT, bool IN_PACKED, bool OUT_PACKED, bool TW,
          bool PROWS>
__global__ void __launch_bounds__(WM * WN * 64, OCC)
bat_gemm_list_kernel(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles) {
  constexpr int BM = WM * MB * 32;
  constexpr int BN = WN * NB * 32;
  __shared__ __attribute__((aligned(1024))) int8_t lds[gemm_lds_bytes<WM, WN, MB, NB, KS, RIGHT, OUT_PACKED>()];
  const int xcd = blockIdx.x & 7, local = blockIdx.x >> 3, per_xcd = gridDim.x >> 3;
  const int lo = (int)((long)ntiles * xcd / 8), hi = (int)((long)ntiles * (xcd + 1) / 8);
  for (int i = lo + local; i < hi; i += per_xcd) {
    const GemmTileRef r = tiles[i];
    const GemmTask k = tasks[r.task];
    TileArgs t{k.table, k.tw, k.src, k.dst, k.src_stride, k.dst_stride, k.q, k.qinv, k.npoly,
               k.log_r, k.log_c, (int)r.tm * BM, (int)r.tn * BN};
    gemm_tile<WM, WN, MB, NB, KS, RIGHT, IN_PACKED, OUT_PACKED, TW, PROWS>(t, lds, lds + 2 * BM * 64 * KS);
  }
}

// Grid of a uniform launch with BM x BN tiles; false if the shape does not tile.
template <int BM, int BN, bool RIGHT>
bool uniform_grid(const GemmLaunch& g, int kdiv, int& tiles_m, int& tiles_n, int& grid) {
  const int U = RIGHT ? (1 << g.log_c) : (1 << g.log_r);
  const int V = RIGHT ? (1 << g.log_r) : (1 << g.log_c);
  const int M = 4 * U, K = 4 * U;
  if (M % BM || K % kdiv) return false;
  // per-lane byte offsets are 32-bit and span at most BN / V + 1 polynomials of a tile
  const uint64_t span = (uint64_t)(BN / V + 2) * 4;
  if (span * g.src_stride >= (1ull << 31) || span * g.dst_stride >= (1ull << 31)) return false;
  tiles_m = M / BM;
  const int ncols = g.npoly * V;
  tiles_n = (ncols + BN - 1) / BN;
  grid = g.njobs * tiles_m * tiles_n;
  return true;
}

// LDS-staged tile: WM x WN waves of MB x NB blocks.
template <int WM, int WN, int MB, int NB, int OCC, int KS = 1>
struct StagedCfg {
  template <bool RIGHT, bool INP, bool OUTP, bool TW, bool PROWS = false, bool WIDE = false, int RED = 0>
  static hipError_t launch(const GemmLaunch& g, hipStream_t s) {
    constexpr int BM = WM * MB * 32, BN = WN * NB * 32;
    int tm, tn, grid;
    if (!uniform_grid<BM, BN, RIGHT>(g, BK * KS, tm, tn, grid)) return hipErrorInvalidValue;
    launch_kernel((bat_gemm_kernel<WM, WN, MB, NB, OCC, KS, RIGHT, INP, OUTP, TW, PROWS, WIDE, RED>), dim3(grid),
                       dim3(WM * WN * 64), 0, s, g, tm, tn);
    return hipGetLastError();
  }
};

// Direct-table tile: WA x WN waves of MA x NBD blocks, stages of KS slabs, unrolled by two.
template <int WA, int WN, int MA, int NBD, int OCC, int KS>
struct DirectCfg {
  template <bool RIGHT, bool INP, bool OUTP, bool TW, bool PROWS = false, bool WIDE = false, int RED = 0>
  static hipError_t launch(const GemmLaunch& g, hipStream_t s) {
    static_assert(!WIDE && RED == 0, "the direct tiles: narrow chunk sums and Montgomery only");
    constexpr int BM = WA * MA * 32, BN = WN * NBD * 32;
    int tm, tn, grid;
    if (!uniform_grid<BM, BN, RIGHT>(g, 2 * BK * KS, tm, tn, grid)) return hipErrorInvalidValue;
    launch_kernel((bat_gemm_direct_kernel<WA, WN, MA, NBD, OCC, KS, RIGHT, INP, OUTP, TW, PROWS>), dim3(grid),
                       dim3(WA * WN * 64), 0, s, g, tm, tn);
    return hipGetLastError();
  }
};

template <class Cfg, bool WIDE = false, int RED = 0>
hipError_t dispatch_flags(const GemmLaunch& g, hipStream_t s) {
  // forward: LEFT(plain in, packed out, twiddle) then RIGHT(packed in, plain out)
  // inverse: RIGHT(plain in, packed out, twiddle) then LEFT(packed in, plain out)
  const bool right = g.kind == kRight;
  if (!right && !g.in_packed && g.out_packed && g.twiddle)
    return Cfg::template launch<false, false, true, true, false, WIDE, RED>(g, s);
  if (right && g.in_packed && !g.out_packed && !g.twiddle)
    return Cfg::template launch<true, true, false, false, false, WIDE, RED>(g, s);
  if (right && !g.in_packed && g.out_packed && g.twiddle)
    return Cfg::template launch<true, false, true, true, false, WIDE, RED>(g, s);
  if (!right && g.in_packed && !g.out_packed && !g.twiddle && g.in_rows)
    return Cfg::template launch<false, true, false, false, true, WIDE, RED>(g, s);
  if (!right && g.in_packed && !g.out_packed && !g.twiddle)
    return Cfg::template launch<false, true, false, false, false, WIDE, RED>(g, s);
  return hipErrorInvalidValue;
}

}  // namespace

namespace {

// Work-list tiles: the staged 256 x 128 (8 waves of 64 x 64, two workgroups per CU),
// 128 x 64 and 64 x 64 (4 waves each, four per CU).  The grid holds as many
// workgroups as are resident, a multiple of 8 (one eighth of the list per XCD).
template <int WM, int WN, int MB, int NB, bool RIGHT, bool INP, bool OUTP, bool TW, bool PROWS>
hipError_t launch_list_tile(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, hipStream_t s) {
  constexpr int NW = WM * WN, OCC = 4;
  int ncu = 256;
  {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n > 0)
      ncu = n;
  }
  const int resident = ((4 * OCC / NW) * ncu + 7) / 8 * 8;
  const int grid = std::min(resident, (ntiles + 7) / 8 * 8);
  launch_kernel((bat_gemm_list_kernel<WM, WN, MB, NB, OCC, 1, RIGHT, INP, OUTP, TW, PROWS>), dim3(grid),
                dim3(NW * 64), 0, s, tasks, tiles, ntiles);
  return hipGetLastError();
}

template <bool RIGHT, bool INP, bool OUTP, bool TW, bool PROWS>
hipError_t launch_list_cfg(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, int tile, hipStream_t s) {
  switch (tile) {
    case kListTile256x128: return launch_list_tile<4, 2, 2, 2, RIGHT, INP, OUTP, TW, PROWS>(tasks, tiles, ntiles, s);
    case kListTile128x64: return launch_list_tile<2, 2, 2, 1, RIGHT, INP, OUTP, TW, PROWS>(tasks, tiles, ntiles, s);
    case kListTile64x64: return launch_list_tile<2, 2, 1, 1, RIGHT, INP, OUTP, TW, PROWS>(tasks, tiles, ntiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool gemm_list_tile_dims(int tile, int* rows, int* cols) {
  switch (tile) {
    case kListTile256x128: *rows = 256; *cols = 128; return true;
    case kListTile128x64: *rows = 128; *cols = 64; return true;
    case kListTile64x64: *rows = 64; *cols = 64; return true;
    default: return false;
  }
}

hipError_t launch_bat_gemm_list(const GemmTask* tasks, const GemmTileRef* tiles, int ntiles, int kind, bool in_packed,
                                bool out_packed, bool twiddle, bool in_rows, int tile, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const bool right = kind == kRight;
  if (in_rows && (right || !in_packed || out_packed || twiddle)) return hipErrorInvalidValue;
  if (!right && !in_packed && out_packed && twiddle)
    return launch_list_cfg<false, false, true, true, false>(tasks, tiles, ntiles, tile, s);
  if (right && in_packed && !out_packed && !twiddle)
    return launch_list_cfg<true, true, false, false, false>(tasks, tiles, ntiles, tile, s);
  if (right && !in_packed && out_packed && twiddle)
    return launch_list_cfg<true, false, true, true, false>(tasks, tiles, ntiles, tile, s);
  if (!right && in_packed && !out_packed && !twiddle && in_rows)
    return launch_list_cfg<false, true, false, false, true>(tasks, tiles, ntiles, tile, s);
  if (!right && in_packed && !out_packed && !twiddle)
    return launch_list_cfg<false, true, false, false, false>(tasks, tiles, ntiles, tile, s);
  return hipErrorInvalidValue;
}

int resolve_gemm_tile(const GemmLaunch& g) {
  const int U = (g.kind == kRight) ? (1 << g.log_c) : (1 << g.log_r);
  const int V = (g.kind == kRight) ? (1 << g.log_r) : (1 << g.log_c);
  const int M = 4 * U;
  const long ncols = (long)g.npoly * V;
  int t = g.tile;
  // wide primes and the Barrett epilogue: the staged 256 x 128 (8 waves), 128 x 64 and
  // 64 x 64 tiles only
  if ((g.wide || g.red) && t != kTile256x128w8 && t != kTile128x64 && t != kTile64x64) t = kTileAuto;
  if ((t == kTile256x256 || t == kTile256x128w8 || t == kTile256x256w16 || t == kTile256x256w16k2) && M < 256)
    t = kTileAuto;
  if (t == kTile256x128 && M < 256) t = kTileAuto;
  if (t == kTile128x64 && M < 128) t = kTileAuto;
  // the direct tiles merge chunk sums in 32 bits only: contractions up to 512 inputs
  if ((t == kTileDirect256x128 || t == kTileDirect256x128n) && (M < 256 || U > 512)) t = kTileAuto;
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
  if (g.wide) {
    // wide primes: LDS-staged tiles only (the direct tiles merge in 32 bits)
    if (U > 4096 || g.red != 0) return hipErrorInvalidValue;   // the 64-bit merge bound; Montgomery only
    switch (resolve_gemm_tile(g)) {
      case kTile256x128w8: return dispatch_flags<StagedCfg<4, 2, 2, 2, 4>, true>(g, s);
      case kTile128x64: return dispatch_flags<StagedCfg<2, 2, 2, 1, 4>, true>(g, s);
      default: return dispatch_flags<StagedCfg<2, 2, 1, 1, 4>, true>(g, s);
    }
  }
  if (g.red == 1) {
    // Barrett epilogue (plain tables): the same three staged tiles
    if (U > 4096) return hipErrorInvalidValue;   // z < U q 508 <= 2^(2k) needs U <= 4096 at q >= 2^21
    switch (resolve_gemm_tile(g)) {
      case kTile256x128w8: return dispatch_flags<StagedCfg<4, 2, 2, 2, 4>, false, 1>(g, s);
      case kTile128x64: return dispatch_flags<StagedCfg<2, 2, 2, 1, 4>, false, 1>(g, s);
      default: return dispatch_flags<StagedCfg<2, 2, 1, 1, 4>, false, 1>(g, s);
    }
  }
  if (g.red != 0) return hipErrorInvalidValue;
  switch (resolve_gemm_tile(g)) {
    case kTile256x256: return dispatch_flags<StagedCfg<2, 4, 4, 2, 2>>(g, s);     // 8 waves of 128x64
    case kTile256x128: return dispatch_flags<StagedCfg<2, 2, 4, 2, 2>>(g, s);     // 4 waves of 128x64
    case kTile128x64: return dispatch_flags<StagedCfg<2, 2, 2, 1, 4>>(g, s);      // 4 waves of 64x32
    case kTile256x128w8: return dispatch_flags<StagedCfg<4, 2, 2, 2, 4>>(g, s);   // 8 waves of 64x64
    case kTile256x256w16: return dispatch_flags<StagedCfg<4, 4, 2, 2, 4>>(g, s);  // 16 waves of 64x64
    case kTile256x256w16k2: return dispatch_flags<StagedCfg<4, 4, 2, 2, 4, 2>>(g, s);  // same, 128-deep K stages
    case kTileDirect256x128: return dispatch_flags<DirectCfg<4, 2, 2, 2, 4, 1>>(g, s);   // 8 waves of 64x64, direct table
    case kTileDirect256x128n: return dispatch_flags<DirectCfg<4, 1, 2, 4, 2, 1>>(g, s);  // 4 waves of 64x128, direct table
    default: return dispatch_flags<StagedCfg<2, 2, 1, 1, 4>>(g, s);               // 64 x 64: 4 waves of 32x32
  }
}

}  // namespace cross
