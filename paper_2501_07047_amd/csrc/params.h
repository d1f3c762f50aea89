// Host-side number theory and table construction for the BAT/MAT NTT.
//
// Everything here runs once per (prime, N, R) on the host ("offline compile"
// of the pre-known operands, Sec. BAT and Sec. MAT of arXiv 2501.07047) and is
// uploaded to the device once.  Pure C++; no device code.
#pragma once
#include <cstdint>
#include <vector>

namespace cross {

constexpr int kChunkBits = 7;   // bp: 7-bit chunks fit non-negative int8 MFMA operands
constexpr int kChunks = 4;      // Kc: four 7-bit chunks hold a residue below 2^28
constexpr int kTileK = 64;      // K extent of one table tile (one 16x16x64 MFMA step)

// Wide primes (2^28 <= q < 2^31) do not fit four 7-bit chunks.  Their tables
// use balanced signed 8-bit digits and the runtime side its four bytes, each
// fed to the MFMA as b - 128 (see bat_expand).  Only the NTT takes them.
constexpr uint32_t kNarrowPrimeLimit = 1u << 28;
constexpr uint32_t kWidePrimeLimit = 1u << 31;
inline bool wide_prime(uint32_t q) { return q >= kNarrowPrimeLimit; }

uint32_t powmod(uint64_t b, uint64_t e, uint32_t q);
bool is_prime_u32(uint32_t n);
uint32_t smallest_generator(uint32_t q);
// Canonical primitive 2N-th root: g^((q-1)/2N) for the smallest generator g.
uint32_t root_2n(uint32_t q, uint32_t log_n);
uint32_t inv_mod_2_32(uint32_t q);       // q^-1 mod 2^32 (q odd)
// A operand (1 KB, MFMA fragment order) of the BAT lazy reduction for prime q.
std::vector<int8_t> lazy_fragment(uint32_t q);
uint32_t bitrev(uint32_t x, int bits);

// BAT-expanded table of a pre-known residue matrix T (rows = "in", cols = "out"):
// dense int8 matrix D[m = out*4 + i][k = in*4 + j] = chunk_i((T[in][out] * 2^32 * 2^(7j)) mod q)
// (without the factor 2^32 when montgomery is false),
// stored in MFMA fragment order (M = 4 * n_out): for 64-deep K slab s = k / 64 and
// 32-row block b = m / 32, two 1 KB fragments (K halves h = (k % 64) / 32) of the
// v_mfma_i32_32x32x32_i8 A operand, byte (m, k) at
// (s * (M / 32) + b) * 2048 + h * 1024 + 16 * (m % 32 + 32 * ((k % 32) / 16)) + k % 16,
// so a workgroup's rows of one K slab are contiguous and load in lane order.
//
// For a wide prime (wide_prime(q)) the same layout holds with
// D[m = out*4 + i][k = in*4 + j] = digit_i(v), v = (T[in][out] * 2^32 * 2^(8j)) mod q,
// where digit_0..3 are the balanced base-256 digits (each in [-128, 127]) of
// the representative of v in [-2155905152, 2139062143] (such a representative
// exists for every residue class, since that range holds 2^32 > q integers),
// and the M * K bytes are followed by M int32 row corrections 128 * sum_k D[m][k]:
// the runtime bytes b enter the MFMA as b - 128, and an accumulator started at
// the correction ends at sum_k D[m][k] * b_k.
// Throws std::invalid_argument unless 4 * n_in is a multiple of 64.
void bat_expand(const std::vector<uint32_t>& T, int n_in, int n_out, uint32_t q,
                std::vector<int8_t>& out, bool montgomery = true);

struct NttTables {
  // forward: step 1 (left-known, rows), step 2 twiddle, step 3 (right-known, cols)
  std::vector<int8_t> fwd_left, fwd_right, inv_left, inv_right;
  // the same four without the Montgomery factor (Barrett epilogue; narrow primes only)
  std::vector<int8_t> fwd_left_plain, fwd_right_plain, inv_left_plain, inv_right_plain;
  std::vector<uint32_t> fwd_tw, inv_tw;      // (w, floor(w 2^32 / q)) pairs for Shoup multiplication
  std::vector<uint32_t> bf_fwd, bf_inv;      // butterfly twiddles, Montgomery form
  uint32_t bf_ninv;                          // N^-1 * 2^32 mod q (butterfly inverse scale)
  // three factors (row transform split as C1 x C2): BAT tables of the two row
  // sub-steps and their twiddle pairs, plus the inverse step-2 twiddles row-major
  std::vector<int8_t> row_fwd_b, row_fwd_c, row_inv_c, row_inv_b;
  // the same four without the Montgomery factor (Barrett epilogue)
  std::vector<int8_t> row_fwd_b_plain, row_fwd_c_plain, row_inv_c_plain, row_inv_b_plain;
  std::vector<uint32_t> row_fwd_t3, row_inv_t3, inv_tw_rows;
  // T3 times 2^32 mod q, as pairs: a forward row transform with these twiddles yields
  // its outputs times 2^32 (Montgomery form), for the fused key-switch inner product
  std::vector<uint32_t> row_fwd_t3_mont;
};
// with_bat = false builds only the butterfly twiddles (sizes below the MFMA minimum).
// log_c1 > 0 selects the three-factor form: the C-point row transform is split as
// C1 x C2 (C1 = 2^log_c1) and the C x C step-3 tables are not built.
void build_ntt_tables(uint32_t q, uint32_t log_n, uint32_t log_r, NttTables& t, bool with_bat = true,
                      uint32_t log_c1 = 0);

}  // namespace cross
