// Host precompute: primality, roots and the MAT-permuted, BAT-expanded twiddle
// tables of the layout-invariant 3-step negacyclic NTT (arXiv 2501.07047,
// Sec. MAT "Bit-reverse shuffling elimination" and Alg. bat_deployment,
// procedures DirectScalarBAT / OfflineCompileLeft).
#include "params.h"

#include <cstring>
#include <stdexcept>

namespace cross {

uint32_t powmod(uint64_t b, uint64_t e, uint32_t q) {
  uint64_t r = 1 % q;
  b %= q;
  while (e) {
    if (e & 1) r = r * b % q;
    b = b * b % q;
    e >>= 1;
  }
  return (uint32_t)r;
}

// Deterministic Miller-Rabin for 32-bit n (bases 2, 7, 61).
bool is_prime_u32(uint32_t n) {
  if (n < 2) return false;
  static const uint32_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 61};
  for (uint32_t p : small) {
    if (n % p == 0) return n == p;
  }
  uint32_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) {
    d >>= 1;
    ++s;
  }
  for (uint32_t a : {2u, 7u, 61u}) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = x * x % n;
      if (x == n - 1) {
        comp = false;
        break;
      }
    }
    if (comp) return false;
  }
  return true;
}

uint32_t smallest_generator(uint32_t q) {
  std::vector<uint32_t> fs;
  uint32_t m = q - 1;
  for (uint32_t p = 2; (uint64_t)p * p <= m; ++p) {
    if (m % p == 0) {
      fs.push_back(p);
      while (m % p == 0) m /= p;
    }
  }
  if (m > 1) fs.push_back(m);
  for (uint32_t g = 2;; ++g) {
    bool ok = true;
    for (uint32_t f : fs) {
      if (powmod(g, (q - 1) / f, q) == 1) {
        ok = false;
        break;
      }
    }
    if (ok) return g;
  }
}

uint32_t root_2n(uint32_t q, uint32_t log_n) {
  uint64_t two_n = 2ull << log_n;
  if ((q - 1) % two_n) throw std::invalid_argument("q != 1 mod 2N");
  return powmod(smallest_generator(q), (q - 1) / two_n, q);
}

uint32_t inv_mod_2_32(uint32_t q) {
  uint32_t x = q;  // Newton iteration: correct to 3 bits, doubles each step
  for (int i = 0; i < 5; ++i) x *= 2u - q * x;
  return x;
}

uint32_t bitrev(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; ++i) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

// Balanced base-256 digits of v: v = sum_i d_i 256^i, d_i in [-128, 127].
static void balanced_digits(int64_t v, int8_t (&d)[kChunks]) {
  for (int i = 0; i < kChunks; ++i) {
    int64_t r = ((v % 256) + 256) % 256;     // v mod 256 in [0, 256)
    if (r >= 128) r -= 256;
    d[i] = (int8_t)r;
    v = (v - r) / 256;
  }
  if (v != 0) throw std::logic_error("balanced_digits: value out of range");
}

void bat_expand(const std::vector<uint32_t>& T, int n_in, int n_out, uint32_t q,
                std::vector<int8_t>& out, bool montgomery) {
  const int M = kChunks * n_out, K = kChunks * n_in;
  if (n_in <= 0 || n_out <= 0 || K % kTileK != 0 || M % 32 != 0 || (size_t)T.size() != (size_t)n_in * n_out)
    throw std::invalid_argument("bat_expand: table shape does not tile");
  const bool wide = wide_prime(q);
  out.assign((size_t)M * K + (wide ? 4 * (size_t)M : 0), 0);
  std::vector<int64_t> rowsum(wide ? M : 0, 0);
  const uint64_t r32 = montgomery ? ((uint64_t)1 << 32) % q : 1;
  // balanced 4-digit range: [-128 * (2^32 - 1) / 255, 127 * (2^32 - 1) / 255]
  const int64_t hi = 127 * (int64_t)0x1010101;
  for (int in = 0; in < n_in; ++in) {
    for (int o = 0; o < n_out; ++o) {
      uint64_t t = (uint64_t)T[(size_t)in * n_out + o] * r32 % q;  // Montgomery form unless plain
      for (int j = 0; j < kChunks; ++j) {
        int8_t c[kChunks];
        if (wide) {
          const uint64_t v = (t << (8 * j)) % q;                      // a * 2^(8 j) mod q: byte j of the input
          balanced_digits((int64_t)v > hi ? (int64_t)v - (int64_t)q : (int64_t)v, c);
        } else {
          const uint64_t v = (t << (kChunkBits * j)) % q;             // a * 2^(bp j) mod q
          for (int i = 0; i < kChunks; ++i) c[i] = (int8_t)((v >> (kChunkBits * i)) & ((1u << kChunkBits) - 1));
        }
        for (int i = 0; i < kChunks; ++i) {
          int m = o * kChunks + i, k = in * kChunks + j;
          if (wide) rowsum[m] += c[i];
          // MFMA fragment order: per 64-deep K slab and 32-row block, two 1 KB
          // fragments (K halves) of 32 rows x 32 K bytes, lane-major
          const size_t blk = (size_t)(k / kTileK) * (M / 32) + m / 32;
          const int half = (k % kTileK) / 32;
          const int lane = (m % 32) + 32 * ((k % 32) / 16);
          out[blk * 2048 + half * 1024 + lane * 16 + (k % 16)] = c[i];
        }
      }
    }
  }
  for (int m = 0; wide && m < M; ++m) {
    const int32_t corr = (int32_t)(128 * rowsum[m]);
    std::memcpy(&out[(size_t)M * K + 4 * (size_t)m], &corr, 4);
  }
}

void build_ntt_tables(uint32_t q, uint32_t log_n, uint32_t log_r, NttTables& t, bool with_bat,
                      uint32_t log_c1) {
  const uint32_t N = 1u << log_n, R = 1u << log_r, C = N / R, N2 = 2 * N;
  const int log_c = (int)(log_n - log_r);
  const uint32_t psi = root_2n(q, log_n);
  std::vector<uint32_t> pw(N2);
  uint64_t x = 1;
  for (uint32_t e = 0; e < N2; ++e) {
    pw[e] = (uint32_t)x;
    x = x * psi % q;
  }
  auto P = [&](int64_t e) { return pw[(uint32_t)(((e % (int64_t)N2) + N2) % N2)]; };
  const uint64_t r32 = ((uint64_t)1 << 32) % q;
  const uint64_t ninv = powmod(N, q - 2, q);

  // Radix-2 butterfly baseline: psi^brv_N(i) and psi^-brv_N(i), Montgomery form.
  t.bf_fwd.resize(N);
  t.bf_inv.resize(N);
  for (uint32_t i = 0; i < N; ++i) {
    uint32_t b = bitrev(i, (int)log_n);
    t.bf_fwd[i] = (uint32_t)(P(b) * r32 % q);
    t.bf_inv[i] = (uint32_t)(P(-(int64_t)b) * r32 % q);
  }
  t.bf_ninv = (uint32_t)(ninv * r32 % q);
  if (!with_bat) return;

  // Step-1 matrix TF1[k][r] = psi^(C r (2 brv_R(k)+1)); as a left-known product
  // Y[k][c] = sum_r TF1[k][r] A[r][c], i.e. "in" = r, "out" = k.
  std::vector<uint32_t> m1((size_t)R * R), im1((size_t)R * R);
  for (uint32_t k = 0; k < R; ++k) {
    int64_t odd = 2 * (int64_t)bitrev(k, (int)log_r) + 1;
    for (uint32_t r = 0; r < R; ++r) {
      m1[(size_t)r * R + k] = P((int64_t)C * r * odd);
      // inverse step 2 (left-known): a[r][c] = sum_k ITF1[r][k] Y[k][c], "in" = k, "out" = r
      im1[(size_t)k * R + r] = (uint32_t)((uint64_t)P(-(int64_t)C * r * odd) * ninv % q);
    }
  }
  bat_expand(m1, R, R, q, t.fwd_left);
  bat_expand(im1, R, R, q, t.inv_left);
  if (!wide_prime(q)) {           // without the Montgomery factor, for the Barrett epilogue
    bat_expand(m1, R, R, q, t.fwd_left_plain, false);
    bat_expand(im1, R, R, q, t.inv_left_plain, false);
  }

  auto shoup = [&](uint32_t w) { return (uint32_t)(((uint64_t)w << 32) / q); };
  if (log_c1 > 0) {
    if (log_c1 >= (uint32_t)log_c) throw std::invalid_argument("three-factor split needs C1 < C");
    // Row transform split as C1 x C2 (c = c1 C2 + c2, c' = m C2 + c2'):
    //   TB[m][c1] = psi^(2R C2 c1 brv_C1(m))    (left product over c1: "in" = c1, "out" = m)
    //   T3[m][c2] = psi^(2R c2 brv_C1(m))       (twiddle, pairs [m][c2])
    //   TC[c2][c2'] = psi^(2R C1 c2 brv_C2(c2')) (right product over c2: "in" = c2, "out" = c2')
    // inverse (no scaling; N^-1 is in the step-1 matrix): ITC over c2' then IT3, ITB over m.
    const uint32_t C1 = 1u << log_c1, C2 = C / C1;
    const int lc1 = (int)log_c1, lc2 = log_c - (int)log_c1;
    std::vector<uint32_t> tb((size_t)C1 * C1), itb((size_t)C1 * C1), tc((size_t)C2 * C2), itc((size_t)C2 * C2);
    for (uint32_t c1 = 0; c1 < C1; ++c1)
      for (uint32_t m = 0; m < C1; ++m) {
        const int64_t e = 2 * (int64_t)R * C2 * c1 * bitrev(m, lc1);
        tb[(size_t)c1 * C1 + m] = P(e);      // in c1, out m
        itb[(size_t)m * C1 + c1] = P(-e);    // in m, out c1
      }
    for (uint32_t c2 = 0; c2 < C2; ++c2)
      for (uint32_t cp = 0; cp < C2; ++cp) {
        const int64_t e = 2 * (int64_t)R * C1 * c2 * bitrev(cp, lc2);
        tc[(size_t)c2 * C2 + cp] = P(e);     // in c2, out c2'
        itc[(size_t)cp * C2 + c2] = P(-e);   // in c2', out c2
      }
    bat_expand(tb, C1, C1, q, t.row_fwd_b);
    bat_expand(tc, C2, C2, q, t.row_fwd_c);
    bat_expand(itc, C2, C2, q, t.row_inv_c);
    bat_expand(itb, C1, C1, q, t.row_inv_b);
    // the same four without the Montgomery factor, for the Barrett epilogue
    // (narrow primes only: the wide form has no Barrett epilogue)
    if (!wide_prime(q)) {
      bat_expand(tb, C1, C1, q, t.row_fwd_b_plain, false);
      bat_expand(tc, C2, C2, q, t.row_fwd_c_plain, false);
      bat_expand(itc, C2, C2, q, t.row_inv_c_plain, false);
      bat_expand(itb, C1, C1, q, t.row_inv_b_plain, false);
    }
    t.row_fwd_t3.resize((size_t)2 * C);
    t.row_fwd_t3_mont.resize((size_t)2 * C);
    t.row_inv_t3.resize((size_t)2 * C);
    for (uint32_t m = 0; m < C1; ++m)
      for (uint32_t c2 = 0; c2 < C2; ++c2) {
        const int64_t e = 2 * (int64_t)R * c2 * bitrev(m, lc1);
        const uint32_t wf = P(e), wi = P(-e);
        // T3 pairs [m][c2], IT3 pairs [c2][m]: each in the order the kernel's
        // lanes read them (consecutive c2, resp. consecutive m, across a wave)
        const size_t f = 2 * ((size_t)m * C2 + c2), g = 2 * ((size_t)c2 * C1 + m);
        t.row_fwd_t3[f] = wf;
        t.row_fwd_t3[f + 1] = shoup(wf);
        const uint32_t wm = (uint32_t)(((uint64_t)wf << 32) % q);
        t.row_fwd_t3_mont[f] = wm;
        t.row_fwd_t3_mont[f + 1] = shoup(wm);
        t.row_inv_t3[g] = wi;
        t.row_inv_t3[g + 1] = shoup(wi);
      }
    // step-2 twiddles: forward [k][c] as in the two-factor form; the inverse ones
    // row-major too (applied by the row kernel's last epilogue)
    t.fwd_tw.resize((size_t)2 * R * C);
    t.inv_tw_rows.resize((size_t)2 * R * C);
    for (uint32_t k = 0; k < R; ++k) {
      int64_t odd = 2 * (int64_t)bitrev(k, (int)log_r) + 1;
      for (uint32_t c = 0; c < C; ++c) {
        const uint32_t wf = P((int64_t)c * odd), wi = P(-(int64_t)c * odd);
        const size_t f = 2 * ((size_t)k * C + c);
        t.fwd_tw[f] = wf;
        t.fwd_tw[f + 1] = shoup(wf);
        t.inv_tw_rows[f] = wi;
        t.inv_tw_rows[f + 1] = shoup(wi);
      }
    }
    return;
  }

  // Step-3 matrix TF3[c][c'] = psi^(2R c brv_C(c')): out[k][c'] = sum_c Y[k][c] TF3[c][c'],
  // "in" = c, "out" = c'.  Inverse step 1: Y[k][c] = sum_c' Ahat[k][c'] ITF3[c'][c].
  std::vector<uint32_t> m3((size_t)C * C), im3((size_t)C * C);
  for (uint32_t c = 0; c < C; ++c) {
    for (uint32_t cp = 0; cp < C; ++cp) {
      int64_t e = 2 * (int64_t)R * c * bitrev(cp, log_c);
      m3[(size_t)c * C + cp] = P(e);
      im3[(size_t)cp * C + c] = P(-e);
    }
  }
  bat_expand(m3, C, C, q, t.fwd_right);
  bat_expand(im3, C, C, q, t.inv_right);
  if (!wide_prime(q)) {
    bat_expand(m3, C, C, q, t.fwd_right_plain, false);
    bat_expand(im3, C, C, q, t.inv_right_plain, false);
  }

  // Step-2 twiddles T2[k][c] = psi^(c (2 brv_R(k)+1)), stored [k][c] (left kernel epilogue);
  // inverse twiddles IT2[k][c] = psi^(-c (2 brv_R(k)+1)), stored transposed [c][k]
  // (right kernel epilogue, whose lanes run along k).  Each entry is the pair
  // (w, floor(w * 2^32 / q)) for Shoup multiplication.
  t.fwd_tw.resize((size_t)2 * R * C);
  t.inv_tw.resize((size_t)2 * R * C);
  for (uint32_t k = 0; k < R; ++k) {
    int64_t odd = 2 * (int64_t)bitrev(k, (int)log_r) + 1;
    for (uint32_t c = 0; c < C; ++c) {
      const uint32_t wf = P((int64_t)c * odd), wi = P(-(int64_t)c * odd);
      const size_t f = 2 * ((size_t)k * C + c), i = 2 * ((size_t)c * R + k);
      t.fwd_tw[f] = wf;
      t.fwd_tw[f + 1] = shoup(wf);
      t.inv_tw[i] = wi;
      t.inv_tw[i + 1] = shoup(wi);
    }
  }
}

}  // namespace cross
