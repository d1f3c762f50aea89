// Host side of VecModMul with a pre-known operand under a chosen modular
// reduction (Sec. Evaluation "Impact of Modular Reduction Algorithm"; App.
// "BAT for Modular Reduction").
#include <cstring>
#include <string>
#include <vector>

#include "context.h"
#include "params.h"

namespace cross {

ModLimb mod_limb(uint32_t q) {
  ModLimb m{};
  uint32_t k = 0;
  while ((1ull << k) <= q) ++k;           // bit length
  m.q = q;
  m.qinv = inv_mod_2_32(q);
  m.bar_k = k;
  m.bar_m = (uint32_t)(((unsigned __int128)1 << (2 * k)) / q);
  m.r32 = (uint32_t)((1ull << 32) % q);
  return m;
}

// A operand of the BAT-lazy MFMA for prime q (1 KB, lane l holding row l % 32
// and K bytes 16 (l / 32) .. +15).  K segment s (bytes 4s .. 4s + 3) carries the
// high chunks c_4 .. c_7 of element s % 4 of the lanes with l / 32 = s / 4; row
// block 2 (s % 4) + s / 4 gets the chunk matrix LC[j][k] = chunk k of
// 2^(7 (4 + j)) mod q at (row 4b + k, byte 4s + j), zero elsewhere.
std::vector<int8_t> lazy_fragment(uint32_t q) {
  uint32_t lc[4][4];
  for (int j = 0; j < 4; ++j) {
    const uint32_t v = powmod(2, 7 * (4 + j), q);
    for (int k = 0; k < 4; ++k) lc[j][k] = (v >> (7 * k)) & 0x7f;
  }
  std::vector<int8_t> f(1024, 0);
  for (int lane = 0; lane < 64; ++lane)
    for (int e = 0; e < 16; ++e) {
      const int row = lane & 31, kb = 16 * (lane >> 5) + e;
      const int s = kb / 4, j = kb % 4, b = row / 4, k = row % 4;
      if (b == 2 * (s % 4) + s / 4) f[lane * 16 + e] = (int8_t)lc[j][k];
    }
  return f;
}

namespace {

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

cross_status modmul_setup(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, int method,
                          const ModLimb** limbs, const int8_t** lazy) {
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  if (!primes) return fail(ctx, CROSS_EINVAL, "null primes");
  if (method < kModredBarrett || method > kModredBatLazy) return fail(ctx, CROSS_EINVAL, "unknown reduction method");
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS)
    return fail(ctx, CROSS_EINVAL, "bad shape");
  if (method == kModredBatLazy && log_n < 8)
    return fail(ctx, CROSS_EUNSUPPORTED, "BAT-lazy reduction needs N >= 256 (one prime per wave)");
  std::vector<ModLimb> m(L);
  std::vector<int8_t> frag;
  for (uint32_t i = 0; i < L; ++i) {
    cross_status st = check_prime(ctx, primes[i], log_n);
    if (st != CROSS_OK) return st;
    m[i] = mod_limb(primes[i]);
    if (method == kModredBatLazy) {
      const std::vector<int8_t> f = lazy_fragment(primes[i]);
      frag.insert(frag.end(), f.begin(), f.end());
    }
  }
  void* d = nullptr;
  cross_status st = cached_device_copy(ctx, m.data(), m.size() * sizeof(ModLimb), &d);
  if (st != CROSS_OK) return st;
  *limbs = (const ModLimb*)d;
  *lazy = nullptr;
  if (method == kModredBatLazy) {
    void* f = nullptr;
    if ((st = cached_device_copy(ctx, frag.data(), frag.size(), &f)) != CROSS_OK) return st;
    *lazy = (const int8_t*)f;
  }
  return CROSS_OK;
}

}  // namespace
}  // namespace cross

using namespace cross;

extern "C" {

cross_status cross_vec_modmul_prepare(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                                      int method, const uint32_t* w, uint32_t* w_prep, void* stream) {
  if (!ctx) return CROSS_EINVAL;
  if (!w || !w_prep) return fail(ctx, CROSS_EINVAL, "null buffer");
  const ModLimb* limbs = nullptr;
  const int8_t* lazy = nullptr;
  cross_status st = modmul_setup(ctx, log_n, primes, L, method, &limbs, &lazy);
  if (st != CROSS_OK) return st;
  const uint64_t n = (uint64_t)L << log_n;
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(w), b0 = reinterpret_cast<uintptr_t>(w_prep);
  if (a0 < b0 + 2 * n * 4 && b0 < a0 + n * 4) return fail(ctx, CROSS_EINVAL, "w_prep must not overlap w");
  hipStream_t s = (hipStream_t)stream;
  if (aligned16(w) && (st = check_residues(ctx, "w", w, n, 1, primes, (int)L, (int)log_n, s)) != CROSS_OK) return st;
  ProfScope ps(ctx, "modmul_prepare", s);
  const hipError_t e = launch_modmul_prepare(w, w_prep, w_prep + n, limbs, (int)L, (int)log_n, method, s);
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("prepare launch: ") + hipGetErrorString(e));
  return CROSS_OK;
}

cross_status cross_vec_modmul(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                              uint32_t npoly, int method, const uint32_t* a, const uint32_t* w_prep,
                              uint32_t* out, void* stream) {
  if (!ctx) return CROSS_EINVAL;
  if (!a || !w_prep || !out || !aligned16(a) || !aligned16(w_prep) || !aligned16(out) || npoly < 1)
    return fail(ctx, CROSS_EINVAL, "null or misaligned buffer, or npoly < 1");
  const ModLimb* limbs = nullptr;
  const int8_t* lazy = nullptr;
  cross_status st = modmul_setup(ctx, log_n, primes, L, method, &limbs, &lazy);
  if (st != CROSS_OK) return st;
  const uint64_t n = (uint64_t)L << log_n;
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_residues(ctx, "a", a, n, (int)npoly, primes, (int)L, (int)log_n, s)) != CROSS_OK) return st;
  ProfScope ps(ctx, "vec_modmul", s);
  const hipError_t e = launch_vec_modmul(a, w_prep, w_prep + n, out, limbs, lazy, (int)L, (int)log_n, (int)npoly,
                                         method, s);
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("vec_modmul launch: ") + hipGetErrorString(e));
  return CROSS_OK;
}

}  // extern "C"
