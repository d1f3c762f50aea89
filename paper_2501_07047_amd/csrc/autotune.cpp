// Autotuner: choose the 3-step split N = R x C and the GEMM workgroup tile for a
// transform size by timing the candidates on the device (the paper sweeps
// (R, C) in {(128,512), (256,256), (512,128)} for its HE operators and keeps
// the best; here every split with R, C >= 16 within a factor 4 of square, and
// every tile, is timed).  Results can be kept in a text cache file, one line
// per choice: "<device> <log_n> <L> <batch> <log_r> <tile> <microseconds>".
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <set>
#include <string>

#include "context.h"
#include "params.h"

using namespace cross;

namespace {

std::string device_tag(int dev) {
  hipDeviceProp_t p;
  if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string s = std::string(p.gcnArchName) + ":" + std::to_string(p.multiProcessorCount) + "cu";
  for (char& c : s)
    if (c == ' ') c = '_';
  return s;
}

bool cache_lookup(const char* path, const std::string& dev, uint32_t log_n, uint32_t L, uint32_t batch,
                  uint32_t* log_r, int* tile, double* us) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string d;
    uint32_t n, l, b, r;
    int t;
    double u;
    if (in >> d >> n >> l >> b >> r >> t >> u)
      if (d == dev && n == log_n && l == L && b == batch) {
        *log_r = r;
        *tile = t;
        *us = u;
        found = true;   // the last matching line wins
      }
  }
  return found;
}

std::vector<uint32_t> tuning_primes(uint32_t count) {
  std::vector<uint32_t> out;
  for (uint32_t m = ((1u << 28) - 2) >> 17; m > 0 && out.size() < count; --m) {
    uint32_t q = (m << 17) + 1;
    if (is_prime_u32(q)) out.push_back(q);
  }
  return out;
}

}  // namespace

extern "C" {

cross_status cross_autotune(cross_ctx ctx, uint32_t log_n, uint32_t L, uint32_t batch, const char* cache_path,
                            uint32_t* log_r_out, int* tile_out, double* us_out) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < 8 || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS || batch < 1)
    return fail(ctx, CROSS_EINVAL, "autotune needs 8 <= log_n <= 16, 1 <= L <= 64, batch >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  const std::string dev = device_tag(ctx->device);
  uint32_t best_r = 0;
  int best_t = 0;
  double best_us = 0;
  if (cache_lookup(cache_path, dev, log_n, L, batch, &best_r, &best_t, &best_us)) {
    ctx->split[(int)log_n] = (int)best_r;
    ctx->tile_by_logn[(int)log_n] = best_t;
    if (log_r_out) *log_r_out = best_r;
    if (tile_out) *tile_out = best_t;
    if (us_out) *us_out = best_us;
    return CROSS_OK;
  }
  const std::vector<uint32_t> primes = tuning_primes(L);
  const uint64_t words = (uint64_t)batch * L << log_n;
  void* data = nullptr;
  if (hipMalloc(&data, words * 4) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CROSS_ENOMEM, "autotune buffer allocation failed");
  }
  (void)hipMemset(data, 0, words * 4);   // zero is a valid residue; timing does not depend on values
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int saved_tile = ctx->gemm_tile;
  best_us = 1e30;
  cross_status st = CROSS_OK;
  const int half = (int)log_n / 2;
  // from N = 2^12 up, keep R, C >= 64 so the batch runtime's 256-row work-list tiles can use the choice
  const int lo_r = std::max(log_n >= 12 ? 6 : 4, half - 1);
  const int hi_r = std::min((int)log_n - (log_n >= 12 ? 6 : 4), half + 1);
  for (int lr = lo_r; lr <= hi_r && st == CROSS_OK; ++lr) {
    ctx->split[(int)log_n] = lr;
    std::set<std::pair<int, int>> timed;   // (row-side, column-side) tiles as launched
    for (int tile = 1; tile < kTileCount && st == CROSS_OK; ++tile) {
      // a tile that does not fit this split falls back to another one: time each pair once
      GemmLaunch g{};
      g.njobs = (int)L;
      g.npoly = (int)batch;
      g.log_r = lr;
      g.log_c = (int)log_n - lr;
      g.tile = tile;
      g.kind = kLeft;
      const int t_left = resolve_gemm_tile(g);
      g.kind = kRight;
      const int t_right = resolve_gemm_tile(g);
      if (!timed.insert({t_left, t_right}).second) continue;
      ctx->gemm_tile = tile;
      for (int w = 0; w < 2 && st == CROSS_OK; ++w) {
        st = cross_ntt_forward(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
        if (st == CROSS_OK) st = cross_ntt_inverse(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
      }
      if (st != CROSS_OK) break;
      const int reps = 5;
      (void)hipEventRecord(e0, nullptr);
      for (int k = 0; k < reps && st == CROSS_OK; ++k) {
        st = cross_ntt_forward(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
        if (st == CROSS_OK) st = cross_ntt_inverse(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
      }
      (void)hipEventRecord(e1, nullptr);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      const double us = ms * 1e3 / reps;
      if (st == CROSS_OK && us < best_us) {
        best_us = us;
        best_r = (uint32_t)lr;
        best_t = tile;
      }
    }
  }
  ctx->gemm_tile = saved_tile;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(data);
  if (st != CROSS_OK) return st;
  ctx->split[(int)log_n] = (int)best_r;
  ctx->tile_by_logn[(int)log_n] = best_t;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %u %u %u %u %d %.3f\n", dev.c_str(), log_n, L, batch, best_r, best_t, best_us);
      std::fclose(f);
    }
  }
  if (log_r_out) *log_r_out = best_r;
  if (tile_out) *tile_out = best_t;
  if (us_out) *us_out = best_us;
  return CROSS_OK;
}

}  // extern "C"
