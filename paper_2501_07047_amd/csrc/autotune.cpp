// Autotuner: choose how a transform size is factored -- the two-factor split
// N = R x C with a GEMM workgroup tile, or a three-factor split R x C1 x C2 --
// by timing the candidates on the device (the paper sweeps (R, C) in
// {(128,512), (256,256), (512,128)} for its HE operators and keeps the best;
// here every two-factor split within a factor 4 of square with every tile, and
// every three-factor split with 16 <= C1, C2 <= 32, is timed).  Results can be
// kept in a text cache file, one line per choice:
// "<device> <log_n> <L> <batch> <log_r> <log_c1> <tile> <microseconds> <two-factor log_r>".
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

struct Choice {
  uint32_t log_r = 0, log_c1 = 0;   // log_c1 = 0: two factors
  int tile = 0;
  double us = 1e30;
  uint32_t log_r2 = 0;              // best two-factor split (the batch runtime's)
};

bool cache_lookup(const char* path, const std::string& dev, uint32_t log_n, uint32_t L, uint32_t batch,
                  Choice* c) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string d;
    uint32_t n, l, b, r, c1, r2;
    int t;
    double u;
    if (in >> d >> n >> l >> b >> r >> c1 >> t >> u >> r2)
      if (d == dev && n == log_n && l == L && b == batch) {
        c->log_r = r;
        c->log_c1 = c1;
        c->tile = t;
        c->us = u;
        c->log_r2 = r2;
        found = true;   // the last matching line wins
      }
  }
  return found;
}

void apply(cross_ctx ctx, uint32_t log_n, const Choice& c) {
  ctx->split[(int)log_n] = (int)c.log_r2;
  ctx->split3[(int)log_n] = std::make_pair((int)c.log_r, (int)c.log_c1);
  ctx->tile_by_logn[(int)log_n] = c.tile;
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
                            uint32_t* log_r_out, uint32_t* log_c1_out, int* tile_out, double* us_out) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < 8 || log_n > CROSS_MAX_LOG_N || L < 1 || L > CROSS_MAX_LIMBS || batch < 1)
    return fail(ctx, CROSS_EINVAL, "autotune needs 8 <= log_n <= 16, 1 <= L <= 64, batch >= 1");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  const std::string dev = device_tag(ctx->device);
  Choice best;
  auto report = [&]() {
    if (log_r_out) *log_r_out = best.log_r;
    if (log_c1_out) *log_c1_out = best.log_c1;
    if (tile_out) *tile_out = best.tile;
    if (us_out) *us_out = best.us;
  };
  if (cache_lookup(cache_path, dev, log_n, L, batch, &best)) {
    apply(ctx, log_n, best);
    report();
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
  const auto saved3 = ctx->split3.find((int)log_n) != ctx->split3.end()
                          ? std::make_pair(true, ctx->split3[(int)log_n]) : std::make_pair(false, std::make_pair(0, 0));
  cross_status st = CROSS_OK;
  // time forward + inverse with the context set to (lr, lc1, tile)
  auto time_one = [&](int lr, int lc1, int tile, double* us) {
    ctx->split3[(int)log_n] = std::make_pair(lr, lc1);
    ctx->gemm_tile = tile;
    for (int w = 0; w < 2 && st == CROSS_OK; ++w) {
      st = cross_ntt_forward(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
      if (st == CROSS_OK) st = cross_ntt_inverse(ctx, log_n, primes.data(), L, batch, (uint32_t*)data, nullptr);
    }
    if (st != CROSS_OK) return;
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
    *us = ms * 1e3 / reps;
  };
  // two factors: splits near square x every distinct tile pair
  double best2 = 1e30;
  const int half = (int)log_n / 2;
  // from N = 2^12 up, keep R, C >= 64 so the batch runtime's 256-row work-list tiles can use the choice
  const int lo_r = std::max(log_n >= 12 ? 6 : 4, half - 1);
  const int hi_r = std::min((int)log_n - (log_n >= 12 ? 6 : 4), half + 1);
  for (int lr = lo_r; lr <= hi_r && st == CROSS_OK; ++lr) {
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
      double us = 1e30;
      time_one(lr, 0, tile, &us);
      if (st != CROSS_OK) break;
      if (us < best2) {
        best2 = us;
        best.log_r2 = (uint32_t)lr;
      }
      if (us < best.us) {
        best.us = us;
        best.log_r = (uint32_t)lr;
        best.log_c1 = 0;
        best.tile = tile;
      }
    }
  }
  // three factors (the row kernels with 16 <= C1, C2 <= 32), row-side tile automatic
  for (int lr = 4; lr <= (int)log_n - 8 && st == CROSS_OK; ++lr)
    for (int lc1 = 4; lc1 <= 5 && st == CROSS_OK; ++lc1) {
      const int lc2 = (int)log_n - lr - lc1;
      if (lc2 < 4 || lc2 > 5 || !rows_split_supported((int)log_n, lr, lc1)) continue;
      double us = 1e30;
      time_one(lr, lc1, 0, &us);
      if (st == CROSS_OK && us < best.us) {
        best.us = us;
        best.log_r = (uint32_t)lr;
        best.log_c1 = (uint32_t)lc1;
        best.tile = 0;
      }
    }
  ctx->gemm_tile = saved_tile;
  if (saved3.first) ctx->split3[(int)log_n] = saved3.second;
  else ctx->split3.erase((int)log_n);
  // batch runtime (log_n >= 12): the work-list tile of its GEMM steps, per direction,
  // timed on one NTT job of the same shape through a batch (the runtime's own split:
  // three factors R x 32 x 32 from 2^14 up, else the best two-factor split above)
  if (st == CROSS_OK && log_n >= 12) {
    ctx->split[(int)log_n] = (int)best.log_r2;
    for (int inv = 0; inv < 2 && st == CROSS_OK; ++inv) {
      const int key = 2 * (int)log_n + inv;
      const auto saved_lt = ctx->list_tile.find(key);
      const bool had = saved_lt != ctx->list_tile.end();
      const int old_lt = had ? saved_lt->second : 0;
      cross_job job{};
      job.op = inv ? CROSS_OP_NTT_INVERSE : CROSS_OP_NTT_FORWARD;
      job.params.log_n = log_n;
      job.params.L = L;
      job.params.primes = primes.data();
      job.batch = batch;
      job.data = (uint32_t*)data;
      double best_us = 1e30;
      int best_tile = -1;
      for (int lt = 0; lt < kListTileCount && st == CROSS_OK; ++lt) {
        ctx->list_tile[key] = lt;
        cross_batch bt = nullptr;
        if (cross_batch_create(ctx, &job, 1, 0, &bt) != CROSS_OK) continue;   // tile does not fit: skip
        double us = 1e30;
        for (int w = 0; w < 2; ++w) (void)cross_batch_run(bt, nullptr);
        const int reps = 5;
        (void)hipEventRecord(e0, nullptr);
        for (int k = 0; k < reps; ++k) (void)cross_batch_run(bt, nullptr);
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) == hipSuccess) us = ms * 1e3 / reps;
        cross_batch_destroy(bt);
        if (us < best_us) {
          best_us = us;
          best_tile = lt;
        }
      }
      if (best_tile >= 0) ctx->list_tile[key] = best_tile;
      else if (had) ctx->list_tile[key] = old_lt;
      else ctx->list_tile.erase(key);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(data);
  if (st != CROSS_OK) return st;
  apply(ctx, log_n, best);
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "a")) {
      std::fprintf(f, "%s %u %u %u %u %u %d %.3f %u\n", dev.c_str(), log_n, L, batch, best.log_r, best.log_c1,
                   best.tile, best.us, best.log_r2);
      std::fclose(f);
    }
  }
  report();
  return CROSS_OK;
}

}  // extern "C"
