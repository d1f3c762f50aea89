// Context, plan cache and the NTT entry points of the C ABI.
#include "context.h"

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <stdexcept>

#include "params.h"

namespace cross {

cross_status fail(cross_ctx ctx, cross_status code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

cross_status check_prime(cross_ctx ctx, uint32_t q, uint32_t log_n, bool wide_ok) {
  if (q >= kWidePrimeLimit || (!wide_ok && wide_prime(q)))
    return fail(ctx, CROSS_ERANGE, "modulus " + std::to_string(q) + (wide_ok ? " >= 2^31" : " >= 2^28"));
  if (q < 3 || !is_prime_u32(q)) return fail(ctx, CROSS_ENOTPRIME, "modulus " + std::to_string(q) + " is not prime");
  if ((q - 1) % (2ull << log_n)) return fail(ctx, CROSS_ENOROOT, "modulus " + std::to_string(q) + " != 1 mod 2N");
  return CROSS_OK;
}

LaunchEvents& launch_events() {
  thread_local LaunchEvents ev;
  return ev;
}

ProfScope::ProfScope(cross_ctx c, const char* name, hipStream_t st, bool mk) : ctx(c), s(st), markers(mk) {
  if (!ctx || !ctx->prof || (!ctx->prof_only.empty() && ctx->prof_only != name)) return;
  cross_ctx_s::ProfRec r{name, nullptr, nullptr, false};
  // events come from the context's pool (creating events per launch costs more host
  // time than the launches themselves)
  auto take = [&](hipEvent_t* e) {
    if (!ctx->prof_pool.empty()) {
      *e = ctx->prof_pool.back();
      ctx->prof_pool.pop_back();
      return true;
    }
    return hipEventCreate(e) == hipSuccess;
  };
  if (!take(&r.a)) return;
  if (!take(&r.b)) {
    ctx->prof_pool.push_back(r.a);
    return;
  }
  if (markers) {
    (void)hipEventRecord(r.a, s);
  } else {
    prev = launch_events();
    launch_events() = LaunchEvents{r.a, r.b, 0};
  }
  idx = (int)ctx->prof_recs.size();
  ctx->prof_recs.push_back(r);
}

ProfScope::~ProfScope() {
  if (idx < 0) return;
  auto& r = ctx->prof_recs[idx];
  if (markers) {
    r.valid = hipEventRecord(r.b, s) == hipSuccess;
  } else {
    r.valid = launch_events().stamped > 0;
    launch_events() = prev;
  }
}

int split_of(cross_ctx ctx, int log_n) {
  auto it = ctx->split.find(log_n);
  if (it != ctx->split.end()) return it->second;
  return log_n / 2;
}

static cross_status dev_alloc(cross_ctx ctx, size_t bytes, void** out) {
  if (hipMalloc(out, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, CROSS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return CROSS_OK;
}

bool default_split3(int log_n, int* log_r, int* log_c1) {
  // measured fastest three-factor splits (N = 2^13 .. 2^16, 24 limbs x 16 polynomials)
  switch (log_n) {
    case 13: *log_r = 5; *log_c1 = 4; return true;
    case 14: *log_r = 5; *log_c1 = 5; return true;
    case 15: *log_r = 6; *log_c1 = 5; return true;
    case 16: *log_r = 6; *log_c1 = 5; return true;
    default: return false;
  }
}

void effective_split(cross_ctx ctx, int log_n, bool allow3, int* log_r, int* log_c1) {
  *log_r = (log_n >= 8) ? split_of(ctx, log_n) : 0;
  *log_c1 = 0;
  if (!allow3 || log_n < 8) return;
  auto s3 = ctx->split3.find(log_n);
  if (s3 != ctx->split3.end()) {
    *log_r = s3->second.first;
    *log_c1 = s3->second.second;
    return;
  }
  int r = 0, c1 = 0;
  if (default_split3(log_n, &r, &c1)) {
    *log_r = r;
    *log_c1 = c1;
  }
}

cross_status get_plan(cross_ctx ctx, uint32_t q, int log_n, Plan** out, bool allow3) {
  int log_r = 0, log_c1 = 0;
  effective_split(ctx, log_n, allow3, &log_r, &log_c1);
  return get_plan_at(ctx, q, log_n, log_r, log_c1, out);
}

cross_status get_plan_at(cross_ctx ctx, uint32_t q, int log_n, int log_r, int log_c1, Plan** out) {
  auto key = std::make_tuple(q, log_n, log_r, log_c1);
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    *out = it->second;
    return CROSS_OK;
  }
  NttTables t;
  try {
    // below N = 2^8 a 3-step split cannot fill one 64-deep MFMA step: butterfly twiddles only
    build_ntt_tables(q, log_n, log_r, t, log_n >= 8, (uint32_t)log_c1);
  } catch (const std::exception& e) {
    return fail(ctx, CROSS_EINVAL, e.what());
  }
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t sz = al(t.fwd_left.size()) + al(t.fwd_right.size()) + al(t.inv_left.size()) +
              al(t.inv_right.size()) + al(t.fwd_tw.size() * 4) + al(t.inv_tw.size() * 4) +
              al(t.bf_fwd.size() * 4) + al(t.bf_inv.size() * 4) + al(t.row_fwd_b.size()) +
              al(t.row_fwd_c.size()) + al(t.row_inv_c.size()) + al(t.row_inv_b.size()) +
              al(t.row_fwd_t3.size() * 4) + al(t.row_inv_t3.size() * 4) + al(t.inv_tw_rows.size() * 4) +
              al(t.row_fwd_t3_mont.size() * 4) +
              al(t.row_fwd_b_plain.size()) + al(t.row_fwd_c_plain.size()) + al(t.row_inv_c_plain.size()) +
              al(t.row_inv_b_plain.size()) + al(t.fwd_left_plain.size()) + al(t.fwd_right_plain.size()) +
              al(t.inv_left_plain.size()) + al(t.inv_right_plain.size());
  Plan* p = new Plan();
  cross_status st = dev_alloc(ctx, sz, &p->block);
  if (st != CROSS_OK) {
    delete p;
    return st;
  }
  char* base = static_cast<char*>(p->block);
  size_t off = 0;
  auto put = [&](const void* src, size_t bytes) -> void* {
    void* dst = base + off;
    if (bytes) (void)hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    off += al(bytes);
    return bytes ? dst : nullptr;
  };
  p->fwd_left = (int8_t*)put(t.fwd_left.data(), t.fwd_left.size());
  p->fwd_right = (int8_t*)put(t.fwd_right.data(), t.fwd_right.size());
  p->inv_left = (int8_t*)put(t.inv_left.data(), t.inv_left.size());
  p->inv_right = (int8_t*)put(t.inv_right.data(), t.inv_right.size());
  p->fwd_left_plain = (int8_t*)put(t.fwd_left_plain.data(), t.fwd_left_plain.size());
  p->fwd_right_plain = (int8_t*)put(t.fwd_right_plain.data(), t.fwd_right_plain.size());
  p->inv_left_plain = (int8_t*)put(t.inv_left_plain.data(), t.inv_left_plain.size());
  p->inv_right_plain = (int8_t*)put(t.inv_right_plain.data(), t.inv_right_plain.size());
  p->fwd_tw = (uint32_t*)put(t.fwd_tw.data(), t.fwd_tw.size() * 4);
  p->inv_tw = (uint32_t*)put(t.inv_tw.data(), t.inv_tw.size() * 4);
  p->bf_fwd = (uint32_t*)put(t.bf_fwd.data(), t.bf_fwd.size() * 4);
  p->bf_inv = (uint32_t*)put(t.bf_inv.data(), t.bf_inv.size() * 4);
  p->row_fwd_b = (int8_t*)put(t.row_fwd_b.data(), t.row_fwd_b.size());
  p->row_fwd_c = (int8_t*)put(t.row_fwd_c.data(), t.row_fwd_c.size());
  p->row_inv_c = (int8_t*)put(t.row_inv_c.data(), t.row_inv_c.size());
  p->row_inv_b = (int8_t*)put(t.row_inv_b.data(), t.row_inv_b.size());
  p->row_fwd_t3 = (uint32_t*)put(t.row_fwd_t3.data(), t.row_fwd_t3.size() * 4);
  p->row_fwd_t3_mont = (uint32_t*)put(t.row_fwd_t3_mont.data(), t.row_fwd_t3_mont.size() * 4);
  p->row_inv_t3 = (uint32_t*)put(t.row_inv_t3.data(), t.row_inv_t3.size() * 4);
  p->inv_tw_rows = (uint32_t*)put(t.inv_tw_rows.data(), t.inv_tw_rows.size() * 4);
  p->row_fwd_b_plain = (int8_t*)put(t.row_fwd_b_plain.data(), t.row_fwd_b_plain.size());
  p->row_fwd_c_plain = (int8_t*)put(t.row_fwd_c_plain.data(), t.row_fwd_c_plain.size());
  p->row_inv_c_plain = (int8_t*)put(t.row_inv_c_plain.data(), t.row_inv_c_plain.size());
  p->row_inv_b_plain = (int8_t*)put(t.row_inv_b_plain.data(), t.row_inv_b_plain.size());
  {
    uint32_t k = 0;
    while ((1ull << k) <= q) ++k;
    p->bar_k = k;
    p->bar_m = (uint32_t)(((unsigned __int128)1 << (2 * k)) / q);
  }
  if (hipGetLastError() != hipSuccess) {
    (void)hipFree(p->block);
    delete p;
    return fail(ctx, CROSS_EDEVICE, "table upload failed");
  }
  p->q = q;
  p->qinv = inv_mod_2_32(q);
  p->psi = root_2n(q, log_n);
  p->log_n = log_n;
  p->log_r = log_r;
  p->log_c1 = log_c1;
  p->bf_ninv = t.bf_ninv;
  p->wide = wide_prime(q);
  ctx->plans[key] = p;
  *out = p;
  return CROSS_OK;
}

cross_status cached_device_copy(cross_ctx ctx, const void* host, size_t bytes, void** out) {
  if (ctx->arena.base) {
    // no-alloc call: a stream-ordered copy into the arena (later calls on the same
    // stream overwrite it only after this call's kernels have run)
    cross_ctx_s::Arena& a = ctx->arena;
    const size_t at = (a.used + 255) & ~(size_t)255;
    if (at + bytes > a.cap) return fail(ctx, CROSS_EINVAL, "job lists exceed the no-alloc scratch head");
    if (bytes && hipMemcpyAsync(a.base + at, host, bytes, hipMemcpyHostToDevice, a.stream) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, CROSS_EDEVICE, "job list copy failed");
    }
    a.used = at + bytes;
    *out = a.base + at;
    return CROSS_OK;
  }
  std::string key(static_cast<const char*>(host), bytes);
  auto it = ctx->job_cache.find(key);
  if (it != ctx->job_cache.end()) {
    *out = it->second;
    return CROSS_OK;
  }
  void* d = nullptr;
  cross_status st = dev_alloc(ctx, bytes ? bytes : 16, &d);
  if (st != CROSS_OK) return st;
  if (hipMemcpy(d, host, bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return fail(ctx, CROSS_EDEVICE, "job list upload failed");
  }
  ctx->job_cache[key] = d;
  *out = d;
  return CROSS_OK;
}

cross_status pinned_acquire(cross_ctx ctx, size_t bytes, int* idx) {
  int best = -1;
  for (size_t i = 0; i < ctx->pinned.size(); ++i) {
    const auto& b = ctx->pinned[i];
    if (!b.busy && b.size >= bytes && (best < 0 || b.size < ctx->pinned[best].size)) best = (int)i;
  }
  if (best < 0) {
    cross_ctx_s::Pinned b;
    b.size = std::max<size_t>(bytes, 64 << 10);
    if (hipHostMalloc(&b.p, b.size, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, CROSS_ENOMEM, "pinned host allocation failed");
    }
    if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(b.p);
      return fail(ctx, CROSS_EDEVICE, "event creation failed");
    }
    ctx->pinned.push_back(b);
    best = (int)ctx->pinned.size() - 1;
  } else if (hipEventSynchronize(ctx->pinned[best].ev) != hipSuccess) {
    // its previous copy must have left the buffer (normally long done)
    (void)hipGetLastError();
    return fail(ctx, CROSS_EDEVICE, "waiting for a pinned buffer's copy failed");
  }
  ctx->pinned[best].busy = true;
  *idx = best;
  return CROSS_OK;
}

void pinned_release(cross_ctx ctx, int idx) {
  if (idx >= 0 && idx < (int)ctx->pinned.size()) ctx->pinned[idx].busy = false;
}

cross_status workspace(cross_ctx ctx, hipStream_t s, size_t bytes, void** out) {
  DevBuf& b = ctx->workspace[s];
  if (b.size < bytes) {
    if (b.ptr) {
      // the old buffer may still be in use by work queued on this stream
      (void)hipStreamSynchronize(s);
      (void)hipFree(b.ptr);
      b.ptr = nullptr;
      b.size = 0;
    }
    cross_status st = dev_alloc(ctx, bytes, &b.ptr);
    if (st != CROSS_OK) return st;
    b.size = bytes;
  }
  *out = b.ptr;
  return CROSS_OK;
}

// Three factors (plans with log_c1 > 0): forward = row-side step 1 (R-point,
// fused step-2 twiddle, packed output) then the row kernel (C1 x C2 transform
// of every row, plain output); inverse = the inverse row kernel (packed output
// with the inverse step-2 twiddle) then the row-side step 1 inverse on packed
// row-major input (N^-1 folded in).
static cross_status ntt_three(cross_ctx ctx, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
                              uint32_t* data, uint64_t stride, int npoly, bool inverse, uint32_t* tmp,
                              hipStream_t s, const RowsTail* tail = nullptr, uint32_t* dst = nullptr,
                              bool left_only = false) {
  if (!dst) dst = data;
  const int log_n = plans[0]->log_n, log_r = plans[0]->log_r, log_c1 = plans[0]->log_c1;
  const int log_c2 = log_n - log_r - log_c1;
  const int red = ctx->ntt_reduction;
  const bool wide = plans[0]->wide;
  if (red == 1)
    for (const Plan* p : plans) {
      if (p->bar_k < 22) return fail(ctx, CROSS_EUNSUPPORTED, "Barrett NTT epilogue needs primes >= 2^21");
      if (p->wide) return fail(ctx, CROSS_EUNSUPPORTED, "Barrett NTT epilogue needs primes < 2^28");
    }
  std::vector<RowsJob> rj(plans.size());
  std::vector<GemmJob> gj(plans.size());
  for (size_t i = 0; i < plans.size(); ++i) {
    const Plan* p = plans[i];
    if (p->log_r != log_r || p->log_c1 != log_c1) return fail(ctx, CROSS_EINVAL, "mixed NTT splits in one call");
    const bool bar = red == 1;
    rj[i] = inverse ? RowsJob{bar ? p->row_inv_c_plain : p->row_inv_c, bar ? p->row_inv_b_plain : p->row_inv_b,
                              p->row_inv_t3, p->inv_tw_rows, offs[i], p->q, p->qinv, p->bar_m, p->bar_k}
                    : RowsJob{bar ? p->row_fwd_b_plain : p->row_fwd_b, bar ? p->row_fwd_c_plain : p->row_fwd_c,
                              p->row_fwd_t3, nullptr, offs[i], p->q, p->qinv, p->bar_m, p->bar_k};
    gj[i] = GemmJob{bar ? (inverse ? p->inv_left_plain : p->fwd_left_plain) : (inverse ? p->inv_left : p->fwd_left),
                    inverse ? nullptr : p->fwd_tw, offs[i], offs[i], p->q, p->qinv, p->bar_m, p->bar_k};
  }
  void *dr = nullptr, *dg = nullptr;
  cross_status st = cached_device_copy(ctx, rj.data(), rj.size() * sizeof(RowsJob), &dr);
  if (st == CROSS_OK) st = cached_device_copy(ctx, gj.data(), gj.size() * sizeof(GemmJob), &dg);
  if (st != CROSS_OK) return st;
  GemmLaunch g{};
  g.jobs = (const GemmJob*)dg;
  g.njobs = (int)plans.size();
  g.src_stride = g.dst_stride = stride;
  g.npoly = npoly;
  g.log_r = log_r;
  g.log_c = log_n - log_r;
  g.kind = kLeft;
  g.wide = wide;
  g.red = red;
  g.tile = ctx->gemm_tile;
  if (g.tile == 0) {
    auto it = ctx->tile_by_logn.find(log_n);
    if (it != ctx->tile_by_logn.end()) g.tile = it->second;
  }
  auto rows = [&](const uint32_t* in, uint32_t* out) -> cross_status {
    hipError_t e;
    {
      ProfScope ps(ctx, "ntt_rows", s);
      e = launch_ntt_rows((const RowsJob*)dr, (int)plans.size(), in, out, stride, npoly, log_r, log_c1, log_c2,
                          inverse, red, wide, s);
    }
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("row transform launch: ") + hipGetErrorString(e));
    return CROSS_OK;
  };
  auto left = [&]() -> cross_status {
    hipError_t e;
    {
      ProfScope ps(ctx, "bat_gemm_left", s);
      e = launch_bat_gemm(g, s);
    }
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("row-side step launch: ") + hipGetErrorString(e));
    return CROSS_OK;
  };
  if (!inverse) {
    g.src = data;
    g.dst = tmp;
    g.out_packed = g.twiddle = true;
    if ((st = left()) != CROSS_OK) return st;
    if (left_only) return CROSS_OK;
    if (!tail) return rows(tmp, dst);
    hipError_t e;
    {
      ProfScope ps(ctx, "ntt_rows", s);
      e = launch_ntt_rows_tail((const RowsJob*)dr, (int)plans.size(), tmp, stride, npoly, log_r, *tail, s);
    }
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("row transform launch: ") + hipGetErrorString(e));
    return CROSS_OK;
  }
  if ((st = rows(data, tmp)) != CROSS_OK) return st;
  g.src = tmp;
  g.dst = dst;
  g.in_packed = g.in_rows = true;
  return left();
}

bool ntt_tail_fusable(cross_ctx ctx, const std::vector<Plan*>& plans) {
  if (plans.empty() || ctx->ntt_engine != CROSS_NTT_ENGINE_MFMA || ctx->ntt_reduction != 0) return false;
  const Plan* p0 = plans[0];
  if (p0->log_n < 8 || p0->log_c1 == 0 || !rows_tail_supported(p0->log_n, p0->log_r, p0->log_c1)) return false;
  for (const Plan* p : plans)
    if (p->wide || p->log_r != p0->log_r || p->log_c1 != p0->log_c1) return false;
  return true;
}

cross_status ntt_limbs_tail(cross_ctx ctx, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
                            uint32_t* data, uint64_t stride, int npoly, uint32_t* tmp, const RowsTail& tail,
                            hipStream_t s) {
  if (!ntt_tail_fusable(ctx, plans)) return fail(ctx, CROSS_EUNSUPPORTED, "no fused tail for this NTT form");
  return ntt_three(ctx, plans, offs, data, stride, npoly, false, tmp, s, &tail);
}

cross_status ntt_rowside_forward(cross_ctx ctx, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
                                 uint32_t* data, uint64_t stride, int npoly, uint32_t* tmp, hipStream_t s) {
  if (!ntt_tail_fusable(ctx, plans)) return fail(ctx, CROSS_EUNSUPPORTED, "no fused row kernel for this NTT form");
  return ntt_three(ctx, plans, offs, data, stride, npoly, false, tmp, s, nullptr, nullptr, true);
}

cross_status ntt_limbs(cross_ctx ctx, const std::vector<Plan*>& plans,
                       const std::vector<uint64_t>& offs, uint32_t* data, uint64_t stride,
                       int npoly, bool inverse, uint32_t* tmp, hipStream_t s, uint32_t* dst) {
  if (plans.empty()) return CROSS_OK;
  if (dst == data) dst = nullptr;
  const int log_n = plans[0]->log_n;
  const int log_r = plans[0]->log_r;
  if (log_n >= 8) {
    // one launch takes one operand form: wide and narrow limbs go in two groups
    bool mixed = false;
    for (const Plan* p : plans) mixed |= p->wide != plans[0]->wide;
    if (mixed) {
      std::vector<Plan*> pw, pn;
      std::vector<uint64_t> ow, on;
      for (size_t i = 0; i < plans.size(); ++i) {
        (plans[i]->wide ? pw : pn).push_back(plans[i]);
        (plans[i]->wide ? ow : on).push_back(offs[i]);
      }
      cross_status st = ntt_limbs(ctx, pn, on, data, stride, npoly, inverse, tmp, s, dst);
      return st != CROSS_OK ? st : ntt_limbs(ctx, pw, ow, data, stride, npoly, inverse, tmp, s, dst);
    }
  }
  if (log_n < 8 || ctx->ntt_engine == CROSS_NTT_ENGINE_BUTTERFLY) {
    // below the MFMA minimum (4R >= 64), or the butterfly engine selected: radix-2
    // kernels, in place (out of place: the limbs are copied to dst first)
    if (dst) {
      void* doff = nullptr;
      cross_status st = cached_device_copy(ctx, offs.data(), offs.size() * 8, &doff);
      if (st != CROSS_OK) return st;
      const hipError_t e = launch_limb_copy(data, stride, (const uint64_t*)doff, dst, stride, (const uint64_t*)doff,
                                            (int)offs.size(), log_n, npoly, s);
      if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("limb copy: ") + hipGetErrorString(e));
      data = dst;
      dst = nullptr;
    }
    std::vector<ButterflyJob> jobs(plans.size());
    for (size_t i = 0; i < plans.size(); ++i)
      jobs[i] = ButterflyJob{inverse ? plans[i]->bf_inv : plans[i]->bf_fwd, offs[i], plans[i]->q,
                             plans[i]->qinv, plans[i]->bf_ninv};
    void* dj = nullptr;
    cross_status st = cached_device_copy(ctx, jobs.data(), jobs.size() * sizeof(ButterflyJob), &dj);
    if (st != CROSS_OK) return st;
    hipError_t e;
    {
      ProfScope ps(ctx, "butterfly_ntt", s);
      e = launch_butterfly((const ButterflyJob*)dj, (int)jobs.size(), data, stride, npoly, log_n, inverse, s);
    }
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("butterfly launch: ") + hipGetErrorString(e));
    return CROSS_OK;
  }
  if (plans[0]->log_c1 > 0) return ntt_three(ctx, plans, offs, data, stride, npoly, inverse, tmp, s, nullptr, dst);
  const int red = ctx->ntt_reduction;
  if (red == 1)
    for (const Plan* p : plans) {
      if (p->bar_k < 22) return fail(ctx, CROSS_EUNSUPPORTED, "Barrett NTT epilogue needs primes >= 2^21");
      if (p->wide) return fail(ctx, CROSS_EUNSUPPORTED, "Barrett NTT epilogue needs primes < 2^28");
    }
  const bool bar = red == 1;
  std::vector<GemmJob> j1(plans.size()), j2(plans.size());
  for (size_t i = 0; i < plans.size(); ++i) {
    const Plan* p = plans[i];
    j1[i] = GemmJob{bar ? (inverse ? p->inv_right_plain : p->fwd_left_plain) : (inverse ? p->inv_right : p->fwd_left),
                    inverse ? p->inv_tw : p->fwd_tw, offs[i], offs[i], p->q, p->qinv, p->bar_m, p->bar_k};
    j2[i] = GemmJob{bar ? (inverse ? p->inv_left_plain : p->fwd_right_plain) : (inverse ? p->inv_left : p->fwd_right),
                    nullptr, offs[i], offs[i], p->q, p->qinv, p->bar_m, p->bar_k};
  }
  void *d1 = nullptr, *d2 = nullptr;
  cross_status st = cached_device_copy(ctx, j1.data(), j1.size() * sizeof(GemmJob), &d1);
  if (st == CROSS_OK) st = cached_device_copy(ctx, j2.data(), j2.size() * sizeof(GemmJob), &d2);
  if (st != CROSS_OK) return st;
  GemmLaunch g{};
  g.njobs = (int)plans.size();
  g.src_stride = g.dst_stride = stride;
  g.npoly = npoly;
  g.log_r = log_r;
  g.log_c = log_n - log_r;
  g.wide = plans[0]->wide;
  g.red = red;
  g.tile = ctx->gemm_tile;
  if (g.tile == 0) {
    auto it = ctx->tile_by_logn.find(log_n);
    if (it != ctx->tile_by_logn.end()) g.tile = it->second;
  }
  // step 1 (data -> tmp, packed chunks, twiddle fused) then step 3 (tmp -> data)
  g.jobs = (const GemmJob*)d1;
  g.src = data;
  g.dst = tmp;
  g.kind = inverse ? kRight : kLeft;
  g.in_packed = false;
  g.out_packed = true;
  g.twiddle = true;
  hipError_t e;
  {
    ProfScope ps(ctx, inverse ? "bat_gemm_right" : "bat_gemm_left", s);
    e = launch_bat_gemm(g, s);
  }
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("step-1 launch: ") + hipGetErrorString(e));
  g.jobs = (const GemmJob*)d2;
  g.src = tmp;
  g.dst = dst ? dst : data;
  g.kind = inverse ? kLeft : kRight;
  g.in_packed = true;
  g.out_packed = false;
  g.twiddle = false;
  {
    ProfScope ps(ctx, inverse ? "bat_gemm_left" : "bat_gemm_right", s);
    e = launch_bat_gemm(g, s);
  }
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("step-3 launch: ") + hipGetErrorString(e));
  return CROSS_OK;
}

cross_status check_residues(cross_ctx ctx, const char* what, const uint32_t* base, uint64_t stride, int npoly,
                            const uint32_t* qs, int nl, int log_n, hipStream_t s) {
  if (!ctx->debug_check || npoly <= 0 || nl <= 0) return CROSS_OK;
  if (!ctx->debug_flag) {
    void* f = nullptr;
    cross_status st = dev_alloc(ctx, sizeof(unsigned long long), &f);
    if (st != CROSS_OK) return st;
    ctx->debug_flag = static_cast<unsigned long long*>(f);
  }
  const uint64_t N = 1ull << log_n;
  std::vector<CheckLimb> limbs(nl);
  for (int i = 0; i < nl; ++i) limbs[i] = CheckLimb{(uint64_t)i * N, qs[i], 0};
  void* dl = nullptr;
  cross_status st = cached_device_copy(ctx, limbs.data(), limbs.size() * sizeof(CheckLimb), &dl);
  if (st != CROSS_OK) return st;
  unsigned long long first = ~0ull;
  hipError_t e = hipMemcpyAsync(ctx->debug_flag, &first, sizeof(first), hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = launch_residue_check(base, stride, npoly, (const CheckLimb*)dl, nl, log_n, ctx->debug_flag, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&first, ctx->debug_flag, sizeof(first), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("debug check: ") + hipGetErrorString(e));
  if (first == ~0ull) return CROSS_OK;
  const uint64_t n = first % N, pl = first / N;
  const uint64_t l = pl % (uint64_t)nl, p = pl / (uint64_t)nl;
  return fail(ctx, CROSS_EDOMAIN, std::string(what) + ": polynomial " + std::to_string(p) + ", limb " +
                                      std::to_string(l) + ", coefficient " + std::to_string(n) +
                                      " is not below its modulus " + std::to_string(qs[l]));
}

// ---- scratch of the allocation-free NTT entry point ------------------------
// A file-scope device array: every device the library runs on holds its own copy
// (loaded with the code object, kept until the process ends).  Host code never
// uses its name as an address: the device address comes from hipGetSymbolAddress,
// taken once per device with that device current, and is kept per device.
constexpr size_t kNoAllocJobBytes = 64 << 10;      // head: the call's job lists
static __device__ __align__(256) uint8_t scratch[kNoAllocJobBytes + CROSS_NOALLOC_MAX_BYTES];

hipError_t noalloc_scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;                  // device -> address of its copy
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  int prev = 0;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if ((e = hipSetDevice(device)) != hipSuccess) return e;
  void* p = nullptr;
  e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return e;
  addr[device] = p;
  *out = p;
  return hipSuccess;
}

static cross_status ntt_common(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                               uint32_t batch, uint32_t* data, void* stream, bool inverse,
                               bool butterfly) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N)
    return fail(ctx, CROSS_EINVAL, "log_n out of range [4, 16]");
  if (!primes || !data) return fail(ctx, CROSS_EINVAL, "null pointer");
  if (L < 1 || L > CROSS_MAX_LIMBS) return fail(ctx, CROSS_EINVAL, "L out of range");
  if (batch < 1) return fail(ctx, CROSS_EINVAL, "batch must be >= 1");
  if (reinterpret_cast<uintptr_t>(data) & 15) return fail(ctx, CROSS_EINVAL, "data not 16-byte aligned");
  for (uint32_t i = 0; i < L; ++i) {
    cross_status st = check_prime(ctx, primes[i], log_n, true);
    if (st != CROSS_OK) return st;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint64_t N = 1ull << log_n;
  {
    cross_status st = check_residues(ctx, "data", data, (uint64_t)L * N, (int)batch, primes, (int)L, (int)log_n, s);
    if (st != CROSS_OK) return st;
  }
  std::vector<Plan*> plans(L);
  std::vector<uint64_t> offs(L);
  for (uint32_t i = 0; i < L; ++i) {
    cross_status st = get_plan(ctx, primes[i], (int)log_n, &plans[i]);
    if (st != CROSS_OK) return st;
    offs[i] = i * N;
  }
  if (butterfly || log_n < 8) {
    std::vector<ButterflyJob> jobs(L);
    for (uint32_t i = 0; i < L; ++i)
      jobs[i] = ButterflyJob{inverse ? plans[i]->bf_inv : plans[i]->bf_fwd, offs[i], plans[i]->q,
                             plans[i]->qinv, plans[i]->bf_ninv};
    void* dj = nullptr;
    cross_status st = cached_device_copy(ctx, jobs.data(), jobs.size() * sizeof(ButterflyJob), &dj);
    if (st != CROSS_OK) return st;
    hipError_t e;
    {
      ProfScope ps(ctx, "butterfly_ntt", s);
      e = launch_butterfly((const ButterflyJob*)dj, (int)L, data, (uint64_t)L * N, (int)batch,
                           (int)log_n, inverse, s);
    }
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("butterfly launch: ") + hipGetErrorString(e));
    return CROSS_OK;
  }
  void* tmp = nullptr;
  cross_status st = workspace(ctx, s, (size_t)batch * L * N * 4, &tmp);
  if (st != CROSS_OK) return st;
  return ntt_limbs(ctx, plans, offs, data, (uint64_t)L * N, (int)batch, inverse, (uint32_t*)tmp, s);
}

}  // namespace cross

using namespace cross;

extern "C" {

cross_status cross_ctx_create(int hip_device, cross_ctx* out) {
  if (!out) return CROSS_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
    (void)hipGetLastError();
    return CROSS_EDEVICE;
  }
  void* scratch_ptr = nullptr;
  if (noalloc_scratch_address(hip_device, &scratch_ptr) != hipSuccess) {
    (void)hipGetLastError();
    return CROSS_EDEVICE;
  }
  cross_ctx c = new cross_ctx_s();
  c->device = hip_device;
  c->noalloc_scratch = scratch_ptr;
  if (const char* v = std::getenv("CROSS_DEBUG_CHECK")) c->debug_check = v[0] == '1';
  *out = c;
  return CROSS_OK;
}

void cross_ctx_destroy(cross_ctx ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : ctx->plans) {
    (void)hipFree(kv.second->block);
    delete kv.second;
  }
  for (auto& kv : ctx->job_cache) (void)hipFree(kv.second);
  for (auto& kv : ctx->const_cache) (void)hipFree(kv.second);
  for (auto& kv : ctx->workspace) (void)hipFree(kv.second.ptr);
  for (auto& b : ctx->pinned) {
    (void)hipEventDestroy(b.ev);
    (void)hipHostFree(b.p);
  }
  if (ctx->debug_flag) (void)hipFree(ctx->debug_flag);
  for (auto& r : ctx->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : ctx->prof_pool) (void)hipEventDestroy(e);
  delete ctx;
}

const char* cross_last_error(cross_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

cross_status cross_root(uint32_t q, uint32_t log_n, uint32_t* psi_out) {
  if (!psi_out || log_n < 1 || log_n > 26) return CROSS_EINVAL;
  cross_status st = check_prime(nullptr, q, log_n, true);
  if (st != CROSS_OK) return st;
  *psi_out = root_2n(q, log_n);
  return CROSS_OK;
}

cross_status cross_set_ntt_split(cross_ctx ctx, uint32_t log_n, uint32_t log_r) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < 8 || log_n > CROSS_MAX_LOG_N || log_r < 4 || log_n - log_r < 4 || log_r > log_n)
    return fail(ctx, CROSS_EINVAL, "split needs 4 <= log_r <= log_n - 4");
  ctx->split[(int)log_n] = (int)log_r;
  ctx->split3[(int)log_n] = std::make_pair((int)log_r, 0);    // explicitly two factors
  return CROSS_OK;
}

cross_status cross_set_ntt_split3(cross_ctx ctx, uint32_t log_n, uint32_t log_r, uint32_t log_c1) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < 8 || log_n > CROSS_MAX_LOG_N) return fail(ctx, CROSS_EINVAL, "log_n out of range");
  if (log_c1 == 0 && log_r == 0) {          // back to the size's default
    ctx->split3.erase((int)log_n);
    return CROSS_OK;
  }
  if (log_c1 == 0) {                        // two factors with R = 2^log_r
    if (log_r < 4 || log_r > log_n || log_n - log_r < 4)
      return fail(ctx, CROSS_EINVAL, "split needs 4 <= log_r <= log_n - 4");
    ctx->split3[(int)log_n] = std::make_pair((int)log_r, 0);
    return CROSS_OK;
  }
  if (log_r > log_n || !rows_split_supported((int)log_n, (int)log_r, (int)log_c1))
    return fail(ctx, CROSS_EINVAL, "three-factor split needs 16 <= C1, C2 <= 64 and R >= max(16, 8192 / (C1 C2))");
  ctx->split3[(int)log_n] = std::make_pair((int)log_r, (int)log_c1);
  return CROSS_OK;
}

cross_status cross_set_ntt_reduction(cross_ctx ctx, int method) {
  if (!ctx) return CROSS_EINVAL;
  if (method != CROSS_NTT_RED_MONTGOMERY && method != CROSS_NTT_RED_BARRETT)
    return fail(ctx, CROSS_EINVAL, "unknown NTT reduction");
  ctx->ntt_reduction = method;
  return CROSS_OK;
}

cross_status cross_ntt_noalloc(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, uint32_t batch,
                               uint32_t* data, int inverse, void* stream) {
  if (!ctx) return CROSS_EINVAL;
  if (log_n < CROSS_MIN_LOG_N || log_n > CROSS_MAX_LOG_N)
    return fail(ctx, CROSS_EINVAL, "log_n out of range [4, 16]");
  if (!primes || !data) return fail(ctx, CROSS_EINVAL, "null pointer");
  if (L < 1 || L > CROSS_MAX_LIMBS) return fail(ctx, CROSS_EINVAL, "L out of range");
  if (batch < 1) return fail(ctx, CROSS_EINVAL, "batch must be >= 1");
  if (reinterpret_cast<uintptr_t>(data) & 15) return fail(ctx, CROSS_EINVAL, "data not 16-byte aligned");
  const uint64_t N = 1ull << log_n, bytes = (uint64_t)batch * L * N * 4;
  if (bytes > CROSS_NOALLOC_MAX_BYTES)
    return fail(ctx, CROSS_EINVAL, "batch * L * N * 4 = " + std::to_string(bytes) +
                                       " bytes exceeds the no-alloc limit CROSS_NOALLOC_MAX_BYTES = " +
                                       std::to_string((uint64_t)CROSS_NOALLOC_MAX_BYTES));
  if (!ctx->noalloc_scratch) return fail(ctx, CROSS_EDEVICE, "no-alloc scratch address unknown");
  std::vector<Plan*> plans(L);
  std::vector<uint64_t> offs(L);
  for (uint32_t i = 0; i < L; ++i) {
    cross_status st = check_prime(ctx, primes[i], log_n, true);
    if (st != CROSS_OK) return st;
    int log_r = 0, log_c1 = 0;
    effective_split(ctx, (int)log_n, true, &log_r, &log_c1);
    auto it = ctx->plans.find(std::make_tuple(primes[i], (int)log_n, log_r, log_c1));
    if (it == ctx->plans.end())
      return fail(ctx, CROSS_EUNSUPPORTED, "no tables for modulus " + std::to_string(primes[i]) +
                                               " at this size on this context: call cross_ntt_forward or "
                                               "cross_ntt_inverse with these primes once first");
    plans[i] = it->second;
    offs[i] = i * N;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* base = static_cast<char*>(ctx->noalloc_scratch);
  ctx->arena = cross_ctx_s::Arena{base, kNoAllocJobBytes, 0, s};
  const cross_status st = ntt_limbs(ctx, plans, offs, data, L * N, (int)batch, inverse != 0,
                                    reinterpret_cast<uint32_t*>(base + kNoAllocJobBytes), s);
  ctx->arena = cross_ctx_s::Arena{};
  return st;
}

cross_status cross_set_debug_check(cross_ctx ctx, int enable) {
  if (!ctx) return CROSS_EINVAL;
  ctx->debug_check = enable != 0;
  return CROSS_OK;
}

cross_status cross_set_ntt_engine(cross_ctx ctx, int engine) {
  if (!ctx) return CROSS_EINVAL;
  if (engine != CROSS_NTT_ENGINE_MFMA && engine != CROSS_NTT_ENGINE_BUTTERFLY)
    return fail(ctx, CROSS_EINVAL, "unknown NTT engine");
  ctx->ntt_engine = engine;
  return CROSS_OK;
}

cross_status cross_get_ntt_split(cross_ctx ctx, uint32_t log_n, uint32_t* log_r, uint32_t* log_c1) {
  if (!ctx || !log_r || !log_c1) return CROSS_EINVAL;
  if (log_n < 8 || log_n > CROSS_MAX_LOG_N) return fail(ctx, CROSS_EINVAL, "log_n out of range");
  int r = 0, c1 = 0;
  effective_split(ctx, (int)log_n, true, &r, &c1);
  *log_r = (uint32_t)r;
  *log_c1 = (uint32_t)c1;
  return CROSS_OK;
}

cross_status cross_set_gemm_tile(cross_ctx ctx, int tile) {
  if (!ctx) return CROSS_EINVAL;
  if (tile < 0 || tile >= kTileCount) return fail(ctx, CROSS_EINVAL, "tile must be 0 (auto) .. 9");
  ctx->gemm_tile = tile;
  return CROSS_OK;
}

cross_status cross_ntt_forward(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                               uint32_t batch, uint32_t* data, void* stream) {
  return ntt_common(ctx, log_n, primes, L, batch, data, stream, false, false);
}
cross_status cross_ntt_inverse(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                               uint32_t batch, uint32_t* data, void* stream) {
  return ntt_common(ctx, log_n, primes, L, batch, data, stream, true, false);
}
cross_status cross_ntt_forward_butterfly(cross_ctx ctx, uint32_t log_n, const uint32_t* primes,
                                         uint32_t L, uint32_t batch, uint32_t* data, void* stream) {
  return ntt_common(ctx, log_n, primes, L, batch, data, stream, false, true);
}
cross_status cross_ntt_inverse_butterfly(cross_ctx ctx, uint32_t log_n, const uint32_t* primes,
                                         uint32_t L, uint32_t batch, uint32_t* data, void* stream) {
  return ntt_common(ctx, log_n, primes, L, batch, data, stream, true, true);
}

cross_status cross_profile_enable(cross_ctx ctx, int enable) {
  if (!ctx) return CROSS_EINVAL;
  ctx->prof = enable != 0;
  return CROSS_OK;
}

cross_status cross_profile_only(cross_ctx ctx, const char* family) {
  if (!ctx) return CROSS_EINVAL;
  ctx->prof_only = family ? family : "";
  return CROSS_OK;
}

cross_status cross_profile_report(cross_ctx ctx, char* buf, uint64_t len) {
  if (!ctx || !buf || len == 0) return CROSS_EINVAL;
  std::map<std::string, std::pair<long, double>> agg;
  for (auto& r : ctx->prof_recs) {
    float ms = 0.f;
    if (r.valid && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& x = agg[r.name];
      x.first += 1;
      x.second += ms;
    }
    ctx->prof_pool.push_back(r.a);
    ctx->prof_pool.push_back(r.b);
  }
  ctx->prof_recs.clear();
  std::string out;
  for (auto& kv : agg) {
    char line[256];
    snprintf(line, sizeof line, "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  size_t n = out.size() < len - 1 ? out.size() : (size_t)(len - 1);
  std::memcpy(buf, out.data(), n);
  buf[n] = 0;
  return CROSS_OK;
}

cross_status cross_host_row_tables(uint32_t q, uint32_t log_n, uint32_t log_r, uint32_t log_c1, uint32_t which,
                                   void* out, uint64_t* bytes) {
  if (!bytes || which > 12 || log_n > CROSS_MAX_LOG_N || log_r > log_n ||
      !rows_split_supported((int)log_n, (int)log_r, (int)log_c1))
    return CROSS_EINVAL;
  cross_status st = check_prime(nullptr, q, log_n, true);
  if (st != CROSS_OK) return st;
  if (which >= 8 && which <= 11 && wide_prime(q)) return CROSS_EINVAL;   // no plain tables in the wide form
  NttTables t;
  try {
    build_ntt_tables(q, log_n, log_r, t, true, log_c1);
  } catch (const std::exception&) {
    return CROSS_EINVAL;
  }
  const void* src = nullptr;
  uint64_t n = 0;
  switch (which) {
    case 0: src = t.row_fwd_b.data(); n = t.row_fwd_b.size(); break;
    case 1: src = t.row_fwd_c.data(); n = t.row_fwd_c.size(); break;
    case 2: src = t.row_inv_c.data(); n = t.row_inv_c.size(); break;
    case 3: src = t.row_inv_b.data(); n = t.row_inv_b.size(); break;
    case 4: src = t.row_fwd_t3.data(); n = t.row_fwd_t3.size() * 4; break;
    case 5: src = t.row_inv_t3.data(); n = t.row_inv_t3.size() * 4; break;
    case 6: src = t.inv_tw_rows.data(); n = t.inv_tw_rows.size() * 4; break;
    case 7: src = t.fwd_tw.data(); n = t.fwd_tw.size() * 4; break;
    case 8: src = t.row_fwd_b_plain.data(); n = t.row_fwd_b_plain.size(); break;
    case 9: src = t.row_fwd_c_plain.data(); n = t.row_fwd_c_plain.size(); break;
    case 10: src = t.row_inv_c_plain.data(); n = t.row_inv_c_plain.size(); break;
    case 11: src = t.row_inv_b_plain.data(); n = t.row_inv_b_plain.size(); break;
    default: src = t.row_fwd_t3_mont.data(); n = t.row_fwd_t3_mont.size() * 4; break;
  }
  if (!out) {
    *bytes = n;
    return CROSS_OK;
  }
  if (*bytes < n) return CROSS_EINVAL;
  std::memcpy(out, src, n);
  *bytes = n;
  return CROSS_OK;
}

cross_status cross_host_tables(uint32_t q, uint32_t log_n, uint32_t log_r, uint32_t which,
                               void* out, uint64_t* bytes) {
  if (!bytes || which > 10 || log_n < 8 || log_n > CROSS_MAX_LOG_N || log_r < 4 || log_n - log_r < 4)
    return CROSS_EINVAL;
  cross_status st = check_prime(nullptr, q, log_n, which != 6);
  if (st != CROSS_OK) return st;
  if (which >= 7 && wide_prime(q)) return CROSS_EINVAL;     // no plain tables in the wide form
  NttTables t;
  std::vector<int8_t> lazy;
  if (which == 6) lazy = lazy_fragment(q);
  else build_ntt_tables(q, log_n, log_r, t);
  const void* src = nullptr;
  uint64_t n = 0;
  switch (which) {
    case 6: src = lazy.data(); n = lazy.size(); break;
    case 0: src = t.fwd_left.data(); n = t.fwd_left.size(); break;
    case 1: src = t.fwd_right.data(); n = t.fwd_right.size(); break;
    case 2: src = t.inv_left.data(); n = t.inv_left.size(); break;
    case 3: src = t.inv_right.data(); n = t.inv_right.size(); break;
    case 4: src = t.fwd_tw.data(); n = t.fwd_tw.size() * 4; break;
    case 5: src = t.inv_tw.data(); n = t.inv_tw.size() * 4; break;
    case 7: src = t.fwd_left_plain.data(); n = t.fwd_left_plain.size(); break;
    case 8: src = t.fwd_right_plain.data(); n = t.fwd_right_plain.size(); break;
    case 9: src = t.inv_left_plain.data(); n = t.inv_left_plain.size(); break;
    default: src = t.inv_right_plain.data(); n = t.inv_right_plain.size(); break;
  }
  if (!out) {
    *bytes = n;
    return CROSS_OK;
  }
  if (*bytes < n) return CROSS_EINVAL;
  std::memcpy(out, src, n);
  *bytes = n;
  return CROSS_OK;
}

}  // extern "C"
