// Batch runtime: many jobs of uneven N, limb count and kind in a fixed
// sequence of work-list launches, optionally captured once as a hipGraph.
//
// Every job is lowered onto the same phases (automorphism, tensor product,
// ModUp copies, INTT of d, BConv, NTT of the extension, inner product, ModDown
// INTT / BConv / NTT, tail).  A phase holds the work of every job that takes
// part in it: vector phases list one task per polynomial; an NTT phase has two
// halves, each a few work-list launches -- BAT GEMM steps as persistent grids
// over (task, tile) lists, one launch per list tile shape, and the row
// transform of the three-factor form as one persistent launch over a task list
// -- where each task carries its own N, split, prime, tables and buffers.
// Sizes from 2^14 up run in three factors, R x 32 x 32 (a quarter of the
// two-factor MAC work at 2^16); 2^12 and 2^13 in two (R, C >= 64).  Launch
// boundaries order the phases, so a batch of any size costs a fixed number of
// launches, and replaying the captured graph costs one.
#include <cstring>
#include <algorithm>
#include <map>
#include <memory>
#include <string>

#include "ckks_plan.h"
#include "context.h"
#include "params.h"

namespace cross {

namespace {

// The NTT phases, in run order.
enum NttPhaseId { kNttInvD, kNttFwdExt, kNttInvP, kNttFwdZ, kNumNtt };

// One work-list GEMM launch.
struct GemmPhase {
  std::vector<GemmTask> tasks;
  std::vector<GemmTileRef> tiles;
  const GemmTask* d_tasks = nullptr;
  const GemmTileRef* d_tiles = nullptr;
};

// One row-kernel launch over a task list.
struct RowsPhase {
  std::vector<RowsTask> tasks;
  int64_t nblocks = 0;
  const RowsTask* d_tasks = nullptr;
};

// Half of an NTT phase: GEMM launches keyed by (list tile, row-major packed input)
// and one row-kernel launch.  The GEMM flags are fixed per half (first / second
// step of the forward / inverse transform).
struct NttHalf {
  std::map<std::pair<int, bool>, GemmPhase> gemm;
  RowsPhase rows;
};

struct NttPhase {
  NttHalf half[2];
};

}  // namespace

}  // namespace cross

struct cross_batch_s {
  cross_ctx ctx = nullptr;
  cross::NttPhase ntt[cross::kNumNtt];
  std::vector<cross::AutoTask> autos;
  std::vector<cross::TensorTask> tensors;
  std::vector<cross::CopyTask> copies;
  std::vector<cross::BconvLaunch> bconv_up, bconv_down;
  std::vector<cross::InnerTask> inners;
  std::vector<cross::TailTask> tails;
  // N >= 2^14 (R x 32 x 32): ModUp NTT + inner product and ModDown NTT + tail fused
  std::vector<cross::IpTask> ips;
  std::vector<cross::RowsTailTask> rtails;
  int64_t ip_blocks = 0, rtail_blocks = 0;
  const cross::IpTask* d_ips = nullptr;
  const cross::RowsTailTask* d_rtails = nullptr;
  const cross::AutoTask* d_autos = nullptr;
  const cross::TensorTask* d_tensors = nullptr;
  const cross::CopyTask* d_copies = nullptr;
  const cross::BconvLaunch *d_bconv_up = nullptr, *d_bconv_down = nullptr;
  const cross::InnerTask* d_inners = nullptr;
  const cross::TailTask* d_tails = nullptr;
  uint64_t max_auto = 0, max_tensor = 0, max_copy = 0, max_inner = 0, max_tail = 0;
  uint64_t max_cols_up = 0, max_cols_down = 0;   // largest npoly << log_n of the BConv tasks
  int max_nsrc_up = 0, max_nsrc_down = 0;
  std::vector<void*> allocs;
  uint64_t ws_bytes = 0;
  bool external = false;        // scratch and task lists live in the caller's workspace
  char* ext_cursor = nullptr;   // next free byte of the caller's workspace (task lists)
  char* ext_end = nullptr;
  char* ext_lists = nullptr;    // first byte of the task lists in the caller's workspace
  std::vector<char> stage;      // task lists as laid out there (host copy)
  int pinned = -1;              // the context's pinned buffer holding their upload's source
  hipStream_t upload_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace cross {

namespace {

uint64_t align256(uint64_t x) { return (x + 255) & ~(uint64_t)255; }

template <typename T>
uint64_t list_bytes(const std::vector<T>& v) { return align256(v.size() * sizeof(T)); }

template <typename T>
cross_status upload(cross_batch b, const std::vector<T>& v, const T** out) {
  *out = nullptr;
  if (v.empty()) return CROSS_OK;
  void* d = nullptr;
  if (b->external) {
    const uint64_t n = list_bytes(v);
    if (b->ext_cursor + n > b->ext_end) return fail(b->ctx, CROSS_EINVAL, "workspace too small for the task lists");
    d = b->ext_cursor;
    b->ext_cursor += n;
    // gathered into the host stage; finish_upload copies every list at once
    const size_t at = b->stage.size();
    b->stage.resize(at + n, 0);
    std::memcpy(b->stage.data() + at, v.data(), v.size() * sizeof(T));
  } else {
    if (hipMalloc(&d, v.size() * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return fail(b->ctx, CROSS_ENOMEM, "batch task list allocation failed");
    }
    b->allocs.push_back(d);
    if (hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
      return fail(b->ctx, CROSS_EDEVICE, "batch task list upload failed");
  }
  *out = static_cast<const T*>(d);
  return CROSS_OK;
}

// Caller's workspace: one stream-ordered copy of all task lists from a pinned
// buffer of the context's pool (released when the batch is destroyed; the copy's
// end is recorded on the buffer's event, so the buffer is reused only after it).
cross_status finish_upload(cross_batch b) {
  if (b->stage.empty()) return CROSS_OK;
  cross_status st = pinned_acquire(b->ctx, b->stage.size(), &b->pinned);
  if (st != CROSS_OK) return st;
  cross_ctx_s::Pinned& pb = b->ctx->pinned[b->pinned];
  std::memcpy(pb.p, b->stage.data(), b->stage.size());
  if (hipMemcpyAsync(b->ext_lists, pb.p, b->stage.size(), hipMemcpyHostToDevice, b->upload_stream) != hipSuccess ||
      hipEventRecord(pb.ev, b->upload_stream) != hipSuccess) {
    (void)hipGetLastError();
    return fail(b->ctx, CROSS_EDEVICE, "batch task list upload failed");
  }
  return CROSS_OK;
}

uint64_t task_list_bytes(cross_batch b) {
  uint64_t n = 0;
  for (auto& ph : b->ntt)
    for (auto& hf : ph.half) {
      for (auto& kv : hf.gemm) n += list_bytes(kv.second.tasks) + list_bytes(kv.second.tiles);
      n += list_bytes(hf.rows.tasks);
    }
  n += list_bytes(b->autos) + list_bytes(b->tensors) + list_bytes(b->copies) + list_bytes(b->bconv_up) +
       list_bytes(b->bconv_down) + list_bytes(b->inners) + list_bytes(b->tails) + list_bytes(b->ips) +
       list_bytes(b->rtails);
  return n;
}

// List tile of a GEMM step with M = 4U output rows: the tuner's choice for the
// transform size and direction where it fits, else the largest that tiles M.
int list_tile_for(cross_ctx ctx, int log_n, bool inverse, int M) {
  auto it = ctx->list_tile.find(2 * log_n + (inverse ? 1 : 0));
  if (it != ctx->list_tile.end()) {
    int rows = 0, cols = 0;
    if (gemm_list_tile_dims(it->second, &rows, &cols) && M % rows == 0) return it->second;
  }
  return M >= 256 ? kListTile256x128 : M >= 128 ? kListTile128x64 : kListTile64x64;
}

// Add one limb's GEMM step to the half's launch for its tile.
void add_gemm_task(cross_ctx ctx, NttHalf& hf, const GemmTask& t, int U, int V, int npoly, bool inverse,
                   bool in_rows, int log_n) {
  const int tile = list_tile_for(ctx, log_n, inverse, 4 * U);
  int rows = 0, cols = 0;
  gemm_list_tile_dims(tile, &rows, &cols);
  GemmPhase& ph = hf.gemm[std::make_pair(tile, in_rows)];
  const int tm_n = 4 * U / rows;
  const long ncols = (long)npoly * V;
  const int tn_n = (int)((ncols + cols - 1) / cols);
  const uint32_t id = (uint32_t)ph.tasks.size();
  ph.tasks.push_back(t);
  for (int tn = 0; tn < tn_n; ++tn)
    for (int tm = 0; tm < tm_n; ++tm) ph.tiles.push_back(GemmTileRef{id, (uint16_t)tm, (uint16_t)tn});
}

// A full NTT of a limb list through `tmp` (same layout as `data`): limb i of
// polynomial p lives at data + p * stride + offs[i].  Two-factor limbs add both
// GEMM steps; three-factor limbs (R x 32 x 32) add the row-side GEMM step and a
// row-kernel task: forward = row-side step (data -> tmp, packed, step-2 twiddle)
// then rows (tmp -> data); inverse = rows (data -> tmp, packed rows, inverse
// step-2 twiddle) then the row-side step on row-major packed input (tmp -> data).
// dst (three factors, inverse): the result goes there instead of back into data.
// first_half_only (three factors, forward): only the row-side step (data -> tmp), for
// a fused row kernel to finish.
void add_ntt(cross_batch b, NttPhase& ph, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
             uint32_t* data, uint32_t* tmp, uint64_t stride, int npoly, bool inverse, uint32_t* dst = nullptr,
             bool first_half_only = false) {
  for (size_t i = 0; i < plans.size(); ++i) {
    const Plan* p = plans[i];
    const int log_r = p->log_r, log_c = p->log_n - p->log_r;
    const int R = 1 << log_r, C = 1 << log_c;
    GemmTask t{};
    t.src_stride = t.dst_stride = stride;
    t.q = p->q;
    t.qinv = p->qinv;
    t.npoly = npoly;
    t.log_r = (int16_t)log_r;
    t.log_c = (int16_t)log_c;
    if (p->log_c1 > 0) {
      RowsTask r{};
      r.stride = stride;
      r.q = p->q;
      r.qinv = p->qinv;
      r.npoly = npoly;
      r.log_r = log_r;
      t.tw = nullptr;
      if (!inverse) {
        t.table = p->fwd_left;
        t.tw = p->fwd_tw;
        t.src = data + offs[i];
        t.dst = tmp + offs[i];
        add_gemm_task(b->ctx, ph.half[0], t, R, C, npoly, false, false, p->log_n);
        if (first_half_only) continue;
        r.tab = p->row_fwd_b;
        r.tw1 = p->row_fwd_t3;
        r.in = tmp + offs[i];
        r.out = data + offs[i];
      } else {
        r.tab = p->row_inv_c;
        r.tw1 = p->row_inv_t3;
        r.tw2 = p->inv_tw_rows;
        r.in = data + offs[i];
        r.out = tmp + offs[i];
        t.table = p->inv_left;
        t.src = tmp + offs[i];
        t.dst = (dst ? dst : data) + offs[i];
        add_gemm_task(b->ctx, ph.half[1], t, R, C, npoly, true, true, p->log_n);
      }
      RowsPhase& rp = ph.half[inverse ? 0 : 1].rows;
      r.first_block = (int32_t)rp.nblocks;
      rp.nblocks += (int64_t)npoly * R / rows_list_rows_per_block();
      rp.tasks.push_back(r);
      continue;
    }
    // two factors: forward = left-known TF1 (+T2) then right-known TF3;
    // inverse = right-known ITF3 (+IT2) then left-known ITF1
    t.table = inverse ? p->inv_right : p->fwd_left;
    t.tw = inverse ? p->inv_tw : p->fwd_tw;
    t.src = data + offs[i];
    t.dst = tmp + offs[i];
    add_gemm_task(b->ctx, ph.half[0], t, inverse ? C : R, inverse ? R : C, npoly, inverse, false, p->log_n);
    t.table = inverse ? p->inv_left : p->fwd_right;
    t.tw = nullptr;
    t.src = tmp + offs[i];
    t.dst = data + offs[i];
    add_gemm_task(b->ctx, ph.half[1], t, inverse ? R : C, inverse ? C : R, npoly, inverse, false, p->log_n);
  }
}

// The batch runtime's plan for prime q at size 2^log_n: three factors R x 32 x 32
// from 2^14 up, else the context's two-factor split (R, C >= 64 for the list tiles).
cross_status batch_plan(cross_ctx ctx, uint32_t q, int log_n, Plan** out) {
  if (log_n >= 14) return get_plan_at(ctx, q, log_n, log_n - 10, 5, out);
  cross_status st = get_plan(ctx, q, log_n, out, false);
  if (st != CROSS_OK) return st;
  if ((*out)->log_r < 6 || log_n - (*out)->log_r < 6)
    return fail(ctx, CROSS_EUNSUPPORTED, "batch runtime needs R, C >= 64 below N = 2^14");
  return CROSS_OK;
}

hipError_t run_ntt(cross_batch b, int phase, bool inverse, hipStream_t s, bool prof) {
  cross_ctx ctx = b->ctx;
  hipError_t e = hipSuccess;
  for (int h = 0; h < 2 && e == hipSuccess; ++h) {
    NttHalf& hf = b->ntt[phase].half[h];
    // step flags: forward = LEFT(plain -> packed, twiddle) then RIGHT(packed -> plain);
    // inverse = RIGHT(plain -> packed, twiddle) then LEFT(packed -> plain)
    const bool first = h == 0;
    const int kind = (inverse == first) ? kRight : kLeft;
    for (auto& kv : hf.gemm) {
      if (e != hipSuccess || kv.second.tiles.empty()) continue;
      ProfScope ps(prof ? ctx : nullptr, kind == kLeft ? "bat_gemm_left" : "bat_gemm_right", s);
      e = launch_bat_gemm_list(kv.second.d_tasks, kv.second.d_tiles, (int)kv.second.tiles.size(), kind,
                               /*in_packed=*/!first, /*out_packed=*/first, /*twiddle=*/first,
                               /*in_rows=*/kv.first.second, kv.first.first, s);
    }
    if (e == hipSuccess && !hf.rows.tasks.empty()) {
      ProfScope ps(prof ? ctx : nullptr, "ntt_rows", s);
      e = launch_ntt_rows_list(hf.rows.d_tasks, (int)hf.rows.tasks.size(), hf.rows.nblocks, inverse, s);
    }
  }
  return e;
}

hipError_t run_phases(cross_batch b, hipStream_t s, bool prof) {
  cross_ctx ctx = b->ctx;
  hipError_t e = hipSuccess;
  auto vec = [&](const char* name, auto fn) {
    if (e != hipSuccess) return;
    ProfScope ps(prof ? ctx : nullptr, name, s);
    e = fn();
  };
  auto ntt = [&](int phase, bool inverse) {
    if (e == hipSuccess) e = run_ntt(b, phase, inverse, s, prof);
  };
  vec("automorphism", [&] { return launch_auto_list(b->d_autos, (int)b->autos.size(), b->max_auto, s); });
  vec("tensor", [&] { return launch_tensor_list(b->d_tensors, (int)b->tensors.size(), b->max_tensor, s); });
  vec("limb_copy", [&] { return launch_copy_list(b->d_copies, (int)b->copies.size(), b->max_copy, s); });
  ntt(kNttInvD, true);
  vec("bconv", [&] {
    return launch_bconv_list(b->d_bconv_up, (int)b->bconv_up.size(), b->max_cols_up, b->max_nsrc_up, s);
  });
  ntt(kNttFwdExt, false);
  vec("ntt_rows_ip", [&] { return launch_ntt_rows_ip_list(b->d_ips, (int)b->ips.size(), b->ip_blocks, s); });
  vec("inner_product", [&] { return launch_inner_list(b->d_inners, (int)b->inners.size(), b->max_inner, s); });
  ntt(kNttInvP, true);
  vec("bconv", [&] {
    return launch_bconv_list(b->d_bconv_down, (int)b->bconv_down.size(), b->max_cols_down, b->max_nsrc_down, s);
  });
  ntt(kNttFwdZ, false);
  vec("ntt_rows", [&] {
    return launch_ntt_rows_tail_list(b->d_rtails, (int)b->rtails.size(), b->rtail_blocks, s);
  });
  vec("moddown_tail", [&] { return launch_tail_list(b->d_tails, (int)b->tails.size(), b->max_tail, s); });
  return e;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

}  // namespace

}  // namespace cross

using namespace cross;

extern "C" {

void cross_batch_destroy(cross_batch b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  if (!b->external) (void)hipDeviceSynchronize();
  pinned_release(b->ctx, b->pinned);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  for (void* p : b->allocs) (void)hipFree(p);
  delete b;
}

}  // extern "C"

namespace cross {
namespace {

// size_only: plan and lower, then report the bytes a caller-provided workspace needs.
cross_status build_batch(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, int use_graph, void* ext_ws,
                         uint64_t ext_bytes, hipStream_t upload_stream, bool size_only, uint64_t* need,
                         cross_batch* out) {
  if (!ctx || (!out && !size_only)) return CROSS_EINVAL;
  if (out) *out = nullptr;
  if (!jobs || njobs == 0) return fail(ctx, CROSS_EINVAL, "empty job list");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  std::unique_ptr<cross_batch_s, void (*)(cross_batch)> b(new cross_batch_s(), cross_batch_destroy);
  b->ctx = ctx;

  // ---- pass 1: validate, plan, size the workspace --------------------------------
  struct JobPlan {
    CkksPlan* c = nullptr;
    std::vector<Plan*> plans;   // NTT plans of the job's limbs (CKKS: all L + K, Q then P)
    uint64_t ws = 0;            // words
  };
  std::vector<JobPlan> jp(njobs);
  uint64_t ws_words = 0;
  for (uint32_t j = 0; j < njobs; ++j) {
    const cross_job& J = jobs[j];
    const cross_ckks_params& P = J.params;
    if (J.batch < 1) return fail(ctx, CROSS_EINVAL, "job " + std::to_string(j) + ": batch must be >= 1");
    if (P.log_n < 12 || P.log_n > CROSS_MAX_LOG_N)
      return fail(ctx, CROSS_EUNSUPPORTED, "job " + std::to_string(j) + ": batch runtime needs 12 <= log_n <= 16");
    const uint64_t N = 1ull << P.log_n;
    if (J.op == CROSS_OP_NTT_FORWARD || J.op == CROSS_OP_NTT_INVERSE) {
      if (!J.data || !aligned16(J.data) || !P.primes || P.L < 1 || P.L > CROSS_MAX_LIMBS)
        return fail(ctx, CROSS_EINVAL, "job " + std::to_string(j) + ": bad NTT job");
      for (uint32_t i = 0; i < P.L; ++i) {
        cross_status st = check_prime(ctx, P.primes[i], P.log_n);
        if (st != CROSS_OK) return st;
        Plan* p = nullptr;
        if ((st = batch_plan(ctx, P.primes[i], (int)P.log_n, &p)) != CROSS_OK) return st;
        jp[j].plans.push_back(p);
      }
      jp[j].ws = (uint64_t)J.batch * P.L * N;
    } else if (J.op == CROSS_OP_HE_MULT || J.op == CROSS_OP_ROTATE) {
      cross_status st = get_ckks_plan(ctx, &P, &jp[j].c);
      if (st != CROSS_OK) return st;
      if (jp[j].c->wide) return fail(ctx, CROSS_ERANGE, "the batch runtime takes primes below 2^28 only");
      for (uint32_t t : jp[j].c->primes) {
        Plan* p = nullptr;
        if ((st = batch_plan(ctx, t, (int)P.log_n, &p)) != CROSS_OK) return st;
        jp[j].plans.push_back(p);
      }
      const bool he = J.op == CROSS_OP_HE_MULT;
      if (!J.ct_a || !J.key || !J.out || (he && !J.ct_b) || !aligned16(J.ct_a) || !aligned16(J.key) ||
          !aligned16(J.out) || (he && !aligned16(J.ct_b)))
        return fail(ctx, CROSS_EINVAL, "job " + std::to_string(j) + ": bad ciphertext job");
      const CkksPlan* c = jp[j].c;
      const uint64_t LK = c->L + c->K;
      const uint64_t nd = (uint64_t)c->L * N, next = (uint64_t)c->dnum * LK * N;
      const uint64_t nacc = 2 * LK * N, nz = 2ull * c->L * N;
      // NTT scratch is used with the layouts of d, ext, acc and z in turn
      const uint64_t ntmp = std::max(next, nacc);
      jp[j].ws = (uint64_t)J.batch * (nd + next + ntmp + nacc + nz);
    } else {
      return fail(ctx, CROSS_EINVAL, "job " + std::to_string(j) + ": unknown op");
    }
    ws_words += (jp[j].ws + 63) & ~(uint64_t)63;
  }
  void* wsp = nullptr;
  const uint64_t scratch = align256(ws_words * 4);
  if (size_only || ext_ws) {
    // lower against the caller's base (or a stand-in aligned base when only sizing)
    wsp = ext_ws ? ext_ws : reinterpret_cast<void*>((uintptr_t)1 << 20);
    b->external = true;
  } else {
    if (hipMalloc(&wsp, ws_words * 4) != hipSuccess) {
      (void)hipGetLastError();
      return fail(ctx, CROSS_ENOMEM, "batch workspace allocation failed");
    }
    b->allocs.push_back(wsp);
  }
  b->ws_bytes = ws_words * 4;

  // ---- pass 2: lower every job onto the phases ------------------------------------
  uint32_t* ws = static_cast<uint32_t*>(wsp);
  for (uint32_t j = 0; j < njobs; ++j) {
    const cross_job& J = jobs[j];
    const uint64_t N = 1ull << J.params.log_n;
    uint32_t* mine = ws;
    ws += (jp[j].ws + 63) & ~(uint64_t)63;
    if (J.op == CROSS_OP_NTT_FORWARD || J.op == CROSS_OP_NTT_INVERSE) {
      const bool inv = J.op == CROSS_OP_NTT_INVERSE;
      std::vector<uint64_t> offs(J.params.L);
      for (uint32_t i = 0; i < J.params.L; ++i) offs[i] = i * N;
      add_ntt(b.get(), b->ntt[inv ? kNttInvD : kNttFwdExt], jp[j].plans, offs, J.data, mine,
              (uint64_t)J.params.L * N, (int)J.batch, inv);
      continue;
    }
    const CkksPlan* c = jp[j].c;
    const bool he = J.op == CROSS_OP_HE_MULT;
    const int L = c->L, K = c->K, LK = L + K, B = (int)J.batch;
    const uint64_t nd = (uint64_t)L * N, next = (uint64_t)c->dnum * LK * N, nacc = 2ull * LK * N;
    const uint64_t ntmp = std::max(next, nacc);
    uint32_t* d = mine;
    uint32_t* ext = d + B * nd;
    uint32_t* tmp = ext + B * next;
    uint32_t* acc = tmp + B * ntmp;
    uint32_t* z = acc + B * nacc;
    const uint64_t ct = 2 * nd;   // words per ciphertext
    const uint32_t* perm = nullptr;
    if (!he) {
      const int64_t half = (int64_t)N / 2;
      const uint64_t r = (uint64_t)((((int64_t)J.steps % half) + half) % half);
      cross_status st = perm_table(ctx, c->log_n, powmod(5, r, (uint32_t)(2 * N)), &perm);
      if (st != CROSS_OK) return st;
    }
    // from 2^14 up (R x 32 x 32) the inner product runs in the ModUp NTT's row kernel and
    // the tail in the ModDown NTT's: no digit copies, no extension limbs stored
    const bool fuse = c->log_n >= 14;
    for (int bb = 0; bb < B; ++bb) {
      const uint32_t* a = J.ct_a + bb * ct;
      uint32_t* o = J.out + bb * ct;
      uint32_t* db = d + bb * nd;
      if (he) {
        b->tensors.push_back(TensorTask{a, J.ct_b + bb * ct, o, db, c->mods, L, c->log_n, nd / 4});
        b->max_tensor = std::max(b->max_tensor, nd / 4);
      } else {
        b->autos.push_back(AutoTask{a, o, perm, c->log_n, nd});            // sigma(c0) -> out[0]
        b->autos.push_back(AutoTask{a + nd, db, perm, c->log_n, nd});      // sigma(c1) -> d
        b->max_auto = std::max(b->max_auto, nd);
      }
      if (fuse) continue;
      // ModUp: digit limbs copied unchanged, inactive digits zeroed
      uint32_t* eb = ext + bb * next;
      for (int dj = 0; dj < c->dnum; ++dj) {
        if (dj < c->ndig) {
          const int lo = dj * c->alpha, hi = std::min(L, (dj + 1) * c->alpha);
          const uint64_t cnt = (uint64_t)(hi - lo) * N / 4;
          b->copies.push_back(CopyTask{db + lo * N, eb + ((uint64_t)dj * LK + lo) * N, cnt});
          b->max_copy = std::max(b->max_copy, cnt);
        } else {
          b->copies.push_back(CopyTask{nullptr, eb + (uint64_t)dj * LK * N, (uint64_t)LK * N / 4});
          b->max_copy = std::max(b->max_copy, (uint64_t)LK * N / 4);
        }
      }
      b->inners.push_back(InnerTask{eb, J.key, acc + bb * nacc, c->mods, LK, c->dnum, c->ndig, c->log_n,
                                    (uint64_t)LK * N / 4});
      b->max_inner = std::max(b->max_inner, (uint64_t)LK * N / 4);
      for (int sidx = 0; sidx < 2; ++sidx) {
        const uint32_t* base = (he || sidx == 0) ? o + sidx * nd : nullptr;
        b->tails.push_back(TailTask{acc + bb * nacc + sidx * (uint64_t)LK * N, z + (bb * 2 + sidx) * nd, base,
                                    o + sidx * nd, c->tail, L, c->log_n, nd / 4});
        b->max_tail = std::max(b->max_tail, nd / 4);
      }
    }
    // INTT of d (all L limbs)
    const std::vector<Plan*>& bp = jp[j].plans;
    std::vector<Plan*> qp(bp.begin(), bp.begin() + L);
    std::vector<uint64_t> qo(L);
    for (int i = 0; i < L; ++i) qo[i] = i * N;
    // (fused: out of place into z, free until the ModDown, so d keeps its NTT form)
    add_ntt(b.get(), b->ntt[kNttInvD], qp, qo, d, tmp, nd, B, true, fuse ? z : nullptr);
    // BConv of each digit, NTT of every converted limb
    std::vector<Plan*> ep;
    std::vector<uint64_t> eo;
    for (int dj = 0; dj < c->ndig; ++dj) {
      const BconvStatic& bs = c->modup[dj];
      BconvLaunch g{bs.src, bs.dst, bs.table, bs.nsrc, bs.ndst, fuse ? z : d, ext, nd, next, B, c->log_n, bs.wide};
      b->bconv_up.push_back(g);
      b->max_cols_up = std::max(b->max_cols_up, (uint64_t)B << c->log_n);
      b->max_nsrc_up = std::max(b->max_nsrc_up, bs.nsrc);
    }
    // the converted limbs target-major (one prime's transforms adjacent: its step-2
    // twiddles are fetched into one L2)
    for (int t = 0; t < LK; ++t)
      for (int dj = 0; dj < c->ndig; ++dj)
        if (std::find(c->targets[dj].begin(), c->targets[dj].end(), t) != c->targets[dj].end()) {
          ep.push_back(bp[t]);
          eo.push_back(((uint64_t)dj * LK + t) * N);
        }
    add_ntt(b.get(), b->ntt[kNttFwdExt], ep, eo, ext, tmp, next, B, false, nullptr, fuse);
    const int log_r = bp[0]->log_r;
    if (fuse) {
      std::vector<IpLimb> lm(LK);
      const std::vector<int> order = ip_limb_order(L, K);
      for (int pos = 0; pos < LK; ++pos) {
        const int t = order[pos];
        // Barrett constants of the key products: k = bit length of q, m = floor(2^(2k) / q)
        const uint32_t q = bp[t]->q;
        uint32_t k = 0;
        while ((1ull << k) <= q) ++k;
        const uint32_t m = (uint32_t)(((unsigned __int128)1 << (2 * k)) / q);
        lm[pos] = IpLimb{bp[t]->row_fwd_b, bp[t]->row_fwd_t3_mont, q, bp[t]->qinv, m, k,
                         t < L ? t / c->alpha : -1, t};
      }
      void* dl = nullptr;
      cross_status st = cached_device_copy(ctx, lm.data(), lm.size() * sizeof(IpLimb), &dl);
      if (st != CROSS_OK) return st;
      IpTask it{};
      it.p = RowsIp{(const IpLimb*)dl, tmp, d, J.key, acc, next, LK, L, B, c->ndig, log_r - 3};
      it.first_block = (int32_t)b->ip_blocks;
      b->ip_blocks += (int64_t)LK * B << (log_r - 3);
      b->ips.push_back(it);
    }
    // ModDown of both accumulators: INTT of P limbs, BConv P -> Q, NTT of Q limbs
    std::vector<Plan*> pp(bp.begin() + L, bp.end());
    std::vector<uint64_t> po(K);
    for (int k = 0; k < K; ++k) po[k] = (uint64_t)(L + k) * N;
    add_ntt(b.get(), b->ntt[kNttInvP], pp, po, acc, tmp, (uint64_t)LK * N, 2 * B, true);
    {
      const BconvStatic& bs = c->moddown;
      BconvLaunch g{bs.src, bs.dst, bs.table, bs.nsrc, bs.ndst, acc, z, (uint64_t)LK * N, nd, 2 * B, c->log_n, bs.wide};
      b->bconv_down.push_back(g);
      b->max_cols_down = std::max(b->max_cols_down, (uint64_t)(2 * B) << c->log_n);
      b->max_nsrc_down = std::max(b->max_nsrc_down, bs.nsrc);
    }
    add_ntt(b.get(), b->ntt[kNttFwdZ], qp, qo, z, tmp, nd, 2 * B, false, nullptr, fuse);
    if (fuse) {
      uint64_t pmod[64];
      for (int i = 0; i < L; ++i) {
        const uint32_t q = c->primes[i];
        uint64_t pm = 1;
        for (int k = 0; k < K; ++k) pm = pm * (c->primes[L + k] % q) % q;
        pmod[i] = pm;
      }
      for (int i = 0; i < L; ++i) {
        const Plan* p = bp[i];
        const uint32_t q = p->q;
        const uint32_t pinv = powmod(pmod[i], q - 2, q);
        RowsTailTask rt{};
        rt.r.tab = p->row_fwd_b;
        rt.r.tw1 = p->row_fwd_t3;
        rt.r.in = tmp + qo[i];
        rt.r.stride = nd;
        rt.r.q = q;
        rt.r.qinv = p->qinv;
        rt.r.npoly = 2 * B;
        rt.r.log_r = log_r;
        rt.r.first_block = (int32_t)b->rtail_blocks;
        rt.acc = acc + qo[i];
        rt.acc_stride = (uint64_t)LK * N;
        rt.base = J.out + qo[i];
        rt.out = J.out + qo[i];
        rt.out_stride = nd;
        rt.pinv = pinv;
        rt.pinv_shoup = (uint32_t)(((uint64_t)pinv << 32) / q);
        rt.base_only_even = he ? 0 : 1;
        b->rtail_blocks += (int64_t)(2 * B) << (log_r - 3);
        b->rtails.push_back(rt);
      }
    }
  }

  // ---- pass 3: device task lists ---------------------------------------------------
  if (size_only) {
    *need = scratch + task_list_bytes(b.get());
    b->external = true;   // nothing was allocated: destroy must not synchronise
    return CROSS_OK;
  }
  if (ext_ws) {
    if ((reinterpret_cast<uintptr_t>(ext_ws) & 255) != 0 || ext_bytes < scratch + task_list_bytes(b.get()))
      return fail(ctx, CROSS_EINVAL, "workspace must be 256-byte aligned and at least cross_batch_workspace_bytes");
    b->ext_cursor = static_cast<char*>(ext_ws) + scratch;
    b->ext_lists = b->ext_cursor;
    b->ext_end = static_cast<char*>(ext_ws) + ext_bytes;
    b->upload_stream = upload_stream;
  }
  cross_status st = CROSS_OK;
  for (auto& ph : b->ntt)
    for (auto& hf : ph.half) {
      for (auto& kv : hf.gemm) {
        if (st == CROSS_OK) st = upload(b.get(), kv.second.tasks, &kv.second.d_tasks);
        if (st == CROSS_OK) st = upload(b.get(), kv.second.tiles, &kv.second.d_tiles);
      }
      if (st == CROSS_OK) st = upload(b.get(), hf.rows.tasks, &hf.rows.d_tasks);
    }
  if (st == CROSS_OK) st = upload(b.get(), b->autos, &b->d_autos);
  if (st == CROSS_OK) st = upload(b.get(), b->tensors, &b->d_tensors);
  if (st == CROSS_OK) st = upload(b.get(), b->copies, &b->d_copies);
  if (st == CROSS_OK) st = upload(b.get(), b->bconv_up, &b->d_bconv_up);
  if (st == CROSS_OK) st = upload(b.get(), b->bconv_down, &b->d_bconv_down);
  if (st == CROSS_OK) st = upload(b.get(), b->inners, &b->d_inners);
  if (st == CROSS_OK) st = upload(b.get(), b->tails, &b->d_tails);
  if (st == CROSS_OK) st = upload(b.get(), b->ips, &b->d_ips);
  if (st == CROSS_OK) st = upload(b.get(), b->rtails, &b->d_rtails);
  if (st == CROSS_OK && b->external) st = finish_upload(b.get());
  if (st != CROSS_OK) return st;

  if (use_graph) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
      return fail(ctx, CROSS_EDEVICE, "capture stream creation failed");
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = run_phases(b.get(), cs, false);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess) e = e2;
    b->graph = g;
    if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  }
  *out = b.release();
  return CROSS_OK;
}

}  // namespace
}  // namespace cross

extern "C" {

cross_status cross_batch_create(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, int use_graph,
                                cross_batch* out) {
  return build_batch(ctx, jobs, njobs, use_graph, nullptr, 0, nullptr, false, nullptr, out);
}

cross_status cross_batch_workspace_bytes(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, uint64_t* bytes) {
  if (!bytes) return CROSS_EINVAL;
  return build_batch(ctx, jobs, njobs, 0, nullptr, 0, nullptr, true, bytes, nullptr);
}

cross_status cross_batch_create_in(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, int use_graph,
                                   void* workspace, uint64_t workspace_bytes, void* stream, cross_batch* out) {
  if (!workspace) return ctx ? fail(ctx, CROSS_EINVAL, "null workspace") : CROSS_EINVAL;
  return build_batch(ctx, jobs, njobs, use_graph, workspace, workspace_bytes, static_cast<hipStream_t>(stream),
                     false, nullptr, out);
}

cross_status cross_get_batch_tile(cross_ctx ctx, uint32_t log_n, int inverse, int* tile, int* tuned) {
  if (!ctx || !tile || !tuned) return CROSS_EINVAL;
  if (log_n < 12 || log_n > CROSS_MAX_LOG_N) return fail(ctx, CROSS_EINVAL, "log_n outside 12..16");
  const bool inv = inverse != 0;
  auto it = ctx->list_tile.find(2 * (int)log_n + (inv ? 1 : 0));
  *tuned = it != ctx->list_tile.end();
  // the first step: the row-side step (U = R) in three factors, else U = R forward, C inverse
  int log_u = (int)log_n - 10;
  if (log_n < 14) {
    const int lr = split_of(ctx, (int)log_n);
    log_u = inv ? (int)log_n - lr : lr;
  }
  *tile = list_tile_for(ctx, (int)log_n, inv, 4 << log_u);
  return CROSS_OK;
}

cross_status cross_batch_run(cross_batch b, void* stream) {
  if (!b) return CROSS_EINVAL;
  cross_ctx ctx = b->ctx;
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, CROSS_EDEVICE, "hipSetDevice failed");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (b->exec) {
    ProfScope ps(ctx, "batch_graph", s, true);
    e = hipGraphLaunch(b->exec, s);
  } else {
    e = run_phases(b, s, true);
  }
  if (e != hipSuccess) return fail(ctx, CROSS_EDEVICE, std::string("batch run: ") + hipGetErrorString(e));
  return CROSS_OK;
}

cross_status cross_batch_info(cross_batch b, uint32_t* launches, uint64_t* workspace_bytes, uint64_t* gemm_tiles) {
  if (!b) return CROSS_EINVAL;
  uint32_t n = 0;
  uint64_t tiles = 0;
  for (auto& ph : b->ntt)
    for (auto& hf : ph.half) {
      for (auto& kv : hf.gemm) {
        n += kv.second.tiles.empty() ? 0 : 1;
        tiles += kv.second.tiles.size();
      }
      n += hf.rows.tasks.empty() ? 0 : 1;
    }
  n += !b->autos.empty() + !b->tensors.empty() + !b->copies.empty() + !b->bconv_up.empty() +
       !b->bconv_down.empty() + !b->inners.empty() + !b->tails.empty() + !b->ips.empty() + !b->rtails.empty();
  if (launches) *launches = n;
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  if (gemm_tiles) *gemm_tiles = tiles;
  return CROSS_OK;
}

}  // extern "C"
