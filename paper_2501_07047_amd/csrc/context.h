// Library context: device tables, job-list cache and per-stream workspace.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cross.h"
#include "kernels.h"

namespace cross {

// Device-resident tables of one (q, N, R) NTT plan.
struct Plan {
  uint32_t q = 0, qinv = 0, psi = 0;
  int log_n = 0, log_r = 0;
  int log_c1 = 0;           // > 0: three factors, the row transform split as C1 x C2
  int8_t *fwd_left = nullptr, *fwd_right = nullptr, *inv_left = nullptr, *inv_right = nullptr;
  int8_t *fwd_left_plain = nullptr, *fwd_right_plain = nullptr;      // without the Montgomery factor
  int8_t *inv_left_plain = nullptr, *inv_right_plain = nullptr;
  uint32_t *fwd_tw = nullptr, *inv_tw = nullptr, *bf_fwd = nullptr, *bf_inv = nullptr;
  int8_t *row_fwd_b = nullptr, *row_fwd_c = nullptr, *row_inv_c = nullptr, *row_inv_b = nullptr;
  int8_t *row_fwd_b_plain = nullptr, *row_fwd_c_plain = nullptr;   // without the Montgomery factor
  int8_t *row_inv_c_plain = nullptr, *row_inv_b_plain = nullptr;
  uint32_t bar_m = 0, bar_k = 0;              // Barrett constants: floor(2^(2k) / q), k = bit length
  uint32_t *row_fwd_t3 = nullptr, *row_inv_t3 = nullptr, *inv_tw_rows = nullptr;
  uint32_t* row_fwd_t3_mont = nullptr;        // T3 x 2^32 (fused ModUp NTT + inner product)
  uint32_t bf_ninv = 0;
  bool wide = false;        // 2^28 <= q < 2^31: signed-digit tables, byte operands
  void* block = nullptr;
};

// A device buffer that only grows; freed when the context goes away.
struct DevBuf {
  void* ptr = nullptr;
  size_t size = 0;
};

struct Status {
  cross_status code;
  std::string msg;
};

// Event bracket around one kernel launch (no-op unless profiling is enabled).
// The library's kernel launches inside the scope stamp its events from their
// dispatches (no extra queue packets); with markers = true (a scope around work
// that is not launched by the library, such as a graph launch) the events are
// recorded on the stream instead.
struct ProfScope {
  cross_ctx ctx;
  hipStream_t s;
  int idx = -1;
  bool markers = false;
  LaunchEvents prev;
  ProfScope(cross_ctx c, const char* name, hipStream_t st, bool markers = false);
  ~ProfScope();
};

}  // namespace cross

struct cross_ctx_s {
  int device = 0;
  std::string err;
  std::map<std::tuple<uint32_t, int, int, int>, cross::Plan*> plans;   // (q, log_n, log_r, log_c1)
  std::map<std::string, void*> job_cache;     // serialised job list -> device copy
  std::map<hipStream_t, cross::DevBuf> workspace;
  std::map<int, int> split;                   // log_n -> log_r override (two factors)
  std::map<int, std::pair<int, int>> split3;  // log_n -> (log_r, log_c1); log_c1 = 0: two factors
                                              // (absent: the size's default)
  int gemm_tile = 0;                          // GemmTile override (0 = auto)
  int ntt_reduction = 0;                      // row-kernel epilogue: 0 Montgomery, 1 Barrett
  int ntt_engine = 0;                         // NTTs inside other operations: 0 MFMA, 1 butterfly
  std::map<int, int> tile_by_logn;            // autotuned GemmTile per transform size
  std::map<int, int> list_tile;               // batch runtime: GemmListTile per (2 log_n + inverse)
  std::map<std::string, void*> const_cache;   // other device-resident constants
  std::map<std::string, std::shared_ptr<void>> ext_plans;   // CKKS plans (host structs)
  // Pinned host buffers for stream-ordered task-list uploads, reused across batches:
  // `ev` is recorded after the last copy out of the buffer, and a buffer is handed
  // out again only once that copy has finished.
  struct Pinned {
    void* p = nullptr;
    size_t size = 0;
    hipEvent_t ev = nullptr;
    bool busy = false;
  };
  std::vector<Pinned> pinned;
  void* noalloc_scratch = nullptr;            // device address of this device's no-alloc scratch
  bool debug_check = false;                   // residue-range check of every input (CROSS_DEBUG_CHECK)
  unsigned long long* debug_flag = nullptr;   // device word of the check
  // While set (cross_ntt_noalloc), job lists go into this arena with stream-ordered
  // copies instead of the allocating cache.
  struct Arena {
    char* base = nullptr;
    size_t cap = 0, used = 0;
    hipStream_t stream = nullptr;
  } arena;
  bool prof = false;
  std::string prof_only;                      // time only this kernel family ("" = all)
  struct ProfRec {
    std::string name;
    hipEvent_t a, b;
    bool valid;           // both events were stamped by this scope
  };
  std::vector<ProfRec> prof_recs;
  std::vector<hipEvent_t> prof_pool;          // events of finished reports, reused
};

namespace cross {

cross_status fail(cross_ctx ctx, cross_status code, const std::string& msg);
// wide_ok: the NTT also takes wide primes, 2^28 <= q < 2^31 (every other operation
// needs q < 2^28).
cross_status check_prime(cross_ctx ctx, uint32_t q, uint32_t log_n, bool wide_ok = false);
// allow3 = false keeps the two-factor form even where a three-factor split is set
// (the batch runtime's work lists implement two factors only).
cross_status get_plan(cross_ctx ctx, uint32_t q, int log_n, Plan** out, bool allow3 = true);
// The plan of an explicit split (log_c1 = 0: two factors); built on first use.
cross_status get_plan_at(cross_ctx ctx, uint32_t q, int log_n, int log_r, int log_c1, Plan** out);
int split_of(cross_ctx ctx, int log_n);
// The (log_r, log_c1) get_plan uses for size 2^log_n (log_c1 = 0: two factors).
void effective_split(cross_ctx ctx, int log_n, bool allow3, int* log_r, int* log_c1);
// Device copy of a POD array, cached by content.
cross_status cached_device_copy(cross_ctx ctx, const void* host, size_t bytes, void** out);
// Debug mode (ctx->debug_check): every coefficient of npoly polynomials `stride`
// apart, limb i at offset i * N with prime qs[i], must be below its prime; checked
// on the device and synchronously on `s`.  CROSS_EDOMAIN names the first offender.
cross_status check_residues(cross_ctx ctx, const char* what, const uint32_t* base, uint64_t stride, int npoly,
                            const uint32_t* qs, int nl, int log_n, hipStream_t s);
// Device address of `device`'s copy of the allocation-free NTT's scratch array
// (looked up once per device).
hipError_t noalloc_scratch_address(int device, void** out);
// Per-stream scratch of at least `bytes`.
cross_status workspace(cross_ctx ctx, hipStream_t s, size_t bytes, void** out);
// A pinned host buffer of at least `bytes` from the context's pool (index in *idx),
// free to overwrite; pinned_release returns it, after its last copy was recorded
// on its event.
cross_status pinned_acquire(cross_ctx ctx, size_t bytes, int* idx);
void pinned_release(cross_ctx ctx, int idx);

// Run forward / inverse NTTs for a list of limbs, each given by (plan, element
// offset) inside `data` with `npoly` polynomials at `stride` elements apart.
// `tmp` must hold (max offset + npoly*stride) elements laid out like data.  With
// dst (laid out like data, overlapping neither data nor tmp) the result goes there
// and data keeps its input (the butterfly path copies the limbs to dst first).
cross_status ntt_limbs(cross_ctx ctx, const std::vector<Plan*>& plans,
                       const std::vector<uint64_t>& offs, uint32_t* data, uint64_t stride,
                       int npoly, bool inverse, uint32_t* tmp, hipStream_t s, uint32_t* dst = nullptr);
// Whether the forward NTT of these limbs can end in the fused ModDown tail: the
// MFMA engine with the Montgomery epilogue, narrow primes, and a three-factor split
// whose row kernel has the fused form.
bool ntt_tail_fusable(cross_ctx ctx, const std::vector<Plan*>& plans);
// Forward NTT of the listed limbs of `data` (as ntt_limbs) whose row kernel applies
// `tail` instead of writing the transform back (data is left in its input state
// except where tail.out overlaps it); CROSS_EUNSUPPORTED when !ntt_tail_fusable.
cross_status ntt_limbs_tail(cross_ctx ctx, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
                            uint32_t* data, uint64_t stride, int npoly, uint32_t* tmp, const RowsTail& tail,
                            hipStream_t s);
// Only the first launch of the forward three-factor NTT of these limbs: the row-side
// step data -> tmp (packed, step-2 twiddle applied), for a fused row kernel to finish;
// CROSS_EUNSUPPORTED when !ntt_tail_fusable.
cross_status ntt_rowside_forward(cross_ctx ctx, const std::vector<Plan*>& plans, const std::vector<uint64_t>& offs,
                                 uint32_t* data, uint64_t stride, int npoly, uint32_t* tmp, hipStream_t s);

}  // namespace cross
