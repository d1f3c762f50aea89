// Baseline: plain radix-2 butterfly negacyclic NTT on the vector ALUs
// (arXiv 2501.07047, App. "Radix-2 Cooley-Tukey NTT (Butterfly NTT)": log N
// stages of N/2 modular multiply/add/subtract with bit-complement shuffles).
//
// Forward: Cooley-Tukey, natural order in, bit-reversed order out; stage with
// m groups of half-width t uses twiddle psi^brv_N(m + group).  Inverse:
// Gentleman-Sande with psi^-brv_N, N^-1 applied in the last stage.  The
// printed algorithm is cyclic and its indices are garbled; this follows the
// textbook negacyclic form, which produces the same bit-reversed order as the
// 3-step MFMA path so the two agree bit for bit.
//
// Deliberately plain: one launch per stage, one butterfly per thread, every
// stage reads and writes the whole array in HBM.  This is the comparison
// baseline, not a tuned NTT.
#include "kernels.h"

namespace cross {

namespace {

__device__ __forceinline__ uint32_t mont_mul(uint32_t a, uint32_t b, uint32_t q, uint32_t qinv) {
  // a < 2q, b < q (Montgomery form): a*b*2^-32 mod q in (0, 2q)
  uint64_t z = (uint64_t)a * b;
  uint32_t t = (uint32_t)z * qinv;
  return (uint32_t)(z >> 32) + q - __umulhi(t, q);
}

__global__ void __launch_bounds__(256)
bf_stage_kernel(const ButterflyJob* jobs, uint32_t* data, uint64_t stride, int npoly, int log_n,
                int log_m, bool inverse, bool last) {
  const int half = 1 << (log_n - 1);
  const int per_poly = half;
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int job_id = blockIdx.y;
  if (idx >= (uint64_t)per_poly * npoly) return;
  const int poly = (int)(idx >> (log_n - 1));
  const int i = (int)(idx & (half - 1));
  const ButterflyJob jb = jobs[job_id];
  uint32_t* a = data + jb.off + (uint64_t)poly * stride;
  const uint32_t q = jb.q, qinv = jb.qinv;
  const int log_t = log_n - 1 - log_m;       // half-width t = N / (2m)
  const int grp = i >> log_t;
  const int j = i & ((1 << log_t) - 1);
  const int j1 = (grp << (log_t + 1)) + j;
  const int j2 = j1 + (1 << log_t);
  const uint32_t w = jb.tw[(1 << log_m) + grp];
  uint32_t u = a[j1], v = a[j2];
  if (!inverse) {
    uint32_t vw = mont_mul(v, w, q, qinv);
    if (vw >= q) vw -= q;
    uint32_t x = u + vw;
    if (x >= q) x -= q;
    uint32_t y = u + q - vw;
    if (y >= q) y -= q;
    a[j1] = x;
    a[j2] = y;
  } else {
    uint32_t x = u + v;
    if (x >= q) x -= q;
    uint32_t y = mont_mul(u + q - v, w, q, qinv);
    if (last) x = mont_mul(x, jb.ninv, q, qinv);
    if (last) y = mont_mul(y, jb.ninv, q, qinv);
    if (x >= q) x -= q;
    if (y >= q) y -= q;
    a[j1] = x;
    a[j2] = y;
  }
}

}  // namespace

hipError_t launch_butterfly(const ButterflyJob* jobs, int njobs, uint32_t* data, uint64_t stride,
                            int npoly, int log_n, bool inverse, hipStream_t s) {
  const uint64_t work = ((uint64_t)1 << (log_n - 1)) * npoly;
  dim3 grid((unsigned)((work + 255) / 256), (unsigned)njobs);
  for (int st = 0; st < log_n; ++st) {
    // forward: m = 1, 2, ..., N/2; inverse: m = N/2, ..., 1
    int log_m = inverse ? (log_n - 1 - st) : st;
    launch_kernel(bf_stage_kernel, grid, dim3(256), 0, s, jobs, data, stride, npoly, log_n,
                       log_m, inverse, inverse && st == log_n - 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace cross
