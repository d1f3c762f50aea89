// Residue-range check of the debug mode (CROSS_DEBUG_CHECK): every input residue
// of an entry point must lie in [0, q) of its limb's prime.  One thread checks
// four consecutive coefficients (one 16-byte load); the first offending position
// (lowest polynomial, limb, coefficient) is kept with a 64-bit atomic minimum.
#include "kernels.h"

namespace cross {

namespace {

__global__ void residue_check_kernel(const uint32_t* base, uint64_t stride, int npoly, const CheckLimb* limbs,
                                     int nl, int log_n, unsigned long long* first) {
  const uint64_t N = 1ull << log_n;
  const uint64_t i4 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i4 >= (N >> 2)) return;
  const int l = blockIdx.y;
  const CheckLimb lm = limbs[l];
  for (int p = blockIdx.z; p < npoly; p += gridDim.z) {
    const uint4 v = *reinterpret_cast<const uint4*>(base + (uint64_t)p * stride + lm.off + 4 * i4);
    const uint32_t x[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (x[k] >= lm.q) {
        const unsigned long long pos = ((unsigned long long)p * nl + l) * N + 4 * i4 + k;
        atomicMin(first, pos);
      }
  }
}

}  // namespace

hipError_t launch_residue_check(const uint32_t* base, uint64_t stride, int npoly, const CheckLimb* limbs, int nl,
                                int log_n, unsigned long long* first, hipStream_t s) {
  if (npoly <= 0 || nl <= 0) return hipSuccess;
  if (log_n < 4 || nl > 65535) return hipErrorInvalidValue;
  const uint64_t n4 = (1ull << log_n) >> 2;
  dim3 grid((unsigned)((n4 + 255) / 256), (unsigned)nl, (unsigned)(npoly < 1024 ? npoly : 1024));
  launch_kernel(residue_check_kernel, grid, dim3(256), 0, s, base, stride, npoly, limbs, nl, log_n, first);
  return hipGetLastError();
}

}  // namespace cross
