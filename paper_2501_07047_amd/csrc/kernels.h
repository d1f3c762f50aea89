// Internal interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cross {

// One limb of one BAT NTT step: all `npoly` polynomials of the limb share the
// prime and therefore the table.  Offsets are in uint32 elements from the
// launch's base pointers, so a job list can be reused for any buffer.
struct GemmJob {
  const int8_t* table;     // tile-major BAT-expanded matrix (params.h, bat_expand)
  const uint32_t* tw;      // step-2 twiddles (Montgomery form) or nullptr
  uint64_t src_off, dst_off;
  uint32_t q, qinv;        // prime and q^-1 mod 2^32
};

// Step kinds of the layout-invariant 3-step NTT.
//  LEFT : out[u][v] = sum_r T[r][u] X[r][v]   (pre-known matrix on the left; step 1)
//  RIGHT: out[v][u] = sum_c X[v][c] T[c][u]   (pre-known matrix on the right; step 3)
// For LEFT, u runs over rows (R of them) and v over columns (C); for RIGHT,
// u runs over columns (C) and v over rows (R).
enum StepKind { kLeft = 0, kRight = 1 };

struct GemmLaunch {
  const GemmJob* jobs;     // device array
  int njobs;
  const uint32_t* src;
  uint32_t* dst;
  uint64_t src_stride, dst_stride;   // elements between successive polynomials of a job
  int npoly;
  int log_r, log_c;
  int kind;                // StepKind
  bool in_packed, out_packed, twiddle;
};

hipError_t launch_bat_gemm(const GemmLaunch& g, hipStream_t s);

struct ButterflyJob {
  const uint32_t* tw;      // psi^brv(i) (or its inverse), Montgomery form, N entries
  uint64_t off;            // element offset of the limb in the launch's buffer
  uint32_t q, qinv, ninv;  // ninv: N^-1 * 2^32 mod q (inverse only)
};
hipError_t launch_butterfly(const ButterflyJob* jobs, int njobs, uint32_t* data, uint64_t stride,
                            int npoly, int log_n, bool inverse, hipStream_t s);

}  // namespace cross
