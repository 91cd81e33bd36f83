// Internal declarations of the manufactured-solution kernels (not ABI).
#pragma once

#include <hip/hip_runtime.h>

namespace adimx {
namespace mms {

constexpr int kMaxErrorBlocks = 2048;

// Size of the fixed device array behind adi_mms_errors_noalloc (one copy per
// GPU, held until the process ends).
constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;

// Device address of the current GPU's copy of that array (looked up with
// hipGetSymbolAddress once per device, then cached).
hipError_t noalloc_scratch(double** out);

// Quadrature tables per axis a (x, y, z): Q_a = N_a q Gauss points, for
// point g the basis functions g/q .. g/q + p (element g/q) with values
// bv[a][g*(p+1) + r] and derivatives bd[a][g*(p+1) + r]; coordinates x[a][g]
// and weights w[a][g].
struct Tables {
  const double* x[3];
  const double* w[3];
  const double* bv[3];
  const double* bd[3];
  int N[3], p, q;
};

// vals[c * Qx Qy Qz + point] = component c (E1..E3, H1..H3) of the
// manufactured solution at time t on the tensor grid of quadrature points
// (x fastest).
hipError_t launch_exact(const Tables& tb, double t, double* vals, hipStream_t s);
// L2 projection right-hand sides (f_c, B_i B_j B_k) into the six state
// components (type T, nx ny nz each), constrained coefficients set to zero.
template <typename T>
hipError_t launch_project_rhs(const Tables& tb, const double* vals, T* state, hipStream_t s);
// Per-block partial sums of the squared errors of the state against the
// manufactured solution at time t: [block][0] E L2, [1] E curl, [2] H L2,
// [3] H curl.  Returns the number of blocks written (nblk <= kMaxErrorBlocks);
// every block writes its four sums (nothing needs clearing).
template <typename T>
hipError_t launch_errors(const Tables& tb, const T* state, double t, double* partial,
                         int* nblk, hipStream_t s);

}  // namespace mms
}  // namespace adimx
