// Internal declarations of the closure network kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include "adimx_internal.h"

#include <cstddef>

namespace adimx {
namespace nn {

struct ConvArgs {
  const __bf16* in;     // [V][CI] channels last (CI = 16 or 32, zero padded)
  const __bf16* wt;     // B operand [COP][27*CI], k = tap*CI + ci
  const float* bias;    // [COP] (forward) or null
  const float* zprev;   // backward data: pre-activation [V][COP] of the layer below
  float* out_f32;       // forward: last layer [V][co_real] / hidden z [V][COP]
  __bf16* out_bf16;     // hidden silu(z) [V][COP] / backward data dz [V][COP]
  int nx, ny, nz;
  int co_real;          // valid output channels of the last layer
};

struct WgradArgs {
  const __bf16* in;     // layer input [V][CI]
  const __bf16* dz;     // gradient of the layer output (pre-activation) [V][COP]
  float* part;          // per-block partials [blocks][27*CI*COP + COP]
  int nx, ny, nz;
};

hipError_t launch_conv(int ci, int cop, int epi, const ConvArgs& a, hipStream_t s);
int wgrad_blocks(int nx, int ny, int nz);
hipError_t launch_wgrad(int ci, int cop, const WgradArgs& a, int cin, int cout, float* grad,
                        hipStream_t s);
hipError_t launch_layout(const float* Wm, const float* bm, int cin, int cout, int CIP, int COP,
                         __bf16* wf, __bf16* wb, float* bias_pad, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s);
hipError_t launch_pack(const float* src, int creal, int CP, size_t V, __bf16* dst, hipStream_t s);
hipError_t launch_mse(const float* y, const float* t, size_t count, float* dy, float* partial,
                      int nblocks, hipStream_t s);

// Solver <-> network glue (state: six n^3 components [c][v] of type T).
constexpr int kFeatures = 16;  // network inputs per coefficient
constexpr int kOutputs = 6;    // corrections of E1..E3, H1..H3
template <typename T>
hipError_t launch_state_scale(const T* state, size_t count, float* partial, int nblk,
                              float* scale, hipStream_t s);
template <typename T, typename O>
hipError_t launch_features(const T* state, const T* prev, const float* mat, int n,
                           const float* scale, const SourceArgs& src, const double* tnow,
                           double dt, O* x, hipStream_t s);
template <typename T>
hipError_t launch_target(const T* fine, const T* coarse, size_t D, const float* scale, float* t,
                         hipStream_t s);
template <typename T>
hipError_t launch_apply(T* state, int n, const float* y, const float* scale, const int* flag,
                        hipStream_t s);
// Gate: flag = (RMS of scale * y > limit * RMS of state - prev); partial
// holds 2 nblk floats.
template <typename T>
hipError_t launch_gate(const float* y, const T* state, const T* prev, size_t count, float* partial,
                       int nblk, const float* scale, float limit, int* flag, int* rejected,
                       hipStream_t s);

}  // namespace nn
}  // namespace adimx

struct adi_nn;
namespace adimx {
namespace nn {
// Network buffers sized for an nx x ny x nz grid (features x [V][cin],
// output y [V][cout], scale and reduction partials), and the forward pass.
int closure_buffers(adi_nn* n, int nx, int ny, int nz, float** x, float** y, float** scale,
                    float** partial);
int closure_forward(adi_nn* n, const float* x, float* y, int nx, int ny, int nz, hipStream_t s);
// The network's packed bf16 input buffer [V][16] (after closure_buffers),
// and an inference forward that starts from it (no packing step).
__bf16* closure_input16(adi_nn* n);
int closure_forward_packed(adi_nn* n, float* y, int nx, int ny, int nz, hipStream_t s);
int closure_cin(const adi_nn* n);
int closure_cout(const adi_nn* n);
}  // namespace nn
}  // namespace adimx
