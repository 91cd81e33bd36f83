// Host side of the learned closure network: parameters (float32 master
// copy, Adam moments), bfloat16 operand layouts, activation buffers, and the
// forward / backward / Adam / loss entry points of the C ABI.
#include "adimx.h"
#include "closure_internal.h"

#include <cmath>
#include <string>
#include <vector>

using namespace adimx::nn;

struct adi_nn {
  hipStream_t stream = nullptr;
  int cin = 9, ch = 32, cout = 6;
  int P = 0;
  int woff[3] = {}, boff[3] = {};
  int lin[3] = {}, lout[3] = {}, CIP[3] = {}, COP[3] = {};
  float *master = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  __bf16* wf[3] = {};
  __bf16* wb[3] = {};
  float* bias[3] = {};
  // activations of the last forward (grid nx, ny, nz)
  int nx = 0, ny = 0, nz = 0;
  size_t V = 0;
  __bf16 *x16 = nullptr, *a1 = nullptr, *a2 = nullptr, *dz3 = nullptr, *dz2 = nullptr, *dz1 = nullptr;
  float *z1 = nullptr, *z2 = nullptr, *part = nullptr, *partial = nullptr;
  float *xbuf = nullptr, *ybuf = nullptr, *scale = nullptr;
  std::vector<void*> owned;
  std::string err;
  bool forward_done = false;
};

namespace {

int nn_fail(adi_nn* n, int code, const std::string& msg) {
  if (n) n->err = msg;
  return code;
}

#define NNCHK(nn, expr)                                                                 \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return nn_fail(nn, ADI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <typename X>
hipError_t dalloc(adi_nn* n, X** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(X));
  if (e == hipSuccess) {
    n->owned.push_back(q);
    *p = static_cast<X*>(q);
  }
  return e;
}

void free_acts(adi_nn* n) {
  void* bufs[] = {n->x16, n->a1, n->a2, n->dz3, n->dz2, n->dz1, n->z1, n->z2, n->part,
                  n->xbuf, n->ybuf};
  for (void* b : bufs) {
    if (!b) continue;
    hipFree(b);
    for (auto& o : n->owned)
      if (o == b) o = nullptr;
  }
  n->x16 = n->a1 = n->a2 = n->dz3 = n->dz2 = n->dz1 = nullptr;
  n->z1 = n->z2 = n->part = n->xbuf = n->ybuf = nullptr;
  n->V = 0;
}

int ensure_acts(adi_nn* n, int nx, int ny, int nz) {
  const size_t V = size_t(nx) * ny * nz;
  if (V == n->V && nx == n->nx && ny == n->ny && nz == n->nz) return ADI_OK;
  free_acts(n);
  NNCHK(n, dalloc(n, &n->x16, V * 16));
  NNCHK(n, dalloc(n, &n->a1, V * 32));
  NNCHK(n, dalloc(n, &n->a2, V * 32));
  NNCHK(n, dalloc(n, &n->dz3, V * 16));
  NNCHK(n, dalloc(n, &n->dz2, V * 32));
  NNCHK(n, dalloc(n, &n->dz1, V * 32));
  NNCHK(n, dalloc(n, &n->z1, V * 32));
  NNCHK(n, dalloc(n, &n->z2, V * 32));
  NNCHK(n, dalloc(n, &n->xbuf, V * size_t(n->cin)));
  NNCHK(n, dalloc(n, &n->ybuf, V * size_t(n->cout)));
  const size_t blocks = size_t(wgrad_blocks(nx, ny, nz));
  NNCHK(n, dalloc(n, &n->part, blocks * (27 * 32 * 32 + 32)));
  n->V = V;
  n->nx = nx;
  n->ny = ny;
  n->nz = nz;
  n->forward_done = false;
  return ADI_OK;
}

int relayout(adi_nn* n, hipStream_t s) {
  for (int l = 0; l < 3; ++l)
    NNCHK(n, launch_layout(n->master + n->woff[l], n->master + n->boff[l], n->lin[l], n->lout[l],
                           n->CIP[l], n->COP[l], n->wf[l], l > 0 ? n->wb[l] : nullptr,
                           n->bias[l], s));
  return ADI_OK;
}

// Forward of the three layers on x (float32 [V][cin], device); output y
// (float32 [V][cout], device).  With keep (training) the hidden layers'
// float32 pre-activations are kept for the backward pass; without it
// (inference) only their bf16 activations are written, the same values.
int forward_on(adi_nn* n, const float* x, float* y, int nx, int ny, int nz, hipStream_t s,
               bool keep = true) {
  int st = ensure_acts(n, nx, ny, nz);
  if (st != ADI_OK) return st;
  if (x) NNCHK(n, launch_pack(x, n->cin, 16, n->V, n->x16, s));  // else x16 is filled
  const int hidden = keep ? 1 : 3;
  ConvArgs a{};
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.in = n->x16; a.wt = n->wf[0]; a.bias = n->bias[0]; a.out_f32 = n->z1; a.out_bf16 = n->a1;
  NNCHK(n, launch_conv(16, 32, hidden, a, s));
  a.in = n->a1; a.wt = n->wf[1]; a.bias = n->bias[1]; a.out_f32 = n->z2; a.out_bf16 = n->a2;
  NNCHK(n, launch_conv(32, 32, hidden, a, s));
  a.in = n->a2; a.wt = n->wf[2]; a.bias = n->bias[2]; a.out_f32 = y; a.out_bf16 = nullptr;
  a.co_real = n->cout;
  NNCHK(n, launch_conv(32, 16, 0, a, s));
  n->forward_done = keep;
  return ADI_OK;
}

}  // namespace

extern "C" {

int adi_nn_create(adi_nn** out, int cin, int chid, int cout, void* hip_stream) {
  if (!out) return ADI_EINVAL;
  *out = nullptr;
  if (cin < 1 || cin > 16 || chid != 32 || cout < 1 || cout > 16) return ADI_EINVAL;
  adi_nn* n = new adi_nn();
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->cin = cin;
  n->ch = chid;
  n->cout = cout;
  const int lin[3] = {cin, chid, chid}, lout[3] = {chid, chid, cout};
  const int CIP[3] = {16, 32, 32}, COP[3] = {32, 32, 16};
  int o = 0;
  for (int l = 0; l < 3; ++l) {
    n->lin[l] = lin[l];
    n->lout[l] = lout[l];
    n->CIP[l] = CIP[l];
    n->COP[l] = COP[l];
    n->woff[l] = o;
    o += 27 * lin[l] * lout[l];
    n->boff[l] = o;
    o += lout[l];
  }
  n->P = o;
  bool ok = dalloc(n, &n->master, o) == hipSuccess && dalloc(n, &n->grad, o) == hipSuccess &&
            dalloc(n, &n->m, o) == hipSuccess && dalloc(n, &n->v, o) == hipSuccess &&
            dalloc(n, &n->partial, 4096) == hipSuccess && dalloc(n, &n->scale, 64) == hipSuccess;
  for (int l = 0; l < 3 && ok; ++l) {
    ok = dalloc(n, &n->wf[l], size_t(COP[l]) * 27 * CIP[l]) == hipSuccess &&
         dalloc(n, &n->bias[l], size_t(COP[l])) == hipSuccess;
    if (ok && l > 0) ok = dalloc(n, &n->wb[l], size_t(CIP[l]) * 27 * COP[l]) == hipSuccess;
  }
  if (!ok) {
    adi_nn_destroy(n);
    return ADI_ENOMEM;
  }
  hipMemset(n->master, 0, size_t(o) * 4);
  hipMemset(n->m, 0, size_t(o) * 4);
  hipMemset(n->v, 0, size_t(o) * 4);
  hipMemset(n->grad, 0, size_t(o) * 4);
  *out = n;
  return relayout(n, n->stream) == ADI_OK ? ADI_OK : ADI_EHIP;
}

int adi_nn_param_count(const adi_nn* n) { return n ? n->P : ADI_EINVAL; }

int adi_nn_set_params(adi_nn* n, const float* host) {
  if (!n || !host) return ADI_EINVAL;
  for (int i = 0; i < n->P; ++i)
    if (!std::isfinite(host[i])) return nn_fail(n, ADI_ENONFINITE, "parameter not finite");
  NNCHK(n, hipStreamSynchronize(n->stream));
  NNCHK(n, hipMemcpy(n->master, host, size_t(n->P) * 4, hipMemcpyHostToDevice));
  NNCHK(n, hipMemset(n->m, 0, size_t(n->P) * 4));
  NNCHK(n, hipMemset(n->v, 0, size_t(n->P) * 4));
  return relayout(n, n->stream);
}

int adi_nn_get_params(adi_nn* n, float* host) {
  if (!n || !host) return ADI_EINVAL;
  NNCHK(n, hipStreamSynchronize(n->stream));
  NNCHK(n, hipMemcpy(host, n->master, size_t(n->P) * 4, hipMemcpyDeviceToHost));
  return ADI_OK;
}

int adi_nn_forward(adi_nn* n, const float* x_dev, float* y_dev, int nx, int ny, int nz) {
  if (!n || !x_dev || !y_dev || nx < 1 || ny < 1 || nz < 1) return ADI_EINVAL;
  return forward_on(n, x_dev, y_dev, nx, ny, nz, n->stream);
}

int adi_nn_backward(adi_nn* n, const float* dy_dev) {
  if (!n || !dy_dev) return ADI_EINVAL;
  if (!n->forward_done) return nn_fail(n, ADI_ESTATE, "adi_nn_forward first");
  hipStream_t s = n->stream;
  NNCHK(n, launch_pack(dy_dev, n->cout, 16, n->V, n->dz3, s));
  WgradArgs w{};
  w.nx = n->nx;
  w.ny = n->ny;
  w.nz = n->nz;
  w.part = n->part;
  // layer 3: dW3 from (a2, dz3); dz2 = (dz3 * W3^T) silu'(z2)
  w.in = n->a2; w.dz = n->dz3;
  NNCHK(n, launch_wgrad(32, 16, w, n->lin[2], n->lout[2], n->grad + n->woff[2], s));
  ConvArgs a{};
  a.nx = n->nx;
  a.ny = n->ny;
  a.nz = n->nz;
  a.in = n->dz3; a.wt = n->wb[2]; a.zprev = n->z2; a.out_bf16 = n->dz2;
  NNCHK(n, launch_conv(16, 32, 2, a, s));
  // layer 2
  w.in = n->a1; w.dz = n->dz2;
  NNCHK(n, launch_wgrad(32, 32, w, n->lin[1], n->lout[1], n->grad + n->woff[1], s));
  a.in = n->dz2; a.wt = n->wb[1]; a.zprev = n->z1; a.out_bf16 = n->dz1;
  NNCHK(n, launch_conv(32, 32, 2, a, s));
  // layer 1 (no input gradient needed)
  w.in = n->x16; w.dz = n->dz1;
  NNCHK(n, launch_wgrad(16, 32, w, n->lin[0], n->lout[0], n->grad + n->woff[0], s));
  return ADI_OK;
}

int adi_nn_get_grads(adi_nn* n, float* host) {
  if (!n || !host) return ADI_EINVAL;
  NNCHK(n, hipStreamSynchronize(n->stream));
  NNCHK(n, hipMemcpy(host, n->grad, size_t(n->P) * 4, hipMemcpyDeviceToHost));
  return ADI_OK;
}

int adi_nn_adam(adi_nn* n, float lr, float b1, float b2, float eps, int t) {
  if (!n || t < 1 || !(lr >= 0.f)) return ADI_EINVAL;
  NNCHK(n, launch_adam(n->master, n->grad, n->m, n->v, n->P, lr, b1, b2, eps, t, n->stream));
  return relayout(n, n->stream);
}

int adi_nn_mse(adi_nn* n, const float* y_dev, const float* t_dev, size_t count, float* dy_dev,
               double* loss) {
  if (!n || !y_dev || !t_dev || !dy_dev || count == 0) return ADI_EINVAL;
  const int nb = 1024;
  NNCHK(n, launch_mse(y_dev, t_dev, count, dy_dev, n->partial, nb, n->stream));
  if (loss) {
    std::vector<float> p(nb);
    NNCHK(n, hipMemcpyAsync(p.data(), n->partial, nb * 4, hipMemcpyDeviceToHost, n->stream));
    NNCHK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (float q : p) s += q;
    *loss = s / double(count);
  }
  return ADI_OK;
}

const char* adi_nn_last_error(const adi_nn* n) { return n ? n->err.c_str() : "invalid handle"; }

void adi_nn_destroy(adi_nn* n) {
  if (!n) return;
  if (n->stream) hipStreamSynchronize(n->stream);
  for (void* p : n->owned)
    if (p) hipFree(p);
  delete n;
}

}  // extern "C"

// --------------------------------------------------------------- internal
namespace adimx {
namespace nn {

// Used by adi_step_closure: network buffers sized for the grid, and the
// forward pass on a given stream.
int closure_buffers(adi_nn* n, int nx, int ny, int nz, float** x, float** y, float** scale,
                    float** partial) {
  int st = ensure_acts(n, nx, ny, nz);
  if (st != ADI_OK) return st;
  *x = n->xbuf;
  *y = n->ybuf;
  *scale = n->scale;
  *partial = n->partial;
  return ADI_OK;
}

int closure_forward(adi_nn* n, const float* x, float* y, int nx, int ny, int nz, hipStream_t s) {
  return forward_on(n, x, y, nx, ny, nz, s, false);
}

__bf16* closure_input16(adi_nn* n) { return n->x16; }

int closure_forward_packed(adi_nn* n, float* y, int nx, int ny, int nz, hipStream_t s) {
  return forward_on(n, nullptr, y, nx, ny, nz, s, false);
}

int closure_cin(const adi_nn* n) { return n->cin; }
int closure_cout(const adi_nn* n) { return n->cout; }

}  // namespace nn
}  // namespace adimx
