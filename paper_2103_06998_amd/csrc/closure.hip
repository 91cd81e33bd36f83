// gfx950 kernels of the learned closure: a three-layer 3x3x3 convolutional
// network on the coefficient grid (channels last, [z][y][x][c]), bfloat16
// operands with float32 accumulation on the MFMA units, trained on the GPU.
//
// Convolutions are implicit GEMMs: M = voxels (16 consecutive x per MFMA
// tile), N = output channels, K = 27 taps x input channels.  A block owns a
// 16 x 4 x 4 voxel tile; its input with a one-voxel halo is staged in LDS.
#include "adimx_internal.h"
#include "closure_internal.h"

#include <hip/hip_bf16.h>

namespace adimx {
namespace nn {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int TX = 16, TY = 4, TZ = 4;  // output tile (one wave per z row)
constexpr int HXX = TX + 2, HYY = TY + 2, HZZ = TZ + 2;
constexpr int HV = HXX * HYY * HZZ;     // staged voxels (648)
constexpr int kThreads = 256;

// The hardware reciprocal (1 ulp) instead of a correctly rounded division:
// the activations are rounded to bfloat16 (8 bits) right after.
__device__ __forceinline__ float sigmoid_f(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}
__device__ __forceinline__ float silu_f(float z) { return z * sigmoid_f(z); }
__device__ __forceinline__ float silu_grad_f(float z) {
  const float s = sigmoid_f(z);
  return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ bf16x8 zero8() {
  bf16x8 z;
#pragma unroll
  for (int j = 0; j < 8; ++j) z[j] = __bf16(0.0f);
  return z;
}

// ---------------------------------------------------------------- conv
// EPI 0: out_f32[v][co_real] = acc + bias                (last layer)
// EPI 1: z = acc + bias -> out_f32[v][COP] = z, out_bf16 = silu(z)  (hidden)
// EPI 2: out_bf16[v][COP] = acc * silu'(zprev[v][COP])   (backward data)
// EPI 3: out_bf16[v][COP] = silu(acc + bias)             (hidden, inference:
//        the float32 pre-activation, needed only by the backward pass, is
//        not written)
template <int CI, int COP, int EPI>
__global__ __launch_bounds__(kThreads) void conv_kernel(ConvArgs a) {
  constexpr int PIT = CI + 8;  // staged bf16 per voxel (16-byte aligned rows)
  constexpr int K = 27 * CI, NK = (K + 31) / 32, NT = COP / 16, CH = CI / 8;
  __shared__ __align__(16) __bf16 tile[HV * PIT];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const __bf16* in = a.in;

  // Stage the halo tile: every thread's loads are issued before any is
  // used (from addresses clamped into the grid), then voxels outside the
  // grid are zeroed as the values go to LDS, so the loads are in flight
  // together instead of one load-then-store round trip per chunk.
  constexpr int NST = HV * CH, NIT = (NST + kThreads - 1) / kThreads;
  bf16x8 sv[NIT];
  bool inb[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = min(tid + it * kThreads, NST - 1);
    const int v = idx / CH, c = idx % CH;
    const int hx = v % HXX, hy = (v / HXX) % HYY, hz = v / (HXX * HYY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    inb[it] = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    const int cx = min(max(gx, 0), nx - 1), cy = min(max(gy, 0), ny - 1),
              cz = min(max(gz, 0), nz - 1);
    sv[it] = *reinterpret_cast<const bf16x8*>(in + ((size_t(cz) * ny + cy) * nx + cx) * CI + c * 8);
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int idx = tid + it * kThreads;
    if (idx < NST) {
      const int v = idx / CH, c = idx % CH;
      *reinterpret_cast<bf16x8*>(tile + v * PIT + c * 8) = inb[it] ? sv[it] : zero8();
    }
  }
  __syncthreads();

  const int m = lane & 15, g = lane >> 4;
  f32x4 acc[TY][NT];
#pragma unroll
  for (int i = 0; i < TY; ++i)
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // Fully unrolled: each step's tap and channel offsets are then constants
  // (with 32 input channels a step is exactly one tap), so the LDS and
  // weight addresses take immediate offsets instead of a division chain per
  // step, and the zero fill of lanes past the last tap is folded away where
  // K is a multiple of 32.
#pragma unroll
  for (int ks = 0; ks < NK; ++ks) {
    const int k0 = ks * 32 + g * 8;  // this lane's 8 consecutive k
    const int t = k0 / CI, c0 = k0 % CI;
    const bool valid = t < 27;
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    bf16x8 b[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
      b[nt] = valid ? *reinterpret_cast<const bf16x8*>(a.wt + size_t(nt * 16 + m) * K + k0) : zero8();
#pragma unroll
    for (int mt = 0; mt < TY; ++mt) {
      bf16x8 av = zero8();
      if (valid) {
        const int hv = ((wave + tz) * HYY + (mt + ty)) * HXX + (m + tx);
        av = *reinterpret_cast<const bf16x8*>(tile + hv * PIT + c0);
      }
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nt], acc[mt][nt], 0, 0, 0);
    }
  }

  const int gz = z0 + wave;
  if constexpr (EPI == 1 || EPI == 3) {
    // The bf16 activations leave through LDS (the staged tile is no longer
    // read): each wave writes its TY x TX x COP outputs channels-last with a
    // row pitch of COP + 4 values (the four 16-lane groups of a 2-byte write
    // fall on disjoint banks), then each lane stores 8 channels of one voxel
    // with one 16-byte write, 4 stores per wave instead of 32 per lane.
    static_assert(COP == 32, "four lanes per voxel");
    constexpr int OP = COP + 4;
    static_assert(4 * TY * TX * OP <= HV * PIT, "fits in the staged tile");
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
    __syncthreads();  // every wave is done with the staged tile
    __bf16* ob = tile + wave * (TY * TX * OP);
#pragma unroll
    for (int mt = 0; mt < TY; ++mt) {
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + m;
        const float bco = a.bias[co];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = 4 * g + r;
          const float z = acc[mt][nt][r] + bco;
          if (EPI == 1) {
            const int gx = x0 + x, gy = y0 + mt;
            if (gx < nx && gy < ny && gz < nz)
              a.out_f32[((size_t(gz) * ny + gy) * nx + gx) * COP + co] = z;
          }
          ob[(mt * TX + x) * OP + co] = __bf16(silu_f(z));
        }
      }
    }
    __syncthreads();
    const int x = lane >> 2, q = lane & 3;  // voxel of the row, 8-channel chunk
    const int gx = x0 + x;
#pragma unroll
    for (int mt = 0; mt < TY; ++mt) {
      const int gy = y0 + mt;
      const __bf16* src = ob + (mt * TX + x) * OP + q * 8;  // 8-byte aligned
      const bf16x4 lo = *reinterpret_cast<const bf16x4*>(src);
      const bf16x4 hi = *reinterpret_cast<const bf16x4*>(src + 4);
      bf16x8 v8;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v8[j] = lo[j];
        v8[j + 4] = hi[j];
      }
      if (gx < nx && gy < ny && gz < nz)
        *reinterpret_cast<bf16x8*>(a.out_bf16 + ((size_t(gz) * ny + gy) * nx + gx) * COP + q * 8) = v8;
    }
  } else if constexpr (EPI == 0) {
    // The network's outputs (co_real <= COP float32 channels per voxel) also
    // leave through LDS: a row of TX voxels is co_real * TX consecutive
    // floats in global memory, written by consecutive lanes.
    static_assert(NT == 1, "one 16-channel tile");
    static_assert(4 * TY * TX * COP * sizeof(float) <= HV * PIT * sizeof(__bf16),
                  "fits in the staged tile");
    const int cr = a.co_real;
    __syncthreads();  // every wave is done with the staged tile
    float* ob = reinterpret_cast<float*>(tile) + wave * (TY * TX * COP);
    if (m < cr) {
      const float bco = a.bias[m];
#pragma unroll
      for (int mt = 0; mt < TY; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) ob[(mt * TX + 4 * g + r) * cr + m] = acc[mt][0][r] + bco;
    }
    __syncthreads();
    const int nvalid = max(0, min(TX, nx - x0)) * cr;  // floats of the row inside the grid
#pragma unroll
    for (int mt = 0; mt < TY; ++mt) {
      const int gy = y0 + mt;
      if (gy >= ny || gz >= nz) continue;
      float* dst = a.out_f32 + ((size_t(gz) * ny + gy) * nx + x0) * cr;
      for (int e = lane; e < nvalid; e += 64) dst[e] = ob[mt * TX * cr + e];
    }
  } else {
#pragma unroll
    for (int mt = 0; mt < TY; ++mt) {
      const int gy = y0 + mt;
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int co = nt * 16 + m;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gx = x0 + 4 * g + r;
          if (gx >= nx || gy >= ny || gz >= nz) continue;
          const size_t v = (size_t(gz) * ny + gy) * nx + gx;
          a.out_bf16[v * COP + co] = __bf16(acc[mt][nt][r] * silu_grad_f(a.zprev[v * COP + co]));
        }
      }
    }
  }
}

// ---------------------------------------------------------------- dW
// Partial weight and bias gradients of one voxel tile:
//   dW[t][ci][co] = sum_v in[v + t - 1][ci] dz[v][co],  db[co] = sum_v dz[v][co]
// as GEMMs with M = ci, N = co, K = the tile's 256 voxels, one tap at a time
// (waves take taps round robin).  Operands are staged channel-major in LDS.
template <int CI, int COP>
__global__ __launch_bounds__(kThreads) void wgrad_kernel(WgradArgs a) {
  constexpr int NV = TX * TY * TZ;  // 256
  constexpr int DP = NV + 8;        // dz row pitch (16-byte aligned)
  constexpr int MT = CI / 16, NT = COP / 16;
  __shared__ __align__(16) __bf16 X[CI * HV];
  __shared__ __align__(16) __bf16 Dz[COP * DP];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
  const size_t blk = (size_t(blockIdx.z) * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;

  // Both operands staged channel-major; as in the forward kernel, every
  // load of a thread is issued (from addresses clamped into the grid) before
  // the values are zeroed outside the grid and written to LDS.
  constexpr int NX8 = HV * (CI / 8), NXI = (NX8 + kThreads - 1) / kThreads;
  constexpr int ND8 = NV * (COP / 8), NDI = (ND8 + kThreads - 1) / kThreads;
  bf16x8 xv[NXI], dv[NDI];
  bool xin[NXI], din[NDI];
#pragma unroll
  for (int it = 0; it < NXI; ++it) {
    const int idx = min(tid + it * kThreads, NX8 - 1);
    const int v = idx / (CI / 8), c = idx % (CI / 8);
    const int hx = v % HXX, hy = (v / HXX) % HYY, hz = v / (HXX * HYY);
    const int gx = x0 - 1 + hx, gy = y0 - 1 + hy, gz = z0 - 1 + hz;
    xin[it] = gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
    const int cx = min(max(gx, 0), nx - 1), cy = min(max(gy, 0), ny - 1),
              cz = min(max(gz, 0), nz - 1);
    xv[it] = *reinterpret_cast<const bf16x8*>(a.in + ((size_t(cz) * ny + cy) * nx + cx) * CI + c * 8);
  }
#pragma unroll
  for (int it = 0; it < NDI; ++it) {
    const int idx = min(tid + it * kThreads, ND8 - 1);
    const int v = idx / (COP / 8), c = idx % (COP / 8);
    const int lx = v % TX, ly = (v / TX) % TY, lz = v / (TX * TY);
    const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    din[it] = gx < nx && gy < ny && gz < nz;
    const int cx = min(gx, nx - 1), cy = min(gy, ny - 1), cz = min(gz, nz - 1);
    dv[it] = *reinterpret_cast<const bf16x8*>(a.dz + ((size_t(cz) * ny + cy) * nx + cx) * COP + c * 8);
  }
#pragma unroll
  for (int it = 0; it < NXI; ++it) {
    const int idx = tid + it * kThreads;
    if (idx < NX8) {
      const int v = idx / (CI / 8), c = idx % (CI / 8);
      const bf16x8 val = xin[it] ? xv[it] : zero8();
#pragma unroll
      for (int j = 0; j < 8; ++j) X[(c * 8 + j) * HV + v] = val[j];
    }
  }
#pragma unroll
  for (int it = 0; it < NDI; ++it) {
    const int idx = tid + it * kThreads;
    if (idx < ND8) {
      const int v = idx / (COP / 8), c = idx % (COP / 8);
      const bf16x8 val = din[it] ? dv[it] : zero8();
#pragma unroll
      for (int j = 0; j < 8; ++j) Dz[(c * 8 + j) * DP + v] = val[j];
    }
  }
  __syncthreads();

  const int m = lane & 15, g = lane >> 4;
  float* part = a.part + blk * size_t(27 * CI * COP + COP);
  for (int t = wave; t < 27; t += 4) {
    const int tz = t / 9, ty = (t / 3) % 3, tx = t % 3;
    f32x4 acc[MT][NT];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
      for (int j = 0; j < NT; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < NV / 32; ++ks) {
      const int k0 = ks * 32 + g * 8;  // 8 consecutive voxels along x
      const int lx = k0 % TX, ly = (k0 / TX) % TY, lz = k0 / (TX * TY);
      const int hbase = ((lz + tz) * HYY + (ly + ty)) * HXX + lx + tx;
      bf16x8 b[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
        b[nt] = *reinterpret_cast<const bf16x8*>(Dz + (nt * 16 + m) * DP + k0);
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        bf16x8 av;
        const __bf16* xr = X + (mt * 16 + m) * HV + hbase;
#pragma unroll
        for (int j = 0; j < 8; ++j) av[j] = xr[j];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[nt], acc[mt][nt], 0, 0, 0);
      }
    }
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ci = mt * 16 + 4 * g + r, co = nt * 16 + m;
          part[(size_t(t) * CI + ci) * COP + co] = acc[mt][nt][r];
        }
  }
  if (tid < COP) {
    float s = 0.f;
    for (int v = 0; v < NV; ++v) s += float(Dz[tid * DP + v]);
    part[size_t(27) * CI * COP + tid] = s;
  }
}

// Sum the per-block partials into the gradient in the master layout
// W[t][ci][co] (ci < cin, co < cout), then b[co].  A block owns 64 outputs;
// its four waves each sum every fourth partial (b = wave, wave + 4, ...) in
// increasing b, and the four sums are added in wave order: a fixed order, so
// the result is bitwise repeatable, with 4x the loads in flight of one
// serial sum per output.
constexpr int kReduceOut = 64, kReduceSplit = 4;
__global__ void __launch_bounds__(kReduceOut * kReduceSplit)
wgrad_reduce_kernel(const float* __restrict__ part, int nblk, int CI, int COP, int cin, int cout,
                    float* __restrict__ grad) {
  __shared__ float acc[kReduceSplit][kReduceOut];
  const int nW = 27 * cin * cout;
  const size_t stride = size_t(27) * CI * COP + COP;
  const int lane = threadIdx.x % kReduceOut, g = threadIdx.x / kReduceOut;
  const int j = blockIdx.x * kReduceOut + lane;
  float s = 0.f;
  if (j < nW + cout) {
    size_t src;
    if (j < nW) {
      const int t = j / (cin * cout), rem = j % (cin * cout), ci = rem / cout, co = rem % cout;
      src = (size_t(t) * CI + ci) * COP + co;
    } else {
      src = size_t(27) * CI * COP + (j - nW);
    }
    const float* q = part + src;
    int b = g;
    for (; b + 3 * kReduceSplit < nblk; b += 4 * kReduceSplit) {
      const float v0 = q[size_t(b) * stride], v1 = q[size_t(b + kReduceSplit) * stride],
                  v2 = q[size_t(b + 2 * kReduceSplit) * stride],
                  v3 = q[size_t(b + 3 * kReduceSplit) * stride];
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; b < nblk; b += kReduceSplit) s += q[size_t(b) * stride];
  }
  acc[g][lane] = s;
  __syncthreads();
  if (g == 0 && j < nW + cout) {
    float r = acc[0][lane];
#pragma unroll
    for (int w = 1; w < kReduceSplit; ++w) r += acc[w][lane];
    grad[j] = r;
  }
}

// ---------------------------------------------------------------- params
// Master (float32) layout per layer: W[t][ci][co] (27 cin cout) then b[cout].
// Forward B operand: wf[co][t*CIP + ci] (bf16, zero padded);
// backward-data B operand: wb[ci][t'*COP + co] = W[26 - t'][ci][co].
__global__ void layout_kernel(const float* __restrict__ Wm, const float* __restrict__ bm, int cin,
                              int cout, int CIP, int COP, __bf16* __restrict__ wf,
                              __bf16* __restrict__ wb, float* __restrict__ bias_pad) {
  const int nf = COP * 27 * CIP, nb = wb ? CIP * 27 * COP : 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nf + nb + COP;
       j += gridDim.x * blockDim.x) {
    if (j < nf) {
      const int co = j / (27 * CIP), k = j % (27 * CIP), t = k / CIP, ci = k % CIP;
      const float w = (ci < cin && co < cout) ? Wm[(size_t(t) * cin + ci) * cout + co] : 0.f;
      wf[j] = __bf16(w);
    } else if (j < nf + nb) {
      const int jj = j - nf;
      const int ci = jj / (27 * COP), k = jj % (27 * COP), tp = k / COP, co = k % COP;
      const int t = 26 - tp;
      const float w = (ci < cin && co < cout) ? Wm[(size_t(t) * cin + ci) * cout + co] : 0.f;
      wb[jj] = __bf16(w);
    } else {
      const int co = j - nf - nb;
      bias_pad[co] = co < cout ? bm[co] : 0.f;
    }
  }
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// float32 [V][creal] -> bf16 [V][CP] (zero padded channels)
__global__ void pack_kernel(const float* __restrict__ src, int creal, int CP, size_t V,
                            __bf16* __restrict__ dst) {
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < V * CP;
       i += size_t(gridDim.x) * blockDim.x) {
    const size_t v = i / CP;
    const int c = int(i % CP);
    dst[i] = __bf16(c < creal ? src[v * creal + c] : 0.f);
  }
}

// dy = 2 (y - t) / count; per-block partial sums of (y - t)^2
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, size_t count,
                           float* __restrict__ dy, float* __restrict__ partial) {
  __shared__ float red[256];
  float s = 0.f;
  const float k = 2.0f / float(count);
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x) {
    const float r = y[i] - t[i];
    dy[i] = k * r;
    s += r * r;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace

hipError_t launch_conv(int ci, int cop, int epi, const ConvArgs& a, hipStream_t s) {
  dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + TZ - 1) / TZ);
  dim3 block(kThreads);
  if (ci == 16 && cop == 32 && epi == 1) hipLaunchKernelGGL((conv_kernel<16, 32, 1>), grid, block, 0, s, a);
  else if (ci == 32 && cop == 32 && epi == 1) hipLaunchKernelGGL((conv_kernel<32, 32, 1>), grid, block, 0, s, a);
  else if (ci == 32 && cop == 16 && epi == 0) hipLaunchKernelGGL((conv_kernel<32, 16, 0>), grid, block, 0, s, a);
  else if (ci == 16 && cop == 32 && epi == 2) hipLaunchKernelGGL((conv_kernel<16, 32, 2>), grid, block, 0, s, a);
  else if (ci == 32 && cop == 32 && epi == 2) hipLaunchKernelGGL((conv_kernel<32, 32, 2>), grid, block, 0, s, a);
  else if (ci == 16 && cop == 32 && epi == 3) hipLaunchKernelGGL((conv_kernel<16, 32, 3>), grid, block, 0, s, a);
  else if (ci == 32 && cop == 32 && epi == 3) hipLaunchKernelGGL((conv_kernel<32, 32, 3>), grid, block, 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

int wgrad_blocks(int nx, int ny, int nz) {
  return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY) * ((nz + TZ - 1) / TZ);
}

hipError_t launch_wgrad(int ci, int cop, const WgradArgs& a, int cin, int cout, float* grad,
                        hipStream_t s) {
  dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + TZ - 1) / TZ);
  dim3 block(kThreads);
  if (ci == 32 && cop == 16) hipLaunchKernelGGL((wgrad_kernel<32, 16>), grid, block, 0, s, a);
  else if (ci == 32 && cop == 32) hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, block, 0, s, a);
  else if (ci == 16 && cop == 32) hipLaunchKernelGGL((wgrad_kernel<16, 32>), grid, block, 0, s, a);
  else return hipErrorInvalidValue;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nblk = int(grid.x * grid.y * grid.z);
  const int n = 27 * cin * cout + cout;
  hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((n + kReduceOut - 1) / kReduceOut),
                     dim3(kReduceOut * kReduceSplit), 0, s, a.part, nblk, ci, cop, cin, cout, grad);
  return hipGetLastError();
}

hipError_t launch_layout(const float* Wm, const float* bm, int cin, int cout, int CIP, int COP,
                         __bf16* wf, __bf16* wb, float* bias_pad, hipStream_t s) {
  const int n = COP * 27 * CIP + (wb ? CIP * 27 * COP : 0) + COP;
  hipLaunchKernelGGL(layout_kernel, dim3((n + 255) / 256), dim3(256), 0, s, Wm, bm, cin, cout, CIP,
                     COP, wf, wb, bias_pad);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, int t, hipStream_t s) {
  const float c1 = 1.f - powf(b1, float(t)), c2 = 1.f - powf(b2, float(t));
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, g, m, v, n, lr, b1,
                     b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack(const float* src, int creal, int CP, size_t V, __bf16* dst, hipStream_t s) {
  const int blocks = int(std::min<size_t>((V * CP + 255) / 256, 8192));
  hipLaunchKernelGGL(pack_kernel, dim3(blocks), dim3(256), 0, s, src, creal, CP, V, dst);
  return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, size_t count, float* dy, float* partial,
                      int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, s, y, t, count, dy, partial);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace adimx

// ====================================================================== glue
namespace adimx {
namespace nn {
namespace {

template <typename T>
__global__ void sumsq_kernel(const T* __restrict__ x, size_t count, float* __restrict__ partial) {
  __shared__ float red[256];
  double s = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x) {
    const double v = double(x[i]);
    s += v * v;
  }
  red[threadIdx.x] = float(s);
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Root mean square of count values from per-block sums of squares.
__device__ float rms_of_partials(const float* __restrict__ partial, int nblk, size_t count) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return float(sqrt(red[0] / double(count)));
}

// scale = RMS of the state (a tiny floor keeps zero states finite)
__global__ void scale_kernel(const float* __restrict__ partial, int nblk, size_t count,
                             float* __restrict__ scale) {
  const float r = rms_of_partials(partial, nblk, count);
  if (threadIdx.x == 0) scale[0] = r + 1e-30f;
}

// x[v][0..5]   = C_c[v] / scale,
// x[v][6..11]  = (C_c[v] - S_c[v]) / scale   (C after the coarse step, S before),
// x[v][12..14] = material features,
// x[v][15]     = source impulse of the step / scale, spread over the
//                coefficients by the tensor-product basis values at the dipole
// (O = float for the API; O = bf16 writes the network's packed input
// directly, the same values as packing the float features)
template <typename T, typename O>
__global__ void features_kernel(const T* __restrict__ state, const T* __restrict__ prev,
                                const float* __restrict__ mat, int n,
                                const float* __restrict__ scale, SourceArgs src,
                                const double* __restrict__ tnow, double dt,
                                O* __restrict__ x) {
  const size_t D = size_t(n) * n * n;
  const float inv = 1.0f / scale[0];
  double jimp = 0.0;  // dt/2 (g(t - 3 dt/4) + g(t - dt/4)) amp, t = time after the step
  if (src.comp >= 0) {
    const double t = *tnow;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double s = t - (h ? 0.25 : 0.75) * dt - src.t0;
      jimp += sin(2.0 * 3.14159265358979323846 * src.f0 * s) *
              exp(-(s / src.width) * (s / src.width));
    }
    jimp *= 0.5 * dt * src.amp;
  }
  for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < D;
       v += size_t(gridDim.x) * blockDim.x) {
    O* o = x + v * kFeatures;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double cur = double(state[c * D + v]);
      o[c] = O(float(cur) * inv);
      o[6 + c] = O(float(cur - double(prev[c * D + v])) * inv);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) o[12 + c] = O(mat[v * 3 + c]);
    float sf = 0.f;
    if (src.comp >= 0) {
      const int i = int(v % n) - src.first[0], j = int((v / n) % n) - src.first[1],
                k = int(v / (size_t(n) * n)) - src.first[2];
      const int P = kMaxP;
      if (i >= 0 && i <= P && j >= 0 && j <= P && k >= 0 && k <= P)
        sf = float(jimp * src.bx[i] * src.by[j] * src.bz[k]) * inv;
    }
    o[15] = O(sf);
  }
}

template <typename T>
__global__ void target_kernel(const T* __restrict__ fine, const T* __restrict__ coarse, size_t D,
                              const float* __restrict__ scale, float* __restrict__ t) {
  const float inv = 1.0f / scale[0];
  for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < D;
       v += size_t(gridDim.x) * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c)
      t[v * 6 + c] = float(double(fine[c * D + v]) - double(coarse[c * D + v])) * inv;
  }
}

// state_c += scale * y_c, except on the constrained boundary coefficients
// (E_c on the faces normal to the other axes, H_c on the faces normal to c);
// skipped entirely when the gate flag is set
template <typename T>
__global__ void apply_kernel(T* __restrict__ state, int n, const float* __restrict__ y,
                             const float* __restrict__ scale, const int* __restrict__ flag) {
  if (flag && flag[0]) return;
  const size_t D = size_t(n) * n * n;
  const float s = scale[0];
  for (size_t v = size_t(blockIdx.x) * blockDim.x + threadIdx.x; v < D;
       v += size_t(gridDim.x) * blockDim.x) {
    const int i = int(v % n), j = int((v / n) % n), k = int(v / (size_t(n) * n));
    const bool b[3] = {i == 0 || i == n - 1, j == 0 || j == n - 1, k == 0 || k == n - 1};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const int comp = c % 3;
      const bool constrained = c < 3 ? (b[(comp + 1) % 3] || b[(comp + 2) % 3]) : b[comp];
      if (!constrained) state[c * D + v] += T(s * y[v * 6 + c]);
    }
  }
}

// Per-block sums of squares of the change a - b (the coarse step's change
// C - S when a is the state after the step and b the marked state before).
template <typename T>
__global__ void diffsq_kernel(const T* __restrict__ a, const T* __restrict__ b, size_t count,
                              float* __restrict__ partial) {
  __shared__ float red[256];
  double s = 0.0;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += size_t(gridDim.x) * blockDim.x) {
    const double v = double(a[i]) - double(b[i]);
    s += v * v;
  }
  red[threadIdx.x] = float(s);
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Gate of the correction, judged against the coarse step it corrects: the
// correction s * y is rejected (flag set, counter raised) when its RMS
// exceeds limit times the RMS of the step's change C - S.  A step that
// changed nothing (a zero state without a source) therefore takes no
// correction at all.
__global__ void gate_kernel(const float* __restrict__ partial_y, const float* __restrict__ partial_d,
                            int nblk, size_t count, const float* __restrict__ scale, float limit,
                            int* __restrict__ flag, int* __restrict__ rejected) {
  const float ry = rms_of_partials(partial_y, nblk, count);
  __syncthreads();
  const float rd = rms_of_partials(partial_d, nblk, count);
  if (threadIdx.x == 0) {
    const float corr = scale[0] * ry;
    const int bad = !(corr <= limit * rd);  // NaN counts as out of range
    flag[0] = bad;
    if (bad) rejected[0] += 1;
  }
}

int blocks_for(size_t n) { return int(std::min<size_t>((n + 255) / 256, 4096)); }

}  // namespace

template <typename T>
hipError_t launch_state_scale(const T* state, size_t count, float* partial, int nblk,
                              float* scale, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel<T>, dim3(nblk), dim3(256), 0, s, state, count, partial);
  hipLaunchKernelGGL(scale_kernel, dim3(1), dim3(256), 0, s, partial, nblk, count, scale);
  return hipGetLastError();
}

template <typename T, typename O>
hipError_t launch_features(const T* state, const T* prev, const float* mat, int n,
                           const float* scale, const SourceArgs& src, const double* tnow,
                           double dt, O* x, hipStream_t s) {
  const size_t D = size_t(n) * n * n;
  hipLaunchKernelGGL((features_kernel<T, O>), dim3(blocks_for(D)), dim3(256), 0, s, state, prev,
                     mat, n, scale, src, tnow, dt, x);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_target(const T* fine, const T* coarse, size_t D, const float* scale, float* t,
                         hipStream_t s) {
  hipLaunchKernelGGL(target_kernel<T>, dim3(blocks_for(D)), dim3(256), 0, s, fine, coarse, D,
                     scale, t);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_apply(T* state, int n, const float* y, const float* scale, const int* flag,
                        hipStream_t s) {
  const size_t D = size_t(n) * n * n;
  hipLaunchKernelGGL(apply_kernel<T>, dim3(blocks_for(D)), dim3(256), 0, s, state, n, y, scale,
                     flag);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gate(const float* y, const T* state, const T* prev, size_t count, float* partial,
                       int nblk, const float* scale, float limit, int* flag, int* rejected,
                       hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel<float>, dim3(nblk), dim3(256), 0, s, y, count, partial);
  hipLaunchKernelGGL(diffsq_kernel<T>, dim3(nblk), dim3(256), 0, s, state, prev, count,
                     partial + nblk);
  hipLaunchKernelGGL(gate_kernel, dim3(1), dim3(256), 0, s, partial, partial + nblk, nblk, count,
                     scale, limit, flag, rejected);
  return hipGetLastError();
}

#define INST(T)                                                                                  \
  template hipError_t launch_state_scale<T>(const T*, size_t, float*, int, float*, hipStream_t);  \
  template hipError_t launch_features<T, float>(const T*, const T*, const float*, int,            \
                                                const float*, const SourceArgs&, const double*,   \
                                                double, float*, hipStream_t);                     \
  template hipError_t launch_features<T, __bf16>(const T*, const T*, const float*, int,           \
                                                 const float*, const SourceArgs&, const double*,  \
                                                 double, __bf16*, hipStream_t);                   \
  template hipError_t launch_target<T>(const T*, const T*, size_t, const float*, float*,          \
                                       hipStream_t);                                              \
  template hipError_t launch_apply<T>(T*, int, const float*, const float*, const int*,            \
                                      hipStream_t);                                               \
  template hipError_t launch_gate<T>(const float*, const T*, const T*, size_t, float*, int,        \
                                     const float*, float, int*, int*, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace nn
}  // namespace adimx
