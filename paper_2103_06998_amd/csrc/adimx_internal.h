// Internal declarations shared by the host driver and the HIP kernels of
// libadimx.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace adimx {

constexpr int kMaxP = 4;    // largest supported B-spline degree
// Segments per line of the partitioned line solve: 4, or 8 for lines of
// more than kSpikeS8MinN rows (segments of at most 36 rows either way in the
// benchmarked sizes; shorter segments need fewer registers per wave).
constexpr int kSpikeS = 4, kSpikeS8 = 8, kSpikeS8MinN = 193;
constexpr int spike_segments(int n) { return n >= kSpikeS8MinN ? kSpikeS8 : kSpikeS; }
// Lines of n rows use the partitioned solve when kSpikeMinN <= n <= kSpikeMaxN.
constexpr int kSpikeMinN = 48, kSpikeMaxN = 288;

// ---------------------------------------------------------------- host (FP64)
struct Gram1D {
  int N = 0, p = 0, n = 0;
  std::vector<double> M, S, A, B;  // bands, n x (2p+1): band[r*(2p+1)+d] = X[r][r+d-p]
};

std::vector<double> open_knots(int N, int p);
int find_span(const std::vector<double>& t, int p, int n, double x);
void basis_on_span(const std::vector<double>& t, int p, int span, double x, double* val,
                   double* der);
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w);
Gram1D build_gram(int N, int p);
void apply_dirichlet(std::vector<double>& band, int n, int p);
double band_lu(const std::vector<double>& band, int n, int p, std::vector<double>& L,
               std::vector<double>& Uoff, std::vector<double>& Uinv);
std::vector<double> greville(int N, int p);
// W[i*V + v]: share of the integral of B_i over [0, 1] that lies in voxel v.
std::vector<double> voxel_weights(int N, int p, int V);

// Partitioned (SPIKE) solve data of one shared banded matrix split into S
// row segments [spike_boundary(n,S,i), spike_boundary(n,S,i+1)):
// block-diagonal LU (L, DU = D*U, D as band_lu, couplings across segment
// boundaries removed), spikes V, W ([r*p + k]) and the inverse R (q x q,
// q = 2p(S-1), row-major) of the reduced system on the unknowns
// z = [U_0, T_1, U_1, T_2, ..., U_{S-2}, T_{S-1}] (U_i: bottom p rows of
// segment i, T_i: top p rows).  Returns false if a segment is shorter than
// 2p, a pivot is tiny, or a self-check against the direct solve fails.
struct SpikeData {
  int S = 0, q = 0;
  std::vector<double> L, DU, D, V, W, R;
};
int spike_boundary(int n, int S, int i);
bool spike_prepare(const std::vector<double>& band, int n, int p, int S, SpikeData& out);
void basis_at(int N, int p, double x, int* first, double* vals);

// ---------------------------------------------------------------- kernels
// Stage kinds of the right-hand-side kernel.
enum RhsStage : int {
  kStageE1 = 0,   // E right-hand sides, substep 1 (eq. discrete1)
  kStageE2 = 1,   // E right-hand sides, substep 2 (eq. discrete3)
  kStageH1 = 2,   // H right-hand sides, substep 1 (eq. discrete2)
  kStageH2 = 3,   // H right-hand sides, substep 2 (eq. discrete4)
  kStageEd1 = 8,  // E increments, substep 1: b - P E (b of eq. discrete1, P the
                  // row-scaled system matrix of eq. dupa1ab)
  kStageEd2 = 9,  // the same for substep 2 (eq. discrete3)
  kStageHd1 = 10, // H increments, substep 1: b - M H (eq. discrete2)
  kStageHd2 = 11, // the same for substep 2 (eq. discrete4)
};

struct SourceArgs {
  int comp = -1;                   // field component carrying the dipole, -1: none
  int first[3] = {0, 0, 0};        // first nonzero basis index per axis
  double bx[kMaxP + 1] = {0}, by[kMaxP + 1] = {0}, bz[kMaxP + 1] = {0};
  double amp = 0, f0 = 0, t0 = 0, width = 1;
};

template <typename T>
struct RhsArgs {
  const void* f[9];       // input fields (E stages: E1..E3,H1..H3; H stages: H1..H3,
                          // E_old1..3, E_new1..3), in the kernel's input type
  void* out[3];           // outputs, in the kernel's output type
  const void* coef[3];    // per-row coefficients, in the kernel's coefficient type:
                          // E: gamma, beta, alpha (increments: gamma - 1, beta,
                          // alpha); H: delta
  const T* bandx;         // x axis: [op][r][2p+1], op 0 = M, 1 = A, 2 = B, 3 = S
  const T* bandy;         // y axis, same layout
  const T* zw;            // z axis: [op][k][2p+1]: weight of input plane k on output
                          // plane k - p + q (band entry Z[k-p+q][k], zero outside)
  int nx, ny, nz;         // coefficients per axis
  int yin0, yin1;         // rows yin0..yin1 of every y operator equal row yrep
  int yrep;               // (translation-invariant interior rows; empty if yin0 > yin1)
  int zchunk;             // output planes per block
  SourceArgs src;
  const double* tnow;     // device time at the start of the step
  double frac_dt;         // (1/4 or 3/4) * dt
};

struct SweepDesc {
  int axis;               // 0 = x, 1 = y, 2 = z
  void* in;               // right-hand sides (T)
  void* out;              // solution (T); may equal in
  const void* acc;        // if non-null, out = solution + acc (element-wise)
  const void* L;          // factors; shared: [r*P + k-1],
                          // modified: [((l/64 * n + r) * P + k-1) * 64 + l%64]
  const void* U;          // D * U (pre-scaled upper factor), same layout as L
  const void* D;          // inverse diagonal; shared: [r], modified: [(l/64 * n + r) * 64 + l%64]
  const void* spk;        // shared factors only: partitioned-solve data (L, DU, D, V, W
                          // as [r*P + k] / [r], then R, q x q), or null
  int segs;               // segments per line of spk (spike_segments(n))
  int modified;           // 0 = shared factors, 1 = per-line factors
  const void* aband;      // SweepArgs::apply: band [r][2p+1] of the 1D operator applied
                          // to `in` before the solve (T)
  double scale;           // SweepArgs::apply: out = acc + scale * solution
};

struct SweepArgs {
  SweepDesc d[3];         // blockIdx.y selects the descriptor
  int dim[3];             // coefficients per axis (nx, ny, nz); a descriptor's
                          // lines have dim[axis] rows, and there are
                          // nx ny nz / dim[axis] of them
  int xaxis;              // 0: y/z lines, 1: x lines (transposing kernel),
                          // 2: both, descriptors of x lines first
  int spike;              // 0, or the segments per line (every descriptor's segs) of
                          // the partitioned solve of shared-factor lines
  int apply;              // 1: each line solves M x = A in (A = the descriptor's aband;
                          // partitioned solve only) and stores acc + scale * x
  double* tick_t;         // if non-null, block (0,0) thread 0 does *tick_t += tick_dt
  double tick_dt;
};

struct FactorArgs {
  const double* Mb;       // band of the base matrix of the axis (Dirichlet rows applied)
  const double* Sb;       // band of the stiffness matrix (Dirichlet rows/cols zero)
  const double* alpha;    // per-DOF coefficient (nx ny nz, x fastest)
  double* L64; double* U64; double* D64;   // per-line factors (float64): L, D*U, D
  float* L32; float* U32; float* D32;      // float32 copies (refine mode) or null
  double* minratio;       // per line: min |U_rr| / |A_rr|
  int n, nlines, axis;    // rows per line (dim[axis]), lines, axis
  int nx, ny;             // coefficients along x and y (line strides)
};

// Launchers (kernels.hip).  All enqueue on `stream` and return hipError_t.
template <typename T>
hipError_t launch_rhs(int stage, int p, const RhsArgs<T>& a, hipStream_t stream);
// Increments of the float32 mode (stages Ed1/Ed2/Hd1/Hd2): float32 fields and
// coefficients, float64 arithmetic (bands and z weights in float64), float32
// outputs.
hipError_t launch_rhs_inc(int stage, int p, const RhsArgs<double>& a, hipStream_t stream);
// The same increments in float32 arithmetic and accumulation (float32 bands).
hipError_t launch_rhs_inc32(int stage, int p, const RhsArgs<float>& a, hipStream_t stream);
template <typename T>
hipError_t launch_sweep(int p, int ndesc, const SweepArgs& a, hipStream_t stream);
hipError_t launch_factor(int p, const FactorArgs& a, hipStream_t stream);
template <typename T>
hipError_t launch_convert(const void* src, void* dst, size_t count, int dir, hipStream_t stream);

}  // namespace adimx
