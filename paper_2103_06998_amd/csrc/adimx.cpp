// Host driver of libadimx: context, device workspace, initialisation
// (Gram matrices, coefficients, factorisations) and the captured time step.
//
// One time step (eqs. scheme1a-scheme1d / discrete1-discrete4) is, per
// substep s = 1, 2:
//   E stage: right-hand sides of E1, E2, E3 (one kernel), then for every
//            component its three 1D solves, the material-modified axis first
//            (that order solves the row-scaled system of eq. dupa1ab
//            exactly; the remaining two axes have shared factors);
//   H stage: right-hand sides of H1, H2, H3, then mass solves along x, y, z.
// In ADI_FP32_REFINE mode every stage is solved in increment form: the
// right-hand-side kernel forms b - P x_old from the float32 state (the
// residual of the old state; float32 arithmetic, or float64 for the stages
// selected by adi_set_residual64, by default the E stage of substep 2), the
// float32 sweeps solve P d = b - P x_old, and the last sweep adds x_old, so
// the float32 solve's rounding scales with the increment d instead of with
// the state.
#include "adimx.h"
#include "adimx_internal.h"
#include "closure_internal.h"
#include "mms_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

using namespace adimx;

namespace {

// Axis carrying the stiffness term of E_c (K1 = diag(MSM, MMS, SMM) in
// substep 1, K2 = diag(MMS, SMM, MSM) in substep 2); 0 = x, 1 = y, 2 = z.
constexpr int kModAxis[2][3] = {{1, 2, 0}, {2, 0, 1}};

bool dirichlet(int kindH, int c, int axis) {
  // PEC: E_c vanishes on the faces normal to the other axes, H_c on the faces
  // normal to axis c.
  return kindH ? (axis == c) : (axis != c);
}

struct Region {
  size_t off, bytes;
};

}  // namespace

struct adi_ctx {
  int Ns[3] = {0, 0, 0};   // elements per axis (x, y, z)
  int ns[3] = {0, 0, 0};   // coefficients per axis, N_a + p
  int N = 0, n = 0;        // elements and coefficients along x (all axes of a cube)
  int p = 0, prec = ADI_FP64;
  size_t D = 0;            // nx ny nz
  size_t esz = 8;          // bytes per field element
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipStream_t side = nullptr;        // second branch of a step: x-line sweeps beside y/z
  hipStream_t hside = nullptr;       // third branch: the H stage's first round beside the E stage
  std::vector<hipEvent_t> fork_ev;   // fork / join events of the branches
  size_t fork_idx = 0;
  std::string err;

  std::vector<double> eps, mu, sig;
  std::vector<double> tau;  // local time step per DOF (empty: dt everywhere)
  bool have_material = false;
  SourceArgs src;
  double src_xs[3] = {0.5, 0.5, 0.5};

  double dt = 0.0, t = 0.0;
  double pivot_floor = 1e-14;  // smallest accepted |U_rr| / |A_rr| of the LU
  // float32 mode: stages whose increment is formed in float64 arithmetic
  // (bit res64_bit(stage, sub)); the others use float32 arithmetic
  int res64 = ADI_RES64_DEFAULT;
  // H stage as two apply-and-solve line rounds (delta = dt / (2 mu) the same
  // in every row; set by adi_factor)
  bool fast_h = false;
  double hdelta = 0.0;
  bool factored = false;

  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;

  // device pointers (into ws)
  void* B[4] = {};          // 4 field buffers of 3 D elements; B0|B1 = state (E|H)
  void* coefT[4] = {};      // alpha, beta, gamma, delta in the field type
  double* coef64[4] = {};   // float64 copies (refine mode), else alias of coefT
  void* gm1T = nullptr;     // gamma - 1 (refine mode: group coefficient of the E increments)
  void* bandT[3] = {};      // per axis: [M,A,B,S][n_a][2p+1] in the field type
  double* band64[3] = {};   // same in float64
  void* zwT = nullptr;      // z weights [M,A,B,S][k][2p+1] in the field type
  double* zw64 = nullptr;   // same in float64
  // rows yin[0]..yin[1] of the y operators' bands equal row yin[2]
  // (translation-invariant interior rows of uniform knots)
  int yin[3] = {1, 0, 0};
  double* fb64[3] = {};     // per axis, factor bands: Mdir, Sdir (n_a (2p+1) each)
  // shared factors per axis: [axis][0] free, [axis][1] Dirichlet
  void* shL[3][2] = {}, *shU[3][2] = {}, *shD[3][2] = {};
  void* spk[3][2] = {};     // partitioned-solve data of the shared factors (same variants)
  bool spike_ok[3] = {};    // spk[axis] holds valid data for the current factorisation
  void* mL[6] = {}, *mU[6] = {}, *mD[6] = {};     // per-line factors, system (s-1)*3 + c
  double* minratio = nullptr;
  double* d_t = nullptr;

  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  // per-launch timing (eager profiling pass): events recorded around every
  // kernel of a step, durations summed over the profiled steps
  bool profiling = false;
  std::vector<hipEvent_t> events;      // 2 per launch
  std::vector<int> launch_kind, launch_ndesc, launch_nmod, launch_nacc;
  std::vector<double> launch_ms_sum;
  int profiled_steps = 0;
  size_t launch_idx = 0;

  // learned closure (allocated on first use)
  void* cl_prev = nullptr;      // state before the last coarse step (6 D, field type)
  float* cl_mat = nullptr;      // material features [D][3]
  float* cl_red = nullptr;      // reduction partials [kClosureBlocks], scale [1]
  int* cl_flag = nullptr;       // [0] gate flag, [1] rejected-correction counter
  bool cl_mat_valid = false;    // cl_mat matches the last factorisation
  bool cl_marked = false;       // cl_prev holds a state

  // manufactured-solution tools (allocated on first use)
  int mms_q = 0;
  double* mms_tab = nullptr;    // x, w, bv, bd of the q-point rule (one axis)
  double* mms_vals = nullptr;   // solution at the Gauss points, 6 Q^3
  double* mms_part = nullptr;   // error partial sums, 4 per block

  bool refine() const { return prec == ADI_FP32_REFINE; }
};

namespace {

// Bit of adi_set_residual64's mask for stage 0 = E, 1 = H of substep sub.
constexpr int res64_bit(int stage, int sub) { return 1 << (2 * (sub - 1) + stage); }

int fail(adi_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, expr)                                                           \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return fail(ctx, ADI_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Walk the workspace layout; if `base` is non-null assign the pointers.
size_t layout(adi_ctx* c, unsigned char* base) {
  size_t cur = 0;
  auto take = [&](size_t bytes) -> unsigned char* {
    cur = (cur + 255) & ~size_t(255);
    unsigned char* ptr = base ? base + cur : nullptr;
    cur += bytes;
    return ptr;
  };
  const size_t D = c->D, es = c->esz;
  const int W = 2 * c->p + 1, P = c->p;
  // B0..B3 contiguous so that B0|B1 (the state) is one 6 D array
  unsigned char* b = take(4 * 3 * D * es);
  for (int i = 0; i < 4; ++i) c->B[i] = b ? b + size_t(i) * 3 * D * es : nullptr;
  for (int i = 0; i < 4; ++i) c->coefT[i] = take(D * es);
  for (int i = 0; i < 4; ++i)
    c->coef64[i] = c->refine() ? reinterpret_cast<double*>(take(D * 8))
                               : reinterpret_cast<double*>(c->coefT[i]);
  c->gm1T = c->refine() ? take(D * es) : nullptr;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = c->ns[ax];
    c->bandT[ax] = take(size_t(4) * n * W * es);
    c->band64[ax] = reinterpret_cast<double*>(take(size_t(4) * n * W * 8));
    c->fb64[ax] = reinterpret_cast<double*>(take(size_t(2) * n * W * 8));
    const int q = 2 * P * (spike_segments(n) - 1);
    for (int v = 0; v < 2; ++v) {
      c->shL[ax][v] = take(size_t(n) * P * es);
      c->shU[ax][v] = take(size_t(n) * P * es);
      c->shD[ax][v] = take(size_t(n) * es);
      c->spk[ax][v] = take((size_t(n) * (4 * P + 1) + size_t(q) * q) * es);
    }
  }
  c->zwT = take(size_t(4) * c->ns[2] * W * es);
  c->zw64 = reinterpret_cast<double*>(take(size_t(4) * c->ns[2] * W * 8));
  // per-line factors of system s (its modified axis a: D / n_a lines of n_a
  // rows) in blocks of 64 lines (the line count padded to 64)
  size_t maxlines = 0;
  for (int s = 0; s < 6; ++s) {
    const int n = c->ns[kModAxis[s / 3][s % 3]];
    const size_t nlpad = (D / size_t(n) + 63) / 64 * 64;
    maxlines = std::max(maxlines, D / size_t(n));
    c->mL[s] = take(size_t(P) * n * nlpad * es);
    c->mU[s] = take(size_t(P) * n * nlpad * es);
    c->mD[s] = take(size_t(n) * nlpad * es);
  }
  c->minratio = reinterpret_cast<double*>(take(maxlines * 8));
  c->d_t = reinterpret_cast<double*>(take(8));
  return cur + 256;
}

void* comp(void* buf, int c, const adi_ctx* x) {
  return static_cast<unsigned char*>(buf) + size_t(c) * x->D * x->esz;
}

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

int upload(adi_ctx* c, void* dst, const std::vector<double>& src) {
  if (c->esz == 8) {
    HIPCHK(c, hipMemcpy(dst, src.data(), src.size() * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f = cast_vec<float>(src);
    HIPCHK(c, hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  return ADI_OK;
}

// The widest run of rows around the middle row of a 1D operator set
// ([op][r][W], four operators) whose band rows all equal the middle row's to
// within a relative 1e-14 of its largest entry (with uniform knots, the rows
// whose basis functions and neighbours are all interior translates):
// out = {first, last, middle}, or an empty range {1, 0, middle}.
void invariant_rows(const std::vector<double>& ops, int n, int W, int out[3]) {
  const int m = n / 2;
  auto same = [&](int r) {
    for (int op = 0; op < 4; ++op) {
      const double* a = &ops[(size_t(op) * n + r) * W];
      const double* b = &ops[(size_t(op) * n + m) * W];
      double big = 0.0;
      for (int d = 0; d < W; ++d) big = std::max(big, std::fabs(b[d]));
      for (int d = 0; d < W; ++d)
        if (std::fabs(a[d] - b[d]) > 1e-14 * big) return false;
    }
    return true;
  };
  int lo = m, hi = m;
  while (lo > 0 && same(lo - 1)) --lo;
  while (hi < n - 1 && same(hi + 1)) ++hi;
  out[0] = lo;
  out[1] = hi;
  out[2] = m;
}

// Output planes per RHS block: the grid is 3 ceil(nx/32) ceil(ny/8)
// ceil(nz/zchunk) blocks of 256 threads (one per tile and output component),
// about two resident per CU; pick the chunk (>= 8 planes, to bound the
// 2p-plane halo) whose block count best fills whole rounds of 512 slots.
int pick_zchunk(const int* ns) {
  const int n = ns[2];
  const long xy = 3L * ((ns[0] + 31) / 32) * ((ns[1] + 7) / 8);
  const long slots = 512;
  int best = n;
  double best_eff = -1.0;
  for (int nz = 1; nz <= std::max(1, n / 8); ++nz) {
    const int z = (n + nz - 1) / nz;  // balanced chunks
    const long blocks = xy * ((n + z - 1) / z);
    const long rounds = (blocks + slots - 1) / slots;
    // efficiency of the rounds, slightly favouring fewer halo planes
    const double eff = double(blocks) / double(rounds * slots) * (double(z) / (z + 6.0));
    if (eff > best_eff + 1e-9) {
      best_eff = eff;
      best = z;
    }
  }
  return best;
}

// ---------------------------------------------------------------- enqueue
// (kind 2 is not used: it named a separate float64 residual kernel)
enum LaunchKind { kKindRhsE = 0, kKindRhsH = 1, kKindSweepX = 3, kKindSweepYZ = 4,
                  kKindSweepXYZ = 5, kKindApply = 6 };

// Run `launch` on stream s; when profiling, bracket it with two events.
template <typename F>
hipError_t timed(adi_ctx* c, hipStream_t s, int kind, int ndesc, int nmod, int nacc,
                 F&& launch) {
  if (!c->profiling) return launch();
  const size_t i = c->launch_idx++;
  while (c->events.size() < 2 * (i + 1)) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return err;
    c->events.push_back(e);
  }
  if (c->launch_kind.size() < i + 1) {
    c->launch_kind.resize(i + 1);
    c->launch_ndesc.resize(i + 1);
    c->launch_nmod.resize(i + 1);
    c->launch_nacc.resize(i + 1);
  }
  c->launch_kind[i] = kind;
  c->launch_ndesc[i] = ndesc;
  c->launch_nmod[i] = nmod;
  c->launch_nacc[i] = nacc;
  hipError_t e = hipEventRecord(c->events[2 * i], s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return hipEventRecord(c->events[2 * i + 1], s);
}

template <typename T>
RhsArgs<T> rhs_args(adi_ctx* c, const void* const* f, int nf, void* const* out, int kindH,
                    int sub) {
  RhsArgs<T> a{};
  for (int i = 0; i < nf; ++i) a.f[i] = f[i];
  for (int i = 0; i < 3; ++i) a.out[i] = out[i];
  if (kindH) {
    a.coef[0] = c->coefT[3];  // delta
  } else {
    a.coef[0] = c->coefT[2];  // gamma
    a.coef[1] = c->coefT[1];  // beta
    a.coef[2] = c->coefT[0];  // alpha
  }
  a.bandx = static_cast<const T*>(c->bandT[0]);
  a.bandy = static_cast<const T*>(c->bandT[1]);
  a.zw = static_cast<const T*>(c->zwT);
  a.nx = c->ns[0];
  a.ny = c->ns[1];
  a.nz = c->ns[2];
  a.yin0 = c->yin[0];
  a.yin1 = c->yin[1];
  a.yrep = c->yin[2];
  a.zchunk = pick_zchunk(c->ns);
  a.src = c->src;
  a.tnow = c->d_t;
  a.frac_dt = (sub == 1 ? 0.25 : 0.75) * c->dt;
  return a;
}

SweepDesc desc_for(adi_ctx* c, int kindH, int sub, int comp_i, int axis, void* in, void* out,
                   const void* acc) {
  SweepDesc d{};
  d.axis = axis;
  d.in = in;
  d.out = out;
  d.acc = acc;
  const bool mod = !kindH && kModAxis[sub - 1][comp_i] == axis;
  if (mod) {
    const int s = (sub - 1) * 3 + comp_i;
    d.L = c->mL[s];
    d.U = c->mU[s];
    d.D = c->mD[s];
    d.modified = 1;
  } else {
    const int v = dirichlet(kindH, comp_i, axis) ? 1 : 0;
    d.L = c->shL[axis][v];
    d.U = c->shU[axis][v];
    d.D = c->shD[axis][v];
    d.spk = c->spike_ok[axis] ? c->spk[axis][v] : nullptr;
    d.segs = spike_segments(c->ns[axis]);
    d.modified = 0;
  }
  return d;
}

// Partitioned solves for a launch: every descriptor shared, with
// partition data for its axis, all with the same segment count (returned;
// 0 = one lane per line).
int spike_for(const SweepArgs& a, int nd) {
  for (int q = 0; q < nd; ++q)
    if (a.d[q].modified || !a.d[q].spk || a.d[q].segs != a.d[0].segs) return 0;
  return nd > 0 ? a.d[0].segs : 0;
}

// Blocks of 64 lines a launch of these descriptors runs per descriptor.
size_t line_blocks(const adi_ctx* c, const SweepDesc* d, int nd) {
  size_t b = 0;
  for (int q = 0; q < nd; ++q) b = std::max(b, (c->D / size_t(c->ns[d[q].axis]) + 63) / 64);
  return b;
}

// Blocks of 64 lines of one H-stage apply-and-solve round (one descriptor
// per axis).
size_t h_round_blocks(const adi_ctx* c) {
  size_t b = 0;
  for (int ax = 0; ax < 3; ++ax) b = std::max(b, (c->D / size_t(c->ns[ax]) + 63) / 64);
  return 3 * b;
}

// Solve order of component c: modified axis first for E, x y z for H.
void axis_order(int kindH, int sub, int c, int order[3]) {
  if (kindH) {
    order[0] = 0; order[1] = 1; order[2] = 2;
    return;
  }
  const int m = kModAxis[sub - 1][c];
  order[0] = m;
  int k = 1;
  for (int a = 0; a < 3; ++a)
    if (a != m) order[k++] = a;
}

hipError_t next_event(adi_ctx* c, hipEvent_t* e) {
  if (c->fork_idx == c->fork_ev.size()) {
    hipEvent_t ev;
    hipError_t err = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (err != hipSuccess) return err;
    c->fork_ev.push_back(ev);
  }
  *e = c->fork_ev[c->fork_idx++];
  return hipSuccess;
}

// Enqueue the three rounds of 1D solves of one stage on the three components
// of `buf` (in place).  If `acc_base` is given, the last solve of each
// component adds the matching component of acc_base to its solution (the
// increment form of the float32 mode: x_new = x_old + d).
// Within a round the x-line launch and the y/z-line launch touch different
// components: outside the profiling pass the x launch runs on a second
// branch (the side stream, forked from and joined back into s).
template <typename T>
hipError_t enqueue_solves(adi_ctx* c, int kindH, int sub, void* buf, const void* acc_base,
                          hipStream_t s) {
  int order[3][3];
  for (int ci = 0; ci < 3; ++ci) axis_order(kindH, sub, ci, order[ci]);
  for (int r = 0; r < 3; ++r) {
    SweepArgs grp[2]{};
    int nd[2] = {0, 0};
    for (int xgroup = 1; xgroup >= 0; --xgroup) {
      SweepArgs& a = grp[xgroup];
      for (int ci = 0; ci < 3; ++ci) {
        const int ax = order[ci][r];
        if ((ax == 0) != (xgroup == 1)) continue;
        void* in = comp(buf, ci, c);
        const void* acc =
            (acc_base && r == 2) ? comp(const_cast<void*>(acc_base), ci, c) : nullptr;
        a.d[nd[xgroup]++] = desc_for(c, kindH, sub, ci, ax, in, in, acc);
      }
      for (int k = 0; k < 3; ++k) a.dim[k] = c->ns[k];
      a.xaxis = xgroup;
      a.tick_t = nullptr;
      a.spike = spike_for(a, nd[xgroup]);
    }
    // x and y/z descriptors of one kind (all modified or all shared), with
    // at most 1024 blocks of 64 lines in all: one launch, x descriptors
    // first (no cross-stream fork and join, which cost 5-9 us per round);
    // larger rounds run better as two concurrent launches
    SweepDesc alld[6];
    for (int q = 0; q < nd[1]; ++q) alld[q] = grp[1].d[q];
    for (int q = 0; q < nd[0]; ++q) alld[nd[1] + q] = grp[0].d[q];
    const size_t blocks = line_blocks(c, alld, nd[0] + nd[1]) * size_t(nd[0] + nd[1]);
    if (nd[0] > 0 && nd[1] > 0 && blocks <= 1024) {
      const int nmod0 = [&] { int m = 0; for (int q = 0; q < nd[0]; ++q) m += grp[0].d[q].modified; return m; }();
      const int nmod1 = [&] { int m = 0; for (int q = 0; q < nd[1]; ++q) m += grp[1].d[q].modified; return m; }();
      const int nall = nd[0] + nd[1], mall = nmod0 + nmod1;
      if (mall == 0 || mall == nall) {
        SweepArgs a = grp[1];
        for (int q = 0; q < nd[0]; ++q) a.d[nd[1] + q] = grp[0].d[q];
        a.xaxis = 2;
        a.spike = spike_for(a, nall);
        const int nacc = (acc_base && r == 2) ? nall : 0;
        hipError_t e = timed(c, s, kKindSweepXYZ, nall, mall, nacc,
                             [&] { return launch_sweep<T>(c->p, nall, a, s); });
        if (e != hipSuccess) return e;
        continue;
      }
    }
    const bool branch = nd[0] > 0 && nd[1] > 0 && !c->profiling && c->side;
    hipEvent_t ev = nullptr;
    if (branch) {
      hipError_t e = next_event(c, &ev);
      if (e == hipSuccess) e = hipEventRecord(ev, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->side, ev, 0);
      if (e != hipSuccess) return e;
    }
    for (int xgroup = 1; xgroup >= 0; --xgroup) {
      if (nd[xgroup] == 0) continue;
      const SweepArgs& a = grp[xgroup];
      int nmod = 0;
      for (int q = 0; q < nd[xgroup]; ++q) nmod += a.d[q].modified;
      hipStream_t ls = (branch && xgroup == 1) ? c->side : s;
      const int nacc = (acc_base && r == 2) ? nd[xgroup] : 0;
      hipError_t e = timed(c, ls, xgroup ? kKindSweepX : kKindSweepYZ, nd[xgroup], nmod, nacc,
                           [&] { return launch_sweep<T>(c->p, nd[xgroup], a, ls); });
      if (e != hipSuccess) return e;
    }
    if (branch) {
      hipError_t e = next_event(c, &ev);
      if (e == hipSuccess) e = hipEventRecord(ev, c->side);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// H stage of substep `sub` with one delta = dt / (2 mu) in every row
// (discrete2 / discrete4).  Each H_c has two curl terms, delta (+-) times
// E_b with the advection matrix A along one axis a != c and M along the
// other two.  Since E_b vanishes on the faces normal to c (PEC) and H_c
// vanishes there too, the mass solve along c and along the third axis
// cancel their M factors exactly, and the Kronecker solve of the term
// reduces to M_a^{-1} A_a along its own axis:
//   H_c' = H_c + sum over the two terms of (+-delta) M_a^{-1} (A_a E_b).
// Two rounds of apply-and-solve line launches (one term per component each,
// the three components on three different axes) replace the right-hand
// side kernel and the three rounds of mass solves.  Round k = 0 takes the
// terms on the E before the stage (Ein, added to Hin), round 1 those on the
// E after it (added in place); this enqueues round k on stream s.  A round
// too large for one launch puts its x lines on the side stream when
// `may_branch`.
template <typename T>
hipError_t enqueue_h_round(adi_ctx* c, int sub, int k, void* Ein, void* Eout, void* Hin,
                           void* Hout, hipStream_t s, bool may_branch) {
  struct Term { int axis, sign, b; bool old; };  // b = E component, old = E before the stage
  static const Term terms[2][3][2] = {
      {{{1, -1, 2, true}, {2, +1, 1, false}},
       {{2, -1, 0, true}, {0, +1, 2, false}},
       {{0, -1, 1, true}, {1, +1, 0, false}}},
      {{{2, +1, 1, true}, {1, -1, 2, false}},
       {{0, +1, 2, true}, {2, -1, 0, false}},
       {{1, +1, 0, true}, {0, -1, 1, false}}}};
  const int W = 2 * c->p + 1;
  SweepDesc d[3];
  for (int ci = 0; ci < 3; ++ci) {
    const Term& t = terms[sub - 1][ci][k];
    const int ax = t.axis, n = c->ns[ax];
    void* io = comp(Hout, ci, c);
    SweepDesc q = desc_for(c, 1, sub, ci, ax, comp(t.old ? Ein : Eout, t.b, c), io,
                           k == 0 ? comp(Hin, ci, c) : io);
    q.aband = static_cast<const T*>(c->bandT[ax]) + size_t(1) * n * W;  // op 1 = A
    q.scale = t.sign * c->hdelta;
    d[ax] = q;  // one term per axis in each round
  }
  SweepArgs a{};
  for (int q = 0; q < 3; ++q) a.d[q] = d[q];  // x descriptor first
  for (int q = 0; q < 3; ++q) a.dim[q] = c->ns[q];
  a.apply = 1;
  a.xaxis = 2;
  a.spike = spike_for(a, 3);
  if (!a.spike) return hipErrorInvalidValue;
  if (sub == 2 && k == 1) {
    a.tick_t = c->d_t;
    a.tick_dt = c->dt;
  }
  if (h_round_blocks(c) <= 1024)
    return timed(c, s, kKindApply, 3, 0, 3, [&] { return launch_sweep<T>(c->p, 3, a, s); });
  // larger rounds: the x lines on the side branch, the y/z lines here
  SweepArgs ax_{}, ayz{};
  ax_.d[0] = d[0];
  ayz.d[0] = d[1];
  ayz.d[1] = d[2];
  for (SweepArgs* g : {&ax_, &ayz}) {
    for (int q = 0; q < 3; ++q) g->dim[q] = c->ns[q];
    g->apply = 1;
  }
  ax_.xaxis = 1;
  ayz.xaxis = 0;
  ax_.spike = spike_for(ax_, 1);
  ayz.spike = spike_for(ayz, 2);
  ayz.tick_t = a.tick_t;
  ayz.tick_dt = a.tick_dt;
  const bool branch = may_branch && !c->profiling && c->side;
  hipEvent_t ev = nullptr;
  if (branch) {
    hipError_t e = next_event(c, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->side, ev, 0);
    if (e != hipSuccess) return e;
  }
  hipStream_t xs = branch ? c->side : s;
  hipError_t e = timed(c, xs, kKindApply, 1, 0, 1, [&] { return launch_sweep<T>(c->p, 1, ax_, xs); });
  if (e == hipSuccess)
    e = timed(c, s, kKindApply, 2, 0, 2, [&] { return launch_sweep<T>(c->p, 2, ayz, s); });
  if (e != hipSuccess) return e;
  if (branch) {
    e = next_event(c, &ev);
    if (e == hipSuccess) e = hipEventRecord(ev, c->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t enqueue_step_t(adi_ctx* c, hipStream_t s) {
  void* const* B = c->B;
  for (int sub = 1; sub <= 2; ++sub) {
    // buffers: substep 1: E=B0, H=B1 -> E'=B2, H'=B3; substep 2: E'=B2, H'=B3 -> E''=B0, H''=B1
    void* Ein = sub == 1 ? B[0] : B[2];
    void* Hin = sub == 1 ? B[1] : B[3];
    void* Eout = sub == 1 ? B[2] : B[0];
    void* Hout = sub == 1 ? B[3] : B[1];
    // With one permeability the H stage's first round reads only the
    // substep's inputs (Ein, Hin) and writes only Hout, which the E stage
    // neither reads nor writes: outside the profiling pass, a round too
    // large for one launch runs on a branch of its own beside the E stage's
    // solves, joined before round 2 (256^3 p=2 float64 step 6.55 -> 6.33 ms).
    // At 128^3 the overlap gains nothing: the two kernels share the memory
    // system (per-line sweep 67 -> 87 us, round 67 us instead of 37) and the
    // fork and the join each leave the GPU idle for 5-10 us.
    const bool hbranch = c->fast_h && !c->profiling && c->hside && h_round_blocks(c) > 1024;
    hipEvent_t hev = nullptr;
    // E stage: right-hand sides (float32 mode: increments b - P E_old) into
    // Eout, then the three solves in place (float32 mode: + E_old)
    {
      const void* f[6] = {comp(Ein, 0, c), comp(Ein, 1, c), comp(Ein, 2, c),
                          comp(Hin, 0, c), comp(Hin, 1, c), comp(Hin, 2, c)};
      void* out[3] = {comp(Eout, 0, c), comp(Eout, 1, c), comp(Eout, 2, c)};
      hipError_t e;
      if (!c->refine()) {
        RhsArgs<T> a = rhs_args<T>(c, f, 6, out, 0, sub);
        e = timed(c, s, kKindRhsE, 3, 0, 0, [&] {
          return launch_rhs<T>(sub == 1 ? kStageE1 : kStageE2, c->p, a, s);
        });
      } else {
        const int stage = sub == 1 ? kStageEd1 : kStageEd2;
        if (c->res64 & res64_bit(0, sub)) {
          RhsArgs<double> a = rhs_args<double>(c, f, 6, out, 0, sub);
          a.coef[0] = c->gm1T;  // gamma - 1: the mass part of P E folded in
          a.bandx = c->band64[0];
          a.bandy = c->band64[1];
          a.zw = c->zw64;
          e = timed(c, s, kKindRhsE, 3, 0, 0, [&] { return launch_rhs_inc(stage, c->p, a, s); });
        } else {
          RhsArgs<float> a = rhs_args<float>(c, f, 6, out, 0, sub);
          a.coef[0] = c->gm1T;
          e = timed(c, s, kKindRhsE, 3, 0, 0, [&] { return launch_rhs_inc32(stage, c->p, a, s); });
        }
      }
      if (e != hipSuccess) return e;
      if (hbranch) {
        e = next_event(c, &hev);
        if (e == hipSuccess) e = hipEventRecord(hev, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(c->hside, hev, 0);
        if (e == hipSuccess) e = enqueue_h_round<T>(c, sub, 0, Ein, Eout, Hin, Hout, c->hside, false);
        if (e == hipSuccess) e = next_event(c, &hev);
        if (e == hipSuccess) e = hipEventRecord(hev, c->hside);
        if (e != hipSuccess) return e;
      }
      e = enqueue_solves<T>(c, 0, sub, Eout, c->refine() ? Ein : nullptr, s);
      if (e != hipSuccess) return e;
    }
    // H stage
    if (c->fast_h) {
      hipError_t e = hbranch ? hipStreamWaitEvent(s, hev, 0)
                             : enqueue_h_round<T>(c, sub, 0, Ein, Eout, Hin, Hout, s, true);
      if (e == hipSuccess) e = enqueue_h_round<T>(c, sub, 1, Ein, Eout, Hin, Hout, s, true);
      if (e != hipSuccess) return e;
    } else {
      const void* f[9] = {comp(Hin, 0, c),  comp(Hin, 1, c),  comp(Hin, 2, c),
                          comp(Ein, 0, c),  comp(Ein, 1, c),  comp(Ein, 2, c),
                          comp(Eout, 0, c), comp(Eout, 1, c), comp(Eout, 2, c)};
      void* out[3] = {comp(Hout, 0, c), comp(Hout, 1, c), comp(Hout, 2, c)};
      hipError_t e;
      if (!c->refine()) {
        RhsArgs<T> a = rhs_args<T>(c, f, 9, out, 1, sub);
        e = timed(c, s, kKindRhsH, 3, 0, 0, [&] {
          return launch_rhs<T>(sub == 1 ? kStageH1 : kStageH2, c->p, a, s);
        });
      } else {
        // increments b - M H_old: the delta terms alone (H_old is not read)
        const int stage = sub == 1 ? kStageHd1 : kStageHd2;
        if (c->res64 & res64_bit(1, sub)) {
          RhsArgs<double> a = rhs_args<double>(c, f, 9, out, 1, sub);
          a.bandx = c->band64[0];
          a.bandy = c->band64[1];
          a.zw = c->zw64;
          e = timed(c, s, kKindRhsH, 3, 0, 0, [&] { return launch_rhs_inc(stage, c->p, a, s); });
        } else {
          RhsArgs<float> a = rhs_args<float>(c, f, 9, out, 1, sub);
          e = timed(c, s, kKindRhsH, 3, 0, 0, [&] { return launch_rhs_inc32(stage, c->p, a, s); });
        }
      }
      if (e != hipSuccess) return e;
      // H: x, y, z (all shared factors); the last launch advances the time
      // and, in the float32 mode, adds H_old
      for (int ax = 0; ax < 3; ++ax) {
        SweepArgs w{};
        const bool add = c->refine() && ax == 2;
        for (int ci = 0; ci < 3; ++ci) {
          void* io = comp(Hout, ci, c);
          w.d[ci] = desc_for(c, 1, sub, ci, ax, io, io, add ? comp(Hin, ci, c) : nullptr);
        }
        for (int k = 0; k < 3; ++k) w.dim[k] = c->ns[k];
        w.xaxis = ax == 0;
        w.spike = spike_for(w, 3);
        if (sub == 2 && ax == 2) {
          w.tick_t = c->d_t;
          w.tick_dt = c->dt;
        }
        e = timed(c, s, ax == 0 ? kKindSweepX : kKindSweepYZ, 3, 0, add ? 3 : 0,
                  [&] { return launch_sweep<T>(c->p, 3, w, s); });
        if (e != hipSuccess) return e;
      }
    }
  }
  return hipSuccess;
}

hipError_t enqueue_step(adi_ctx* c, hipStream_t s) {
  return c->refine() ? enqueue_step_t<float>(c, s) : enqueue_step_t<double>(c, s);
}

void drop_graph(adi_ctx* c) {
  if (c->exec) hipGraphExecDestroy(c->exec);
  if (c->graph) hipGraphDestroy(c->graph);
  c->exec = nullptr;
  c->graph = nullptr;
}

int capture(adi_ctx* c) {
  drop_graph(c);
  c->launch_idx = 0;
  c->fork_idx = 0;
  HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
  hipError_t e = enqueue_step(c, c->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess) return fail(c, ADI_EHIP, std::string("step capture: ") + hipGetErrorString(e));
  if (e2 != hipSuccess) return fail(c, ADI_EHIP, std::string("end capture: ") + hipGetErrorString(e2));
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0));
  return ADI_OK;
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int ensure_stream(adi_ctx* c) {
  if (c->cap) return ADI_OK;
  HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  HIPCHK(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  HIPCHK(c, hipStreamCreateWithFlags(&c->hside, hipStreamNonBlocking));
  return ADI_OK;
}

int ensure_workspace(adi_ctx* c) {
  int st = ensure_stream(c);
  if (st != ADI_OK) return st;
  if (c->ws) return ADI_OK;
  const size_t bytes = layout(c, nullptr);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(c, ADI_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->ws = static_cast<unsigned char*>(p);
  c->ws_bytes = bytes;
  c->own_ws = true;
  const size_t aligned = (reinterpret_cast<uintptr_t>(c->ws) + 255) & ~uintptr_t(255);
  layout(c, reinterpret_cast<unsigned char*>(aligned));
  // a defined initial state: zero fields at t = 0 (not part of any graph)
  HIPCHK(c, hipMemset(c->B[0], 0, 6 * c->D * c->esz));
  HIPCHK(c, hipMemset(c->d_t, 0, 8));
  return ADI_OK;
}

}  // namespace

// ====================================================================== ABI
extern "C" {

int adi_create(adi_ctx** out, int nx, int ny, int nz, int p, int precision, void* hip_stream) {
  if (!out) return ADI_EINVAL;
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || p < 1 || p > kMaxP) return ADI_EINVAL;
  if (precision != ADI_FP64 && precision != ADI_FP32_REFINE) return ADI_EINVAL;
  // coefficients per component below 2^31 (32-bit line and column indices)
  const size_t D = size_t(nx + p) * size_t(ny + p) * size_t(nz + p);
  if (D >= (size_t(1) << 31)) return ADI_EINVAL;
  adi_ctx* c = new adi_ctx();
  const int Ns[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    c->Ns[a] = Ns[a];
    c->ns[a] = Ns[a] + p;
  }
  c->N = nx;
  c->p = p;
  c->n = nx + p;
  c->D = D;
  c->prec = precision;
  c->esz = precision == ADI_FP64 ? 8 : 4;
  c->stream = static_cast<hipStream_t>(hip_stream);
  // the private capture stream is created on first device use, so that
  // argument validation never touches the GPU
  *out = c;
  return ADI_OK;
}

int adi_ncoef(const adi_ctx* c) { return c ? c->n : ADI_EINVAL; }

int adi_dims(const adi_ctx* c, int* n_out) {
  if (!c || !n_out) return ADI_EINVAL;
  for (int a = 0; a < 3; ++a) n_out[a] = c->ns[a];
  return ADI_OK;
}

size_t adi_workspace_bytes(const adi_ctx* c) {
  if (!c) return 0;
  adi_ctx tmp;
  for (int a = 0; a < 3; ++a) {
    tmp.Ns[a] = c->Ns[a];
    tmp.ns[a] = c->ns[a];
  }
  tmp.N = c->N; tmp.p = c->p; tmp.n = c->n; tmp.D = c->D; tmp.prec = c->prec; tmp.esz = c->esz;
  return layout(&tmp, nullptr);
}

int adi_bind_workspace(adi_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return ADI_EINVAL;
  if (c->ws) return fail(c, ADI_ESTATE, "workspace already set");
  const size_t need = layout(c, nullptr);
  if (bytes < need) return fail(c, ADI_ENOMEM, "workspace too small");
  int st = ensure_stream(c);
  if (st != ADI_OK) return st;
  c->ws = static_cast<unsigned char*>(dev_ptr);
  c->ws_bytes = bytes;
  c->own_ws = false;
  const size_t aligned = (reinterpret_cast<uintptr_t>(c->ws) + 255) & ~uintptr_t(255);
  layout(c, reinterpret_cast<unsigned char*>(aligned));
  HIPCHK(c, hipMemset(c->B[0], 0, 6 * c->D * c->esz));
  HIPCHK(c, hipMemset(c->d_t, 0, 8));
  return ADI_OK;
}

int adi_set_material_dof(adi_ctx* c, const double* eps, const double* mu, const double* sig) {
  if (!c || !eps || !mu || !sig) return ADI_EINVAL;
  for (size_t i = 0; i < c->D; ++i) {
    if (!std::isfinite(eps[i]) || !std::isfinite(mu[i]) || !std::isfinite(sig[i]))
      return fail(c, ADI_EINVAL, "material value not finite");
    if (!(eps[i] > 0.0) || !(mu[i] > 0.0) || sig[i] < 0.0)
      return fail(c, ADI_EINVAL, "need eps > 0, mu > 0, sigma >= 0");
  }
  c->eps.assign(eps, eps + c->D);
  c->mu.assign(mu, mu + c->D);
  c->sig.assign(sig, sig + c->D);
  c->have_material = true;
  c->factored = false;
  return ADI_OK;
}

int adi_set_material(adi_ctx* c, const double* eps_r, const double* mu_r, const double* sigma_nd,
                     int vx, int vy, int vz, int map_mode) {
  if (!c || !eps_r || !mu_r || !sigma_nd || vx < 1 || vy < 1 || vz < 1) return ADI_EINVAL;
  if (map_mode != ADI_MAP_GREVILLE && map_mode != ADI_MAP_BSPLINE_AVG)
    return fail(c, ADI_EINVAL, "unknown material map mode");
  const size_t V = size_t(vx) * vy * vz;
  for (size_t i = 0; i < V; ++i) {
    if (!std::isfinite(eps_r[i]) || !std::isfinite(mu_r[i]) || !std::isfinite(sigma_nd[i]))
      return fail(c, ADI_EINVAL, "material value not finite");
    if (!(eps_r[i] > 0.0) || !(mu_r[i] > 0.0) || sigma_nd[i] < 0.0)
      return fail(c, ADI_EINVAL, "need eps > 0, mu > 0, sigma >= 0");
  }
  if (map_mode == ADI_MAP_BSPLINE_AVG) {
    // DOF (i,j,k) takes the voxel values averaged with the weights of its
    // test function B_i B_j B_k, one axis at a time (x, then y, then z)
    const int nx = c->ns[0], ny = c->ns[1], nz = c->ns[2];
    const std::vector<double> wx = voxel_weights(c->Ns[0], c->p, vx),
                              wy = voxel_weights(c->Ns[1], c->p, vy),
                              wz = voxel_weights(c->Ns[2], c->p, vz);
    auto avg = [&](const double* m, std::vector<double>& out) {
      std::vector<double> a(size_t(vz) * vy * nx, 0.0), b(size_t(vz) * ny * nx, 0.0);
      for (int k = 0; k < vz; ++k)
        for (int j = 0; j < vy; ++j) {
          const double* row = m + (size_t(k) * vy + j) * vx;
          double* o = a.data() + (size_t(k) * vy + j) * nx;
          for (int i = 0; i < nx; ++i) {
            const double* w = wx.data() + size_t(i) * vx;
            double s = 0.0;
            for (int v = 0; v < vx; ++v) s += w[v] * row[v];
            o[i] = s;
          }
        }
      for (int k = 0; k < vz; ++k)
        for (int jj = 0; jj < ny; ++jj) {
          const double* w = wy.data() + size_t(jj) * vy;
          double* o = b.data() + (size_t(k) * ny + jj) * nx;
          for (int v = 0; v < vy; ++v) {
            if (w[v] == 0.0) continue;
            const double* src = a.data() + (size_t(k) * vy + v) * nx;
            for (int i = 0; i < nx; ++i) o[i] += w[v] * src[i];
          }
        }
      out.assign(c->D, 0.0);
      const size_t plane = size_t(nx) * ny;
      for (int kk = 0; kk < nz; ++kk) {
        const double* w = wz.data() + size_t(kk) * vz;
        double* o = out.data() + size_t(kk) * plane;
        for (int v = 0; v < vz; ++v) {
          if (w[v] == 0.0) continue;
          const double* src = b.data() + size_t(v) * plane;
          for (size_t q = 0; q < plane; ++q) o[q] += w[v] * src[q];
        }
      }
    };
    avg(eps_r, c->eps);
    avg(mu_r, c->mu);
    avg(sigma_nd, c->sig);
    c->have_material = true;
    c->factored = false;
    return ADI_OK;
  }
  // Greville sampling: DOF (i,j,k) takes the voxel containing (xi_i, xi_j, xi_k).
  auto vox = [](double x, int V) { return std::min(int(std::floor(x * V)), V - 1); };
  const int V3[3] = {vx, vy, vz};
  std::vector<int> idx[3];
  for (int ax = 0; ax < 3; ++ax) {
    const std::vector<double> xi = greville(c->Ns[ax], c->p);
    idx[ax].resize(c->ns[ax]);
    for (int i = 0; i < c->ns[ax]; ++i) idx[ax][i] = vox(xi[i], V3[ax]);
  }
  c->eps.resize(c->D);
  c->mu.resize(c->D);
  c->sig.resize(c->D);
  const int nx = c->ns[0], ny = c->ns[1], nz = c->ns[2];
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t o = i + size_t(nx) * (j + size_t(ny) * k);
        const size_t v = idx[0][i] + size_t(vx) * (idx[1][j] + size_t(vy) * idx[2][k]);
        c->eps[o] = eps_r[v];
        c->mu[o] = mu_r[v];
        c->sig[o] = sigma_nd[v];
      }
  c->have_material = true;
  c->factored = false;
  return ADI_OK;
}

int adi_set_local_dt(adi_ctx* c, const double* tau) {
  if (!c) return ADI_EINVAL;
  if (!tau) {
    c->tau.clear();
  } else {
    for (size_t i = 0; i < c->D; ++i)
      if (!std::isfinite(tau[i]) || tau[i] < 0.0)
        return fail(c, ADI_EINVAL, "local time steps must be finite and >= 0");
    c->tau.assign(tau, tau + c->D);
  }
  c->factored = false;
  return ADI_OK;
}

int adi_set_source(adi_ctx* c, const double xs[3], int comp_i, double amp, double f0, double t0,
                   double width) {
  if (!c || !xs || comp_i < 0 || comp_i > 2) return ADI_EINVAL;
  if (!(width > 0.0)) return fail(c, ADI_EINVAL, "source width must be > 0");
  for (int a = 0; a < 3; ++a)
    if (!(xs[a] >= 0.0 && xs[a] <= 1.0)) return fail(c, ADI_EINVAL, "source outside the domain");
  SourceArgs s{};
  if (amp == 0.0) {
    s.comp = -1;
  } else {
    s.comp = comp_i;
    s.amp = amp;
    s.f0 = f0;
    s.t0 = t0;
    s.width = width;
    double vals[kMaxP + 1];
    int first;
    basis_at(c->Ns[0], c->p, xs[0], &first, vals);
    s.first[0] = first;
    for (int r = 0; r <= c->p; ++r) s.bx[r] = vals[r];
    basis_at(c->Ns[1], c->p, xs[1], &first, vals);
    s.first[1] = first;
    for (int r = 0; r <= c->p; ++r) s.by[r] = vals[r];
    basis_at(c->Ns[2], c->p, xs[2], &first, vals);
    s.first[2] = first;
    for (int r = 0; r <= c->p; ++r) s.bz[r] = vals[r];
  }
  c->src = s;
  for (int a = 0; a < 3; ++a) c->src_xs[a] = xs[a];
  c->factored = false;
  return ADI_OK;
}

int adi_factor(adi_ctx* c, double dt) {
  if (!c) return ADI_EINVAL;
  if (!c->have_material) return fail(c, ADI_ESTATE, "set the material before factor");
  if (!std::isfinite(dt) || dt < 0.0) return fail(c, ADI_EINVAL, "dt must be finite and >= 0");
  c->factored = false;  // until this factorisation has succeeded
  int st = ensure_workspace(c);
  if (st != ADI_OK) return st;
  const int p = c->p, W = 2 * p + 1;
  const size_t D = c->D;
  c->dt = dt;
  c->cl_mat_valid = false;

  // per axis: 1D operators (float64, exact Gauss quadrature), shared factors
  // of M (free) and M with Dirichlet rows/columns, their partitioned-solve
  // data (long lines only; any failed self-check keeps the one-lane-per-line
  // solve) and the bands the per-line factors are built from
  Gram1D gz;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = c->ns[ax];
    Gram1D g = build_gram(c->Ns[ax], p);
    std::vector<double> ops(size_t(4) * n * W);
    std::copy(g.M.begin(), g.M.end(), ops.begin());
    std::copy(g.A.begin(), g.A.end(), ops.begin() + size_t(n) * W);
    std::copy(g.B.begin(), g.B.end(), ops.begin() + size_t(2) * n * W);
    std::copy(g.S.begin(), g.S.end(), ops.begin() + size_t(3) * n * W);
    if ((st = upload(c, c->bandT[ax], ops)) != ADI_OK) return st;
    HIPCHK(c, hipMemcpy(c->band64[ax], ops.data(), ops.size() * 8, hipMemcpyHostToDevice));
    if (ax == 1) invariant_rows(ops, n, W, c->yin);
    if (ax == 2) {
      // z weights: input plane k contributes Z[k-p+q][k] to output plane k-p+q
      std::vector<double> zw(size_t(4) * n * W, 0.0);
      for (int op = 0; op < 4; ++op)
        for (int k = 0; k < n; ++k)
          for (int q = 0; q < W; ++q) {
            const int t = k - p + q;
            if (t < 0 || t >= n) continue;
            zw[(size_t(op) * n + k) * W + q] = ops[(size_t(op) * n + t) * W + (k - t + p)];
          }
      if ((st = upload(c, c->zwT, zw)) != ADI_OK) return st;
      HIPCHK(c, hipMemcpy(c->zw64, zw.data(), zw.size() * 8, hipMemcpyHostToDevice));
    }
    for (int v = 0; v < 2; ++v) {
      std::vector<double> band = g.M;
      if (v) apply_dirichlet(band, n, p);
      std::vector<double> L, U, Dinv;
      const double r = band_lu(band, n, p, L, U, Dinv);
      if (!(r > c->pivot_floor))
        return fail(c, ADI_ESINGULAR, "pivot at or below the floor in a mass matrix factor");
      for (int i = 0; i < n; ++i)  // pre-scale the upper factor: D * U
        for (int k = 0; k < p; ++k) U[size_t(i) * p + k] *= Dinv[i];
      if ((st = upload(c, c->shL[ax][v], L)) != ADI_OK) return st;
      if ((st = upload(c, c->shU[ax][v], U)) != ADI_OK) return st;
      if ((st = upload(c, c->shD[ax][v], Dinv)) != ADI_OK) return st;
    }
    c->spike_ok[ax] = false;
    if (n >= kSpikeMinN && n <= kSpikeMaxN) {
      bool ok = true;
      std::vector<double> pack[2];
      for (int v = 0; v < 2 && ok; ++v) {
        std::vector<double> band = g.M;
        if (v) apply_dirichlet(band, n, p);
        SpikeData sd;
        ok = spike_prepare(band, n, p, spike_segments(n), sd);
        if (!ok) break;
        for (const std::vector<double>* part : {&sd.L, &sd.DU, &sd.D, &sd.V, &sd.W, &sd.R})
          pack[v].insert(pack[v].end(), part->begin(), part->end());
      }
      if (ok) {
        for (int v = 0; v < 2; ++v)
          if ((st = upload(c, c->spk[ax][v], pack[v])) != ADI_OK) return st;
        c->spike_ok[ax] = true;
      }
    }
    // bands of the material-modified systems along this axis (always
    // Dirichlet: the modified axis of E_c is never axis c)
    std::vector<double> fb(size_t(2) * n * W);
    std::vector<double> Mb = g.M, Sb = g.S;
    apply_dirichlet(Mb, n, p);
    apply_dirichlet(Sb, n, p);
    for (int b : {0, n - 1}) Sb[size_t(b) * W + p] = 0.0;  // identity rows carry no alpha S
    std::copy(Mb.begin(), Mb.end(), fb.begin());
    std::copy(Sb.begin(), Sb.end(), fb.begin() + size_t(n) * W);
    HIPCHK(c, hipMemcpy(c->fb64[ax], fb.data(), fb.size() * 8, hipMemcpyHostToDevice));
  }

  // per-row coefficients (material attached to test functions), with the
  // trapezoidal conductivity term: c = sigma dt / (4 eps),
  // alpha = dt^2/(4 eps mu (1+c)), beta = dt/(2 eps (1+c)),
  // gamma = (1-c)/(1+c), delta = dt/(2 mu)
  std::vector<double> co[5];
  for (auto& v : co) v.resize(D);
  // (a local time step per test function replaces dt in its row)
  for (size_t i = 0; i < D; ++i) {
    const double e = c->eps[i], m = c->mu[i], s = c->sig[i];
    const double tt = c->tau.empty() ? dt : c->tau[i];
    const double cc = s * tt / (4.0 * e);
    co[0][i] = tt * tt / (4.0 * e * m * (1.0 + cc));
    co[1][i] = tt / (2.0 * e * (1.0 + cc));
    co[2][i] = (1.0 - cc) / (1.0 + cc);
    co[3][i] = tt / (2.0 * m);
    co[4][i] = -2.0 * cc / (1.0 + cc);  // gamma - 1 without cancellation
  }
  for (int i = 0; i < 4; ++i) {
    if ((st = upload(c, c->coefT[i], co[i])) != ADI_OK) return st;
    if (c->refine())
      HIPCHK(c, hipMemcpy(c->coef64[i], co[i].data(), D * 8, hipMemcpyHostToDevice));
  }
  if (c->refine() && (st = upload(c, c->gm1T, co[4])) != ADI_OK) return st;

  // per-line factors of the modified systems
  double worst = 1e300;
  for (int sub = 1; sub <= 2; ++sub)
    for (int ci = 0; ci < 3; ++ci) {
      const int s = (sub - 1) * 3 + ci;
      const int ax = kModAxis[sub - 1][ci], n = c->ns[ax];
      FactorArgs f{};
      f.Mb = c->fb64[ax];
      f.Sb = c->fb64[ax] + size_t(n) * W;
      f.alpha = c->coef64[0];
      if (c->refine()) {
        f.L32 = static_cast<float*>(c->mL[s]);
        f.U32 = static_cast<float*>(c->mU[s]);
        f.D32 = static_cast<float*>(c->mD[s]);
      } else {
        f.L64 = static_cast<double*>(c->mL[s]);
        f.U64 = static_cast<double*>(c->mU[s]);
        f.D64 = static_cast<double*>(c->mD[s]);
      }
      f.minratio = c->minratio;
      f.n = n;
      f.nlines = int(D / size_t(n));
      f.axis = ax;
      f.nx = c->ns[0];
      f.ny = c->ns[1];
      std::vector<double> ratios(size_t(f.nlines));
      HIPCHK(c, launch_factor(p, f, c->cap));
      HIPCHK(c, hipMemcpyAsync(ratios.data(), c->minratio, ratios.size() * 8,
                               hipMemcpyDeviceToHost, c->cap));
      HIPCHK(c, hipStreamSynchronize(c->cap));
      for (double r : ratios) worst = std::min(worst, r);
    }
  if (!(worst > c->pivot_floor))
    return fail(c, ADI_ESINGULAR, "pivot at or below the floor in a material-modified factor");

  // the H stage's shortcut needs one delta for all rows and partitioned
  // solves with one segment count on every axis
  bool one_delta = true;
  for (size_t i = 1; i < D && one_delta; ++i) one_delta = co[3][i] == co[3][0];
  c->fast_h = one_delta && c->spike_ok[0] && c->spike_ok[1] && c->spike_ok[2] &&
              spike_segments(c->ns[0]) == spike_segments(c->ns[1]) &&
              spike_segments(c->ns[0]) == spike_segments(c->ns[2]);
  c->hdelta = co[3][0];

  st = capture(c);
  if (st != ADI_OK) return st;
  c->factored = true;
  return ADI_OK;
}

int adi_set_pivot_floor(adi_ctx* c, double floor) {
  if (!c) return ADI_EINVAL;
  if (!std::isfinite(floor) || floor < 0.0) return fail(c, ADI_EINVAL, "pivot floor must be finite and >= 0");
  c->pivot_floor = floor;
  c->factored = false;
  return ADI_OK;
}

int adi_set_residual64(adi_ctx* c, int mask) {
  if (!c) return ADI_EINVAL;
  if (mask < 0 || mask > 15) return fail(c, ADI_EINVAL, "residual mask must be in [0, 15]");
  c->res64 = mask;
  c->factored = false;  // the captured step changes
  return ADI_OK;
}

int adi_set_fields(adi_ctx* c, const double* EH, double t) {
  if (!c || !EH) return ADI_EINVAL;
  if (!finite_all(EH, 6 * c->D) || !std::isfinite(t))
    return fail(c, ADI_ENONFINITE, "field value not finite");
  if (!c->ws) {
    int st = ensure_workspace(c);
    if (st != ADI_OK) return st;
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // the state lives in the constrained space: E_c is zero on the faces
  // normal to the two other axes, H_c on the faces normal to axis c (PEC,
  // imposed strongly)
  std::vector<double> v(EH, EH + 6 * c->D);
  const int nx = c->ns[0], ny = c->ns[1], nz = c->ns[2];
  for (int f = 0; f < 6; ++f) {
    const int cc = f % 3;
    double* a = v.data() + size_t(f) * c->D;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          const bool b[3] = {i == 0 || i == nx - 1, j == 0 || j == ny - 1, k == 0 || k == nz - 1};
          const bool zero = f < 3 ? (b[(cc + 1) % 3] || b[(cc + 2) % 3]) : b[cc];
          if (zero) a[(size_t(k) * ny + j) * nx + i] = 0.0;
        }
  }
  if (c->esz == 8) {
    HIPCHK(c, hipMemcpy(c->B[0], v.data(), 6 * c->D * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(v.begin(), v.end());
    HIPCHK(c, hipMemcpy(c->B[0], f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  HIPCHK(c, hipMemcpy(c->d_t, &t, 8, hipMemcpyHostToDevice));
  c->t = t;
  return ADI_OK;
}

int adi_step(adi_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return ADI_EINVAL;
  if (!c->factored || !c->exec) return fail(c, ADI_ESTATE, "adi_factor must succeed before adi_step");
  for (int i = 0; i < nsteps; ++i) HIPCHK(c, hipGraphLaunch(c->exec, c->stream));
  c->t += nsteps * c->dt;
  return ADI_OK;
}

int adi_get_fields(adi_ctx* c, double* EH_out, double* t_out) {
  if (!c || !EH_out) return ADI_EINVAL;
  if (!c->ws) return fail(c, ADI_ESTATE, "no state");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (c->esz == 8) {
    HIPCHK(c, hipMemcpy(EH_out, c->B[0], 6 * c->D * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(6 * c->D);
    HIPCHK(c, hipMemcpy(f.data(), c->B[0], f.size() * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < f.size(); ++i) EH_out[i] = f[i];
  }
  double t = 0.0;
  HIPCHK(c, hipMemcpy(&t, c->d_t, 8, hipMemcpyDeviceToHost));
  if (t_out) *t_out = t;
  return ADI_OK;
}

int adi_fields_device(adi_ctx* c, void** dev, int* dtype) {
  if (!c || !dev || !dtype) return ADI_EINVAL;
  if (!c->ws) return fail(c, ADI_ESTATE, "no state");
  *dev = c->B[0];
  *dtype = c->esz == 8 ? 0 : 1;
  return ADI_OK;
}

int adi_sync(adi_ctx* c) {
  if (!c) return ADI_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return ADI_OK;
}

int adi_profile_run(adi_ctx* c, int nsteps) {
  if (!c || nsteps < 1) return ADI_EINVAL;
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor must succeed before profiling");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->profiling = true;
  c->launch_ms_sum.clear();
  c->profiled_steps = 0;
  int st = ADI_OK;
  for (int k = 0; k < nsteps && st == ADI_OK; ++k) {
    c->launch_idx = 0;
    hipError_t e = enqueue_step(c, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      st = fail(c, ADI_EHIP, std::string("profiled step: ") + hipGetErrorString(e));
      break;
    }
    const size_t n = c->launch_idx;
    c->launch_ms_sum.resize(n, 0.0);
    for (size_t i = 0; i < n; ++i) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, c->events[2 * i], c->events[2 * i + 1]);
      if (e != hipSuccess) {
        st = fail(c, ADI_EHIP, std::string("hipEventElapsedTime: ") + hipGetErrorString(e));
        break;
      }
      c->launch_ms_sum[i] += ms;
    }
    ++c->profiled_steps;
  }
  c->profiling = false;
  c->t += c->profiled_steps * c->dt;
  return st;
}

int adi_profile_read(adi_ctx* c, int cap, int* nout, int* kind, int* ndesc, int* nmod,
                     int* nacc, float* ms) {
  if (!c || !nout) return ADI_EINVAL;
  if (c->profiled_steps == 0) return fail(c, ADI_ESTATE, "run adi_profile_run first");
  const int n = int(c->launch_ms_sum.size());
  *nout = n;
  for (int i = 0; i < n && i < cap; ++i) {
    if (kind) kind[i] = c->launch_kind[i];
    if (ndesc) ndesc[i] = c->launch_ndesc[i];
    if (nmod) nmod[i] = c->launch_nmod[i];
    if (nacc) nacc[i] = c->launch_nacc[i];
    if (ms) ms[i] = float(c->launch_ms_sum[i] / c->profiled_steps);
  }
  return ADI_OK;
}

const char* adi_last_error(const adi_ctx* c) { return c ? c->err.c_str() : "invalid handle"; }

void adi_destroy(adi_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  drop_graph(c);
  for (hipEvent_t e : c->events) hipEventDestroy(e);
  if (c->own_ws && c->ws) hipFree(c->ws);
  if (c->cl_prev) hipFree(c->cl_prev);
  if (c->cl_mat) hipFree(c->cl_mat);
  if (c->cl_red) hipFree(c->cl_red);
  if (c->cl_flag) hipFree(c->cl_flag);
  if (c->mms_tab) hipFree(c->mms_tab);
  if (c->mms_vals) hipFree(c->mms_vals);
  if (c->mms_part) hipFree(c->mms_part);
  if (c->cap) hipStreamDestroy(c->cap);
  if (c->side) hipStreamDestroy(c->side);
  if (c->hside) hipStreamDestroy(c->hside);
  for (hipEvent_t e : c->fork_ev) hipEventDestroy(e);
  delete c;
}

// ------------------------------------------------------------- test hooks
int adi_rhs(adi_ctx* c, int stage, int sub, const double* in, double t, double* out) {
  if (!c || !in || !out || (stage != 0 && stage != 1) || (sub != 1 && sub != 2)) return ADI_EINVAL;
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor first");
  const int nf = stage == 0 ? 6 : 9;
  const size_t D = c->D, es = c->esz;
  void* din = nullptr;
  void* dout = nullptr;
  HIPCHK(c, hipMalloc(&din, nf * D * es));
  HIPCHK(c, hipMalloc(&dout, 3 * D * es));
  int st = ADI_OK;
  do {
    std::vector<double> v(in, in + nf * D);
    if ((st = upload(c, din, v)) != ADI_OK) break;
    double tt = t;
    if (hipMemcpy(c->d_t, &tt, 8, hipMemcpyHostToDevice) != hipSuccess) { st = fail(c, ADI_EHIP, "copy t"); break; }
    const void* f[9];
    for (int i = 0; i < nf; ++i) f[i] = static_cast<unsigned char*>(din) + size_t(i) * D * es;
    void* o[3] = {dout, static_cast<unsigned char*>(dout) + D * es,
                  static_cast<unsigned char*>(dout) + 2 * D * es};
    const int kind = stage == 0 ? (sub == 1 ? kStageE1 : kStageE2) : (sub == 1 ? kStageH1 : kStageH2);
    hipError_t e;
    if (es == 8) e = launch_rhs<double>(kind, c->p, rhs_args<double>(c, f, nf, o, stage, sub), c->cap);
    else e = launch_rhs<float>(kind, c->p, rhs_args<float>(c, f, nf, o, stage, sub), c->cap);
    if (e != hipSuccess || hipStreamSynchronize(c->cap) != hipSuccess) { st = fail(c, ADI_EHIP, "rhs kernel"); break; }
    if (es == 8) {
      if (hipMemcpy(out, dout, 3 * D * 8, hipMemcpyDeviceToHost) != hipSuccess) { st = fail(c, ADI_EHIP, "copy"); break; }
    } else {
      std::vector<float> f32(3 * D);
      if (hipMemcpy(f32.data(), dout, 3 * D * 4, hipMemcpyDeviceToHost) != hipSuccess) { st = fail(c, ADI_EHIP, "copy"); break; }
      for (size_t i = 0; i < f32.size(); ++i) out[i] = f32[i];
    }
    double t0 = c->t;
    hipMemcpy(c->d_t, &t0, 8, hipMemcpyHostToDevice);
  } while (false);
  hipFree(din);
  hipFree(dout);
  return st;
}

int adi_solve(adi_ctx* c, int stage, int sub, double* inout) {
  if (!c || !inout || (stage != 0 && stage != 1) || (sub != 1 && sub != 2)) return ADI_EINVAL;
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor first");
  const size_t D = c->D, es = c->esz;
  void* d = nullptr;
  HIPCHK(c, hipMalloc(&d, 3 * D * es));
  int st = ADI_OK;
  do {
    std::vector<double> v(inout, inout + 3 * D);
    if ((st = upload(c, d, v)) != ADI_OK) break;
    c->fork_idx = 0;
    hipError_t e = es == 8 ? enqueue_solves<double>(c, stage, sub, d, nullptr, c->cap)
                           : enqueue_solves<float>(c, stage, sub, d, nullptr, c->cap);
    if (e != hipSuccess || hipStreamSynchronize(c->cap) != hipSuccess) { st = fail(c, ADI_EHIP, "solve kernels"); break; }
    if (es == 8) {
      if (hipMemcpy(inout, d, 3 * D * 8, hipMemcpyDeviceToHost) != hipSuccess) { st = fail(c, ADI_EHIP, "copy"); break; }
    } else {
      std::vector<float> f32(3 * D);
      if (hipMemcpy(f32.data(), d, 3 * D * 4, hipMemcpyDeviceToHost) != hipSuccess) { st = fail(c, ADI_EHIP, "copy"); break; }
      for (size_t i = 0; i < f32.size(); ++i) inout[i] = f32[i];
    }
  } while (false);
  hipFree(d);
  return st;
}

}  // extern "C"

// ------------------------------------------------------------ closure glue
namespace {

constexpr int kClosureBlocks = 1024;

int closure_ready(adi_ctx* c) {
  // the network's features index the coefficient grid as a cube
  if (c->ns[0] != c->ns[1] || c->ns[0] != c->ns[2])
    return fail(c, ADI_EINVAL, "the learned closure needs a cubic patch (nx = ny = nz)");
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor first");
  const size_t D = c->D;
  if (!c->cl_prev) {
    void* p = nullptr;
    HIPCHK(c, hipMalloc(&p, 6 * D * c->esz));
    c->cl_prev = p;
    HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->cl_mat), D * 3 * sizeof(float)));
    HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->cl_red), (kClosureBlocks + 64) * sizeof(float)));
    HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->cl_flag), 64 * sizeof(int)));
    HIPCHK(c, hipMemset(c->cl_flag, 0, 64 * sizeof(int)));
  }
  if (!c->cl_mat_valid) {
    // per-coefficient material features: log eps, log mu, c / (1 + c) with
    // the conductivity number c = sigma dt / (4 eps) of the trapezoidal rule
    std::vector<float> f(D * 3);
    for (size_t i = 0; i < D; ++i) {
      const double cc = c->sig[i] * c->dt / (4.0 * c->eps[i]);
      f[i * 3 + 0] = float(std::log(c->eps[i]));
      f[i * 3 + 1] = float(std::log(c->mu[i]));
      f[i * 3 + 2] = float(cc / (1.0 + cc));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->cl_mat, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
    c->cl_mat_valid = true;
  }
  return ADI_OK;
}

float* cl_scale(adi_ctx* c) { return c->cl_red + kClosureBlocks; }

hipError_t enqueue_mark(adi_ctx* c) {
  return hipMemcpyAsync(c->cl_prev, c->B[0], 6 * c->D * c->esz, hipMemcpyDeviceToDevice, c->stream);
}

// scale = RMS of the state; x = features of (state, cl_prev, material, source)
// (float32, or the network's packed bf16 input)
template <typename O>
hipError_t enqueue_features(adi_ctx* c, O* x, float* scale) {
  hipError_t e;
  if (c->esz == 8) {
    const double* st = static_cast<const double*>(c->B[0]);
    e = nn::launch_state_scale<double>(st, 6 * c->D, c->cl_red, kClosureBlocks, scale, c->stream);
    if (e == hipSuccess)
      e = nn::launch_features(st, static_cast<const double*>(c->cl_prev), c->cl_mat, c->n, scale,
                              c->src, c->d_t, c->dt, x, c->stream);
  } else {
    const float* st = static_cast<const float*>(c->B[0]);
    e = nn::launch_state_scale<float>(st, 6 * c->D, c->cl_red, kClosureBlocks, scale, c->stream);
    if (e == hipSuccess)
      e = nn::launch_features(st, static_cast<const float*>(c->cl_prev), c->cl_mat, c->n, scale,
                              c->src, c->d_t, c->dt, x, c->stream);
  }
  return e;
}

hipError_t enqueue_apply(adi_ctx* c, const float* y, const float* scale, const int* flag) {
  if (c->esz == 8)
    return nn::launch_apply<double>(static_cast<double*>(c->B[0]), c->n, y, scale, flag, c->stream);
  return nn::launch_apply<float>(static_cast<float*>(c->B[0]), c->n, y, scale, flag, c->stream);
}

}  // namespace

extern "C" {

int adi_copy_state(adi_ctx* dst, const adi_ctx* src) {
  if (!dst || !src) return ADI_EINVAL;
  if (dst->ns[0] != src->ns[0] || dst->ns[1] != src->ns[1] || dst->ns[2] != src->ns[2])
    return fail(dst, ADI_EINVAL, "grids differ");
  if (!src->ws) return fail(dst, ADI_ESTATE, "source has no state");
  if (!dst->ws) {
    int st = ensure_workspace(dst);
    if (st != ADI_OK) return st;
  }
  if (src->stream != dst->stream) HIPCHK(dst, hipStreamSynchronize(src->stream));
  const size_t count = 6 * dst->D;
  if (dst->esz == src->esz) {
    HIPCHK(dst, hipMemcpyAsync(dst->B[0], src->B[0], count * dst->esz, hipMemcpyDeviceToDevice,
                               dst->stream));
  } else {
    HIPCHK(dst, launch_convert<float>(src->B[0], dst->B[0], count, src->esz == 8 ? 0 : 1,
                                      dst->stream));
  }
  HIPCHK(dst, hipMemcpyAsync(dst->d_t, src->d_t, 8, hipMemcpyDeviceToDevice, dst->stream));
  dst->t = src->t;
  return ADI_OK;
}

int adi_closure_mark(adi_ctx* c) {
  if (!c) return ADI_EINVAL;
  int st = closure_ready(c);
  if (st != ADI_OK) return st;
  HIPCHK(c, enqueue_mark(c));
  c->cl_marked = true;
  return ADI_OK;
}

int adi_closure_features(adi_ctx* c, float* x_dev, float* scale_dev) {
  if (!c || !x_dev || !scale_dev) return ADI_EINVAL;
  int st = closure_ready(c);
  if (st != ADI_OK) return st;
  if (!c->cl_marked) return fail(c, ADI_ESTATE, "adi_closure_mark first");
  HIPCHK(c, enqueue_features(c, x_dev, scale_dev));
  return ADI_OK;
}

int adi_closure_target(adi_ctx* fine, adi_ctx* coarse, const float* scale_dev, float* t_dev) {
  if (!fine || !coarse || !scale_dev || !t_dev) return ADI_EINVAL;
  if (fine->ns[0] != coarse->ns[0] || fine->ns[1] != coarse->ns[1] ||
      fine->ns[2] != coarse->ns[2] || !fine->ws || !coarse->ws)
    return fail(coarse, ADI_EINVAL, "grids differ or no state");
  if (fine->esz != coarse->esz) return fail(coarse, ADI_EINVAL, "precisions differ");
  if (fine->stream != coarse->stream) HIPCHK(coarse, hipStreamSynchronize(fine->stream));
  if (coarse->esz == 8)
    HIPCHK(coarse, nn::launch_target<double>(static_cast<const double*>(fine->B[0]),
                                             static_cast<const double*>(coarse->B[0]), coarse->D,
                                             scale_dev, t_dev, coarse->stream));
  else
    HIPCHK(coarse, nn::launch_target<float>(static_cast<const float*>(fine->B[0]),
                                            static_cast<const float*>(coarse->B[0]), coarse->D,
                                            scale_dev, t_dev, coarse->stream));
  return ADI_OK;
}

int adi_closure_apply(adi_ctx* c, const float* y_dev, const float* scale_dev) {
  if (!c || !y_dev || !scale_dev) return ADI_EINVAL;
  if (c->ns[0] != c->ns[1] || c->ns[0] != c->ns[2])
    return fail(c, ADI_EINVAL, "the learned closure needs a cubic patch (nx = ny = nz)");
  if (!c->ws) return fail(c, ADI_ESTATE, "no state");
  HIPCHK(c, enqueue_apply(c, y_dev, scale_dev, nullptr));
  return ADI_OK;
}

int adi_step_closure(adi_ctx* c, adi_nn* nn_, int nsteps, float gate) {
  if (!c || !nn_ || nsteps < 0) return ADI_EINVAL;
  if (!c->factored || !c->exec) return fail(c, ADI_ESTATE, "adi_factor must succeed first");
  if (nn::closure_cin(nn_) != nn::kFeatures || nn::closure_cout(nn_) != nn::kOutputs)
    return fail(c, ADI_EINVAL, "network must map 16 features to 6 corrections");
  int st = closure_ready(c);
  if (st != ADI_OK) return st;
  const int n = c->n;
  float *x = nullptr, *y = nullptr, *scale = nullptr, *partial = nullptr;
  st = nn::closure_buffers(nn_, n, n, n, &x, &y, &scale, &partial);
  if (st != ADI_OK) return fail(c, st, "network buffers");
  for (int i = 0; i < nsteps; ++i) {
    HIPCHK(c, enqueue_mark(c));
    HIPCHK(c, hipGraphLaunch(c->exec, c->stream));
    HIPCHK(c, enqueue_features(c, nn::closure_input16(nn_), scale));
    st = nn::closure_forward_packed(nn_, y, n, n, n, c->stream);
    if (st != ADI_OK) return fail(c, st, "network forward");
    const int* flag = nullptr;
    if (gate > 0.f) {
      const size_t count = c->D * nn::kOutputs;
      if (c->esz == 8)
        HIPCHK(c, nn::launch_gate<double>(y, static_cast<const double*>(c->B[0]),
                                          static_cast<const double*>(c->cl_prev), count, partial,
                                          kClosureBlocks, scale, gate, c->cl_flag, c->cl_flag + 1,
                                          c->stream));
      else
        HIPCHK(c, nn::launch_gate<float>(y, static_cast<const float*>(c->B[0]),
                                         static_cast<const float*>(c->cl_prev), count, partial,
                                         kClosureBlocks, scale, gate, c->cl_flag, c->cl_flag + 1,
                                         c->stream));
      flag = c->cl_flag;
    }
    HIPCHK(c, enqueue_apply(c, y, scale, flag));
  }
  c->cl_marked = true;
  c->t += nsteps * c->dt;
  return ADI_OK;
}

int adi_closure_rejected(adi_ctx* c, int* count) {
  if (!c || !count) return ADI_EINVAL;
  *count = 0;
  if (!c->cl_flag) return ADI_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(count, c->cl_flag + 1, sizeof(int), hipMemcpyDeviceToHost));
  return ADI_OK;
}

}  // extern "C"

// ------------------------------------------------ manufactured solution
namespace {

// Gauss tables of the q-point rule on every element, axis after axis
// (x, y, z): for axis a with Q_a = N_a q points, coordinates x[Q_a],
// weights w[Q_a], then the p + 1 basis values bv[Q_a][p+1] and derivatives
// bd[Q_a][p+1] of each point's element.
size_t mms_table_size(const int* Ns, int p, int q) {
  return size_t(Ns[0] + Ns[1] + Ns[2]) * q * (2 + 2 * (p + 1));
}

void mms_host_tables(const int* Ns, int p, int q, std::vector<double>& tab) {
  std::vector<double> gx, gw;
  gauss_legendre(q, gx, gw);
  tab.assign(mms_table_size(Ns, p, q), 0.0);
  double* base = tab.data();
  std::vector<double> v(p + 1), d(p + 1);
  for (int ax = 0; ax < 3; ++ax) {
    const int N = Ns[ax], Q = N * q;
    const std::vector<double> t = open_knots(N, p);
    double* X = base;
    double* Wt = X + Q;
    double* BV = Wt + Q;
    double* BD = BV + size_t(Q) * (p + 1);
    for (int e = 0; e < N; ++e)
      for (int g = 0; g < q; ++g) {
        const int a = e * q + g;
        X[a] = (e + 0.5 * (gx[g] + 1.0)) / N;
        Wt[a] = 0.5 * gw[g] / N;
        basis_on_span(t, p, e + p, X[a], v.data(), d.data());
        for (int r = 0; r <= p; ++r) {
          BV[size_t(a) * (p + 1) + r] = v[r];
          BD[size_t(a) * (p + 1) + r] = d[r];
        }
      }
    base += size_t(Q) * (2 + 2 * (p + 1));
  }
}

// The device tables of mms_host_tables at `base`.
mms::Tables tables_at(const double* base, const int* Ns, int p, int q) {
  mms::Tables tb{};
  for (int ax = 0; ax < 3; ++ax) {
    const int Q = Ns[ax] * q;
    tb.x[ax] = base;
    tb.w[ax] = base + Q;
    tb.bv[ax] = base + 2 * Q;
    tb.bd[ax] = base + 2 * Q + size_t(Q) * (p + 1);
    tb.N[ax] = Ns[ax];
    base += size_t(Q) * (2 + 2 * (p + 1));
  }
  tb.p = p;
  tb.q = q;
  return tb;
}

size_t quad_points(const adi_ctx* c, int q) {
  return size_t(c->Ns[0]) * q * size_t(c->Ns[1]) * q * size_t(c->Ns[2]) * q;
}

// Tables on the device, and the buffers of the projection and errors
// (allocated on first use and whenever q changes).
int mms_ready(adi_ctx* c, int q) {
  if (q < 1 || q > 16) return fail(c, ADI_EINVAL, "quadrature points per element must be 1..16");
  if (c->mms_q == q) return ADI_OK;
  std::vector<double> tab;
  mms_host_tables(c->Ns, c->p, q, tab);
  if (c->mms_tab) hipFree(c->mms_tab);
  if (c->mms_vals) hipFree(c->mms_vals);
  c->mms_tab = nullptr;
  c->mms_vals = nullptr;
  c->mms_q = 0;
  HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->mms_tab), tab.size() * 8));
  HIPCHK(c, hipMemcpy(c->mms_tab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->mms_vals), 6 * quad_points(c, q) * 8));
  if (!c->mms_part)
    HIPCHK(c, hipMalloc(reinterpret_cast<void**>(&c->mms_part), mms::kMaxErrorBlocks * 4 * 8));
  c->mms_q = q;
  return ADI_OK;
}

mms::Tables mms_tables(const adi_ctx* c) { return tables_at(c->mms_tab, c->Ns, c->p, c->mms_q); }

// Sum the per-block partial sums of the error kernel (in block order) into
// out: ||E_h - E||, its H(curl) norm, the same for H.
void errors_from_partials(const std::vector<double>& part, int nblk, double* out) {
  double sum[4] = {0, 0, 0, 0};
  for (int b = 0; b < nblk; ++b)
    for (int k = 0; k < 4; ++k) sum[k] += part[size_t(b) * 4 + k];
  out[0] = std::sqrt(sum[0]);
  out[1] = std::sqrt(sum[0] + sum[1]);
  out[2] = std::sqrt(sum[2]);
  out[3] = std::sqrt(sum[2] + sum[3]);
}

// (M (x) M (x) M)^-1 on the three components of buf (E or H boundary rows).
template <typename T>
hipError_t enqueue_mass_solves(adi_ctx* c, int kindH, void* buf, hipStream_t s) {
  for (int ax = 0; ax < 3; ++ax) {
    SweepArgs w{};
    for (int ci = 0; ci < 3; ++ci) {
      void* io = comp(buf, ci, c);
      const int v = dirichlet(kindH, ci, ax) ? 1 : 0;
      SweepDesc& d = w.d[ci];
      d.axis = ax;
      d.in = io;
      d.out = io;
      d.L = c->shL[ax][v];
      d.U = c->shU[ax][v];
      d.D = c->shD[ax][v];
      d.spk = c->spike_ok[ax] ? c->spk[ax][v] : nullptr;
      d.segs = spike_segments(c->ns[ax]);
      d.modified = 0;
    }
    for (int k = 0; k < 3; ++k) w.dim[k] = c->ns[k];
    w.xaxis = ax == 0;
    w.spike = spike_for(w, 3);
    hipError_t e = launch_sweep<T>(c->p, 3, w, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// State = L2 projection of the six component fields held at the Gauss points
// in c->mms_vals (projection right-hand sides, then mass solves), time t.
int project_from_vals(adi_ctx* c, double t, hipStream_t s) {
  const mms::Tables tb = mms_tables(c);
  hipError_t e;
  if (c->esz == 8) {
    e = mms::launch_project_rhs<double>(tb, c->mms_vals, static_cast<double*>(c->B[0]), s);
    if (e == hipSuccess) e = enqueue_mass_solves<double>(c, 0, c->B[0], s);
    if (e == hipSuccess) e = enqueue_mass_solves<double>(c, 1, c->B[1], s);
  } else {
    e = mms::launch_project_rhs<float>(tb, c->mms_vals, static_cast<float*>(c->B[0]), s);
    if (e == hipSuccess) e = enqueue_mass_solves<float>(c, 0, c->B[0], s);
    if (e == hipSuccess) e = enqueue_mass_solves<float>(c, 1, c->B[1], s);
  }
  HIPCHK(c, e);
  HIPCHK(c, hipMemcpyAsync(c->d_t, &t, 8, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipStreamSynchronize(s));
  c->t = t;
  return ADI_OK;
}

}  // namespace

extern "C" {

int adi_mms_project(adi_ctx* c, int q, double t) {
  if (!c || !std::isfinite(t)) return ADI_EINVAL;
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor first");
  int st = mms_ready(c, q);
  if (st != ADI_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, mms::launch_exact(mms_tables(c), t, c->mms_vals, c->cap));
  return project_from_vals(c, t, c->cap);
}

int adi_project(adi_ctx* c, const double* vals_qp, int q, double t) {
  if (!c || !vals_qp || !std::isfinite(t)) return ADI_EINVAL;
  if (!c->factored) return fail(c, ADI_ESTATE, "adi_factor first");
  int st = mms_ready(c, q);
  if (st != ADI_OK) return st;
  const size_t count = 6 * quad_points(c, q);
  if (!finite_all(vals_qp, count)) return fail(c, ADI_ENONFINITE, "value not finite");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->mms_vals, vals_qp, count * 8, hipMemcpyHostToDevice));
  return project_from_vals(c, t, c->cap);
}

int adi_mms_errors(adi_ctx* c, int q, double* out) {
  if (!c || !out) return ADI_EINVAL;
  if (!c->ws) return fail(c, ADI_ESTATE, "no state");
  int st = mms_ready(c, q);
  if (st != ADI_OK) return st;
  const mms::Tables tb = mms_tables(c);
  int nblk = 0;
  HIPCHK(c, c->esz == 8
                ? mms::launch_errors<double>(tb, static_cast<const double*>(c->B[0]), c->t,
                                             c->mms_part, &nblk, c->stream)
                : mms::launch_errors<float>(tb, static_cast<const float*>(c->B[0]), c->t,
                                            c->mms_part, &nblk, c->stream));
  std::vector<double> part(size_t(nblk) * 4);
  HIPCHK(c, hipMemcpyAsync(part.data(), c->mms_part, part.size() * 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  errors_from_partials(part, nblk, out);
  return ADI_OK;
}

int adi_mms_errors_noalloc(adi_ctx* c, int q, double* out) {
  if (!c || !out) return ADI_EINVAL;
  if (q < 1 || q > 16) return fail(c, ADI_EINVAL, "quadrature points per element must be 1..16");
  const size_t ntab = mms_table_size(c->Ns, c->p, q);
  const size_t part_off = (ntab + 31) / 32 * 32;  // partials 256-byte aligned
  if ((part_off + size_t(mms::kMaxErrorBlocks) * 4) * 8 > mms::kNoAllocScratchBytes)
    return fail(c, ADI_ENOMEM, "quadrature tables and partial sums exceed the fixed scratch");
  if (!c->ws) return fail(c, ADI_ESTATE, "no state");
  double* scr = nullptr;  // this GPU's copy of the library's fixed device array
  HIPCHK(c, mms::noalloc_scratch(&scr));
  std::vector<double> tab;
  mms_host_tables(c->Ns, c->p, q, tab);
  HIPCHK(c, hipMemcpyAsync(scr, tab.data(), ntab * 8, hipMemcpyHostToDevice, c->stream));
  const mms::Tables tb = tables_at(scr, c->Ns, c->p, q);
  double* partial = scr + part_off;
  int nblk = 0;
  HIPCHK(c, c->esz == 8
                ? mms::launch_errors<double>(tb, static_cast<const double*>(c->B[0]), c->t,
                                             partial, &nblk, c->stream)
                : mms::launch_errors<float>(tb, static_cast<const float*>(c->B[0]), c->t,
                                            partial, &nblk, c->stream));
  std::vector<double> part(size_t(nblk) * 4);
  HIPCHK(c, hipMemcpyAsync(part.data(), partial, part.size() * 8, hipMemcpyDeviceToHost,
                           c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));  // also keeps `tab` alive until its copy is done
  errors_from_partials(part, nblk, out);
  return ADI_OK;
}

}  // extern "C"
