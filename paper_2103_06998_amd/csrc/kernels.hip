// gfx950 kernels of the ADI step: right-hand-side assembly, banded line
// sweeps and the per-line float64 factorisation of material-modified rows.
//
// Data layout: every field component is an n^3 array, x fastest ([z][y][x]),
// the paper's reordering of a right-hand side into N_x-long rows.
#include "adimx_internal.h"

#include <algorithm>
#include <type_traits>
#include <utility>

namespace adimx {

namespace {

// ------------------------------------------------------------ term tables
// One sum-factorised term of a right-hand side: output component `out`,
// coefficient group `grp`, sign, input field, and the 1D operators acting on
// x, y and z (0 = M mass, 1 = A trial derivative, 2 = B = A^T test
// derivative, 3 = S stiffness).  Each output value is
//   sum_g coef_g[row] * sum_{terms in g} sign * (X (x) Y (x) Z) field.
struct Term {
  int out, grp, sign, field, x, y, z;
};
constexpr int OM = 0, OA = 1, OB = 2, OS = 3;

// Stage kinds and their tables.
//  E stages (fields E1,E2,E3,H1,H2,H3; groups gamma, beta, alpha):
//    discrete1 / dupa1ab: RE1 = g MMM E1 + b (MAM H3 - MMA H2) + a ABM E2, ...
//    discrete3:           alpha terms AMB E3, BAM E1, MBA E2.
//  E increment stages (groups gamma - 1, beta, alpha): the same terms minus
//    the row-scaled system matrix applied to the old E_c, i.e. b - P E with
//    P = MMM + alpha (S on the modified axis); the MMM part folds into the
//    group coefficient gamma - 1, the stiffness part is one more term:
//    substep 1: - a MSM E1, - a MMS E2, - a SMM E3; substep 2: - a MMS E1,
//    - a SMM E2, - a MSM E3.
//  H stages (fields H1..3, E_old1..3, E_new1..3; groups 1, delta):
//    discrete2: RH1 = MMM H1 - d MAM E3 + d MMA E2', ...
//    discrete4: RH1 = MMM H1 + d MMA E2' - d MAM E3'', ... (sign of scheme1d)
//  H increment stages: the delta terms alone (b - MMM H).
template <int STAGE>
struct StageInfo;
template <> struct StageInfo<kStageE1> { static constexpr int NT = 12, NG = 3; };
template <> struct StageInfo<kStageE2> { static constexpr int NT = 12, NG = 3; };
template <> struct StageInfo<kStageEd1> { static constexpr int NT = 15, NG = 3; };
template <> struct StageInfo<kStageEd2> { static constexpr int NT = 15, NG = 3; };
template <> struct StageInfo<kStageH1> { static constexpr int NT = 9, NG = 2; };
template <> struct StageInfo<kStageH2> { static constexpr int NT = 9, NG = 2; };
template <> struct StageInfo<kStageHd1> { static constexpr int NT = 6, NG = 2; };
template <> struct StageInfo<kStageHd2> { static constexpr int NT = 6, NG = 2; };

template <int STAGE>
constexpr bool is_h_stage() {
  return STAGE == kStageH1 || STAGE == kStageH2 || STAGE == kStageHd1 || STAGE == kStageHd2;
}

template <int STAGE>
__host__ __device__ constexpr Term get_term(int i) {
  constexpr Term curl_and_mass[9] = {
      {0, 0, +1, 0, OM, OM, OM}, {0, 1, +1, 5, OM, OA, OM}, {0, 1, -1, 4, OM, OM, OA},
      {1, 0, +1, 1, OM, OM, OM}, {1, 1, +1, 3, OM, OM, OA}, {1, 1, -1, 5, OA, OM, OM},
      {2, 0, +1, 2, OM, OM, OM}, {2, 1, +1, 4, OA, OM, OM}, {2, 1, -1, 3, OM, OA, OM}};
  constexpr Term r_sub1[3] = {{0, 2, +1, 1, OA, OB, OM}, {1, 2, +1, 2, OM, OA, OB},
                              {2, 2, +1, 0, OB, OM, OA}};
  constexpr Term r_sub2[3] = {{0, 2, +1, 2, OA, OM, OB}, {1, 2, +1, 0, OB, OA, OM},
                              {2, 2, +1, 1, OM, OB, OA}};
  // stiffness part of P E_c on the modified axis (substep 1: E1 y, E2 z,
  // E3 x; substep 2: E1 z, E2 x, E3 y)
  constexpr Term s_sub1[3] = {{0, 2, -1, 0, OM, OS, OM}, {1, 2, -1, 1, OM, OM, OS},
                              {2, 2, -1, 2, OS, OM, OM}};
  constexpr Term s_sub2[3] = {{0, 2, -1, 0, OM, OM, OS}, {1, 2, -1, 1, OS, OM, OM},
                              {2, 2, -1, 2, OM, OS, OM}};
  constexpr Term h_sub1[9] = {
      {0, 0, +1, 0, OM, OM, OM}, {0, 1, -1, 5, OM, OA, OM}, {0, 1, +1, 7, OM, OM, OA},
      {1, 0, +1, 1, OM, OM, OM}, {1, 1, -1, 3, OM, OM, OA}, {1, 1, +1, 8, OA, OM, OM},
      {2, 0, +1, 2, OM, OM, OM}, {2, 1, -1, 4, OA, OM, OM}, {2, 1, +1, 6, OM, OA, OM}};
  constexpr Term h_sub2[9] = {
      {0, 0, +1, 0, OM, OM, OM}, {0, 1, +1, 4, OM, OM, OA}, {0, 1, -1, 8, OM, OA, OM},
      {1, 0, +1, 1, OM, OM, OM}, {1, 1, +1, 5, OA, OM, OM}, {1, 1, -1, 6, OM, OM, OA},
      {2, 0, +1, 2, OM, OM, OM}, {2, 1, +1, 3, OM, OA, OM}, {2, 1, -1, 7, OA, OM, OM}};
  if (STAGE == kStageH1) return h_sub1[i];
  if (STAGE == kStageH2) return h_sub2[i];
  if (STAGE == kStageHd1) return h_sub1[i + 1 + i / 2];  // the two delta terms of each output
  if (STAGE == kStageHd2) return h_sub2[i + 1 + i / 2];
  if (i < 9) return curl_and_mass[i];
  constexpr bool sub2 = STAGE == kStageE2 || STAGE == kStageEd2;
  if (i < 12) return sub2 ? r_sub2[i - 9] : r_sub1[i - 9];
  return sub2 ? s_sub2[i - 12] : s_sub1[i - 12];
}

// Per output component: the input fields it reads (local slots) and its
// distinct (field, y-operator) pairs, each applied once per plane.  The y
// pass gives each field slot one wave, which applies the pairs of that
// field (at most two) to the same loaded column values.
struct CompTab {
  int nf[3] = {};           // fields read by component c
  int field[3][8] = {};     // slot -> field index
  int np[3] = {};           // pairs of component c
  int pslot[3][16] = {};    // pair -> field slot
  int pyop[3][16] = {};     // pair -> y operator
  int nsp[3][8] = {};       // slot -> number of its pairs
  int spair[3][8][2] = {};  // slot -> its pairs
  int term_pair[24] = {};   // term -> pair index within its component
  int maxnf = 0, maxnp = 0, maxsp = 0;
};

template <int STAGE>
constexpr CompTab make_comp_tab() {
  CompTab t{};
  for (int i = 0; i < StageInfo<STAGE>::NT; ++i) {
    const Term tm = get_term<STAGE>(i);
    const int c = tm.out;
    int slot = -1;
    for (int k = 0; k < t.nf[c]; ++k)
      if (t.field[c][k] == tm.field) slot = k;
    if (slot < 0) {
      slot = t.nf[c]++;
      t.field[c][slot] = tm.field;
    }
    int pr = -1;
    for (int k = 0; k < t.np[c]; ++k)
      if (t.pslot[c][k] == slot && t.pyop[c][k] == tm.y) pr = k;
    if (pr < 0) {
      pr = t.np[c]++;
      t.pslot[c][pr] = slot;
      t.pyop[c][pr] = tm.y;
      t.spair[c][slot][t.nsp[c][slot]++] = pr;
    }
    t.term_pair[i] = pr;
  }
  for (int c = 0; c < 3; ++c) {
    t.maxnf = t.nf[c] > t.maxnf ? t.nf[c] : t.maxnf;
    t.maxnp = t.np[c] > t.maxnp ? t.np[c] : t.maxnp;
    for (int k = 0; k < t.nf[c]; ++k) t.maxsp = t.nsp[c][k] > t.maxsp ? t.nsp[c][k] : t.maxsp;
  }
  return t;
}

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// A value the same in every lane of the wave, held in scalar registers.
template <typename T>
__device__ __forceinline__ T wave_uniform(T v) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
  } else {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(unsigned(u))));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(unsigned(u >> 32))));
    return __builtin_bit_cast(T, (static_cast<unsigned long long>(hi) << 32) | lo);
  }
}

constexpr int kTX = 32, kTY = 8, kCols = kTX * kTY;
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, one L2 each
constexpr int kRhsThreads = kCols;  // one block per (tile, output component)

// LDS of one RHS block: y-pass results (two buffers), the y band rows of
// the tile and the z weights of the chunk's input planes.
template <typename TC, int P, int STAGE>
size_t rhs_lds_bytes(int zchunk) {
  constexpr int HX = kTX + 2 * P, W = 2 * P + 1;
  constexpr CompTab CT = make_comp_tab<STAGE>();
  return sizeof(TC) * (2 * size_t(CT.maxnp) * kTY * HX + size_t(4) * kTY * W +
                       size_t(zchunk + 2 * P) * 4 * W);
}

// ------------------------------------------------------------ RHS kernel
// Block = one output component of a kTX x kTY tile of (x, y) output columns
// and a chunk of z planes, mapped so that the three components of a tile and
// its x neighbours run on one XCD and share their inputs in its L2.  Input
// planes are marched along z.  The y operators are applied by one wave per
// (field, operator) pair of the component: lane = x column of the tile with
// its p-halo, holding the 2p + kTY values of its column (loaded straight
// from global memory two planes ahead) and producing kTY values into
// LDS (double buffered, so one barrier per plane suffices).  The x operators
// are then applied per output column with the thread's band rows in
// registers, and each result is scattered into a register queue of 2p+1
// pending output planes with the z operator's weights.  When the oldest
// pending plane is complete it is scaled by the per-row coefficients and
// written.  TI: input type, TC: arithmetic type, TO: output type, TK:
// coefficient type.
// One block's work: the tile (bx, by), z chunk bz of output component
// COMP, or of comp_rt when COMP < 0.  With a compile-time component its
// terms, field slots and boundary rule are fixed in the code and no term is
// skipped by a branch, which lets the compiler batch the LDS reads of all
// its terms: float32 arithmetic takes that form (E right-hand side 136 ->
// 126 us at 128^3 p=3), and so does float64 arithmetic up to p = 2 (the
// 256^3 p=2 step: 4.22 -> 4.13 ms in the float32 mode).  In float64
// arithmetic at p >= 3 the batched reads need more registers than there are
// and the kernel slows down (128^3 p=3: 150 -> 218 us), so it keeps the
// runtime component.
template <typename TI, typename TC, typename TO, typename TK, int P, int STAGE, int COMP>
__device__ __forceinline__ void rhs_tile(const RhsArgs<TC>& a, const TC* __restrict__ bandx,
                                         const TC* __restrict__ bandy,
                                         const TC* __restrict__ zw, int bx, int by, int bz,
                                         int comp_rt) {
  const int comp = COMP >= 0 ? COMP : comp_rt;
  constexpr int W = 2 * P + 1, HX = kTX + 2 * P, HY = kTY + 2 * P;
  constexpr int NT = StageInfo<STAGE>::NT, NG = StageInfo<STAGE>::NG;
  constexpr CompTab CT = make_comp_tab<STAGE>();
  constexpr bool kE = !is_h_stage<STAGE>();
  constexpr int NWAVES = kRhsThreads / 64;
  static_assert(CT.maxnf <= NWAVES, "one field per wave in the y pass");
  static_assert(CT.maxsp <= 2, "at most two y operators per field");
  static_assert(HX <= 64, "one lane per x column in the y pass");
  constexpr int GSZ = CT.maxnp * kTY * HX;  // one y-pass buffer
  constexpr int NCF = kE ? 3 : 1;           // per-row coefficients of an output

  extern __shared__ __align__(16) unsigned char smem[];
  TC* sG = reinterpret_cast<TC*>(smem);  // [2][pair][yy][x]
  TC* sYB = sG + 2 * GSZ;                // y band rows [op][yy][d] of the tile
  TC* sZW = sYB + 4 * kTY * W;           // z weights [plane - kbeg][op][q]

  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t plane = size_t(nx) * ny;
  const int tid = threadIdx.x;
  const int wave = tid / 64, lane = tid % 64;
  const int tx = tid % kTX, ty = tid / kTX;
  const int i0 = bx * kTX, j0 = by * kTY;
  const int t0 = bz * a.zchunk;
  const int t1 = min(nz, t0 + a.zchunk);
  const int i = i0 + tx, j = j0 + ty;

  // x band rows of this thread's output column (registers)
  TC xb[4][W];
#pragma unroll
  for (int op = 0; op < 4; ++op)
#pragma unroll
    for (int d = 0; d < W; ++d) xb[op][d] = (i < nx) ? bandx[(size_t(op) * nx + i) * W + d] : TC(0);

  // y band rows of the tile and z weights of the chunk's input planes (read
  // by every lane: LDS broadcasts instead of scalar loads in the plane loop)
  const int kbeg = max(t0 - P, 0), kend = min(t1 + P, nz);  // input planes to read
  for (int idx = tid; idx < 4 * kTY * W; idx += kRhsThreads) {
    const int op = idx / (kTY * W), rem = idx % (kTY * W), yy = rem / W, d = rem % W;
    sYB[idx] = bandy[(size_t(op) * ny + min(j0 + yy, ny - 1)) * W + d];
  }
  // (four loads of a thread in flight before their LDS writes: one
  // load-then-store round trip per value had delayed the plane loop's start)
  {
    const int nzw = (kend - kbeg) * 4 * W;
    for (int base = tid; base < nzw; base += 4 * kRhsThreads) {
      TC v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int idx = min(base + u * kRhsThreads, nzw - 1);
        const int kk = idx / (4 * W), rem = idx % (4 * W), op = rem / W, q = rem % W;
        v[u] = zw[(size_t(op) * nz + kbeg + kk) * W + q];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (base + u * kRhsThreads < nzw) sZW[base + u * kRhsThreads] = v[u];
    }
  }

  // This wave's field slot (its one or two y operators) and this lane's
  // column x = i0 - P + lane, rows y = j0 - P + m (m < HY).  Every global
  // load in the plane loop is issued unconditionally: columns and rows
  // outside the grid are clamped to its edge (their band weights are zero,
  // so the values read there never contribute), a wave without a field reads
  // a single address, and planes past the chunk re-read its last one.  With
  // no load skipped by a branch the compiler counts the loads in flight
  // exactly, and each wait for a plane or a coefficient leaves the younger
  // prefetches in flight.
  const bool on = wave < CT.nf[comp];
  const int slot = on ? wave : 0;
  const int nsp = on ? CT.nsp[comp][slot] : 0;  // pairs of this wave's field
  const int pr0 = CT.spair[comp][slot][0], pr1 = CT.spair[comp][slot][1];
  const int yop0 = CT.pyop[comp][pr0], yop1 = CT.pyop[comp][pr1];
  // A tile whose output rows all have the band rows of row yrep (interior
  // rows of uniform knots) takes the wave's y weights from scalar registers
  // instead of reading 8 band rows per operator from LDS on every plane.
  const bool yin = j0 >= a.yin0 && j0 + kTY - 1 <= a.yin1;
  TC wy0[W], wy1[W];
#pragma unroll
  for (int d = 0; d < W; ++d) {
    wy0[d] = wave_uniform(bandy[(size_t(wave_uniform(yop0)) * ny + a.yrep) * W + d]);
    wy1[d] = wave_uniform(bandy[(size_t(wave_uniform(yop1)) * ny + a.yrep) * W + d]);
  }
  // Addresses are a block-uniform row or plane pointer plus a 32-bit lane
  // offset (nx ny < 2^31), which keeps one offset register per lane.
  const TI* fsrc = static_cast<const TI*>(a.f[CT.field[comp][slot]]);
  const unsigned loff = on ? unsigned(min(max(i0 - P + lane, 0), nx - 1)) : 0u;
  const size_t pstride = on ? plane : 0;
  int rows[HY];
#pragma unroll
  for (int m = 0; m < HY; ++m) rows[m] = on ? min(max(j0 - P + m, 0), ny - 1) * nx : 0;
  auto load_plane = [&](int k, TI (&v)[HY]) {
    const TI* pp = fsrc + pstride * size_t(min(k, kend - 1));
#pragma unroll
    for (int m = 0; m < HY; ++m) v[m] = (pp + rows[m])[loff];
  };
  // per-row coefficients of output plane te (clamped; used only when written)
  const unsigned colo = unsigned(min(i, nx - 1)) + unsigned(nx) * unsigned(min(j, ny - 1));
  auto load_cf = [&](int te, TC (&c)[NCF]) {
    const size_t po = plane * size_t(min(max(te, 0), nz - 1));
#pragma unroll
    for (int q = 0; q < NCF; ++q) c[q] = TC((static_cast<const TK*>(a.coef[q]) + po)[colo]);
  };

  TC acc[NG][W];
#pragma unroll
  for (int g = 0; g < NG; ++g)
#pragma unroll
    for (int q = 0; q < W; ++q) acc[g][q] = TC(0);

  // source value at the midpoint of the substep times this column's x and y
  // basis values (zero for columns outside the source's support)
  double jsrc = 0.0;
  bool srccol = false;
  if (kE && a.src.comp == comp) {
    const int ri = i - a.src.first[0], rj = j - a.src.first[1];
    srccol = ri >= 0 && ri <= P && rj >= 0 && rj <= P;
    const double tm = *a.tnow + a.frac_dt;
    const double s = tm - a.src.t0;
    const double amp = a.src.amp * sin(2.0 * 3.14159265358979323846 * a.src.f0 * s) *
                       exp(-(s / a.src.width) * (s / a.src.width));
    if (srccol) jsrc = amp * a.src.by[rj] * a.src.bx[ri];
  }

  // write the complete output plane te (acc[.][0]) of this thread's column
  auto emit = [&](int te, const TC (&cf)[NCF]) {
    const unsigned o = unsigned(i) + unsigned(nx) * unsigned(j);
    const size_t po = plane * size_t(te);
    const bool bi = (i == 0 || i == nx - 1), bj = (j == 0 || j == ny - 1),
               bk = (te == 0 || te == nz - 1);
    if (kE) {
      const TC g = cf[0], b = cf[kE ? 1 : 0], al = cf[kE ? 2 : 0];
      TC v = g * acc[0][0] + b * acc[1][0] + al * acc[2 % NG][0];
      if (srccol) {
        const int rk = te - a.src.first[2];
        if (rk >= 0 && rk <= P) v -= b * TC(jsrc * a.src.bz[rk]);
      }
      // E_c is constrained on the faces normal to the two other axes
      const bool bnd = (comp == 0) ? (bj || bk) : (comp == 1) ? (bi || bk) : (bi || bj);
      (static_cast<TO*>(a.out[comp]) + po)[o] = bnd ? TO(0) : TO(v);
    } else {
      const TC v = acc[0][0] + cf[0] * acc[1][0];
      // H_c is constrained on the faces normal to axis c
      const bool bnd = (comp == 0) ? bi : (comp == 1) ? bj : bk;
      (static_cast<TO*>(a.out[comp]) + po)[o] = bnd ? TO(0) : TO(v);
    }
  };
  auto shift = [&]() {
#pragma unroll
    for (int g = 0; g < NG; ++g) {
#pragma unroll
      for (int q = 0; q < W - 1; ++q) acc[g][q] = acc[g][q + 1];
      acc[g][W - 1] = TC(0);
    }
  };
  const bool inplane = i < nx && j < ny;

  // Input plane k (kbeg <= k < kend) is held in ring slot (k - kbeg) & 1 and
  // its y-pass result in LDS buffer (k - kbeg) & 1; the loop is unrolled by
  // two so that both slots are static registers (no copies, which would wait
  // for the loads in flight).  Plane k + 2 is loaded into the slot as soon
  // as plane k has been consumed, and the coefficients of an output plane
  // one iteration before it is written.
  TI pre[2][HY];
  TC cfr[2][NCF];
  load_plane(kbeg, pre[0]);
  load_plane(kbeg + 1, pre[1]);
  load_cf(kbeg - P, cfr[0]);
  __syncthreads();  // band rows and z weights staged
  auto body = [&](auto sc, int k) {
    constexpr int S = decltype(sc)::value;
    const int te = k - P;
    load_cf(te + 1, cfr[S ^ 1]);
    TC* G = sG + S * GSZ;
    // y pass from registers: the wave's one or two y operators on its field
    if (on && lane < HX && yin) {
#pragma unroll
      for (int yy = 0; yy < kTY; ++yy) {
        TC s = TC(0);
#pragma unroll
        for (int d = 0; d < W; ++d) s += wy0[d] * TC(pre[S][yy + d]);
        G[(pr0 * kTY + yy) * HX + lane] = s;
      }
      if (CT.maxsp > 1 && nsp > 1) {  // wave-uniform
#pragma unroll
        for (int yy = 0; yy < kTY; ++yy) {
          TC s = TC(0);
#pragma unroll
          for (int d = 0; d < W; ++d) s += wy1[d] * TC(pre[S][yy + d]);
          G[(pr1 * kTY + yy) * HX + lane] = s;
        }
      }
    } else if (on && lane < HX) {
      const TC* yb0 = sYB + yop0 * kTY * W;
#pragma unroll
      for (int yy = 0; yy < kTY; ++yy) {
        TC s = TC(0);
#pragma unroll
        for (int d = 0; d < W; ++d) s += yb0[yy * W + d] * TC(pre[S][yy + d]);
        G[(pr0 * kTY + yy) * HX + lane] = s;
      }
      if (CT.maxsp > 1 && nsp > 1) {  // wave-uniform
        const TC* yb1 = sYB + yop1 * kTY * W;
#pragma unroll
        for (int yy = 0; yy < kTY; ++yy) {
          TC s = TC(0);
#pragma unroll
          for (int d = 0; d < W; ++d) s += yb1[yy * W + d] * TC(pre[S][yy + d]);
          G[(pr1 * kTY + yy) * HX + lane] = s;
        }
      }
    }
    load_plane(k + 2, pre[S]);
    __syncthreads();
    const TC* zk = sZW + (k - kbeg) * 4 * W;
    static_for<NT>([&](auto ic) {
      constexpr int it = decltype(ic)::value;
      constexpr Term tm = get_term<STAGE>(it);
      constexpr int tp = CT.term_pair[it];
      if (tm.out == comp) {
        TC v = TC(0);
#pragma unroll
        for (int d = 0; d < W; ++d) v += xb[tm.x][d] * G[(tp * kTY + ty) * HX + tx + d];
        if (tm.sign < 0) v = -v;
        const TC* zq = zk + tm.z * W;
#pragma unroll
        for (int q = 0; q < W; ++q) acc[tm.grp][q] += zq[q] * v;
      }
    });
    if (te >= t0 && te < t1 && inplane) emit(te, cfr[S]);
    shift();
  };
  int k = kbeg;
  for (; k + 1 < kend; k += 2) {
    body(std::integral_constant<int, 0>{}, k);
    body(std::integral_constant<int, 1>{}, k + 1);
  }
  if (k < kend) {
    body(std::integral_constant<int, 0>{}, k);
    ++k;
  }
  // output planes past the last input plane (top of the grid)
  for (; k < t1 + P; ++k) {
    const int te = k - P;
    if (te >= t0 && te < t1 && inplane) {
      TC c[NCF];
      load_cf(te, c);
      emit(te, c);
    }
    shift();
  }
}

template <typename TI, typename TC, typename TO, typename TK, int P, int STAGE>
__global__ __launch_bounds__(kRhsThreads) void rhs_kernel(RhsArgs<TC> a,
                                                          const TC* __restrict__ bandx,
                                                          const TC* __restrict__ bandy,
                                                          const TC* __restrict__ zw) {
  // Work item of this block.  Workgroups are dealt to the 8 XCDs (each with
  // its own L2) round robin by linear id; item w = ((zc * nty + ty) * ntx +
  // tx) * 3 + component is assigned so that each XCD runs a contiguous range
  // of items: the three components of a tile and its x neighbours share
  // their inputs in one L2.
  int comp, bx, by, bz;
  {
    const int ntx = gridDim.x / 3, nty = gridDim.y;
    const int total = gridDim.x * gridDim.y * gridDim.z;
    const int b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int xcd = b % kXcds, k = b / kXcds;
    const int q = total / kXcds, r = total % kXcds;
    int w = xcd * q + min(xcd, r) + k;
    comp = w % 3;
    w /= 3;
    bx = w % ntx;
    w /= ntx;
    by = w % nty;
    bz = w / nty;
  }
  if constexpr (sizeof(TC) == 4 || P <= 2) {
    if (comp == 0) rhs_tile<TI, TC, TO, TK, P, STAGE, 0>(a, bandx, bandy, zw, bx, by, bz, 0);
    else if (comp == 1) rhs_tile<TI, TC, TO, TK, P, STAGE, 1>(a, bandx, bandy, zw, bx, by, bz, 1);
    else rhs_tile<TI, TC, TO, TK, P, STAGE, 2>(a, bandx, bandy, zw, bx, by, bz, 2);
  } else {
    rhs_tile<TI, TC, TO, TK, P, STAGE, -1>(a, bandx, bandy, zw, bx, by, bz, comp);
  }
}

// Copy count values from global memory to LDS with NTH threads, eight loads
// in flight per thread.
template <typename T, int NTH>
__device__ __forceinline__ void stage_batched(T* dst, const T* __restrict__ src, int count,
                                              int tid) {
  constexpr int B = 8;
  for (int base = tid; base < count; base += NTH * B) {
    T v[B];
#pragma unroll
    for (int j = 0; j < B; ++j) v[j] = src[min(base + j * NTH, count - 1)];
#pragma unroll
    for (int j = 0; j < B; ++j)
      if (base + j * NTH < count) dst[base + j * NTH] = v[j];
  }
}

// ------------------------------------------------------------ sweeps
// One wave (64 lanes) solves 64 lines: lane = line.  The 64 x n tile is
// staged through LDS (row pitch 65 elements: conflict-free column access and
// transposed stores for x lines), the forward and backward substitutions run
// in LDS, and the tile is written back.  Lines along y and z are loaded with
// consecutive lanes on consecutive x (coalesced); lines along x are contiguous
// in memory and are transposed through LDS.
// rows per lane loaded together (float tiles: every row of a 64-row chunk in flight)
template <typename T>
struct SweepLoadRows { static constexpr int value = sizeof(T) == 8 ? 32 : 64; };
constexpr int kCH = 8;       // rows per compute chunk of the LDS part
// register slots of per-line factor chunks (float64: two, as its register
// rows leave no room for a third without spilling)
template <typename T, int P>
constexpr int fac_ring() { return sizeof(T) == 8 ? 2 : 3; }

// Rows of a line kept in registers (the rest in LDS): float64 tiles would
// limit a CU to two waves by LDS alone, so their first rows stay in
// registers (72 for shared factors; 40 for per-line factors, whose
// prefetch slots need the registers and whose launches have at most a few
// waves per CU); float32 tiles fit four waves per CU entirely in LDS.
template <typename T, bool MOD>
struct SweepRegRows { static constexpr int value = sizeof(T) == 8 ? (MOD ? 40 : 72) : 0; };

__host__ __device__ constexpr int sweep_pitch(bool xax) { return xax ? 65 : 64; }

// Rows of the LDS buffer: the LDS part of the lines, and for x lines also the
// transposition of the register part.
__host__ __device__ inline int sweep_buf_rows(int n, bool xax, int rr) {
  const int nlds = n > rr ? n - rr : 0;
  const int nreg = n < rr ? n : rr;
  return xax ? (nlds > nreg ? nlds : nreg) : nlds;
}

// One wave (64 lanes) solves 64 lines, lane = line.  Rows [0, kRR) of a line
// live in registers, rows [kRR, n) in an LDS column private to the lane.
// Lines along y and z are read with consecutive lanes on consecutive x
// (coalesced); lines along x are contiguous in memory and are transposed
// through LDS (row pitch 65: conflict-free transposed access), in two parts.
// Forward: y_r = b_r - sum_k L[r][k] y_{r-1-k}; backward:
// x_r = D_r y_r - sum_k DU[r][k] x_{r+1+k}, DU = D * U pre-scaled, so each row
// adds one dependent FMA.  Shared factors [r*P + k] / [r] are staged in LDS;
// per-line factors are read as [((l/64 * n + r) * P + k) * 64 + l%64].
template <typename T, int P, bool XAX, bool MOD>
__device__ __forceinline__ void sweep_body(const SweepArgs& a) {
  constexpr int kLoadCH = SweepLoadRows<T>::value;
  constexpr int PIT = sweep_pitch(XAX);
  constexpr int kRR = SweepRegRows<T, MOD>::value;
  constexpr int kRA = kRR > 0 ? kRR : 1;  // register array extent
  extern __shared__ __align__(16) unsigned char smem[];
  T* buf = reinterpret_cast<T*>(smem);
  const SweepDesc& ds = a.d[blockIdx.y];
  const int nx = a.dim[0];
  const size_t nxy = size_t(nx) * a.dim[1];
  const int n = a.dim[ds.axis];                                   // rows per line
  const int nl = int(nxy * size_t(a.dim[2]) / size_t(n));         // lines
  const int lane = threadIdx.x;
  const int l0 = blockIdx.x * 64, l = l0 + lane;
  if (l0 >= nl) return;  // the grid covers the descriptor with the most lines
  T* sfac = buf + size_t(sweep_buf_rows(n, XAX, kRR)) * PIT;  // shared: L[n*P], DU[n*P], D[n]
  const bool act = l < nl;
  const int nll = min(64, nl - l0);  // lines in this tile
  const T* __restrict__ in = static_cast<const T*>(ds.in);
  T* __restrict__ out = static_cast<T*>(ds.out);
  const T* __restrict__ accp = static_cast<const T*>(ds.acc);
  const int lc = act ? l : 0;
  // y lines: line (i, k) starts at i + k nx ny, stride nx; z lines: line
  // i + j nx starts there, stride nx ny
  const size_t lbase = (ds.axis == 1) ? size_t(lc % nx) + size_t(lc / nx) * nxy : size_t(lc);
  const size_t rstride = (ds.axis == 1) ? size_t(nx) : nxy;
  const int nreg = min(n, kRR);

  if (!MOD) {
    stage_batched<T, 64>(sfac, static_cast<const T*>(ds.L), n * P, lane);
    stage_batched<T, 64>(sfac + n * P, static_cast<const T*>(ds.U), n * P, lane);
    stage_batched<T, 64>(sfac + 2 * n * P, static_cast<const T*>(ds.D), n, lane);
  }

  // x lines: copy columns [c0, c1) of the nll contiguous lines into
  // buf[(r - c0) * PIT + line] (coalesced global reads)
  auto stage_cols = [&](int c0, int c1) {
    const int wdt = c1 - c0, total = nll * wdt;
    const float inv = 1.0f / float(wdt);
    const T* src = in + size_t(l0) * n;
    for (int e0 = 0; e0 < total; e0 += 64 * kLoadCH) {
      T v[kLoadCH];
#pragma unroll
      for (int c = 0; c < kLoadCH; ++c) {
        const int e = min(e0 + c * 64 + lane, total - 1);
        int ll = int((float(e) + 0.5f) * inv);
        int r = e - ll * wdt;
        if (r < 0) { --ll; r += wdt; }
        if (r >= wdt) { ++ll; r -= wdt; }
        v[c] = src[size_t(ll) * n + c0 + r];
      }
#pragma unroll
      for (int c = 0; c < kLoadCH; ++c) {
        const int e = e0 + c * 64 + lane;
        int ll = int((float(e) + 0.5f) * inv);
        int r = e - ll * wdt;
        if (r < 0) { --ll; r += wdt; }
        if (r >= wdt) { ++ll; r -= wdt; }
        if (e < total) buf[r * PIT + ll] = v[c];
      }
    }
  };
  auto unstage_cols = [&](int c0, int c1) {
    const int wdt = c1 - c0, total = nll * wdt;
    const float inv = 1.0f / float(wdt);
    T* dst = out + size_t(l0) * n;
    const T* ac = accp ? accp + size_t(l0) * n : nullptr;
    for (int e0 = 0; e0 < total; e0 += 64 * kLoadCH) {
#pragma unroll
      for (int c = 0; c < kLoadCH; ++c) {
        const int e = e0 + c * 64 + lane;
        int ll = int((float(e) + 0.5f) * inv);
        int r = e - ll * wdt;
        if (r < 0) { --ll; r += wdt; }
        if (r >= wdt) { ++ll; r -= wdt; }
        if (e < total) {
          const size_t o = size_t(ll) * n + c0 + r;
          T v = buf[r * PIT + ll];
          if (ac) v += ac[o];
          dst[o] = v;
        }
      }
    }
  };

  // ---- load: registers for rows [0, nreg), LDS for rows [kRR, n)
  T yr[kRA];
  if (XAX) {
    if (kRR > 0) {
      stage_cols(0, nreg);
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRR; ++r) yr[r] = (r < nreg) ? buf[r * PIT + lane] : T(0);
      __syncthreads();
    }
    if (n > kRR) stage_cols(kRR, n);
    __syncthreads();
  } else {
#pragma unroll
    for (int r = 0; r < kRR; ++r) yr[r] = in[lbase + size_t(min(r, n - 1)) * rstride];
    for (int r0 = kRR; r0 < n; r0 += kLoadCH) {
      T v[kLoadCH];
#pragma unroll
      for (int c = 0; c < kLoadCH; ++c) v[c] = in[lbase + size_t(min(r0 + c, n - 1)) * rstride];
#pragma unroll
      for (int c = 0; c < kLoadCH; ++c)
        if (r0 + c < n) buf[(r0 + c - kRR) * PIT + lane] = v[c];
    }
    __syncthreads();  // shared factors
  }

  const T* __restrict__ Lm = static_cast<const T*>(ds.L);
  const T* __restrict__ Um = static_cast<const T*>(ds.U);
  const T* __restrict__ Dm = static_cast<const T*>(ds.D);
  // per-line factors: [line / 64][row][k][line % 64], so that a wave's
  // factors are one contiguous stream
  const size_t fb = size_t(blockIdx.x) * n;
  auto fL = [&](int r, int k) -> T {
    if (MOD) return Lm[((fb + r) * P + k) * 64 + lane];
    return sfac[r * P + k];
  };
  auto fU = [&](int r, int k) -> T {
    if (MOD) return Um[((fb + r) * P + k) * 64 + lane];
    return sfac[n * P + r * P + k];
  };
  auto fD = [&](int r) -> T {
    if (MOD) return Dm[(fb + r) * 64 + lane];
    return sfac[2 * n * P + r];
  };

  T h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = T(0);
  // ---- forward, register rows (rows >= n are padding and never stored).
  // Per-line factors: a chunk's loads are issued while the chunk before it
  // is computed (two fixed register slots, unconditional clamped loads).
  if (!MOD || P < 3) {
#pragma unroll
    for (int r = 0; r < kRR; ++r) {
      const int rf = min(r, n - 1);
      T s = yr[r];
#pragma unroll
      for (int k = P - 1; k >= 0; --k) s -= fL(rf, k) * h[k];
#pragma unroll
      for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
      h[0] = s;
      yr[r] = s;
    }
  } else if (kRR > 0) {
    constexpr int NRC = (kRR + kCH - 1) / kCH;
    T gl[2][kCH][P];
    auto load_r = [&](int q, T (&g)[kCH][P]) {
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        const int rf = min(q * kCH + c, n - 1);
#pragma unroll
        for (int k = 0; k < P; ++k) g[c][k] = fL(rf, k);
      }
    };
    load_r(0, gl[0]);
    static_for<NRC>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if (q + 1 < NRC) load_r(q + 1, gl[(q + 1) & 1]);
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        constexpr int r0 = q * kCH;
        if (r0 + c < kRR) {
          T s = yr[r0 + c];
#pragma unroll
          for (int k = P - 1; k >= 0; --k) s -= gl[q & 1][c][k] * h[k];
#pragma unroll
          for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
          h[0] = s;
          yr[r0 + c] = s;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each chunk's loads in its slot
    });
  }
  // ---- forward, LDS rows.  Shared factors come from LDS.  Per-line factors
  // (global memory) go through a ring of kD register slots of kCH rows: the
  // loads of chunk j + kD - 1 are issued before chunk j is computed, all
  // unconditionally (rows clamped), and the chunk loop is unrolled by the
  // ring length so that every slot is a fixed set of registers; a wave so
  // keeps kD - 1 chunks of factors in flight.
  constexpr int kD = MOD ? fac_ring<T, P>() : 1;
  const int nch = n > kRR ? (n - kRR + kCH - 1) / kCH : 0;  // chunks of LDS rows
  {
    T f[kD][kCH][P];
    auto load_f = [&](int j, T (&g)[kCH][P]) {
      const int r0 = kRR + j * kCH;
#pragma unroll
      for (int c = 0; c < kCH; ++c)
#pragma unroll
        for (int k = 0; k < P; ++k) g[c][k] = fL(min(r0 + c, n - 1), k);
    };
    auto fwd_chunk = [&](int j, const T (&g)[kCH][P]) {
      const int r0 = kRR + j * kCH;
      T v[kCH];
#pragma unroll
      for (int c = 0; c < kCH; ++c) v[c] = buf[(min(r0 + c, n - 1) - kRR) * PIT + lane];
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        T s = v[c];
#pragma unroll
        for (int k = P - 1; k >= 0; --k) s -= g[c][k] * h[k];
#pragma unroll
        for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
        h[0] = s;
        v[c] = s;
      }
#pragma unroll
      for (int c = 0; c < kCH; ++c)
        if (r0 + c < n) buf[(r0 + c - kRR) * PIT + lane] = v[c];
    };
    if (MOD) {
      if (nch > 0) {
#pragma unroll
        for (int s = 0; s + 1 < kD; ++s) load_f(s, f[s]);
        for (int j0 = 0; j0 < nch; j0 += kD) {
          static_for<kD>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            const int j = j0 + S;
            load_f(j + kD - 1, f[(S + kD - 1) % kD]);
            if (j < nch) fwd_chunk(j, f[S]);  // uniform
          });
        }
      }
    } else {
      for (int j = 0; j < nch; ++j) {
        load_f(j, f[0]);
        fwd_chunk(j, f[0]);
      }
    }
  }
  // ---- backward, LDS rows (from the last row down to kRR), same ring
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = T(0);
  {
    T f[kD][kCH][P], d[kD][kCH];
    // chunk j holds rows n-1-j*kCH, n-2-j*kCH, ... (descending, clamped at kRR)
    auto load_f = [&](int j, T (&g)[kCH][P], T (&e)[kCH]) {
      const int r0 = n - 1 - j * kCH;
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        const int rf = max(r0 - c, kRR);
#pragma unroll
        for (int k = 0; k < P; ++k) g[c][k] = fU(rf, k);
        e[c] = fD(rf);
      }
    };
    auto bwd_chunk = [&](int j, const T (&g)[kCH][P], const T (&e)[kCH]) {
      const int r0 = n - 1 - j * kCH;
      T v[kCH];
#pragma unroll
      for (int c = 0; c < kCH; ++c) v[c] = buf[(max(r0 - c, kRR) - kRR) * PIT + lane];
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        if (r0 - c >= kRR) {  // uniform
          T s = e[c] * v[c];
#pragma unroll
          for (int k = P - 1; k >= 0; --k) s -= g[c][k] * h[k];
#pragma unroll
          for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
          h[0] = s;
          v[c] = s;
        }
      }
#pragma unroll
      for (int c = 0; c < kCH; ++c)
        if (r0 - c >= kRR) buf[(r0 - c - kRR) * PIT + lane] = v[c];
    };
    if (MOD) {
      if (nch > 0) {
#pragma unroll
        for (int s = 0; s + 1 < kD; ++s) load_f(s, f[s], d[s]);
        for (int j0 = 0; j0 < nch; j0 += kD) {
          static_for<kD>([&](auto sc) {
            constexpr int S = decltype(sc)::value;
            const int j = j0 + S;
            load_f(j + kD - 1, f[(S + kD - 1) % kD], d[(S + kD - 1) % kD]);
            if (j < nch) bwd_chunk(j, f[S], d[S]);  // uniform
          });
        }
      }
    } else {
      for (int j = 0; j < nch; ++j) {
        load_f(j, f[0], d[0]);
        bwd_chunk(j, f[0], d[0]);
      }
    }
  }
  // ---- backward, register rows (padding rows r >= n are skipped).  Per-line
  // factors of a chunk of kCH rows are loaded, unconditionally (rows
  // clamped), while the chunk before it is computed; a load inside the
  // per-row branch would be waited for row by row.
  if (!MOD || P < 3) {
#pragma unroll
    for (int r = kRR - 1; r >= 0; --r) {
      if (r < n) {  // uniform
        T s = fD(r) * yr[r];
#pragma unroll
        for (int k = P - 1; k >= 0; --k) s -= fU(r, k) * h[k];
#pragma unroll
        for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
        h[0] = s;
        yr[r] = s;
      }
    }
  } else if (kRR > 0) {
    constexpr int NRC = (kRR + kCH - 1) / kCH;
    T gu[2][kCH][P], gd[2][kCH];
    auto load_r = [&](int q, T (&g)[kCH][P], T (&e)[kCH]) {
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        const int rf = min(max(kRR - 1 - q * kCH - c, 0), n - 1);
#pragma unroll
        for (int k = 0; k < P; ++k) g[c][k] = fU(rf, k);
        e[c] = fD(rf);
      }
    };
    load_r(0, gu[0], gd[0]);
    static_for<NRC>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      if (q + 1 < NRC) load_r(q + 1, gu[(q + 1) & 1], gd[(q + 1) & 1]);
#pragma unroll
      for (int c = 0; c < kCH; ++c) {
        constexpr int r0 = kRR - 1 - q * kCH;
        const int r = r0 - c;
        if (r >= 0 && r < n) {  // uniform
          T s = gd[q & 1][c] * yr[r];
#pragma unroll
          for (int k = P - 1; k >= 0; --k) s -= gu[q & 1][c][k] * h[k];
#pragma unroll
          for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
          h[0] = s;
          yr[r] = s;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each chunk's loads in its slot
    });
  }

  // ---- store
  if (XAX) {
    __syncthreads();
    if (n > kRR) unstage_cols(kRR, n);
    if (kRR > 0) {
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRR; ++r)
        if (r < nreg) buf[r * PIT + lane] = yr[r];
      __syncthreads();
      unstage_cols(0, nreg);
    }
  } else if (act) {
#pragma unroll
    for (int r = 0; r < kRR; ++r) {
      if (r < n) {
        const size_t o = lbase + size_t(r) * rstride;
        T v = yr[r];
        if (accp) v += accp[o];
        out[o] = v;
      }
    }
    for (int r = kRR; r < n; ++r) {
      const size_t o = lbase + size_t(r) * rstride;
      T v = buf[(r - kRR) * PIT + lane];
      if (accp) v += accp[o];
      out[o] = v;
    }
  }
  if (a.tick_t && blockIdx.x == 0 && blockIdx.y == 0 && lane == 0) *a.tick_t += a.tick_dt;
}

// ------------------------------------------------------------ partitioned sweep
// Shared-factor lines, each split into S row segments (4, or 8 for long
// lines) solved by the S waves of a block (wave = segment, lane = line, 64
// lines per block); a segment's rows stay in registers.  Per line:
//   1. g = A_s^{-1} b on every segment (block-diagonal LU, forward and
//      backward recurrences of m = n / S rows instead of n);
//   2. the p values at both ends of every segment go through LDS, and each
//      segment forms the 2p interface unknowns it needs from the
//      precomputed inverse R of the reduced system: T (top p rows of the
//      next segment) and U (bottom p rows of the previous one);
//   3. x = g - V T - W U with the precomputed spikes V, W.
// The factors, spikes and R of the descriptor are staged in LDS (broadcast
// reads: every lane of a wave reads the same row).
// With AP the right-hand side is A v for the line's values v (A = the
// descriptor's banded operator, staged in LDS behind R): each segment loads
// its rows with a p-row halo on both sides and forms its rows of A v before
// the solve, and the store writes acc + scale * x.
template <typename T, int P, bool XAX, int MR, int S, bool AP>
__device__ __forceinline__ void spike_body(const SweepArgs& a) {
  constexpr int Q = 2 * P * (S - 1), W = 2 * P + 1;
  constexpr int MRV = AP ? MR + 2 * P : MR;  // rows of the line a segment loads
  extern __shared__ __align__(16) unsigned char smem[];
  T* sf = reinterpret_cast<T*>(smem);
  const SweepDesc& ds = a.d[blockIdx.y];
  const int nx = a.dim[0];
  const size_t nxy = size_t(nx) * a.dim[1];
  const int n = a.dim[ds.axis];                                   // rows per line
  const int nl = int(nxy * size_t(a.dim[2]) / size_t(n));         // lines
  if (int(blockIdx.x) * 64 >= nl) return;  // block-uniform: before any barrier
  const int nf0 = n * (4 * P + 1) + Q * Q;
  const int nf = nf0 + (AP ? n * W : 0);
  T* gex = sf + nf;  // [Q][64] boundary values of g
  // the segment is the wave: wave-uniform, so its row offsets stay scalar
  const int tid = threadIdx.x, seg = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const T* sL = sf;
  const T* sDU = sf + n * P;
  const T* sD = sf + 2 * n * P;
  const T* sV = sD + n;
  const T* sW = sV + n * P;
  const T* sR = sW + n * P;

  const T* __restrict__ in = static_cast<const T*>(ds.in);
  T* __restrict__ out = static_cast<T*>(ds.out);
  const T* __restrict__ accp = static_cast<const T*>(ds.acc);
  const int l = blockIdx.x * 64 + lane;
  const bool act = l < nl;
  const int lc = act ? l : 0;
  size_t lbase, rstride;
  if (XAX) {
    lbase = size_t(lc) * n;
    rstride = 1;
  } else if (ds.axis == 1) {
    lbase = size_t(lc % nx) + size_t(lc / nx) * nxy;
    rstride = nx;
  } else {
    lbase = size_t(lc);
    rstride = nxy;
  }
  const int b0 = (seg * n) / S, b1 = ((seg + 1) * n) / S, m = b1 - b0;  // m <= MR

  // unconditional loads (rows past the segment repeat its last row) keep
  // every load of the segment in flight at once
  // x lines (contiguous in memory) go through a per-wave LDS tile of 8 rows
  // x 64 lines: lanes read runs of 8 consecutive values (coalesced) and each
  // lane then takes its own line's rows.  LDS operations of one wave execute
  // in order, so the tile needs no barrier.
  T* xt = gex + Q * 64 + seg * (8 * 65);
  const int l0 = blockIdx.x * 64;
  // line row held in load slot r: the segment's rows (slots past it repeat
  // its last row), or with AP the segment's rows with a p-row halo on both
  // sides, clamped to the line (the band of A is zero outside the line)
  const int mv = AP ? m + 2 * P : m;
  auto rowof = [&](int r) {
    return AP ? min(max(b0 - P + r, 0), n - 1) : b0 + min(r, m - 1);
  };
  T yv[MRV];
  if (XAX && (AP ? MRV <= 48 : MR <= 40)) {
    // short segments: every chunk's loads in flight at once (rows clamped),
    // then the chunks go through the tile one by one
    constexpr int NC = (MRV + 7) / 8;
    T v[NC][8];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int e = lane + 64 * j, ln = e >> 3, rr = e & 7;
        v[c][j] = in[size_t(min(l0 + ln, nl - 1)) * n + rowof(8 * c + rr)];
      }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      if (8 * c < mv) {  // uniform
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = lane + 64 * j;
          xt[(e & 7) * 65 + (e >> 3)] = v[c][j];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
          if (8 * c + rr < MRV) yv[8 * c + rr] = xt[rr * 65 + lane];
        __builtin_amdgcn_wave_barrier();
      }
    }
  } else if (XAX) {
#pragma unroll
    for (int c0 = 0; c0 < MRV; c0 += 8) {
      if (c0 < mv) {  // uniform
        T v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = lane + 64 * j, ln = e >> 3, rr = e & 7;
          v[j] = in[size_t(min(l0 + ln, nl - 1)) * n + rowof(c0 + rr)];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = lane + 64 * j;
          xt[(e & 7) * 65 + (e >> 3)] = v[j];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
          if (c0 + rr < MRV) yv[c0 + rr] = xt[rr * 65 + lane];
        __builtin_amdgcn_wave_barrier();
      }
    }
  } else {
#pragma unroll
    for (int r = 0; r < MRV; ++r) yv[r] = in[lbase + size_t(rowof(r)) * rstride];
  }
  stage_batched<T, 64 * S>(sf, static_cast<const T*>(ds.spk), nf0, tid);
  if constexpr (AP) stage_batched<T, 64 * S>(sf + nf0, static_cast<const T*>(ds.aband), n * W, tid);
  __syncthreads();  // factors staged
  T y[MR];
  if constexpr (AP) {
    // rows of A v: padding rows (r >= m) read band rows past the line, which
    // lie inside the block's LDS; their results are never stored
    const T* sA = sf + nf0;
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      const T* Ar = sA + (b0 + r) * W;
      T acc = T(0);
#pragma unroll
      for (int d = 0; d < W; ++d) acc += Ar[d] * yv[r + d];
      y[r] = acc;
    }
  } else {
#pragma unroll
    for (int r = 0; r < MR; ++r) y[r] = yv[r];
  }

  // Forward and backward recurrences over all MR rows without a branch per
  // row, so that the compiler issues the factor reads of later rows (at
  // fixed offsets from one base) ahead of the dependent arithmetic.  Rows
  // r >= m (padding) read factors past the segment (the staged arrays are
  // followed by others, so every read stays inside the block's LDS) and
  // their results are never stored; in the backward pass they are set to
  // zero, so the segment's last row starts from h = 0.  Long float64
  // segments keep a branch per row: without it they need every register
  // and ran slower (256^3, p = 2: 0.23 -> 0.31 ms per y/z launch).
  constexpr bool kFlat = sizeof(T) * MR <= 8 * 48;
  T h[P];
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = T(0);
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    if (kFlat || r < m) {  // compile-time, or wave-uniform
      const T* Lr = sL + (b0 + r) * P;
      T s = y[r];
#pragma unroll
      for (int k = P - 1; k >= 0; --k) s -= Lr[k] * h[k];
#pragma unroll
      for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
      h[0] = s;
      y[r] = s;
    }
  }
#pragma unroll
  for (int k = 0; k < P; ++k) h[k] = T(0);
#pragma unroll
  for (int r = MR - 1; r >= 0; --r) {
    if (kFlat || r < m) {
      const int g = b0 + r;
      T s = sD[g] * y[r];
#pragma unroll
      for (int k = P - 1; k >= 0; --k) s -= sDU[g * P + k] * h[k];
      if (kFlat) s = (r < m) ? s : T(0);
#pragma unroll
      for (int k = P - 1; k > 0; --k) h[k] = h[k - 1];
      h[0] = s;
      y[r] = s;
    }
  }

  // boundary values: z layout [U_0, T_1, U_1, T_2, ...], p each
#pragma unroll
  for (int r = 0; r < MR; ++r) {
    if (seg > 0 && r < P) gex[(2 * P * (seg - 1) + P + r) * 64 + lane] = y[r];
    if (seg < S - 1 && r >= m - P && r < m) gex[(2 * P * seg + r - (m - P)) * 64 + lane] = y[r];
  }
  __syncthreads();
  T tn[P], up[P];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    tn[k] = T(0);
    up[k] = T(0);
  }
  if (seg < S - 1) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const T* Rr = sR + (2 * P * seg + P + k) * Q;
      T s = T(0);
#pragma unroll
      for (int c = 0; c < Q; ++c) s += Rr[c] * gex[c * 64 + lane];
      tn[k] = s;
    }
  }
  if (seg > 0) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const T* Rr = sR + (2 * P * (seg - 1) + k) * Q;
      T s = T(0);
#pragma unroll
      for (int c = 0; c < Q; ++c) s += Rr[c] * gex[c * 64 + lane];
      up[k] = s;
    }
  }
  // correction x = g - V T - W U in groups of four rows, each group behind a
  // wave-uniform branch: the rows of a group read their spikes together,
  // while the branches keep the compiler from holding every row's spikes in
  // registers at once
  constexpr int kGroup = kFlat ? 4 : 1;
#pragma unroll
  for (int r0 = 0; r0 < MR; r0 += kGroup) {
    if (r0 < m) {  // uniform
#pragma unroll
      for (int r = r0; r < r0 + kGroup && r < MR; ++r) {
        const int g = b0 + r;  // padding rows read past the segment, never stored
        T x = y[r];
#pragma unroll
        for (int k = 0; k < P; ++k) x -= sV[g * P + k] * tn[k] + sW[g * P + k] * up[k];
        y[r] = x;
      }
    }
  }
  if constexpr (AP) {
    const T sc = T(ds.scale);
#pragma unroll
    for (int r = 0; r < MR; ++r) y[r] *= sc;
  }
  if (XAX) {
    // the values to add (x_old) in the stores' own pattern, every chunk's
    // loads in flight at once (rows and lines clamped) instead of one wait
    // per chunk
    constexpr int NCS = (MR + 7) / 8;
    T av[NCS][8];
    if (accp) {  // uniform
#pragma unroll
      for (int c = 0; c < NCS; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = lane + 64 * j, ln = e >> 3, rr = e & 7;
          av[c][j] = accp[size_t(min(l0 + ln, nl - 1)) * n + b0 + min(8 * c + rr, m - 1)];
        }
    }
#pragma unroll
    for (int c0 = 0; c0 < MR; c0 += 8) {
      if (c0 < m) {  // uniform
#pragma unroll
        for (int rr = 0; rr < 8; ++rr)
          if (c0 + rr < MR) xt[rr * 65 + lane] = y[c0 + rr];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int e = lane + 64 * j, ln = e >> 3, rr = e & 7;
          if (l0 + ln < nl && c0 + rr < m) {
            const size_t o = size_t(l0 + ln) * n + b0 + c0 + rr;
            T x = xt[rr * 65 + ln];
            if (accp) x += av[c0 / 8][j];
            out[o] = x;
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  } else {
    if (kFlat && accp) {  // uniform: the old state's rows (clamped, no branch per row)
#pragma unroll
      for (int r = 0; r < MR; ++r) y[r] += accp[lbase + size_t(b0 + min(r, m - 1)) * rstride];
    }
#pragma unroll
    for (int r = 0; r < MR; ++r) {
      if (r < m) {
        const size_t o = lbase + size_t(b0 + r) * rstride;
        T x = y[r];
        if (!kFlat && accp) x += accp[o];
        if (act) out[o] = x;
      }
    }
  }
  if (a.tick_t && blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) *a.tick_t += a.tick_dt;
}

// Kernels of the two line solvers.  A solve round whose descriptors mix x
// lines with y/z lines runs as one launch (the descriptor's axis selects the
// code path per block, x descriptors first so that the longer x blocks start
// first) instead of two launches on two streams joined by events: the
// cross-stream waits left the GPU idle for 5-9 us per round.
template <typename T, int P, bool XAX, bool MOD>
__global__ __launch_bounds__(64) void sweep_kernel(SweepArgs a) {
  sweep_body<T, P, XAX, MOD>(a);
}
template <typename T, int P, bool MOD>
__global__ __launch_bounds__(64) void sweep_mixed_kernel(SweepArgs a) {
  if (a.d[blockIdx.y].axis == 0) sweep_body<T, P, true, MOD>(a);
  else sweep_body<T, P, false, MOD>(a);
}
template <typename T, int P, bool XAX, int MR, int S, bool AP>
__global__ __launch_bounds__(64 * S) void spike_kernel(SweepArgs a) {
  spike_body<T, P, XAX, MR, S, AP>(a);
}
template <typename T, int P, int MR, int S, bool AP>
__global__ __launch_bounds__(64 * S) void spike_mixed_kernel(SweepArgs a) {
  if (a.d[blockIdx.y].axis == 0) spike_body<T, P, true, MR, S, AP>(a);
  else spike_body<T, P, false, MR, S, AP>(a);
}

// ------------------------------------------------------------ factorisation
// Pivot-free banded Doolittle LU of the material-modified 1D matrices, one
// line per thread, in float64.  Row r of line l is Mb[r,:] + alpha[pos] Sb[r,:]
// with alpha read at the row's own position (the row's test function), so
// the factors are those of the row-scaled 1D system of eq. dupa1abcdefg.
template <int P>
__global__ __launch_bounds__(64) void factor_kernel(FactorArgs a) {
  constexpr int W = 2 * P + 1;
  const int l = blockIdx.x * 64 + threadIdx.x;
  if (l >= a.nlines) return;
  const int n = a.n;
  const size_t nxy = size_t(a.nx) * a.ny;
  size_t lbase, rstride;
  if (a.axis == 0) { lbase = size_t(l) * n; rstride = 1; }
  else if (a.axis == 1) { lbase = size_t(l % a.nx) + size_t(l / a.nx) * nxy; rstride = a.nx; }
  else { lbase = l; rstride = nxy; }

  double up[P + 1][P + 1];  // up[m][c] = U_{i-m, i-m+c}
#pragma unroll
  for (int m = 0; m <= P; ++m)
#pragma unroll
    for (int c = 0; c <= P; ++c) up[m][c] = 0.0;
  double minr = 1e300;
  for (int i = 0; i < n; ++i) {
    const double al = a.alpha[lbase + size_t(i) * rstride];
    double A[W];
#pragma unroll
    for (int d = 0; d < W; ++d) A[d] = a.Mb[size_t(i) * W + d] + al * a.Sb[size_t(i) * W + d];
    double Lr[P + 1];
    Lr[0] = 1.0;
#pragma unroll
    for (int m = P; m >= 1; --m) {
      if (i - m < 0) {
        Lr[m] = 0.0;
        continue;
      }
      double s = A[P - m];
#pragma unroll
      for (int mp = m + 1; mp <= P; ++mp) s -= Lr[mp] * up[mp][mp - m];
      Lr[m] = s / up[m][0];
    }
    double ur[P + 1];
#pragma unroll
    for (int c = 0; c <= P; ++c) {
      double s = A[P + c];
#pragma unroll
      for (int mp = 1; mp <= P - c; ++mp) s -= Lr[mp] * up[mp][c + mp];
      ur[c] = s;
    }
    const double dinv = 1.0 / ur[0];
    const size_t ob = size_t(l >> 6) * n + i;  // per-line factors: [line / 64][row][k][line % 64]
#pragma unroll
    for (int m = 1; m <= P; ++m) {
      const size_t o = (ob * P + (m - 1)) * 64 + (l & 63);
      const double du = dinv * ur[m];  // pre-scaled for the backward substitution
      if (a.L64) {
        a.L64[o] = Lr[m];
        a.U64[o] = du;
      }
      if (a.L32) {
        a.L32[o] = float(Lr[m]);
        a.U32[o] = float(du);
      }
    }
    if (a.D64) a.D64[ob * 64 + (l & 63)] = dinv;
    if (a.D32) a.D32[ob * 64 + (l & 63)] = float(dinv);
    const double ratio = fabs(ur[0]) / fabs(A[P]);
    minr = ratio < minr ? ratio : minr;
#pragma unroll
    for (int m = P; m >= 2; --m)
#pragma unroll
      for (int c = 0; c <= P; ++c) up[m][c] = up[m - 1][c];
#pragma unroll
    for (int c = 0; c <= P; ++c) up[1][c] = ur[c];
  }
  a.minratio[l] = minr;
}

template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ src, D* __restrict__ dst, size_t count) {
  const size_t stride = size_t(gridDim.x) * blockDim.x;
  for (size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count; i += stride)
    dst[i] = D(src[i]);
}

template <typename K>
hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
}

template <typename TI, typename TC, typename TO, typename TK, int P, int STAGE>
hipError_t launch_rhs_t(const RhsArgs<TC>& a, hipStream_t s) {
  auto k = rhs_kernel<TI, TC, TO, TK, P, STAGE>;
  const size_t lds = rhs_lds_bytes<TC, P, STAGE>(a.zchunk);
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  dim3 grid(3 * ((a.nx + kTX - 1) / kTX), (a.ny + kTY - 1) / kTY, (a.nz + a.zchunk - 1) / a.zchunk);
  hipLaunchKernelGGL(k, grid, dim3(kRhsThreads), lds, s, a, a.bandx, a.bandy, a.zw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_rhs_p(int stage, const RhsArgs<T>& a, hipStream_t s) {
  switch (stage) {
    case kStageE1: return launch_rhs_t<T, T, T, T, P, kStageE1>(a, s);
    case kStageE2: return launch_rhs_t<T, T, T, T, P, kStageE2>(a, s);
    case kStageH1: return launch_rhs_t<T, T, T, T, P, kStageH1>(a, s);
    case kStageH2: return launch_rhs_t<T, T, T, T, P, kStageH2>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int P>
hipError_t launch_inc_p(int stage, const RhsArgs<double>& a, hipStream_t s) {
  switch (stage) {
    case kStageEd1: return launch_rhs_t<float, double, float, float, P, kStageEd1>(a, s);
    case kStageEd2: return launch_rhs_t<float, double, float, float, P, kStageEd2>(a, s);
    case kStageHd1: return launch_rhs_t<float, double, float, float, P, kStageHd1>(a, s);
    case kStageHd2: return launch_rhs_t<float, double, float, float, P, kStageHd2>(a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, int P, bool XAX, bool MOD>
size_t sweep_lds(int n) {
  return (size_t(sweep_buf_rows(n, XAX, SweepRegRows<T, MOD>::value)) * sweep_pitch(XAX) +
          (MOD ? 0 : size_t(n) * (2 * P + 1))) * sizeof(T);
}

// Longest line and largest line count over the descriptors of a launch: the
// LDS is sized for the longest line, the grid for the most lines (blocks
// past a descriptor's lines return at once).
struct LaunchShape {
  int nmax = 0, lines = 0;
};
inline LaunchShape launch_shape(int ndesc, const SweepArgs& a) {
  LaunchShape r;
  const size_t D = size_t(a.dim[0]) * a.dim[1] * a.dim[2];
  for (int i = 0; i < ndesc; ++i) {
    const int n = a.dim[a.d[i].axis];
    r.nmax = std::max(r.nmax, n);
    r.lines = std::max(r.lines, int(D / size_t(n)));
  }
  return r;
}

template <typename T, int P, bool XAX, bool MOD>
hipError_t launch_sweep_k(int ndesc, const SweepArgs& a, hipStream_t s) {
  const LaunchShape sh = launch_shape(ndesc, a);
  const size_t lds = sweep_lds<T, P, XAX, MOD>(sh.nmax);
  dim3 grid((sh.lines + 63) / 64, ndesc);
  auto k = sweep_kernel<T, P, XAX, MOD>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(64), lds, s, a);
  return hipGetLastError();
}
template <typename T, int P, bool MOD>
hipError_t launch_sweep_mixed(int ndesc, const SweepArgs& a, hipStream_t s) {
  const LaunchShape sh = launch_shape(ndesc, a);
  const size_t lds =
      std::max(sweep_lds<T, P, true, MOD>(sh.nmax), sweep_lds<T, P, false, MOD>(sh.nmax));
  dim3 grid((sh.lines + 63) / 64, ndesc);
  auto k = sweep_mixed_kernel<T, P, MOD>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(64), lds, s, a);
  return hipGetLastError();
}

template <typename T, int P, bool XAX, int MR, int S, bool AP>
hipError_t launch_spike_k(int ndesc, const SweepArgs& a, hipStream_t s) {
  constexpr int Q = 2 * P * (S - 1);
  const LaunchShape sh = launch_shape(ndesc, a);
  const size_t lds = (size_t(sh.nmax) * (4 * P + 1 + (AP ? 2 * P + 1 : 0)) + Q * Q +
                      size_t(Q) * 64 + (XAX ? size_t(S) * 8 * 65 : 0)) * sizeof(T);
  dim3 grid((sh.lines + 63) / 64, ndesc);
  auto k = spike_kernel<T, P, XAX, MR, S, AP>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(64 * S), lds, s, a);
  return hipGetLastError();
}

template <typename T, int P, int MR, int S, bool AP>
hipError_t launch_spike_mixed_k(int ndesc, const SweepArgs& a, hipStream_t s) {
  constexpr int Q = 2 * P * (S - 1);
  const LaunchShape sh = launch_shape(ndesc, a);
  const size_t lds = (size_t(sh.nmax) * (4 * P + 1 + (AP ? 2 * P + 1 : 0)) + Q * Q +
                      size_t(Q) * 64 + size_t(S) * 8 * 65) * sizeof(T);
  dim3 grid((sh.lines + 63) / 64, ndesc);
  auto k = spike_mixed_kernel<T, P, MR, S, AP>;
  hipError_t e = set_lds(k, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k, grid, dim3(64 * S), lds, s, a);
  return hipGetLastError();
}

template <typename T, int P, int MR, int S, bool AP>
hipError_t launch_spike_xsa(int xaxis, int ndesc, const SweepArgs& a, hipStream_t s) {
  if (xaxis == 2) return launch_spike_mixed_k<T, P, MR, S, AP>(ndesc, a, s);
  return xaxis ? launch_spike_k<T, P, true, MR, S, AP>(ndesc, a, s)
               : launch_spike_k<T, P, false, MR, S, AP>(ndesc, a, s);
}

template <typename T, int P, int MR, int S>
hipError_t launch_spike_xs(int xaxis, int ndesc, const SweepArgs& a, hipStream_t s) {
  return a.apply ? launch_spike_xsa<T, P, MR, S, true>(xaxis, ndesc, a, s)
                 : launch_spike_xsa<T, P, MR, S, false>(xaxis, ndesc, a, s);
}

// xaxis: 0 = y/z lines, 1 = x lines, 2 = both (descriptor axis per block)
template <typename T, int P>
hipError_t launch_spike_x(int xaxis, int ndesc, const SweepArgs& a, hipStream_t s) {
  // register rows per segment: ceil(n / S) of the longest line, rounded up
  // to the nearest instantiated length (padding rows cost work); lines of
  // n >= kSpikeS8MinN (<= kSpikeMaxN) have 8 segments of at most 36 rows
  const int nmax = launch_shape(ndesc, a).nmax;
  if (a.spike == kSpikeS8) {
    if ((nmax + kSpikeS8 - 1) / kSpikeS8 > 36) return hipErrorInvalidValue;
    return launch_spike_xs<T, P, 36, kSpikeS8>(xaxis, ndesc, a, s);
  }
  if (a.spike != kSpikeS) return hipErrorInvalidValue;
  const int m = (nmax + kSpikeS - 1) / kSpikeS;
  if (m <= 24) return launch_spike_xs<T, P, 24, kSpikeS>(xaxis, ndesc, a, s);
  if (m <= 36) return launch_spike_xs<T, P, 36, kSpikeS>(xaxis, ndesc, a, s);
  if (m <= 48) return launch_spike_xs<T, P, 48, kSpikeS>(xaxis, ndesc, a, s);
  return hipErrorInvalidValue;
}

template <typename T, int P>
hipError_t launch_sweep_p(int ndesc, const SweepArgs& a, hipStream_t s) {
  // every descriptor of one launch is either modified or shared
  const bool mod = a.d[0].modified != 0;
  for (int i = 1; i < ndesc; ++i)
    if ((a.d[i].modified != 0) != mod) return hipErrorInvalidValue;
  if (a.apply && (!a.spike || mod)) return hipErrorInvalidValue;  // partitioned solve only
  if (a.spike && !mod) {
    for (int i = 0; i < ndesc; ++i) {
      if (a.apply && !a.d[i].aband) return hipErrorInvalidValue;
      const int n = a.dim[a.d[i].axis];
      if (!a.d[i].spk || a.d[i].segs != a.spike || spike_segments(n) != a.spike ||
          n < kSpikeMinN || n > kSpikeMaxN)
        return hipErrorInvalidValue;
    }
    return launch_spike_x<T, P>(a.xaxis, ndesc, a, s);
  }
  if (a.xaxis == 2)
    return mod ? launch_sweep_mixed<T, P, true>(ndesc, a, s)
               : launch_sweep_mixed<T, P, false>(ndesc, a, s);
  if (a.xaxis)
    return mod ? launch_sweep_k<T, P, true, true>(ndesc, a, s)
               : launch_sweep_k<T, P, true, false>(ndesc, a, s);
  return mod ? launch_sweep_k<T, P, false, true>(ndesc, a, s)
             : launch_sweep_k<T, P, false, false>(ndesc, a, s);
}

}  // namespace

template <typename T>
hipError_t launch_rhs(int stage, int p, const RhsArgs<T>& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_rhs_p<T, 1>(stage, a, s);
    case 2: return launch_rhs_p<T, 2>(stage, a, s);
    case 3: return launch_rhs_p<T, 3>(stage, a, s);
    case 4: return launch_rhs_p<T, 4>(stage, a, s);
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_rhs<double>(int, int, const RhsArgs<double>&, hipStream_t);
template hipError_t launch_rhs<float>(int, int, const RhsArgs<float>&, hipStream_t);

template <int P>
hipError_t launch_inc32_p(int stage, const RhsArgs<float>& a, hipStream_t s) {
  switch (stage) {
    case kStageEd1: return launch_rhs_t<float, float, float, float, P, kStageEd1>(a, s);
    case kStageEd2: return launch_rhs_t<float, float, float, float, P, kStageEd2>(a, s);
    case kStageHd1: return launch_rhs_t<float, float, float, float, P, kStageHd1>(a, s);
    case kStageHd2: return launch_rhs_t<float, float, float, float, P, kStageHd2>(a, s);
  }
  return hipErrorInvalidValue;
}

// Increments of the float32 mode in float32 arithmetic and accumulation.
hipError_t launch_rhs_inc32(int stage, int p, const RhsArgs<float>& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_inc32_p<1>(stage, a, s);
    case 2: return launch_inc32_p<2>(stage, a, s);
    case 3: return launch_inc32_p<3>(stage, a, s);
    case 4: return launch_inc32_p<4>(stage, a, s);
  }
  return hipErrorInvalidValue;
}

// Increments of the float32 mode: float32 fields and coefficients, float64
// arithmetic, float32 outputs.
hipError_t launch_rhs_inc(int stage, int p, const RhsArgs<double>& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_inc_p<1>(stage, a, s);
    case 2: return launch_inc_p<2>(stage, a, s);
    case 3: return launch_inc_p<3>(stage, a, s);
    case 4: return launch_inc_p<4>(stage, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_sweep(int p, int ndesc, const SweepArgs& a, hipStream_t s) {
  switch (p) {
    case 1: return launch_sweep_p<T, 1>(ndesc, a, s);
    case 2: return launch_sweep_p<T, 2>(ndesc, a, s);
    case 3: return launch_sweep_p<T, 3>(ndesc, a, s);
    case 4: return launch_sweep_p<T, 4>(ndesc, a, s);
  }
  return hipErrorInvalidValue;
}
template hipError_t launch_sweep<double>(int, int, const SweepArgs&, hipStream_t);
template hipError_t launch_sweep<float>(int, int, const SweepArgs&, hipStream_t);

hipError_t launch_factor(int p, const FactorArgs& a, hipStream_t s) {
  dim3 grid((a.nlines + 63) / 64);
  switch (p) {
    case 1: hipLaunchKernelGGL(factor_kernel<1>, grid, dim3(64), 0, s, a); break;
    case 2: hipLaunchKernelGGL(factor_kernel<2>, grid, dim3(64), 0, s, a); break;
    case 3: hipLaunchKernelGGL(factor_kernel<3>, grid, dim3(64), 0, s, a); break;
    case 4: hipLaunchKernelGGL(factor_kernel<4>, grid, dim3(64), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// dir 0: double -> float, dir 1: float -> double
template <typename T>
hipError_t launch_convert(const void* src, void* dst, size_t count, int dir, hipStream_t s) {
  const int blocks = int(std::min<size_t>((count + 255) / 256, 4096));
  if (count == 0) return hipSuccess;
  if (dir == 0) {
    auto k = convert_kernel<double, float>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, static_cast<const double*>(src),
                       static_cast<float*>(dst), count);
  } else {
    auto k = convert_kernel<float, double>;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, s, static_cast<const float*>(src),
                       static_cast<double*>(dst), count);
  }
  return hipGetLastError();
}
template hipError_t launch_convert<float>(const void*, void*, size_t, int, hipStream_t);

}  // namespace adimx
