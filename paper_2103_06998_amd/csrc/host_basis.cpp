// Host-side (float64) B-spline basis, Gauss-Legendre rules, 1D Gram band
// matrices and pivot-free banded LU.  Initialisation work only.
//
// Basis: degree-p B-splines with maximal continuity on the open uniform knot
// vector of N elements on [0, 1] (p+1 repeated end knots), n = N + p functions
// (the patch discretisation of the section "Variational formulation").  The
// p+1 functions that are nonzero on a knot span and their first derivatives
// are evaluated with the triangular (inverted-triangle) scheme on that span.
//
// Gram matrices, row = test function, column = trial function:
//   M[l][i] = int B_l B_i,  S[l][i] = int B_l' B_i',  A[l][i] = int B_l B_i',
//   B = A^T (derivative on the test function; the matrix list after eqs.
//   discrete1-discrete4 names it twice as a trial derivative, but the weak
//   form weak1 term (d1 E2, d2 V1) = A (x) B (x) M fixes B = A^T).
// Band storage: band[r * (2p+1) + d] = X[r][r + d - p].
#include "adimx_internal.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace adimx {

std::vector<double> open_knots(int N, int p) {
  std::vector<double> t;
  for (int i = 0; i <= p; ++i) t.push_back(0.0);
  for (int i = 1; i < N; ++i) t.push_back(double(i) / double(N));
  for (int i = 0; i <= p; ++i) t.push_back(1.0);
  return t;
}

int find_span(const std::vector<double>& t, int p, int n, double x) {
  // index s with t[s] <= x < t[s+1], p <= s <= n-1; x = 1 maps to the last span
  if (x >= t[n]) return n - 1;
  if (x <= t[p]) return p;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) / 2;
    if (x < t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

// The p+1 B-splines of degree p that are nonzero on knot span `span` at x,
// and their first derivatives: the triangular Cox-de Boor evaluation with
// the knot differences kept in the lower triangle, as published in
// L. Piegl and W. Tiller, The NURBS Book (2nd ed., Springer 1997),
// algorithms A2.2 (basis functions) and A2.3 (derivatives), restated here
// for the first derivative only.
void basis_on_span(const std::vector<double>& t, int p, int span, double x, double* val,
                   double* der) {
  // ndu[j][r]: values of degree-j functions (upper triangle) and knot
  // differences (lower triangle), for j, r in 0..p.
  double ndu[kMaxP + 1][kMaxP + 1];
  double left[kMaxP + 1], right[kMaxP + 1];
  ndu[0][0] = 1.0;
  for (int j = 1; j <= p; ++j) {
    left[j] = x - t[span + 1 - j];
    right[j] = t[span + j] - x;
    double saved = 0.0;
    for (int r = 0; r < j; ++r) {
      ndu[j][r] = right[r + 1] + left[j - r];
      double tmp = ndu[r][j - 1] / ndu[j][r];
      ndu[r][j] = saved + right[r + 1] * tmp;
      saved = left[j - r] * tmp;
    }
    ndu[j][j] = saved;
  }
  for (int r = 0; r <= p; ++r) val[r] = ndu[r][p];
  if (!der) return;
  if (p == 0) {
    der[0] = 0.0;
    return;
  }
  // d/dx N_{s-p+r,p} = p (N_{s-p+r,p-1}/(t_{s+r}-t_{s-p+r}) - N_{s-p+r+1,p-1}/(t_{s+r+1}-t_{s-p+r+1}))
  for (int r = 0; r <= p; ++r) {
    double d = 0.0;
    // degree p-1 functions nonzero on the span: ndu[k][p-1], k = 0..p-1, index s-p+1+k
    if (r >= 1) {
      double den = ndu[p][r - 1];  // t[s+r] - t[s-p+r]
      d += ndu[r - 1][p - 1] / den;
    }
    if (r <= p - 1) {
      double den = ndu[p][r];      // t[s+r+1] - t[s-p+r+1]
      d -= ndu[r][p - 1] / den;
    }
    der[r] = p * d;
  }
}

// q-point Gauss-Legendre rule on [-1, 1]: the textbook Newton iteration on
// the Legendre polynomial P_q (three-term recurrence for P_q and P_q') from
// the initial guesses cos(pi (i + 3/4) / (q + 1/2)), weights
// 2 / ((1 - x^2) P_q'(x)^2) (as in, e.g., Press et al., Numerical Recipes,
// section 4.6 (3rd ed.: 4.6.1)).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  // Newton iteration on P_q from the Chebyshev-like initial guesses.
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < (q + 1) / 2; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));
    double pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= q; ++j) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = q * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (std::fabs(z - z1) < 1e-16) break;
    }
    x[i] = -z;
    x[q - 1 - i] = z;
    w[i] = w[q - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

Gram1D build_gram(int N, int p) {
  Gram1D g;
  g.N = N;
  g.p = p;
  g.n = N + p;
  const int n = g.n, w = 2 * p + 1;
  g.M.assign(size_t(n) * w, 0.0);
  g.S.assign(size_t(n) * w, 0.0);
  g.A.assign(size_t(n) * w, 0.0);
  g.B.assign(size_t(n) * w, 0.0);
  std::vector<double> t = open_knots(N, p);
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);  // exact for the degree <= 2p integrands
  double val[kMaxP + 1], der[kMaxP + 1];
  const double h = 1.0 / N;
  for (int e = 0; e < N; ++e) {
    const int span = p + e;
    for (int q = 0; q <= p; ++q) {
      const double x = (e + 0.5 * (gx[q] + 1.0)) * h;
      const double wq = 0.5 * h * gw[q];
      basis_on_span(t, p, span, x, val, der);
      for (int a = 0; a <= p; ++a) {      // test function span-p+a
        const int l = span - p + a;
        for (int b = 0; b <= p; ++b) {    // trial function span-p+b
          const int i = span - p + b;
          const int d = i - l + p;
          g.M[size_t(l) * w + d] += wq * val[a] * val[b];
          g.S[size_t(l) * w + d] += wq * der[a] * der[b];
          g.A[size_t(l) * w + d] += wq * val[a] * der[b];
        }
      }
    }
  }
  for (int r = 0; r < n; ++r)
    for (int d = 0; d < w; ++d) {
      const int c = r + d - p;
      if (c < 0 || c >= n) continue;
      g.B[size_t(r) * w + d] = g.A[size_t(c) * w + (2 * p - d)];
    }
  return g;
}

void apply_dirichlet(std::vector<double>& band, int n, int p) {
  const int w = 2 * p + 1;
  for (int b : {0, n - 1}) {
    for (int d = 0; d < w; ++d) band[size_t(b) * w + d] = 0.0;
    band[size_t(b) * w + p] = 1.0;
    for (int d = 0; d < w; ++d) {  // column b of the other rows
      const int r = b - (d - p);
      if (r >= 0 && r < n && r != b) band[size_t(r) * w + d] = 0.0;
    }
  }
}

double band_lu(const std::vector<double>& band, int n, int p, std::vector<double>& L,
               std::vector<double>& Uoff, std::vector<double>& Uinv) {
  // Doolittle without pivoting on the band.  Outputs, per row r:
  //   L[r*p + k-1]    = L_{r, r-k}   (k = 1..p)
  //   Uoff[r*p + k-1] = U_{r, r+k}   (k = 1..p)
  //   Uinv[r]         = 1 / U_{r,r}
  // Returns min_r |U_rr| / |A_rr|.
  const int w = 2 * p + 1;
  L.assign(size_t(n) * p, 0.0);
  Uoff.assign(size_t(n) * p, 0.0);
  Uinv.assign(n, 0.0);
  std::vector<double> Ud(n, 0.0);
  auto A = [&](int i, int j) { return band[size_t(i) * w + (j - i + p)]; };
  auto U = [&](int k, int j) -> double { return j == k ? Ud[k] : Uoff[size_t(k) * p + (j - k - 1)]; };
  auto Lg = [&](int i, int k) -> double { return L[size_t(i) * p + (i - k - 1)]; };
  double minratio = 1e300;
  for (int i = 0; i < n; ++i) {
    for (int j = std::max(0, i - p); j < i; ++j) {
      double s = A(i, j);
      for (int k = std::max(0, i - p); k < j; ++k)
        if (j - k <= p) s -= Lg(i, k) * U(k, j);
      L[size_t(i) * p + (i - j - 1)] = s / Ud[j];
    }
    for (int j = i; j <= std::min(n - 1, i + p); ++j) {
      double s = A(i, j);
      for (int k = std::max({0, i - p, j - p}); k < i; ++k) s -= Lg(i, k) * U(k, j);
      if (j == i) Ud[i] = s;
      else Uoff[size_t(i) * p + (j - i - 1)] = s;
    }
    const double ratio = std::fabs(Ud[i]) / std::fabs(A(i, i));
    if (ratio < minratio) minratio = ratio;
    Uinv[i] = 1.0 / Ud[i];
  }
  return minratio;
}

// ------------------------------------------------------------ partitioned solve
// A banded matrix (bandwidth p each side) split into S row segments
// [b_i, b_{i+1}) is solved as: local solves with the block diagonal, then a
// small reduced system for the p unknowns on either side of every segment
// boundary, then a correction with the spikes (the block diagonal's inverse
// applied to the couplings across the boundaries).
namespace {

// Forward / backward substitution with the factors of band_lu (DU = D * U).
void lu_solve(const std::vector<double>& L, const std::vector<double>& DU,
              const std::vector<double>& D, int n, int p, std::vector<double>& x) {
  for (int r = 0; r < n; ++r)
    for (int k = 1; k <= p && r - k >= 0; ++k) x[r] -= L[size_t(r) * p + k - 1] * x[r - k];
  for (int r = n - 1; r >= 0; --r) {
    double s = D[r] * x[r];
    for (int k = 1; k <= p && r + k < n; ++k) s -= DU[size_t(r) * p + k - 1] * x[r + k];
    x[r] = s;
  }
}

// Gauss-Jordan inverse with partial pivoting (q x q, row-major); false if singular.
bool dense_inverse(std::vector<double> a, int q, std::vector<double>& inv) {
  inv.assign(size_t(q) * q, 0.0);
  for (int i = 0; i < q; ++i) inv[size_t(i) * q + i] = 1.0;
  for (int c = 0; c < q; ++c) {
    int piv = c;
    for (int r = c + 1; r < q; ++r)
      if (std::fabs(a[size_t(r) * q + c]) > std::fabs(a[size_t(piv) * q + c])) piv = r;
    if (!(std::fabs(a[size_t(piv) * q + c]) > 1e-300)) return false;
    if (piv != c)
      for (int j = 0; j < q; ++j) {
        std::swap(a[size_t(c) * q + j], a[size_t(piv) * q + j]);
        std::swap(inv[size_t(c) * q + j], inv[size_t(piv) * q + j]);
      }
    const double d = 1.0 / a[size_t(c) * q + c];
    for (int j = 0; j < q; ++j) {
      a[size_t(c) * q + j] *= d;
      inv[size_t(c) * q + j] *= d;
    }
    for (int r = 0; r < q; ++r) {
      if (r == c) continue;
      const double f = a[size_t(r) * q + c];
      if (f == 0.0) continue;
      for (int j = 0; j < q; ++j) {
        a[size_t(r) * q + j] -= f * a[size_t(c) * q + j];
        inv[size_t(r) * q + j] -= f * inv[size_t(c) * q + j];
      }
    }
  }
  return true;
}

}  // namespace

int spike_boundary(int n, int S, int i) { return int((long(i) * n) / S); }

bool spike_prepare(const std::vector<double>& band, int n, int p, int S, SpikeData& out) {
  const int w = 2 * p + 1, q = 2 * p * (S - 1);
  for (int i = 0; i < S; ++i)
    if (spike_boundary(n, S, i + 1) - spike_boundary(n, S, i) < 2 * p) return false;
  std::vector<int> seg(n);
  for (int i = 0; i < S; ++i)
    for (int r = spike_boundary(n, S, i); r < spike_boundary(n, S, i + 1); ++r) seg[r] = i;
  auto A = [&](int r, int c) -> double {
    if (c < 0 || c >= n || c - r > p || r - c > p) return 0.0;
    return band[size_t(r) * w + (c - r + p)];
  };
  // block diagonal (couplings across segment boundaries removed) and its LU
  std::vector<double> blk(band);
  for (int r = 0; r < n; ++r)
    for (int d = 0; d < w; ++d) {
      const int c = r + d - p;
      if (c >= 0 && c < n && seg[c] != seg[r]) blk[size_t(r) * w + d] = 0.0;
    }
  std::vector<double> L, U, Dinv;
  const double ratio = band_lu(blk, n, p, L, U, Dinv);
  if (!(ratio > 1e-14)) return false;
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < p; ++k) U[size_t(r) * p + k] *= Dinv[r];
  // spikes: V[:, k] = blockdiag^-1 (coupling to x[b_{i+1} + k]) for rows of
  // segment i < S-1; W[:, k] = blockdiag^-1 (coupling to x[b_i - p + k]) for i > 0
  std::vector<double> V(size_t(n) * p, 0.0), Wv(size_t(n) * p, 0.0), col(n);
  for (int k = 0; k < p; ++k) {
    for (int r = 0; r < n; ++r) {
      const int i = seg[r];
      col[r] = (i < S - 1) ? A(r, spike_boundary(n, S, i + 1) + k) : 0.0;
    }
    lu_solve(L, U, Dinv, n, p, col);
    for (int r = 0; r < n; ++r) V[size_t(r) * p + k] = col[r];
    for (int r = 0; r < n; ++r) {
      const int i = seg[r];
      col[r] = (i > 0) ? A(r, spike_boundary(n, S, i) - p + k) : 0.0;
    }
    lu_solve(L, U, Dinv, n, p, col);
    for (int r = 0; r < n; ++r) Wv[size_t(r) * p + k] = col[r];
  }
  // reduced system on z = [U_0, T_1, U_1, T_2, ..., U_{S-2}, T_{S-1}] (p each):
  // U_i = bottom p rows of segment i, T_i = top p rows of segment i;
  // x_i = g_i - V_i T_{i+1} - W_i U_{i-1} restricted to those rows.
  auto zU = [&](int i, int j) { return 2 * p * i + j; };
  auto zT = [&](int i, int j) { return 2 * p * (i - 1) + p + j; };
  std::vector<double> K(size_t(q) * q, 0.0);
  for (int i = 0; i < S; ++i) {
    const int b0 = spike_boundary(n, S, i), b1 = spike_boundary(n, S, i + 1);
    for (int side = 0; side < 2; ++side) {  // 0: U_i (bottom rows), 1: T_i (top rows)
      if (side == 0 && i == S - 1) continue;
      if (side == 1 && i == 0) continue;
      for (int j = 0; j < p; ++j) {
        const int r = side == 0 ? b1 - p + j : b0 + j;
        const int row = side == 0 ? zU(i, j) : zT(i, j);
        K[size_t(row) * q + row] += 1.0;
        for (int k = 0; k < p; ++k) {
          if (i < S - 1) K[size_t(row) * q + zT(i + 1, k)] += V[size_t(r) * p + k];
          if (i > 0) K[size_t(row) * q + zU(i - 1, k)] += Wv[size_t(r) * p + k];
        }
      }
    }
  }
  std::vector<double> R;
  if (!dense_inverse(K, q, R)) return false;

  // self-check against the direct banded solve on a fixed right-hand side
  std::vector<double> La, Ua, Da;
  band_lu(band, n, p, La, Ua, Da);
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < p; ++k) Ua[size_t(r) * p + k] *= Da[r];
  std::vector<double> b(n), ref(n), g(n);
  for (int r = 0; r < n; ++r) b[r] = std::sin(0.7 * r + 0.3) + 0.25 * std::cos(2.1 * r);
  ref = b;
  lu_solve(La, Ua, Da, n, p, ref);
  g = b;
  lu_solve(L, U, Dinv, n, p, g);
  std::vector<double> gz(q), z(q, 0.0);
  for (int i = 0; i + 1 < S; ++i) {
    const int b1 = spike_boundary(n, S, i + 1);
    for (int j = 0; j < p; ++j) {
      gz[zU(i, j)] = g[b1 - p + j];
      gz[zT(i + 1, j)] = g[b1 + j];
    }
  }
  for (int r = 0; r < q; ++r)
    for (int c = 0; c < q; ++c) z[r] += R[size_t(r) * q + c] * gz[c];
  double err = 0.0, nrm = 0.0;
  for (int r = 0; r < n; ++r) {
    const int i = seg[r];
    double x = g[r];
    for (int k = 0; k < p; ++k) {
      if (i < S - 1) x -= V[size_t(r) * p + k] * z[zT(i + 1, k)];
      if (i > 0) x -= Wv[size_t(r) * p + k] * z[zU(i - 1, k)];
    }
    err = std::max(err, std::fabs(x - ref[r]));
    nrm = std::max(nrm, std::fabs(ref[r]));
  }
  if (!(err <= 1e-12 * nrm)) return false;

  out.S = S;
  out.q = q;
  out.L = std::move(L);
  out.DU = std::move(U);
  out.D = std::move(Dinv);
  out.V = std::move(V);
  out.W = std::move(Wv);
  out.R = std::move(R);
  return true;
}

std::vector<double> voxel_weights(int N, int p, int V) {
  // Fraction of the integral of each B-spline over each voxel: pieces of
  // the voxel between knots are integrated with (p+1)-point Gauss rules
  // (exact on polynomial pieces), then every row is normalised.
  const int n = N + p;
  const std::vector<double> t = open_knots(N, p);
  std::vector<double> gx, gw;
  gauss_legendre(p + 1, gx, gw);
  std::vector<double> W(size_t(n) * V, 0.0), vals(p + 1);
  for (int v = 0; v < V; ++v) {
    const double a = double(v) / V, b = double(v + 1) / V;
    std::vector<double> cuts{a};
    for (int e = 1; e < N; ++e) {
      const double k = double(e) / N;
      if (k > a && k < b) cuts.push_back(k);
    }
    cuts.push_back(b);
    for (size_t c = 0; c + 1 < cuts.size(); ++c) {
      const double lo = cuts[c], hi = cuts[c + 1], half = 0.5 * (hi - lo);
      for (int g = 0; g <= p; ++g) {
        const double x = 0.5 * (lo + hi) + half * gx[g];
        const int span = find_span(t, p, n, x);
        basis_on_span(t, p, span, x, vals.data(), nullptr);
        for (int r = 0; r <= p; ++r) W[size_t(span - p + r) * V + v] += half * gw[g] * vals[r];
      }
    }
  }
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int v = 0; v < V; ++v) s += W[size_t(i) * V + v];
    for (int v = 0; v < V; ++v) W[size_t(i) * V + v] /= s;
  }
  return W;
}

std::vector<double> greville(int N, int p) {
  std::vector<double> t = open_knots(N, p), xi(N + p);
  for (int i = 0; i < N + p; ++i) {
    if (p == 0) {
      xi[i] = 0.5 * (t[i] + t[i + 1]);
      continue;
    }
    double s = 0.0;
    for (int k = 1; k <= p; ++k) s += t[i + k];
    xi[i] = s / p;
  }
  return xi;
}

void basis_at(int N, int p, double x, int* first, double* vals) {
  std::vector<double> t = open_knots(N, p);
  const int n = N + p;
  const int span = find_span(t, p, n, x);
  basis_on_span(t, p, span, x, vals, nullptr);
  *first = span - p;
}

}  // namespace adimx
