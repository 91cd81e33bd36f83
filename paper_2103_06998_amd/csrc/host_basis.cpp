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
