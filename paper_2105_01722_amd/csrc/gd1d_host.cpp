// Host construction of the 1D Galerkin-difference element data (FP64).
//
// Sec. 2.1 (eq. GD_basis_lagrange and the nodal form) with the extrapolation
// closure of Sec. 2.1.1: on cell k of a unit-spaced grid 0..N the GD function is
// the degree-p interpolant on the p+1 nodes starting at
// s_k = clamp(k - (p-1)/2, 0, N-p).  In the interior that is the centred stencil of
// the generating function; next to a boundary every stencil value lies on the
// degree-p extrapolant through the first (last) p+1 nodes, so the cell polynomial
// is that extrapolant.
//
// Produced (unit spacing; the caller scales by h = H/N):
//   M_hat[i][j] = sum_k int_k^{k+1} phi_i phi_j,  S_hat[i][j] = sum_k int phi_i' phi_j'
//   (Sec. 3.1), and the non-zeros of D-tilde: dL[i] = phi_i'(0), dR[i] = phi_i'(N)
//   (Sec. 3.2).  phi_i(0) = delta_i0 and phi_i(N) = delta_iN (interpolatory basis).
#include <cmath>
#include <vector>

#include "gdw_internal.h"

namespace gdw {

// Gauss-Legendre rule with n points on [0, 1] (Newton iteration on P_n).
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = pk;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = pk;
    }
    if (n == 1) { p1 = z; p0 = 1.0; }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);   // 2/((1-z^2)P'^2) on [-1,1], halved
  }
}

// Lagrange basis on nodes[0..m-1] at t: values and first derivatives.
static void lagrange(const double* nodes, int m, double t, double* val, double* der) {
  for (int a = 0; a < m; ++a) {
    double v = 1.0;
    for (int b = 0; b < m; ++b)
      if (b != a) v *= (t - nodes[b]) / (nodes[a] - nodes[b]);
    val[a] = v;
    double d = 0.0;
    for (int b = 0; b < m; ++b) {
      if (b == a) continue;
      double prod = 1.0 / (nodes[a] - nodes[b]);
      for (int c = 0; c < m; ++c)
        if (c != a && c != b) prod *= (t - nodes[c]) / (nodes[a] - nodes[c]);
      d += prod;
    }
    der[a] = d;
  }
}

int gd_window_start(int k, int N, int p) {
  int s = k - (p - 1) / 2;
  if (s < 0) s = 0;
  if (s > N - p) s = N - p;
  return s;
}

void gd1d_unit(int N, int p, double* M, double* S, double* dL, double* dR) {
  const int n1 = N + 1, m = p + 1;
  std::vector<double> xg(m), wg(m), nodes(m), val(m), der(m);
  gauss_legendre01(m, xg.data(), wg.data());
  for (int i = 0; i < n1 * n1; ++i) M[i] = S[i] = 0.0;
  for (int k = 0; k < N; ++k) {
    const int s = gd_window_start(k, N, p);
    for (int a = 0; a < m; ++a) nodes[a] = double(s + a);
    for (int g = 0; g < m; ++g) {
      lagrange(nodes.data(), m, k + xg[g], val.data(), der.data());
      for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
          M[(s + a) * n1 + (s + b)] += wg[g] * val[a] * val[b];
          S[(s + a) * n1 + (s + b)] += wg[g] * der[a] * der[b];
        }
    }
  }
  for (int i = 0; i < n1; ++i) dL[i] = dR[i] = 0.0;
  {
    for (int a = 0; a < m; ++a) nodes[a] = double(a);
    lagrange(nodes.data(), m, 0.0, val.data(), der.data());
    for (int a = 0; a < m; ++a) dL[a] = der[a];
    const int s = N - p;
    for (int a = 0; a < m; ++a) nodes[a] = double(s + a);
    lagrange(nodes.data(), m, double(N), val.data(), der.data());
    for (int a = 0; a < m; ++a) dR[s + a] = der[a];
  }
}

// Basis values / t-derivatives of all N+1 functions at a point t in cell k.
void gd1d_eval_cell(int N, int p, int k, double t, double* val, double* der) {
  const int n1 = N + 1, m = p + 1;
  double nodes[64], v[64], d[64];
  const int s = gd_window_start(k, N, p);
  for (int a = 0; a < m; ++a) nodes[a] = double(s + a);
  lagrange(nodes, m, t, v, d);
  for (int i = 0; i < n1; ++i) val[i] = der[i] = 0.0;
  for (int a = 0; a < m; ++a) {
    val[s + a] = v[a];
    der[s + a] = d[a];
  }
}

}  // namespace gdw
