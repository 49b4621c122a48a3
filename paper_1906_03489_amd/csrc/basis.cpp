// Host-side 1-D quadrature and basis tables (section 2.1 of arXiv 1906.03489).
//
// GLL points: the interior points are the zeros of L_N' (L_N the Legendre
// polynomial of degree N = Q-1), found by Newton's method from the
// Chebyshev-Gauss-Lobatto points, with L_N'' taken from Legendre's
// differential equation.  Weights w_i = 2 / (N (N+1) L_N(x_i)^2).
//
// Modified basis: the bubble of the section 2.1 display equals
//   phi_p(x) = (1-x)/2 (1+x)/2 P^{1,1}_{p-1}(x) = (1 - x^2) L_p'(x) / (2 (p+1)),
// since P^{1,1}_{p-1} = 2 L_p' / (p+1); Legendre's equation then gives the
// derivative in closed form, phi_p'(x) = -(p/2) L_p(x).  Both need only the
// Legendre three-term recurrence.
#include <cmath>
#include <vector>

#include "nk_internal.h"

namespace nk {

// L_k(x) and L_k'(x) for k = 0..kmax.
static void legendre_all(int kmax, double x, double* L, double* dL) {
  L[0] = 1.0;
  dL[0] = 0.0;
  if (kmax >= 1) {
    L[1] = x;
    dL[1] = 1.0;
  }
  for (int k = 1; k < kmax; ++k) {
    L[k + 1] = ((2.0 * k + 1.0) * x * L[k] - k * L[k - 1]) / (k + 1.0);
    // derivative recurrence: L_{k+1}' = L_{k-1}' + (2k+1) L_k
    dL[k + 1] = dL[k - 1] + (2.0 * k + 1.0) * L[k];
  }
}

void gll_points(int Q, double* x, double* w) {
  const int N = Q - 1;
  std::vector<double> L(N + 2), dL(N + 2);
  for (int i = 0; i < Q; ++i) {
    double xi;
    if (i == 0) {
      xi = -1.0;
    } else if (i == N) {
      xi = 1.0;
    } else {
      xi = -std::cos(M_PI * i / N);
      for (int it = 0; it < 100; ++it) {
        legendre_all(N, xi, L.data(), dL.data());
        // L_N'' from (1 - x^2) L'' - 2 x L' + N (N+1) L = 0
        double d2 = (2.0 * xi * dL[N] - N * (N + 1.0) * L[N]) / (1.0 - xi * xi);
        double dx = dL[N] / d2;
        xi -= dx;
        if (std::fabs(dx) < 1e-17) break;
      }
    }
    x[i] = xi;
  }
  // symmetrise (points come in +-pairs) and evaluate weights
  for (int i = 0; i < Q / 2; ++i) {
    double a = 0.5 * (x[Q - 1 - i] - x[i]);
    x[i] = -a;
    x[Q - 1 - i] = a;
  }
  if (Q % 2 == 1) x[Q / 2] = 0.0;
  for (int i = 0; i < Q; ++i) {
    legendre_all(N, x[i], L.data(), dL.data());
    w[i] = 2.0 / (N * (N + 1.0) * L[N] * L[N]);
  }
}

void modified_basis(int P, int Q, const double* x, double* B, double* DB) {
  const int n = P + 1;
  std::vector<double> L(P + 2), dL(P + 2);
  for (int i = 0; i < Q; ++i) {
    const double xi = x[i];
    legendre_all(P, xi, L.data(), dL.data());
    for (int p = 0; p < n; ++p) {
      double b, db;
      if (p == 0) {
        b = 0.5 * (1.0 - xi);
        db = -0.5;
      } else if (p == P) {
        b = 0.5 * (1.0 + xi);
        db = 0.5;
      } else {
        b = (1.0 - xi * xi) * dL[p] / (2.0 * (p + 1.0));
        db = -0.5 * p * L[p];
      }
      B[i * n + p] = b;
      DB[i * n + p] = db;
    }
  }
}

}  // namespace nk
