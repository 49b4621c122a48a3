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
#include <utility>
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

// Derivative matrix of the Lagrange interpolant through the Q nodes x:
// Dc[i*Q + j] = l_j'(x_i), from the barycentric weights b_j = 1 / prod_{k != j}
// (x_j - x_k): l_j'(x_i) = (b_j / b_i) / (x_i - x_j) off the diagonal, and each
// row sums to zero (constants have zero derivative).
void collocation_derivative(int Q, const double* x, double* Dc) {
  std::vector<double> b(Q, 1.0);
  for (int j = 0; j < Q; ++j)
    for (int k = 0; k < Q; ++k)
      if (k != j) b[j] *= x[j] - x[k];
  for (int j = 0; j < Q; ++j) b[j] = 1.0 / b[j];
  for (int i = 0; i < Q; ++i) {
    double diag = 0.0;
    for (int j = 0; j < Q; ++j) {
      if (j == i) continue;
      const double v = (b[j] / b[i]) / (x[i] - x[j]);
      Dc[i * Q + j] = v;
      diag -= v;
    }
    Dc[i * Q + i] = diag;
  }
}

// Eigen-decomposition of the symmetric n x n matrix A (row-major) by cyclic
// Jacobi rotations: A = V diag(lam) V^T, eigenvectors in the columns of V.
void symmetric_eigen(int n, const double* A, double* V, double* lam) {
  std::vector<double> a(A, A + n * n);
  for (int i = 0; i < n * n; ++i) V[i] = 0.0;
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += a[i * n + j] * a[i * n + j];
        if (i != j) off += a[i * n + j] * a[i * n + j];
      }
    if (off <= 1e-34 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        // rotation angle that annihilates a[p][q]
        const double theta = (a[q * n + q] - a[p * n + p]) / (2.0 * apq);
        const double tt = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          const double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) lam[i] = a[i * n + i];
}

// P_k^{(a,b)}(x) by the textbook three-term recurrence in k.
static double jacobi_poly(int k, double a, double b, double x) {
  if (k < 0) return 0.0;
  double p0 = 1.0;
  if (k == 0) return p0;
  double p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
  for (int n = 1; n < k; ++n) {
    const double c = 2.0 * n + a + b;
    const double a1 = 2.0 * (n + 1) * (n + a + b + 1) * c;
    const double a2 = (c + 1) * (a * a - b * b);
    const double a3 = c * (c + 1) * (c + 2);
    const double a4 = 2.0 * (n + a) * (n + b) * (c + 2);
    const double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Collapsed triangle quadrature: Q Gauss-Lobatto-Legendre points in eta_1
// and Q-1 Gauss-Radau points of the weight (1 - eta_2) in eta_2 (-1
// included).  The Radau interior points are the roots of P^{1,1}_{Q-2}, i.e.
// the interior GLL points of order Q; the weights are fixed by exactness on
// 1, x, ..., x^{Q-2} (moments of (1-x) in closed form), solved by Gaussian
// elimination with partial pivoting.
void tri_points(int Q, double* e1, double* w1, double* e2, double* w2) {
  gll_points(Q, e1, w1);
  const int n = Q - 1;
  e2[0] = -1.0;
  for (int k = 1; k < n; ++k) e2[k] = e1[k];
  std::vector<double> A(n * n), rhs(n);
  for (int k = 0; k < n; ++k) {
    const double ik = (k % 2 == 0) ? 2.0 / (k + 1) : 0.0;        // int x^k
    const double ik1 = ((k + 1) % 2 == 0) ? 2.0 / (k + 2) : 0.0; // int x^(k+1)
    rhs[k] = ik - ik1;
    for (int j = 0; j < n; ++j) A[k * n + j] = std::pow(e2[j], k);
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(rhs[c], rhs[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      rhs[r] -= f * rhs[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = rhs[c];
    for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * w2[j];
    w2[c] = s / A[c * n + c];
  }
}

// eta_2 factor of every triangle mode at the points z (values and
// derivatives, [nz][nmodes]); modes grouped by the eta_1 index p: p = 0 with
// q = 0..P (q = P the collapsed vertex (1+z)/2), 0 < p < P with
// q = 0..P-1-p, p = P with q = 0..P-1.
void tri_btable(int P, int nz, const double* z, double* Bt, double* dBt) {
  const int nm = (P + 1) * (P + 2) / 2;
  std::vector<double> L(P + 2), dL(P + 2);
  for (int j = 0; j < nz; ++j) {
    const double x = z[j];
    legendre_all(P, x, L.data(), dL.data());
    int m = 0;
    for (int p = 0; p <= P; ++p) {
      const int nq = p == 0 ? P + 1 : (p == P ? P : P - p);
      for (int q = 0; q < nq; ++q, ++m) {
        double v, d;
        if (p == 0 || p == P) {
          if (q == 0) {
            v = 0.5 * (1.0 - x);
            d = -0.5;
          } else if (p == 0 && q == P) {
            v = 0.5 * (1.0 + x);
            d = 0.5;
          } else {  // 1-D bubble q
            v = (1.0 - x * x) * dL[q] / (2.0 * (q + 1.0));
            d = -0.5 * q * L[q];
          }
        } else {
          const double a = 0.5 * (1.0 - x);
          const double ap = std::pow(a, p), ap1 = ap * a;
          if (q == 0) {
            v = ap1;
            d = -0.5 * (p + 1) * ap;
          } else {
            const double f = ap1 * 0.5 * (1.0 + x);
            const double df = -0.5 * (p + 1) * ap * 0.5 * (1.0 + x) + 0.5 * ap1;
            const double J = jacobi_poly(q - 1, 2.0 * p + 1, 1.0, x);
            const double dJ = q >= 2 ? 0.5 * (q + 2.0 * p + 2) * jacobi_poly(q - 2, 2.0 * p + 2, 2.0, x) : 0.0;
            v = f * J;
            d = df * J + f * dJ;
          }
        }
        Bt[j * nm + m] = v;
        dBt[j * nm + m] = d;
      }
    }
  }
}

}  // namespace nk
