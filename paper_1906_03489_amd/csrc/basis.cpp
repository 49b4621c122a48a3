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
#include <algorithm>
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

// n Gauss-Radau points (x = -1 included) and weights of the weight
// (1-x)^alpha on [-1, 1] (the eta_3 rule of tetrahedra uses alpha = 2).  The
// interior points are the roots of P^{alpha,1}_{n-1}: eigenvalues of its
// symmetric tridiagonal recurrence matrix (Golub-Welsch), found by
// symmetric_eigen and polished by Newton steps on the three-term recurrence;
// the weights are fixed by exactness on 1, x, ..., x^{n-1}, the moments of
// (1-x)^alpha in closed form (binomial expansion), solved by Gaussian
// elimination with partial pivoting.
void radau_points(int n, int alpha, double* x, double* w) {
  x[0] = -1.0;
  const int m = n - 1;
  if (m > 0) {
    const double a = alpha, b = 1.0;
    std::vector<double> T(m * m, 0.0), V(m * m), lam(m);
    for (int k = 0; k < m; ++k) {
      const double c = 2.0 * k + a + b;
      T[k * m + k] = (k == 0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (c * (c + 2.0));
      if (k + 1 < m) {
        const double kk = k + 1.0, c1 = 2.0 * kk + a + b;
        const double off = std::sqrt(4.0 * kk * (kk + a) * (kk + b) * (kk + a + b) /
                                     (c1 * c1 * (c1 + 1.0) * (c1 - 1.0)));
        T[k * m + k + 1] = T[(k + 1) * m + k] = off;
      }
    }
    symmetric_eigen(m, T.data(), V.data(), lam.data());
    std::sort(lam.begin(), lam.end());
    for (int k = 0; k < m; ++k) {
      double r = lam[k];
      for (int it = 0; it < 20; ++it) {   // Newton: P' = (m + a + b + 1)/2 P^{a+1,b+1}_{m-1}
        const double f = jacobi_poly(m, a, b, r);
        const double df = 0.5 * (m + a + b + 1.0) * jacobi_poly(m - 1, a + 1.0, b + 1.0, r);
        const double dr = f / df;
        r -= dr;
        if (std::fabs(dr) < 1e-16) break;
      }
      x[k + 1] = r;
    }
  }
  // moments int_{-1}^{1} x^k (1-x)^alpha dx = sum_l binom(alpha, l) (-1)^l int x^{k+l}
  std::vector<double> A(n * n), rhs(n);
  for (int k = 0; k < n; ++k) {
    double mk = 0.0, bin = 1.0;
    for (int l = 0; l <= alpha; ++l) {
      const int d = k + l;
      const double ik = (d % 2 == 0) ? 2.0 / (d + 1) : 0.0;
      mk += ((l % 2) ? -bin : bin) * ik;
      bin = bin * (alpha - l) / (l + 1.0);
    }
    rhs[k] = mk;
    for (int j = 0; j < n; ++j) A[k * n + j] = std::pow(x[j], k);
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
    for (int j = c + 1; j < n; ++j) s -= A[c * n + j] * w[j];
    w[c] = s / A[c * n + c];
  }
}

// Collapsed tetrahedron quadrature: GLL (Q) in eta_1, Radau of (1-x) (Q-1)
// in eta_2, Radau of (1-x)^2 (Q-1) in eta_3.
void tet_points(int Q, double* e1, double* w1, double* e2, double* w2, double* e3, double* w3) {
  tri_points(Q, e1, w1, e2, w2);
  radau_points(Q - 1, 2, e3, w3);
}

// Total polynomial degree of triangle mode (p, q) of order P.
int tri_mode_degree(int P, int p, int q) {
  if ((p == 0 || p == P) && q == 0) return 1;   // vertices A, B
  if (p == 0 && q == P) return 1;               // vertex C
  if (p == 0 || p == P) return q + 1;           // edges AC, BC
  if (q == 0) return p + 1;                     // edge AB
  return p + q + 1;                             // interior
}

// The eta_3 factor of a collapsed-shape mode whose lower part has degree s:
// ((1-x)/2)^s for r = 0, times (1+x)/2 P^{2s-1,1}_{r-1}(x) for r >= 1; value
// and derivative.
static void cfactor(int s, int r, double x, double* v, double* d) {
  const double a = 0.5 * (1.0 - x), g = 0.5 * (1.0 + x);
  const double f = std::pow(a, s), df = s > 0 ? -0.5 * s * std::pow(a, s - 1) : 0.0;
  if (r == 0) {
    *v = f;
    *d = df;
    return;
  }
  const double J = jacobi_poly(r - 1, 2.0 * s - 1.0, 1.0, x);
  const double dJ = r >= 2 ? 0.5 * (r + 2.0 * s) * jacobi_poly(r - 2, 2.0 * s, 2.0, x) : 0.0;
  *v = f * g * J;
  *d = df * g * J + f * 0.5 * J + f * g * dJ;
}

// eta_3 factor of every tetrahedron mode at the points z (values and
// derivatives, [nz][nm3]): modes grouped by triangle mode t (degree s),
// r = 0..P-s; the top vertex (1+z)/2 last.
void tet_ctable(int P, int nz, const double* z, double* Ct, double* dCt) {
  const int nm3 = (P + 1) * (P + 2) * (P + 3) / 6;
  for (int k = 0; k < nz; ++k) {
    int m = 0;
    for (int p = 0; p <= P; ++p) {
      const int nq = p == 0 ? P + 1 : (p == P ? P : P - p);
      for (int q = 0; q < nq; ++q) {
        const int s = tri_mode_degree(P, p, q);
        for (int r = 0; r <= P - s; ++r, ++m) cfactor(s, r, z[k], &Ct[k * nm3 + m], &dCt[k * nm3 + m]);
      }
    }
    Ct[k * nm3 + m] = 0.5 * (1.0 + z[k]);   // top vertex
    dCt[k * nm3 + m] = 0.5;
  }
}

// Degree of the 1-D modified basis function p of order P.
int mod_degree(int P, int p) { return (p == 0 || p == P) ? 1 : p + 1; }

// eta_3 factor of every pyramid mode at the points z ([nz][nm]): modes
// grouped by base mode (p slow, q fast) with s = max(deg p, deg q),
// r = 0..P-s; the apex (1+z)/2 last.
void pyr_ctable(int P, int nz, const double* z, double* Ct, double* dCt) {
  const int nm = (P + 1) * (P + 2) * (2 * P + 3) / 6;
  for (int k = 0; k < nz; ++k) {
    int m = 0;
    for (int p = 0; p <= P; ++p)
      for (int q = 0; q <= P; ++q) {
        const int s = std::max(mod_degree(P, p), mod_degree(P, q));
        for (int r = 0; r <= P - s; ++r, ++m) cfactor(s, r, z[k], &Ct[k * nm + m], &dCt[k * nm + m]);
      }
    Ct[k * nm + m] = 0.5 * (1.0 + z[k]);   // apex
    dCt[k * nm + m] = 0.5;
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
