// Per-point geometric factors of the element maps chi_e (section 2.1) and the
// elemental Helmholtz diagonal used by the Jacobi preconditioner.
#include "nk_internal.h"

namespace nk {

// One thread per (element, point).  J[e][c][a][q] = d x_c / d xi_a.  Writes
// factor f of point q = i + Q t (t = j + Q k in 3-D, t = j in 2-D) at
// ((e*NF + f)*Q + i)*Q^(d-1) + t, with f = 0: w detJ, then the upper triangle
// of w detJ kappa J^{-1} J^{-T} row by row.  The derivative factors go to
// dfac[(e*(d*d+1) + g)*Q^d + q]: g = a*d + c for (J^{-1})_{ac} = d xi_a / d x_c,
// g = d*d for w detJ.
template <int D>
__global__ void __launch_bounds__(256)
    k_geom(int Q, int64_t nelem, const double* __restrict__ jac, const double* __restrict__ kappa,
           const double* __restrict__ wq, double* __restrict__ fac64, float* __restrict__ fac32,
           double* __restrict__ dfac64, float* __restrict__ dfac32, int* __restrict__ bad) {
  const int QD = D == 3 ? Q * Q * Q : Q * Q;
  const int QT = QD / Q;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * QD) return;
  const int64_t e = id / QD;
  const int q = (int)(id - e * QD);
  const int i = q % Q, t = q / Q;
  double J[D][D];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int a = 0; a < D; ++a) J[c][a] = jac[((e * D + c) * D + a) * QD + q];
  double w = wq[i];
  {
    int r = t;
#pragma unroll
    for (int a = 1; a < D; ++a) {
      w *= wq[r % Q];
      r /= Q;
    }
  }
  const double kap = kappa ? kappa[e * QD + q] : 1.0;
  constexpr int NF = D == 3 ? kNF3 : kNF2;
  double f[NF];
  double det;
  if constexpr (D == 3) {
    // inverse by cofactors: Jinv[a][c] = cof(J)[c][a] / det
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id_ = 1.0 / det;
    double Ji[3][3];
    Ji[0][0] = c00 * id_;
    Ji[1][0] = c01 * id_;
    Ji[2][0] = c02 * id_;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id_;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id_;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id_;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id_;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id_;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id_;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t o = (e * 10 + a * 3 + c) * QD + q;
        dfac64[o] = Ji[a][c];
        dfac32[o] = (float)Ji[a][c];
      }
    const double s = w * det * kap;
    int k = 1;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = a; b < 3; ++b) {
        f[k++] = s * (Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1] + Ji[a][2] * Ji[b][2]);
      }
  } else {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double id_ = 1.0 / det;
    const double Ji[2][2] = {{J[1][1] * id_, -J[0][1] * id_}, {-J[1][0] * id_, J[0][0] * id_}};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int64_t o = (e * 5 + a * 2 + c) * QD + q;
        dfac64[o] = Ji[a][c];
        dfac32[o] = (float)Ji[a][c];
      }
    const double s = w * det * kap;
    f[1] = s * (Ji[0][0] * Ji[0][0] + Ji[0][1] * Ji[0][1]);
    f[2] = s * (Ji[0][0] * Ji[1][0] + Ji[0][1] * Ji[1][1]);
    f[3] = s * (Ji[1][0] * Ji[1][0] + Ji[1][1] * Ji[1][1]);
  }
  f[0] = w * det;
  {
    const int64_t o = (e * (D * D + 1) + D * D) * QD + q;
    dfac64[o] = w * det;
    dfac32[o] = (float)(w * det);
  }
  if (!(det > 0.0) || !(kap > 0.0)) atomicOr(bad, 1);
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int64_t o = ((e * NF + k) * Q + i) * QT + t;
    fac64[o] = f[k];
    fac32[o] = (float)f[k];
  }
}

hipError_t launch_geom(int dim, int Q, int64_t nelem, const double* jac, const double* kappa,
                       const double* wq, double* fac64, float* fac32, double* dfac64,
                       float* dfac32, int* bad, hipStream_t s) {
  const int64_t QD = dim == 3 ? (int64_t)Q * Q * Q : (int64_t)Q * Q;
  const int64_t n = nelem * QD;
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  if (dim == 3)
    hipLaunchKernelGGL(k_geom<3>, dim3((unsigned)nb), dim3(256), 0, s, Q, nelem, jac, kappa, wq,
                       fac64, fac32, dfac64, dfac32, bad);
  else
    hipLaunchKernelGGL(k_geom<2>, dim3((unsigned)nb), dim3(256), 0, s, Q, nelem, jac, kappa, wq,
                       fac64, fac32, dfac64, dfac32, bad);
  return hipGetLastError();
}

// Elemental Helmholtz diagonal, scattered to the global numbering.  One
// thread per (element, mode); loops over the points.  With v_a the reference
// gradient of phi_m and phi_m its value at a point,
//   diag H_e[m] = sum_points ( sum_ab G'_ab v_a v_b + lambda w detJ phi_m^2 ).
// B and D are the 1-D tables [Q][n] in device memory.
template <int D>
__global__ void __launch_bounds__(256)
    k_diag(int P, int Q, int64_t nelem, const double* __restrict__ Bt, const double* __restrict__ Dt,
           const double* __restrict__ fac, const double* __restrict__ lam, double lam0,
           const int32_t* __restrict__ l2g, double* __restrict__ diag) {
  const int n = P + 1;
  const int ND = D == 3 ? n * n * n : n * n;
  const int QD = D == 3 ? Q * Q * Q : Q * Q;
  const int QT = QD / Q;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * ND) return;
  const int64_t e = id / ND;
  const int m = (int)(id - e * ND);
  const int32_t g = l2g[e * ND + m];
  if (g < 0) return;  // Dirichlet: row replaced by the identity
  const int p = m % n, q = (m / n) % n, r = m / (n * n);
  const double lm = lam ? lam[e] : lam0;
  constexpr int NF = D == 3 ? kNF3 : kNF2;
  const double* fe = fac + e * (int64_t)NF * QD;
  double s = 0.0;
  if constexpr (D == 3) {
    for (int k = 0; k < Q; ++k) {
      const double b3 = Bt[k * n + r], d3 = Dt[k * n + r];
      for (int j = 0; j < Q; ++j) {
        const double b2 = Bt[j * n + q], d2 = Dt[j * n + q];
        const int t = j + Q * k;
        for (int i = 0; i < Q; ++i) {
          const double b1 = Bt[i * n + p], d1 = Dt[i * n + p];
          const double v1 = d1 * b2 * b3, v2 = b1 * d2 * b3, v3 = b1 * b2 * d3, ph = b1 * b2 * b3;
          const double* fp = fe + (int64_t)i * QT + t;
          const double wj = fp[0], G11 = fp[QD], G12 = fp[2 * QD], G13 = fp[3 * QD],
                       G22 = fp[4 * QD], G23 = fp[5 * QD], G33 = fp[6 * QD];
          s += G11 * v1 * v1 + G22 * v2 * v2 + G33 * v3 * v3 +
               2.0 * (G12 * v1 * v2 + G13 * v1 * v3 + G23 * v2 * v3) + lm * wj * ph * ph;
        }
      }
    }
  } else {
    for (int j = 0; j < Q; ++j) {
      const double b2 = Bt[j * n + q], d2 = Dt[j * n + q];
      for (int i = 0; i < Q; ++i) {
        const double b1 = Bt[i * n + p], d1 = Dt[i * n + p];
        const double v1 = d1 * b2, v2 = b1 * d2, ph = b1 * b2;
        const double* fp = fe + (int64_t)i * QT + j;
        s += fp[QD] * v1 * v1 + 2.0 * fp[2 * QD] * v1 * v2 + fp[3 * QD] * v2 * v2 +
             lm * fp[0] * ph * ph;
      }
    }
  }
  unsafeAtomicAdd(diag + l2g_dof(g), s);
}

hipError_t launch_diag(int dim, int P, int Q, int64_t nelem, const double* Bt, const double* Dt,
                       const double* fac, const double* lam, double lam0, const int32_t* l2g,
                       double* diag, hipStream_t s) {
  const int n = P + 1;
  const int64_t ND = dim == 3 ? (int64_t)n * n * n : (int64_t)n * n;
  const int64_t tot = nelem * ND;
  if (tot == 0) return hipSuccess;
  const int64_t nb = (tot + 255) / 256;
  if (dim == 3)
    hipLaunchKernelGGL(k_diag<3>, dim3((unsigned)nb), dim3(256), 0, s, P, Q, nelem, Bt, Dt, fac,
                       lam, lam0, l2g, diag);
  else
    hipLaunchKernelGGL(k_diag<2>, dim3((unsigned)nb), dim3(256), 0, s, P, Q, nelem, Bt, Dt, fac,
                       lam, lam0, l2g, diag);
  return hipGetLastError();
}

}  // namespace nk
