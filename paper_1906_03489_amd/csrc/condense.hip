// Static condensation of the assembled hexahedral Helmholtz system onto the
// elemental boundary DOFs (section 2.1 of arXiv 1906.03489: the modified
// basis splits each element's modes into boundary modes, shared with
// neighbours, and interior bubbles owned by the element alone).
//
// The condensed operator S = sum_e R_e^T (H_bb - H_bi H_ii^{-1} H_ib) R_e is
// applied matrix-free in three launches:
//   pass 1  gather the boundary values (interior modes are Dirichlet entries
//           of the condensed map, so they read 0), sum-factorised Helmholtz,
//           store the interior outputs (H_ib x_b) per element;
//   inverse z = -H_ii^{-1} (H_ib x_b), one dense product per element;
//   pass 2  gather the boundary values again with the interior inputs taken
//           from z, Helmholtz, scatter-add the boundary outputs
//           (H_bb x_b + H_bi z = S_e x_b) and the element energies.
// The dense inverses are formed once: H_ii column by column from the local
// Helmholtz kernel applied to interior unit vectors, then inverted in place
// by Gauss-Jordan elimination (H_ii is symmetric positive definite, so no
// pivoting is needed).
#include "engine.h"
#include "system.h"
#include "tables.h"
#include "tiles.h"

namespace nk {

constexpr int sc_ni(int P) { return (P - 1) * (P - 1) * (P - 1); }
constexpr int sc_threads(int ni) { return ni <= 64 ? 64 : (ni + 63) / 64 * 64; }

// ------------------------------------------------------------ operator passes

template <int N, int Q, int EPB, int PASS>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_sc_pass(const Tab<double, N, Q> tb, const DevArgs<double> a) {
  constexpr int NT = slot_threads<Q>(), S = Q * Q * N;
  __shared__ double smem[EPB * 3 * S];
  __shared__ double red[NT != 64 ? EPB * NT : 1];
  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && seg_converged(a.elem_seg, a.seg_done, e)) live = false;
  helm3_body<double, N, Q, NT, true, 2, true, PASS>(tb, smem + slot * 3 * S, red, slot, t, live,
                                                     e, a);
}

template <int P, int PASS>
static hipError_t run_pass(const CondOp& c, const double* x, double* y, double* dots,
                           const int32_t* dslot, const int32_t* seg_done, hipStream_t s) {
  constexpr int N = P + 1, Q = P + 2, EPB = kTileEPB3[P][0];
  DevArgs<double> d{};
  d.nelem = c.nelem;
  d.in = x;
  d.out = y;
  d.fac = c.fac;
  d.lam = c.lam;
  d.lam0 = c.lam0;
  d.l2g = c.l2g;
  d.dots = dots;
  d.dslot = dslot;
  d.seg_done = seg_done;
  d.in2 = c.t;
  d.out2 = c.t;
  const int64_t nblk = (c.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  if (nblk == 0) return hipSuccess;
  hipLaunchKernelGGL((k_sc_pass<N, Q, EPB, PASS>), dim3((unsigned)nblk),
                     dim3(EPB * slot_threads<Q>()), 0, s, host_tab<double, N, Q>(), d);
  return hipGetLastError();
}

hipError_t sc_pass(const CondOp& c, int pass, const double* x, double* y, double* dots,
                   const int32_t* dslot, const int32_t* seg_done, hipStream_t s) {
  if (pass != 1 && pass != 2) return hipErrorInvalidValue;
#define NK_SC_CASE(P)                                                        \
  case P:                                                                    \
    return pass == 1 ? run_pass<P, 1>(c, x, y, dots, dslot, seg_done, s)     \
                     : run_pass<P, 2>(c, x, y, dots, dslot, seg_done, s);
  switch (c.P) {
    NK_SC_CASE(2)
    NK_SC_CASE(3)
    NK_SC_CASE(4)
    NK_SC_CASE(5)
    NK_SC_CASE(6)
    default: return hipErrorInvalidValue;
  }
#undef NK_SC_CASE
}

// --------------------------------------------------------- interior inverse
// One block per element.  y_k = alpha T[e][k] + beta sign_k b[dof_k] (terms
// with a zero coefficient are not read), z = gamma H_ii^{-1} y; z goes back
// to T[e] or, with xadd, is added to xadd at the interior DOFs (sign
// applied).  The inverse is symmetric, so thread k reads column k of row j:
// for each j the block reads one contiguous row.
template <int NI>
__global__ void __launch_bounds__(sc_threads(NI))
    k_sc_ainv(const double* __restrict__ A, double* __restrict__ T, const double* __restrict__ b,
              const int32_t* __restrict__ iidx, double alpha, double beta, double gamma,
              double* __restrict__ xadd, const int32_t* __restrict__ seg_done) {
  __shared__ double ys[NI];
  if (seg_done != nullptr && seg_done[0] != 0) return;   // uniform over the grid
  const int64_t e = blockIdx.x;
  const int k = threadIdx.x;
  int32_t ik = 0;
  if (k < NI) {
    double yk = 0.0;
    if (alpha != 0.0) yk = alpha * T[e * NI + k];
    if (beta != 0.0 || xadd != nullptr) ik = iidx[e * NI + k];
    if (beta != 0.0) yk += beta * l2g_sign(ik, b[l2g_dof(ik)]);
    ys[k] = yk;
  }
  __syncthreads();
  if (k < NI) {
    const double* Ak = A + e * (int64_t)(NI * NI) + k;
    double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
    int j = 0;
#pragma unroll 4
    for (; j + 4 <= NI; j += 4) {
      z0 += Ak[(j + 0) * NI] * ys[j + 0];
      z1 += Ak[(j + 1) * NI] * ys[j + 1];
      z2 += Ak[(j + 2) * NI] * ys[j + 2];
      z3 += Ak[(j + 3) * NI] * ys[j + 3];
    }
    for (; j < NI; ++j) z0 += Ak[j * NI] * ys[j];
    const double z = gamma * ((z0 + z1) + (z2 + z3));
    if (xadd != nullptr)
      xadd[l2g_dof(ik)] += l2g_sign(ik, z);
    else
      T[e * NI + k] = z;
  }
}

template <int P>
static hipError_t run_ainv(const CondOp& c, const double* b, const int32_t* iidx, double alpha,
                           double beta, double gamma, double* xadd, const int32_t* seg_done,
                           hipStream_t s) {
  constexpr int NI = sc_ni(P);
  if (c.nelem > 0x7fffffff) return hipErrorInvalidValue;
  if (c.nelem == 0) return hipSuccess;
  hipLaunchKernelGGL((k_sc_ainv<NI>), dim3((unsigned)c.nelem), dim3(sc_threads(NI)), 0, s, c.ainv,
                     c.t, b, iidx, alpha, beta, gamma, xadd, seg_done);
  return hipGetLastError();
}

hipError_t sc_ainv(const CondOp& c, const double* b, const int32_t* iidx, double alpha, double beta,
                   double gamma, double* xadd, const int32_t* seg_done, hipStream_t s) {
  switch (c.P) {
    case 2: return run_ainv<2>(c, b, iidx, alpha, beta, gamma, xadd, seg_done, s);
    case 3: return run_ainv<3>(c, b, iidx, alpha, beta, gamma, xadd, seg_done, s);
    case 4: return run_ainv<4>(c, b, iidx, alpha, beta, gamma, xadd, seg_done, s);
    case 5: return run_ainv<5>(c, b, iidx, alpha, beta, gamma, xadd, seg_done, s);
    case 6: return run_ainv<6>(c, b, iidx, alpha, beta, gamma, xadd, seg_done, s);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------------- setup

// local mode index of interior mode k (numbering as in sc_inner / sc_k)
__device__ __forceinline__ int sc_mode(int P, int k) {
  const int n = P + 1, m = P - 1;
  const int r = k / (m * m) + 1, hi = (k / m) % m + 1, lo = k % m + 1;
  return (r * n + hi) * n + lo;
}

// c[e][mode(k)] = 1 and c[e][mode(k - 1)] = 0 for every element: walks a
// zeroed coefficient vector through the interior unit vectors.
__global__ void k_sc_unit(int P, int64_t nelem, double* __restrict__ c, int k) {
  const int n3 = (P + 1) * (P + 1) * (P + 1);
  const int mk = sc_mode(P, k), mp = k > 0 ? sc_mode(P, k - 1) : -1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nelem;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (mp >= 0) c[e * n3 + mp] = 0.0;
    c[e * n3 + mk] = 1.0;
  }
}

// Row k of H_ii (= column k, H is symmetric) from y = H e_k.
__global__ void k_sc_column(int P, int64_t nelem, const double* __restrict__ y,
                            double* __restrict__ A, int k) {
  const int n3 = (P + 1) * (P + 1) * (P + 1), ni = (P - 1) * (P - 1) * (P - 1);
  const int64_t total = nelem * ni;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = idx / ni;
    const int i = (int)(idx - e * ni);
    A[(e * ni + k) * ni + i] = y[e * n3 + sc_mode(P, i)];
  }
}

// In-place Gauss-Jordan inversion of each element's NI x NI block (one block
// of threads per element, the matrix in global memory).  A pivot that is not
// positive sets *bad.
template <int NI>
__global__ void __launch_bounds__(256) k_sc_invert(double* __restrict__ A, int* __restrict__ bad) {
  __shared__ double rowk[NI], colk[NI];
  double* M = A + (int64_t)blockIdx.x * (NI * NI);
  for (int kk = 0; kk < NI; ++kk) {
    const double piv = M[kk * NI + kk];
    if (!(piv > 0.0)) {
      if (threadIdx.x == 0) atomicOr(bad, 1);
    }
    const double ip = 1.0 / piv;
    for (int j = threadIdx.x; j < NI; j += blockDim.x) {
      rowk[j] = j == kk ? ip : M[kk * NI + j] * ip;
      colk[j] = M[j * NI + kk];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NI * NI; idx += blockDim.x) {
      const int i = idx / NI, j = idx - i * NI;
      double v;
      if (i == kk)
        v = rowk[j];
      else if (j == kk)
        v = -colk[i] * ip;
      else
        v = M[idx] - colk[i] * rowk[j];
      M[idx] = v;
    }
    __syncthreads();
  }
}

static unsigned grid_for(int64_t n) {
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  return (unsigned)(nb > 0 ? nb : 1);
}

hipError_t sc_unit(int P, int64_t nelem, double* c, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_unit, dim3(grid_for(nelem)), dim3(256), 0, s, P, nelem, c, k);
  return hipGetLastError();
}

hipError_t sc_column(int P, int64_t nelem, const double* y, double* A, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_column, dim3(grid_for(nelem * sc_ni(P))), dim3(256), 0, s, P, nelem, y,
                     A, k);
  return hipGetLastError();
}

hipError_t sc_invert(int P, int64_t nelem, double* A, int* bad, hipStream_t s) {
  if (nelem > 0x7fffffff) return hipErrorInvalidValue;
  if (nelem == 0) return hipSuccess;
  const dim3 g((unsigned)nelem), b(256);
  switch (P) {
    case 2: hipLaunchKernelGGL(k_sc_invert<sc_ni(2)>, g, b, 0, s, A, bad); break;
    case 3: hipLaunchKernelGGL(k_sc_invert<sc_ni(3)>, g, b, 0, s, A, bad); break;
    case 4: hipLaunchKernelGGL(k_sc_invert<sc_ni(4)>, g, b, 0, s, A, bad); break;
    case 5: hipLaunchKernelGGL(k_sc_invert<sc_ni(5)>, g, b, 0, s, A, bad); break;
    case 6: hipLaunchKernelGGL(k_sc_invert<sc_ni(6)>, g, b, 0, s, A, bad); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------ boundary <-> full vectors

// cond[c] = full[bmap[c]] on the condensed free DOFs (dinv_c != 0), 0 on
// its Dirichlet, dummy and padding entries.
__global__ void k_sc_restrict(int64_t nb, int64_t npad, const int32_t* __restrict__ bmap,
                              const double* __restrict__ full, const double* __restrict__ dinv_c,
                              double* __restrict__ cond) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < npad;
       c += (int64_t)gridDim.x * blockDim.x)
    cond[c] = (c < nb && dinv_c[c] != 0.0) ? full[bmap[c]] : 0.0;
}

// full[bmap[c]] += cond[c]
__global__ void k_sc_expand_add(int64_t nb, const int32_t* __restrict__ bmap,
                                const double* __restrict__ cond, double* __restrict__ full) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nb;
       c += (int64_t)gridDim.x * blockDim.x)
    full[bmap[c]] += cond[c];
}

hipError_t sc_restrict(int64_t nb, int64_t npad, const int32_t* bmap, const double* full,
                       const double* dinv_c, double* cond, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_restrict, dim3(grid_for(npad)), dim3(256), 0, s, nb, npad, bmap, full,
                     dinv_c, cond);
  return hipGetLastError();
}

hipError_t sc_expand_add(int64_t nb, const int32_t* bmap, const double* cond, double* full,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_sc_expand_add, dim3(grid_for(nb)), dim3(256), 0, s, nb, bmap, cond, full);
  return hipGetLastError();
}

}  // namespace nk
