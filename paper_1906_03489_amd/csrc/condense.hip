// Static condensation of the assembled hexahedral Helmholtz system onto the
// elemental boundary DOFs (section 2.1 of arXiv 1906.03489: the modified
// basis splits each element's modes into boundary modes, shared with
// neighbours, and interior bubbles owned by the element alone).
//
// The condensed operator S = sum_e R_e^T (H_bb - H_bi H_ii^{-1} H_ib) R_e is
// applied matrix-free, per element (one fused launch; the three steps are
// also separate launches, used for the right-hand side and the interior
// recovery):
//   pass 1  gather the boundary values (interior modes are Dirichlet entries
//           of the condensed map, so they read 0), sum-factorised Helmholtz,
//           store the interior outputs (H_ib x_b) per element;
//   inverse z = -H_ii^{-1} (H_ib x_b), one dense product per element;
//   pass 2  gather the boundary values again with the interior inputs taken
//           from z, Helmholtz, scatter-add the boundary outputs
//           (H_bb x_b + H_bi z = S_e x_b) and the element energies.
// The dense inverses are formed once: H_ii row by row from the local
// Helmholtz kernel applied to interior unit vectors, then inverted by
// Gauss-Jordan elimination in LDS (H_ii is symmetric positive definite, so no
// pivoting is needed).
#include "engine.h"
#include "system.h"
#include "tables.h"
#include "tiles.h"

namespace nk {

constexpr int sc_ni(int P) { return (P - 1) * (P - 1) * (P - 1); }
constexpr int sc_threads(int ni) { return ni <= 64 ? 64 : (ni + 63) / 64 * 64; }

// The symmetric interior inverse A of an element is stored by diagonals:
// D[s][k] = A[k][(k + s) mod NI] for s = 0 .. NI/2, (NI/2 + 1) NI values,
// about half of NI^2.  Row k of A y is the sum over s of D[s][k] y[k + s]
// and, for 0 < s < NI - s, of D[s][k - s] y[k - s] (indices mod NI; the
// second term is the transposed half, read from the same diagonal).  Both
// reads of a diagonal are contiguous across k, so a slot's loads coalesce
// and the second one hits the cache lines of the first.
// Rows k = t, t + NT, .. (R of them) of one thread, in one pass over the
// diagonals so that the loads of all its rows are in flight together; rows
// past NI read row NI - 1 and their result is not used.
template <typename T, int NI, int NT, int R>
__device__ __forceinline__ void sc_symv_rows(const T* __restrict__ D, const T* y, int t, T (&z)[R]) {
  constexpr int H = NI / 2;
  int k[R], kp[R], km[R];   // row, (k + s) mod NI, (k - s) mod NI
  T zt[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    k[i] = t + i * NT < NI ? t + i * NT : NI - 1;
    kp[i] = km[i] = k[i];
    z[i] = zt[i] = T(0);
  }
#pragma unroll 32
  for (int s = 0; s <= H; ++s) {
    const T* Ds = D + s * NI;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      z[i] += Ds[k[i]] * y[kp[i]];
      if (s > 0 && s < NI - s) zt[i] += Ds[km[i]] * y[km[i]];
      kp[i] = kp[i] + 1 == NI ? 0 : kp[i] + 1;
      km[i] = km[i] == 0 ? NI - 1 : km[i] - 1;
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) z[i] += zt[i];
}

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
  constexpr int NI = (N - 2) * (N - 2) * (N - 2);
  double* scb = a.out2 + (live ? e : 0) * (int64_t)NI;
  helm3_body<double, N, Q, NT, true, 2, true, PASS>(tb, smem + slot * 3 * S, red, slot, t, live,
                                                     e, a, scb);
}

// The whole condensed operator of one element per slot in one launch:
// pass 1 into the slot's LDS block y, z = -H_ii^{-1} y (the slot's threads
// take the rows k = t, t + NT, ...; the inverse in its diagonal storage),
// pass 2 from z.  The interior values never
// leave LDS; pass 2 re-reads the element's factors and map right after
// pass 1.
// T: FP64, or FP32 (factors and an FP32 copy of the inverses) for the inner
// iterations of the refined condensed solve.  PF / EOI: the Helmholtz
// body's factor prefetch depth and I-stage form (two variants per order and
// precision are compiled; setup times both).  ASM = false is
// the elemental form S_e x_e on local vectors (local input with zero
// interior entries, every local output stored), used to probe diag(S_e).
template <typename T, int N, int Q, int EPB, int PF, bool EOI, bool ASM = true>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_sc_fused(const Tab<T, N, Q> tb, const DevArgs<T> a, const T* __restrict__ A) {
  constexpr int NT = slot_threads<Q>(), S = Q * Q * N, NI = (N - 2) * (N - 2) * (N - 2);
  __shared__ T smem[EPB * 3 * S];
  __shared__ double red[NT != 64 ? EPB * NT : 1];
  __shared__ T ib[EPB][2][NI];
  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && seg_converged(a.elem_seg, a.seg_done, e)) live = false;
  T* y = ib[slot][0];
  T* z = ib[slot][1];
  helm3_body<T, N, Q, NT, ASM, PF, EOI, 1>(tb, smem + slot * 3 * S, red, slot, t, live, e, a, y);
  slot_sync<NT>();
  if (live) {
    constexpr int R = (NI + NT - 1) / NT;
    T zr[R];
    sc_symv_rows<T, NI, NT, R>(A + e * (int64_t)sc_packed(NI), y, t, zr);
#pragma unroll
    for (int i = 0; i < R; ++i)
      if (t + i * NT < NI) z[t + i * NT] = -zr[i];
  }
  slot_sync<NT>();
  helm3_body<T, N, Q, NT, ASM, PF, EOI, 2>(tb, smem + slot * 3 * S, red, slot, t, live, e, a, z);
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

template <typename T, int P, int PF, bool EOI, bool ASM = true>
static hipError_t run_fused(const CondOp& c, const T* x, T* y, double* dots, const int32_t* dslot,
                            const int32_t* seg_done, hipStream_t s) {
  constexpr int N = P + 1, Q = P + 2, EPB = kTileEPB3[P][0];
  DevArgs<T> d{};
  d.nelem = c.nelem;
  d.in = x;
  d.out = y;
  d.fac = sizeof(T) == 8 ? (const T*)c.fac : (const T*)c.fac32;
  d.lam = c.lam;
  d.lam0 = c.lam0;
  d.l2g = c.l2g;
  d.dots = dots;
  d.dslot = dslot;
  d.seg_done = seg_done;
  const int64_t nblk = (c.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  if (nblk == 0) return hipSuccess;
  const T* A = sizeof(T) == 8 ? (const T*)c.ainv : (const T*)c.ainv32;
  hipLaunchKernelGGL((k_sc_fused<T, N, Q, EPB, PF, EOI, ASM>), dim3((unsigned)nblk),
                     dim3(EPB * slot_threads<Q>()), 0, s, host_tab<T, N, Q>(), d, A);
  return hipGetLastError();
}

template <typename T>
static hipError_t sc_apply_t(const CondOp& c, const T* x, T* y, double* dots, const int32_t* dslot,
                             const int32_t* seg_done, hipStream_t s) {
  const int v = sizeof(T) == 8 ? c.variant : c.variant32;
#define NK_SC_FUSED(P)                                                                  \
  case P:                                                                               \
    return v == 0 ? run_fused<T, P, 2, true>(c, x, y, dots, dslot, seg_done, s)         \
                  : run_fused<T, P, 1, false>(c, x, y, dots, dslot, seg_done, s);
  switch (c.P) {
    NK_SC_FUSED(2)
    NK_SC_FUSED(3)
    NK_SC_FUSED(4)
    NK_SC_FUSED(5)
    NK_SC_FUSED(6)
    default: return hipErrorInvalidValue;
  }
#undef NK_SC_FUSED
}

hipError_t sc_apply(const CondOp& c, nk_dtype t, const void* x, void* y, double* dots,
                    const int32_t* dslot, const int32_t* seg_done, hipStream_t s) {
  if (t == NK_F64)
    return sc_apply_t<double>(c, (const double*)x, (double*)y, dots, dslot, seg_done, s);
  if (c.ainv32 == nullptr) return hipErrorInvalidValue;
  return sc_apply_t<float>(c, (const float*)x, (float*)y, dots, dslot, seg_done, s);
}

hipError_t sc_local(const CondOp& c, const double* x, double* y, hipStream_t s) {
  switch (c.P) {
    case 2: return run_fused<double, 2, 1, false, false>(c, x, y, nullptr, nullptr, nullptr, s);
    case 3: return run_fused<double, 3, 1, false, false>(c, x, y, nullptr, nullptr, nullptr, s);
    case 4: return run_fused<double, 4, 1, false, false>(c, x, y, nullptr, nullptr, nullptr, s);
    case 5: return run_fused<double, 5, 1, false, false>(c, x, y, nullptr, nullptr, nullptr, s);
    case 6: return run_fused<double, 6, 1, false, false>(c, x, y, nullptr, nullptr, nullptr, s);
    default: return hipErrorInvalidValue;
  }
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
// with a zero coefficient are not read), z = gamma H_ii^{-1} y (the inverse
// in its diagonal storage); z goes back to T[e] or, with xadd, is added to
// xadd at the interior DOFs (sign applied).
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
    double zr[1];
    sc_symv_rows<double, NI, sc_threads(NI), 1>(A + e * (int64_t)sc_packed(NI), ys, k, zr);
    const double z = gamma * zr[0];
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

// c[e][m_new] = 1 and c[e][m_old] = 0 (m_old < 0: none) for every element.
__global__ void k_sc_unit_mode(int n3, int64_t nelem, double* __restrict__ c, int m_new, int m_old) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nelem;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (m_old >= 0) c[e * n3 + m_old] = 0.0;
    c[e * n3 + m_new] = 1.0;
  }
}

// diag[g] += y[e][m] where local mode m of element e is the free DOF g of
// the boundary map (its sign squares away).
__global__ void k_sc_diag_add(int n3, int64_t nelem, const double* __restrict__ y, int m,
                              const int32_t* __restrict__ l2g, double* __restrict__ diag) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nelem;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = l2g[e * n3 + m];
    if (g >= 0) atomicAdd(diag + l2g_dof(g), y[e * n3 + m]);
  }
}

// Jacobi preconditioner from diag: on the free DOFs (dinv64 != 0) dinv =
// 1/diag and diag_out = diag.
__global__ void k_sc_dinv(int64_t n, const double* __restrict__ diag, double* __restrict__ dinv64,
                          float* __restrict__ dinv32, double* __restrict__ diag_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (dinv64[i] != 0.0) {
      dinv64[i] = 1.0 / diag[i];
      dinv32[i] = (float)(1.0 / diag[i]);
      diag_out[i] = diag[i];
    }
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

// Gauss-Jordan inversion of each element's NI x NI block H_ii (one block of
// sc_inv_threads threads per element, the matrix in LDS: at most 125 x 125 doubles, within
// gfx950's 160 KB per workgroup), written out in the diagonal storage of
// sc_symv_rows.  H_ii is symmetric positive definite, so no pivoting is
// needed; a pivot that is not positive sets *bad.
// Threads per element: the elimination steps are latency-bound, and with
// the largest blocks one workgroup fills the CU's LDS, so it brings its own
// waves.
constexpr int sc_inv_threads(int ni) { return ni >= 64 ? 1024 : 256; }

template <int NI>
__global__ void __launch_bounds__(sc_inv_threads(NI))
    k_sc_invert(const double* __restrict__ A, double* __restrict__ D, int* __restrict__ bad) {
  __shared__ double M[NI * NI];
  __shared__ double rowk[NI], colk[NI];
  const double* Ae = A + (int64_t)blockIdx.x * (NI * NI);
  for (int i = threadIdx.x; i < NI * NI; i += blockDim.x) M[i] = Ae[i];
  __syncthreads();
  for (int kk = 0; kk < NI; ++kk) {
    const double piv = M[kk * NI + kk];
    if (!(piv > 0.0) && threadIdx.x == 0) atomicOr(bad, 1);
    const double ip = 1.0 / piv;
    for (int j = threadIdx.x; j < NI; j += blockDim.x) {
      rowk[j] = j == kk ? ip : M[kk * NI + j] * ip;
      colk[j] = M[j * NI + kk];
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NI * NI; idx += blockDim.x) {
      const int i = idx / NI, j = idx - i * NI;
      M[idx] = i == kk ? rowk[j] : j == kk ? -colk[i] * ip : M[idx] - colk[i] * rowk[j];
    }
    __syncthreads();
  }
  double* De = D + (int64_t)blockIdx.x * sc_packed(NI);
  for (int idx = threadIdx.x; idx < sc_packed(NI); idx += blockDim.x) {
    const int sd = idx / NI, k = idx - sd * NI;
    const int j = k + sd < NI ? k + sd : k + sd - NI;
    De[idx] = M[k * NI + j];
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

hipError_t sc_unit_mode(int P, int64_t nelem, double* c, int m_new, int m_old, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_unit_mode, dim3(grid_for(nelem)), dim3(256), 0, s, (P + 1) * (P + 1) * (P + 1),
                     nelem, c, m_new, m_old);
  return hipGetLastError();
}

hipError_t sc_diag_add(int P, int64_t nelem, const double* y, int m, const int32_t* l2g,
                       double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_diag_add, dim3(grid_for(nelem)), dim3(256), 0, s, (P + 1) * (P + 1) * (P + 1),
                     nelem, y, m, l2g, diag);
  return hipGetLastError();
}

hipError_t sc_dinv(int64_t n, const double* diag, double* dinv64, float* dinv32, double* diag_out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_sc_dinv, dim3(grid_for(n)), dim3(256), 0, s, n, diag, dinv64, dinv32,
                     diag_out);
  return hipGetLastError();
}

hipError_t sc_column(int P, int64_t nelem, const double* y, double* A, int k, hipStream_t s) {
  hipLaunchKernelGGL(k_sc_column, dim3(grid_for(nelem * sc_ni(P))), dim3(256), 0, s, P, nelem, y,
                     A, k);
  return hipGetLastError();
}

hipError_t sc_invert(int P, int64_t nelem, const double* A, double* D, int* bad, hipStream_t s) {
  if (nelem > 0x7fffffff) return hipErrorInvalidValue;
  if (nelem == 0) return hipSuccess;
  const dim3 g((unsigned)nelem);
#define NK_SC_INV(P)                                                                    \
  case P:                                                                               \
    hipLaunchKernelGGL(k_sc_invert<sc_ni(P)>, g, dim3(sc_inv_threads(sc_ni(P))), 0, s, A, D, bad); \
    break;
  switch (P) {
    NK_SC_INV(2)
    NK_SC_INV(3)
    NK_SC_INV(4)
    NK_SC_INV(5)
    NK_SC_INV(6)
    default: return hipErrorInvalidValue;
  }
#undef NK_SC_INV
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
