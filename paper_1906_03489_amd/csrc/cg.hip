// Vector kernels of the Jacobi-preconditioned conjugate-gradient solver and
// the assembly helpers.  Each block of kVecBlock threads owns kSegAlign
// consecutive DOFs of one system, so per-system reductions are block sums
// finished by the last block of that system (fixed summation order, hence
// deterministic).
#include "system.h"

namespace nk {

constexpr int kPer = kSegAlign / kVecBlock;  // DOFs per thread

__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kVecBlock / 64; ++i) s += sh[i];
  return s;  // valid in thread 0
}

// Register the block's partials (a, b); returns true in thread 0 of the last
// block of system `s` to arrive, which then sees every block's partials.
__device__ __forceinline__ bool last_block(double a, double b, double* part, int32_t* cnt, int s,
                                           int64_t nb_s) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    __hip_atomic_store(part + 2 * blockIdx.x, a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(part + 2 * blockIdx.x + 1, b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const int prev = atomicAdd(cnt + s, 1);
    is_last = (prev == nb_s - 1);
    if (is_last) __threadfence();
  }
  __syncthreads();
  return is_last != 0;
}

// Sum partials of blocks [b0, b1) in order (whole block cooperates); result in thread 0.
__device__ __forceinline__ void sum_parts(double* part, int64_t b0, int64_t b1, double* sh,
                                          double& a, double& b) {
  double sa = 0.0, sb = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kVecBlock) {
    sa += __hip_atomic_load(part + 2 * i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sb += __hip_atomic_load(part + 2 * i + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  a = block_sum(sa, sh);
  b = block_sum(sb, sh);
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_p(const int32_t* __restrict__ blk_seg, CgState st, const T* __restrict__ r,
           const T* __restrict__ dinv, T* __restrict__ p) {
  const int s = blk_seg[blockIdx.x];
  if (st.done[s]) return;
  const T beta = (T)st.beta[s];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    p[i] = r[i] * dinv[i] + beta * p[i];
  }
}

template <typename T>
hipError_t cg_p_update(const VecLayout& L, CgState st, const T* r, const T* dinv, T* p,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg, st, r,
                     dinv, p);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_cg_alpha(const int64_t* __restrict__ elem_off, const double* __restrict__ dots, CgState st,
               int fatal) {
  __shared__ double sh[kVecBlock / 64];
  const int s = blockIdx.x;
  if (st.done[s]) return;
  double v = 0.0;
  for (int64_t e = elem_off[s] + threadIdx.x; e < elem_off[s + 1]; e += kVecBlock) v += dots[e];
  const double pAp = block_sum(v, sh);
  if (threadIdx.x == 0) {
    if (!(pAp > 0.0) || !isfinite(pAp)) {
      st.alpha[s] = 0.0;
      st.done[s] = 1;
      if (fatal) st.status[s] = NK_EBREAKDOWN;
    } else {
      st.alpha[s] = st.rz[s] / pAp;
    }
  }
}

template <typename T>
hipError_t cg_alpha(int nsys, const int64_t* elem_off, const double* dots, CgState st,
                    bool fatal_breakdown, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(nsys), dim3(kVecBlock), 0, s, elem_off, dots, st,
                     fatal_breakdown ? 1 : 0);
  return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_upd(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ blk_first, CgState st,
             int maxit, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
             T* __restrict__ y, const T* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double sh[kVecBlock / 64];
  const int s = blk_seg[blockIdx.x];
  if (st.done[s]) return;
  const T alpha = (T)st.alpha[s];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    x[i] += alpha * p[i];
    const T ri = r[i] - alpha * y[i];
    r[i] = ri;
    y[i] = T(0);
    const double rd = (double)ri;
    rz += rd * rd * (double)dinv[i];
    rr += rd * rd;
  }
  const double a = block_sum(rz, sh), b = block_sum(rr, sh);
  const int64_t b0 = blk_first[s], b1 = blk_first[s + 1];
  if (!last_block(a, b, part, st.cnt, s, b1 - b0)) return;
  double rzn, rrn;
  sum_parts(part, b0, b1, sh, rzn, rrn);
  if (threadIdx.x == 0) {
    st.beta[s] = rzn / st.rz[s];
    st.rz[s] = rzn;
    st.rr[s] = rrn;
    const int it = st.iters[s] + 1;
    st.iters[s] = it;
    if (rrn <= st.tol2[s]) {
      st.done[s] = 1;
    } else if (it >= maxit || !isfinite(rrn)) {
      st.done[s] = 1;
      st.status[s] = isfinite(rrn) ? NK_ENOCONV : NK_EBREAKDOWN;
    }
    st.cnt[s] = 0;
  }
}

template <typename T>
hipError_t cg_update(const VecLayout& L, CgState st, int maxit, T* x, T* r, const T* p, T* y,
                     const T* dinv, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_upd<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg,
                     L.blk_first, st, maxit, x, r, p, y, dinv, part);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_resid(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ blk_first, CgState st,
            const double* __restrict__ b, double* __restrict__ y,
            const double* __restrict__ dinv, double* __restrict__ r, double* __restrict__ p,
            double* __restrict__ part) {
  __shared__ double sh[kVecBlock / 64];
  const int s = blk_seg[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const double di = dinv[i];
    const double ri = di != 0.0 ? b[i] - y[i] : 0.0;
    r[i] = ri;
    y[i] = 0.0;
    if (p) p[i] = 0.0;
    rz += ri * ri * di;
    rr += ri * ri;
  }
  const double a = block_sum(rz, sh), bsum = block_sum(rr, sh);
  const int64_t b0 = blk_first[s], b1 = blk_first[s + 1];
  if (!last_block(a, bsum, part, st.cnt, s, b1 - b0)) return;
  double rzn, rrn;
  sum_parts(part, b0, b1, sh, rzn, rrn);
  if (threadIdx.x == 0) {
    if (st.rz) st.rz[s] = rzn;
    st.rr[s] = rrn;
    if (st.beta) st.beta[s] = 0.0;
    if (st.iters) st.iters[s] = 0;
    if (st.done) st.done[s] = (st.tol2[s] >= 0.0 && rrn <= st.tol2[s]) ? 1 : 0;
    st.cnt[s] = 0;
  }
}

hipError_t cg_residual(const VecLayout& L, CgState st, const double* b, double* y,
                       const double* dinv, double* r, double* p, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_resid, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg,
                     L.blk_first, st, b, y, dinv, r, p, part);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_norm2(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ blk_first,
            const double* __restrict__ v, double* __restrict__ part, int32_t* cnt, double* out,
            double rtol2, double* tol2) {
  __shared__ double sh[kVecBlock / 64];
  const int s = blk_seg[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double a = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const double vi = v[base + c * kVecBlock];
    a += vi * vi;
  }
  a = block_sum(a, sh);
  const int64_t b0 = blk_first[s], b1 = blk_first[s + 1];
  if (!last_block(a, 0.0, part, cnt, s, b1 - b0)) return;
  double tot, dummy;
  sum_parts(part, b0, b1, sh, tot, dummy);
  if (threadIdx.x == 0) {
    out[s] = tot;
    if (tol2) tol2[s] = rtol2 * tot;
    cnt[s] = 0;
  }
}

hipError_t vec_norm2(const VecLayout& L, const double* v, double* part, int32_t* cnt, double* out,
                     double rtol, double* tol2, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg,
                     L.blk_first, v, part, cnt, out, rtol * rtol, tol2);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_inner_init(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ blk_first,
                 CgState st, const int32_t* __restrict__ outer_done, double tau2,
                 const double* __restrict__ r64, const float* __restrict__ dinv32,
                 float* __restrict__ r32, float* __restrict__ d32, float* __restrict__ p32,
                 float* __restrict__ y32, double* __restrict__ part) {
  __shared__ double sh[kVecBlock / 64];
  const int s = blk_seg[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double rz = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const float ri = (float)r64[i];
    r32[i] = ri;
    d32[i] = 0.f;
    p32[i] = 0.f;
    y32[i] = 0.f;
    const double rd = (double)ri;
    rz += rd * rd * (double)dinv32[i];
    rr += rd * rd;
  }
  const double a = block_sum(rz, sh), b = block_sum(rr, sh);
  const int64_t b0 = blk_first[s], b1 = blk_first[s + 1];
  if (!last_block(a, b, part, st.cnt, s, b1 - b0)) return;
  double rzn, rrn;
  sum_parts(part, b0, b1, sh, rzn, rrn);
  if (threadIdx.x == 0) {
    st.rz[s] = rzn;
    st.rr[s] = rrn;
    st.tol2[s] = tau2 * rrn;
    st.beta[s] = 0.0;
    st.iters[s] = 0;
    st.status[s] = 0;
    st.done[s] = (outer_done[s] || rrn == 0.0) ? 1 : 0;
    st.cnt[s] = 0;
  }
}

hipError_t cg_inner_init(const VecLayout& L, CgState st, const int32_t* outer_done, double tau,
                         const double* r64, const float* dinv32, float* r32, float* d32,
                         float* p32, float* y32, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_inner_init, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg,
                     L.blk_first, st, outer_done, tau * tau, r64, dinv32, r32, d32, p32, y32,
                     part);
  return hipGetLastError();
}

__global__ void __launch_bounds__(kVecBlock)
    k_correct(const int32_t* __restrict__ blk_seg, const int32_t* __restrict__ outer_done,
              const float* __restrict__ d32, double* __restrict__ x) {
  const int s = blk_seg[blockIdx.x];
  if (outer_done[s]) return;
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    x[i] += (double)d32[i];
  }
}

hipError_t cg_correct(const VecLayout& L, const int32_t* outer_done, const float* d32, double* x,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_correct, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg,
                     outer_done, d32, x);
  return hipGetLastError();
}

template <typename T>
__global__ void k_fill(T* __restrict__ v, int64_t n, T val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    v[i] = val;
}

template <typename T>
hipError_t vec_fill(T* v, int64_t n, T val, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)nb), dim3(256), 0, s, v, n, val);
  return hipGetLastError();
}

// padded[i] for i in system k's padded range <- user[dof_off[k] + (i - pdof_off[k])],
// zero on Dirichlet (dinv == 0) and padding entries.
template <typename T>
__global__ void k_pad_in(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ dof_off,
                         const int64_t* __restrict__ pdof_off, const T* __restrict__ user,
                         const double* __restrict__ dinv, T* __restrict__ padded) {
  const int s = blk_seg[blockIdx.x];
  const int64_t n_s = dof_off[s + 1] - dof_off[s];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const int64_t li = i - pdof_off[s];
    padded[i] = (li < n_s && dinv[i] != 0.0) ? user[dof_off[s] + li] : T(0);
  }
}

template <typename T>
hipError_t pad_in(int nsys, const int64_t* dof_off, const int64_t* pdof_off, const VecLayout& L,
                  const T* user, const double* dinv, T* padded, hipStream_t s) {
  (void)nsys;
  hipLaunchKernelGGL(k_pad_in<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, s, L.blk_seg, dof_off,
                     pdof_off, user, dinv, padded);
  return hipGetLastError();
}

// user[j] <- padded[...] for every user index j (binary search of its system).
template <typename T>
__global__ void k_pad_out(int nsys, const int64_t* __restrict__ dof_off,
                          const int64_t* __restrict__ pdof_off, int64_t nuser,
                          const T* __restrict__ padded, T* __restrict__ user) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nuser;
       j += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = nsys;  // dof_off[lo] <= j < dof_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (dof_off[mid] <= j) lo = mid; else hi = mid;
    }
    user[j] = padded[pdof_off[lo] + (j - dof_off[lo])];
  }
}

template <typename T>
hipError_t pad_out(int nsys, const int64_t* dof_off, const int64_t* pdof_off, int64_t nuser,
                   const T* padded, T* user, hipStream_t s) {
  if (nuser == 0) return hipSuccess;
  int64_t nb = (nuser + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_pad_out<T>, dim3((unsigned)nb), dim3(256), 0, s, nsys, dof_off, pdof_off, nuser,
                     padded, user);
  return hipGetLastError();
}

// Internal l2g: user global index g of system s -> padded index gi, stored as
// gi (free) or -1-gi (Dirichlet).  Out-of-range indices set *bad.
__global__ void k_build_l2g(int64_t nelem, int nloc, const int32_t* __restrict__ elem_seg,
                            const int64_t* __restrict__ dof_off,
                            const int64_t* __restrict__ pdof_off,
                            const int32_t* __restrict__ l2g_user,
                            const uint8_t* __restrict__ dirichlet, int32_t* __restrict__ l2g_int,
                            int* bad) {
  const int64_t tot = nelem * nloc;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = id / nloc;
    const int s = elem_seg[e];
    const int64_t g = l2g_user[id];
    if (g < dof_off[s] || g >= dof_off[s + 1]) {
      atomicOr(bad, 1);
      l2g_int[id] = -1 - (int32_t)pdof_off[s];
      continue;
    }
    const int64_t gi = g - dof_off[s] + pdof_off[s];
    l2g_int[id] = dirichlet[g] ? (int32_t)(-1 - gi) : (int32_t)gi;
  }
}

hipError_t build_l2g(int64_t nelem, int nloc, const int32_t* elem_seg, const int64_t* dof_off,
                     const int64_t* pdof_off, const int32_t* l2g_user, const uint8_t* dirichlet,
                     int32_t* l2g_int, int* bad, hipStream_t s) {
  const int64_t tot = nelem * nloc;
  if (tot == 0) return hipSuccess;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_build_l2g, dim3((unsigned)nb), dim3(256), 0, s, nelem, nloc, elem_seg,
                     dof_off, pdof_off, l2g_user, dirichlet, l2g_int, bad);
  return hipGetLastError();
}

// diag holds accumulated free-DOF diagonals, mark is nonzero on free DOFs:
// dinv = 1/diag on free DOFs and exactly 0 on Dirichlet/padding rows (so
// dinv != 0 is the free-DOF mask everywhere), whose diagonal is reported as 1.
__global__ void k_diag_finish(int64_t n, const double* diag, const double* __restrict__ mark,
                              double* __restrict__ dinv64, float* __restrict__ dinv32,
                              double* diag_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double d = diag[i];
    const bool free_ = mark[i] != 0.0;
    dinv64[i] = free_ ? 1.0 / d : 0.0;
    dinv32[i] = free_ ? (float)(1.0 / d) : 0.f;
    diag_out[i] = free_ ? d : 1.0;
  }
}

hipError_t diag_finish(const VecLayout& L, const double* diag, const double* mark,
                       double* dinv64, float* dinv32, double* diag_out, hipStream_t s) {
  int64_t nb = (L.npad + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_diag_finish, dim3((unsigned)nb), dim3(256), 0, s, L.npad, diag, mark,
                     dinv64, dinv32, diag_out);
  return hipGetLastError();
}

// mark[g] = 1 for every free global DOF referenced by an element
__global__ void k_mark(int64_t tot, const int32_t* __restrict__ l2g, double* __restrict__ mark) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = l2g[id];
    if (g >= 0) mark[g] = 1.0;
  }
}

hipError_t mark_free(int64_t nelem, int nloc, const int32_t* l2g_int, double* mark, hipStream_t s) {
  const int64_t tot = nelem * nloc;
  if (tot == 0) return hipSuccess;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_mark, dim3((unsigned)nb), dim3(256), 0, s, tot, l2g_int, mark);
  return hipGetLastError();
}

__global__ void k_gather(int64_t tot, const int32_t* __restrict__ l2g,
                         const double* __restrict__ x, double* __restrict__ xl) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = l2g[id];
    xl[id] = x[g >= 0 ? g : -1 - g];
  }
}

hipError_t gather_user(int64_t nelem, int nloc, const int32_t* l2g_int, const double* xpad,
                       double* xloc, hipStream_t s) {
  const int64_t tot = nelem * nloc;
  if (tot == 0) return hipSuccess;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_gather, dim3((unsigned)nb), dim3(256), 0, s, tot, l2g_int, xpad, xloc);
  return hipGetLastError();
}

__global__ void k_scatter(int64_t tot, const int32_t* __restrict__ l2g,
                          const double* __restrict__ yl, double* __restrict__ y) {
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int32_t g = l2g[id];
    if (g >= 0) unsafeAtomicAdd(y + g, yl[id]);
  }
}

hipError_t scatter_add(int64_t nelem, int nloc, const int32_t* l2g_int, const double* yloc,
                       double* ypad, hipStream_t s) {
  const int64_t tot = nelem * nloc;
  if (tot == 0) return hipSuccess;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb), dim3(256), 0, s, tot, l2g_int, yloc, ypad);
  return hipGetLastError();
}

template <typename A, typename B>
__global__ void k_cast(const A* __restrict__ src, B* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (B)src[i];
}

hipError_t cast_copy(const double* src, float* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_cast<double, float>), dim3((unsigned)nb), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t cast_copy(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL((k_cast<float, double>), dim3((unsigned)nb), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

template hipError_t cg_p_update<double>(const VecLayout&, CgState, const double*, const double*,
                                        double*, hipStream_t);
template hipError_t cg_p_update<float>(const VecLayout&, CgState, const float*, const float*,
                                       float*, hipStream_t);
template hipError_t cg_alpha<double>(int, const int64_t*, const double*, CgState, bool,
                                     hipStream_t);
template hipError_t cg_alpha<float>(int, const int64_t*, const double*, CgState, bool, hipStream_t);
template hipError_t cg_update<double>(const VecLayout&, CgState, int, double*, double*,
                                      const double*, double*, const double*, double*, hipStream_t);
template hipError_t cg_update<float>(const VecLayout&, CgState, int, float*, float*, const float*,
                                     float*, const float*, double*, hipStream_t);
template hipError_t pad_in<double>(int, const int64_t*, const int64_t*, const VecLayout&,
                                   const double*, const double*, double*, hipStream_t);
template hipError_t pad_in<float>(int, const int64_t*, const int64_t*, const VecLayout&,
                                  const float*, const double*, float*, hipStream_t);
template hipError_t pad_out<double>(int, const int64_t*, const int64_t*, int64_t, const double*,
                                    double*, hipStream_t);
template hipError_t pad_out<float>(int, const int64_t*, const int64_t*, int64_t, const float*,
                                   float*, hipStream_t);
template hipError_t vec_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t vec_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t vec_fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);

}  // namespace nk
