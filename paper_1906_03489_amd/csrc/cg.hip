// Vector kernels of the Jacobi-preconditioned conjugate-gradient solver and
// the assembly helpers.  Each block of kVecBlock threads owns kSegAlign
// consecutive DOFs of one system, so per-system reductions are block sums
// finished by the last block of that system (fixed summation order, hence
// deterministic).
#include "system.h"

namespace nk {

constexpr int kPer = kSegAlign / kVecBlock;  // DOFs per thread

template <int NTH = kVecBlock>
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NTH / 64; ++i) s += sh[i];
  return s;  // valid in thread 0
}

constexpr int kFinThreads = 1024;

// K block sums at once (one barrier round for all of them), valid in thread 0.
template <int NTH, int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k * (NTH / 64) + w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int i = 0; i < NTH / 64; ++i) t += sh[k * (NTH / 64) + i];
      v[k] = t;
    }
  }
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

// ---------------------------------------------------------------------------
// Preconditioned CG with one reduction phase per iteration (the Chronopoulos-
// Gear arrangement of the textbook recurrences): with u = M^{-1} r, w = A u,
//   gamma = (r, u), delta = (w, u),
//   beta = gamma / gamma_old,  alpha = gamma / (delta - beta gamma / alpha_old),
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s.
// One iteration = cg_update (vectors; partial sums of gamma and r.r),
// the assembled operator w = A u (per-element u_e.(H_e u_e) into dots), and
// cg_finish (one block per system sums the partials and the dots, tests
// convergence and forms alpha, beta).  Block partials are plain stores read by
// the next kernel, so no grid-wide fence is needed.

// Writes the block's two partial sums; thread 0 holds the block sums.
__device__ __forceinline__ void store_parts(double a, double b, double* part) {
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_update(const int32_t* __restrict__ blk_seg, CgState st, T* __restrict__ x,
                T* __restrict__ r, T* __restrict__ u, T* __restrict__ p, T* __restrict__ s,
                T* __restrict__ w, const T* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double sh[2 * (kVecBlock / 64)];
  const int sg = blk_seg[blockIdx.x];
  if (st.done[sg]) return;
  const T alpha = (T)st.alpha[sg], beta = (T)st.beta[sg];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double g = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const T di = dinv[i];
    const T ri = r[i];
    const T pi = ri * di + beta * p[i];
    const T si = w[i] + beta * s[i];
    x[i] += alpha * pi;
    const T rn = ri - alpha * si;
    const T un = rn * di;
    p[i] = pi;
    s[i] = si;
    r[i] = rn;
    u[i] = un;
    w[i] = T(0);
    g += (double)rn * (double)un;
    rr += (double)rn * (double)rn;
  }
  double v[2] = {g, rr};
  block_sums<kVecBlock, 2>(v, sh);
  store_parts(v[0], v[1], part);
}

template <typename T>
hipError_t cg_update(const VecLayout& L, CgState st, T* x, T* r, T* u, T* p, T* s, T* w,
                     const T* dinv, double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_update<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream,
                     L.blk_seg, st, x, r, u, p, s, w, dinv, part);
  return hipGetLastError();
}

// Start of a solve: r = (b - w) on free DOFs (w = A x0, or 0), u = M^{-1} r,
// p = s = w = 0, partial sums of (r, u) and (r, r).
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_start(const int32_t* __restrict__ blk_seg, const double* __restrict__ b,
               T* __restrict__ w, T* __restrict__ r, T* __restrict__ u, T* __restrict__ p,
               T* __restrict__ s, const T* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double sh[2 * (kVecBlock / 64)];
  (void)blk_seg;
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double g = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const T di = dinv[i];
    const T ri = di != T(0) ? (T)(b[i] - (double)w[i]) : T(0);
    const T ui = ri * di;
    r[i] = ri;
    u[i] = ui;
    p[i] = T(0);
    s[i] = T(0);
    w[i] = T(0);
    g += (double)ri * (double)ui;
    rr += (double)ri * (double)ri;
  }
  double v[2] = {g, rr};
  block_sums<kVecBlock, 2>(v, sh);
  store_parts(v[0], v[1], part);
}

template <typename T>
hipError_t cg_start(const VecLayout& L, const double* b, T* w, T* r, T* u, T* p, T* s,
                    const T* dinv, double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_start<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream,
                     L.blk_seg, b, w, r, u, p, s, dinv, part);
  return hipGetLastError();
}

// One block per system: gamma = sum of (r,u) partials, rr = sum of (r,r)
// partials, delta = sum of the system's dots.  mode 0: iteration, mode 1:
// first step of a solve (tol2 is set from rr when tau2 > 0, for the inner
// solves of the refinement), mode 2: the last iteration's step again after
// its residual was replaced by the true one (reliable update: gamma and
// delta are new, beta and alpha come from the saved gamma and alpha of the
// iteration before; the search directions p, s are kept).
__global__ void __launch_bounds__(kFinThreads)
    k_cg_finish(const int64_t* __restrict__ blk_first, const int64_t* __restrict__ dblk_first,
                const double* __restrict__ part, const double* __restrict__ dots, CgState st,
                int fatal, int start, double tau2, const int32_t* __restrict__ outer_done,
                const double* __restrict__ outer_tol2, const double* __restrict__ outer_rr) {
  __shared__ double sh[3 * (kFinThreads / 64)];
  const int sg = blockIdx.x;
  if (start == 0 && st.done[sg]) return;
  // Every thread requests kFinLoads values per round before adding any (the
  // indices are clamped into the range, so every load is in bounds and
  // needs no branch), so a system of up to kFinLoads * kFinThreads elements
  // takes one memory round trip instead of one per value.
  constexpr int kFinLoads = 16;
  double dl = 0.0, g = 0.0, rr = 0.0;
  // dots are padded per system to whole kSegAlign blocks (padding is zero)
  const int64_t d0 = dblk_first[sg] * kSegAlign, d1 = dblk_first[sg + 1] * kSegAlign;
  for (int64_t i0 = d0 + threadIdx.x; i0 < d1; i0 += (int64_t)kFinLoads * kFinThreads) {
    double v[kFinLoads];
#pragma unroll
    for (int k = 0; k < kFinLoads; ++k) {
      const int64_t i = i0 + (int64_t)k * kFinThreads;
      v[k] = dots[i < d1 ? i : d1 - 1];
    }
#pragma unroll
    for (int k = 0; k < kFinLoads; ++k) dl += i0 + (int64_t)k * kFinThreads < d1 ? v[k] : 0.0;
  }
  const int64_t b0 = blk_first[sg], b1 = blk_first[sg + 1];
  for (int64_t j0 = b0 + threadIdx.x; j0 < b1; j0 += (int64_t)kFinLoads * kFinThreads) {
    double va[kFinLoads], vb[kFinLoads];
#pragma unroll
    for (int k = 0; k < kFinLoads; ++k) {
      const int64_t j = j0 + (int64_t)k * kFinThreads, jc = j < b1 ? j : b1 - 1;
      va[k] = part[2 * jc];
      vb[k] = part[2 * jc + 1];
    }
#pragma unroll
    for (int k = 0; k < kFinLoads; ++k) {
      const bool in = j0 + (int64_t)k * kFinThreads < b1;
      g += in ? va[k] : 0.0;
      rr += in ? vb[k] : 0.0;
    }
  }
  double v3[3] = {g, rr, dl};
  block_sums<kFinThreads, 3>(v3, sh);
  g = v3[0];
  rr = v3[1];
  dl = v3[2];
  if (threadIdx.x != 0) return;
  if (start == 2) {
    st.rr[sg] = rr;
    if ((outer_done != nullptr && outer_done[sg] != 0) || rr <= st.tol2[sg] || rr == 0.0 ||
        st.iters[sg] >= st.maxit[sg]) {
      st.done[sg] = 1;
      return;
    }
    if (!isfinite(rr) || !isfinite(g) || !isfinite(dl)) {
      st.done[sg] = 1;
      st.status[sg] = NK_EBREAKDOWN;
      return;
    }
    // The recurrence for p.Ap assumes the new residual is orthogonal to the
    // old directions; where rounding has spoilt that (the residual is at the
    // noise level of the low precision, e.g. a Krylov space that is used up)
    // the direction restarts from u (beta = 0, p = u, s = A u).
    const double gp = st.rz_prev[sg];
    double beta = gp > 0.0 ? g / gp : 0.0;
    double den = gp > 0.0 ? dl - beta * g / st.alpha_prev[sg] : dl;
    if (!(den > 0.0) || !isfinite(den)) {
      beta = 0.0;
      den = dl;
    }
    if (!(den > 0.0)) {
      st.done[sg] = 1;
      st.status[sg] = NK_EBREAKDOWN;
      return;
    }
    st.done[sg] = 0;
    st.beta[sg] = beta;
    st.alpha[sg] = g / den;
    st.rz[sg] = g;
    return;
  }
  if (start) {
    st.iters[sg] = 0;
    st.rz_prev[sg] = 0.0;
    st.alpha_prev[sg] = 0.0;
    st.status[sg] = 0;
    st.rr[sg] = rr;
    if (tau2 > 0.0) {
      // inner solve of the refinement: reduce by tau, or only as far as the
      // outer tolerance still needs (with a factor 1/2 of margin)
      const double need = outer_rr[sg] > 0.0 ? 0.25 * outer_tol2[sg] / outer_rr[sg] : 0.0;
      st.tol2[sg] = (need > tau2 ? need : tau2) * rr;
    }
    const bool od = outer_done != nullptr && outer_done[sg] != 0;
    if (od || rr <= st.tol2[sg] || rr == 0.0) {
      st.done[sg] = 1;
      return;
    }
    st.done[sg] = 0;
    if (!(dl > 0.0) || !isfinite(dl) || !isfinite(g)) {
      st.done[sg] = 1;
      if (fatal) st.status[sg] = NK_EBREAKDOWN;
      return;
    }
    st.rz[sg] = g;
    st.alpha[sg] = g / dl;
    st.beta[sg] = 0.0;
    return;
  }
  const int it = st.iters[sg] + 1;
  st.iters[sg] = it;
  st.rr[sg] = rr;
  st.rz_prev[sg] = st.rz[sg];
  st.alpha_prev[sg] = st.alpha[sg];
  if (rr <= st.tol2[sg]) {
    st.done[sg] = 1;
    return;
  }
  if (!isfinite(rr) || !isfinite(g) || !isfinite(dl)) {
    st.done[sg] = 1;
    st.status[sg] = NK_EBREAKDOWN;
    return;
  }
  if (it >= st.maxit[sg]) {
    st.done[sg] = 1;
    if (fatal) st.status[sg] = NK_ENOCONV;
    return;
  }
  const double beta = g / st.rz[sg];
  const double den = dl - beta * g / st.alpha[sg];
  if (!(den > 0.0)) {
    st.done[sg] = 1;
    if (fatal) st.status[sg] = NK_EBREAKDOWN;
    return;
  }
  st.beta[sg] = beta;
  st.alpha[sg] = g / den;
  st.rz[sg] = g;
}

hipError_t cg_finish(int nsys, const VecLayout& L, const VecLayout& Ld, const double* part,
                     const double* dots, CgState st, bool fatal, bool start,
                     double tau2, const int32_t* outer_done, const double* outer_tol2,
                     const double* outer_rr, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_finish, dim3(nsys), dim3(kFinThreads), 0, stream, L.blk_first,
                     Ld.blk_first, part, dots, st, fatal ? 1 : 0, start ? 1 : 0, tau2,
                     outer_done, outer_tol2, outer_rr);
  return hipGetLastError();
}

hipError_t cg_finish_reliable(int nsys, const VecLayout& L, const VecLayout& Ld, const double* part,
                              const double* dots, CgState st, const int32_t* outer_done,
                              hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_finish, dim3(nsys), dim3(kFinThreads), 0, stream, L.blk_first,
                     Ld.blk_first, part, dots, st, 0, 2, 0.0, outer_done, nullptr, nullptr);
  return hipGetLastError();
}

// Reliable update of the low-precision CG: r = the true residual r64 (FP64,
// zero off the free DOFs) rounded to T, u = M^{-1} r, w = 0, partial sums of
// (r, u) and (r, r); p and s are left as they are.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_reliable(const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ u,
                  T* __restrict__ w, const T* __restrict__ dinv, double* __restrict__ part) {
  __shared__ double sh[2 * (kVecBlock / 64)];
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  double g = 0.0, rr = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const T ri = (T)r64[i];
    const T ui = ri * dinv[i];
    r[i] = ri;
    u[i] = ui;
    w[i] = T(0);
    g += (double)ri * (double)ui;
    rr += (double)ri * (double)ri;
  }
  double v[2] = {g, rr};
  block_sums<kVecBlock, 2>(v, sh);
  store_parts(v[0], v[1], part);
}

hipError_t cg_reliable(const VecLayout& L, const double* r64, float* r, float* u, float* w,
                       const float* dinv, double* part, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_reliable<float>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream, r64,
                     r, u, w, dinv, part);
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

// Internal l2g: user global index g of system s -> padded index gi, with the
// sign flag (bit 30) for sign[id] = -1, stored as gi (free) or -1-gi
// (Dirichlet).  Out-of-range indices or signs other than +-1 set *bad.
__global__ void k_build_l2g(int64_t nelem, int nloc, const int32_t* __restrict__ elem_seg,
                            const int64_t* __restrict__ dof_off,
                            const int64_t* __restrict__ pdof_off,
                            const int32_t* __restrict__ l2g_user, const int8_t* __restrict__ sign,
                            const uint8_t* __restrict__ dirichlet, int32_t* __restrict__ l2g_int,
                            int* bad) {
  const int64_t tot = nelem * nloc;
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < tot;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = id / nloc;
    const int s = elem_seg[e];
    const int64_t g = l2g_user[id];
    const int sg = sign ? sign[id] : 1;
    if (g < dof_off[s] || g >= dof_off[s + 1] || (sg != 1 && sg != -1)) {
      atomicOr(bad, 1);
      l2g_int[id] = -1 - (int32_t)pdof_off[s];
      continue;
    }
    const int32_t gi = (int32_t)(g - dof_off[s] + pdof_off[s]) | (sg < 0 ? kL2gNeg : 0);
    l2g_int[id] = dirichlet[g] ? -1 - gi : gi;
  }
}

hipError_t build_l2g(int64_t nelem, int nloc, const int32_t* elem_seg, const int64_t* dof_off,
                     const int64_t* pdof_off, const int32_t* l2g_user, const int8_t* sign,
                     const uint8_t* dirichlet, int32_t* l2g_int, int* bad, hipStream_t s) {
  const int64_t tot = nelem * nloc;
  if (tot == 0) return hipSuccess;
  int64_t nb = (tot + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_build_l2g, dim3((unsigned)nb), dim3(256), 0, s, nelem, nloc, elem_seg,
                     dof_off, pdof_off, l2g_user, sign, dirichlet, l2g_int, bad);
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
    if (g >= 0) mark[l2g_dof(g)] = 1.0;
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
    xl[id] = l2g_sign(g, x[l2g_dof(g)]);
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
    if (g >= 0) unsafeAtomicAdd(y + l2g_dof(g), l2g_sign(g, yl[id]));
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

// Internal l2g entries of a one-system system back to the user form it was
// built from: global DOF + off, orientation sign, Dirichlet flag of the DOF
// (dirichlet must be zero on entry; entries of one DOF agree, so concurrent
// writes store the same byte).
__global__ void k_decode_l2g(int64_t n, const int32_t* __restrict__ l2g_int, int64_t off,
                             int32_t* __restrict__ l2g_user, int8_t* __restrict__ sign,
                             uint8_t* __restrict__ dirichlet) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = l2g_int[i];
    const int64_t g = (int64_t)l2g_dof(v) + off;
    l2g_user[i] = (int32_t)g;
    sign[i] = l2g_neg(v) ? int8_t(-1) : int8_t(1);
    if (v < 0) dirichlet[g] = 1;
  }
}

hipError_t decode_l2g(int64_t n, const int32_t* l2g_int, int64_t off, int32_t* l2g_user,
                      int8_t* sign, uint8_t* dirichlet, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_decode_l2g, dim3((unsigned)nb), dim3(256), 0, s, n, l2g_int, off, l2g_user,
                     sign, dirichlet);
  return hipGetLastError();
}

// One system's padded segment from its own user vector: padded[i] = user[i]
// for i < n on free DOFs (dinv != 0), 0 on Dirichlet and padding entries.
template <typename T>
__global__ void k_seg_in(int64_t n, int64_t npad, const T* __restrict__ user,
                         const double* __restrict__ dinv, T* __restrict__ padded) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * blockDim.x)
    padded[i] = (i < n && dinv[i] != 0.0) ? user[i] : T(0);
}

hipError_t seg_in(int64_t n, int64_t npad, const double* user, const double* dinv, double* padded,
                  hipStream_t s) {
  if (npad == 0) return hipSuccess;
  int64_t nb = (npad + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_seg_in<double>, dim3((unsigned)nb), dim3(256), 0, s, n, npad, user, dinv,
                     padded);
  return hipGetLastError();
}

template <typename T>
__global__ void k_seg_out(int64_t n, const T* __restrict__ padded, T* __restrict__ user) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    user[i] = padded[i];
}

hipError_t seg_out(int64_t n, const double* padded, double* user, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_seg_out<double>, dim3((unsigned)nb), dim3(256), 0, s, n, padded, user);
  return hipGetLastError();
}

template hipError_t cg_update<double>(const VecLayout&, CgState, double*, double*, double*,
                                      double*, double*, double*, const double*, double*,
                                      hipStream_t);
template hipError_t cg_update<float>(const VecLayout&, CgState, float*, float*, float*, float*,
                                     float*, float*, const float*, double*, hipStream_t);
template hipError_t cg_start<double>(const VecLayout&, const double*, double*, double*, double*,
                                     double*, double*, const double*, double*, hipStream_t);
template hipError_t cg_start<float>(const VecLayout&, const double*, float*, float*, float*,
                                    float*, float*, const float*, double*, hipStream_t);
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
