// Vector kernels of the Jacobi-preconditioned conjugate-gradient solver and
// the assembly helpers.  Each block of kVecBlock threads owns kSegAlign
// consecutive DOFs of one system.  The CG iteration's reductions go through
// per-system accumulation slots (below); the residual and norm kernels finish
// their per-system sums in the last block of the system.
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
// One iteration j is two kernels: cg_update (every block first forms the
// system's gamma, r.r, delta, alpha and beta itself from kSlots accumulation
// slots, then updates its vectors and adds its partials of the next gamma and
// r.r to the slots) and the assembled operator w = A u (each element adds
// u_e.(H_e u_e) to a slot).  No separate reduction kernel and no grid-wide
// fence: the slots are filled with atomics by one kernel and read by the next.
// Slot sets rotate so that no kernel reads a set that is being filled or
// cleared: gamma / r.r sets by j mod 3 (iteration j reads set j, fills j+1,
// clears j+2), delta sets by j mod 2 (iteration j's update reads set j and
// clears j+1, its operator fills j+1), and the carried scalars (gamma, alpha,
// iterations, stopped) by j mod 2 (read j-1, written j by the system's first
// block).  Captured graphs hold a multiple of 6 iterations, so iteration j of
// every launch sees the same sets.
constexpr int kGS = 2 * kSlots;   // gamma slots then r.r slots, per system and set

__device__ __forceinline__ double* gslot(const CgState& st, int nsys, int q, int s) {
  return st.gsl + ((int64_t)q * nsys + s) * kGS;
}
__device__ __forceinline__ double* dslot_set(const CgState& st, int nsys, int q, int s) {
  return st.dsl + ((int64_t)q * nsys + s) * kSlots;
}

// Sums of a system's slots (one per thread: kSlots = kVecBlock), broadcast
// to every thread of the block.
__device__ __forceinline__ void slot_sums(const double* g, const double* d, double* sh,
                                          double& gam, double& rr, double& del) {
  static_assert(kSlots == kVecBlock, "one slot per thread");
  const int t = threadIdx.x;
  double v[3] = {g[t], g[kSlots + t], d[t]};
  block_sums<kVecBlock, 3>(v, sh);
  __shared__ double bc[3];
  if (t == 0) {
    bc[0] = v[0];
    bc[1] = v[1];
    bc[2] = v[2];
  }
  __syncthreads();
  gam = bc[0];
  rr = bc[1];
  del = bc[2];
}

// The leader block of a system clears the slot sets it owns this iteration.
__device__ __forceinline__ void clear_slots(double* g, double* d) {
  const int t = threadIdx.x;
  g[t] = 0.0;
  g[kSlots + t] = 0.0;
  d[t] = 0.0;
}

template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_update(const int32_t* __restrict__ blk_seg, const int64_t* __restrict__ blk_first,
                CgState st, int nsys, int j, int fatal, const int32_t* __restrict__ skip,
                T* __restrict__ x, T* __restrict__ r, T* __restrict__ u, T* __restrict__ p,
                T* __restrict__ s, T* __restrict__ w, const T* __restrict__ dinv) {
  __shared__ double sh[3 * (kVecBlock / 64)];
  const int sg = blk_seg[blockIdx.x];
  const bool leader = blockIdx.x == blk_first[sg];
  const int qg = j % 3, qd = j & 1, qp = (j + 1) & 1;   // qp: the set written last iteration
  const int64_t cur = (int64_t)qd * nsys + sg, prev = (int64_t)qp * nsys + sg;
  // the block's vectors are requested first, so their loads overlap the
  // reduction of the slots that decides the step
  const int64_t base = (int64_t)blockIdx.x * kSegAlign + threadIdx.x;
  T vd[kPer], vr[kPer], vp[kPer], vw[kPer], vs[kPer];
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    vd[c] = dinv[i];
    vr[c] = r[i];
    vp[c] = p[i];
    vw[c] = w[i];
    vs[c] = s[i];
  }
  const double gp = st.sgam[prev], ap = st.salp[prev];
  const int itp = st.sit[prev], dnp = st.sdn[prev];
  double gam, rr, del;
  slot_sums(gslot(st, nsys, qg, sg), dslot_set(st, nsys, qd, sg), sh, gam, rr, del);
  if (leader) clear_slots(gslot(st, nsys, (j + 2) % 3, sg), dslot_set(st, nsys, qp, sg));
  if (dnp || (skip && skip[sg])) {
    // stopped: carry the state to this iteration's set
    if (leader && threadIdx.x == 0) {
      st.sgam[cur] = gp;
      st.salp[cur] = ap;
      st.sit[cur] = itp;
      st.sdn[cur] = 1;
      st.done[sg] = 1;
    }
    return;
  }
  bool stop = false;
  int status = 0;
  double beta = 0.0, alpha = 0.0;
  if (!isfinite(rr) || !isfinite(gam) || !isfinite(del)) {
    stop = true;
    status = NK_EBREAKDOWN;
  } else if (rr <= st.tol2[sg] || rr == 0.0) {
    stop = true;
  } else if (itp >= st.maxit[sg]) {
    stop = true;
    if (fatal) status = NK_ENOCONV;
  } else {
    // After a reliable update the new residual is not orthogonal to the old
    // directions to working precision; where that spoils p.Ap (or in the low
    // precision, where rounding does), the direction restarts from u.
    beta = gp > 0.0 ? gam / gp : 0.0;
    double den = gp > 0.0 ? del - beta * gam / ap : del;
    if (!(den > 0.0) || !isfinite(den)) {
      if (fatal) {
        stop = true;
        status = NK_EBREAKDOWN;
      } else {
        beta = 0.0;
        den = del;
        if (!(den > 0.0)) {
          stop = true;
          status = NK_EBREAKDOWN;
        }
      }
    }
    if (!stop) alpha = gam / den;
  }
  if (leader && threadIdx.x == 0) {
    st.sgam[cur] = stop ? gp : gam;
    st.salp[cur] = stop ? ap : alpha;
    st.sit[cur] = stop ? itp : itp + 1;
    st.sdn[cur] = stop ? 1 : 0;
    st.done[sg] = stop ? 1 : 0;
    st.iters[sg] = stop ? itp : itp + 1;
    st.rr[sg] = rr;
    st.rz[sg] = gam;
    st.alpha[sg] = alpha;
    if (status) st.status[sg] = status;
  }
  if (stop) return;
  const T a = (T)alpha, b = (T)beta;
  double g = 0.0, r2 = 0.0;
#pragma unroll
  for (int c = 0; c < kPer; ++c) {
    const int64_t i = base + c * kVecBlock;
    const T pi = vr[c] * vd[c] + b * vp[c];
    const T si = vw[c] + b * vs[c];
    x[i] += a * pi;
    const T rn = vr[c] - a * si;
    const T un = rn * vd[c];
    p[i] = pi;
    s[i] = si;
    r[i] = rn;
    u[i] = un;
    w[i] = T(0);
    g += (double)rn * (double)un;
    r2 += (double)rn * (double)rn;
  }
  double v[2] = {g, r2};
  block_sums<kVecBlock, 2>(v, sh);
  if (threadIdx.x == 0) {
    double* gs = gslot(st, nsys, (j + 1) % 3, sg);
    const int k = blockIdx.x % kSlots;
    unsafeAtomicAdd(gs + k, v[0]);
    unsafeAtomicAdd(gs + kSlots + k, v[1]);
  }
}

template <typename T>
hipError_t cg_update(const VecLayout& L, CgState st, int nsys, int j, bool fatal,
                     const int32_t* skip, T* x, T* r, T* u, T* p, T* s, T* w, const T* dinv,
                     hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_update<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream,
                     L.blk_seg, L.blk_first, st, nsys, j, fatal ? 1 : 0, skip, x, r, u, p, s, w,
                     dinv);
  return hipGetLastError();
}

// Start of a solve: r = (b - w) on free DOFs (w = A x0, or 0), u = M^{-1} r,
// p = s = w = 0, partial sums of (r, u) and (r, r) into gamma set 0.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_start(const int32_t* __restrict__ blk_seg, CgState st, int nsys,
               const double* __restrict__ b, T* __restrict__ w, T* __restrict__ r,
               T* __restrict__ u, T* __restrict__ p, T* __restrict__ s,
               const T* __restrict__ dinv) {
  __shared__ double sh[2 * (kVecBlock / 64)];
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
  if (threadIdx.x == 0) {
    double* gs = gslot(st, nsys, 0, blk_seg[blockIdx.x]);
    const int k = blockIdx.x % kSlots;
    unsafeAtomicAdd(gs + k, v[0]);
    unsafeAtomicAdd(gs + kSlots + k, v[1]);
  }
}

template <typename T>
hipError_t cg_start(const VecLayout& L, CgState st, int nsys, const double* b, T* w, T* r, T* u,
                    T* p, T* s, const T* dinv, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_start<T>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream,
                     L.blk_seg, st, nsys, b, w, r, u, p, s, dinv);
  return hipGetLastError();
}

// One block per system after the start kernel and the first operator (which
// filled gamma set 0 and delta set 0): iteration counters, the starting
// residual, tol2 for the inner solves of the refinement (tau2 > 0: reduce by
// tau, or only as far as the outer tolerance still needs, with a factor 1/2
// of margin), and the carried scalars the first update reads (set 1: no
// previous gamma, so beta = 0).
__global__ void __launch_bounds__(kVecBlock)
    k_cg_begin(CgState st, int nsys, double tau2, const int32_t* __restrict__ skip,
               const double* __restrict__ outer_tol2, const double* __restrict__ outer_rr) {
  __shared__ double sh[3 * (kVecBlock / 64)];
  const int sg = blockIdx.x;
  double gam, rr, del;
  slot_sums(gslot(st, nsys, 0, sg), dslot_set(st, nsys, 0, sg), sh, gam, rr, del);
  (void)gam;
  (void)del;
  if (threadIdx.x != 0) return;
  st.iters[sg] = 0;
  st.status[sg] = 0;
  st.rr[sg] = rr;
  if (tau2 > 0.0) {
    const double need = outer_rr[sg] > 0.0 ? 0.25 * outer_tol2[sg] / outer_rr[sg] : 0.0;
    st.tol2[sg] = (need > tau2 ? need : tau2) * rr;
  }
  const bool stop = (skip != nullptr && skip[sg] != 0) || rr <= st.tol2[sg] || rr == 0.0;
  const int64_t q1 = (int64_t)nsys + sg;
  st.sgam[q1] = 0.0;
  st.salp[q1] = 1.0;
  st.sit[q1] = 0;
  st.sdn[q1] = stop ? 1 : 0;
  st.done[sg] = stop ? 1 : 0;
}

hipError_t cg_begin_scalars(CgState st, int nsys, double tau2, const int32_t* skip,
                            const double* outer_tol2, const double* outer_rr, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_begin, dim3(nsys), dim3(kVecBlock), 0, stream, st, nsys, tau2, skip,
                     outer_tol2, outer_rr);
  return hipGetLastError();
}

// Reliable update of the low-precision CG: r = the true residual r64 (FP64,
// zero off the free DOFs) rounded to T, u = M^{-1} r, w = 0, partial sums of
// (r, u) and (r, r) into gamma set 0 (cleared beforehand with delta set 0);
// p and s are left as they are.  The next update (iteration 0 of a graph
// launch) then redoes the last step with the new gamma and delta.
template <typename T>
__global__ void __launch_bounds__(kVecBlock)
    k_cg_reliable(const int32_t* __restrict__ blk_seg, CgState st, int nsys,
                  const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ u,
                  T* __restrict__ w, const T* __restrict__ dinv) {
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
  if (threadIdx.x == 0) {
    double* gs = gslot(st, nsys, 0, blk_seg[blockIdx.x]);
    const int k = blockIdx.x % kSlots;
    unsafeAtomicAdd(gs + k, v[0]);
    unsafeAtomicAdd(gs + kSlots + k, v[1]);
  }
}

hipError_t cg_reliable(const VecLayout& L, CgState st, int nsys, const double* r64, float* r,
                       float* u, float* w, const float* dinv, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_reliable<float>, dim3((unsigned)L.nblk), dim3(kVecBlock), 0, stream,
                     L.blk_seg, st, nsys, r64, r, u, w, dinv);
  return hipGetLastError();
}

// Re-arm the systems that are still running after a reliable update: the
// next update (which reads carried set 1) continues them from the new
// residual; skipped systems stay stopped.
__global__ void k_cg_rearm(CgState st, int nsys, const int32_t* __restrict__ skip) {
  const int sg = blockIdx.x * blockDim.x + threadIdx.x;
  if (sg >= nsys) return;
  const int stop = skip != nullptr && skip[sg] != 0;
  st.sdn[(int64_t)nsys + sg] = stop;
  st.done[sg] = stop;
}

hipError_t cg_rearm(CgState st, int nsys, const int32_t* skip, hipStream_t stream) {
  hipLaunchKernelGGL(k_cg_rearm, dim3((nsys + 255) / 256), dim3(256), 0, stream, st, nsys, skip);
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

template hipError_t cg_update<double>(const VecLayout&, CgState, int, int, bool, const int32_t*,
                                      double*, double*, double*, double*, double*, double*,
                                      const double*, hipStream_t);
template hipError_t cg_update<float>(const VecLayout&, CgState, int, int, bool, const int32_t*,
                                     float*, float*, float*, float*, float*, float*, const float*,
                                     hipStream_t);
template hipError_t cg_start<double>(const VecLayout&, CgState, int, const double*, double*,
                                     double*, double*, double*, double*, const double*, hipStream_t);
template hipError_t cg_start<float>(const VecLayout&, CgState, int, const double*, float*, float*,
                                    float*, float*, float*, const float*, hipStream_t);
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
