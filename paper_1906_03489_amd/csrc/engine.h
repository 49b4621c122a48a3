// Sum-factorised elemental operators on tensor-product elements (device code).
//
// Section 3.3 of arXiv 1906.03489 evaluates an expansion at the quadrature
// points by contracting one direction at a time (the sum-factorisation
// display), across many elements of one collection concurrently ("SumFac").
//
// CDNA4 mapping.  One element is handled by one "slot" of NT >= Q*Q threads.
// Each thread owns a pencil (a line of values along one direction) in
// registers, so every contraction is a register-local product with a 1-D
// matrix that is uniform across the wavefront.  The stages loop over pairs of
// mirrored points (k and Q-1-k, even-odd form below) and unroll the mode
// index, so each iteration needs one row of B and of DB, which the scalar
// unit loads from the kernel arguments; the FP64/FP32 FMAs take it as their
// scalar operand.  Between directions the pencils are re-oriented through
// LDS.
//
// Forward (coefficients -> values and reference gradient at the points):
//   K: thread (p,q)  r -> k with B and DB           -> t_B, t_D   [k][q][p]
//   J: thread (p,k)  q -> j                         -> s_BB, s_DB, s_BD [k][j][p]
//   I: thread (j,k)  p -> i, fused with the pointwise factors and with the
//      transposed I stage, one pair of points (or one point) per iteration
// Backward (transpose), summing m and the three flux components:
//   I': thread (j,k) i -> p                         -> s'_BB, s'_DB, s'_BD
//   J': thread (p,k) j -> q                         -> t'_B, t'_D
//   K': thread (p,q) k -> r                         -> coefficients
// y = (B(x)B(x)B)^T m + sum_a (D_a(B(x)B(x)B))^T g_a, with the derivative
// factors carried as separate tensors so no collocation-derivative pass is
// needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nk_internal.h"
#include "tiles.h"

namespace nk {

// 1-D tables: B and D at the Q GLL points, and X[i] = -x_i/2 for the first
// H = ceil(Q/2) points.
//
// The GLL points are symmetric, x_{Q-1-i} = -x_i, and of the modified modes
// the interior ones phi_p (0 < p < P) are even functions for odd p and odd
// functions for even p, while the vertex pair splits into the even sum
// phi_0 + phi_P (= 1) and the odd difference phi_0 - phi_P (= -x).  The
// contractions use this as the even-odd decomposition of a matrix that
// commutes with the reflection (Solomonoff, "A fast algorithm for spectral
// differentiation", J. Comput. Phys. 98, 1992), reading only the rows of the
// first H points.  Coefficients c split into
//   ce = (c_0 + c_P, c_1, c_3, ...)   (KE = P/2 + 1 entries)
//   co = (c_0 - c_P, c_2, c_4, ...)   (KO = (P-1)/2 + 1 entries)
// whose members at x_i are (1/2, phi_1, phi_3, ...) and (-x_i/2, phi_2, ...),
// with derivatives (0, phi'_1, ...) and (-1/2, phi'_2, ...).  With E, O the
// even and odd sums: u(x_i) = E + O, u(x_{Q-1-i}) = E - O, and likewise for
// u' from the derivative sums (Ed from co, Od from ce), so a pair of points
// costs N products instead of 2N.  The transposed contraction takes
// v_i + v_{Q-1-i} and v_i - v_{Q-1-i} against the same rows and unpacks the
// vertex pair; the middle point of an odd Q (x = 0) meets only the even
// members and the derivatives of the odd ones.
template <typename T, int N, int Q>
struct Tab {
  T B[Q * N];            // B[i*N + p] = phi_p(x_i)
  T D[Q * N];            // D[i*N + p] = phi_p'(x_i)
  T X[(Q + 1) / 2];      // X[i] = -x_i / 2
};

template <int N>
struct EO {
  static constexpr int P = N - 1;
  static constexpr int KE = P / 2 + 1;
  static constexpr int KO = (P - 1) / 2 + 1;
};

template <typename T, int N>
__device__ __forceinline__ void eo_split(const T (&c)[N], T (&ce)[EO<N>::KE], T (&co)[EO<N>::KO]) {
  ce[0] = c[0] + c[N - 1];
  co[0] = c[0] - c[N - 1];
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) ce[m] = c[2 * m - 1];
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) co[m] = c[2 * m];
}

template <typename T, int N>
__device__ __forceinline__ void eo_join(const T (&ye)[EO<N>::KE], const T (&yo)[EO<N>::KO], T (&y)[N]) {
  y[0] = ye[0] + yo[0];
  y[N - 1] = ye[0] - yo[0];
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) y[2 * m - 1] = ye[m];
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) y[2 * m] = yo[m];
}

// values at x_h and x_{Q-1-h}
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_val(const Tab<T, N, Q>& tb, int h, const T (&ce)[EO<N>::KE],
                                       const T (&co)[EO<N>::KO], T& lo, T& hi) {
  const T* b = tb.B + h * N;
  T e = T(0.5) * ce[0], o = tb.X[h] * co[0];
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) e += b[2 * m - 1] * ce[m];
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) o += b[2 * m] * co[m];
  lo = e + o;
  hi = e - o;
}

// derivatives at x_h and x_{Q-1-h}
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_der(const Tab<T, N, Q>& tb, int h, const T (&ce)[EO<N>::KE],
                                       const T (&co)[EO<N>::KO], T& lo, T& hi) {
  const T* d = tb.D + h * N;
  T e = T(-0.5) * co[0], o = T(0);
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) e += d[2 * m] * co[m];
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) o += d[2 * m - 1] * ce[m];
  lo = e + o;
  hi = e - o;
}

// value and derivative at the middle point of an odd Q
template <typename T, int N, int Q>
__device__ __forceinline__ T eo_mid_val(const Tab<T, N, Q>& tb, const T (&ce)[EO<N>::KE]) {
  const T* b = tb.B + (Q / 2) * N;
  T e = T(0.5) * ce[0];
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) e += b[2 * m - 1] * ce[m];
  return e;
}
template <typename T, int N, int Q>
__device__ __forceinline__ T eo_mid_der(const Tab<T, N, Q>& tb, const T (&co)[EO<N>::KO]) {
  const T* d = tb.D + (Q / 2) * N;
  T e = T(-0.5) * co[0];
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) e += d[2 * m] * co[m];
  return e;
}

// transposed: ye += (even members at x_h) vp, yo += (odd members) vm, with
// vp = v_h + v_{Q-1-h}, vm = v_h - v_{Q-1-h}
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_acc(const Tab<T, N, Q>& tb, int h, T vp, T vm,
                                       T (&ye)[EO<N>::KE], T (&yo)[EO<N>::KO]) {
  const T* b = tb.B + h * N;
  ye[0] += T(0.5) * vp;
  yo[0] += tb.X[h] * vm;
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) ye[m] += b[2 * m - 1] * vp;
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) yo[m] += b[2 * m] * vm;
}
// transposed derivative: ye += (even members)' wm, yo += (odd members)' wp
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_acc_d(const Tab<T, N, Q>& tb, int h, T wp, T wm,
                                         T (&ye)[EO<N>::KE], T (&yo)[EO<N>::KO]) {
  const T* d = tb.D + h * N;
  yo[0] += T(-0.5) * wp;
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) ye[m] += d[2 * m - 1] * wm;
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) yo[m] += d[2 * m] * wp;
}
// the middle point of an odd Q: value v, derivative weight w
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_acc_mid(const Tab<T, N, Q>& tb, T v, T (&ye)[EO<N>::KE]) {
  const T* b = tb.B + (Q / 2) * N;
  ye[0] += T(0.5) * v;
#pragma unroll
  for (int m = 1; m < EO<N>::KE; ++m) ye[m] += b[2 * m - 1] * v;
}
template <typename T, int N, int Q>
__device__ __forceinline__ void eo_acc_mid_d(const Tab<T, N, Q>& tb, T w, T (&yo)[EO<N>::KO]) {
  const T* d = tb.D + (Q / 2) * N;
  yo[0] += T(-0.5) * w;
#pragma unroll
  for (int m = 1; m < EO<N>::KO; ++m) yo[m] += d[2 * m] * w;
}

template <typename T, int K>
__device__ __forceinline__ void zero(T (&v)[K]) {
#pragma unroll
  for (int m = 0; m < K; ++m) v[m] = T(0);
}

template <typename T>
struct DevArgs {
  int64_t nelem;
  const T* in;
  T* out;
  const T* fac;
  const double* lam;
  double lam0;
  const int32_t* l2g;
  double* dots;
  const double* in2;
  double* out2;
  const double* kappa;
  const int32_t* elem_seg;
  const int32_t* seg_done;
  const int32_t* dslot;
};

template <typename T>
inline DevArgs<T> dev_args(const OpArgs& a) {
  DevArgs<T> d;
  d.nelem = a.nelem;
  d.in = static_cast<const T*>(a.in);
  d.out = static_cast<T*>(a.out);
  d.fac = static_cast<const T*>(a.fac);
  d.lam = a.lam;
  d.lam0 = a.lam0;
  d.l2g = a.l2g;
  d.dots = a.dots;
  d.in2 = a.in2;
  d.out2 = a.out2;
  d.kappa = a.kappa;
  d.elem_seg = a.elem_seg;
  d.seg_done = a.seg_done;
  d.dslot = a.dslot;
  return d;
}

// Blocks are dispatched round-robin over the 8 XCDs (each with its own L2).
// Remap so that every XCD processes one contiguous range of elements, which
// keeps neighbouring elements (sharing global DOFs in assembled operators)
// in the same L2.  Bijective for any nblk.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t nblk) {
  const int64_t per = nblk >> 3, rem = nblk & 7;
  const int64_t x = b & 7, i = b >> 3;
  return x * per + (x < rem ? x : rem) + i;
}

__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
// An assembled operator's element energy u_e.(H_e u_e) is added to the CG
// accumulation slot dslot[e] of its system.
__device__ __forceinline__ void add_dot(double* dots, const int32_t* dslot, int64_t e, double v) {
  unsafeAtomicAdd(dots + dslot[e], v);
}

// Slot synchronisation.  When every slot lies inside one wavefront (NT
// divides 64) only the owning wavefront touches the slot's LDS, and LDS
// operations of a wavefront complete in program order, so a compiler-level
// fence is enough; otherwise the whole block synchronises.
template <int NT>
__device__ __forceinline__ void slot_sync() {
  if constexpr (64 % NT == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

// LDS scalars per slot: three tensors of Q*Q*N.
template <int N, int Q>
constexpr int slot_lds() {
  return 3 * Q * Q * N;
}

// ---------------------------------------------------------------- stages
// Every stage is executed by all threads of the block (barriers inside);
// `act` masks the threads that own a pencil of a live element.

// I-stage inputs of thread (j,k) = t < Q^2: s_BB, s_DB, s_BD [k][j][p].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void load_i(const T* __restrict__ sm, int t, T (&av)[N], T (&bv)[N],
                                       T (&cv)[N]) {
  constexpr int S = Q * Q * N;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    av[p] = sm[t * N + p];
    if constexpr (DER) {
      bv[p] = sm[S + t * N + p];
      cv[p] = sm[2 * S + t * N + p];
    }
  }
}

// Store the I' accumulators of thread (j,k) as s'_BB, s'_DB, s'_BD [k][j][p].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void store_i(T* __restrict__ sm, int t, const T (&sa)[N],
                                        const T (&sb)[N], const T (&sc)[N]) {
  constexpr int S = Q * Q * N;
#pragma unroll
  for (int p = 0; p < N; ++p) {
    sm[t * N + p] = sa[p];
    if constexpr (DER) {
      sm[S + t * N + p] = sb[p];
      sm[2 * S + t * N + p] = sc[p];
    }
  }
}

// The four contraction stages, each with the even-odd tables: every output
// pair (k, Q-1-k) from one pass over the split pencil.
// K: thread t = p + N q (< N^2) holds xin[r]; writes t_B (and t_D) [k][q][p].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void stage_k(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool act,
                                        const T (&xin)[N]) {
  constexpr int NN = N * N, S = Q * Q * N, HP = Q / 2;
  if (act && t < NN) {
    T xe[EO<N>::KE], xo[EO<N>::KO];
    eo_split<T, N>(xin, xe, xo);
#pragma unroll 2
    for (int h = 0; h < HP; ++h) {
      T lo, hi;
      eo_val(tb, h, xe, xo, lo, hi);
      sm[h * NN + t] = lo;
      sm[(Q - 1 - h) * NN + t] = hi;
      if constexpr (DER) {
        eo_der(tb, h, xe, xo, lo, hi);
        sm[S + h * NN + t] = lo;
        sm[S + (Q - 1 - h) * NN + t] = hi;
      }
    }
    if constexpr (Q & 1) {
      sm[HP * NN + t] = eo_mid_val(tb, xe);
      if constexpr (DER) sm[S + HP * NN + t] = eo_mid_der(tb, xo);
    }
  }
}

// J: thread (p,k) = t < N Q reads t_B, t_D; writes s_BB, s_DB, s_BD [k][j][p].
template <typename T, int N, int Q, int NT, bool DER>
__device__ __forceinline__ void stage_j(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool act) {
  constexpr int NN = N * N, S = Q * Q * N, HP = Q / 2, KE = EO<N>::KE, KO = EO<N>::KO;
  const int pj = t % N, kj = t / N;
  const bool me = act && t < N * Q;
  T ae[KE], ao[KO], be[KE], bo[KO];
  if (me) {
    T av[N], bv[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      av[q] = sm[kj * NN + q * N + pj];
      if constexpr (DER) bv[q] = sm[S + kj * NN + q * N + pj];
    }
    eo_split<T, N>(av, ae, ao);
    if constexpr (DER) eo_split<T, N>(bv, be, bo);
  }
  slot_sync<NT>();
  if (me) {
    const int o0 = kj * Q * N + pj;
#pragma unroll 2
    for (int h = 0; h < HP; ++h) {
      const int ol = o0 + h * N, oh = o0 + (Q - 1 - h) * N;
      T lo, hi;
      eo_val(tb, h, ae, ao, lo, hi);
      sm[ol] = lo;
      sm[oh] = hi;
      if constexpr (DER) {
        eo_der(tb, h, ae, ao, lo, hi);
        sm[S + ol] = lo;
        sm[S + oh] = hi;
        eo_val(tb, h, be, bo, lo, hi);
        sm[2 * S + ol] = lo;
        sm[2 * S + oh] = hi;
      }
    }
    if constexpr (Q & 1) {
      const int om = o0 + HP * N;
      sm[om] = eo_mid_val(tb, ae);
      if constexpr (DER) {
        sm[S + om] = eo_mid_der(tb, ao);
        sm[2 * S + om] = eo_mid_val(tb, be);
      }
    }
  }
}

// J': thread (p,k) = t < N Q sums over j; writes t'_B, t'_D [k][q][p].
template <typename T, int N, int Q, int NT, bool DER>
__device__ __forceinline__ void stage_jt(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t,
                                         bool act) {
  constexpr int NN = N * N, S = Q * Q * N, HP = Q / 2, KE = EO<N>::KE, KO = EO<N>::KO;
  const int pj = t % N, kj = t / N;
  const bool me = act && t < N * Q;
  T tBe[KE], tBo[KO], tDe[KE], tDo[KO];
  zero(tBe);
  zero(tBo);
  zero(tDe);
  zero(tDo);
  if (me) {
    const int o0 = kj * Q * N + pj;
#pragma unroll 2
    for (int h = 0; h < HP; ++h) {
      const int ol = o0 + h * N, oh = o0 + (Q - 1 - h) * N;
      const T a1 = sm[ol], a2 = sm[oh];
      eo_acc(tb, h, a1 + a2, a1 - a2, tBe, tBo);
      if constexpr (DER) {
        const T b1 = sm[S + ol], b2 = sm[S + oh], c1 = sm[2 * S + ol], c2 = sm[2 * S + oh];
        eo_acc_d(tb, h, b1 + b2, b1 - b2, tBe, tBo);
        eo_acc(tb, h, c1 + c2, c1 - c2, tDe, tDo);
      }
    }
    if constexpr (Q & 1) {
      const int om = o0 + HP * N;
      eo_acc_mid(tb, sm[om], tBe);
      if constexpr (DER) {
        eo_acc_mid_d(tb, sm[S + om], tBo);
        eo_acc_mid(tb, sm[2 * S + om], tDe);
      }
    }
  }
  slot_sync<NT>();
  if (me) {
    T tB[N];
    eo_join<T, N>(tBe, tBo, tB);
#pragma unroll
    for (int q = 0; q < N; ++q) sm[kj * NN + q * N + pj] = tB[q];
    if constexpr (DER) {
      T tD[N];
      eo_join<T, N>(tDe, tDo, tD);
#pragma unroll
      for (int q = 0; q < N; ++q) sm[S + kj * NN + q * N + pj] = tD[q];
    }
  }
}

// K': thread (p,q) = t < N^2 sums over k into y[r].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void stage_kt(const Tab<T, N, Q>& tb, const T* __restrict__ sm, int t,
                                         bool act, T (&yv)[N]) {
  constexpr int NN = N * N, S = Q * Q * N, HP = Q / 2, KE = EO<N>::KE, KO = EO<N>::KO;
  T ye[KE], yo[KO];
  zero(ye);
  zero(yo);
  if (act && t < NN) {
#pragma unroll 2
    for (int h = 0; h < HP; ++h) {
      const T a1 = sm[h * NN + t], a2 = sm[(Q - 1 - h) * NN + t];
      eo_acc(tb, h, a1 + a2, a1 - a2, ye, yo);
      if constexpr (DER) {
        const T b1 = sm[S + h * NN + t], b2 = sm[S + (Q - 1 - h) * NN + t];
        eo_acc_d(tb, h, b1 + b2, b1 - b2, ye, yo);
      }
    }
    if constexpr (Q & 1) {
      eo_acc_mid(tb, sm[HP * NN + t], ye);
      if constexpr (DER) eo_acc_mid_d(tb, sm[S + HP * NN + t], yo);
    }
  }
  eo_join<T, N>(ye, yo, yv);
}

// Sum of v over the threads of a slot, valid in thread t == 0 of the slot.
template <int NT>
__device__ __forceinline__ double slot_sum(double v, double* red, int slot, int t) {
  if constexpr (NT == 64) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  } else {
    __syncthreads();
    red[slot * NT + t] = v;
    __syncthreads();
    double s = 0.0;
    if (t == 0) {
      for (int i = 0; i < NT; ++i) s += red[slot * NT + i];
    }
    return s;
  }
}

// The paired I stage of the Helmholtz operator along one pencil: at each
// pair of points (h, Q-1-h), then the middle one of an odd Q, the forward
// contraction of the split inputs (a: the pencil, giving the value and the
// derivative along it; b, c: the tensors of the other two reference
// derivatives), the 7 factors with the lambda mass term, and the transposed
// contraction into the split accumulators (sa: mass and first gradient
// component, sb, sc: the other two).  load(i, f) fetches the factors of point
// i.  Sequence position s is point s/2 (even s) or Q-1-s/2 (odd s); PF
// register sets hold positions s .. s+PF-1, and before position s is
// computed the loads of s+PF-1 go into the set that s-1 has just released.
// One loop trip covers a multiple of 2 (a pair) and of PF positions, so that
// every set index is a constant.
template <typename T, int N, int Q, int PF, typename Load>
__device__ __forceinline__ void eo_helm_row(
    const Tab<T, N, Q>& tb, T lam, const T (&ae)[EO<N>::KE], const T (&ao)[EO<N>::KO],
    const T (&be)[EO<N>::KE], const T (&bo)[EO<N>::KO], const T (&ce)[EO<N>::KE],
    const T (&co)[EO<N>::KO], Load load, T (&sae)[EO<N>::KE], T (&sao)[EO<N>::KO],
    T (&sbe)[EO<N>::KE], T (&sbo)[EO<N>::KO], T (&sce)[EO<N>::KE], T (&sco)[EO<N>::KO]) {
  constexpr int HP = Q / 2;
  auto ld = [&](int s, T (&f)[kNF3]) {
    const int sc = s < Q ? s : Q - 1;
    load((sc & 1) ? Q - 1 - (sc >> 1) : (sc >> 1), f);
  };
  // r = (m, g1, g2, g3) at one point
  auto pointwise = [&](const T (&f)[kNF3], T u, T u1, T u2, T u3, T (&r)[4]) {
    r[0] = lam * f[0] * u;
    r[1] = f[1] * u1 + f[2] * u2 + f[3] * u3;
    r[2] = f[2] * u1 + f[4] * u2 + f[5] * u3;
    r[3] = f[3] * u1 + f[5] * u2 + f[6] * u3;
  };
  constexpr int L = (PF % 2 == 0) ? PF : 2 * PF;
  constexpr int PP = L / 2;
  T f[PF][kNF3];
#pragma unroll
  for (int s = 0; s + 1 < PF; ++s) ld(s, f[s]);
#pragma unroll 1
  for (int h0 = 0; h0 < HP; h0 += PP) {
#pragma unroll
    for (int q = 0; q < PP; ++q) {
      const int h = h0 + q;
      if (HP % PP == 0 || h < HP) {
        T ul[4], uh[4], rl[4], rh[4];
        eo_val(tb, h, ae, ao, ul[0], uh[0]);
        eo_der(tb, h, ae, ao, ul[1], uh[1]);
        eo_val(tb, h, be, bo, ul[2], uh[2]);
        eo_val(tb, h, ce, co, ul[3], uh[3]);
        ld(2 * h + PF - 1, f[(2 * q + PF - 1) % PF]);
        pointwise(f[(2 * q) % PF], ul[0], ul[1], ul[2], ul[3], rl);
        ld(2 * h + PF, f[(2 * q + PF) % PF]);
        pointwise(f[(2 * q + 1) % PF], uh[0], uh[1], uh[2], uh[3], rh);
        eo_acc(tb, h, rl[0] + rh[0], rl[0] - rh[0], sae, sao);
        eo_acc_d(tb, h, rl[1] + rh[1], rl[1] - rh[1], sae, sao);
        eo_acc(tb, h, rl[2] + rh[2], rl[2] - rh[2], sbe, sbo);
        eo_acc(tb, h, rl[3] + rh[3], rl[3] - rh[3], sce, sco);
      }
    }
  }
  if constexpr (Q & 1) {
    ld(2 * HP + PF - 1, f[(2 * HP + PF - 1) % PF]);
    T r[4];
    pointwise(f[(2 * HP) % PF], eo_mid_val(tb, ae), eo_mid_der(tb, ao), eo_mid_val(tb, be),
              eo_mid_val(tb, ce), r);
    eo_acc_mid(tb, r[0], sae);
    eo_acc_mid_d(tb, r[1], sao);
    eo_acc_mid(tb, r[2], sbe);
    eo_acc_mid(tb, r[3], sce);
  }
}

// The point-by-point I stage of the Helmholtz operator along one pencil, the
// unsplit counterpart of eo_helm_row (same inputs, factors and outputs, more
// products, fewer live registers).  PF register sets hold the factors of
// points i .. i+PF-1: before point i is computed, the loads of point i+PF-1
// go into the set that point i-1 has just released.  Loads are unconditional
// (clamped index) so that their waits sit right before their first use.
template <typename T, int N, int Q, int PF, typename Load>
__device__ __forceinline__ void plain_helm_row(const Tab<T, N, Q>& tb, T lam, const T (&a)[N],
                                               const T (&b)[N], const T (&c)[N], Load load,
                                               T (&sa)[N], T (&sb)[N], T (&sc)[N]) {
  auto point = [&](int i, const T (&f)[kNF3]) {
    const T* Bi = tb.B + i * N;
    const T* Di = tb.D + i * N;
    T u = 0, u1 = 0, u2 = 0, u3 = 0;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      u += Bi[p] * a[p];
      u1 += Di[p] * a[p];
      u2 += Bi[p] * b[p];
      u3 += Bi[p] * c[p];
    }
    const T m = lam * f[0] * u;
    const T g1 = f[1] * u1 + f[2] * u2 + f[3] * u3;
    const T g2 = f[2] * u1 + f[4] * u2 + f[5] * u3;
    const T g3 = f[3] * u1 + f[5] * u2 + f[6] * u3;
#pragma unroll
    for (int p = 0; p < N; ++p) {
      sa[p] += Bi[p] * m + Di[p] * g1;
      sb[p] += Bi[p] * g2;
      sc[p] += Bi[p] * g3;
    }
  };
  T f[PF][kNF3];
#pragma unroll
  for (int s = 0; s + 1 < PF; ++s) load(s < Q ? s : Q - 1, f[s]);
#pragma unroll 1
  for (int i = 0; i < Q; i += PF) {
#pragma unroll
    for (int s = 0; s < PF; ++s) {
      const int nx = i + s + PF - 1;
      load(nx < Q ? nx : Q - 1, f[(s + PF - 1) % PF]);
      if (Q % PF == 0 || i + s < Q) point(i + s, f[s]);
    }
  }
}

// Interior modes of the statically condensed operator: a slot thread t holds
// the modes (r, t / N, t % N), r = 0..N-1, and the element's (N-2)^3 interior
// modes (every index in 1..N-2) are numbered with r slowest, then t / N, then
// t % N (increasing local mode index).
template <int N>
__device__ __forceinline__ bool sc_inner(int t) {
  const int hi = t / N, lo = t - hi * N;
  return hi >= 1 && hi <= N - 2 && lo >= 1 && lo <= N - 2;
}
template <int N>
__device__ __forceinline__ int sc_k(int t) {
  const int hi = t / N, lo = t - hi * N;
  return (hi - 1) * (N - 2) + (lo - 1);
}

// Helmholtz of one element per slot.  The I stage, the pointwise geometric
// factors with the lambda mass term and the transposed I stage run as one
// loop over the point index i; PF register sets hold the factors of points
// i .. i+PF-1, so the loads of the next PF-1 points are in flight while point
// i is processed (PF = 1: none, fewest registers).  Local store or (ASM)
// atomic scatter-add into the global vector with the element's
// p_e . (H_e p_e).
// SC selects a pass of the statically condensed operator (assembled maps
// whose interior modes are Dirichlet entries, so their gathered values are
// 0 and their scatter is skipped; local inputs whose interior entries are
// 0): 1 stores the element's interior outputs into scb[k] and writes nothing
// else; 2 takes the interior inputs from scb[k], then scatters the boundary
// outputs and sums the energy over the free boundary modes only (ASM) or
// stores every output locally.  scb is the element's block of (N-2)^3
// interior values (global or LDS memory).
template <typename T, int N, int Q, int NT, bool ASM, int PF = 2, bool EOI = true, int SC = 0>
__device__ __forceinline__ void helm3_body(const Tab<T, N, Q>& tb, T* __restrict__ sm,
                                           double* red, int slot, int t, bool live, int64_t e,
                                           const DevArgs<T>& a, T* scb = nullptr) {
  constexpr int NN = N * N, N3 = N * N * N, Q3 = Q * Q * Q, QQ = Q * Q;
  const int64_t ee = live ? e : 0;
  const bool pq = live && t < NN;
  int32_t gidx[N];
  T xin[N];
  if (pq) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if constexpr (ASM) {
        const int32_t g = a.l2g[ee * N3 + r * NN + t];
        gidx[r] = g;
        xin[r] = a.in[l2g_dof(g)];
      } else {
        xin[r] = a.in[ee * N3 + r * NN + t];
      }
    }
    if constexpr (ASM) {
#pragma unroll
      for (int r = 0; r < N; ++r) xin[r] = l2g_value(gidx[r], xin[r]);
    }
    if constexpr (SC == 2) {
      static_assert(N >= 3, "condensed pass");
      constexpr int NI2 = (N - 2) * (N - 2);
      if (sc_inner<N>(t)) {
        const T* ti = scb + sc_k<N>(t);
#pragma unroll
        for (int r = 1; r < N - 1; ++r) xin[r] = ti[(r - 1) * NI2];
      }
    }
  }
  stage_k<T, N, Q, true>(tb, sm, t, live, xin);
  slot_sync<NT>();
  stage_j<T, N, Q, NT, true>(tb, sm, t, live);
  slot_sync<NT>();
  const bool jk = live && t < QQ;
  T sa[N], sb[N], sc[N];
  if constexpr (EOI) {
    constexpr int KE = EO<N>::KE, KO = EO<N>::KO;
    // accumulators of the transposed I contraction, in split form
    T sae[KE], sao[KO], sbe[KE], sbo[KO], sce[KE], sco[KO];
    zero(sae);
    zero(sao);
    zero(sbe);
    zero(sbo);
    zero(sce);
    zero(sco);
    if (jk) {
      T ae[KE], ao[KO], be[KE], bo[KO], ce[KE], co[KO];
      {
        T av[N], bv[N], cv[N];
        load_i<T, N, Q, true>(sm, t, av, bv, cv);
        eo_split<T, N>(av, ae, ao);
        eo_split<T, N>(bv, be, bo);
        eo_split<T, N>(cv, ce, co);
      }
      const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
      const T* fp = a.fac + ee * (int64_t)(kNF3 * Q3) + t;
      eo_helm_row<T, N, Q, PF>(
          tb, lam, ae, ao, be, bo, ce, co,
          [&](int i, T (&f)[kNF3]) {
#pragma unroll
            for (int c = 0; c < kNF3; ++c) f[c] = fp[c * Q3 + i * QQ];
          },
          sae, sao, sbe, sbo, sce, sco);
    }
    eo_join<T, N>(sae, sao, sa);
    eo_join<T, N>(sbe, sbo, sb);
    eo_join<T, N>(sce, sco, sc);
  } else {
#pragma unroll
    for (int p = 0; p < N; ++p) sa[p] = sb[p] = sc[p] = T(0);
    if (jk) {
      T av[N], bv[N], cv[N];
      load_i<T, N, Q, true>(sm, t, av, bv, cv);
      const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
      const T* fp = a.fac + ee * (int64_t)(kNF3 * Q3) + t;
      plain_helm_row<T, N, Q, PF>(
          tb, lam, av, bv, cv,
          [&](int i, T (&f)[kNF3]) {
#pragma unroll
            for (int c = 0; c < kNF3; ++c) f[c] = fp[c * Q3 + i * QQ];
          },
          sa, sb, sc);
    }
  }
  slot_sync<NT>();
  if (jk) store_i<T, N, Q, true>(sm, t, sa, sb, sc);
  slot_sync<NT>();
  stage_jt<T, N, Q, NT, true>(tb, sm, t, live);
  slot_sync<NT>();
  T yv[N];
  stage_kt<T, N, Q, true>(tb, sm, t, live, yv);
  if constexpr (SC == 1) {
    static_assert(N >= 3, "condensed pass");
    constexpr int NI2 = (N - 2) * (N - 2);
    if (pq && sc_inner<N>(t)) {
      T* to = scb + sc_k<N>(t);
#pragma unroll
      for (int r = 1; r < N - 1; ++r) to[(r - 1) * NI2] = yv[r];
    }
  } else if constexpr (ASM) {
    double dp = 0.0;
    if (pq) {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if (gidx[r] >= 0) atomic_add(a.out + l2g_dof(gidx[r]), l2g_sign(gidx[r], yv[r]));
        if (SC != 2 || gidx[r] >= 0) dp += (double)xin[r] * (double)yv[r];
      }
    }
    const double s = slot_sum<NT>(dp, red, slot, t);
    if (live && t == 0 && a.dots) add_dot(a.dots, a.dslot, e, s);
  } else {
    if (pq) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[ee * N3 + r * NN + t] = yv[r];
    }
  }
}

// Threads per slot: Q^2 rounded up to a divisor of 64 when that keeps a slot
// inside one wavefront (then no block barriers are needed), else Q^2.
template <int Q>
constexpr int slot_threads() {
  return Q * Q <= 1 ? 1 : Q * Q <= 4 ? 4 : Q * Q <= 16 ? 16 : Q * Q <= 64 ? 64 : Q * Q;
}

// NTX: threads per slot, 0 for slot_threads<Q>(); Q*Q packs slots without
// idle lanes at the price of block barriers (Q*Q does not divide 64).  EOI:
// the Helmholtz I stage in even-odd pairs (else point by point).
template <typename T, int N, int Q, int EPB, int OP, int PF = 2, int NTX = 0, bool EOI = true>
__global__ void __launch_bounds__(EPB * (NTX ? NTX : slot_threads<Q>()))
    k_op3(const Tab<T, N, Q> tb, const DevArgs<T> a) {
  constexpr int NN = N * N, N3 = N * N * N, Q3 = Q * Q * Q, QQ = Q * Q, S = Q * Q * N;
  constexpr int NT = NTX ? NTX : slot_threads<Q>();
  constexpr bool DER = (OP == OP_HELM || OP == OP_HELM_ASM || OP == OP_GRAD || OP == OP_RHS);
  constexpr int NTEN = DER ? 3 : 1;
  constexpr bool ASM = (OP == OP_HELM_ASM);
  // BwdTrans / IProduct stage whole point arrays (Q^3) for coalesced access
  constexpr int SLOT = (NTEN * S > Q3) ? NTEN * S : Q3;
  __shared__ T smem[EPB * SLOT];
  __shared__ double red[((ASM || OP == OP_GRAD) && NT != 64) ? EPB * NT : 1];

  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && seg_converged(a.elem_seg, a.seg_done, e)) live = false;
  const int64_t ee = live ? e : 0;
  T* sm = smem + slot * SLOT;
  const T* fe = a.fac + ee * (int64_t)(kNF3 * Q3) + t;

  if constexpr (OP == OP_BWD) {
    T xin[N];
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) xin[r] = a.in[ee * N3 + r * NN + t];
    }
    stage_k<T, N, Q, false>(tb, sm, t, live, xin);
    slot_sync<NT>();
    stage_j<T, N, Q, NT, false>(tb, sm, t, live);
    slot_sync<NT>();
    T ae[EO<N>::KE], ao[EO<N>::KO];
    if (live && t < QQ) {
      T av[N], bv[N], cv[N];
      load_i<T, N, Q, false>(sm, t, av, bv, cv);
      eo_split<T, N>(av, ae, ao);
    }
    slot_sync<NT>();
    if (live && t < QQ) {
#pragma unroll 2
      for (int h = 0; h < Q / 2; ++h) {
        T lo, hi;
        eo_val(tb, h, ae, ao, lo, hi);
        sm[t * Q + h] = lo;
        sm[t * Q + Q - 1 - h] = hi;
      }
      if constexpr (Q & 1) sm[t * Q + Q / 2] = eo_mid_val(tb, ae);
    }
    slot_sync<NT>();
    // the slot writes its Q^3 point values contiguously
    if (live) {
      T* o = a.out + ee * Q3;
      for (int c = t; c < Q3; c += NT) o[c] = sm[c];
    }
  } else if constexpr (OP == OP_IPROD) {
    if (live) {
      const T* f = a.in + ee * Q3;
      for (int c = t; c < Q3; c += NT) sm[c] = f[c];
    }
    slot_sync<NT>();
    T se[EO<N>::KE], so[EO<N>::KO];
    zero(se);
    zero(so);
    if (live && t < QQ) {
#pragma unroll 2
      for (int h = 0; h < Q / 2; ++h) {
        const T ml = fe[h * QQ] * sm[t * Q + h];
        const T mh = fe[(Q - 1 - h) * QQ] * sm[t * Q + Q - 1 - h];
        eo_acc(tb, h, ml + mh, ml - mh, se, so);
      }
      if constexpr (Q & 1) eo_acc_mid(tb, fe[(Q / 2) * QQ] * sm[t * Q + Q / 2], se);
    }
    T sa[N];
    eo_join<T, N>(se, so, sa);
    slot_sync<NT>();
    if (live && t < QQ) store_i<T, N, Q, false>(sm, t, sa, sa, sa);
    slot_sync<NT>();
    stage_jt<T, N, Q, NT, false>(tb, sm, t, live);
    slot_sync<NT>();
    T yv[N];
    stage_kt<T, N, Q, false>(tb, sm, t, live, yv);
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[ee * N3 + r * NN + t] = yv[r];
    }
  } else if constexpr (OP == OP_HELM || OP == OP_HELM_ASM) {
    helm3_body<T, N, Q, NT, ASM, PF, EOI>(tb, sm, red, slot, t, live, e, a);
  } else if constexpr (OP == OP_RHS) {
    const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
    constexpr int KE = EO<N>::KE, KO = EO<N>::KO;
    T sae[KE], sao[KO], sbe[KE], sbo[KO], sce[KE], sco[KO];
    zero(sae);
    zero(sao);
    zero(sbe);
    zero(sbo);
    zero(sce);
    zero(sco);
    if (live && t < QQ) {
      const T* uu = a.in + ee * Q3 + t * Q;
      const double* du = a.in2 + ee * 3 * Q3 + t * Q;
      // (m, g1, g2, g3) at point i
      auto point = [&](int i, T (&r)[4]) {
        const T* fp = fe + i * QQ;
        const T d1 = du[i], d2 = du[Q3 + i], d3 = du[2 * Q3 + i];
        r[0] = lam * fp[0] * uu[i];
        r[1] = fp[Q3] * d1 + fp[2 * Q3] * d2 + fp[3 * Q3] * d3;
        r[2] = fp[2 * Q3] * d1 + fp[4 * Q3] * d2 + fp[5 * Q3] * d3;
        r[3] = fp[3 * Q3] * d1 + fp[5 * Q3] * d2 + fp[6 * Q3] * d3;
      };
#pragma unroll 1
      for (int h = 0; h < Q / 2; ++h) {
        T rl[4], rh[4];
        point(h, rl);
        point(Q - 1 - h, rh);
        eo_acc(tb, h, rl[0] + rh[0], rl[0] - rh[0], sae, sao);
        eo_acc_d(tb, h, rl[1] + rh[1], rl[1] - rh[1], sae, sao);
        eo_acc(tb, h, rl[2] + rh[2], rl[2] - rh[2], sbe, sbo);
        eo_acc(tb, h, rl[3] + rh[3], rl[3] - rh[3], sce, sco);
      }
      if constexpr (Q & 1) {
        T r[4];
        point(Q / 2, r);
        eo_acc_mid(tb, r[0], sae);
        eo_acc_mid_d(tb, r[1], sao);
        eo_acc_mid(tb, r[2], sbe);
        eo_acc_mid(tb, r[3], sce);
      }
      T sa[N], sb[N], sc[N];
      eo_join<T, N>(sae, sao, sa);
      eo_join<T, N>(sbe, sbo, sb);
      eo_join<T, N>(sce, sco, sc);
      store_i<T, N, Q, true>(sm, t, sa, sb, sc);
    }
    slot_sync<NT>();
    stage_jt<T, N, Q, NT, true>(tb, sm, t, live);
    slot_sync<NT>();
    T yv[N];
    stage_kt<T, N, Q, true>(tb, sm, t, live, yv);
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[ee * N3 + r * NN + t] = yv[r];
    }
  } else if constexpr (OP == OP_GRAD) {
    // in = z_loc, in2 = u_loc; out = dkappa [E][Q^3] (may be null), out2 = dlambda [E]
    T zv[3][N], uv[3][N];
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const T* src = pass == 0 ? a.in : (const T*)a.in2;
      T xin[N];
      if (live && t < NN) {
#pragma unroll
        for (int r = 0; r < N; ++r) xin[r] = src[ee * N3 + r * NN + t];
      }
      if (pass == 1) slot_sync<NT>();
      stage_k<T, N, Q, true>(tb, sm, t, live, xin);
      slot_sync<NT>();
      stage_j<T, N, Q, NT, true>(tb, sm, t, live);
      slot_sync<NT>();
      if (live && t < QQ) {
        if (pass == 0)
          load_i<T, N, Q, true>(sm, t, zv[0], zv[1], zv[2]);
        else
          load_i<T, N, Q, true>(sm, t, uv[0], uv[1], uv[2]);
      }
    }
    double dl = 0.0;
    if (live && t < QQ) {
      constexpr int KE = EO<N>::KE, KO = EO<N>::KO;
      T ze[3][KE], zo[3][KO], ue[3][KE], uo[3][KO];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        eo_split<T, N>(zv[c], ze[c], zo[c]);
        eo_split<T, N>(uv[c], ue[c], uo[c]);
      }
      const double* kap = a.kappa ? a.kappa + ee * Q3 + t * Q : nullptr;
      // z, dz (reference gradient), u, du at point i -> dkappa, and the mass
      // term's share of dlambda
      auto point = [&](int i, T z, T z1, T z2, T z3, T u, T u1, T u2, T u3) {
        const T* fp = fe + i * QQ;
        const T ik = kap ? T(1) / (T)kap[i] : T(1);
        const T G11 = fp[Q3] * ik, G12 = fp[2 * Q3] * ik, G13 = fp[3 * Q3] * ik,
                G22 = fp[4 * Q3] * ik, G23 = fp[5 * Q3] * ik, G33 = fp[6 * Q3] * ik;
        const T q1 = G11 * u1 + G12 * u2 + G13 * u3;
        const T q2 = G12 * u1 + G22 * u2 + G23 * u3;
        const T q3 = G13 * u1 + G23 * u2 + G33 * u3;
        if (a.out) a.out[ee * Q3 + t * Q + i] = -(z1 * q1 + z2 * q2 + z3 * q3);
        dl += (double)(fp[0] * z * u);
      };
#pragma unroll 1
      for (int h = 0; h < Q / 2; ++h) {
        T zl[4], zh[4], ul[4], uh[4];
        eo_val(tb, h, ze[0], zo[0], zl[0], zh[0]);
        eo_der(tb, h, ze[0], zo[0], zl[1], zh[1]);
        eo_val(tb, h, ze[1], zo[1], zl[2], zh[2]);
        eo_val(tb, h, ze[2], zo[2], zl[3], zh[3]);
        eo_val(tb, h, ue[0], uo[0], ul[0], uh[0]);
        eo_der(tb, h, ue[0], uo[0], ul[1], uh[1]);
        eo_val(tb, h, ue[1], uo[1], ul[2], uh[2]);
        eo_val(tb, h, ue[2], uo[2], ul[3], uh[3]);
        point(h, zl[0], zl[1], zl[2], zl[3], ul[0], ul[1], ul[2], ul[3]);
        point(Q - 1 - h, zh[0], zh[1], zh[2], zh[3], uh[0], uh[1], uh[2], uh[3]);
      }
      if constexpr (Q & 1) {
        point(Q / 2, eo_mid_val(tb, ze[0]), eo_mid_der(tb, zo[0]), eo_mid_val(tb, ze[1]),
              eo_mid_val(tb, ze[2]), eo_mid_val(tb, ue[0]), eo_mid_der(tb, uo[0]),
              eo_mid_val(tb, ue[1]), eo_mid_val(tb, ue[2]));
      }
    }
    const double s = slot_sum<NT>(dl, red, slot, t);
    if (live && t == 0 && a.out2) a.out2[e] = -s;
  }
}

}  // namespace nk
