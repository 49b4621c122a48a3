// Sum-factorised elemental operators on tensor-product elements (device code).
//
// Section 3.3 of arXiv 1906.03489 evaluates an expansion at the quadrature
// points by contracting one direction at a time (the sum-factorisation
// display), across many elements of one collection concurrently ("SumFac").
// On CDNA4 one element is handled by one "slot" of Q*Q threads.  Each thread
// owns a pencil: a line of values along one direction, held in registers, so
// every contraction is a register-local product with a uniform 1-D matrix
// (read from the kernel arguments through the scalar cache).  Between the
// three directions the pencils are re-oriented through LDS.
//
// Forward (coefficients -> values and reference gradient at the points):
//   K: thread (p,q)  contracts r -> k with B and DB        (n^2 pencils)
//   J: thread (p,k)  contracts q -> j                      (n Q pencils)
//   I: thread (j,k)  contracts p -> i                      (Q^2 pencils)
// producing u, du/dxi_1, du/dxi_2, du/dxi_3 at points (i, j, k) in thread
// (j, k).  The backward (transpose) sweep runs I', J', K' in reverse and sums
// the four point fields into one set of coefficients:
//   y = (B (x) B (x) B)^T m + sum_a (D_a (B (x) B (x) B))^T g_a.
// Derivative factors are carried as separate tensors (t_B, t_D after K;
// s_BB, s_DB, s_BD after J) so that no collocation-derivative pass is needed.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "nk_internal.h"

namespace nk {

template <typename T, int N, int Q>
struct Tab {
  T B[Q * N];  // B[i*N + p] = phi_p(x_i)
  T D[Q * N];  // D[i*N + p] = phi_p'(x_i)
};

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

// ---------------------------------------------------------------- 3-D engine

// Forward sweep of one element.  `in` is the element's coefficient array (or
// the global vector when ASM, indexed through l2g_e).  Results for thread t
// = j + Q k: u[i], u1[i], u2[i], u3[i] at points (i, j, k).  Without DER only
// u is produced.  Must be called by every thread of the block.
template <typename T, int N, int Q, bool DER, bool ASM>
__device__ __forceinline__ void fwd3(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool live,
                                     const T* __restrict__ in, const int32_t* __restrict__ l2g_e,
                                     int32_t (&gidx)[N], T (&xin)[N], T (&u)[Q], T (&u1)[Q],
                                     T (&u2)[Q], T (&u3)[Q]) {
  constexpr int NN = N * N, S = Q * Q * N;
  // K: thread (p,q) = t < N^2 contracts r -> k
  if (live && t < NN) {
#pragma unroll
    for (int r = 0; r < N; ++r) {
      if constexpr (ASM) {
        const int32_t g = l2g_e[r * NN + t];
        gidx[r] = g;
        xin[r] = g >= 0 ? in[g] : T(0);
      } else {
        xin[r] = in[r * NN + t];
      }
    }
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T sb = 0, sd = 0;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        sb += tb.B[k * N + r] * xin[r];
        if constexpr (DER) sd += tb.D[k * N + r] * xin[r];
      }
      sm[k * NN + t] = sb;
      if constexpr (DER) sm[S + k * NN + t] = sd;
    }
  }
  __syncthreads();
  // J: thread (p,k) = t < N Q contracts q -> j
  T sBB[Q], sDB[Q], sBD[Q];
  const int pj = t % N, kj = t / N;
  if (live && t < N * Q) {
    T av[N], bv[N];
#pragma unroll
    for (int q = 0; q < N; ++q) {
      av[q] = sm[kj * NN + q * N + pj];
      if constexpr (DER) bv[q] = sm[S + kj * NN + q * N + pj];
    }
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        s0 += tb.B[j * N + q] * av[q];
        if constexpr (DER) {
          s1 += tb.D[j * N + q] * av[q];
          s2 += tb.B[j * N + q] * bv[q];
        }
      }
      sBB[j] = s0;
      if constexpr (DER) {
        sDB[j] = s1;
        sBD[j] = s2;
      }
    }
  }
  __syncthreads();
  if (live && t < N * Q) {
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      sm[(kj * Q + j) * N + pj] = sBB[j];
      if constexpr (DER) {
        sm[S + (kj * Q + j) * N + pj] = sDB[j];
        sm[2 * S + (kj * Q + j) * N + pj] = sBD[j];
      }
    }
  }
  __syncthreads();
  // I: thread (j,k) = t < Q^2 contracts p -> i
  if (live) {
    T av[N], bv[N], cv[N];
#pragma unroll
    for (int p = 0; p < N; ++p) {
      av[p] = sm[t * N + p];
      if constexpr (DER) {
        bv[p] = sm[S + t * N + p];
        cv[p] = sm[2 * S + t * N + p];
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        s0 += tb.B[i * N + p] * av[p];
        if constexpr (DER) {
          s1 += tb.D[i * N + p] * av[p];
          s2 += tb.B[i * N + p] * bv[p];
          s3 += tb.B[i * N + p] * cv[p];
        }
      }
      u[i] = s0;
      if constexpr (DER) {
        u1[i] = s1;
        u2[i] = s2;
        u3[i] = s3;
      }
    }
  }
}

// Backward (transpose) sweep: from m, g1, g2, g3 at points (i, j, k) of
// thread t = j + Q k to coefficients yv[r] of thread (p,q) = t < N^2.
// Without DER only m is used.  Must be called by every thread; the caller
// has synchronised so that sm may be overwritten.
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void bwd3(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool live,
                                     const T (&m)[Q], const T (&g1)[Q], const T (&g2)[Q],
                                     const T (&g3)[Q], T (&yv)[N]) {
  constexpr int NN = N * N, S = Q * Q * N;
  // I': thread (j,k) contracts i -> p
  if (live) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        s0 += tb.B[i * N + p] * m[i];
        if constexpr (DER) {
          s0 += tb.D[i * N + p] * g1[i];
          s1 += tb.B[i * N + p] * g2[i];
          s2 += tb.B[i * N + p] * g3[i];
        }
      }
      sm[t * N + p] = s0;
      if constexpr (DER) {
        sm[S + t * N + p] = s1;
        sm[2 * S + t * N + p] = s2;
      }
    }
  }
  __syncthreads();
  // J': thread (p,k) = t < N Q contracts j -> q
  const int pj = t % N, kj = t / N;
  T tB[N], tD[N];
  if (live && t < N * Q) {
    T av[Q], bv[Q], cv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      av[j] = sm[(kj * Q + j) * N + pj];
      if constexpr (DER) {
        bv[j] = sm[S + (kj * Q + j) * N + pj];
        cv[j] = sm[2 * S + (kj * Q + j) * N + pj];
      }
    }
#pragma unroll
    for (int q = 0; q < N; ++q) {
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        s0 += tb.B[j * N + q] * av[j];
        if constexpr (DER) {
          s0 += tb.D[j * N + q] * bv[j];
          s1 += tb.B[j * N + q] * cv[j];
        }
      }
      tB[q] = s0;
      if constexpr (DER) tD[q] = s1;
    }
  }
  __syncthreads();
  if (live && t < N * Q) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      sm[kj * NN + q * N + pj] = tB[q];
      if constexpr (DER) sm[S + kj * NN + q * N + pj] = tD[q];
    }
  }
  __syncthreads();
  // K': thread (p,q) = t < N^2 contracts k -> r
  if (live && t < NN) {
    T av[Q], bv[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      av[k] = sm[k * NN + t];
      if constexpr (DER) bv[k] = sm[S + k * NN + t];
    }
#pragma unroll
    for (int r = 0; r < N; ++r) {
      T s0 = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        s0 += tb.B[k * N + r] * av[k];
        if constexpr (DER) s0 += tb.D[k * N + r] * bv[k];
      }
      yv[r] = s0;
    }
  }
}

// Sum of v over the threads of a slot (NT threads), result valid in thread
// t == 0 of the slot.  `red` is a block-shared scratch of blockDim doubles.
template <int NT>
__device__ __forceinline__ double slot_sum(double v, double* red, int slot, int t) {
  __syncthreads();
  red[slot * NT + t] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0) {
    for (int i = 0; i < NT; ++i) s += red[slot * NT + i];
  }
  return s;
}

// Helmholtz of one element per slot: forward sweep, pointwise geometric
// factors and lambda mass term, backward sweep; local store or (ASM) atomic
// scatter-add into the global vector with the element's p_e . (H_e p_e).
template <typename T, int N, int Q, int NT, bool ASM>
__device__ __forceinline__ void helm3_body(const Tab<T, N, Q>& tb, T* __restrict__ sm,
                                           double* red, int slot, int t, bool live, int64_t e,
                                           const DevArgs<T>& a) {
  constexpr int NN = N * N, N3 = N * N * N, Q3 = Q * Q * Q, QQ = Q * Q;
  const int64_t ee = live ? e : 0;
  const T* fe = a.fac + ee * (int64_t)(kNF3 * Q3);
  int32_t gidx[N];
  T xin[N];
  T u[Q], u1[Q], u2[Q], u3[Q];
  const T* src = ASM ? a.in : a.in + ee * N3;
  fwd3<T, N, Q, true, ASM>(tb, sm, t, live, src, ASM ? a.l2g + ee * N3 : nullptr, gidx, xin, u,
                           u1, u2, u3);
  const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
  T m[Q], g1[Q], g2[Q], g3[Q], yv[N];
  if (live) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      const T* fp = fe + i * QQ + t;
      const T wj = fp[0], G11 = fp[Q3], G12 = fp[2 * Q3], G13 = fp[3 * Q3], G22 = fp[4 * Q3],
              G23 = fp[5 * Q3], G33 = fp[6 * Q3];
      m[i] = lam * wj * u[i];
      g1[i] = G11 * u1[i] + G12 * u2[i] + G13 * u3[i];
      g2[i] = G12 * u1[i] + G22 * u2[i] + G23 * u3[i];
      g3[i] = G13 * u1[i] + G23 * u2[i] + G33 * u3[i];
    }
  }
  __syncthreads();
  bwd3<T, N, Q, true>(tb, sm, t, live, m, g1, g2, g3, yv);
  if constexpr (ASM) {
    double dp = 0.0;
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if (gidx[r] >= 0) atomic_add(a.out + gidx[r], yv[r]);
        dp += (double)xin[r] * (double)yv[r];
      }
    }
    const double s = slot_sum<NT>(dp, red, slot, t);
    if (live && t == 0 && a.dots) a.dots[e] = s;
  } else {
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[e * N3 + r * NN + t] = yv[r];
    }
  }
}

template <typename T, int N, int Q, int EPB, int OP>
__global__ void __launch_bounds__(EPB * Q * Q)
    k_op3(const Tab<T, N, Q> tb, const DevArgs<T> a) {
  constexpr int NN = N * N, N3 = N * N * N, Q3 = Q * Q * Q, QQ = Q * Q, S = Q * Q * N;
  constexpr int NT = QQ;
  constexpr bool DER = (OP == OP_HELM || OP == OP_HELM_ASM || OP == OP_GRAD || OP == OP_RHS);
  constexpr int NTEN = DER ? 3 : 1;
  constexpr bool ASM = (OP == OP_HELM_ASM);
  __shared__ T smem[EPB * NTEN * S];
  __shared__ double red[(ASM || OP == OP_GRAD) ? EPB * NT : 1];

  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && a.elem_seg != nullptr) live = a.seg_done[a.elem_seg[e]] == 0;
  T* sm = smem + slot * NTEN * S;
  // factor f at point (i, t) of element e
  const T* fe = a.fac + (live ? e : 0) * (int64_t)(kNF3 * Q3);
  auto F = [&](int f, int i) -> T { return fe[(f * Q + i) * QQ + t]; };

  int32_t gidx[N];
  T xin[N];
  T u[Q], u1[Q], u2[Q], u3[Q];

  if constexpr (OP == OP_BWD) {
    fwd3<T, N, Q, false, false>(tb, sm, t, live, a.in + (live ? e : 0) * N3, nullptr, gidx, xin, u,
                                u1, u2, u3);
    if (live) {
      T* o = a.out + e * Q3 + t * Q;
#pragma unroll
      for (int i = 0; i < Q; ++i) o[i] = u[i];
    }
  } else if constexpr (OP == OP_IPROD) {
    T m[Q], yv[N];
    if (live) {
      const T* f = a.in + e * Q3 + t * Q;
#pragma unroll
      for (int i = 0; i < Q; ++i) m[i] = F(0, i) * f[i];
    }
    bwd3<T, N, Q, false>(tb, sm, t, live, m, m, m, m, yv);
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[e * N3 + r * NN + t] = yv[r];
    }
  } else if constexpr (OP == OP_HELM || OP == OP_HELM_ASM) {
    helm3_body<T, N, Q, NT, ASM>(tb, sm, red, slot, t, live, e, a);
  } else if constexpr (OP == OP_RHS) {
    const T lam = (T)(a.lam ? a.lam[live ? e : 0] : a.lam0);
    T m[Q], g1[Q], g2[Q], g3[Q], yv[N];
    if (live) {
      const T* uu = a.in + e * Q3 + t * Q;
      const double* du = a.in2 + e * 3 * Q3 + t * Q;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T d1 = du[i], d2 = du[Q3 + i], d3 = du[2 * Q3 + i];
        m[i] = lam * F(0, i) * uu[i];
        g1[i] = F(1, i) * d1 + F(2, i) * d2 + F(3, i) * d3;
        g2[i] = F(2, i) * d1 + F(4, i) * d2 + F(5, i) * d3;
        g3[i] = F(3, i) * d1 + F(5, i) * d2 + F(6, i) * d3;
      }
    }
    bwd3<T, N, Q, true>(tb, sm, t, live, m, g1, g2, g3, yv);
    if (live && t < NN) {
#pragma unroll
      for (int r = 0; r < N; ++r) a.out[e * N3 + r * NN + t] = yv[r];
    }
  } else if constexpr (OP == OP_GRAD) {
    // in = z_loc, in2 = u_loc; out = dkappa [E][Q^3] (may be null), out2 = dlambda [E]
    T z[Q], z1[Q], z2[Q], z3[Q];
    fwd3<T, N, Q, true, false>(tb, sm, t, live, a.in + (live ? e : 0) * N3, nullptr, gidx, xin, z,
                               z1, z2, z3);
    __syncthreads();
    fwd3<T, N, Q, true, false>(tb, sm, t, live, (const T*)a.in2 + (live ? e : 0) * N3, nullptr,
                               gidx, xin, u, u1, u2, u3);
    double dl = 0.0;
    if (live) {
      const double* kap = a.kappa ? a.kappa + e * Q3 + t * Q : nullptr;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T wj = F(0, i);
        const T ik = kap ? T(1) / (T)kap[i] : T(1);
        const T G11 = F(1, i) * ik, G12 = F(2, i) * ik, G13 = F(3, i) * ik, G22 = F(4, i) * ik,
                G23 = F(5, i) * ik, G33 = F(6, i) * ik;
        const T q1 = G11 * u1[i] + G12 * u2[i] + G13 * u3[i];
        const T q2 = G12 * u1[i] + G22 * u2[i] + G23 * u3[i];
        const T q3 = G13 * u1[i] + G23 * u2[i] + G33 * u3[i];
        if (a.out) a.out[e * Q3 + t * Q + i] = -(z1[i] * q1 + z2[i] * q2 + z3[i] * q3);
        dl += (double)(wj * z[i] * u[i]);
      }
    }
    const double s = slot_sum<NT>(dl, red, slot, t);
    if (live && t == 0 && a.out2) a.out2[e] = -s;
  }
}

}  // namespace nk
