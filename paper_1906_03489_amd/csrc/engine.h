// Sum-factorised elemental operators on tensor-product elements (device code).
//
// Section 3.3 of arXiv 1906.03489 evaluates an expansion at the quadrature
// points by contracting one direction at a time (the sum-factorisation
// display), across many elements of one collection concurrently ("SumFac").
//
// CDNA4 mapping.  One element is handled by one "slot" of NT >= Q*Q threads.
// Each thread owns a pencil (a line of values along one direction) in
// registers, so every contraction is a register-local product with a 1-D
// matrix that is uniform across the wavefront.  The stages loop over the
// point index (k, j or i) without unrolling and unroll the mode index, so each
// iteration needs exactly one row of B and of DB, which the scalar unit loads
// from the kernel arguments; the FP64/FP32 FMAs take it as their scalar
// operand.  Between directions the pencils are re-oriented through LDS.
//
// Forward (coefficients -> values and reference gradient at the points):
//   K: thread (p,q)  r -> k with B and DB           -> t_B, t_D   [k][q][p]
//   J: thread (p,k)  q -> j                         -> s_BB, s_DB, s_BD [k][j][p]
//   I: thread (j,k)  p -> i, fused with the pointwise factors and with the
//      transposed I stage, one point i per loop iteration
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

// K: thread t = p + N q (< N^2) holds xin[r]; writes t_B (and t_D) [k][q][p].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void stage_k(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool act,
                                        const T (&xin)[N]) {
  constexpr int NN = N * N, S = Q * Q * N;
  if (act && t < NN) {
#pragma unroll 2
    for (int k = 0; k < Q; ++k) {
      const T* Bk = tb.B + k * N;
      const T* Dk = tb.D + k * N;
      T sb = 0, sd = 0;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        sb += Bk[r] * xin[r];
        if constexpr (DER) sd += Dk[r] * xin[r];
      }
      sm[k * NN + t] = sb;
      if constexpr (DER) sm[S + k * NN + t] = sd;
    }
  }
}

// J: thread (p,k) = t < N Q reads t_B, t_D; writes s_BB, s_DB, s_BD [k][j][p].
template <typename T, int N, int Q, int NT, bool DER>
__device__ __forceinline__ void stage_j(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t, bool act) {
  constexpr int NN = N * N, S = Q * Q * N;
  const int pj = t % N, kj = t / N;
  const bool me = act && t < N * Q;
  T av[N], bv[N];
  if (me) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      av[q] = sm[kj * NN + q * N + pj];
      if constexpr (DER) bv[q] = sm[S + kj * NN + q * N + pj];
    }
  }
  slot_sync<NT>();
  if (me) {
#pragma unroll 2
    for (int j = 0; j < Q; ++j) {
      const T* Bj = tb.B + j * N;
      const T* Dj = tb.D + j * N;
      T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        s0 += Bj[q] * av[q];
        if constexpr (DER) {
          s1 += Dj[q] * av[q];
          s2 += Bj[q] * bv[q];
        }
      }
      const int o = (kj * Q + j) * N + pj;
      sm[o] = s0;
      if constexpr (DER) {
        sm[S + o] = s1;
        sm[2 * S + o] = s2;
      }
    }
  }
}

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

// J': thread (p,k) = t < N Q sums over j; writes t'_B, t'_D [k][q][p].
template <typename T, int N, int Q, int NT, bool DER>
__device__ __forceinline__ void stage_jt(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t,
                                         bool act) {
  constexpr int NN = N * N, S = Q * Q * N;
  const int pj = t % N, kj = t / N;
  const bool me = act && t < N * Q;
  T tB[N], tD[N];
#pragma unroll
  for (int q = 0; q < N; ++q) tB[q] = tD[q] = T(0);
  if (me) {
#pragma unroll 2
    for (int j = 0; j < Q; ++j) {
      const int o = (kj * Q + j) * N + pj;
      const T a = sm[o];
      T b = 0, c = 0;
      if constexpr (DER) {
        b = sm[S + o];
        c = sm[2 * S + o];
      }
      const T* Bj = tb.B + j * N;
      const T* Dj = tb.D + j * N;
#pragma unroll
      for (int q = 0; q < N; ++q) {
        tB[q] += Bj[q] * a;
        if constexpr (DER) {
          tB[q] += Dj[q] * b;
          tD[q] += Bj[q] * c;
        }
      }
    }
  }
  slot_sync<NT>();
  if (me) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
      sm[kj * NN + q * N + pj] = tB[q];
      if constexpr (DER) sm[S + kj * NN + q * N + pj] = tD[q];
    }
  }
}

// K': thread (p,q) = t < N^2 sums over k into y[r].
template <typename T, int N, int Q, bool DER>
__device__ __forceinline__ void stage_kt(const Tab<T, N, Q>& tb, const T* __restrict__ sm, int t,
                                         bool act, T (&yv)[N]) {
  constexpr int NN = N * N, S = Q * Q * N;
#pragma unroll
  for (int r = 0; r < N; ++r) yv[r] = T(0);
  if (act && t < NN) {
#pragma unroll 2
    for (int k = 0; k < Q; ++k) {
      const T a = sm[k * NN + t];
      const T b = DER ? sm[S + k * NN + t] : T(0);
      const T* Bk = tb.B + k * N;
      const T* Dk = tb.D + k * N;
#pragma unroll
      for (int r = 0; r < N; ++r) {
        yv[r] += Bk[r] * a;
        if constexpr (DER) yv[r] += Dk[r] * b;
      }
    }
  }
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

// Helmholtz of one element per slot.  The I stage, the pointwise geometric
// factors with the lambda mass term and the transposed I stage run as one
// loop over the point index i; PF register sets hold the factors of points
// i .. i+PF-1, so the loads of the next PF-1 points are in flight while point
// i is processed (PF = 1: none, fewest registers).  Local store or (ASM)
// atomic scatter-add into the global vector with the element's
// p_e . (H_e p_e).
template <typename T, int N, int Q, int NT, bool ASM, int PF = 2>
__device__ __forceinline__ void helm3_body(const Tab<T, N, Q>& tb, T* __restrict__ sm,
                                           double* red, int slot, int t, bool live, int64_t e,
                                           const DevArgs<T>& a) {
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
  }
  stage_k<T, N, Q, true>(tb, sm, t, live, xin);
  slot_sync<NT>();
  stage_j<T, N, Q, NT, true>(tb, sm, t, live);
  slot_sync<NT>();
  const bool jk = live && t < QQ;
  T av[N], bv[N], cv[N], sa[N], sb[N], sc[N];
#pragma unroll
  for (int p = 0; p < N; ++p) sa[p] = sb[p] = sc[p] = T(0);
  if (jk) {
    load_i<T, N, Q, true>(sm, t, av, bv, cv);
    const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
    const T* fp = a.fac + ee * (int64_t)(kNF3 * Q3) + t;
    // one point: forward I contraction, factors, transposed I contraction
    auto point = [&](int i, const T (&f)[kNF3]) {
      const T* Bi = tb.B + i * N;
      const T* Di = tb.D + i * N;
      T u = 0, u1 = 0, u2 = 0, u3 = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        u += Bi[p] * av[p];
        u1 += Di[p] * av[p];
        u2 += Bi[p] * bv[p];
        u3 += Bi[p] * cv[p];
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
    auto load = [&](int i, T (&f)[kNF3]) {
#pragma unroll
      for (int c = 0; c < kNF3; ++c) f[c] = fp[c * Q3 + i * QQ];
    };
    if constexpr (PF == 1) {
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        T f[kNF3];
        load(i, f);
        point(i, f);
      }
    } else {
      // set s holds point i+s; before point i+s is computed, the loads of
      // point i+s+PF-1 go into the set that point i+s-1 has just released.
      // Loads are unconditional (clamped index) so that the waits for them
      // can be placed right before their first use.
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
  }
  slot_sync<NT>();
  if (jk) store_i<T, N, Q, true>(sm, t, sa, sb, sc);
  slot_sync<NT>();
  stage_jt<T, N, Q, NT, true>(tb, sm, t, live);
  slot_sync<NT>();
  T yv[N];
  stage_kt<T, N, Q, true>(tb, sm, t, live, yv);
  if constexpr (ASM) {
    double dp = 0.0;
    if (pq) {
#pragma unroll
      for (int r = 0; r < N; ++r) {
        if (gidx[r] >= 0) atomic_add(a.out + l2g_dof(gidx[r]), l2g_sign(gidx[r], yv[r]));
        dp += (double)xin[r] * (double)yv[r];
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
// idle lanes at the price of block barriers (Q*Q does not divide 64).
template <typename T, int N, int Q, int EPB, int OP, int PF = 2, int NTX = 0>
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
    T av[N], bv[N], cv[N];
    if (live && t < QQ) load_i<T, N, Q, false>(sm, t, av, bv, cv);
    slot_sync<NT>();
    if (live && t < QQ) {
#pragma unroll 2
      for (int i = 0; i < Q; ++i) {
        const T* Bi = tb.B + i * N;
        T u = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) u += Bi[p] * av[p];
        sm[t * Q + i] = u;
      }
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
    T sa[N];
#pragma unroll
    for (int p = 0; p < N; ++p) sa[p] = T(0);
    if (live && t < QQ) {
#pragma unroll 2
      for (int i = 0; i < Q; ++i) {
        const T m = fe[i * QQ] * sm[t * Q + i];
        const T* Bi = tb.B + i * N;
#pragma unroll
        for (int p = 0; p < N; ++p) sa[p] += Bi[p] * m;
      }
    }
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
    helm3_body<T, N, Q, NT, ASM, PF>(tb, sm, red, slot, t, live, e, a);
  } else if constexpr (OP == OP_RHS) {
    const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
    T sa[N], sb[N], sc[N];
#pragma unroll
    for (int p = 0; p < N; ++p) sa[p] = sb[p] = sc[p] = T(0);
    if (live && t < QQ) {
      const T* uu = a.in + ee * Q3 + t * Q;
      const double* du = a.in2 + ee * 3 * Q3 + t * Q;
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        const T* fp = fe + i * QQ;
        const T d1 = du[i], d2 = du[Q3 + i], d3 = du[2 * Q3 + i];
        const T m = lam * fp[0] * uu[i];
        const T g1 = fp[Q3] * d1 + fp[2 * Q3] * d2 + fp[3 * Q3] * d3;
        const T g2 = fp[2 * Q3] * d1 + fp[4 * Q3] * d2 + fp[5 * Q3] * d3;
        const T g3 = fp[3 * Q3] * d1 + fp[5 * Q3] * d2 + fp[6 * Q3] * d3;
        const T* Bi = tb.B + i * N;
        const T* Di = tb.D + i * N;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          sa[p] += Bi[p] * m + Di[p] * g1;
          sb[p] += Bi[p] * g2;
          sc[p] += Bi[p] * g3;
        }
      }
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
      const double* kap = a.kappa ? a.kappa + ee * Q3 + t * Q : nullptr;
#pragma unroll 1
      for (int i = 0; i < Q; ++i) {
        const T* Bi = tb.B + i * N;
        const T* Di = tb.D + i * N;
        T z = 0, z1 = 0, z2 = 0, z3 = 0, u = 0, u1 = 0, u2 = 0, u3 = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          z += Bi[p] * zv[0][p];
          z1 += Di[p] * zv[0][p];
          z2 += Bi[p] * zv[1][p];
          z3 += Bi[p] * zv[2][p];
          u += Bi[p] * uv[0][p];
          u1 += Di[p] * uv[0][p];
          u2 += Bi[p] * uv[1][p];
          u3 += Bi[p] * uv[2][p];
        }
        const T* fp = fe + i * QQ;
        const T ik = kap ? T(1) / (T)kap[i] : T(1);
        const T G11 = fp[Q3] * ik, G12 = fp[2 * Q3] * ik, G13 = fp[3 * Q3] * ik,
                G22 = fp[4 * Q3] * ik, G23 = fp[5 * Q3] * ik, G33 = fp[6 * Q3] * ik;
        const T q1 = G11 * u1 + G12 * u2 + G13 * u3;
        const T q2 = G12 * u1 + G22 * u2 + G23 * u3;
        const T q3 = G13 * u1 + G23 * u2 + G33 * u3;
        if (a.out) a.out[ee * Q3 + t * Q + i] = -(z1 * q1 + z2 * q2 + z3 * q3);
        dl += (double)(fp[0] * z * u);
      }
    }
    const double s = slot_sum<NT>(dl, red, slot, t);
    if (live && t == 0 && a.out2) a.out2[e] = -s;
  }
}

}  // namespace nk
