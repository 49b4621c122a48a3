// 2-D (quadrilateral) sum-factorised operators.  One slot of Q threads per
// element: thread p (< n) contracts q -> j for the pencil of mode p; thread j
// contracts p -> i.  Factors per point: w detJ, then w detJ kappa G_11, G_12,
// G_22, stored [e][f][i][j] so thread j reads them coalesced.
#include "engine.h"
#include "tables.h"
#include "tiles.h"

namespace nk {

template <typename T, int N, int Q, int EPB, int OP>
__global__ void __launch_bounds__(EPB * Q)
    k_op2(const Tab<T, N, Q> tb, const DevArgs<T> a) {
  constexpr int N2 = N * N, Q2 = Q * Q, S = Q * N, NT = Q;
  constexpr bool DER = (OP == OP_HELM || OP == OP_HELM_ASM || OP == OP_RHS || OP == OP_GRAD);
  constexpr bool ASM = (OP == OP_HELM_ASM);
  constexpr int NTEN = DER ? 2 : 1;
  __shared__ T smem[EPB * NTEN * S];
  __shared__ double red[(ASM || OP == OP_GRAD) ? EPB * NT : 1];
  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && seg_converged(a.elem_seg, a.seg_done, e)) live = false;
  T* sm = smem + slot * NTEN * S;
  const int64_t ee = live ? e : 0;
  const T* fe = a.fac + ee * (int64_t)(kNF2 * Q2);
  auto F = [&](int f, int i) -> T { return fe[(f * Q + i) * Q + t]; };

  // forward sweep of coefficient array `in` (element base, or global + l2g)
  auto fwd = [&](const T* in, const int32_t* l2g_e, int32_t(&gidx)[N], T(&xin)[N], T(&u)[Q],
                 T(&u1)[Q], T(&u2)[Q]) {
    if (live && t < N) {
#pragma unroll
      for (int q = 0; q < N; ++q) {
        if constexpr (ASM) {
          const int32_t g = l2g_e[q * N + t];
          gidx[q] = g;
          xin[q] = in[l2g_dof(g)];
        } else {
          xin[q] = in[q * N + t];
        }
      }
      if constexpr (ASM) {
#pragma unroll
        for (int q = 0; q < N; ++q) xin[q] = l2g_value(gidx[q], xin[q]);
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        T sb = 0, sd = 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          sb += tb.B[j * N + q] * xin[q];
          if constexpr (DER) sd += tb.D[j * N + q] * xin[q];
        }
        sm[j * N + t] = sb;
        if constexpr (DER) sm[S + j * N + t] = sd;
      }
    }
    __syncthreads();
    if (live) {
      T av[N], bv[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        av[p] = sm[t * N + p];
        if constexpr (DER) bv[p] = sm[S + t * N + p];
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        T s0 = 0, s1 = 0, s2 = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          s0 += tb.B[i * N + p] * av[p];
          if constexpr (DER) {
            s1 += tb.D[i * N + p] * av[p];
            s2 += tb.B[i * N + p] * bv[p];
          }
        }
        u[i] = s0;
        if constexpr (DER) {
          u1[i] = s1;
          u2[i] = s2;
        }
      }
    }
  };
  // backward sweep from m, g1, g2 at points (i, t) to coefficients yv[q] of thread p = t < N
  auto bwd = [&](const T(&m)[Q], const T(&g1)[Q], const T(&g2)[Q], T(&yv)[N]) {
    if (live) {
#pragma unroll
      for (int p = 0; p < N; ++p) {
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          s0 += tb.B[i * N + p] * m[i];
          if constexpr (DER) {
            s0 += tb.D[i * N + p] * g1[i];
            s1 += tb.B[i * N + p] * g2[i];
          }
        }
        sm[t * N + p] = s0;
        if constexpr (DER) sm[S + t * N + p] = s1;
      }
    }
    __syncthreads();
    if (live && t < N) {
      T av[Q], bv[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        av[j] = sm[j * N + t];
        if constexpr (DER) bv[j] = sm[S + j * N + t];
      }
#pragma unroll
      for (int q = 0; q < N; ++q) {
        T s0 = 0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          s0 += tb.B[j * N + q] * av[j];
          if constexpr (DER) s0 += tb.D[j * N + q] * bv[j];
        }
        yv[q] = s0;
      }
    }
  };

  int32_t gidx[N];
  T xin[N];
  T u[Q], u1[Q], u2[Q], yv[N];
  if constexpr (OP == OP_BWD) {
    fwd(a.in + ee * N2, nullptr, gidx, xin, u, u1, u2);
    if (live) {
#pragma unroll
      for (int i = 0; i < Q; ++i) a.out[e * Q2 + t * Q + i] = u[i];
    }
  } else if constexpr (OP == OP_IPROD) {
    T m[Q];
    if (live) {
#pragma unroll
      for (int i = 0; i < Q; ++i) m[i] = F(0, i) * a.in[e * Q2 + t * Q + i];
    }
    bwd(m, m, m, yv);
    if (live && t < N) {
#pragma unroll
      for (int q = 0; q < N; ++q) a.out[e * N2 + q * N + t] = yv[q];
    }
  } else if constexpr (OP == OP_HELM || OP == OP_HELM_ASM) {
    fwd(ASM ? a.in : a.in + ee * N2, ASM ? a.l2g + ee * N2 : nullptr, gidx, xin, u, u1, u2);
    const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
    T m[Q], g1[Q], g2[Q];
    if (live) {
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        m[i] = lam * F(0, i) * u[i];
        g1[i] = F(1, i) * u1[i] + F(2, i) * u2[i];
        g2[i] = F(2, i) * u1[i] + F(3, i) * u2[i];
      }
    }
    __syncthreads();
    bwd(m, g1, g2, yv);
    if constexpr (ASM) {
      double dp = 0.0;
      if (live && t < N) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
          if (gidx[q] >= 0) atomic_add(a.out + l2g_dof(gidx[q]), l2g_sign(gidx[q], yv[q]));
          dp += (double)xin[q] * (double)yv[q];
        }
      }
      const double s = slot_sum<NT>(dp, red, slot, t);
      if (live && t == 0 && a.dots) add_dot(a.dots, a.dslot, e, s);
    } else {
      if (live && t < N) {
#pragma unroll
        for (int q = 0; q < N; ++q) a.out[e * N2 + q * N + t] = yv[q];
      }
    }
  } else if constexpr (OP == OP_RHS) {
    const T lam = (T)(a.lam ? a.lam[ee] : a.lam0);
    T m[Q], g1[Q], g2[Q];
    if (live) {
      const T* uu = a.in + e * Q2 + t * Q;
      const double* du = a.in2 + e * 2 * Q2 + t * Q;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T d1 = du[i], d2 = du[Q2 + i];
        m[i] = lam * F(0, i) * uu[i];
        g1[i] = F(1, i) * d1 + F(2, i) * d2;
        g2[i] = F(2, i) * d1 + F(3, i) * d2;
      }
    }
    bwd(m, g1, g2, yv);
    if (live && t < N) {
#pragma unroll
      for (int q = 0; q < N; ++q) a.out[e * N2 + q * N + t] = yv[q];
    }
  } else if constexpr (OP == OP_GRAD) {
    T z[Q], z1[Q], z2[Q];
    fwd(a.in + ee * N2, nullptr, gidx, xin, z, z1, z2);
    __syncthreads();
    fwd((const T*)a.in2 + ee * N2, nullptr, gidx, xin, u, u1, u2);
    double dl = 0.0;
    if (live) {
      const double* kap = a.kappa ? a.kappa + e * Q2 + t * Q : nullptr;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const T ik = kap ? T(1) / (T)kap[i] : T(1);
        const T q1 = (F(1, i) * u1[i] + F(2, i) * u2[i]) * ik;
        const T q2 = (F(2, i) * u1[i] + F(3, i) * u2[i]) * ik;
        if (a.out) a.out[e * Q2 + t * Q + i] = -(z1[i] * q1 + z2[i] * q2);
        dl += (double)(F(0, i) * z[i] * u[i]);
      }
    }
    const double s = slot_sum<NT>(dl, red, slot, t);
    if (live && t == 0 && a.out2) a.out2[e] = -s;
  }
}

template <typename T, int P, int EPB, int OP>
static hipError_t run2(const OpArgs& a) {
  constexpr int N = P + 1, Q = P + 2;
  const Tab<T, N, Q>& tb = host_tab<T, N, Q>();
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_op2<T, N, Q, EPB, OP>), dim3((unsigned)nblk), dim3(EPB * Q), 0, a.stream,
                     tb, dev_args<T>(a));
  return hipGetLastError();
}

template <typename T, int P, int OP>
static hipError_t run2_tiled(const OpArgs& a) {
  constexpr int E0 = kTileEPB2[P][0], E1 = kTileEPB2[P][1];
  if (a.tile == 1 && E1 > 0) return run2<T, P, (E1 > 0 ? E1 : 1), OP>(a);
  return run2<T, P, E0, OP>(a);
}

template <int P>
static hipError_t run2_p(nk_dtype t, const OpArgs& a) {
  if (t == NK_F64) {
    switch (a.op) {
      case OP_BWD: return run2_tiled<double, P, OP_BWD>(a);
      case OP_IPROD: return run2_tiled<double, P, OP_IPROD>(a);
      case OP_HELM: return run2_tiled<double, P, OP_HELM>(a);
      case OP_HELM_ASM: return run2_tiled<double, P, OP_HELM_ASM>(a);
      case OP_RHS: return run2<double, P, kTileEPB2[P][0], OP_RHS>(a);
      case OP_GRAD: return run2<double, P, kTileEPB2[P][0], OP_GRAD>(a);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.op) {
    case OP_BWD: return run2_tiled<float, P, OP_BWD>(a);
    case OP_IPROD: return run2_tiled<float, P, OP_IPROD>(a);
    case OP_HELM: return run2_tiled<float, P, OP_HELM>(a);
    case OP_HELM_ASM: return run2_tiled<float, P, OP_HELM_ASM>(a);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_op2(nk_dtype t, const OpArgs& a) {
  switch (a.P) {
    case 1: return run2_p<1>(t, a);
    case 2: return run2_p<2>(t, a);
    case 3: return run2_p<3>(t, a);
    case 4: return run2_p<4>(t, a);
    case 5: return run2_p<5>(t, a);
    case 6: return run2_p<6>(t, a);
    case 7: return run2_p<7>(t, a);
    case 8: return run2_p<8>(t, a);
    case 9: return run2_p<9>(t, a);
    case 10: return run2_p<10>(t, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace nk
