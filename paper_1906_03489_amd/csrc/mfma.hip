// Helmholtz operator with the sum-factorisation contractions on the matrix
// cores (v_mfma_*_16x16x4), for orders with Q <= 8.
//
// One element per wavefront.  Every contraction of section 3.3's
// sum-factorisation is a small GEMM  out[row][col] = sum_kappa A[row][kappa] X[kappa][col]:
// the columns are the pencils of the stage (up to 64 = 4 column tiles of
// 16), kappa runs over the contracted index (padded to multiples of 4) and
// the 16 rows hold the output index of one or two result tensors (e.g. the
// B and DB contractions of the same data).  A comes from the 1-D tables and
// is the same for every element: the host builds, for every stage, chain
// and k-step, the value each lane must feed (fragments), so the kernel only
// loads them.  X comes from global memory (first stage), from LDS (the
// re-oriented output of the previous stage) or directly from registers
// (the pointwise results, whose lane placement already matches).
//
// MFMA lane layout (gfx950, 16x16x4): lane l feeds A[l%16][l/16] and
// B[l/16][l%16]; it receives D rows R(g,v) of column l%16 for items v=0..3
// with g = l/16: FP32 R = 4g+v, FP64 R = g+4v.  The kernel names results by
// (g, v); the host maps them to rows when it builds the fragments.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "tables.h"
#include "tiles.h"

namespace nk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct V4;
template <>
struct V4<double> {
  typedef d4 type;
};
template <>
struct V4<float> {
  typedef f4 type;
};

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Fragment slots (k-steps) per stage and chain, in buffer order.
enum : int {
  FK = 0,          // K: 2 k-steps (r)
  FJA = 2,         // J chain a (t_B -> s_BB, s_DB): 2
  FJB = 4,         // J chain b (t_D -> s_BD): 2
  FIA = 6,         // I chain a (s_BB -> u, u1): 2
  FIB = 8,         // I chain b ([s_DB; s_BD] -> u2, u3): 4
  FPA = 12,        // I' chain a (m, g1, g2 -> s'_BB, s'_DB): 6
  FPB = 18,        // I' chain b (g3 -> s'_BD): 2
  FJT = 20,        // J' (s'_BB, s'_DB, s'_BD -> t'_B, t'_D): 6
  FKT = 26,        // K' (t'_B, t'_D -> y): 4
  FNUM = 30
};

// --------------------------------------------------------------- host side

// A[rho][kappa] for one k-step of one chain: out(g, v) and in(kappa) give the
// semantic of the row and of the contracted index; coef() combines them.
template <typename T>
static void build_fragments(int P, std::vector<T>& frag) {
  const int N = P + 1, Q = P + 2;
  std::vector<double> x(Q), w(Q), B(Q * N), D(Q * N);
  gll_points(Q, x.data(), w.data());
  modified_basis(P, Q, x.data(), B.data(), D.data());
  auto b = [&](int i, int p) { return (i < Q && p < N) ? B[i * N + p] : 0.0; };
  auto d = [&](int i, int p) { return (i < Q && p < N) ? D[i * N + p] : 0.0; };
  const bool f64 = sizeof(T) == 8;
  frag.assign(FNUM * 64, T(0));
  // rho -> (g, v)
  auto gv = [&](int rho, int& g, int& v) {
    if (f64) {
      g = rho % 4;
      v = rho / 4;
    } else {
      g = rho / 4;
      v = rho % 4;
    }
  };
  for (int l = 0; l < 64; ++l) {
    const int rho = l % 16, kk = l / 16;
    int g, v;
    gv(rho, g, v);
    const int lo = g < 2, o4 = 4 * (g % 2) + v;  // output index 0..7 within a tensor
    // K: rows (g<2: t_B[k=o4], else t_D[k=o4]); kappa = r = 4s + kk
    for (int s = 0; s < 2; ++s) {
      const int r = 4 * s + kk;
      frag[(FK + s) * 64 + l] = (T)(lo ? b(o4, r) : d(o4, r));
    }
    // J a: rows (s_BB[j=o4] | s_DB[j=o4]), data t_B[q = 4s+kk]
    // J b: rows (s_BD[j=o4] | 0), data t_D[q]
    for (int s = 0; s < 2; ++s) {
      const int q = 4 * s + kk;
      frag[(FJA + s) * 64 + l] = (T)(lo ? b(o4, q) : d(o4, q));
      frag[(FJB + s) * 64 + l] = (T)(lo ? b(o4, q) : 0.0);
    }
    // I a: item v: even -> u[i], odd -> u1[i], i = 2g + v/2; data s_BB[p = 4s+kk]
    // I b: even -> u2[i] from s_DB (s = 0,1), odd -> u3[i] from s_BD (s = 2,3)
    {
      const int i = 2 * g + v / 2;
      for (int s = 0; s < 2; ++s) {
        const int p = 4 * s + kk;
        frag[(FIA + s) * 64 + l] = (T)((v % 2 == 0) ? b(i, p) : d(i, p));
      }
      for (int s = 0; s < 4; ++s) {
        const int p = 4 * (s % 2) + kk;
        const bool from_sdb = s < 2;
        frag[(FIB + s) * 64 + l] = (T)(((v % 2 == 0) == from_sdb) ? b(i, p) : 0.0);
      }
    }
    // I': k-step s feeds quantity s/2 (m, g1, g2, g3) at point i = 2*kk + s%2.
    // a: rows (s'_BB[p=o4] | s'_DB[p=o4]); b: rows (s'_BD[p=o4] | 0)
    for (int s = 0; s < 6; ++s) {
      const int qty = s / 2, i = 2 * kk + s % 2;
      double c = 0.0;
      if (lo) c = qty == 0 ? b(i, o4) : qty == 1 ? d(i, o4) : 0.0;
      else c = qty == 2 ? b(i, o4) : 0.0;
      frag[(FPA + s) * 64 + l] = (T)c;
    }
    for (int s = 0; s < 2; ++s) {
      const int i = 2 * kk + s;
      frag[(FPB + s) * 64 + l] = (T)(lo ? b(i, o4) : 0.0);
    }
    // J': k-step s feeds tensor s/2 (s'_BB, s'_DB, s'_BD) at j = 4(s%2) + kk;
    // rows (t'_B[q=o4] | t'_D[q=o4])
    for (int s = 0; s < 6; ++s) {
      const int t = s / 2, j = 4 * (s % 2) + kk;
      double c = 0.0;
      if (lo) c = t == 0 ? b(j, o4) : t == 1 ? d(j, o4) : 0.0;
      else c = t == 2 ? b(j, o4) : 0.0;
      frag[(FJT + s) * 64 + l] = (T)c;
    }
    // K': k-step s feeds tensor s/2 (t'_B, t'_D) at k = 4(s%2) + kk; rows (y[r=o4] | 0)
    for (int s = 0; s < 4; ++s) {
      const int t = s / 2, k = 4 * (s % 2) + kk;
      frag[(FKT + s) * 64 + l] = (T)(lo ? (t == 0 ? b(k, o4) : d(k, o4)) : 0.0);
    }
  }
}

// Device copy of the fragments of order P, built once per (device, P, T).
template <typename T>
static const T* device_fragments(int P) {
  static std::mutex mu;
  static std::unordered_map<long, T*> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const long key = dev * 64L + P;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  std::vector<T> h;
  build_fragments<T>(P, h);
  T* d = nullptr;
  if (hipMalloc((void**)&d, h.size() * sizeof(T)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  cache[key] = d;
  return d;
}

// ------------------------------------------------------------- device side

template <typename T, int N, int Q, int EPB, bool ASM>
__global__ void __launch_bounds__(EPB * 64)
    k_helm_mfma(const T* __restrict__ frag, const DevArgs<T> a) {
  static_assert(Q <= 8, "one 16-row block per stage needs Q <= 8");
  typedef typename V4<T>::type vec;
  constexpr int NN = N * N, N3 = N * N * N, Q3 = Q * Q * Q, QQ = Q * Q, S = Q * Q * N;
  __shared__ T smem[EPB * 3 * S];
  const int slot = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int g = l >> 4, cl = l & 15;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  bool live = e < a.nelem;
  if (live && seg_converged(a.elem_seg, a.seg_done, e)) live = false;
  if (!live) return;  // the slot is one whole wavefront: nothing else waits for it
  T* sm = smem + slot * 3 * S;
  T* sA = sm;
  T* sB = sm + S;
  T* sC = sm + 2 * S;
  auto F = [&](int k) { return frag[k * 64 + l]; };
  auto wsync = [] {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };
  const vec zero = {0, 0, 0, 0};

  // ---- K: X[r][(q,p)] from global (gathered when ASM) ----
  const int32_t* l2ge = ASM ? a.l2g + e * N3 : nullptr;
  const T* xe = ASM ? a.in : a.in + e * N3;
  {
    const T f0 = F(FK), f1 = F(FK + 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 16 * c + cl;  // (q,p) = col
      T x0 = 0, x1 = 0;
      if (col < NN) {
        const int r0 = g, r1 = 4 + g;
        if constexpr (ASM) {
          int32_t g0 = -1, g1 = -1;
          if (r0 < N) {
            g0 = l2ge[r0 * NN + col];
            x0 = xe[l2g_dof(g0)];
          }
          if (r1 < N) {
            g1 = l2ge[r1 * NN + col];
            x1 = xe[l2g_dof(g1)];
          }
          x0 = l2g_value(g0, x0);
          x1 = l2g_value(g1, x1);
        } else {
          if (r0 < N) x0 = xe[r0 * NN + col];
          if (r1 < N) x1 = xe[r1 * NN + col];
        }
      }
      vec acc = mfma(f0, x0, zero);
      acc = mfma(f1, x1, acc);
      if (col < NN) {
        // g<2: t_B[k = 4g+v], else t_D[k = 4(g-2)+v]
        T* dst = g < 2 ? sA : sB;
        const int k0 = 4 * (g % 2);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (k0 + v < Q) dst[(k0 + v) * NN + col] = acc[v];
      }
    }
  }
  wsync();
  // ---- J: X[q][(p,k)] = t[k][q][p] ----
  vec ja[4], jb[4];
  {
    const T fa0 = F(FJA), fa1 = F(FJA + 1), fb0 = F(FJB), fb1 = F(FJB + 1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 16 * c + cl;  // (p,k): p = col % N, k = col / N
      const int p = col % N, k = col / N;
      const bool ok = col < N * Q;
      const int q0 = g, q1 = 4 + g;
      const T a0 = (ok && q0 < N) ? sA[k * NN + q0 * N + p] : T(0);
      const T a1 = (ok && q1 < N) ? sA[k * NN + q1 * N + p] : T(0);
      const T b0 = (ok && q0 < N) ? sB[k * NN + q0 * N + p] : T(0);
      const T b1 = (ok && q1 < N) ? sB[k * NN + q1 * N + p] : T(0);
      ja[c] = mfma(fa1, a1, mfma(fa0, a0, zero));
      jb[c] = mfma(fb1, b1, mfma(fb0, b0, zero));
    }
  }
  wsync();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = 16 * c + cl;
    if (col < N * Q) {
      const int p = col % N, k = col / N;
      const int j0 = 4 * (g % 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = j0 + v;
        if (j < Q) {
          const int o = (k * Q + j) * N + p;
          if (g < 2) {
            sA[o] = ja[c][v];  // s_BB
            sC[o] = jb[c][v];  // s_BD
          } else {
            sB[o] = ja[c][v];  // s_DB
          }
        }
      }
    }
  }
  wsync();
  // ---- I: X[p][(j,k)] = s[k][j][p]; pointwise; I' from registers ----
  const T lam = (T)(a.lam ? a.lam[e] : a.lam0);
  const T* fe = a.fac + e * (int64_t)(kNF3 * Q3);
  {
    const T fia0 = F(FIA), fia1 = F(FIA + 1);
    const T fib0 = F(FIB), fib1 = F(FIB + 1), fib2 = F(FIB + 2), fib3 = F(FIB + 3);
    T fp[8];
#pragma unroll
    for (int s = 0; s < 6; ++s) fp[s] = F(FPA + s);
    fp[6] = F(FPB);
    fp[7] = F(FPB + 1);
    // factors of this lane's two points per column tile; tile c+1's loads
    // are issued before tile c is computed (double buffer)
    auto load_f = [&](int c, T (&dst)[2][kNF3]) {
      const int col = 16 * c + cl;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * g + h;
        const bool okp = col < QQ && i < Q;
        const T* fq = fe + (okp ? i * QQ + col : 0);
#pragma unroll
        for (int f = 0; f < kNF3; ++f) dst[h][f] = fq[f * Q3];
      }
    };
    T fcur[2][kNF3], fnxt[2][kNF3];
    load_f(0, fcur);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c + 1 < 4) load_f(c + 1, fnxt);
      const int col = 16 * c + cl;  // (j,k) = col
      const bool ok = col < QQ;
      const int p0 = g, p1 = 4 + g;
      const int base = col * N;   // (k*Q + j)*N with col = j + Q k
      const T x0 = (ok && p0 < N) ? sA[base + p0] : T(0);
      const T x1 = (ok && p1 < N) ? sA[base + p1] : T(0);
      const T y0 = (ok && p0 < N) ? sB[base + p0] : T(0);
      const T y1 = (ok && p1 < N) ? sB[base + p1] : T(0);
      const T z0 = (ok && p0 < N) ? sC[base + p0] : T(0);
      const T z1 = (ok && p1 < N) ? sC[base + p1] : T(0);
      const vec uu = mfma(fia1, x1, mfma(fia0, x0, zero));               // u, u1
      const vec vv = mfma(fib3, z1, mfma(fib2, z0, mfma(fib1, y1, mfma(fib0, y0, zero))));  // u2, u3
      // two points i = 2g + h, h = 0, 1 at column (j,k)
      T q[4][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int i = 2 * g + h;
        const T u = uu[2 * h], u1 = uu[2 * h + 1], u2 = vv[2 * h], u3 = vv[2 * h + 1];
        const bool okp = ok && i < Q;
        const T* f = fcur[h];
        q[0][h] = okp ? lam * f[0] * u : T(0);
        q[1][h] = okp ? f[1] * u1 + f[2] * u2 + f[3] * u3 : T(0);
        q[2][h] = okp ? f[2] * u1 + f[4] * u2 + f[5] * u3 : T(0);
        q[3][h] = okp ? f[3] * u1 + f[5] * u2 + f[6] * u3 : T(0);
      }
      // I': k-step s feeds quantity s/2 at point 2g + s%2 (this lane's own points)
      vec acc = zero;
#pragma unroll
      for (int s = 0; s < 6; ++s) acc = mfma(fp[s], q[s / 2][s % 2], acc);
      const vec accb = mfma(fp[7], q[3][1], mfma(fp[6], q[3][0], zero));
      // column (j,k) was read above by this wavefront only, so its results
      // can overwrite it in place (LDS operations of one wave stay in order)
      if (ok) {
        const int p0 = 4 * (g % 2);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = p0 + v;
          if (p < N) {
            const int o = base + p;
            if (g < 2) {
              sA[o] = acc[v];   // s'_BB
              sC[o] = accb[v];  // s'_BD
            } else {
              sB[o] = acc[v];   // s'_DB
            }
          }
        }
      }
      if (c + 1 < 4) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int f = 0; f < kNF3; ++f) fcur[h][f] = fnxt[h][f];
      }
    }
  }
  wsync();
  // ---- J': X[(t, j)][(p,k)], t in {s'_BB, s'_DB, s'_BD} ----
  vec jt[4];
  {
    T fj[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) fj[s] = F(FJT + s);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 16 * c + cl;
      const int p = col % N, k = col / N;
      const bool ok = col < N * Q;
      vec acc = zero;
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int j = 4 * (s % 2) + g;
        const T* src = s / 2 == 0 ? sA : s / 2 == 1 ? sB : sC;
        const T xv = (ok && j < Q) ? src[(k * Q + j) * N + p] : T(0);
        acc = mfma(fj[s], xv, acc);
      }
      jt[c] = acc;
    }
  }
  wsync();
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int col = 16 * c + cl;
    if (col < N * Q) {
      const int p = col % N, k = col / N;
      const int q0 = 4 * (g % 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int q = q0 + v;
        if (q < N) (g < 2 ? sA : sB)[k * NN + q * N + p] = jt[c][v];  // t'_B | t'_D
      }
    }
  }
  wsync();
  // ---- K': X[(t, k)][(q,p)], t in {t'_B, t'_D}; y[r][(q,p)] ----
  {
    T fk[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) fk[s] = F(FKT + s);
    double dp = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int col = 16 * c + cl;
      const bool ok = col < NN;
      vec acc = zero;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int k = 4 * (s % 2) + g;
        const T* src = s / 2 == 0 ? sA : sB;
        const T xv = (ok && k < Q) ? src[k * NN + col] : T(0);
        acc = mfma(fk[s], xv, acc);
      }
      if (ok && g < 2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 4 * g + v;
          if (r < N) {
            if constexpr (ASM) {
              const int32_t gi = l2ge[r * NN + col];
              if (gi >= 0) {
                const T yv = l2g_sign(gi, acc[v]);
                atomic_add(a.out + l2g_dof(gi), yv);
                dp += (double)xe[l2g_dof(gi)] * (double)yv;
              }
            } else {
              a.out[e * N3 + r * NN + col] = acc[v];
            }
          }
        }
      }
    }
    if constexpr (ASM) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) dp += __shfl_xor(dp, o);
      if (l == 0 && a.dots) add_dot(a.dots, a.dslot, e, dp);
    }
  }
}

template <typename T, int P, int EPB, bool ASM>
static hipError_t run_mfma(const OpArgs& a) {
  constexpr int N = P + 1, Q = P + 2;
  const T* frag = device_fragments<T>(P);
  if (!frag) return hipErrorOutOfMemory;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_helm_mfma<T, N, Q, EPB, ASM>), dim3((unsigned)nblk), dim3(EPB * 64), 0,
                     a.stream, frag, dev_args<T>(a));
  return hipGetLastError();
}

template <int P>
static hipError_t run_mfma_p(nk_dtype t, const OpArgs& a) {
  const bool asmb = a.op == OP_HELM_ASM;
  if (t == NK_F64)
    return asmb ? run_mfma<double, P, 2, true>(a) : run_mfma<double, P, 2, false>(a);
  return asmb ? run_mfma<float, P, 2, true>(a) : run_mfma<float, P, 2, false>(a);
}

bool mfma_supported(int dim, int P) { return dim == 3 && P >= 2 && P <= 6; }

hipError_t launch_helm_mfma(nk_dtype t, const OpArgs& a) {
  if (a.op != OP_HELM && a.op != OP_HELM_ASM) return hipErrorInvalidValue;
  if (a.nelem == 0) return hipSuccess;
  switch (a.P) {
    case 2: return run_mfma_p<2>(t, a);
    case 3: return run_mfma_p<3>(t, a);
    case 4: return run_mfma_p<4>(t, a);
    case 5: return run_mfma_p<5>(t, a);
    case 6: return run_mfma_p<6>(t, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace nk
