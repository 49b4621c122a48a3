// Collapsed-coordinate triangles (section 2.1: a quadrilateral with one
// direction collapsed through the Duffy map; section 3.3: the expansion
// factors in the collapsed coordinates, so the operators stay
// sum-factorised).  Elemental BwdTrans, IProductWRTBase and Helmholtz.
//
// Basis: phi_m(eta_1, eta_2) = a_p(eta_1) b_m(eta_2) with modes grouped by the
// eta_1 index p (p = 0: q = 0..P, q = P the collapsed vertex (1+eta_2)/2
// which carries no eta_1 factor; 0 < p < P: q = 0..P-1-p; p = P: q = 0..P-1);
// a_p the 1-D modified basis, b_m the eta_2 factors.  Points: Q GLL points in
// eta_1 times Q-1 Radau points in eta_2, q = i + Q j.  The collapsed vertex is
// evaluated as a_0 b + a_P b (a_0 + a_P = 1), so every stage is a plain
// per-p contraction.
//
// Per element (one slot): coefficients -> LDS; eta_2 stage (thread j: v_p and
// dv_p/deta_2 at point row j for every p); eta_1 stage (thread per point: u,
// du/deta_1, du/deta_2); pointwise factors; transposed eta_1 stage (thread
// j); transposed eta_2 stage (thread per mode).  Factors per point (built at
// space creation): w detJ, then w detJ kappa (T^T G T) with T the Duffy
// chain rule d xi / d eta, so the kernel works in collapsed derivatives.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "tables.h"

namespace nk {

template <int P>
struct TriShape {
  static constexpr int N = P + 1, Q = P + 2, Q2 = Q - 1, NP = Q * Q2, NM = N * (N + 1) / 2;
  static constexpr int need0 = NP > NM ? NP : NM;
  static constexpr int need = need0 > Q2 * N ? need0 : Q2 * N;
  static constexpr int NT = need <= 8 ? 8 : need <= 16 ? 16 : need <= 32 ? 32 : need <= 64 ? 64
                                                          : (need + 63) / 64 * 64;
  static constexpr int EPB = NT <= 64 ? 512 / NT : 1;   // amortises the table copy
  static constexpr int cnt(int p) { return p == 0 ? P + 1 : (p == P ? P : P - p); }
  static constexpr int off(int p) {
    int o = 0;
    for (int k = 0; k < p; ++k) o += cnt(k);
    return o;
  }
  static constexpr int TAB = 2 * Q * N + 2 * Q2 * NM + Q2;   // A, DA, B2, dB2, (1+eta_2)/2
  static constexpr int SLOT = NM + 2 * Q2 * N + 3 * NP;
};

// Device table of order P: A [Q][N], DA [Q][N], B2 [Q2][NM], dB2 [Q2][NM],
// c [Q2] = (1 + eta_2)/2.
template <typename T>
static const T* tri_table(int P) {
  static std::mutex mu;
  static std::unordered_map<long, T*> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const long key = dev * 64L + P;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int N = P + 1, Q = P + 2, Q2 = Q - 1, NM = N * (N + 1) / 2;
  std::vector<double> e1(Q), w1(Q), e2(Q2), w2(Q2), A(Q * N), DA(Q * N), B2(Q2 * NM), dB2(Q2 * NM);
  tri_points(Q, e1.data(), w1.data(), e2.data(), w2.data());
  modified_basis(P, Q, e1.data(), A.data(), DA.data());
  tri_btable(P, Q2, e2.data(), B2.data(), dB2.data());
  std::vector<T> h;
  for (double v : A) h.push_back((T)v);
  for (double v : DA) h.push_back((T)v);
  for (double v : B2) h.push_back((T)v);
  for (double v : dB2) h.push_back((T)v);
  for (double v : e2) h.push_back((T)(0.5 * (1.0 + v)));
  T* d = nullptr;
  if (hipMalloc((void**)&d, h.size() * sizeof(T)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  cache[key] = d;
  return d;
}

template <typename T, int P, int OP>
__global__ void __launch_bounds__(TriShape<P>::EPB * TriShape<P>::NT)
    k_tri(const Tab<T, P + 1, P + 2> tb, const T* __restrict__ tab, const DevArgs<T> a) {
  using S = TriShape<P>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, NP = S::NP, NM = S::NM, NT = S::NT;
  constexpr int EPB = S::EPB;
  constexpr bool HELM = OP == OP_HELM;
  __shared__ T stab[S::TAB];
  __shared__ T smem[EPB * S::SLOT];
  for (int k = threadIdx.x; k < S::TAB; k += EPB * NT) stab[k] = tab[k];
  __syncthreads();
  const T* A = stab;
  const T* DA = stab + Q * N;
  const T* B2 = stab + 2 * Q * N;
  const T* dB2 = B2 + Q2 * NM;
  const T* cz = dB2 + Q2 * NM;
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool live = e < a.nelem;
  T* C = smem + slot * S::SLOT;   // coefficients [NM]
  T* V = C + NM;                   // [Q2][N]
  T* dV = V + Q2 * N;              // [Q2][N]
  T* Mq = dV + Q2 * N;             // [NP] each
  T* G1 = Mq + NP;
  T* G2 = G1 + NP;
  if constexpr (OP == OP_BWD || HELM) {
    if (live && t < NM) C[t] = a.in[e * NM + t];
    slot_sync<NT>();
    // eta_2 stage: thread (j, p) forms v_p(eta_2j) (and its derivative)
    if (live && t < Q2 * N) {
      const int j = t / N, p = t - (t / N) * N;
      const int m0 = p == 0 ? 0 : (P + 1) + (p - 1) * P - (p - 1) * p / 2;
      const int nq = p == 0 ? P + 1 : (p == P ? P : P - p);
      T v = 0, dv = 0;
      for (int q = 0; q < nq; ++q) {
        v += B2[j * NM + m0 + q] * C[m0 + q];
        if constexpr (HELM) dv += dB2[j * NM + m0 + q] * C[m0 + q];
      }
      if (p == P) {   // the collapsed vertex also multiplies a_P
        v += cz[j] * C[P];
        if constexpr (HELM) dv += T(0.5) * C[P];
      }
      V[j * N + p] = v;
      if constexpr (HELM) dV[j * N + p] = dv;
    }
    slot_sync<NT>();
    // eta_1 stage: thread per point
    if (live && t < NP) {
      const int i = t % Q, j = t / Q;
      T u = 0, u1 = 0, u2 = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        u += A[i * N + p] * V[j * N + p];
        if constexpr (HELM) {
          u1 += DA[i * N + p] * V[j * N + p];
          u2 += A[i * N + p] * dV[j * N + p];
        }
      }
      if constexpr (OP == OP_BWD) {
        a.out[e * NP + t] = u;
      } else {
        const T* f = a.fac + e * (int64_t)(4 * NP) + t;
        const T lam = (T)(a.lam ? a.lam[e] : a.lam0);
        Mq[t] = lam * f[0] * u;
        G1[t] = f[NP] * u1 + f[2 * NP] * u2;
        G2[t] = f[2 * NP] * u1 + f[3 * NP] * u2;
      }
    }
    if constexpr (OP == OP_BWD) return;
  } else {  // IProductWRTBase: point values times w detJ
    if (live && t < NP) Mq[t] = a.fac[e * (int64_t)(4 * NP) + t] * a.in[e * NP + t];
  }
  slot_sync<NT>();
  // transposed eta_1 stage: thread (j, p) accumulates over i
  if (live && t < Q2 * N) {
    const int j = t / N, p = t - (t / N) * N;
    T sa = 0, sb = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      sa += A[i * N + p] * Mq[i + Q * j];
      if constexpr (HELM) {
        sa += DA[i * N + p] * G1[i + Q * j];
        sb += A[i * N + p] * G2[i + Q * j];
      }
    }
    V[j * N + p] = sa;
    if constexpr (HELM) dV[j * N + p] = sb;
  }
  slot_sync<NT>();
  // transposed eta_2 stage: thread per mode
  if (live && t < NM) {
    int p = 0;
#pragma unroll
    for (int k = 1; k < N; ++k) p += (t >= S::off(k)) ? 1 : 0;
    T y = 0;
#pragma unroll 4
    for (int j = 0; j < Q2; ++j) {
      y += B2[j * NM + t] * V[j * N + p];
      if constexpr (HELM) y += dB2[j * NM + t] * dV[j * N + p];
    }
    if (t == P) {   // the collapsed vertex: its a_P part
#pragma unroll 4
      for (int j = 0; j < Q2; ++j) {
        y += cz[j] * V[j * N + P];
        if constexpr (HELM) y += T(0.5) * dV[j * N + P];
      }
    }
    a.out[e * NM + t] = y;
  }
}

template <typename T, int P>
static hipError_t run_tri(const OpArgs& a) {
  using S = TriShape<P>;
  const T* tab = tri_table<T>(P);
  if (!tab) return hipErrorOutOfMemory;
  const int64_t nblk = (a.nelem + S::EPB - 1) / S::EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const Tab<T, P + 1, P + 2>& tb = host_tab<T, P + 1, P + 2>();
  const DevArgs<T> d = dev_args<T>(a);
  const dim3 g((unsigned)nblk), b(S::EPB * S::NT);
  switch (a.op) {
    case OP_BWD: hipLaunchKernelGGL((k_tri<T, P, OP_BWD>), g, b, 0, a.stream, tb, tab, d); break;
    case OP_IPROD: hipLaunchKernelGGL((k_tri<T, P, OP_IPROD>), g, b, 0, a.stream, tb, tab, d); break;
    case OP_HELM: hipLaunchKernelGGL((k_tri<T, P, OP_HELM>), g, b, 0, a.stream, tb, tab, d); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int P>
static hipError_t run_tri_p(nk_dtype t, const OpArgs& a) {
  return t == NK_F64 ? run_tri<double, P>(a) : run_tri<float, P>(a);
}

hipError_t launch_tri(nk_dtype t, const OpArgs& a) {
  if (a.nelem == 0) return hipSuccess;
  switch (a.P) {
    case 1: return run_tri_p<1>(t, a);
    case 2: return run_tri_p<2>(t, a);
    case 3: return run_tri_p<3>(t, a);
    case 4: return run_tri_p<4>(t, a);
    case 5: return run_tri_p<5>(t, a);
    case 6: return run_tri_p<6>(t, a);
    case 7: return run_tri_p<7>(t, a);
    case 8: return run_tri_p<8>(t, a);
    case 9: return run_tri_p<9>(t, a);
    case 10: return run_tri_p<10>(t, a);
  }
  return hipErrorInvalidValue;
}

// Factors of the collapsed triangle at every point (thread per point):
// f0 = w detJ with w = w1_i w2_j / 2 (the Radau weight carries 1 - eta_2),
// f1..f3 = w detJ kappa (T^T G T)_{11,12,22}, G = J^{-1} J^{-T}, T = d xi / d eta.
__global__ void __launch_bounds__(256)
    k_geom_tri(int Q, int64_t nelem, const double* __restrict__ jac, const double* __restrict__ kappa,
               const double* __restrict__ pts, double* __restrict__ fac64, float* __restrict__ fac32,
               int* __restrict__ bad) {
  const int Q2 = Q - 1, NP = Q * Q2;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * NP) return;
  const int64_t e = id / NP;
  const int q = (int)(id - e * NP);
  const int i = q % Q, j = q / Q;
  const double e1 = pts[i], w1 = pts[Q + i], e2 = pts[2 * Q + j], w2 = pts[2 * Q + Q2 + j];
  double J[2][2];
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b) J[c][b] = jac[((e * 2 + c) * 2 + b) * NP + q];
  const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double id_ = 1.0 / det;
  const double Ji[2][2] = {{J[1][1] * id_, -J[0][1] * id_}, {-J[1][0] * id_, J[0][0] * id_}};
  double G[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) G[a][b] = Ji[a][0] * Ji[b][0] + Ji[a][1] * Ji[b][1];
  // T[a][b] = d xi_a / ... : grad_xi = T grad_eta
  const double T[2][2] = {{2.0 / (1.0 - e2), 0.0}, {(1.0 + e1) / (1.0 - e2), 1.0}};
  double H[2][2];   // T^T G T
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double s = 0.0;
      for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) s += T[c][a] * G[c][d] * T[d][b];
      H[a][b] = s;
    }
  const double kap = kappa ? kappa[e * NP + q] : 1.0;
  const double wj = 0.5 * w1 * w2 * det;
  const double f[4] = {wj, wj * kap * H[0][0], wj * kap * H[0][1], wj * kap * H[1][1]};
  if (!(det > 0.0) || !(kap > 0.0)) atomicOr(bad, 1);
  for (int k = 0; k < 4; ++k) {
    fac64[(e * 4 + k) * NP + q] = f[k];
    fac32[(e * 4 + k) * NP + q] = (float)f[k];
  }
}

hipError_t launch_geom_tri(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s) {
  const int64_t n = nelem * Q * (Q - 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geom_tri, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q, nelem, jac,
                     kappa, pts, fac64, fac32, bad);
  return hipGetLastError();
}

}  // namespace nk
