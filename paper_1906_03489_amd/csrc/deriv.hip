// Derivative and projection operators around the Helmholtz path (the
// explicit-type building blocks of section 2.2 and the projection of the
// listing in section 3.5):
//
//   PhysDeriv             du/dx_c at the quadrature points: collocation
//                         derivative of the point values along each reference
//                         direction, then the chain rule with J^{-1}.
//   IProductWRTDerivBase  sum_q w detJ grad phi_m . f: the per-point
//                         transform g_a = w detJ sum_c (J^{-1})_{ac} f_c, then
//                         the transposed sum-factorisation sweeps (D along
//                         direction a, B along the others).
//   FwdTrans              u^_e = M_e^{-1} IProductWRTBase(f): per element,
//                         conjugate gradients on the sum-factorised mass
//                         operator, preconditioned with the exact inverse of
//                         the tensor-product mass at the element's mean
//                         Jacobian determinant (fast diagonalisation: the 1-D
//                         reference mass M1 = V diag(lam) V^T gives
//                         (M1 x M1 x M1)^{-1} = (V x V x V) diag(1/(lam lam lam))
//                         (V x V x V)^T, V block diagonal in the even and odd
//                         modes).  The whole iteration stays on chip;
//                         HBM sees the point values, w detJ and the result.
//
// Element data layouts as for the other operators: points [E][Q^d] with
// q = i + Q(j + Q k), coefficients [E][n^d] with m = p + n(q + n r); vector
// fields [E][d][Q^d].  Derivative factors [E][d*d+1][Q^d] (J^{-1} entry
// (a,c) at a*d + c, then w detJ) in point order.
#include <cmath>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "tables.h"

namespace nk {

// ----------------------------------------------------------- device tables

// Device copy of a host-built table, built once per (device, key).
template <typename T, typename Build>
static const T* cached_table(long key, Build build) {
  static std::mutex mu;
  static std::unordered_map<long, T*> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  const long k = key * 64 + dev;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(k);
  if (it != cache.end()) return it->second;
  std::vector<double> h = build();
  std::vector<T> ht(h.begin(), h.end());
  T* d = nullptr;
  if (hipMalloc((void**)&d, ht.size() * sizeof(T)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, ht.data(), ht.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  cache[k] = d;
  return d;
}

// Collocation derivative matrix on the Q GLL points, row-major [Q][Q].
template <typename T>
static const T* colloc_table(int Q) {
  return cached_table<T>(Q, [Q] {
    std::vector<double> x(Q), w(Q), Dc(Q * Q);
    gll_points(Q, x.data(), w.data());
    collocation_derivative(Q, x.data(), Dc.data());
    return Dc;
  });
}

// Fast-diagonalisation tables of order P.  2-D: VT [N][N] (VT[o][m] =
// V[m][o]), V [N][N], then S [N^2] with S[p + N q] = 1 / (lam_p lam_q), from
// the 1-D modal mass M1 = V diag(lam) V^T.  3-D: M1 commutes with the
// reflection of the modes (the vertex swap and the sign of the odd interior
// modes; see the even-odd tables of engine.h), so in the orthonormal basis of
// even members ((d_0 + d_P)/sqrt 2, d_1, d_3, ...) and odd members
// ((d_0 - d_P)/sqrt 2, d_2, ...) it is block diagonal, M_e = V_e L_e V_e^T and
// M_o = V_o L_o V_o^T, and the eigenvector transforms act on the split
// coefficients of eo_split / eo_join: FE [KE][KE] and FO [KO][KO] with
// F[a][k] = V[k][a] (column k = 0 divided by sqrt 2, which maps the split's
// c_0 +- c_P onto the orthonormal vertex members), GE and GO their
// transposes (the same scaling on row 0), then S [N^3] with
// S[a + N(b + N c)] = 1 / (lam_a lam_b lam_c) in the eigen ordering (the KE
// even eigenvalues, then the KO odd ones).
template <typename T>
static const T* fastdiag_table(int P, int Q, int dim) {
  return cached_table<T>(1000L * dim + 32L * P + Q, [P, Q, dim] {
    const int N = P + 1;
    std::vector<double> x(Q), w(Q), B(Q * N), D(Q * N), M(N * N, 0.0), V(N * N), lam(N);
    gll_points(Q, x.data(), w.data());
    modified_basis(P, Q, x.data(), B.data(), D.data());
    for (int p = 0; p < N; ++p)
      for (int pp = 0; pp < N; ++pp)
        for (int i = 0; i < Q; ++i) M[p * N + pp] += w[i] * B[i * N + p] * B[i * N + pp];
    if (dim == 2) {
      symmetric_eigen(N, M.data(), V.data(), lam.data());
      std::vector<double> t(2 * N * N + N * N);
      for (int o = 0; o < N; ++o)
        for (int m = 0; m < N; ++m) {
          t[o * N + m] = V[m * N + o];
          t[N * N + o * N + m] = V[o * N + m];
        }
      for (int id = 0; id < N * N; ++id) {
        const int p = id % N, q = id / N;
        t[2 * N * N + id] = 1.0 / (lam[p] * lam[q]);
      }
      return t;
    }
    const int KE = P / 2 + 1, KO = (P - 1) / 2 + 1;
    const double r2 = std::sqrt(0.5);
    // orthonormal basis vectors (columns), even members then odd members
    auto basis = [&](int col, int k) {   // component k of basis vector col
      if (col == 0) return (k == 0 || k == P) ? r2 : 0.0;
      if (col < KE) return k == 2 * col - 1 ? 1.0 : 0.0;
      const int m = col - KE;
      if (m == 0) return k == 0 ? r2 : (k == P ? -r2 : 0.0);
      return k == 2 * m ? 1.0 : 0.0;
    };
    auto block = [&](int c0, int n, std::vector<double>& Vb, std::vector<double>& lb) {
      std::vector<double> Mb(n * n, 0.0);
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
          for (int k = 0; k < N; ++k)
            for (int l = 0; l < N; ++l)
              Mb[a * n + b] += basis(c0 + a, k) * M[k * N + l] * basis(c0 + b, l);
      Vb.assign(n * n, 0.0);
      lb.assign(n, 0.0);
      symmetric_eigen(n, Mb.data(), Vb.data(), lb.data());
    };
    std::vector<double> Ve, le, Vo, lo;
    block(0, KE, Ve, le);
    block(KE, KO, Vo, lo);
    std::vector<double> t;
    for (int a = 0; a < KE; ++a)        // FE[a][k] = Ve[k][a] (k = 0 scaled)
      for (int k = 0; k < KE; ++k) t.push_back(Ve[k * KE + a] * (k == 0 ? r2 : 1.0));
    for (int a = 0; a < KO; ++a)        // FO
      for (int k = 0; k < KO; ++k) t.push_back(Vo[k * KO + a] * (k == 0 ? r2 : 1.0));
    for (int k = 0; k < KE; ++k)        // GE[k][a] = Ve[k][a] (k = 0 scaled)
      for (int a = 0; a < KE; ++a) t.push_back(Ve[k * KE + a] * (k == 0 ? r2 : 1.0));
    for (int k = 0; k < KO; ++k)        // GO
      for (int a = 0; a < KO; ++a) t.push_back(Vo[k * KO + a] * (k == 0 ? r2 : 1.0));
    auto ev = [&](int i) { return i < KE ? le[i] : lo[i - KE]; };
    for (int id = 0; id < N * N * N; ++id) {
      const int a = id % N, b = (id / N) % N, c = id / (N * N);
      t.push_back(1.0 / (ev(a) * ev(b) * ev(c)));
    }
    return t;
  });
}

// Slot-wide sum visible to every thread of the slot.  Slots that fit in a
// wavefront reduce with lane shuffles inside their lane group; larger slots
// (one per block) combine per-wavefront partials through LDS.
template <int NT>
__device__ __forceinline__ double slot_allsum(double v, double* red) {
  if constexpr (NT <= 64) {
#pragma unroll
    for (int o = NT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  } else {
    constexpr int NW = (NT + 63) / 64;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k];
    return s;
  }
}

template <int Q>
constexpr int deriv_epb() {
  return slot_threads<Q>() >= 64 ? (slot_threads<Q>() > 64 ? 1 : 4) : 256 / slot_threads<Q>();
}

// --------------------------------------------------------------- PhysDeriv

// 3-D: thread t = i + Q j of a slot owns the column (i, j) over k.
template <typename T, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_phys_deriv3(const T* __restrict__ dc, int64_t nelem, const T* __restrict__ in,
                  T* __restrict__ out, const T* __restrict__ dfac) {
  constexpr int QQ = Q * Q, Q3 = QQ * Q, NT = slot_threads<Q>();
  __shared__ T smem[EPB * Q3];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool act = e < nelem && t < QQ;
  T* sm = smem + slot * Q3;
  const int i = t % Q, j = t / Q;
  T col[Q];
  if (act) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      col[k] = in[e * Q3 + t + QQ * k];
      sm[t + QQ * k] = col[k];
    }
  }
  slot_sync<NT>();
  if (!act) return;
  T di[Q], dj[Q];
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    di[m] = dc[i * Q + m];
    dj[m] = dc[j * Q + m];
  }
  const T* fe = dfac + e * (int64_t)(10 * Q3) + t;
  T* oe = out + e * (int64_t)(3 * Q3) + t;
#pragma unroll 2
  for (int k = 0; k < Q; ++k) {
    const T* row = sm + QQ * k;
    const T* dk = dc + k * Q;
    T d1 = 0, d2 = 0, d3 = 0;
#pragma unroll
    for (int m = 0; m < Q; ++m) {
      d1 += di[m] * row[m + Q * j];
      d2 += dj[m] * row[i + Q * m];
      d3 += dk[m] * col[m];
    }
    const T* f = fe + QQ * k;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      oe[c * Q3 + QQ * k] = f[c * Q3] * d1 + f[(3 + c) * Q3] * d2 + f[(6 + c) * Q3] * d3;
  }
}

// 2-D: thread t = i + Q j of a slot owns point (i, j).
template <typename T, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_phys_deriv2(const T* __restrict__ dc, int64_t nelem, const T* __restrict__ in,
                  T* __restrict__ out, const T* __restrict__ dfac) {
  constexpr int QQ = Q * Q, NT = slot_threads<Q>();
  __shared__ T smem[EPB * QQ];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool act = e < nelem && t < QQ;
  T* sm = smem + slot * QQ;
  if (act) sm[t] = in[e * QQ + t];
  slot_sync<NT>();
  if (!act) return;
  const int i = t % Q, j = t / Q;
  T d1 = 0, d2 = 0;
#pragma unroll
  for (int m = 0; m < Q; ++m) {
    d1 += dc[i * Q + m] * sm[m + Q * j];
    d2 += dc[j * Q + m] * sm[i + Q * m];
  }
  const T* f = dfac + e * (int64_t)(5 * QQ) + t;
  T* o = out + e * (int64_t)(2 * QQ) + t;
  o[0] = f[0] * d1 + f[2 * QQ] * d2;
  o[QQ] = f[QQ] * d1 + f[3 * QQ] * d2;
}

// ---------------------------------------------------- IProductWRTDerivBase

// 3-D.  Pass 1, thread t = i + Q j over k: g_a = w detJ sum_c (J^{-1})_{ac}
// f_c into LDS [a][Q^3].  Pass 2, thread t = j + Q k along i: the transposed
// I stage with D for g_1 and B for g_2, g_3, then the engine's J' and K'.
template <typename T, int N, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_iprod_deriv3(const Tab<T, N, Q> tb, int64_t nelem, const T* __restrict__ in,
                   T* __restrict__ out, const T* __restrict__ dfac) {
  constexpr int NN = N * N, N3 = NN * N, QQ = Q * Q, Q3 = QQ * Q, NT = slot_threads<Q>();
  static_assert(3 * Q3 >= slot_lds<N, Q>(), "LDS slot");
  __shared__ T smem[EPB * 3 * Q3];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool live = e < nelem;
  const bool act = live && t < QQ;
  const int64_t ee = live ? e : 0;
  T* sm = smem + slot * 3 * Q3;
  if (act) {
    const T* fe = dfac + ee * (int64_t)(10 * Q3) + t;
    const T* xe = in + ee * (int64_t)(3 * Q3) + t;
#pragma unroll 2
    for (int k = 0; k < Q; ++k) {
      const int o = QQ * k;
      const T f1 = xe[o], f2 = xe[Q3 + o], f3 = xe[2 * Q3 + o];
      const T* f = fe + o;
      const T wj = f[9 * Q3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        sm[a * Q3 + t + o] = wj * (f[(3 * a) * Q3] * f1 + f[(3 * a + 1) * Q3] * f2 +
                                   f[(3 * a + 2) * Q3] * f3);
    }
  }
  slot_sync<NT>();
  // transposed I stage in even-odd pairs: D for g_1, B for g_2, g_3
  constexpr int KE = EO<N>::KE, KO = EO<N>::KO;
  T sae[KE], sao[KO], sbe[KE], sbo[KO], sce[KE], sco[KO];
  zero(sae);
  zero(sao);
  zero(sbe);
  zero(sbo);
  zero(sce);
  zero(sco);
  if (act) {
    const T* g = sm + Q * t;
#pragma unroll 2
    for (int h = 0; h < Q / 2; ++h) {
      const int l = h, u = Q - 1 - h;
      const T a1 = g[l], a2 = g[u], b1 = g[Q3 + l], b2 = g[Q3 + u], c1 = g[2 * Q3 + l],
              c2 = g[2 * Q3 + u];
      eo_acc_d(tb, h, a1 + a2, a1 - a2, sae, sao);
      eo_acc(tb, h, b1 + b2, b1 - b2, sbe, sbo);
      eo_acc(tb, h, c1 + c2, c1 - c2, sce, sco);
    }
    if constexpr (Q & 1) {
      eo_acc_mid_d(tb, g[Q / 2], sao);
      eo_acc_mid(tb, g[Q3 + Q / 2], sbe);
      eo_acc_mid(tb, g[2 * Q3 + Q / 2], sce);
    }
  }
  T sa[N], sb[N], sc[N];
  eo_join<T, N>(sae, sao, sa);
  eo_join<T, N>(sbe, sbo, sb);
  eo_join<T, N>(sce, sco, sc);
  slot_sync<NT>();
  if (act) store_i<T, N, Q, true>(sm, t, sa, sb, sc);
  slot_sync<NT>();
  stage_jt<T, N, Q, NT, true>(tb, sm, t, live);
  slot_sync<NT>();
  T yv[N];
  stage_kt<T, N, Q, true>(tb, sm, t, live, yv);
  if (live && t < NN) {
#pragma unroll
    for (int r = 0; r < N; ++r) out[e * N3 + r * NN + t] = yv[r];
  }
}

// 2-D: thread t = i + Q j computes g_a at its point; then thread j sums
// over i (D for g_1, B for g_2) into h_a[p][j], and thread p sums over j
// (B for h_1, D for h_2).  Table rows are indexed by the loop counter only.
template <typename T, int N, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_iprod_deriv2(const Tab<T, N, Q> tb, int64_t nelem, const T* __restrict__ in,
                   T* __restrict__ out, const T* __restrict__ dfac) {
  constexpr int QQ = Q * Q, NT = slot_threads<Q>();
  __shared__ T smem[EPB * 2 * QQ];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool live = e < nelem;
  T* sm = smem + slot * 2 * QQ;
  if (live && t < QQ) {
    const T* f = dfac + e * (int64_t)(5 * QQ) + t;
    const T* x = in + e * (int64_t)(2 * QQ) + t;
    const T f1 = x[0], f2 = x[QQ], wj = f[4 * QQ];
    sm[t] = wj * (f[0] * f1 + f[QQ] * f2);                // g_1
    sm[QQ + t] = wj * (f[2 * QQ] * f1 + f[3 * QQ] * f2);  // g_2
  }
  slot_sync<NT>();
  T h1[N], h2[N];
#pragma unroll
  for (int p = 0; p < N; ++p) h1[p] = h2[p] = T(0);
  if (live && t < Q) {
#pragma unroll 2
    for (int i = 0; i < Q; ++i) {
      const T g1 = sm[i + Q * t], g2 = sm[QQ + i + Q * t];
      const T* Bi = tb.B + i * N;
      const T* Di = tb.D + i * N;
#pragma unroll
      for (int p = 0; p < N; ++p) {
        h1[p] += Di[p] * g1;
        h2[p] += Bi[p] * g2;
      }
    }
  }
  slot_sync<NT>();
  if (live && t < Q) {
#pragma unroll
    for (int p = 0; p < N; ++p) {
      sm[p * Q + t] = h1[p];
      sm[QQ + p * Q + t] = h2[p];
    }
  }
  slot_sync<NT>();
  if (live && t < N) {
    T y[N];
#pragma unroll
    for (int q = 0; q < N; ++q) y[q] = T(0);
#pragma unroll 2
    for (int j = 0; j < Q; ++j) {
      const T a = sm[t * Q + j], b = sm[QQ + t * Q + j];
      const T* Bj = tb.B + j * N;
      const T* Dj = tb.D + j * N;
#pragma unroll
      for (int q = 0; q < N; ++q) y[q] += Bj[q] * a + Dj[q] * b;
    }
#pragma unroll
    for (int q = 0; q < N; ++q) out[e * (N * N) + q * N + t] = y[q];
  }
}

// ----------------------------------------------------------------- FwdTrans

// y = M_e x for the slot's element: BwdTrans stages, w detJ at the points,
// IProductWRTBase stages.  Vectors are columns over r of thread t = p + N q.
template <typename T, int N, int Q, int NT>
__device__ __forceinline__ void fd_mass(const Tab<T, N, Q>& tb, T* __restrict__ sm, int t,
                                        bool live, const T (&x)[N], const T (&wj)[Q], T (&y)[N]) {
  stage_k<T, N, Q, false>(tb, sm, t, live, x);
  slot_sync<NT>();
  stage_j<T, N, Q, NT, false>(tb, sm, t, live);
  slot_sync<NT>();
  T se[EO<N>::KE], so[EO<N>::KO];
  zero(se);
  zero(so);
  if (live && t < Q * Q) {
    T ae[EO<N>::KE], ao[EO<N>::KO];
    {
      T av[N], dum[N];
      load_i<T, N, Q, false>(sm, t, av, dum, dum);
      eo_split<T, N>(av, ae, ao);
    }
    // point pairs (h, Q-1-h); wj is indexed by constants only (full unroll)
#pragma unroll
    for (int h = 0; h < Q / 2; ++h) {
      T ul, uh;
      eo_val(tb, h, ae, ao, ul, uh);
      const T ml = wj[h] * ul, mh = wj[Q - 1 - h] * uh;
      eo_acc(tb, h, ml + mh, ml - mh, se, so);
    }
    if constexpr (Q & 1) eo_acc_mid(tb, wj[Q / 2] * eo_mid_val(tb, ae), se);
  }
  T sa[N];
  eo_join<T, N>(se, so, sa);
  slot_sync<NT>();
  if (live && t < Q * Q) store_i<T, N, Q, false>(sm, t, sa, sa, sa);
  slot_sync<NT>();
  stage_jt<T, N, Q, NT, false>(tb, sm, t, live);
  slot_sync<NT>();
  stage_kt<T, N, Q, false>(tb, sm, t, live, y);
  slot_sync<NT>();
}

// The even or odd block transform of one split pencil: FWD applies FE / FO
// to the split coefficients, else GE / GO to eigen-coordinates.
template <typename T, int N, bool FWD>
__device__ __forceinline__ void fd_eo_apply(const T* __restrict__ tab, const T (&ie)[EO<N>::KE],
                                            const T (&io)[EO<N>::KO], T (&oe)[EO<N>::KE],
                                            T (&oo)[EO<N>::KO]) {
  constexpr int KE = EO<N>::KE, KO = EO<N>::KO;
  const T* Ae = tab + (FWD ? 0 : KE * KE + KO * KO);
  const T* Ao = Ae + KE * KE;
#pragma unroll
  for (int o = 0; o < KE; ++o) {
    T v = 0;
#pragma unroll
    for (int m = 0; m < KE; ++m) v += Ae[o * KE + m] * ie[m];
    oe[o] = v;
  }
#pragma unroll
  for (int o = 0; o < KO; ++o) {
    T v = 0;
#pragma unroll
    for (int m = 0; m < KO; ++m) v += Ao[o * KO + m] * io[m];
    oo[o] = v;
  }
}

// One direction of the even-odd fast diagonalisation on the n^3 array X in
// LDS (layout [r][q][p]); thread t < N^2 owns the pencil along DIR.  FWD:
// split the pencil, apply FE / FO, store the KE even then the KO odd
// eigen-coordinates; else read those, apply GE / GO and join.
template <typename T, int N, int NT, int DIR, bool FWD>
__device__ __forceinline__ void fd_eo_contract(T* __restrict__ X, const T* __restrict__ tab, int t,
                                               bool act) {
  constexpr int NN = N * N, KE = EO<N>::KE, KO = EO<N>::KO;
  constexpr int stride = DIR == 0 ? 1 : DIR == 1 ? N : NN;
  const int a = t % N, b = t / N;
  const int base = DIR == 0 ? a * N + b * NN : DIR == 1 ? a + b * NN : a + b * N;
  const bool me = act && t < NN;
  T x[N];
  if (me) {
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = X[base + m * stride];
  }
  slot_sync<NT>();
  if (me) {
    T ie[KE], io[KO];
    if constexpr (FWD) {
      eo_split<T, N>(x, ie, io);
    } else {
#pragma unroll
      for (int m = 0; m < KE; ++m) ie[m] = x[m];
#pragma unroll
      for (int m = 0; m < KO; ++m) io[m] = x[KE + m];
    }
    T oe[KE], oo[KO];
    fd_eo_apply<T, N, FWD>(tab, ie, io, oe, oo);
    if constexpr (FWD) {
#pragma unroll
      for (int m = 0; m < KE; ++m) X[base + m * stride] = oe[m];
#pragma unroll
      for (int m = 0; m < KO; ++m) X[base + (KE + m) * stride] = oo[m];
    } else {
      T y[N];
      eo_join<T, N>(oe, oo, y);
#pragma unroll
      for (int m = 0; m < N; ++m) X[base + m * stride] = y[m];
    }
  }
  slot_sync<NT>();
}

// Direction p of the preconditioner: forward transform, the diagonal
// scaling, backward transform, all in the registers of the thread that owns
// the pencil (t = q + N r).
template <typename T, int N, int NT>
__device__ __forceinline__ void fd_eo_middle(T* __restrict__ X, const T* __restrict__ tab,
                                             const T* __restrict__ S, T inv_c, int t, bool act) {
  constexpr int NN = N * N, KE = EO<N>::KE, KO = EO<N>::KO;
  const int base = (t % N) * N + (t / N) * NN;
  const bool me = act && t < NN;
  if (me) {
    T x[N], ie[KE], io[KO], ye[KE], yo[KO];
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = X[base + m];
    eo_split<T, N>(x, ie, io);
    fd_eo_apply<T, N, true>(tab, ie, io, ye, yo);
#pragma unroll
    for (int m = 0; m < KE; ++m) ye[m] *= inv_c * S[base + m];
#pragma unroll
    for (int m = 0; m < KO; ++m) yo[m] *= inv_c * S[base + KE + m];
    fd_eo_apply<T, N, false>(tab, ye, yo, ie, io);
    eo_join<T, N>(ie, io, x);
#pragma unroll
    for (int m = 0; m < N; ++m) X[base + m] = x[m];
  }
  slot_sync<NT>();
}

// z = P^{-1} r = (1/c) (V x V x V) S (V x V x V)^T r, each 1-D transform in
// its even and odd blocks (half the products of a dense N x N one).  The
// thread t = p + N q holding r along direction r transforms it in registers;
// direction q goes through LDS both ways, direction p does forward, scaling
// and backward in one pass.
template <typename T, int N, int NT>
__device__ __forceinline__ void fd_precond(const T* __restrict__ tab, T* __restrict__ X, int t,
                                           bool live, T inv_c, const T (&r)[N], T (&z)[N]) {
  constexpr int NN = N * N, KE = EO<N>::KE, KO = EO<N>::KO;
  const bool me = live && t < NN;
  const T* S = tab + 2 * (KE * KE + KO * KO);
  if (me) {
    T ie[KE], io[KO], ye[KE], yo[KO];
    eo_split<T, N>(r, ie, io);
    fd_eo_apply<T, N, true>(tab, ie, io, ye, yo);
#pragma unroll
    for (int m = 0; m < KE; ++m) X[m * NN + t] = ye[m];
#pragma unroll
    for (int m = 0; m < KO; ++m) X[(KE + m) * NN + t] = yo[m];
  }
  slot_sync<NT>();
  fd_eo_contract<T, N, NT, 1, true>(X, tab, t, live);
  fd_eo_middle<T, N, NT>(X, tab, S, inv_c, t, live);
  fd_eo_contract<T, N, NT, 1, false>(X, tab, t, live);
  if (me) {
    T ye[KE], yo[KO], oe[KE], oo[KO];
#pragma unroll
    for (int m = 0; m < KE; ++m) ye[m] = X[m * NN + t];
#pragma unroll
    for (int m = 0; m < KO; ++m) yo[m] = X[(KE + m) * NN + t];
    fd_eo_apply<T, N, false>(tab, ye, yo, oe, oo);
    eo_join<T, N>(oe, oo, z);
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) z[k] = T(0);
  }
  slot_sync<NT>();
}

template <typename T, int N>
__device__ __forceinline__ double col_dot(const T (&a)[N], const T (&b)[N]) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) s += (double)a[k] * (double)b[k];
  return s;
}

// 3-D FwdTrans, one element per slot; all slots of a block are either one
// wavefront's lane groups (no block barriers) or the block itself.
template <typename T, int N, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot_threads<Q>())
    k_fwd_trans3(const Tab<T, N, Q> tb, const T* __restrict__ tab, int64_t nelem,
                 const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ dfac,
                 double rtol2, int maxit) {
  constexpr int NN = N * N, N3 = NN * N, QQ = Q * Q, Q3 = QQ * Q, NT = slot_threads<Q>();
  static_assert(NT <= 64 ? (64 % NT == 0 && EPB * NT <= 64) : EPB == 1, "slot layout");
  static_assert(Q3 >= slot_lds<N, Q>() / 3, "LDS slot");
  __shared__ T smem[EPB * Q3];
  __shared__ double red[(NT + 63) / 64];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool live = e < nelem;
  const int64_t ee = live ? e : 0;
  T* sm = smem + slot * Q3;
  // w detJ along this thread's pencil (j,k) = t over i, and the element's
  // mean Jacobian determinant c = sum(w detJ) / 2^3
  T wj[Q];
  {
    const T* we = dfac + ee * (int64_t)(10 * Q3) + 9 * Q3;
    if (live && t < QQ) {
#pragma unroll
      for (int k = 0; k < Q; ++k) sm[t + QQ * k] = we[t + QQ * k];
    }
    slot_sync<NT>();
    double ws = 0.0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      wj[i] = (live && t < QQ) ? sm[i + Q * t] : T(0);
      ws += (double)wj[i];
    }
    slot_sync<NT>();
    ws = slot_allsum<NT>(ws, red);
    // b = I_e(f): stage f through LDS for coalesced loads, then I', J', K'
    const T* fe = in + ee * (int64_t)Q3;
    if (live && t < QQ) {
#pragma unroll
      for (int k = 0; k < Q; ++k) sm[t + QQ * k] = fe[t + QQ * k];
    }
    slot_sync<NT>();
    T se[EO<N>::KE], so[EO<N>::KO];
    zero(se);
    zero(so);
    if (live && t < QQ) {
#pragma unroll
      for (int h = 0; h < Q / 2; ++h) {
        const T ml = wj[h] * sm[h + Q * t], mh = wj[Q - 1 - h] * sm[Q - 1 - h + Q * t];
        eo_acc(tb, h, ml + mh, ml - mh, se, so);
      }
      if constexpr (Q & 1) eo_acc_mid(tb, wj[Q / 2] * sm[Q / 2 + Q * t], se);
    }
    T sa[N];
    eo_join<T, N>(se, so, sa);
    slot_sync<NT>();
    if (live && t < QQ) store_i<T, N, Q, false>(sm, t, sa, sa, sa);
    slot_sync<NT>();
    stage_jt<T, N, Q, NT, false>(tb, sm, t, live);
    slot_sync<NT>();
    T b[N];
    stage_kt<T, N, Q, false>(tb, sm, t, live, b);
    slot_sync<NT>();
    const T inv_c = (T)(8.0 / ws);
    // preconditioned CG on M_e x = b, x0 = 0
    T x[N], r[N], p[N], q[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      x[k] = T(0);
      r[k] = b[k];
    }
    const double bb = slot_allsum<NT>(col_dot(b, b), red);
    fd_precond<T, N, NT>(tab, sm, t, live, inv_c, r, p);
    double rz = slot_allsum<NT>(col_dot(r, p), red);
    bool done = !(bb > 0.0);
    // every thread of a slot holds the same sums, so the slot leaves the
    // loop as a whole (a slot of more than 64 threads is its whole block)
    for (int it = 0; it < maxit && !done; ++it) {
      fd_mass<T, N, Q, NT>(tb, sm, t, live, p, wj, q);
      const double pq = slot_allsum<NT>(col_dot(p, q), red);
      if (!(pq > 0.0)) break;
      const T alpha = (T)(rz / pq);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        x[k] += alpha * p[k];
        r[k] -= alpha * q[k];
      }
      const double rr = slot_allsum<NT>(col_dot(r, r), red);
      if (rr <= rtol2 * bb) {
        done = true;
        continue;
      }
      fd_precond<T, N, NT>(tab, sm, t, live, inv_c, r, q);   // q <- z
      const double rzn = slot_allsum<NT>(col_dot(r, q), red);
      const T beta = (T)(rzn / rz);
      rz = rzn;
#pragma unroll
      for (int k = 0; k < N; ++k) p[k] = q[k] + beta * p[k];
    }
    if (live && t < NN) {
#pragma unroll
      for (int k = 0; k < N; ++k) out[e * N3 + k * NN + t] = x[k];
    }
  }
}

// 2-D FwdTrans.  A slot is the smallest power of two >= Q threads (so the
// slot-wide sums are lane-group shuffles); modal vectors are columns over q
// held by thread p < N (mode m = p + N q); point arrays by thread j < Q as
// columns over i.  Tables are read only at loop-uniform rows.
template <int Q>
constexpr int slot2_threads() {
  return Q <= 4 ? 4 : Q <= 8 ? 8 : 16;
}

// Contract direction DIR (0: p, 1: q) of the N x N array X (layout [q][p])
// with the table A: thread t < N owns the pencil along DIR.
template <typename T, int N, int DIR>
__device__ __forceinline__ void fd2_contract(T* __restrict__ X, const T* __restrict__ A, int t,
                                             bool act) {
  constexpr int stride = DIR == 0 ? 1 : N;
  const int base = DIR == 0 ? t * N : t;
  const bool me = act && t < N;
  T x[N];
  if (me) {
#pragma unroll
    for (int m = 0; m < N; ++m) x[m] = X[base + m * stride];
  }
  slot_sync<64>();
  if (me) {
#pragma unroll 2
    for (int o = 0; o < N; ++o) {
      const T* Ao = A + o * N;
      T s = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) s += Ao[m] * x[m];
      X[base + o * stride] = s;
    }
  }
  slot_sync<64>();
}

template <typename T, int N, int Q, int EPB>
__global__ void __launch_bounds__(EPB * slot2_threads<Q>())
    k_fwd_trans2(const Tab<T, N, Q> tb, const T* __restrict__ tab, int64_t nelem,
                 const T* __restrict__ in, T* __restrict__ out, const T* __restrict__ dfac,
                 double rtol2, int maxit) {
  constexpr int NN = N * N, QQ = Q * Q, NT = slot2_threads<Q>();
  static_assert(EPB * NT == 64, "one wavefront per block");
  __shared__ T smem[EPB * QQ];
  const int slot = threadIdx.x / NT, t = threadIdx.x - slot * NT;
  const int64_t nblk = (nelem + EPB - 1) / EPB;
  const int64_t e = xcd_remap(blockIdx.x, nblk) * EPB + slot;
  const bool live = e < nelem;
  const int64_t ee = live ? e : 0;
  T* sm = smem + slot * QQ;
  const bool pj = live && t < Q;   // point column j = t
  const bool pm = live && t < N;   // modal column p = t
  // w detJ along column j = t, and the mean Jacobian determinant c = sum / 2^2
  T wj[Q];
  const T* we = dfac + ee * (int64_t)(5 * QQ) + 4 * QQ;
  if (live) {
    for (int k = t; k < QQ; k += NT) sm[k] = we[k];
  }
  slot_sync<64>();
  double ws = 0.0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    wj[i] = pj ? sm[i + Q * t] : T(0);
    ws += (double)wj[i];
  }
  ws = slot_allsum<NT>(ws, nullptr);
  const T inv_c = (T)(4.0 / ws);
  slot_sync<64>();
  // y = (B^T x B^T)(wj * (B x B) x) for the column layout of thread p
  auto mass = [&](const T (&x)[N], T (&y)[N], bool with_bwd) {
    if (with_bwd) {
      // q -> j: thread p writes T1[j][p]
      if (pm) {
#pragma unroll 2
        for (int j = 0; j < Q; ++j) {
          const T* Bj = tb.B + j * N;
          T s = 0;
#pragma unroll
          for (int q = 0; q < N; ++q) s += Bj[q] * x[q];
          sm[j * N + t] = s;
        }
      }
      slot_sync<64>();
    }
    // p -> i, times w detJ, i -> p: thread j
    T s[N];
#pragma unroll
    for (int p = 0; p < N; ++p) s[p] = T(0);
    if (pj) {
      T a[N];
      if (with_bwd) {
#pragma unroll
        for (int p = 0; p < N; ++p) a[p] = sm[t * N + p];
      }
#pragma unroll 2
      for (int i = 0; i < Q; ++i) {
        const T* Bi = tb.B + i * N;
        T u;
        if (with_bwd) {
          u = 0;
#pragma unroll
          for (int p = 0; p < N; ++p) u += Bi[p] * a[p];
        } else {
          u = sm[i + Q * t];   // point values staged in LDS
        }
        const T mm = wj[i] * u;
#pragma unroll
        for (int p = 0; p < N; ++p) s[p] += Bi[p] * mm;
      }
    }
    slot_sync<64>();
    if (pj) {
#pragma unroll
      for (int p = 0; p < N; ++p) sm[t * N + p] = s[p];
    }
    slot_sync<64>();
    // j -> q: thread p
#pragma unroll
    for (int q = 0; q < N; ++q) y[q] = T(0);
    if (pm) {
#pragma unroll 2
      for (int j = 0; j < Q; ++j) {
        const T* Bj = tb.B + j * N;
        const T v = sm[j * N + t];
#pragma unroll
        for (int q = 0; q < N; ++q) y[q] += Bj[q] * v;
      }
    }
    slot_sync<64>();
  };
  auto precond = [&](const T (&r)[N], T (&z)[N]) {
    const T* VT = tab;
    const T* V = tab + NN;
    const T* S = tab + 2 * NN;
    if (pm) {
#pragma unroll
      for (int q = 0; q < N; ++q) sm[q * N + t] = r[q];
    }
    slot_sync<64>();
    fd2_contract<T, N, 1>(sm, VT, t, live);
    fd2_contract<T, N, 0>(sm, VT, t, live);
    if (pm) {
#pragma unroll
      for (int q = 0; q < N; ++q) sm[q * N + t] *= inv_c * S[q * N + t];
    }
    slot_sync<64>();
    fd2_contract<T, N, 0>(sm, V, t, live);
    fd2_contract<T, N, 1>(sm, V, t, live);
#pragma unroll
    for (int q = 0; q < N; ++q) z[q] = pm ? sm[q * N + t] : T(0);
    slot_sync<64>();
  };
  // b = I_e(f): stage f in LDS, then the transposed sweeps
  const T* fe = in + ee * (int64_t)QQ;
  if (live) {
    for (int k = t; k < QQ; k += NT) sm[k] = fe[k];
  }
  slot_sync<64>();
  T b[N], dummy[N];
#pragma unroll
  for (int q = 0; q < N; ++q) dummy[q] = T(0);
  mass(dummy, b, false);
  T x[N], r[N], p[N], q[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    x[k] = T(0);
    r[k] = b[k];
  }
  const double bb = slot_allsum<NT>(col_dot(b, b), nullptr);
  precond(r, p);
  double rz = slot_allsum<NT>(col_dot(r, p), nullptr);
  bool done = !(bb > 0.0);
  for (int it = 0; it < maxit && !done; ++it) {
    mass(p, q, true);
    const double pq = slot_allsum<NT>(col_dot(p, q), nullptr);
    if (!(pq > 0.0)) break;
    const T alpha = (T)(rz / pq);
#pragma unroll
    for (int k = 0; k < N; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * q[k];
    }
    const double rr = slot_allsum<NT>(col_dot(r, r), nullptr);
    if (rr <= rtol2 * bb) {
      done = true;
      continue;
    }
    precond(r, q);
    const double rzn = slot_allsum<NT>(col_dot(r, q), nullptr);
    const T beta = (T)(rzn / rz);
    rz = rzn;
#pragma unroll
    for (int k = 0; k < N; ++k) p[k] = q[k] + beta * p[k];
  }
  if (pm) {
#pragma unroll
    for (int k = 0; k < N; ++k) out[e * NN + k * N + t] = x[k];
  }
}

// ----------------------------------------------------------------- launchers

template <typename T, int P>
static hipError_t run_deriv(int which, int dim, const DerivArgs& a) {
  constexpr int N = P + 1, Q = P + 2;
  constexpr int EPB = deriv_epb<Q>();
  constexpr int NT = slot_threads<Q>();
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  const T* in = static_cast<const T*>(a.in);
  T* out = static_cast<T*>(a.out);
  const T* df = static_cast<const T*>(a.dfac);
  hipStream_t s = a.stream;
  if (which == DERIV_PHYS) {
    const T* dc = colloc_table<T>(Q);
    if (!dc) return hipErrorOutOfMemory;
    if (dim == 3)
      hipLaunchKernelGGL((k_phys_deriv3<T, Q, EPB>), dim3((unsigned)nblk), dim3(EPB * NT), 0, s, dc,
                         a.nelem, in, out, df);
    else
      hipLaunchKernelGGL((k_phys_deriv2<T, Q, EPB>), dim3((unsigned)nblk), dim3(EPB * NT), 0, s, dc,
                         a.nelem, in, out, df);
    return hipGetLastError();
  }
  const Tab<T, N, Q>& tb = host_tab<T, N, Q>();
  if (which == DERIV_IPROD) {
    if (dim == 3)
      hipLaunchKernelGGL((k_iprod_deriv3<T, N, Q, EPB>), dim3((unsigned)nblk), dim3(EPB * NT), 0, s,
                         tb, a.nelem, in, out, df);
    else
      hipLaunchKernelGGL((k_iprod_deriv2<T, N, Q, EPB>), dim3((unsigned)nblk), dim3(EPB * NT), 0, s,
                         tb, a.nelem, in, out, df);
    return hipGetLastError();
  }
  if (which == DERIV_FWD && dim == 2) {
    constexpr int NT2 = slot2_threads<Q>();
    constexpr int EPB2 = 64 / NT2;
    const int64_t nb2 = (a.nelem + EPB2 - 1) / EPB2;
    if (nb2 > 0x7fffffff) return hipErrorInvalidValue;
    const T* tab = fastdiag_table<T>(P, Q, 2);
    if (!tab) return hipErrorOutOfMemory;
    const double rtol = sizeof(T) == 8 ? 1e-13 : 2e-6;
    hipLaunchKernelGGL((k_fwd_trans2<T, N, Q, EPB2>), dim3((unsigned)nb2), dim3(64), 0, s, tb, tab,
                       a.nelem, in, out, df, rtol * rtol, kFwdMaxIt);
    return hipGetLastError();
  }
  if (which == DERIV_FWD && dim == 3) {
    constexpr int EPBF = NT <= 64 ? 64 / NT : 1;
    const int64_t nbf = (a.nelem + EPBF - 1) / EPBF;
    if (nbf > 0x7fffffff) return hipErrorInvalidValue;
    const T* tab = fastdiag_table<T>(P, Q, 3);
    if (!tab) return hipErrorOutOfMemory;
    const double rtol = sizeof(T) == 8 ? 1e-13 : 2e-6;
    hipLaunchKernelGGL((k_fwd_trans3<T, N, Q, EPBF>), dim3((unsigned)nbf), dim3(EPBF * NT), 0, s,
                       tb, tab, a.nelem, in, out, df, rtol * rtol, kFwdMaxIt);
    return hipGetLastError();
  }
  return hipErrorInvalidValue;
}

template <int P>
static hipError_t run_deriv_p(nk_dtype t, int which, int dim, const DerivArgs& a) {
  return t == NK_F64 ? run_deriv<double, P>(which, dim, a) : run_deriv<float, P>(which, dim, a);
}

hipError_t launch_deriv(nk_dtype t, int which, int dim, int P, const DerivArgs& a) {
  if (a.nelem == 0) return hipSuccess;
  switch (P) {
    case 1: return run_deriv_p<1>(t, which, dim, a);
    case 2: return run_deriv_p<2>(t, which, dim, a);
    case 3: return run_deriv_p<3>(t, which, dim, a);
    case 4: return run_deriv_p<4>(t, which, dim, a);
    case 5: return run_deriv_p<5>(t, which, dim, a);
    case 6: return run_deriv_p<6>(t, which, dim, a);
    case 7: return run_deriv_p<7>(t, which, dim, a);
    case 8: return run_deriv_p<8>(t, which, dim, a);
    case 9: return run_deriv_p<9>(t, which, dim, a);
    case 10: return run_deriv_p<10>(t, which, dim, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace nk
