// Collapsed-coordinate tetrahedra, prisms and pyramids (section 2.1: shapes
// reached from the hexahedron through the Duffy map, collapsing two
// directions for the tetrahedron and one for the prism and the pyramid;
// section 3.3: the expansion factors in the collapsed coordinates, so the
// operators stay sum-factorised).  Elemental BwdTrans, IProductWRTBase and
// Helmholtz, the assembled Helmholtz operator (gather, Helmholtz,
// scatter-add, per-element energies) and its Jacobi diagonal.
//
// Prisms: the triangle of tri.hip in (xi_1, xi_2) extruded along xi_3, every
// mode a triangle mode times the 1-D modified basis phi_r(xi_3), r = 0..P
// (r fastest); Q GLL points in xi_3.  Pyramids: the lower part is the
// tensor-product quadrilateral phi_p(eta_1) phi_q(eta_2) (GLL points in both)
// instead of a triangle, with s = max(deg phi_p, deg phi_q) and the apex
// (1+eta_3)/2 riding on the four base vertex modes.  The kernel below serves
// all three shapes: the "lower" stages are the triangle's (tetrahedron,
// prism) or the quadrilateral's (pyramid), and the eta_3 table holds the
// shape's third-direction factors.
//
// Basis: every mode is a triangle mode T_t(eta_1, eta_2) of the order-P
// triangle (tri.hip), of total degree s_t, times an eta_3 factor c_{s,r}:
// ((1-eta_3)/2)^s for r = 0, times (1+eta_3)/2 P^{2s-1,1}_{r-1}(eta_3) for
// 1 <= r <= P - s; plus the top vertex D = (1+eta_3)/2, evaluated as
// (A + B + C)_triangle * D since the triangle's vertex modes sum to one.
// Coefficients are grouped by triangle mode (r fastest), D last.  Points: Q
// GLL points in eta_1, Q-1 Radau points of (1-x) in eta_2 and Q-1 of (1-x)^2
// in eta_3, q = i + Q (j + (Q-1) k).
//
// So a tetrahedron is Q-1 triangle expansions, one per eta_3 point k, whose
// coefficients w_t(k) = sum_r c_{s_t,r}(eta_3k) u_{t,r} come from an eta_3
// stage.  A thread owns the eta_1 row (j, k) of one tetrahedron: after the
// eta_3 stage (threads over (k, t) pairs), the triangle stages run as in
// tri.hip with the eta_1 tables as scalar operands; the transposed stages
// mirror them.  Helmholtz carries dw/deta_3 through the triangle stage too,
// for the third collapsed derivative.  Factors per point (built at space
// creation): w detJ, then the 6 entries of w detJ kappa M G M^T with M the
// collapsed chain rule d eta / d xi.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "tables.h"

namespace nk {

constexpr int kTet = 0, kPrism = 1, kPyr = 2;

template <int P, int SH>
struct TetShape {
  static constexpr int N = P + 1, Q = P + 2;
  static constexpr int Q2 = SH == kPyr ? Q : Q - 1;      // points in eta_2
  static constexpr int Q3 = SH == kPrism ? Q : Q - 1;    // points in the third direction
  static constexpr int NS = Q2 * Q3, NPT = Q * NS;
  // modes of the lower part: triangle modes, or the pyramid's base modes
  static constexpr int NMT = SH == kPyr ? N * N : N * (N + 1) / 2;
  static constexpr int NM3 = SH == kTet     ? N * (N + 1) * (N + 2) / 6
                             : SH == kPrism ? NMT * N
                                            : N * (N + 1) * (2 * N + 1) / 6;
  static constexpr bool APEX = SH != kPrism;   // a top vertex riding on the lower vertices
  // columns of the third-direction table.  A tetrahedron or pyramid mode's
  // third-direction factor depends only on the degree s >= 1 of its lower
  // mode and on r (0 <= r <= P - s), so the table holds one column per (s, r)
  // pair, s slow, then the top vertex; a prism's depends on r only
  static constexpr int NC = SH == kPrism ? N : P * (P + 1) / 2 + 1;
  // columns of the eta_2 table: one per lower mode, or one per 1-D mode q
  // for pyramids (phi_q(eta_2) depends on q only)
  static constexpr int NB = SH == kPyr ? N : NMT;
  static constexpr int bcol(int t) { return SH == kPyr ? t % N : t; }
  // LDS row strides (in scalars), odd so that distinct rows fall into
  // distinct banks
  static constexpr int TS = NB | 1, CS = NC | 1;
  // LDS tables B2, C3, then dB2, dC3 for Helmholtz only (the other
  // operators read no derivatives)
  static constexpr int ntab(int op) {
    return (op == OP_HELM || op == OP_HELM_ASM ? 2 : 1) * (Q2 * TS + Q3 * CS);
  }
  // vertex modes of the lower part (the apex rides on them)
  static constexpr bool lower_vertex(int t) {
    return SH == kPyr ? (t == 0 || t == P || t == P * N || t == P * N + P)
                      : (t == 0 || t == P || t == NMT - P);
  }
  static constexpr int NITAB = 3 * NMT + 1 + NM3;               // toff3, tp, mt, tcol
  // Per-element LDS of operator OP, in scalars: the coefficients u (not for
  // IProductWRTBase), w, w' (Helmholtz only), then the transposed eta_1
  // buffer [NS][N] (one of SA, SB, SC at a time).  BwdTrans stages its point
  // rows [NS][Q | 1] over u and w, which are dead once the eta_2 stage has
  // read them: the smaller slot lets half as many blocks again share a CU
  static constexpr int RS = Q | 1;
  static constexpr int u_off(int) { return 0; }
  static constexpr int w_off(int op) { return op == OP_IPROD ? 0 : NM3; }
  static constexpr int w3_off(int op) { return w_off(op) + Q3 * NMT; }
  static constexpr int ss_off(int op) {
    return op == OP_BWD ? 0 : w3_off(op) + (op == OP_HELM || op == OP_HELM_ASM ? Q3 * NMT : 0);
  }
  static constexpr int slot(int op) {
    return op == OP_BWD ? (w3_off(op) > NS * RS ? w3_off(op) : NS * RS) : ss_off(op) + NS * N;
  }
  // elements that fit in ~150 KB of LDS beside the tables
  template <typename T>
  static constexpr int by_lds(int op) {
    return (int)((150000 / sizeof(T) - ntab(op)) / slot(op));
  }
  // Wavefront-aligned elements: when an element's NS rows fit in one
  // wavefront, each wavefront holds EPW whole elements (lanes past EPW NS
  // idle) and every exchange between an element's threads stays inside its
  // wavefront, so the stages need no block barriers.  Used where at most 8
  // of 64 lanes idle: measured on MI355X, prisms and pyramids at P = 4, 6
  // (60 and 56 busy lanes) gain 2-10%, tetrahedra at P = 4, 6 (50 and 49)
  // lose 9% against the packed block layout.
  static constexpr int EPW = NS <= 64 ? 64 / NS : 0;
  template <typename T>
  static constexpr bool wave(int op) {
    return EPW > 0 && EPW * NS >= 56 && by_lds<T>(op) >= EPW;
  }
  // elements per block: up to 256 threads (four wavefronts of EPW elements
  // when wavefront-aligned), within the LDS budget
  template <typename T>
  static constexpr int epb(int op) {
    if (wave<T>(op)) {
      const int nw = by_lds<T>(op) / (EPW > 0 ? EPW : 1);
      return (nw < 4 ? nw : 4) * EPW;
    }
    const int by_threads = 256 / NS > 0 ? 256 / NS : 1;
    const int e = by_threads < by_lds<T>(op) ? by_threads : by_lds<T>(op);
    return e > 0 ? e : 1;
  }
  template <typename T>
  static constexpr int threads(int op) {
    return wave<T>(op) ? epb<T>(op) / (EPW > 0 ? EPW : 1) * 64 : (epb<T>(op) * NS + 63) / 64 * 64;
  }
  static constexpr int cnt(int p) { return SH == kPyr ? N : (p == 0 ? P + 1 : (p == P ? P : P - p)); }
  static constexpr int off(int p) {
    int o = 0;
    for (int k = 0; k < p; ++k) o += cnt(k);
    return o;
  }
};

// Device tables of order P (scalars of type T): B2 [Q2][NB], dB2 [Q2][NB] at
// the eta_2 points (NB = NMT lower modes, or P+1 for pyramids); C3 [Q3][NC],
// dC3 [Q3][NC] at the third-direction points (one column per (degree, r)
// pair and the top vertex for tetrahedra and pyramids, P+1 for prisms).
// Integer maps: toff3 [NMT+1] (first coefficient of each lower mode), tp
// [NMT] (eta_1 index p of each lower mode), mt [NM3] (lower mode of each
// coefficient, -1 for the top vertex), tcol [NMT] (first C3 column of each
// lower mode).
struct TetTables {
  const void* tab = nullptr;
  const int* itab = nullptr;
};

template <typename T>
static TetTables tet_tables(int P, int sh) {
  static std::mutex mu;
  static std::unordered_map<long, TetTables> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return {};
  const long key = (dev * 64L + P) * 4 + sh;   // sh < 4
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  const int N = P + 1, Q = P + 2, Q2 = sh == kPyr ? Q : Q - 1, Q3 = sh == kPrism ? Q : Q - 1;
  const int NMT = sh == kPyr ? N * N : N * (N + 1) / 2;
  const int NM3 = sh == kTet ? N * (N + 1) * (N + 2) / 6 : sh == kPrism ? NMT * N : N * (N + 1) * (2 * N + 1) / 6;
  std::vector<double> e1(Q), w1(Q), e2(Q2), w2(Q2), e3(Q3), w3(Q3);
  if (sh == kTet) {
    tet_points(Q, e1.data(), w1.data(), e2.data(), w2.data(), e3.data(), w3.data());
  } else if (sh == kPrism) {
    tri_points(Q, e1.data(), w1.data(), e2.data(), w2.data());
    gll_points(Q, e3.data(), w3.data());
  } else {
    gll_points(Q, e2.data(), w2.data());
    radau_points(Q3, 2, e3.data(), w3.data());
  }
  const int NC = sh == kPrism ? N : P * (P + 1) / 2 + 1;
  const int NB = sh == kPyr ? N : NMT;
  std::vector<double> B2(Q2 * NB), dB2(Q2 * NB), C3(Q3 * NC), dC3(Q3 * NC);
  if (sh == kPyr)   // base mode (p, q) = p N + q: phi_q(eta_2), one column per q
    modified_basis(P, Q, e2.data(), B2.data(), dB2.data());
  else
    tri_btable(P, Q2, e2.data(), B2.data(), dB2.data());
  // per-mode third-direction factors [Q3][NM3] (prisms: phi_r(xi_3), [Q3][N])
  std::vector<double> F3(Q3 * (sh == kPrism ? N : NM3)), dF3(F3.size());
  if (sh == kTet)
    tet_ctable(P, Q2, e3.data(), F3.data(), dF3.data());
  else if (sh == kPrism)
    modified_basis(P, Q, e3.data(), F3.data(), dF3.data());
  else
    pyr_ctable(P, Q3, e3.data(), F3.data(), dF3.data());
  // integer maps, and the columns (s, r) -> sum_{s' < s} (P - s' + 1) + r of
  // the compressed third-direction table (the top vertex last)
  std::vector<int> it_(3 * NMT + 1 + NM3);
  auto coff = [P](int s_) { return (s_ - 1) * (P + 1) - (s_ - 1) * s_ / 2; };
  int t = 0, m = 0;
  for (int p = 0; p <= P; ++p) {
    const int nq = sh == kPyr ? N : (p == 0 ? P + 1 : (p == P ? P : P - p));
    for (int q = 0; q < nq; ++q, ++t) {
      it_[t] = m;                 // toff3
      it_[NMT + 1 + t] = p;       // tp
      const int deg = sh == kTet     ? tri_mode_degree(P, p, q)
                      : sh == kPrism ? 1
                                     : std::max(mod_degree(P, p), mod_degree(P, q));
      const int nr = sh == kPrism ? N : P - deg + 1;
      const int c0 = sh == kPrism ? 0 : coff(deg);
      if (deg < 1 || deg > P || (sh != kPrism && c0 + nr > NC - 1)) return {};
      it_[2 * NMT + 1 + NM3 + t] = c0;   // tcol
      for (int r = 0; r < nr; ++r, ++m) {
        it_[2 * NMT + 1 + m] = t;   // mt
        if (sh != kPrism) {
          for (int kk = 0; kk < Q3; ++kk) {
            C3[kk * NC + c0 + r] = F3[kk * NM3 + m];
            dC3[kk * NC + c0 + r] = dF3[kk * NM3 + m];
          }
        }
      }
    }
  }
  it_[NMT] = m;                   // end of the last group
  if (sh != kPrism) {
    it_[2 * NMT + 1 + m] = -1;    // m = NM3 - 1: the top vertex
    for (int kk = 0; kk < Q3; ++kk) {
      C3[kk * NC + NC - 1] = F3[kk * NM3 + m];
      dC3[kk * NC + NC - 1] = dF3[kk * NM3 + m];
    }
  } else {
    C3 = F3;
    dC3 = dF3;
  }
  std::vector<T> h;
  for (const auto* v : {&B2, &dB2, &C3, &dC3})
    for (double x : *v) h.push_back((T)x);
  TetTables out;
  T* d = nullptr;
  int* di = nullptr;
  if (hipMalloc((void**)&d, h.size() * sizeof(T)) != hipSuccess) return {};
  if (hipMalloc((void**)&di, it_.size() * sizeof(int)) != hipSuccess) {
    (void)hipFree(d);
    return {};
  }
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(di, it_.data(), it_.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    (void)hipFree(di);
    return {};
  }
  out.tab = d;
  out.itab = di;
  cache[key] = out;
  return out;
}

// Local Helmholtz with the factors of the next point in flight while the
// current point is computed.  The second factor set costs 14-30 VGPRs (FP64)
// and sometimes a wave per SIMD; measured per shape and order on MI355X, it
// loses for FP64 tetrahedra at P <= 4, prisms at P >= 8 and pyramids at
// P >= 6, for FP32 tetrahedra at P = 6 and pyramids at P >= 8, and for the
// assembled tetrahedron operator (one wave per SIMD fewer at P = 6); FP64 at
// P = 6 trades it for a fourth wave per SIMD instead (tet_min_waves).
template <typename T>
constexpr bool tet_helm_prefetch(int P, int SH, int OP) {
  if (OP != OP_HELM) return false;
  if (sizeof(T) == 8 && P == 6) return false;   // held to 128 VGPRs instead (below)
  if (sizeof(T) == 8)
    return !((SH == kTet && P <= 4) || (SH == kPrism && P >= 8) || (SH == kPyr && P >= 6));
  return !((SH == kTet && P == 6) || (SH == kPyr && P >= 8));
}

// FP64 Helmholtz at P = 6 asks the compiler for four waves per SIMD (at most
// 128 VGPRs, instead of 134-162 and three waves): measured 4-5% faster for
// tetrahedra and prisms (the compiler keeps 150-160 for the pyramid and the
// assembled tetrahedron operator, which are unchanged).  Elsewhere no target.
template <typename T>
constexpr int tet_min_waves(int P, int OP) {
  return sizeof(T) == 8 && P == 6 && (OP == OP_HELM || OP == OP_HELM_ASM) ? 4 : 1;
}

// Pyramids hold a row's N eta_2 factors in registers (measured on MI355X,
// FP64: BwdTrans 6-8% faster at P = 4, 6, 8, Helmholtz 2-3% at P = 6), except
// the local Helmholtz operator at P <= 4, where the extra registers cost it a
// wave per SIMD (10% slower at P = 4)
constexpr bool pyr_hold_b2(int P, int SH, int OP) { return SH == kPyr && !(OP == OP_HELM && P <= 4); }

template <typename T, int P, int SH, int OP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(tet_min_waves<T>(P, OP))))
    k_tet(const Tab<T, P + 1, P + 2> tb, const T* __restrict__ tab, const int* __restrict__ itab,
          const DevArgs<T> a) {
  using S = TetShape<P, SH>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, NS = S::NS, NPT = S::NPT;
  constexpr bool APEX = S::APEX, TRI = SH != kPyr;   // TRI: triangle lower part
  constexpr int NMT = S::NMT, NM3 = S::NM3, TS = S::TS, CS = S::CS, NC = S::NC, NB = S::NB;
  constexpr int EPB = S::template epb<T>(OP), SLOT = S::slot(OP);
  constexpr bool WAVE = S::template wave<T>(OP);         // elements never straddle a wavefront
  constexpr int EPW = S::EPW;
  constexpr bool ASM = OP == OP_HELM_ASM;                // gathered input, scattered output
  constexpr bool HELM = OP == OP_HELM || ASM;
  constexpr bool HPF = HELM && tet_helm_prefetch<T>(P, SH, OP);
  __shared__ T stab[S::ntab(OP)];
  __shared__ int sit[S::NITAB];
  __shared__ T smem[EPB * SLOT];
  __shared__ double sred[ASM ? 256 : 1];                 // per-thread energy parts
  constexpr int DT = Q2 * TS + Q3 * CS;                  // offset of dB2, dC3
  for (int k = threadIdx.x; k < Q2 * NB; k += blockDim.x) {
    const int r = k / NB, m = k - r * NB;
    stab[r * TS + m] = tab[k];
    if constexpr (HELM) stab[DT + r * TS + m] = tab[Q2 * NB + k];
  }
  for (int k = threadIdx.x; k < Q3 * NC; k += blockDim.x) {
    const int r = k / NC, m = k - r * NC;
    stab[Q2 * TS + r * CS + m] = tab[2 * Q2 * NB + k];
    if constexpr (HELM) stab[DT + Q2 * TS + r * CS + m] = tab[2 * Q2 * NB + Q3 * NC + k];
  }
  for (int k = threadIdx.x; k < S::NITAB; k += blockDim.x) sit[k] = itab[k];
  __syncthreads();
  const T* B2 = stab;
  const T* C3 = stab + Q2 * TS;
  const T* dB2 = HELM ? stab + DT : B2;             // read by Helmholtz only
  const T* dC3 = HELM ? dB2 + Q2 * TS : C3;
  const int* toff3 = sit;
  const int* tp = sit + NMT + 1;
  const int* mt = tp + NMT;
  const int* tcol = mt + NM3;                       // first C3 column of each lower mode
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // element slot of this thread and its row lane t = j + Q2 k; threads past
  // the slots (past EPW NS lanes of a wavefront, or past EPB NS threads) only
  // synchronise, reading their wavefront's first slot
  const int slot0 = WAVE ? wv * EPW + lane / NS : threadIdx.x / NS;
  const bool act = WAVE ? lane / NS < EPW : slot0 < EPB;
  const int slot = act ? slot0 : (WAVE ? wv * EPW : 0);
  const int t = WAVE ? lane % NS : threadIdx.x - slot0 * NS;
  const int j = act ? t % Q2 : 0, k = act ? t / Q2 : 0;
  T* U = smem + slot * SLOT + S::u_off(OP);         // [NM3] coefficients
  T* W = smem + slot * SLOT + S::w_off(OP);         // [Q3][NMT] w, later z
  T* W3 = smem + slot * SLOT + S::w3_off(OP);       // [Q3][NMT] dw/deta_3, later z'
  constexpr int SSO = S::ss_off(OP);                // offset of SS in a slot
  T* SS = smem + slot * SLOT + SSO;                 // [NS][N]; point staging [NS][RS]
  constexpr int RS = S::RS;                         // staged row stride (odd)
  const int64_t ngrp = (a.nelem + EPB - 1) / EPB;
  // synchronisation of the threads that exchange an element's data through
  // LDS: its wavefront (LDS operations of a wavefront complete in order, so
  // a compiler fence suffices), else the block
  auto esync = [] {
    if constexpr (WAVE) {
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
    } else {
      __syncthreads();
    }
  };
  // the element's coefficients, NL per thread (m = t + l NS), all requested
  // before any is used
  constexpr int NL = (NM3 + NS - 1) / NS;
  auto load_u = [&](int64_t eg, T (&r)[NL]) {
    int32_t gv[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int m = t + l * NS;
      r[l] = T(0);
      gv[l] = -1;
      if (act && eg < a.nelem && m < NM3) {
        if constexpr (ASM) {
          gv[l] = a.l2g[eg * NM3 + m];
          r[l] = a.in[l2g_dof(gv[l])];
        } else {
          r[l] = a.in[eg * NM3 + m];
        }
      }
    }
    if constexpr (ASM) {
#pragma unroll
      for (int l = 0; l < NL; ++l) r[l] = l2g_value(gv[l], r[l]);
    }
  };
  // BwdTrans requests the next group's coefficients while it computes the
  // current group (its loads are otherwise the one long wait per group)
  constexpr bool PREFETCH = OP == OP_BWD;
  T un[NL];
  if constexpr (PREFETCH) load_u(blockIdx.x * (int64_t)EPB + slot, un);
  for (int64_t g = blockIdx.x; g < ngrp; g += gridDim.x) {
    // a converged system skips its operator (one system per collapsed space)
    if (ASM && seg_converged(a.elem_seg, a.seg_done, g * EPB)) continue;
    const int64_t e = g * EPB + slot;
    const bool live = act && e < a.nelem;
    T SA[N], SB[N], SC[N];
#pragma unroll
    for (int p = 0; p < N; ++p) SA[p] = SB[p] = SC[p] = T(0);
    if constexpr (OP != OP_IPROD) {
      T uc[NL];
      if constexpr (PREFETCH) {
#pragma unroll
        for (int l = 0; l < NL; ++l) uc[l] = un[l];
        load_u((g + gridDim.x) * EPB + slot, un);
      } else {
        load_u(e, uc);
      }
      if (live) {
#pragma unroll
        for (int l = 0; l < NL; ++l)
          if (t + l * NS < NM3) U[t + l * NS] = uc[l];
      }
      esync();
      // eta_3 stage: w_t(k') (and dw/deta_3) for every (k', t) pair
      if (live) {
        for (int idx = t; idx < Q3 * NMT; idx += NS) {
          const int kk = idx / NMT, tt = idx - kk * NMT;
          const int o = toff3[tt], c = toff3[tt + 1] - o;
          const T* cr = C3 + kk * CS + tcol[tt];
          const T* dcr = dC3 + kk * CS + tcol[tt];
          T w = T(0), w3 = T(0);
          if constexpr (SH == kPrism) {
            // every triangle mode has all N factors: a fixed-length sum whose
            // LDS reads are issued together (measured 2-4% faster; unrolling
            // the variable-length sums of the other shapes with zero-weighted
            // padding did not pay)
#pragma unroll
            for (int r = 0; r < N; ++r) {
              w += cr[r] * U[o + r];
              if constexpr (HELM) w3 += dcr[r] * U[o + r];
            }
          } else {
            for (int r = 0; r < c; ++r) {
              w += cr[r] * U[o + r];
              if constexpr (HELM) w3 += dcr[r] * U[o + r];
            }
          }
          if constexpr (APEX) {
            if (S::lower_vertex(tt)) {   // the top vertex rides on the lower vertex modes
              w += C3[kk * CS + NC - 1] * U[NM3 - 1];
              if constexpr (HELM) w3 += dC3[kk * CS + NC - 1] * U[NM3 - 1];
            }
          }
          W[kk * NMT + tt] = w;
          if constexpr (HELM) W3[kk * NMT + tt] = w3;
        }
      }
      esync();
      // eta_2 stage of slice k, row j
      T V[N], dV[N], V3[N];
#pragma unroll
      for (int p = 0; p < N; ++p) V[p] = dV[p] = V3[p] = T(0);
      const T* w = W + k * NMT;
      const T* w3 = W3 + k * NMT;
      const T* b2 = B2 + j * TS;
      const T* db2 = dB2 + j * TS;
      // a pyramid row's eta_2 factors depend on q only: N values, held in
      // registers rather than re-read for every p behind the group fences
      constexpr bool HOLD = pyr_hold_b2(P, SH, OP);
      T hb[HOLD ? N : 1], hdb[HOLD && HELM ? N : 1];
      if constexpr (HOLD) {
#pragma unroll
        for (int q = 0; q < N; ++q) {
          hb[q] = b2[q];
          if constexpr (HELM) hdb[q] = db2[q];
        }
      }
#pragma unroll
      for (int p = 0; p < N; ++p) {
#pragma unroll
        for (int q = 0; q < S::cnt(p); ++q) {
          const int m = S::off(p) + q, mb = S::bcol(m);
          const T bq = HOLD ? hb[HOLD ? q : 0] : b2[mb];
          V[p] += bq * w[m];
          if constexpr (HELM) {
            dV[p] += (HOLD ? hdb[HOLD && HELM ? q : 0] : db2[mb]) * w[m];
            V3[p] += bq * w3[m];
          }
        }
        // finish one mode group before the next group's loads are issued
        if constexpr (HELM) {
          __asm__ volatile("" : "+v"(V[p]), "+v"(dV[p]), "+v"(V3[p])::"memory");
        } else {
          __asm__ volatile("" : "+v"(V[p])::"memory");
        }
      }
      if constexpr (TRI) {   // the collapsed triangle vertex C also multiplies a_P
        V[P] += b2[P] * w[P];
        if constexpr (HELM) {
          dV[P] += db2[P] * w[P];
          V3[P] += b2[P] * w3[P];
        }
      }
      if constexpr (OP == OP_BWD) {
        // rows staged in LDS (row stride RS) over u and w, once every thread
        // of the element has read them; then the block's contiguous run of
        // point values leaves in one coalesced sweep
        esync();
        {
          // eta_1 stage in even-odd point pairs (the GLL points are symmetric)
          T ve[EO<N>::KE], vo[EO<N>::KO];
          eo_split<T, N>(V, ve, vo);
#pragma unroll 1
          for (int h = 0; h < Q / 2; ++h) {
            T lo, hi;
            eo_val(tb, h, ve, vo, lo, hi);
            if (act) {
              SS[t * RS + h] = lo;
              SS[t * RS + Q - 1 - h] = hi;
            }
          }
          if constexpr (Q & 1) {
            const T mid = eo_mid_val(tb, ve);
            if (act) SS[t * RS + Q / 2] = mid;
          }
        }
        esync();
        // the block's (or, wavefront-aligned, the wavefront's) elements are
        // consecutive, so their point values leave as one contiguous run
        const int s0 = WAVE ? wv * EPW : 0, sn = WAVE ? EPW : EPB;
        const int64_t e0 = g * EPB + s0;
        const int ne = a.nelem - e0 < sn ? (int)(a.nelem - e0) : sn;
        const int i0 = WAVE ? lane : threadIdx.x, di = WAVE ? 64 : blockDim.x;
        for (int idx = i0; idx < ne * NPT; idx += di) {
          const int sl = idx / NPT, q = idx - sl * NPT, row = q / Q;
          a.out[e0 * NPT + idx] = smem[(s0 + sl) * SLOT + SSO + row * RS + (q - row * Q)];
        }
        esync();
        continue;
      } else {
        const T lam = (T)(a.lam ? a.lam[live ? e : 0] : a.lam0);
        const T* f = a.fac + (live ? e : 0) * (int64_t)(7 * NPT) + t;
        // eta_1 stage, the 7 factors and the transposed eta_1 stage, point by
        // point (the paired even-odd form costs these register-bound kernels
        // up to 80 VGPRs); f points into element 0 for threads without a live
        // element, so every load is in bounds (their results are never used)
        plain_helm_row<T, N, Q, (HPF ? 2 : 1)>(
            tb, lam, V, dV, V3,
            [&](int i, T (&fv)[kNF3]) {
#pragma unroll
              for (int c = 0; c < kNF3; ++c) fv[c] = f[(c * Q + i) * NS];
            },
            SA, SB, SC);
      }
    } else {   // IProductWRTBase: point values times w detJ, read by rows
               // straight into registers (staging them through LDS measured
               // slower: its barriers serialise the loads behind the arithmetic)
      const T* x = a.in + (live ? e : 0) * (int64_t)NPT + Q * t;
      const T* f = a.fac + (live ? e : 0) * (int64_t)(7 * NPT) + t;
      // the row's Q values and weights are all requested before the first use
      T xv[Q], wv[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        xv[i] = live ? x[i] : T(0);
        wv[i] = live ? f[i * NS] : T(0);
      }
      T se[EO<N>::KE], so[EO<N>::KO];
      zero(se);
      zero(so);
#pragma unroll
      for (int h = 0; h < Q / 2; ++h) {
        const T ml = wv[h] * xv[h], mh = wv[Q - 1 - h] * xv[Q - 1 - h];
        eo_acc(tb, h, ml + mh, ml - mh, se, so);
      }
      if constexpr (Q & 1) eo_acc_mid(tb, wv[Q / 2] * xv[Q / 2], se);
      eo_join<T, N>(se, so, SA);
    }
    // transposed eta_2 stage, z_t(k') and z'_t(k') for every (k', t) pair,
    // from the transposed eta_1 results SA (with B2), SB (with dB2) and SC
    // (with B2, into z'), which pass through one LDS buffer in turn so that a
    // tetrahedron holds a third of them at a time
    auto tpass = [&](const T (&R)[N], const T* tab2, T* dst, bool accumulate) {
      if (act) {
#pragma unroll
        for (int p = 0; p < N; ++p) SS[t * N + p] = R[p];
      }
      esync();
      if (live) {
        for (int idx = t; idx < Q3 * NMT; idx += NS) {
          const int kk = idx / NMT, tt = idx - kk * NMT, p = tp[tt], tb_ = S::bcol(tt);
          T z = accumulate ? dst[kk * NMT + tt] : T(0);
#pragma unroll
          for (int jj = 0; jj < Q2; ++jj) z += tab2[jj * TS + tb_] * SS[(jj + Q2 * kk) * N + p];
          if (TRI && tt == P) {   // the collapsed triangle vertex C: its a_P part
#pragma unroll
            for (int jj = 0; jj < Q2; ++jj) z += tab2[jj * TS + P] * SS[(jj + Q2 * kk) * N + P];
          }
          dst[kk * NMT + tt] = z;
        }
      }
      esync();
    };
    tpass(SA, B2, W, false);
    if constexpr (HELM) {
      tpass(SB, dB2, W, true);
      tpass(SC, B2, W3, false);
    }
    // transposed eta_3 stage: one output coefficient per iteration
    double dp = 0.0;   // this thread's part of x_e . (H_e x_e)
    if (live) {
      for (int m = t; m < NM3; m += NS) {
        const int tt = mt[m];
        T y = T(0);
        if (!APEX || tt >= 0) {
          const int cm = tcol[tt] + (m - toff3[tt]);
#pragma unroll
          for (int kk = 0; kk < Q3; ++kk) {
            y += C3[kk * CS + cm] * W[kk * NMT + tt];
            if constexpr (HELM) y += dC3[kk * CS + cm] * W3[kk * NMT + tt];
          }
        } else {   // top vertex
#pragma unroll
          for (int kk = 0; kk < Q3; ++kk) {
            const T* zr = W + kk * NMT;
            T zs = zr[0] + zr[P] + (TRI ? zr[NMT - P] : zr[P * N] + zr[P * N + P]);
            y += C3[kk * CS + NC - 1] * zs;
            if constexpr (HELM) {
              const T* z3r = W3 + kk * NMT;
              zs = z3r[0] + z3r[P] + (TRI ? z3r[NMT - P] : z3r[P * N] + z3r[P * N + P]);
              y += dC3[kk * CS + NC - 1] * zs;
            }
          }
        }
        if constexpr (ASM) {
          dp += (double)U[m] * (double)y;
          const int32_t gv = a.l2g[e * NM3 + m];
          if (gv >= 0) atomic_add(a.out + l2g_dof(gv), l2g_sign(gv, y));
        } else {
          a.out[e * NM3 + m] = y;
        }
      }
    }
    if constexpr (ASM) {   // per-element energy for the CG step length
      if (act) sred[slot * NS + t] = dp;
      esync();
      if (live && t == 0 && a.dots) {
        double s_ = 0.0;
        for (int k2 = 0; k2 < NS; ++k2) s_ += sred[slot * NS + k2];
        add_dot(a.dots, a.dslot, e, s_);
      }
    }
    esync();
  }
}

// The assembled operator of every collapsed shape.
template <typename T, int P, int SH>
static const void* asm_kernel() {
  return (const void*)k_tet<T, P, SH, OP_HELM_ASM>;
}

template <typename T, int P, int SH>
static int64_t tet_grid(int op) {
  static std::unordered_map<int, int64_t> cached;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0, cus = 0, nb = 0;
  (void)hipGetDevice(&dev);
  const int key = dev * 4 + (op == OP_BWD ? 0 : op == OP_IPROD ? 1 : op == OP_HELM ? 2 : 3);
  auto it = cached.find(key);
  if (it != cached.end()) return it->second;
  using S = TetShape<P, SH>;
  const int threads = op == OP_BWD     ? S::template threads<T>(OP_BWD)
                      : op == OP_IPROD ? S::template threads<T>(OP_IPROD)
                      : op == OP_HELM  ? S::template threads<T>(OP_HELM)
                                       : S::template threads<T>(OP_HELM_ASM);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = op == OP_BWD     ? (const void*)k_tet<T, P, SH, OP_BWD>
                   : op == OP_IPROD ? (const void*)k_tet<T, P, SH, OP_IPROD>
                   : op == OP_HELM  ? (const void*)k_tet<T, P, SH, OP_HELM>
                                    : asm_kernel<T, P, SH>();
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, threads, 0);
  const int64_t grid = (int64_t)(cus > 0 ? cus : 256) * (nb > 0 ? nb : 1) * 4;
  cached[key] = grid;
  return grid;
}

template <typename T, int P, int SH, int OP>
static hipError_t run_tet_op(const OpArgs& a, const TetTables& tt) {
  using S = TetShape<P, SH>;
  constexpr int EPB = S::template epb<T>(OP);
  constexpr int threads = S::template threads<T>(OP);
  static_assert(threads <= 256, "block size");
  const int64_t ngrp = (a.nelem + EPB - 1) / EPB;
  const int64_t gmax = tet_grid<T, P, SH>(OP);
  const int64_t nb = ngrp < gmax ? ngrp : gmax;
  hipLaunchKernelGGL((k_tet<T, P, SH, OP>), dim3((unsigned)nb), dim3(threads), 0, a.stream,
                     host_tab<T, P + 1, P + 2>(), static_cast<const T*>(tt.tab), tt.itab,
                     dev_args<T>(a));
  return hipGetLastError();
}

template <typename T, int P, int SH>
static hipError_t run_tet(const OpArgs& a) {
  const TetTables tt = tet_tables<T>(P, SH);
  if (!tt.tab) return hipErrorOutOfMemory;
  switch (a.op) {
    case OP_BWD: return run_tet_op<T, P, SH, OP_BWD>(a, tt);
    case OP_IPROD: return run_tet_op<T, P, SH, OP_IPROD>(a, tt);
    case OP_HELM: return run_tet_op<T, P, SH, OP_HELM>(a, tt);
    case OP_HELM_ASM: return run_tet_op<T, P, SH, OP_HELM_ASM>(a, tt);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int SH>
static hipError_t run_tet_p(nk_dtype t, const OpArgs& a) {
  return t == NK_F64 ? run_tet<double, P, SH>(a) : run_tet<float, P, SH>(a);
}

template <int SH>
static hipError_t launch_col(nk_dtype t, const OpArgs& a) {
  if (a.nelem == 0) return hipSuccess;
  switch (a.P) {
    case 1: return run_tet_p<1, SH>(t, a);
    case 2: return run_tet_p<2, SH>(t, a);
    case 3: return run_tet_p<3, SH>(t, a);
    case 4: return run_tet_p<4, SH>(t, a);
    case 5: return run_tet_p<5, SH>(t, a);
    case 6: return run_tet_p<6, SH>(t, a);
    case 7: return run_tet_p<7, SH>(t, a);
    case 8: return run_tet_p<8, SH>(t, a);
    case 9: return run_tet_p<9, SH>(t, a);
    case 10: return run_tet_p<10, SH>(t, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_tet(nk_dtype t, const OpArgs& a) { return launch_col<kTet>(t, a); }
hipError_t launch_prism(nk_dtype t, const OpArgs& a) { return launch_col<kPrism>(t, a); }
hipError_t launch_pyr(nk_dtype t, const OpArgs& a) { return launch_col<kPyr>(t, a); }

// Diagonal of the tetrahedron, prism or pyramid Helmholtz operator, thread
// per (element, mode), scatter-added into the padded global diagonal (Dirichlet modes
// skipped): diag H_e[m] = sum_points (lambda f0 phi_m^2 + d^T G' d) with d the
// three collapsed derivatives of phi_m and G' the 6 stored factors.  A mode
// is T_t(eta_1, eta_2) c(eta_3) (the collapsed triangle vertex C as
// (a_0 + a_P) times its eta_2 factor), the top vertex c(eta_3) alone.
template <int P, int SH>
__global__ void __launch_bounds__(256)
    k_diag_col(const Tab<double, P + 1, P + 2> tb, const double* __restrict__ tab,
               const int* __restrict__ itab, int64_t nelem, const double* __restrict__ fac,
               const double* __restrict__ lam, double lam0, const int32_t* __restrict__ l2g,
               double* __restrict__ diag) {
  using S = TetShape<P, SH>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, Q3 = S::Q3, NS = S::NS, NPT = S::NPT;
  constexpr int NMT = S::NMT, NM3 = S::NM3, NC = S::NC, NB = S::NB;
  constexpr bool TRI = SH != kPyr;   // triangle lower part (else the pyramid's base)
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * NM3) return;
  const int64_t e = id / NM3;
  const int m = (int)(id - e * NM3);
  const int32_t g = l2g[id];
  if (g < 0) return;  // Dirichlet: row replaced by the identity
  const double* B2 = tab;
  const double* dB2 = tab + Q2 * NB;
  const double* C3 = tab + 2 * Q2 * NB;
  const double* dC3 = C3 + Q3 * NC;
  const int tt = itab[2 * NMT + 1 + m];       // lower mode, -1 for the top vertex
  const int p = tt >= 0 ? itab[NMT + 1 + tt] : 0;
  // column of the compressed eta_3 table
  const int cm = tt >= 0 ? itab[2 * NMT + 1 + NM3 + tt] + (m - itab[tt]) : NC - 1;
  const double* f = fac + e * (int64_t)(7 * NPT);
  const double lm = lam ? lam[e] : lam0;
  double s = 0.0;
  for (int k = 0; k < Q3; ++k) {
    const double c = C3[k * NC + cm], dc = dC3[k * NC + cm];
    for (int j = 0; j < Q2; ++j) {
      double b = 1.0, db = 0.0;
      if (tt >= 0) {
        b = B2[j * NB + S::bcol(tt)];
        db = dB2[j * NB + S::bcol(tt)];
      }
      for (int i = 0; i < Q; ++i) {
        double av = 1.0, dav = 0.0;
        if (tt >= 0) {
          av = tb.B[i * N + p];
          dav = tb.D[i * N + p];
          if (TRI && tt == P) {   // collapsed triangle vertex
            av += tb.B[i * N + P];
            dav += tb.D[i * N + P];
          }
        }
        const double ph = av * b * c, d1 = dav * b * c, d2 = av * db * c, d3 = av * b * dc;
        const double* fp = f + (int64_t)i * NS + j + Q2 * k;
        const double f0 = fp[0], g11 = fp[NPT], g12 = fp[2 * NPT], g13 = fp[3 * NPT],
                     g22 = fp[4 * NPT], g23 = fp[5 * NPT], g33 = fp[6 * NPT];
        s += lm * f0 * ph * ph + g11 * d1 * d1 + g22 * d2 * d2 + g33 * d3 * d3 +
             2.0 * (g12 * d1 * d2 + g13 * d1 * d3 + g23 * d2 * d3);
      }
    }
  }
  unsafeAtomicAdd(diag + l2g_dof(g), s);
}

template <int P, int SH>
static hipError_t run_diag_col(int64_t nelem, const double* fac, const double* lam, double lam0,
                               const int32_t* l2g, double* diag, hipStream_t st) {
  const TetTables tt = tet_tables<double>(P, SH);
  if (!tt.tab) return hipErrorOutOfMemory;
  const int64_t tot = nelem * TetShape<P, SH>::NM3;
  hipLaunchKernelGGL((k_diag_col<P, SH>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     host_tab<double, P + 1, P + 2>(), static_cast<const double*>(tt.tab), tt.itab,
                     nelem, fac, lam, lam0, l2g, diag);
  return hipGetLastError();
}

template <int SH>
static hipError_t diag_col(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st) {
  if (nelem == 0) return hipSuccess;
  switch (P) {
    case 1: return run_diag_col<1, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 2: return run_diag_col<2, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 3: return run_diag_col<3, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 4: return run_diag_col<4, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 5: return run_diag_col<5, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 6: return run_diag_col<6, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 7: return run_diag_col<7, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 8: return run_diag_col<8, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 9: return run_diag_col<9, SH>(nelem, fac, lam, lam0, l2g, diag, st);
    case 10: return run_diag_col<10, SH>(nelem, fac, lam, lam0, l2g, diag, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_diag_tet(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st) {
  return diag_col<kTet>(P, nelem, fac, lam, lam0, l2g, diag, st);
}

hipError_t launch_diag_prism(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                             const int32_t* l2g, double* diag, hipStream_t st) {
  return diag_col<kPrism>(P, nelem, fac, lam, lam0, l2g, diag, st);
}

hipError_t launch_diag_pyr(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st) {
  return diag_col<kPyr>(P, nelem, fac, lam, lam0, l2g, diag, st);
}

// Factors of the collapsed tetrahedron, prism or pyramid at every point
// (thread per point): f0 = w |detJ| (tetrahedra, whose sorted vertex orders
// may be left-handed) or w detJ, f1..f6 = the same times kappa
// (M G M^T)_{11,12,13,22,23,33} with G = J^{-1} J^{-T} and M_ba = d eta_b /
// d xi_a.  Tetrahedron: w = w1_i (w2_j / 2) (w3_k / 4) (the Radau weights
// carry (1 - eta_2) and (1 - eta_3)^2); prism: w = w1_i (w2_j / 2) w3_k;
// pyramid: w = w1_i w2_j (w3_k / 4).  Layout [E][7][Q][NS]: for each factor
// and eta_1 index i, the rows j + Q2 k are contiguous, the order in which the
// operator's threads read them.
template <int SH>
__global__ void __launch_bounds__(256)
    k_geom_tet(int Q, int64_t nelem, const double* __restrict__ jac, const double* __restrict__ kappa,
               const double* __restrict__ pts, double* __restrict__ fac64, float* __restrict__ fac32,
               int* __restrict__ bad) {
  const int Q2 = SH == kPyr ? Q : Q - 1, Q3 = SH == kPrism ? Q : Q - 1, NS = Q2 * Q3, NP = Q * NS;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * NP) return;
  const int64_t e = id / NP;
  const int q = (int)(id - e * NP);
  const int i = q % Q, row = q / Q, j = row % Q2, k = row / Q2;
  const double e1 = pts[i], w1 = pts[Q + i];
  const double e2 = pts[2 * Q + j], w2 = pts[2 * Q + Q2 + j];
  const double e3 = pts[2 * Q + 2 * Q2 + k], w3 = pts[2 * Q + 2 * Q2 + Q3 + k];
  double J[3][3];
  for (int c = 0; c < 3; ++c)
    for (int b = 0; b < 3; ++b) J[c][b] = jac[((e * 3 + c) * 3 + b) * NP + q];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double id_ = 1.0 / det;
  double Ji[3][3];   // Ji[a][c] = d xi_a / d x_c
  Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id_;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id_;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id_;
  Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id_;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id_;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id_;
  Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id_;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id_;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id_;
  double G[3][3];
  for (int a_ = 0; a_ < 3; ++a_)
    for (int b = 0; b < 3; ++b)
      G[a_][b] = Ji[a_][0] * Ji[b][0] + Ji[a_][1] * Ji[b][1] + Ji[a_][2] * Ji[b][2];
  // M[b][a] = d eta_b / d xi_a of the collapsed map
  double M[3][3];
  if (SH == kTet) {
    const double g = 2.0 / ((1.0 - e2) * (1.0 - e3));
    const double Mt[3][3] = {{2.0 * g, (1.0 + e1) * g, (1.0 + e1) * g},
                             {0.0, 2.0 / (1.0 - e3), (1.0 + e2) / (1.0 - e3)},
                             {0.0, 0.0, 1.0}};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[r][c] = Mt[r][c];
  } else if (SH == kPrism) {   // eta_1 = 2 (1 + xi_1)/(1 - xi_2) - 1, eta_2 = xi_2, xi_3
    const double Mp[3][3] = {{2.0 / (1.0 - e2), (1.0 + e1) / (1.0 - e2), 0.0},
                             {0.0, 1.0, 0.0},
                             {0.0, 0.0, 1.0}};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[r][c] = Mp[r][c];
  } else {   // pyramid: eta_a = 2 (1 + xi_a)/(1 - xi_3) - 1 (a = 1, 2), eta_3 = xi_3
    const double g = 2.0 / (1.0 - e3);
    const double My[3][3] = {{g, 0.0, (1.0 + e1) / (1.0 - e3)},
                             {0.0, g, (1.0 + e2) / (1.0 - e3)},
                             {0.0, 0.0, 1.0}};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) M[r][c] = My[r][c];
  }
  double H[3][3];   // M G M^T
  for (int a_ = 0; a_ < 3; ++a_)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) s += M[a_][c] * G[c][d] * M[b][d];
      H[a_][b] = s;
    }
  const double kap = kappa ? kappa[e * NP + q] : 1.0;
  // tetrahedra may be left-handed (sorted vertex orders give det J < 0 in
  // half the elements of a mesh): the integrals take |det J|, and only a zero
  // or non-finite determinant is rejected
  const double adet = SH == kTet ? fabs(det) : det;
  if (!(adet > 0.0) || !(adet < 1e300) || !(kap > 0.0)) atomicOr(bad, 1);
  // the Radau weights carry (1 - eta_2) (tetrahedron, prism) and
  // (1 - eta_3)^2 (tetrahedron, pyramid)
  const double wj = w1 * (SH == kPyr ? 1.0 : 0.5) * w2 * (SH == kPrism ? 1.0 : 0.25) * w3 * adet;
  const double ck = wj * kap;
  const double f[7] = {wj, ck * H[0][0], ck * H[0][1], ck * H[0][2], ck * H[1][1], ck * H[1][2], ck * H[2][2]};
  for (int c = 0; c < 7; ++c) {
    const int64_t o = (e * 7 + c) * (int64_t)NP + (int64_t)i * NS + row;
    fac64[o] = f[c];
    fac32[o] = (float)f[c];
  }
}

hipError_t launch_geom_tet(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s) {
  const int64_t n = nelem * Q * (Q - 1) * (Q - 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geom_tet<kTet>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q, nelem,
                     jac, kappa, pts, fac64, fac32, bad);
  return hipGetLastError();
}

hipError_t launch_geom_prism(int Q, int64_t nelem, const double* jac, const double* kappa,
                             const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s) {
  const int64_t n = nelem * Q * (Q - 1) * Q;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geom_tet<kPrism>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q,
                     nelem, jac, kappa, pts, fac64, fac32, bad);
  return hipGetLastError();
}


hipError_t launch_geom_pyr(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s) {
  const int64_t n = nelem * Q * Q * (Q - 1);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_geom_tet<kPyr>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, Q, nelem,
                     jac, kappa, pts, fac64, fac32, bad);
  return hipGetLastError();
}

}  // namespace nk
