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
// Lanes own (triangle, eta_2 row) pairs, so the eta_1 stages, which use the
// same 1-D tables for every lane, run from registers with scalar table
// operands; only the eta_2 stages read per-lane table rows from LDS.  Factors
// per point (built at space creation): w detJ, then w detJ kappa (T^T G T)
// with T the Duffy chain rule d xi / d eta, so the kernel works in collapsed
// derivatives.
#include <mutex>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "tables.h"

namespace nk {

template <int P>
struct TriShape {
  static constexpr int N = P + 1, Q = P + 2, Q2 = Q - 1, NP = Q * Q2, NM = N * (N + 1) / 2;
  static constexpr int EPW = tri_epw(Q);        // triangles per wavefront
  static constexpr int LANES = EPW * Q2;        // lane = (triangle, eta_2 row)
  static constexpr int WPB = 4;                 // wavefronts per block
  // LDS strides (in scalars), odd so that the distinct addresses a wave
  // reads at once fall into distinct banks
  static constexpr int TS = NM | 1;             // eta_2 table row
  static constexpr int CS = NM | 1;             // one triangle's coefficients
  static constexpr int RS = Q | 1;              // one eta_2 row of point values
  // per-triangle staging: point values (BwdTrans out, IProductWRTBase in)
  // and the transposed eta_1 results SA (and SB for Helmholtz)
  static constexpr int xs(int op) {
    return (op == OP_BWD ? Q2 * RS
            : op == OP_IPROD ? (Q2 * RS > Q2 * N ? Q2 * RS : Q2 * N)
                             : 2 * Q2 * N) | 1;
  }
  static constexpr bool helm(int op) { return op == OP_HELM || op == OP_HELM_ASM; }
  static constexpr int ntab(int op) { return helm(op) ? 2 : 1; }   // B2 (, dB2)
  // a wavefront's LDS; BwdTrans stages its point values over the coefficients,
  // which are dead once its eta_2 stage has read them
  static constexpr int wave_lds(int op) {
    return op == OP_BWD ? EPW * (CS > xs(op) ? CS : xs(op)) : EPW * (CS + xs(op));
  }
  static constexpr int cnt(int p) { return p == 0 ? P + 1 : (p == P ? P : P - p); }
  static constexpr int off(int p) {
    int o = 0;
    for (int k = 0; k < p; ++k) o += cnt(k);
    return o;
  }
};

// Device table of order P: B2 [Q2][NM] and dB2 [Q2][NM], the eta_2 factor of
// every mode and its derivative at the Radau points.
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
  const int Q = P + 2, Q2 = Q - 1, NM = (P + 1) * (P + 2) / 2;
  std::vector<double> e1(Q), w1(Q), e2(Q2), w2(Q2), B2(Q2 * NM), dB2(Q2 * NM);
  tri_points(Q, e1.data(), w1.data(), e2.data(), w2.data());
  tri_btable(P, Q2, e2.data(), B2.data(), dB2.data());
  std::vector<T> h;
  for (double v : B2) h.push_back((T)v);
  for (double v : dB2) h.push_back((T)v);
  T* d = nullptr;
  if (hipMalloc((void**)&d, h.size() * sizeof(T)) != hipSuccess) return nullptr;
  if (hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(d);
    return nullptr;
  }
  cache[key] = d;
  return d;
}

// Per wavefront: groups of EPW consecutive triangles, lane (el, j) owning
// eta_2 row j of triangle el.  Stages per group:
//  1. the group's inputs (coefficients, or point values for IProductWRTBase;
//     one contiguous run through registers) -> LDS;
//  2. eta_2 stage: v_p(eta_2j) and dv_p/deta_2 for every p, from the LDS
//     table rows of j (registers V[N], dV[N]);
//  3. one loop over the eta_1 points i: the eta_1 stage (values and both
//     collapsed derivatives), the 4 pointwise factors, and the transposed
//     eta_1 stage accumulated into registers SA[N], SB[N]; the eta_1 tables
//     are the same for every lane, so they are scalar operands;
//  4. SA, SB -> LDS; transposed eta_2 stage with lane (el, t) forming the
//     modes t, t + Q2, ...; results staged in LDS and stored contiguously.
// Each wavefront works only in its own LDS region, so stages are separated
// by wavefront-level fences.
// FP64 Helmholtz at P = 6 fits four waves per SIMD (126 VGPRs, no spill)
// when asked for them, instead of 134 VGPRs and three.
template <typename T>
constexpr int tri_min_waves(int P, int OP) {
  return sizeof(T) == 8 && P == 6 && OP == OP_HELM ? 4 : 1;
}

template <typename T, int P, int OP>
__global__ void __launch_bounds__(TriShape<P>::WPB * 64) __attribute__((amdgpu_waves_per_eu(tri_min_waves<T>(P, OP))))
    k_tri(const Tab<T, P + 1, P + 2> tb, const T* __restrict__ tab, const DevArgs<T> a) {
  using S = TriShape<P>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, NP = S::NP, NM = S::NM, EPW = S::EPW;
  constexpr int LANES = S::LANES, XS = S::xs(OP), WAVE = S::wave_lds(OP);
  constexpr bool HELM = S::helm(OP);
  constexpr bool ASM = OP == OP_HELM_ASM;                 // gathered input, scattered output
  constexpr int NIN = OP == OP_IPROD ? NP : NM;          // inputs per triangle
  constexpr int KIN = (EPW * NIN + 63) / 64;             // inputs per lane per group
  __shared__ T stab[S::ntab(OP) * Q2 * S::TS];
  __shared__ T smem[S::WPB * WAVE];
  __shared__ double sdot[ASM ? S::WPB * 64 : 1];        // per-lane parts of x_e . (H_e x_e)
  for (int k = threadIdx.x; k < S::ntab(OP) * Q2 * NM; k += S::WPB * 64) {
    const int r = k / NM;
    stab[r * S::TS + (k - r * NM)] = tab[k];
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int el = lane / Q2, j = lane - el * Q2;
  const bool row = lane < LANES;
  const int ela = row ? el : 0;           // addressing: idle lanes use triangle 0
  T* Cw = smem + wave * WAVE;             // [EPW][CS] coefficients, later results
  T* Xw = Cw + (OP == OP_BWD ? 0 : EPW * S::CS);   // [EPW][XS] point values / SA, SB
  const T* B2 = stab + j * S::TS;
  const T* dB2 = stab + (Q2 + j) * S::TS;
  const int64_t ngrp = (a.nelem + EPW - 1) / EPW;
  const int64_t nwave = (int64_t)gridDim.x * S::WPB;
  const int64_t per = (ngrp + nwave - 1) / nwave;
  const int64_t g0 = ((int64_t)blockIdx.x * S::WPB + wave) * per;
  const int64_t g1 = g0 + per < ngrp ? g0 + per : ngrp;
  auto group_size = [&](int64_t g) {
    const int64_t left = a.nelem - g * EPW;
    return left < EPW ? (int)left : EPW;
  };
  T pre[KIN];
  auto load_in = [&](int64_t g) {
    const int lim = group_size(g) * NIN;
    const T* src = a.in + g * EPW * NIN;
#pragma unroll
    for (int r = 0; r < KIN; ++r) {
      const int k = lane + 64 * r;
      pre[r] = k < lim ? src[k] : T(0);
    }
  };
  // BwdTrans and IProductWRTBase request the next group's inputs before
  // computing the current one; Helmholtz loads its group at the start, since
  // its factor loads inside the point loop would wait for the prefetch anyway
  // (loads retire in order) and the prefetch registers cost occupancy.
  constexpr bool PREFETCH = !HELM;
  if (PREFETCH && g0 < g1) load_in(g0);
  for (int64_t g = g0; g < g1; ++g) {
    const int64_t e0 = g * EPW;
    const int ne = group_size(g);                       // live triangles
    const int64_t e = e0 + (el < ne ? el : 0);
    const bool live = row && el < ne;
    // a converged system skips its operator (one system per triangle space)
    if (ASM && seg_converged(a.elem_seg, a.seg_done, e0)) continue;
    if constexpr (PREFETCH) {
#pragma unroll
      for (int r = 0; r < KIN; ++r) {
        const int k = lane + 64 * r;
        if (k < ne * NIN) {
          const int ee = k / NIN, q = k - ee * NIN;
          if constexpr (OP == OP_IPROD) {
            const int jj = q / Q;
            Xw[ee * XS + jj * S::RS + (q - jj * Q)] = pre[r];
          } else {
            Cw[ee * S::CS + q] = pre[r];
          }
        }
      }
      slot_sync<64>();
      if (g + 1 < g1) load_in(g + 1);
    } else {
      // the group's coefficients, all requested before any is stored
      constexpr int KM = (EPW * NM + 63) / 64;
      T v[KM];
      int32_t gv[KM];
#pragma unroll
      for (int r = 0; r < KM; ++r) {
        const int k = lane + 64 * r;
        v[r] = T(0);
        gv[r] = -1;
        if (k < ne * NM) {
          if constexpr (ASM) {
            gv[r] = a.l2g[e0 * NM + k];
            v[r] = a.in[l2g_dof(gv[r])];
          } else {
            v[r] = a.in[e0 * NM + k];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < KM; ++r) {
        const int k = lane + 64 * r;
        if (k < ne * NM) {
          const int ee = k / NM;
          Cw[ee * S::CS + (k - ee * NM)] = ASM ? l2g_value(gv[r], v[r]) : v[r];
        }
      }
      slot_sync<64>();
    }
    T SA[N], SB[N];
#pragma unroll
    for (int p = 0; p < N; ++p) SA[p] = SB[p] = T(0);
    if constexpr (OP == OP_BWD || HELM) {
      T V[N], dV[N];
#pragma unroll
      for (int p = 0; p < N; ++p) V[p] = dV[p] = T(0);
      const T* c = Cw + ela * S::CS;
#pragma unroll
      for (int p = 0; p < N; ++p) {
#pragma unroll
        for (int q = 0; q < S::cnt(p); ++q) {
          const T cm = c[S::off(p) + q];
          V[p] += B2[S::off(p) + q] * cm;
          if constexpr (HELM) dV[p] += dB2[S::off(p) + q] * cm;
        }
        // finish one mode group before the next group's loads are issued, so
        // only one group's table entries are held in registers
        if constexpr (HELM) {
          __asm__ volatile("" : "+v"(V[p]), "+v"(dV[p])::"memory");
        } else {
          __asm__ volatile("" : "+v"(V[p])::"memory");
        }
      }
      {   // the collapsed vertex (mode P of group p = 0) also multiplies a_P
        const T cm = c[P];
        V[P] += B2[P] * cm;
        if constexpr (HELM) dV[P] += dB2[P] * cm;
      }
      if constexpr (OP == OP_BWD) {
        slot_sync<64>();   // every lane has read the coefficients under Xw
        T* x = Xw + ela * XS + j * S::RS;
        // eta_1 stage in even-odd point pairs (the GLL points are symmetric)
        T ve[EO<N>::KE], vo[EO<N>::KO];
        eo_split<T, N>(V, ve, vo);
#pragma unroll 1
        for (int h = 0; h < Q / 2; ++h) {
          T lo, hi;
          eo_val(tb, h, ve, vo, lo, hi);
          if (row) {
            x[h] = lo;
            x[Q - 1 - h] = hi;
          }
        }
        if constexpr (Q & 1) {
          const T mid = eo_mid_val(tb, ve);
          if (row) x[Q / 2] = mid;
        }
        slot_sync<64>();
        for (int k = lane; k < ne * NP; k += 64) {
          const int ee = k / NP, q = k - ee * NP, jj = q / Q;
          a.out[e0 * NP + k] = Xw[ee * XS + jj * S::RS + (q - jj * Q)];
        }
        slot_sync<64>();
        continue;
      } else {
        const T lam = (T)(a.lam ? a.lam[e] : a.lam0);
        const T* f = a.fac + g * (int64_t)(4 * Q * LANES) + lane;
#pragma unroll 1
        for (int i = 0; i < Q; ++i) {
          T fa[4] = {T(0), T(0), T(0), T(0)};
          if (row) {
#pragma unroll
            for (int k = 0; k < 4; ++k) fa[k] = f[(k * Q + i) * LANES];
          }
          T u = T(0), u1 = T(0), u2 = T(0);
#pragma unroll
          for (int p = 0; p < N; ++p) {
            u += tb.B[i * N + p] * V[p];
            u1 += tb.D[i * N + p] * V[p];
            u2 += tb.B[i * N + p] * dV[p];
          }
          const T mq = lam * fa[0] * u;
          const T g1_ = fa[1] * u1 + fa[2] * u2;
          const T g2_ = fa[2] * u1 + fa[3] * u2;
#pragma unroll
          for (int p = 0; p < N; ++p) {
            SA[p] += tb.B[i * N + p] * mq + tb.D[i * N + p] * g1_;
            SB[p] += tb.B[i * N + p] * g2_;
          }
        }
      }
    } else {   // IProductWRTBase: staged point values times w detJ
      const T* x = Xw + ela * XS + j * S::RS;
      const T* f = a.fac + g * (int64_t)(4 * Q * LANES) + lane;
      // transposed eta_1 stage in even-odd point pairs
      T se[EO<N>::KE], so[EO<N>::KO];
      zero(se);
      zero(so);
#pragma unroll 1
      for (int h = 0; h < Q / 2; ++h) {
        const T fl = row ? f[h * LANES] : T(0), fh = row ? f[(Q - 1 - h) * LANES] : T(0);
        const T ml = row ? fl * x[h] : T(0), mh = row ? fh * x[Q - 1 - h] : T(0);
        eo_acc(tb, h, ml + mh, ml - mh, se, so);
      }
      if constexpr (Q & 1) {
        const T fm = row ? f[(Q / 2) * LANES] : T(0);
        eo_acc_mid(tb, row ? fm * x[Q / 2] : T(0), se);
      }
      eo_join<T, N>(se, so, SA);
      slot_sync<64>();
    }
    // transposed eta_2 stage
    {
      T* s = Xw + ela * XS;
      if (row) {
#pragma unroll
        for (int p = 0; p < N; ++p) {
          s[j * N + p] = SA[p];
          if constexpr (HELM) s[(Q2 + j) * N + p] = SB[p];
        }
      }
      slot_sync<64>();
      double dp = 0.0;
      if (live) {
        const T* sa = Xw + el * XS;
        for (int mm = j; mm < NM; mm += Q2) {
          int p = 0;
#pragma unroll
          for (int k = 1; k < N; ++k) p += (mm >= S::off(k)) ? 1 : 0;
          T y = T(0);
#pragma unroll
          for (int jj = 0; jj < Q2; ++jj) {
            y += stab[jj * S::TS + mm] * sa[jj * N + p];
            if constexpr (HELM) y += stab[(Q2 + jj) * S::TS + mm] * sa[(Q2 + jj) * N + p];
          }
          if (mm == P) {   // the collapsed vertex: its a_P part
#pragma unroll
            for (int jj = 0; jj < Q2; ++jj) {
              y += stab[jj * S::TS + P] * sa[jj * N + P];
              if constexpr (HELM) y += stab[(Q2 + jj) * S::TS + P] * sa[(Q2 + jj) * N + P];
            }
          }
          if constexpr (ASM) dp += (double)Cw[el * S::CS + mm] * (double)y;   // x_m y_m
          Cw[el * S::CS + mm] = y;
        }
      }
      if constexpr (ASM) sdot[wave * 64 + lane] = dp;
      slot_sync<64>();
      if constexpr (ASM) {
        if (live && j == 0 && a.dots) {
          double s = 0.0;
#pragma unroll
          for (int jj = 0; jj < Q2; ++jj) s += sdot[wave * 64 + lane + jj];
          add_dot(a.dots, a.dslot, e, s);
        }
      }
      for (int k = lane; k < ne * NM; k += 64) {
        const int ee = k / NM;
        const T y = Cw[ee * S::CS + (k - ee * NM)];
        if constexpr (ASM) {
          const int32_t gv = a.l2g[e0 * NM + k];
          if (gv >= 0) atomic_add(a.out + l2g_dof(gv), l2g_sign(gv, y));
        } else {
          a.out[e0 * NM + k] = y;
        }
      }
      slot_sync<64>();
    }
  }
}

// Persistent grid: every resident block of the device, times kTriWaves so a
// block finishing early still leaves work for the scheduler to balance.
constexpr int kTriWaves = 4;

template <typename T, int P>
static int64_t tri_grid(int op) {
  static std::unordered_map<int, int64_t> cached;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  int dev = 0, cus = 0, nb = 0;
  (void)hipGetDevice(&dev);
  const int key = dev * 4 + (op == OP_BWD ? 0 : op == OP_IPROD ? 1 : op == OP_HELM ? 2 : 3);
  auto it = cached.find(key);
  if (it != cached.end()) return it->second;
  using S = TriShape<P>;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = op == OP_BWD     ? (const void*)k_tri<T, P, OP_BWD>
                   : op == OP_IPROD ? (const void*)k_tri<T, P, OP_IPROD>
                   : op == OP_HELM  ? (const void*)k_tri<T, P, OP_HELM>
                                    : (const void*)k_tri<T, P, OP_HELM_ASM>;
  (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, S::WPB * 64, 0);
  const int64_t grid = (int64_t)(cus > 0 ? cus : 256) * (nb > 0 ? nb : 1) * kTriWaves;
  cached[key] = grid;
  return grid;
}

template <typename T, int P>
static hipError_t run_tri(const OpArgs& a) {
  using S = TriShape<P>;
  const T* tab = tri_table<T>(P);
  if (!tab) return hipErrorOutOfMemory;
  const int64_t ngrp = (a.nelem + S::EPW - 1) / S::EPW;
  const int64_t need = (ngrp + S::WPB - 1) / S::WPB;
  const Tab<T, P + 1, P + 2>& tb = host_tab<T, P + 1, P + 2>();
  const DevArgs<T> d = dev_args<T>(a);
  const int64_t nb = need < tri_grid<T, P>(a.op) ? need : tri_grid<T, P>(a.op);
  const dim3 g((unsigned)nb), b(S::WPB * 64);
  switch (a.op) {
    case OP_BWD: hipLaunchKernelGGL((k_tri<T, P, OP_BWD>), g, b, 0, a.stream, tb, tab, d); break;
    case OP_IPROD: hipLaunchKernelGGL((k_tri<T, P, OP_IPROD>), g, b, 0, a.stream, tb, tab, d); break;
    case OP_HELM: hipLaunchKernelGGL((k_tri<T, P, OP_HELM>), g, b, 0, a.stream, tb, tab, d); break;
    case OP_HELM_ASM:
      hipLaunchKernelGGL((k_tri<T, P, OP_HELM_ASM>), g, b, 0, a.stream, tb, tab, d);
      break;
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

// Diagonal of the triangle Helmholtz operator, thread per (triangle, mode),
// scatter-added into the padded global diagonal (Dirichlet modes skipped):
//   diag H_e[m] = sum_points ( lambda f0 phi_m^2 + f1 d1^2 + 2 f2 d1 d2 + f3 d2^2 )
// with d1, d2 the collapsed derivatives of phi_m; the collapsed vertex is
// evaluated as (a_0 + a_P) times its eta_2 factor, as in the operator.
template <int P>
__global__ void __launch_bounds__(256)
    k_diag_tri(const Tab<double, P + 1, P + 2> tb, const double* __restrict__ tab, int64_t nelem,
               const double* __restrict__ fac, const double* __restrict__ lam, double lam0,
               const int32_t* __restrict__ l2g, double* __restrict__ diag) {
  using S = TriShape<P>;
  constexpr int N = S::N, Q = S::Q, Q2 = S::Q2, NM = S::NM;
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nelem * NM) return;
  const int64_t e = id / NM;
  const int m = (int)(id - e * NM);
  const int32_t g = l2g[id];
  if (g < 0) return;  // Dirichlet: row replaced by the identity
  int p = 0;
  for (int k = 1; k < N; ++k) p += (m >= S::off(k)) ? 1 : 0;
  const double* B2 = tab;
  const double* dB2 = tab + Q2 * NM;
  const int64_t grp = e / S::EPW;
  const int lane0 = (int)(e - grp * S::EPW) * Q2;
  const double* f = fac + grp * (int64_t)(4 * Q * S::LANES) + lane0;
  const double lm = lam ? lam[e] : lam0;
  double s = 0.0;
  for (int j = 0; j < Q2; ++j) {
    const double b = B2[j * NM + m], db = dB2[j * NM + m];
    for (int i = 0; i < Q; ++i) {
      double av = tb.B[i * N + p], dav = tb.D[i * N + p];
      if (m == P) {
        av += tb.B[i * N + P];
        dav += tb.D[i * N + P];
      }
      const double ph = av * b, d1 = dav * b, d2 = av * db;
      const double* fp = f + (int64_t)i * S::LANES + j;
      const double f0 = fp[0], f1 = fp[Q * S::LANES], f2 = fp[2 * Q * S::LANES],
                   f3 = fp[3 * Q * S::LANES];
      s += lm * f0 * ph * ph + f1 * d1 * d1 + 2.0 * f2 * d1 * d2 + f3 * d2 * d2;
    }
  }
  unsafeAtomicAdd(diag + l2g_dof(g), s);
}

template <int P>
static hipError_t run_diag_tri(int64_t nelem, const double* fac, const double* lam, double lam0,
                               const int32_t* l2g, double* diag, hipStream_t st) {
  const double* tab = tri_table<double>(P);
  if (!tab) return hipErrorOutOfMemory;
  const int64_t tot = nelem * TriShape<P>::NM;
  hipLaunchKernelGGL(k_diag_tri<P>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st,
                     host_tab<double, P + 1, P + 2>(), tab, nelem, fac, lam, lam0, l2g, diag);
  return hipGetLastError();
}

hipError_t launch_diag_tri(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st) {
  if (nelem == 0) return hipSuccess;
  switch (P) {
    case 1: return run_diag_tri<1>(nelem, fac, lam, lam0, l2g, diag, st);
    case 2: return run_diag_tri<2>(nelem, fac, lam, lam0, l2g, diag, st);
    case 3: return run_diag_tri<3>(nelem, fac, lam, lam0, l2g, diag, st);
    case 4: return run_diag_tri<4>(nelem, fac, lam, lam0, l2g, diag, st);
    case 5: return run_diag_tri<5>(nelem, fac, lam, lam0, l2g, diag, st);
    case 6: return run_diag_tri<6>(nelem, fac, lam, lam0, l2g, diag, st);
    case 7: return run_diag_tri<7>(nelem, fac, lam, lam0, l2g, diag, st);
    case 8: return run_diag_tri<8>(nelem, fac, lam, lam0, l2g, diag, st);
    case 9: return run_diag_tri<9>(nelem, fac, lam, lam0, l2g, diag, st);
    case 10: return run_diag_tri<10>(nelem, fac, lam, lam0, l2g, diag, st);
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
  // wavefront-blocked layout: group g of EPW triangles holds [4][Q][EPW * Q2],
  // lane (el, j) of the operator kernels reading one contiguous run per (k, i)
  const int epw = tri_epw(Q), lanes = epw * Q2;
  const int64_t g = e / epw;
  const int lane = (int)(e - g * epw) * Q2 + j;
  for (int k = 0; k < 4; ++k) {
    const int64_t o = (g * 4 * Q + k * Q + i) * lanes + lane;
    fac64[o] = f[k];
    fac32[o] = (float)f[k];
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
