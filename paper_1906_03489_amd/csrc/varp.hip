// Mixed-order Helmholtz operator in ONE persistent launch (spatially variable
// polynomial order, section 4.2 of arXiv 1906.03489).  Elements are grouped
// by order; each group is cut into work items of kVarpEPB[P] elements, and a
// grid sized to the machine strides over the item list (largest orders first)
// dispatching each item to the sum-factorised body compiled for its order.
// The 1-D tables of every order live in __constant__ memory so that the
// uniform table reads go through the scalar cache.
#include <cstring>
#include <vector>

#include "engine.h"
#include "tables.h"
#include "tiles.h"

namespace nk {

// scalars of the tables of order p (Tab<T, p + 1, p + 2>)
constexpr int varp_tab_len(int p) {
  return 2 * (p + 2) * (p + 1) + (p + 3) / 2;
}
constexpr int varp_tab_off(int P) {
  int off = 0;
  for (int p = 1; p < P; ++p) off += varp_tab_len(p);
  return off;
}
constexpr int kVarpTabLen = varp_tab_off(kMaxP + 1);

__constant__ double c_tab64[kVarpTabLen];
__constant__ float c_tab32[kVarpTabLen];

template <typename T>
__device__ __forceinline__ const T* ctab();
template <>
__device__ __forceinline__ const double* ctab<double>() { return c_tab64; }
template <>
__device__ __forceinline__ const float* ctab<float>() { return c_tab32; }

template <typename T>
constexpr int varp_smem() {
  int m = 0;
  for (int P = 1; P <= kMaxP; ++P) {
    const int v = kVarpEPB[P] * 3 * (P + 2) * (P + 2) * (P + 1);
    m = v > m ? v : m;
  }
  return m;
}

template <typename T>
struct VarpDev {
  const VarpGroup* groups;
  const int64_t* item_start;
  const int64_t* lam_off;
  int ngroups;
  int64_t nitems;
  const T* x;
  T* y;
  const T* fac;
  const double* lam;
  double lam0;
};

template <typename T, int P>
__device__ __forceinline__ void varp_body(const VarpDev<T>& a, const VarpGroup& G, int64_t li,
                                          int64_t lam_off, T* smem) {
  constexpr int N = P + 1, Q = P + 2, NT = slot_threads<Q>(), EPB = kVarpEPB[P];
  static_assert(EPB * NT <= kVarpThreads, "varp tile");
  const int slot = threadIdx.x / NT;
  const int t = threadIdx.x - slot * NT;
  const int64_t e = li * EPB + slot;
  const bool live = slot < EPB && e < G.nelem;
  static_assert(sizeof(Tab<T, N, Q>) == sizeof(T) * varp_tab_len(P), "varp table layout");
  const Tab<T, N, Q>& tb = *reinterpret_cast<const Tab<T, N, Q>*>(ctab<T>() + varp_tab_off(P));
  DevArgs<T> d{};
  d.nelem = G.nelem;
  d.in = a.x + G.c0;
  d.out = a.y + G.c0;
  d.fac = a.fac + G.f0;
  d.lam = a.lam ? a.lam + lam_off : nullptr;
  d.lam0 = a.lam0;
  T* sm = smem + (slot < EPB ? slot : 0) * 3 * Q * Q * N;
  helm3_body<T, N, Q, NT, false, (P >= 8 ? 1 : 2)>(tb, sm, nullptr, slot, t, live, e, d);
}

// MINB = minimum resident blocks per CU requested from the compiler (1 or 2):
// 2 caps registers so two 256-thread blocks fit per CU, at the price of
// spills in the largest orders.
template <typename T, int MINB>
__global__ void __launch_bounds__(kVarpThreads, MINB) k_helm_varp(const VarpDev<T> a) {
  __shared__ T smem[varp_smem<T>()];
  for (int64_t item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    int g = 0;
    while (g + 1 < a.ngroups && item >= a.item_start[g + 1]) ++g;
    const VarpGroup G = a.groups[g];
    const int64_t li = item - a.item_start[g];
    const int64_t lo = a.lam_off[g];
    switch (G.P) {
      case 1: varp_body<T, 1>(a, G, li, lo, smem); break;
      case 2: varp_body<T, 2>(a, G, li, lo, smem); break;
      case 3: varp_body<T, 3>(a, G, li, lo, smem); break;
      case 4: varp_body<T, 4>(a, G, li, lo, smem); break;
      case 5: varp_body<T, 5>(a, G, li, lo, smem); break;
      case 6: varp_body<T, 6>(a, G, li, lo, smem); break;
      case 7: varp_body<T, 7>(a, G, li, lo, smem); break;
      case 8: varp_body<T, 8>(a, G, li, lo, smem); break;
      case 9: varp_body<T, 9>(a, G, li, lo, smem); break;
      case 10: varp_body<T, 10>(a, G, li, lo, smem); break;
      default: break;
    }
    __syncthreads();
  }
}

int varp_items_per_group(int P, int64_t nelem) {
  const int epb = kVarpEPB[P];
  return (int)((nelem + epb - 1) / epb);
}

template <int P>
static void put_tabs(double* t64, float* t32) {
  if constexpr (P <= kMaxP) {
    constexpr int N = P + 1, Q = P + 2;
    std::memcpy(t64 + varp_tab_off(P), &host_tab<double, N, Q>(), sizeof(Tab<double, N, Q>));
    std::memcpy(t32 + varp_tab_off(P), &host_tab<float, N, Q>(), sizeof(Tab<float, N, Q>));
    put_tabs<P + 1>(t64, t32);
  }
}

// Upload the tables of every order to this device's __constant__ memory once.
static hipError_t ensure_varp_tables() {
  static thread_local int done_dev_mask = 0;  // per-thread cache; cheap to redo
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 30 && (done_dev_mask >> dev) & 1) return hipSuccess;
  std::vector<double> t64(kVarpTabLen);
  std::vector<float> t32(kVarpTabLen);
  put_tabs<1>(t64.data(), t32.data());
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab64), t64.data(), sizeof(double) * kVarpTabLen);
  if (e != hipSuccess) return e;
  e = hipMemcpyToSymbol(HIP_SYMBOL(c_tab32), t32.data(), sizeof(float) * kVarpTabLen);
  if (e != hipSuccess) return e;
  if (dev < 30) done_dev_mask |= 1 << dev;
  return hipSuccess;
}

hipError_t launch_helm_varp(const VarpArgs& a) {
  hipError_t e = ensure_varp_tables();
  if (e != hipSuccess) return e;
  if (a.nitems == 0) return hipSuccess;
  if (a.t == NK_F64) {
    VarpDev<double> d{a.groups_dev, a.item_start_dev, a.lam_off_dev, a.ngroups, a.nitems,
                      (const double*)a.x, (double*)a.y, (const double*)a.fac, a.lam, a.lam0};
    if (a.minb == 2)
      hipLaunchKernelGGL((k_helm_varp<double, 2>), dim3(a.grid), dim3(kVarpThreads), 0, a.stream, d);
    else
      hipLaunchKernelGGL((k_helm_varp<double, 1>), dim3(a.grid), dim3(kVarpThreads), 0, a.stream, d);
  } else {
    VarpDev<float> d{a.groups_dev, a.item_start_dev, a.lam_off_dev, a.ngroups, a.nitems,
                     (const float*)a.x, (float*)a.y, (const float*)a.fac, a.lam, a.lam0};
    if (a.minb == 2)
      hipLaunchKernelGGL((k_helm_varp<float, 2>), dim3(a.grid), dim3(kVarpThreads), 0, a.stream, d);
    else
      hipLaunchKernelGGL((k_helm_varp<float, 1>), dim3(a.grid), dim3(kVarpThreads), 0, a.stream, d);
  }
  return hipGetLastError();
}

int varp_blocks_per_cu(nk_dtype t, int minb) {
  int nb = 0;
  if (t == NK_F64)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, minb == 2 ? k_helm_varp<double, 2> : k_helm_varp<double, 1>, kVarpThreads, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, minb == 2 ? k_helm_varp<float, 2> : k_helm_varp<float, 1>, kVarpThreads, 0);
  return nb > 0 ? nb : 1;
}

}  // namespace nk
