// Instantiation and launch of the 3-D operator kernels for one set of
// polynomial orders.  Compiled once per order set (NK_PSET) so the build can
// run in parallel; each object exports launch_op3_set<NK_PSET>.
#include <mutex>

#include "engine.h"
#include "tables.h"
#include "tiles.h"

#ifndef NK_PSET
#error "NK_PSET must be defined"
#endif

namespace nk {

template <typename T, int P, int EPB, int OP, int PF = 2, int NTX = 0, bool EOI = true>
static hipError_t run3(const OpArgs& a) {
  constexpr int N = P + 1, Q = P + 2;
  static_assert(EPB > 0, "tile");
  const Tab<T, N, Q>& tb = host_tab<T, N, Q>();
  const int64_t nblk = (a.nelem + EPB - 1) / EPB;
  if (nblk > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_op3<T, N, Q, EPB, OP, PF, NTX, EOI>), dim3((unsigned)nblk),
                     dim3(EPB * (NTX ? NTX : slot_threads<Q>())), 0,
                     a.stream, tb, dev_args<T>(a));
  return hipGetLastError();
}

// The Helmholtz candidates of one I-stage form (EOI: even-odd pairs, else
// point by point); tile counts from 0 within the form.
template <typename T, int P, int OP, bool EOI>
static hipError_t run3_helm(const OpArgs& a) {
  constexpr int E0 = kTileEPB3[P][0], E1 = kTileEPB3[P][1], E2 = kTileEPB3[P][2];
  constexpr int NE = epb3_count(P);
  constexpr int EPK = packed_epb3(P);
  if constexpr (EPK > 0) {   // the packed slots, after the three factor-set forms
    if (a.tile == kHelmForms * NE) return run3<T, P, EPK, OP, 2, (P + 2) * (P + 2), EOI>(a);
  }
  if (a.tile >= NE) {   // candidates NE.. : one factor set, then four
    const int k = (a.tile - NE) % NE;
    if (a.tile >= 2 * NE) {
      if (k == 1 && E1 > 0) return run3<T, P, (E1 > 0 ? E1 : 1), OP, kDeepPF, 0, EOI>(a);
      if (k == 2 && E2 > 0) return run3<T, P, (E2 > 0 ? E2 : 1), OP, kDeepPF, 0, EOI>(a);
      return run3<T, P, E0, OP, kDeepPF, 0, EOI>(a);
    }
    if (k == 1 && E1 > 0) return run3<T, P, (E1 > 0 ? E1 : 1), OP, 1, 0, EOI>(a);
    if (k == 2 && E2 > 0) return run3<T, P, (E2 > 0 ? E2 : 1), OP, 1, 0, EOI>(a);
    return run3<T, P, E0, OP, 1, 0, EOI>(a);
  }
  if (a.tile == 1 && E1 > 0) return run3<T, P, (E1 > 0 ? E1 : 1), OP, 2, 0, EOI>(a);
  if (a.tile == 2 && E2 > 0) return run3<T, P, (E2 > 0 ? E2 : 1), OP, 2, 0, EOI>(a);
  return run3<T, P, E0, OP, 2, 0, EOI>(a);
}

template <typename T, int P, int OP>
static hipError_t run3_tiled(const OpArgs& a) {
  constexpr int E0 = kTileEPB3[P][0], E1 = kTileEPB3[P][1], E2 = kTileEPB3[P][2];
  constexpr int NE = epb3_count(P);
  if constexpr (op_has_lean(OP)) {
    constexpr int NH = kHelmForms * NE + (packed_epb3(P) > 0 ? 1 : 0);   // candidates per form
    if constexpr (helm_has_pt(P)) {
      if (a.tile >= NH) {
        OpArgs b = a;
        b.tile -= NH;
        return run3_helm<T, P, OP, false>(b);
      }
    }
    return run3_helm<T, P, OP, true>(a);
  }
  if (a.tile == 1 && E1 > 0) return run3<T, P, (E1 > 0 ? E1 : 1), OP>(a);
  if (a.tile == 2 && E2 > 0) return run3<T, P, (E2 > 0 ? E2 : 1), OP>(a);
  return run3<T, P, E0, OP>(a);
}

template <int P>
static hipError_t run3_p(nk_dtype t, const OpArgs& a) {
  if (t == NK_F64) {
    switch (a.op) {
      case OP_BWD: return run3_tiled<double, P, OP_BWD>(a);
      case OP_IPROD: return run3_tiled<double, P, OP_IPROD>(a);
      case OP_HELM: return run3_tiled<double, P, OP_HELM>(a);
      case OP_HELM_ASM: return run3_tiled<double, P, OP_HELM_ASM>(a);
      case OP_RHS: return run3<double, P, kTileEPB3[P][0], OP_RHS>(a);
      case OP_GRAD: return run3<double, P, kTileEPB3[P][0], OP_GRAD>(a);
      default: return hipErrorInvalidValue;
    }
  }
  switch (a.op) {
    case OP_BWD: return run3_tiled<float, P, OP_BWD>(a);
    case OP_IPROD: return run3_tiled<float, P, OP_IPROD>(a);
    case OP_HELM: return run3_tiled<float, P, OP_HELM>(a);
    case OP_HELM_ASM: return run3_tiled<float, P, OP_HELM_ASM>(a);
    default: return hipErrorInvalidValue;
  }
}

#define NK_CAT2(a, b) a##b
#define NK_CAT(a, b) NK_CAT2(a, b)

hipError_t NK_CAT(launch_op3_set, NK_PSET)(nk_dtype t, const OpArgs& a) {
#if NK_PSET == 0
  switch (a.P) {
    case 1: return run3_p<1>(t, a);
    case 2: return run3_p<2>(t, a);
    case 3: return run3_p<3>(t, a);
    case 4: return run3_p<4>(t, a);
  }
#elif NK_PSET == 1
  if (a.P == 5) return run3_p<5>(t, a);
#elif NK_PSET == 2
  if (a.P == 6) return run3_p<6>(t, a);
#elif NK_PSET == 3
  if (a.P == 7) return run3_p<7>(t, a);
#elif NK_PSET == 4
  if (a.P == 8) return run3_p<8>(t, a);
#elif NK_PSET == 5
  if (a.P == 9) return run3_p<9>(t, a);
#elif NK_PSET == 6
  if (a.P == 10) return run3_p<10>(t, a);
#endif
  return hipErrorInvalidValue;
}

}  // namespace nk
