// Internal declarations shared by the library's host and device sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/nk.h"

namespace nk {

// ------------------------------------------------------------------ limits
constexpr int kMinP = 1;
constexpr int kMaxP = 10;          // n = P+1 <= 11, Q = P+2 <= 12
constexpr int kNF3 = 7;            // per-point factors in 3-D
constexpr int kNF2 = 4;            // per-point factors in 2-D
constexpr int kVecBlock = 256;     // threads per block of the CG vector kernels
constexpr int64_t kSegAlign = 2048;  // DOF ranges of each system padded to this (one vector block)

// Internal l2g entries of assembled systems: v >= 0 is the free padded DOF v,
// v < 0 the Dirichlet padded DOF -1-v.  In both, bit 30 of the DOF marks a
// local mode whose global function is the negative of the local one (an edge
// or face that the element traverses against its global direction); the DOF
// index is the value with that bit cleared, so padded systems stay below 2^30.
constexpr int32_t kL2gNeg = 1 << 30;
__host__ __device__ __forceinline__ int32_t l2g_dof(int32_t v) {
  return (v >= 0 ? v : -1 - v) & (kL2gNeg - 1);
}
__host__ __device__ __forceinline__ bool l2g_neg(int32_t v) {
  return ((v >= 0 ? v : -1 - v) & kL2gNeg) != 0;
}
template <typename T>
__host__ __device__ __forceinline__ T l2g_sign(int32_t v, T x) {
  return l2g_neg(v) ? -x : x;
}
// Gathers read x[l2g_dof(v)] for every entry, Dirichlet ones included (their
// -1-g also names a valid DOF), with no branch, so that the loads of all of a
// thread's entries are in flight together; l2g_value then turns the raw value
// into the local one (0 for a Dirichlet entry, sign flipped for a negative
// orientation).  Applying the sign inside a per-entry branch made the
// compiler wait for each load in turn.
template <typename T>
__host__ __device__ __forceinline__ T l2g_value(int32_t v, T raw) {
  return v >= 0 ? l2g_sign(v, raw) : T(0);
}

// Whether element e belongs to a converged system (its operator work is
// skipped).  Batched systems look the flag up through the element's system
// index; a single system passes no index and its one flag is a uniform
// (scalar) load, so no per-element chain of two dependent loads precedes
// the element's gather.
__device__ __forceinline__ bool seg_converged(const int32_t* elem_seg, const int32_t* seg_done,
                                              int64_t e) {
  if (seg_done == nullptr) return false;
  return (elem_seg != nullptr ? seg_done[elem_seg[e]] : seg_done[0]) != 0;
}

// ------------------------------------------------------------ host tables
void gll_points(int Q, double* x, double* w);
void modified_basis(int P, int Q, const double* x, double* B, double* DB);
void collocation_derivative(int Q, const double* x, double* Dc);
void symmetric_eigen(int n, const double* A, double* V, double* lam);
void tri_points(int Q, double* e1, double* w1, double* e2, double* w2);
void tri_btable(int P, int nz, const double* z, double* Bt, double* dBt);
void radau_points(int n, int alpha, double* x, double* w);
void tet_points(int Q, double* e1, double* w1, double* e2, double* w2, double* e3, double* w3);
int tri_mode_degree(int P, int p, int q);
void tet_ctable(int P, int nz, const double* z, double* Ct, double* dCt);
int mod_degree(int P, int p);
void pyr_ctable(int P, int nz, const double* z, double* Ct, double* dCt);

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
nk_status fail(nk_status st, const std::string& msg);
nk_status hip_fail(hipError_t e, const char* what);

#define NK_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return ::nk::hip_fail(e_, #call); \
  } while (0)

// ------------------------------------------------------------- operators
enum OpKind : int {
  OP_BWD = 0,        // coeffs -> point values
  OP_IPROD = 1,      // point values -> coeffs (w detJ weighted)
  OP_HELM = 2,       // local Helmholtz
  OP_HELM_ASM = 3,   // gather -> Helmholtz -> scatter-add, per-element p.Ap
  OP_RHS = 4,        // weak Helmholtz form of a point field (FP64)
  OP_GRAD = 5,       // adjoint parameter gradient (FP64)
  OP_DIAG = 6,       // elemental Helmholtz diagonal scattered to global (FP64)
  OP_COUNT = 7
};

// Everything one operator launch needs; pointers are device pointers of the
// element group being processed (already offset to the group's start).
struct OpArgs {
  int op = 0;
  int dim = 3, P = 0, Q = 0;
  int64_t nelem = 0;
  const void* in = nullptr;     // coefficients or point values (dtype)
  void* out = nullptr;          // point values, coefficients, or global y (dtype)
  const void* fac = nullptr;    // geometric factors (dtype)
  const double* lam = nullptr;  // per-element lambda or null
  double lam0 = 0.0;
  const int32_t* l2g = nullptr; // signed local-to-global (assembled ops): -1-g marks Dirichlet
  double* dots = nullptr;       // per-element p_e . (H_e p_e) (assembled ops)
  const double* in2 = nullptr;  // RHS: reference gradient; GRAD: u_loc
  double* out2 = nullptr;       // GRAD: dlambda; DIAG: unused
  const double* kappa = nullptr;  // GRAD: kappa per point (null = 1)
  const int32_t* elem_seg = nullptr;  // batched: segment of each element
  const int32_t* seg_done = nullptr;  // batched: converged flag per segment
  const int32_t* dslot = nullptr;     // assembled ops: where element e's p.Ap goes in dots
  int tile = 0;                 // tile configuration index
  hipStream_t stream = nullptr;
};

// Matrix-core variant of the Helmholtz operator (local and assembled) for
// 3-D orders with Q <= 8; selected as the last tile candidate of OP_HELM.
bool mfma_supported(int dim, int P);
hipError_t launch_helm_mfma(nk_dtype t, const OpArgs& a);

// Number of compiled tile configurations for an operator and its names.
int tile_count(int op, int dim, int P);
const char* tile_name(int op, int dim, int P, int tile);

// Launch one operator on one element group.  Returns hipErrorInvalidValue
// for (dim, P) combinations that are not compiled.
hipError_t launch_op3(nk_dtype t, const OpArgs& a);
hipError_t launch_op2(nk_dtype t, const OpArgs& a);
bool op_supported(int dim, int P, int Q);

// Mixed-order Helmholtz: all groups in one persistent launch.
struct VarpGroup {
  int P = 0;
  int64_t nelem = 0, c0 = 0, f0 = 0;   // coefficient / factor offsets (elements of scalars)
};
struct VarpArgs {
  nk_dtype t = NK_F64;
  int ngroups = 0;
  const VarpGroup* groups_dev = nullptr;   // device array of groups
  const int64_t* item_start_dev = nullptr; // device prefix sum of work items per group
  int64_t nitems = 0;
  const void* x = nullptr;
  void* y = nullptr;
  const void* fac = nullptr;
  const double* lam = nullptr;  // per element over the concatenated elements, or null
  const int64_t* lam_off_dev = nullptr;    // element offset of each group
  double lam0 = 0.0;
  int grid = 0;
  int minb = 1;                 // minimum resident blocks per CU (register cap)
  hipStream_t stream = nullptr;
};
hipError_t launch_helm_varp(const VarpArgs& a);

// Strategies for operators on a mixed-order space (chosen by the autotuner):
enum VarpStrategy : int {
  VARP_PERSISTENT = 0,      // one persistent launch over all order groups
  VARP_PERSISTENT_2 = 1,    // same, registers capped for two blocks per CU
  VARP_CONCURRENT = 2,      // one launch per order group, all groups concurrent
  VARP_SEQUENTIAL = 3,      // one launch per order group, in order (reference)
  VARP_COUNT = 4
};
int varp_items_per_group(int P, int64_t nelem);   // work items of one group
int varp_blocks_per_cu(nk_dtype t, int minb);

// One entry point per compiled order set (objects built from ops3d_inst.hip).
hipError_t launch_op3_set0(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set1(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set2(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set3(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set4(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set5(nk_dtype t, const OpArgs& a);
hipError_t launch_op3_set6(nk_dtype t, const OpArgs& a);

// PhysDeriv / IProductWRTDerivBase / FwdTrans (deriv.hip).
enum DerivKind : int { DERIV_PHYS = 0, DERIV_IPROD = 1, DERIV_FWD = 2 };
constexpr int kFwdMaxIt = 100;   // CG iterations per element in FwdTrans
struct DerivArgs {
  int64_t nelem = 0;
  const void* in = nullptr;
  void* out = nullptr;
  const void* dfac = nullptr;   // derivative factors of the group, dtype of the call
  hipStream_t stream = nullptr;
};
hipError_t launch_deriv(nk_dtype t, int which, int dim, int P, const DerivArgs& a);

// Collapsed triangles (tri.hip): BwdTrans, IProductWRTBase, Helmholtz.  The
// operator kernels give each lane one eta_2 point row of a triangle, so a
// wavefront holds tri_epw(Q) triangles, and the geometric factors are stored
// in groups of that many triangles ([group][4][Q][tri_epw(Q) * (Q-1)]).
constexpr int tri_epw(int Q) { return 64 / (Q - 1); }
inline int64_t tri_fac_count(int Q, int64_t nelem) {
  const int64_t g = (nelem + tri_epw(Q) - 1) / tri_epw(Q);
  return g * tri_epw(Q) * 4 * (int64_t)Q * (Q - 1);
}
hipError_t launch_tri(nk_dtype t, const OpArgs& a);   // also OP_HELM_ASM (assembled)
hipError_t launch_diag_tri(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st);
// Collapsed tetrahedra and prisms (collapsed3d.hip): BwdTrans,
// IProductWRTBase, Helmholtz; pyramids too.  pts: e1, w1 (Q), e2, w2 (Q-1,
// Q for pyramids), e3, w3 (Q-1, Q for prisms).
hipError_t launch_tet(nk_dtype t, const OpArgs& a);
hipError_t launch_prism(nk_dtype t, const OpArgs& a);
hipError_t launch_pyr(nk_dtype t, const OpArgs& a);
hipError_t launch_diag_tet(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st);
hipError_t launch_diag_prism(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                             const int32_t* l2g, double* diag, hipStream_t st);
hipError_t launch_diag_pyr(int P, int64_t nelem, const double* fac, const double* lam, double lam0,
                           const int32_t* l2g, double* diag, hipStream_t st);
hipError_t launch_geom_tet(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s);
hipError_t launch_geom_prism(int Q, int64_t nelem, const double* jac, const double* kappa,
                             const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s);
hipError_t launch_geom_pyr(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s);
hipError_t launch_geom_tri(int Q, int64_t nelem, const double* jac, const double* kappa,
                           const double* pts, double* fac64, float* fac32, int* bad, hipStream_t s);

// Geometry: per-point factors from Jacobians.
hipError_t launch_geom(int dim, int Q, int64_t nelem, const double* jac, const double* kappa,
                       const double* wq, double* fac64, float* fac32, double* dfac64,
                       float* dfac32, int* bad, hipStream_t s);

// ------------------------------------------------------------------- space
struct Group {
  int P = 0, Q = 0, n = 0;
  int64_t nelem = 0;
  int64_t e0 = 0;   // first element (global element index)
  int64_t c0 = 0;   // first coefficient
  int64_t q0 = 0;   // first point value
  int64_t f0 = 0;   // first factor entry
  int64_t d0 = 0;   // first derivative-factor entry
};

}  // namespace nk

struct nk_space_s {
  int dim = 3;
  int shape = 0;             // 0: quadrilaterals / hexahedra, 1: collapsed triangles
  int device = 0;
  std::vector<nk::Group> groups;
  int64_t nelem = 0, ncoeff = 0, npoint = 0, nfac = 0;
  double* fac64 = nullptr;
  float* fac32 = nullptr;
  // derivative factors [E][d*d + 1][Q^d], standard point order: J^{-1}
  // (d xi_a / d x_c at index a*d + c), then w detJ
  int64_t ndfac = 0;
  double* dfac64 = nullptr;
  float* dfac32 = nullptr;
  double* kappa = nullptr;   // copy of kappa per point (null = 1)
  // variable-order persistent launch tables
  nk::VarpGroup* varp_groups = nullptr;
  int64_t* varp_item_start = nullptr;
  int64_t* varp_lam_off = nullptr;
  int64_t varp_nitems = 0;
  int varp_strategy[2] = {nk::VARP_PERSISTENT, nk::VARP_PERSISTENT};   // per dtype
  // fork/join streams of the concurrent strategy (created on first use)
  std::vector<hipStream_t> gstreams;
  std::vector<hipEvent_t> gevents;
  hipEvent_t fork = nullptr;
};
