// Assembled C0 system state and CG solver internals.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "nk_internal.h"

namespace nk {

// Per-system CG scalars, structure of arrays over the nsys systems.
// Accumulation slots per system for the CG reductions: one per thread of a
// vector block, so that the atomics of a system's elements and blocks spread
// over many addresses (13 824 elements put 54 additions on each).
constexpr int kSlots = 256;

struct CgState {
  double* rz = nullptr;     // r . z of the latest update (host-visible)
  double* rr = nullptr;     // r . r entering the latest update
  double* tol2 = nullptr;   // stop when rr <= tol2
  double* alpha = nullptr;
  int32_t* done = nullptr;
  int32_t* iters = nullptr;
  int32_t* status = nullptr;
  int32_t* cnt = nullptr;   // finished-block counter of the fused reductions (k_resid, k_norm2)
  int32_t* maxit = nullptr; // iteration budget of the current CG run (device, per system)
  // rotating sets (see cg.hip): gamma / r.r slots [3][nsys][2][kSlots],
  // delta slots [2][nsys][kSlots], carried scalars [2][nsys]
  double* gsl = nullptr;
  double* dsl = nullptr;
  double* sgam = nullptr;
  double* salp = nullptr;
  int32_t* sit = nullptr;
  int32_t* sdn = nullptr;
};

// Vector-kernel geometry: DOF ranges of every system are padded to multiples
// of kSegAlign so that each block of a vector kernel belongs to one system.
struct VecLayout {
  int64_t npad = 0;          // padded length
  int64_t nblk = 0;          // npad / kSegAlign
  const int32_t* blk_seg = nullptr;    // system of each block
  const int64_t* blk_first = nullptr;  // first block of each system (nsys+1)
};

// Kernel launchers (cg.hip).
template <typename T>
hipError_t cg_update(const VecLayout& L, CgState st, int nsys, int j, bool fatal,
                     const int32_t* skip, T* x, T* r, T* u, T* p, T* s, T* w, const T* dinv,
                     hipStream_t stream);
template <typename T>
hipError_t cg_start(const VecLayout& L, CgState st, int nsys, const double* b, T* w, T* r, T* u,
                    T* p, T* s, const T* dinv, hipStream_t stream);
hipError_t cg_begin_scalars(CgState st, int nsys, double tau2, const int32_t* skip,
                            const double* outer_tol2, const double* outer_rr, hipStream_t stream);
// r = (float) r64, u = M^{-1} r, w = 0, partial sums of (r, u) and (r, r)
hipError_t cg_reliable(const VecLayout& L, CgState st, int nsys, const double* r64, float* r,
                       float* u, float* w, const float* dinv, hipStream_t stream);
hipError_t cg_rearm(CgState st, int nsys, const int32_t* skip, hipStream_t stream);
// r = (b - y) on free DOFs (dinv > 0), 0 elsewhere; y is reset to 0; optionally
// p = 0; per system rz = r.dinv.r, rr = r.r; done = rr <= tol2.
hipError_t cg_residual(const VecLayout& L, CgState st, const double* b, double* y,
                       const double* dinv, double* r, double* p, double* part, hipStream_t s);
// per-system squared norm of v into out[s] (and tol2 = rtol^2 * out when tol2 != null)
hipError_t vec_norm2(const VecLayout& L, const double* v, double* part, int32_t* cnt, double* out,
                     double rtol, double* tol2, hipStream_t s);
// x += d on systems not yet converged
hipError_t cg_correct(const VecLayout& L, const int32_t* outer_done, const float* d32, double* x,
                      hipStream_t s);
template <typename T>
hipError_t vec_fill(T* v, int64_t n, T val, hipStream_t s);
// padded <-> user layouts (per system contiguous ranges)
template <typename T>
hipError_t pad_in(int nsys, const int64_t* dof_off, const int64_t* pdof_off, const VecLayout& L,
                  const T* user, const double* dinv, T* padded, hipStream_t s);
template <typename T>
hipError_t pad_out(int nsys, const int64_t* dof_off, const int64_t* pdof_off, int64_t nuser,
                   const T* padded, T* user, hipStream_t s);
hipError_t build_l2g(int64_t nelem, int nloc, const int32_t* elem_seg, const int64_t* dof_off,
                     const int64_t* pdof_off, const int32_t* l2g_user, const int8_t* sign,
                     const uint8_t* dirichlet, int32_t* l2g_int, int* bad, hipStream_t s);
// user form (global DOF + off, sign, Dirichlet flags) of a one-system
// internal l2g; dirichlet must be zeroed first
hipError_t decode_l2g(int64_t n, const int32_t* l2g_int, int64_t off, int32_t* l2g_user,
                      int8_t* sign, uint8_t* dirichlet, hipStream_t s);
// padded segment of one system from / to its own user vector
hipError_t seg_in(int64_t n, int64_t npad, const double* user, const double* dinv, double* padded,
                  hipStream_t s);
hipError_t seg_out(int64_t n, const double* padded, double* user, hipStream_t s);
hipError_t diag_finish(const VecLayout& L, const double* diag, const double* mark,
                       double* dinv64, float* dinv32, double* diag_out, hipStream_t s);
hipError_t mark_free(int64_t nelem, int nloc, const int32_t* l2g_int, double* mark, hipStream_t s);
hipError_t gather_user(int64_t nelem, int nloc, const int32_t* l2g_int, const double* xpad,
                       double* xloc, hipStream_t s);
hipError_t scatter_add(int64_t nelem, int nloc, const int32_t* l2g_int, const double* yloc,
                       double* ypad, hipStream_t s);
hipError_t cast_copy(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t cast_copy(const float* src, double* dst, int64_t n, hipStream_t s);
hipError_t launch_diag(int dim, int P, int Q, int64_t nelem, const double* Bt, const double* Dt,
                       const double* fac, const double* lam, double lam0, const int32_t* l2g,
                       double* diag, hipStream_t s);

// Statically condensed operator of a hexahedral system (condense.hip).
constexpr int kCondMinP = 2;
constexpr int kCondMaxP = 6;
// scalars of one element's interior inverse in its diagonal storage
constexpr int sc_packed(int ni) { return (ni / 2 + 1) * ni; }
struct CondOp {
  int P = 0;
  int64_t nelem = 0;
  const double* ainv = nullptr;   // [E][NI/2 + 1][NI] interior inverses by diagonals, NI = (P-1)^3
  double* t = nullptr;            // [E][NI] interior values between the passes
  const double* fac = nullptr;    // FP64 geometric factors
  const float* fac32 = nullptr;   // FP32 geometric factors
  const float* ainv32 = nullptr;  // FP32 copy of ainv (null until a refined condensed solve needs it)
  const double* lam = nullptr;
  double lam0 = 0.0;
  const int32_t* l2g = nullptr;   // internal map of the boundary system
  int variant = 0;                // fused kernel: 0 paired I stage, two factor sets; 1 point by
                                  // point, one set (fewer registers)
  int variant32 = 0;              // the same for the FP32 kernel
};
// y += S x (boundary numbering) in one fused launch, element energies into dots
// (FP32 needs ainv32)
hipError_t sc_apply(const CondOp& c, nk_dtype t, const void* x, void* y, double* dots,
                    const int32_t* dslot, const int32_t* seg_done, hipStream_t s);
// pass 1: t = interior part of H [x_b; 0]; pass 2: y += boundary part of
// H [x_b; t], element energies into dots
hipError_t sc_pass(const CondOp& c, int pass, const double* x, double* y, double* dots,
                   const int32_t* dslot, const int32_t* seg_done, hipStream_t s);
// z = gamma H_ii^{-1} (alpha t + beta b_i) into t, or added into xadd at the
// interior DOFs (iidx: DOF | sign bit per interior mode)
hipError_t sc_ainv(const CondOp& c, const double* b, const int32_t* iidx, double alpha, double beta,
                   double gamma, double* xadd, const int32_t* seg_done, hipStream_t s);
// y_e = S_e x_e on local vectors (x_e with zero interior entries)
hipError_t sc_local(const CondOp& c, const double* x, double* y, hipStream_t s);
hipError_t sc_unit(int P, int64_t nelem, double* c, int k, hipStream_t s);
hipError_t sc_unit_mode(int P, int64_t nelem, double* c, int m_new, int m_old, hipStream_t s);
hipError_t sc_diag_add(int P, int64_t nelem, const double* y, int m, const int32_t* l2g,
                       double* diag, hipStream_t s);
hipError_t sc_dinv(int64_t n, const double* diag, double* dinv64, float* dinv32, double* diag_out,
                   hipStream_t s);
hipError_t sc_column(int P, int64_t nelem, const double* y, double* A, int k, hipStream_t s);
// D = diagonal storage of the inverses of the blocks A ([E][NI][NI])
hipError_t sc_invert(int P, int64_t nelem, const double* A, double* D, int* bad, hipStream_t s);
hipError_t sc_restrict(int64_t nb, int64_t npad, const int32_t* bmap, const double* full,
                       const double* dinv_c, double* cond, hipStream_t s);
hipError_t sc_expand_add(int64_t nb, const int32_t* bmap, const double* cond, double* full,
                         hipStream_t s);

// What a system keeps of its condensed form: the boundary system and the
// arrays that connect it to the full one.
struct CondData {
  nk_system bsys = nullptr;       // boundary system (its operator is ops)
  std::vector<CondOp> ops;        // per order group
  std::vector<int64_t> ioff;      // per order group: first entry in iidx and t
  int64_t nb = 0;                 // boundary DOFs (the boundary system has nb + 1: a dummy)
  int32_t* bmap = nullptr;        // [nb] full DOF of each boundary DOF
  int32_t* iidx = nullptr;        // per group [E_g][NI_g]: full DOF | sign bit of each interior mode
  double* ainv = nullptr;
  float* ainv32 = nullptr;
  double* t = nullptr;
  double* zero = nullptr;         // boundary-length zeros
};

}  // namespace nk

struct nk_system_s {
  nk_space space = nullptr;
  int device = 0;
  int nsys = 1;
  int64_t nuser = 0;                      // user global length (sum of system DOFs)
  std::vector<int64_t> dof_off, pdof_off, elem_off, blk_first;
  nk::VecLayout L;
  int32_t* dslot = nullptr;               // CG accumulation slot of each element
  int64_t* d_dof_off = nullptr;
  int64_t* d_pdof_off = nullptr;
  int64_t* d_elem_off = nullptr;
  int64_t* d_blk_first = nullptr;
  int32_t* d_blk_seg = nullptr;
  int32_t* elem_seg = nullptr;
  int32_t* l2g = nullptr;                 // internal signed l2g into the padded numbering
  double* lam = nullptr;                  // per-element lambda copy (or null)
  double lam0 = 0.0;
  double* diag = nullptr;                 // padded, Dirichlet/padding rows = 1
  double* dinv64 = nullptr;               // 1/diag on free DOFs, exactly 0 elsewhere (the mask)
  float* dinv32 = nullptr;
  // work vectors (padded)
  double *b = nullptr, *x = nullptr, *r = nullptr, *p = nullptr, *y = nullptr;
  double *u = nullptr, *s = nullptr;
  float *r32 = nullptr, *p32 = nullptr, *y32 = nullptr, *d32 = nullptr;
  float *u32 = nullptr, *s32 = nullptr;
  double* part = nullptr;                 // per vector block x 2
  // per-system scalars
  nk::CgState st64, st32;
  double* bb = nullptr;                   // ||b||^2
  double* rr_true = nullptr;
  int32_t* cnt_aux = nullptr;
  int32_t* outer_done = nullptr;
  double* outer_tol2 = nullptr;
  double* outer_rr = nullptr;
  int32_t* outer_cnt = nullptr;
  int32_t* outer_status = nullptr;
  // host staging (pinned)
  int32_t* h_flags = nullptr;             // 2 nsys (two int32 arrays read together)
  int32_t* h_budget = nullptr;            // nsys: iteration budgets on their way to the device
  double* h_d = nullptr;                  // nsys
  hipStream_t cs = nullptr;               // private stream (graphs are captured here)
  std::vector<hipStream_t> ostreams;      // side streams of order groups 1.. (made on first use)
  std::vector<hipEvent_t> oevents;        // their join events
  hipEvent_t ofork = nullptr;             // fork event of the order groups
  hipEvent_t ev = nullptr;
  hipGraphExec_t g64 = nullptr, g32 = nullptr;
  int g64_iters = 0, g32_iters = 0;
  std::vector<int> tiles64, tiles32;   // assembled-operator tile per order group
  nk::CondData* cond = nullptr;           // statically condensed form (built on first use)
  const nk::CondOp* sc = nullptr;         // set on a boundary system: its operator is condensed
                                          // (one CondOp per order group)
};
