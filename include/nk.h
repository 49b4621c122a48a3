/*
 * nk.h -- C ABI of the matrix-free spectral/hp operator library for MI355X
 * (gfx950).
 *
 * The library evaluates, for many same-shape tensor-product elements at once,
 * the operators that section 3.3 ("Collective linear algebra operations") of
 * Moxey et al., "Nektar++: enhancing the capability and application of
 * high-fidelity spectral/hp element methods" (arXiv 1906.03489) groups into
 * collections: the backward transform (elemental expansion evaluated at the
 * quadrature points), the inner product with respect to the basis, and the
 * Helmholtz operator of the weak problem a(u, v) = l(v) of Eqs. (1)-(2), all
 * by sum-factorisation (the display in section 3.3).  On top of these it
 * assembles the C0 system (section 2.1, assembly operator) and solves it with
 * Jacobi-preconditioned conjugate gradients (FP64, FP32 with FP64 residual
 * updates, or FP64 on the system statically condensed onto the elemental
 * boundary DOFs), batches independent systems and mixed orders, and
 * differentiates the solve with respect to kappa and lambda.  Besides
 * quadrilaterals and hexahedra it covers the collapsed-coordinate triangles,
 * tetrahedra, prisms and pyramids of section 2.1 (their elemental operators
 * and assembled solves; nk_space_create_tri / _tet / _prism / _pyr).
 *
 * Discretisation (section 2.1):
 *   - 1-D modified hierarchical C0 basis phi_p, 0 <= p <= P (P = polynomial
 *     order, n = P + 1 modes per direction): phi_0 = (1-x)/2 and
 *     phi_P = (1+x)/2 are the vertex modes, phi_p = (1-x)/2 (1+x)/2
 *     P^{1,1}_{p-1}(x) the bubbles; tensor products on quads and hexes;
 *   - Q Gauss-Lobatto-Legendre points per direction (currently Q = P + 2);
 *   - the map chi_e of each element enters through its Jacobian
 *     J = dx/dxi at every quadrature point.
 * The Helmholtz operator is  y_e = (L_e + lambda_e M_e) x_e  with
 *   M_e = B^T diag(w detJ) B,
 *   L_e = sum_{a,b} (D_a B)^T diag(w detJ kappa (J^{-1} J^{-T})_{ab}) (D_b B),
 * i.e. the weak form of -div(kappa grad u) + lambda u (symmetric positive
 * definite for lambda >= 0).
 *
 * Layouts (all arrays row-major, element index slowest):
 *   coefficients  [E][n^d]  mode m = p + n*(q + n*r), direction 1 fastest;
 *   point values  [E][Q^d]  point k = i + Q*(j + Q*l), direction 1 fastest;
 *   Jacobians     [E][d][d][Q^d], entry [e][c][a][k] = d x_c / d xi_a;
 *   kappa         [E][Q^d];  lambda  [E].
 * For a variable-order space the groups' arrays are concatenated in group
 * order.
 *
 * Ownership: every buffer argument is owned by the caller; "device" means
 * GPU memory of the current HIP device, "host" means CPU memory.  Create
 * calls copy or derive what they need; no call keeps a caller pointer after
 * it returns.  Handles own their GPU memory and free it on destroy.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Operator
 * calls are asynchronous on it.  Create calls and solves synchronise it.
 *
 * Errors: every call returns an nk_status; nothing throws across the ABI.
 * Arguments are validated before any device work; on a non-OK status
 * nk_last_error() returns a thread-local message.  NK_EDEVICE means no usable
 * HIP device is present.
 */
#ifndef NK_H
#define NK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NK_OK = 0,
  NK_EINVAL = 1,        /* bad argument (null pointer, bad size, bad enum) */
  NK_ENOMEM = 2,        /* device allocation failed                        */
  NK_EDEVICE = 3,       /* no usable HIP device                            */
  NK_EHIP = 4,          /* a HIP runtime call failed                       */
  NK_ENOCONV = 5,       /* true residual above rtol when the iteration
                           budget ran out; x holds the last iterate         */
  NK_EBREAKDOWN = 6,    /* CG breakdown (p.Ap <= 0 or non-finite)          */
  NK_EUNSUPPORTED = 7   /* (dim, P, Q) combination not compiled in         */
} nk_status;

typedef enum { NK_F64 = 0, NK_F32 = 1 } nk_dtype;

typedef enum {
  NK_SOLVE_F64 = 0,
  NK_SOLVE_F32_REFINED = 1,
  NK_SOLVE_CONDENSED = 2,
  NK_SOLVE_CONDENSED_F32_REFINED = 3
} nk_solve_mode;

typedef struct nk_space_s* nk_space;
typedef struct nk_system_s* nk_system;

typedef struct {
  int iters;             /* CG iterations summed over restarts (FP64 mode) or inner
                            FP32 iterations summed over refinement steps            */
  int outer_iters;       /* FP64 residual updates (FP32-refined mode), condensation
                            passes (condensed modes), 0 otherwise                      */
  double rel_resid;      /* true ||b - A x||_2 / ||b||_2 recomputed in FP64 at exit    */
  double solve_ms;       /* wall time of the solve on the host clock                   */
  int status;            /* nk_status of this system                                   */
} nk_solve_info;

/* Thread-local message describing the last non-OK status of this thread. */
const char* nk_last_error(void);

/* Library version, as 10000*major + 100*minor + patch. */
int nk_version(void);

/* Number of usable HIP devices (0 if none); never fails. */
int nk_device_count(void);

/* Host-side 1-D tables (section 2.1): Q GLL points x[Q] and weights w[Q],
 * B[Q][P+1] = phi_p(x_i) and DB[Q][P+1] = phi_p'(x_i).  Any output may be
 * NULL.  Host memory.  1 <= P, P + 1 <= Q <= 32.  Useful to evaluate a
 * mesh's Jacobians at the library's quadrature points. */
nk_status nk_basis_tables(int P, int Q, double* x, double* w, double* B, double* DB);

/* Create a space of `nelem` elements of one shape (dim = 2: quads, 3: hexes)
 * at order P with Q points per direction -- one collection in the sense of
 * section 3.3.  jac: device [E][d][d][Q^d]; kappa: device [E][Q^d] or NULL
 * (kappa = 1).  Computes and stores the per-point geometric factors
 * w detJ and w detJ kappa (J^{-1} J^{-T})_{ab} in FP64 and FP32.  Returns
 * NK_EINVAL if any detJ <= 0, NK_EUNSUPPORTED if (dim, P, Q) is not built. */
nk_status nk_space_create(nk_space* out, int dim, int64_t nelem, int P, int Q,
                          const double* jac, const double* kappa, void* stream);

/* Variable polynomial order (section 4.2): `ngroups` groups, group g holding
 * nelem[g] elements at order P[g] with Q[g] points (host arrays); jac[g] and
 * kappa[g] (kappa may be NULL) are device pointers laid out as for
 * nk_space_create.  Operators on such a space take the groups' arrays
 * concatenated in group order and run as ONE persistent launch. */
nk_status nk_space_create_varp(nk_space* out, int dim, int ngroups, const int* P,
                               const int* Q, const int64_t* nelem,
                               const double* const* jac, const double* const* kappa,
                               void* stream);

nk_status nk_space_destroy(nk_space s);

/* Evaluation strategy of the Helmholtz operator on a mixed-order space, per
 * dtype (section 3.3 picks among evaluation strategies by timing them at
 * start-up; nk_autotune does the same):
 *   0  one persistent launch over all order groups (work items of the
 *      largest orders first),
 *   1  the same with registers capped for two resident blocks per CU,
 *   2  one launch per order group, all groups on concurrent streams
 *      (fork/join with the caller's stream),
 *   3  one launch per order group in sequence.
 * BwdTrans and IProductWRTBase on mixed-order spaces always use 2.  Calls on
 * one space from several host threads at once must not use strategy 2. */
nk_status nk_space_set_strategy(nk_space s, nk_dtype t, int strategy);
int nk_space_get_strategy(nk_space s, nk_dtype t);   /* -1 on bad arguments */

/* Collapsed-coordinate triangles (section 2.1: a quadrilateral with one
 * direction collapsed by the Duffy map; the expansion factors in the collapsed
 * coordinates eta_1 = 2(1+xi_1)/(1-xi_2) - 1, eta_2 = xi_2 on the reference
 * triangle xi_1, xi_2 >= -1, xi_1 + xi_2 <= 0).  Quadrature: Q GLL points in
 * eta_1 and Q-1 Gauss-Radau points of the weight (1 - eta_2) in eta_2 (-1
 * included); point q = i + Q j.  nk_tri_points returns them (host arrays of
 * Q, Q, Q-1, Q-1 doubles; the eta_2 weights include the factor (1 - eta_2)).
 * Modes ((P+1)(P+2)/2 per element) are grouped by the eta_1 index p: p = 0
 * with q = 0..P (q = P the collapsed vertex (1+eta_2)/2), 0 < p < P with
 * q = 0..P-1-p, p = P with q = 0..P-1.
 * nk_space_create_tri: nelem triangles of order P (1..10, Q = P + 2); jac:
 * device [E][2][2][Q(Q-1)] FP64, jac[e][c][a][q] = d x_c / d xi_a at the
 * points; kappa: device [E][Q(Q-1)] or NULL.  Such a space supports
 * nk_bwd_trans, nk_iprod_wrt_base and nk_helmholtz (coefficients [E][nmodes],
 * points [E][Q(Q-1)]); other calls return NK_EUNSUPPORTED. */
nk_status nk_tri_points(int Q, double* eta1, double* w1, double* eta2, double* w2);
nk_status nk_space_create_tri(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream);

/* Collapsed-coordinate tetrahedra (section 2.1: the tetrahedron reached from
 * the hexahedron by collapsing two directions, eta_1 = 2(1+xi_1)/(-xi_2-xi_3)
 * - 1, eta_2 = 2(1+xi_2)/(1-xi_3) - 1, eta_3 = xi_3 on the reference
 * tetrahedron xi_a >= -1, xi_1 + xi_2 + xi_3 <= -1).  Quadrature: Q GLL points
 * in eta_1, Q-1 Gauss-Radau points of the weight (1 - eta_2) in eta_2 and Q-1
 * of the weight (1 - eta_3)^2 in eta_3 (-1 included in both); point
 * q = i + Q (j + (Q-1) k).  nk_tet_points returns them (host arrays of Q, Q,
 * Q-1 (x4) doubles; the Radau weights include their weight functions).
 * Modes ((P+1)(P+2)(P+3)/6 per element): each triangle mode t of the order-P
 * triangle (nk_space_create_tri's order), of total degree s, times
 * ((1-eta_3)/2)^s for r = 0 and ((1-eta_3)/2)^s (1+eta_3)/2
 * P^{2s-1,1}_{r-1}(eta_3) for 1 <= r <= P - s, grouped by t with r fastest;
 * the top vertex (1+eta_3)/2 last.
 * nk_space_create_tet: nelem tetrahedra of order P (1..10, Q = P + 2); jac:
 * device [E][3][3][Q(Q-1)^2] FP64, jac[e][c][a][q] = d x_c / d xi_a at the
 * points; kappa: device [E][Q(Q-1)^2] or NULL.  Elements may be left-handed
 * (det J < 0, as ordering every element's vertices by increasing global id
 * produces): the integrals take |det J|; a zero or non-finite determinant
 * or a non-positive kappa returns NK_EINVAL.  Such a space supports
 * nk_bwd_trans, nk_iprod_wrt_base and nk_helmholtz (coefficients [E][nmodes],
 * points [E][Q(Q-1)^2]) and one assembled system (nk_system_create[_signed]);
 * with sorted vertex orders the expansion is C0 without signs (every shared
 * edge and face is seen with the same vertex order).  Other calls return
 * NK_EUNSUPPORTED. */
nk_status nk_tet_points(int Q, double* eta1, double* w1, double* eta2, double* w2, double* eta3,
                        double* w3);
nk_status nk_space_create_tet(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream);

/* Prisms (section 2.1: the hexahedron with one direction collapsed): the
 * triangle of nk_space_create_tri in (xi_1, xi_2), extruded along xi_3 in
 * [-1, 1].  Quadrature: the triangle's points (nk_tri_points) times Q GLL
 * points in xi_3 (nk_basis_tables); point q = i + Q (j + (Q-1) k).  Modes
 * ((P+1)^2 (P+2)/2 per element): each triangle mode times the 1-D modified
 * basis phi_r(xi_3), r = 0..P, grouped by triangle mode with r fastest.
 * jac: device [E][3][3][Q^2 (Q-1)] FP64, kappa: device [E][Q^2 (Q-1)] or
 * NULL.  Supports nk_bwd_trans, nk_iprod_wrt_base, nk_helmholtz and
 * assembled systems (nk_system_create, nk_system_create_signed); other
 * calls return NK_EUNSUPPORTED; a non-positive Jacobian determinant or kappa
 * returns NK_EINVAL. */
nk_status nk_space_create_prism(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                                const double* kappa, void* stream);

/* Pyramids (section 2.1: the hexahedron with its top face collapsed to a
 * point): base [-1, 1]^2 at xi_3 = -1, apex (-1, -1, 1); eta_a = 2(1+xi_a)/
 * (1-xi_3) - 1 (a = 1, 2), eta_3 = xi_3.  Quadrature: Q GLL points in eta_1
 * and eta_2 (nk_basis_tables), Q-1 Gauss-Radau points of (1-eta_3)^2 in
 * eta_3 (nk_tet_points' third set); point q = i + Q (j + Q k).  Modes
 * ((P+1)(P+2)(2P+3)/6 per element): each base mode phi_p(eta_1)
 * phi_q(eta_2) (p slow, q fast) with s = max(deg phi_p, deg phi_q), times
 * ((1-eta_3)/2)^s for r = 0 and ((1-eta_3)/2)^s (1+eta_3)/2
 * P^{2s-1,1}_{r-1}(eta_3) for 1 <= r <= P - s (r fastest); the apex
 * (1+eta_3)/2 last.  jac: device [E][3][3][Q^2 (Q-1)] FP64, kappa: device
 * [E][Q^2 (Q-1)] or NULL; supported calls and errors as for prisms. */
nk_status nk_space_create_pyr(nk_space* out, int64_t nelem, int P, int Q, const double* jac,
                              const double* kappa, void* stream);

/* Sizes of a space: total elements, coefficients (sum n^d) and points
 * (sum Q^d).  Any output may be NULL. */
nk_status nk_space_sizes(nk_space s, int64_t* nelem, int64_t* ncoeffs, int64_t* npoints);

/* BwdTrans (section 2.1 elemental expansion; section 3.3 sum-factorisation):
 * phys_e = (B (x) B (x) B) coeffs_e.  coeffs: device [E][n^d], phys: device
 * [E][Q^d], both of type t. */
nk_status nk_bwd_trans(nk_space s, nk_dtype t, const void* coeffs, void* phys, void* stream);

/* IProductWRTBase: coeffs_e = B^T diag(w detJ) phys_e (section 3.3 operator
 * set).  phys: device [E][Q^d], coeffs: device [E][n^d], type t. */
nk_status nk_iprod_wrt_base(nk_space s, nk_dtype t, const void* phys, void* coeffs, void* stream);

/* Local Helmholtz operator y_e = (L_e + lambda_e M_e) x_e, matrix-free.
 * lambda: device [E] FP64 per-element coefficients, or NULL to use lambda0
 * for every element.  x, y: device [E][n^d] of type t (x and y must not
 * overlap). */
nk_status nk_helmholtz(nk_space s, nk_dtype t, const double* lambda, double lambda0,
                       const void* x, void* y, void* stream);

/* PhysDeriv (differentiation, one of the core elemental operations listed in
 * section 2.3): deriv[e][c][q] = d u / d x_c at quadrature point q of the
 * interpolant of element e's point values, i.e. the collocation derivative
 * along each reference direction followed by the chain rule with J^{-1}.
 * phys: device [E][Q^d], deriv: device [E][d][Q^d], both of type t (must not
 * overlap).  Exact for fields of degree <= Q-1 per reference direction. */
nk_status nk_phys_deriv(nk_space s, nk_dtype t, const void* phys, void* deriv, void* stream);

/* IProductWRTDerivBase (the volume term of the weak form in section 2.2):
 * coeffs[e][m] = sum_q w_q detJ_q sum_c (d phi_m / d x_c)(x_q) f[e][c][q] for a
 * vector field f given at the quadrature points.  f: device [E][d][Q^d],
 * coeffs: device [E][n^d], type t. */
nk_status nk_iprod_wrt_deriv_base(nk_space s, nk_dtype t, const void* f, void* coeffs,
                                  void* stream);

/* FwdTrans (the projection called in the listing of section 3.5): the
 * coefficients of each element's L2 projection of its point values,
 * coeffs_e = M_e^{-1} IProductWRTBase(phys)_e.  Each element's mass system
 * is solved on chip by conjugate gradients preconditioned with the exact
 * inverse of the tensor-product mass at the element's mean Jacobian
 * determinant, from a zero start, until the residual falls below 1e-13 (FP64)
 * or 2e-6 (FP32) of the right-hand side or after 100 iterations.  phys:
 * device [E][Q^d], coeffs: device [E][n^d], type t. */
nk_status nk_fwd_trans(nk_space s, nk_dtype t, const void* phys, void* coeffs, void* stream);

/* Weak form of the Helmholtz operator of a field given at the quadrature
 * points: y_e[m] = a_e(U, phi_m) = sum_a (D_a B)^T (w detJ kappa sum_b G_ab dU_b)
 * + lambda_e B^T (w detJ U), the right-hand side l(v) = a(U, v) of Eq. (1)
 * for a manufactured U.  u: device [E][Q^d] values; du: device [E][d][Q^d]
 * reference-coordinate gradient dU/dxi_a; y: device [E][n^d].  FP64. */
nk_status nk_helmholtz_weak_rhs(nk_space s, const double* lambda, double lambda0,
                                const double* u, const double* du, double* y,
                                void* stream);

/* Assembled C0 system (section 2.1, assembly operator) over a space with a
 * single group: nglobal global coefficients, l2g device int32 [E][n^d]
 * mapping local to global modes (no sign flips), dirichlet device uint8
 * [nglobal] (1 = homogeneous Dirichlet DOF, fixed at zero), lambda device
 * [E] or NULL (lambda0).  Builds the Jacobi diagonal on the GPU.  Triangle
 * spaces take l2g [E][(P+1)(P+2)/2], tetrahedron spaces l2g
 * [E][(P+1)(P+2)(P+3)/6], prism spaces l2g [E][(P+1)^2 (P+2)/2] and
 * pyramid spaces l2g [E][(P+1)(P+2)(2P+3)/6] in the space's mode order (one
 * system each).  The global functions of unstructured triangle and prism
 * meshes generally need nk_system_create_signed.
 * The padded system (each system's DOFs rounded up to 2048) must stay below
 * 2^30 DOFs (NK_EINVAL otherwise). */
nk_status nk_system_create(nk_system* out, nk_space s, int64_t nglobal, const int32_t* l2g,
                           const uint8_t* dirichlet, const double* lambda, double lambda0,
                           void* stream);

/* As nk_system_create, with orientation signs for unstructured meshes
 * (section 2.1: the assembly operator maps local to global modes, and an
 * edge or face that an element traverses against the global direction sees
 * the odd-parity bubbles of that edge or face negated).  sign: device int8
 * [E][modes] with entries +1 or -1 (NULL = all +1): the local mode equals
 * sign times the global function l2g names, so gathering reads sign * x[g]
 * and scattering adds sign * y_local.  Any other sign value or an l2g index
 * outside [0, nglobal) returns NK_EINVAL.  Index permutations (a face seen
 * transposed) are expressed through l2g itself.  Nothing is retained: the
 * map and signs are copied into the system. */
nk_status nk_system_create_signed(nk_system* out, nk_space s, int64_t nglobal,
                                  const int32_t* l2g, const int8_t* sign,
                                  const uint8_t* dirichlet, const double* lambda, double lambda0,
                                  void* stream);

/* Many independent systems solved together (the union is block diagonal):
 * system k owns elements [elem_off[k], elem_off[k+1]) of the space and global
 * DOFs [dof_off[k], dof_off[k+1]) (host int64 arrays of nsys+1 entries); l2g
 * holds indices into the union numbering.  Each system keeps its own CG
 * scalars and convergence test. */
nk_status nk_system_create_batched(nk_system* out, nk_space s, int nsys,
                                   const int64_t* elem_off, const int64_t* dof_off,
                                   const int32_t* l2g, const uint8_t* dirichlet,
                                   const double* lambda, double lambda0, void* stream);

nk_status nk_system_destroy(nk_system sys);

/* y = R A R x for the assembled operator (R zeroes Dirichlet entries) in the
 * given precision.  x, y: device [nglobal] of type t. */
nk_status nk_system_apply(nk_system sys, nk_dtype t, const void* x, void* y, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * y = R A R x as nk_system_apply, same kernels and arguments, but the padded
 * input and output staging lives in a static device array of the library
 * (64 MiB per GPU, held until the process ends) instead of the system's work
 * vectors.  The call allocates nothing, does not synchronise (it is ordered
 * on `stream` only) and needs the system's device to be current.  Limit:
 * 2 x padded DOFs x scalar size <= 64 MiB (4 Mi padded DOFs in FP64, 8 Mi in
 * FP32); larger systems return NK_EINVAL with the sizes in nk_last_error.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (different streams or threads without ordering between them) race. */
nk_status nk_system_apply_noalloc(nk_system sys, nk_dtype t, const void* x, void* y, void* stream);

/* b = R (sum_e A_e^T y_loc_e): scatter-add of local vectors into the global
 * numbering with Dirichlet entries zeroed.  FP64 device arrays. */
nk_status nk_assemble(nk_system sys, const double* y_loc, double* b, void* stream);

/* x_loc_e = A_e x: gather of global coefficients to local ones.  FP64. */
nk_status nk_gather(nk_system sys, const double* x, double* x_loc, void* stream);

/* Jacobi diagonal of the assembled operator (Dirichlet rows = 1).  FP64
 * device [nglobal]. */
nk_status nk_system_diagonal(nk_system sys, double* diag, void* stream);

/* Solve R A R x = b by Jacobi-preconditioned CG.  b, x: device FP64
 * [nglobal] (x: initial guess in, solution out; Dirichlet entries of x are
 * forced to zero).  NK_OK means that the true residual, recomputed in FP64
 * from the returned x, satisfies ||b - A x||_2 <= rtol ||b||_2 for every
 * system (info.rel_resid is that ratio).  maxit bounds the CG iterations of a
 * system in total.  NK_SOLVE_F64: FP64 throughout; CG stops on its recursive
 * residual, and while the true residual is still above rtol (the two drift
 * apart by rounding) it restarts from the current x, within the budget.
 * NK_SOLVE_F32_REFINED: one CG whose operator and vectors run in FP32 (dot
 * products accumulated in FP64), with reliable updates in FP64: whenever the
 * FP32 residual has fallen by NK_RELIABLE_DELTA (default 0.3) since the last
 * update (or the FP32
 * iteration stops), its solution increment is added to the FP64 x and its
 * residual is replaced by the true FP64 residual b - A x, keeping the search
 * direction; the solve ends on the true residual of the returned x, and maxit
 * bounds the FP32 iterations.  (Environment NK_REFINE=restart selects plain
 * iterative refinement instead: FP32 CG solves of the FP64 residual equation,
 * each reducing its residual by NK_INNER_TOL, default 1e-4.)
 * NK_SOLVE_CONDENSED (section 2.1, static condensation): FP64 CG on the
 * system condensed onto the elemental boundary DOFs (nk_system_condense,
 * built on first use), preconditioned by the diagonal of S;
 * the interiors follow element by element, and the pass repeats on the full
 * residual b - A x until it meets rtol (iters: boundary CG iterations summed
 * over passes).  NK_SOLVE_CONDENSED_F32_REFINED: the same, with the boundary
 * system solved as NK_SOLVE_F32_REFINED solves (FP32 condensed operator from
 * an FP32 copy of the interior inverses, made on first use, with FP64
 * reliable updates; iters: FP32 boundary iterations).  Both: one-system
 * hexahedral systems (uniform or variable order) with every 2 <= P <= 6 only
 * (NK_EUNSUPPORTED otherwise).  Iterations run as captured HIP graphs that
 * do not depend on rtol or maxit.  info (host, may be NULL) receives one
 * entry per system (nsys entries for a batched system).  Returns NK_ENOCONV
 * (budget spent with the true residual above rtol) or NK_EBREAKDOWN if any
 * system did not converge. */
nk_status nk_cg_solve(nk_system sys, nk_solve_mode mode, const double* b, double* x,
                      double rtol, int maxit, nk_solve_info* info, void* stream);

/* Static condensation (section 2.1): the modified basis splits each
 * hexahedron's modes into boundary modes (index 0 or P in some direction,
 * shared with neighbours) and (P-1)^3 interior modes owned by the element, so
 * the system condenses onto the boundary DOFs with the elemental Schur
 * complements S_e = H_bb - H_bi H_ii^{-1} H_ib.  Builds (once per system;
 * later calls reuse it) the boundary system and the dense inverses H_ii^{-1}
 * of every element (symmetric, stored by diagonals: E (NI/2 + 1) NI doubles
 * of device memory, NI = (P-1)^3), and returns the
 * number of boundary DOFs in *nboundary (host).  bmap (device int32
 * [nboundary], may be NULL) receives the global DOF of each boundary DOF, in
 * increasing order; bdiag (device FP64 [nboundary], may be NULL) the
 * diagonal of S that preconditions the condensed solve (1 on Dirichlet
 * DOFs).  Requires a one-system system on a hexahedral space, uniform or
 * variable order (section 4.2: each order group has its own interior modes
 * and inverses), every order 2 <= P <= 6 with Q = P + 2 (else
 * NK_EUNSUPPORTED), and a map
 * whose interior modes each reference a DOF no other mode references and that
 * is not Dirichlet (else NK_EUNSUPPORTED).  Synchronises the stream. */
nk_status nk_system_condense(nk_system sys, int64_t* nboundary, int32_t* bmap, double* bdiag,
                             void* stream);

/* yb = S xb, the assembled condensed operator over the boundary numbering of
 * nk_system_condense (Dirichlet entries of xb read as zero, Dirichlet entries
 * of yb zero).  Device FP64 [nboundary].  Matrix-free: two sum-factorised
 * Helmholtz passes and one dense H_ii^{-1} product per element.  Requires a
 * prior nk_system_condense.  Synchronises the stream. */
nk_status nk_condensed_apply(nk_system sys, const double* xb, double* yb, void* stream);

/* Several separately created systems (their own spaces, orders and maps)
 * solved in one call, as nk_cg_solve solves each: sys, b, x are host arrays
 * of nsys entries (b[k], x[k]: device FP64 [nglobal of system k]); info
 * (host, may be NULL) receives one entry per system, NK_OK meaning the same
 * per-system true-residual criterion.  One-system hexahedral/quadrilateral
 * systems of one (dim, P, Q) are solved together as one batched system (the
 * library concatenates their factors, maps and coefficients into a cached
 * union), so each CG iteration runs one assembled-operator launch per order
 * class with per-system CG scalars, in captured HIP graphs; other systems
 * (mixed-order, collapsed shapes, already batched: their entry reports the
 * sub-system with the largest residual) run alongside, each on its own
 * stream.  The union of a member list is built on first use (a copy of the
 * members' factors: device memory comparable to their spaces) and kept for
 * later calls with the same list, at most four lists, until a member is
 * destroyed.  A system may appear once per call; all must live on the
 * current device.  NK_SOLVE_CONDENSED is not taken here (NK_EUNSUPPORTED).
 * Synchronises like nk_cg_solve. */
nk_status nk_cg_solve_batched(nk_system* sys, int nsys, nk_solve_mode mode,
                              const double* const* b, double* const* x, double rtol, int maxit,
                              nk_solve_info* info, void* stream);

/* Adjoint-gradient kernel for a loss of a Helmholtz solve: with u_loc and
 * z_loc the local (gathered) forward and adjoint solutions, writes
 *   dkappa[e][k] = -w_k detJ_k (grad_xi z)^T G (grad_xi u) at point k,
 *   dlambda[e]   = -z_e^T M_e u_e,
 * i.e. -z^T (dA/dtheta) u for theta = kappa (per point) and lambda (per
 * element).  Device FP64: z_loc, u_loc [E][n^d], dkappa [E][Q^d] (may be
 * NULL), dlambda [E] (may be NULL).  Requires a single-group 3-D or 2-D
 * space created with kappa (NULL kappa means kappa = 1). */
nk_status nk_helmholtz_param_grad(nk_space s, const double* z_loc, const double* u_loc,
                                  double* dkappa, double* dlambda, void* stream);

/* Time every compiled tile configuration of the operators in op_mask
 * (bit 0 BwdTrans, 1 IProductWRTBase, 2 Helmholtz, 3 assembled operator)
 * for this space's orders with HIP events and keep the fastest; results are
 * cached per (op, dim, P, Q, dtype, device name) in the file named by
 * NK_AUTOTUNE_CACHE (default: no file). */
nk_status nk_autotune(nk_space s, int op_mask, void* stream);

/* Name of the tile configuration currently selected for (op, dim, P, dtype)
 * ("" if none).  Host string owned by the library (thread-local buffer). */
const char* nk_tile_config(int op, int dim, int P, nk_dtype t);

/* Number of compiled tile configurations of (op, dim, P) (0 for a bad op). */
int nk_tile_count(int op, int dim, int P);

/* Force tile configuration `tile` (0 <= tile < nk_tile_count) for (op, dim,
 * P, dtype), op in {0 BwdTrans, 1 IProductWRTBase, 2 Helmholtz}; the
 * assembled operator follows the Helmholtz choice for systems created
 * afterwards.  NK_EINVAL for out-of-range arguments. */
nk_status nk_set_tile_config(int op, int dim, int P, nk_dtype t, int tile);

#ifdef __cplusplus
}
#endif

#endif /* NK_H */
