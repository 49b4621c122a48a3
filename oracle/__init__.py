"""Plain FP64 CPU oracle for the matrix-free spectral/hp operators.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the GPU library; both sides
read the same seeded inputs from `workloads`.

What it computes, and from which passage of Moxey et al., "Nektar++:
enhancing the capability and application of high-fidelity spectral/hp element
methods" (arXiv 1906.03489):

  basis      1-D Gauss-Lobatto-Legendre points and weights; the modified
             hierarchical C0 basis of section 2.1 (the unnumbered display
             defining phi_p) and its derivative.
  element    tensor-product bases (section 2.1 and the sum-factorisation
             display of section 3.3), geometric factors of the map chi_e
             (section 2.1), and the dense elemental matrices of BwdTrans,
             IProductWRTBase, mass, Laplacian and Helmholtz; PhysDeriv
             (collocation derivative and chain rule), IProductWRTDerivBase
             (the volume term of section 2.2) and FwdTrans (the projection of
             the listing in section 3.5, a dense solve with M_e).  Each operator is
             applied as a dense matrix-vector product: this is the "StdMat"
             strategy of section 3.3, the plain definition that
             sum-factorisation reorders exactly.
  assembly   C0 gather/scatter (section 2.1, assembly operator), Dirichlet
             restriction, Jacobi-preconditioned CG and a sparse direct solve of
             the weak problem of Eqs. (1)-(2).
  condense   static condensation of the assembled system onto the elemental
             boundary DOFs and the element-by-element interior recovery
             (section 2.1).
  grad       gradients of a solve's loss with respect to the per-element
             Helmholtz coefficient and the per-point diffusion coefficient.

Every function's docstring names the passage it follows or the reading taken
where the paper is silent.
"""
from .basis import gll, modified_basis, lagrange_derivative, jacobi_p
from .element import (tensor_bases, geometry, inverse_jacobian, collocation_derivatives,
                      ElementOps, bwd_trans, iprod_wrt_base, phys_deriv, iprod_deriv, fwd_trans,
                      helmholtz_apply, helmholtz_matrices, mass_matrices, weak_rhs)
from .assembly import (assemble_vector, gather, assembled_matrix, pcg, direct_solve,
                       jacobi_diagonal)
from .condense import Condensed, condensed_solve, interior_modes, schur_complement
from .grad import param_grad, loss_and_solution

__all__ = [
    "gll", "modified_basis", "lagrange_derivative", "jacobi_p",
    "tensor_bases", "geometry", "inverse_jacobian", "collocation_derivatives",
    "ElementOps", "bwd_trans", "iprod_wrt_base", "phys_deriv", "iprod_deriv", "fwd_trans",
    "helmholtz_apply", "helmholtz_matrices", "mass_matrices", "weak_rhs",
    "assemble_vector", "gather", "assembled_matrix", "pcg", "direct_solve",
    "jacobi_diagonal", "param_grad", "loss_and_solution",
    "Condensed", "condensed_solve", "interior_modes", "schur_complement",
]
