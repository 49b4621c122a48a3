"""MI355X-native matrix-free spectral/hp element operators.

The package is a thin binding over the HIP library libnk.so (C ABI in
include/nk.h): sum-factorised BwdTrans, IProductWRTBase and Helmholtz over
collections of same-shape elements (section 3.3 of arXiv 1906.03489),
PhysDeriv, IProductWRTDerivBase and an on-chip FwdTrans, the C0
assembled system and its Jacobi-preconditioned CG solve, a mixed-order
persistent launch, an FP32 solve inside FP64 iterative refinement, and
adjoint gradients behind torch.autograd.
"""
from .nk import (  # noqa: F401
    F32, F64, SOLVE_F32_REFINED, SOLVE_F64, OP_BWD, OP_IPROD, OP_HELM, OP_HELM_ASM,
    NkError, Space, System, autotune, basis_tables, bwd_trans, device_count, filtered_fwd_trans, fwd_trans, helmholtz,
    helmholtz_weak_rhs, iprod_wrt_base, iprod_wrt_deriv_base, lib, param_grad, phys_deriv,
    set_tile_config, tile_config, tile_count,
)
