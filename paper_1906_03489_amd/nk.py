"""ctypes binding of the C ABI declared in include/nk.h.

Argument marshalling only: every operator, assembly step and solve runs in
the HIP library libnk.so.  Torch tensors provide device memory and the
current stream.  If the library is missing the import fails loudly; there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnk.so")

NK_OK, NK_EINVAL, NK_ENOMEM, NK_EDEVICE, NK_EHIP, NK_ENOCONV, NK_EBREAKDOWN, NK_EUNSUPPORTED = range(8)
F64, F32 = 0, 1
SOLVE_F64, SOLVE_F32_REFINED, SOLVE_CONDENSED, SOLVE_CONDENSED_F32_REFINED = 0, 1, 2, 3
OP_BWD, OP_IPROD, OP_HELM, OP_HELM_ASM = 0, 1, 2, 3
STATUS_NAMES = {0: "NK_OK", 1: "NK_EINVAL", 2: "NK_ENOMEM", 3: "NK_EDEVICE", 4: "NK_EHIP",
                5: "NK_ENOCONV", 6: "NK_EBREAKDOWN", 7: "NK_EUNSUPPORTED"}

# every symbol the header declares (checked by the host tests)
EXPORTS = [
    "nk_last_error", "nk_version", "nk_device_count", "nk_basis_tables", "nk_space_create",
    "nk_space_create_varp", "nk_space_destroy", "nk_space_sizes", "nk_bwd_trans",
    "nk_iprod_wrt_base", "nk_helmholtz", "nk_helmholtz_weak_rhs", "nk_system_create",
    "nk_system_create_batched", "nk_system_create_signed", "nk_system_destroy", "nk_system_apply",
    "nk_system_apply_noalloc", "nk_assemble", "nk_gather", "nk_system_diagonal", "nk_cg_solve",
    "nk_cg_solve_batched", "nk_helmholtz_param_grad", "nk_autotune",
    "nk_tile_config", "nk_tile_count", "nk_set_tile_config", "nk_space_set_strategy",
    "nk_space_get_strategy", "nk_phys_deriv", "nk_iprod_wrt_deriv_base", "nk_fwd_trans",
    "nk_tri_points", "nk_space_create_tri", "nk_tet_points", "nk_space_create_tet",
    "nk_space_create_prism", "nk_space_create_pyr", "nk_system_condense", "nk_condensed_apply",
]


class NkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("rel_resid", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("status", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load libnk.so (built in-tree by paper_1906_03489_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} missing "
                          "(run `python -m paper_1906_03489_amd.build`)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "nk_last_error": (ctypes.c_char_p, []),
        "nk_version": (i32, []),
        "nk_device_count": (i32, []),
        "nk_basis_tables": (i32, [i32, i32, vp, vp, vp, vp]),
        "nk_space_create": (i32, [pp, i32, i64, i32, i32, vp, vp, vp]),
        "nk_space_create_varp": (i32, [pp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "nk_space_destroy": (i32, [vp]),
        "nk_space_sizes": (i32, [vp, vp, vp, vp]),
        "nk_bwd_trans": (i32, [vp, i32, vp, vp, vp]),
        "nk_iprod_wrt_base": (i32, [vp, i32, vp, vp, vp]),
        "nk_helmholtz": (i32, [vp, i32, vp, dbl, vp, vp, vp]),
        "nk_helmholtz_weak_rhs": (i32, [vp, vp, dbl, vp, vp, vp, vp]),
        "nk_system_create": (i32, [pp, vp, i64, vp, vp, vp, dbl, vp]),
        "nk_system_create_batched": (i32, [pp, vp, i32, vp, vp, vp, vp, vp, dbl, vp]),
        "nk_system_create_signed": (i32, [pp, vp, i64, vp, vp, vp, vp, dbl, vp]),
        "nk_system_destroy": (i32, [vp]),
        "nk_system_apply": (i32, [vp, i32, vp, vp, vp]),
        "nk_system_apply_noalloc": (i32, [vp, i32, vp, vp, vp]),
        "nk_assemble": (i32, [vp, vp, vp, vp]),
        "nk_gather": (i32, [vp, vp, vp, vp]),
        "nk_system_diagonal": (i32, [vp, vp, vp]),
        "nk_cg_solve": (i32, [vp, i32, vp, vp, dbl, i32, vp, vp]),
        "nk_cg_solve_batched": (i32, [vp, i32, i32, vp, vp, dbl, i32, vp, vp]),
        "nk_helmholtz_param_grad": (i32, [vp, vp, vp, vp, vp, vp]),
        "nk_autotune": (i32, [vp, i32, vp]),
        "nk_tile_config": (ctypes.c_char_p, [i32, i32, i32, i32]),
        "nk_tile_count": (i32, [i32, i32, i32]),
        "nk_set_tile_config": (i32, [i32, i32, i32, i32, i32]),
        "nk_space_set_strategy": (i32, [vp, i32, i32]),
        "nk_space_get_strategy": (i32, [vp, i32]),
        "nk_phys_deriv": (i32, [vp, i32, vp, vp, vp]),
        "nk_iprod_wrt_deriv_base": (i32, [vp, i32, vp, vp, vp]),
        "nk_fwd_trans": (i32, [vp, i32, vp, vp, vp]),
        "nk_tri_points": (i32, [i32, vp, vp, vp, vp]),
        "nk_space_create_tri": (i32, [pp, i64, i32, i32, vp, vp, vp]),
        "nk_tet_points": (i32, [i32, vp, vp, vp, vp, vp, vp]),
        "nk_space_create_tet": (i32, [pp, i64, i32, i32, vp, vp, vp]),
        "nk_space_create_prism": (i32, [pp, i64, i32, i32, vp, vp, vp]),
        "nk_space_create_pyr": (i32, [pp, i64, i32, i32, vp, vp, vp]),
        "nk_system_condense": (i32, [vp, ctypes.POINTER(i64), vp, vp, vp]),
        "nk_condensed_apply": (i32, [vp, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status: int):
    if status != NK_OK:
        raise NkError(status, lib().nk_last_error().decode(errors="replace"))


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _tdtype(code):
    import torch
    return torch.float64 if code == F64 else torch.float32


def device_count() -> int:
    return int(lib().nk_device_count())


def tri_points(Q: int):
    """(eta1, w1, eta2, w2) of the library's collapsed triangle quadrature."""
    import numpy as np
    e1, w1 = np.zeros(Q), np.zeros(Q)
    e2, w2 = np.zeros(Q - 1), np.zeros(Q - 1)
    _check(lib().nk_tri_points(Q, e1.ctypes.data_as(ctypes.c_void_p), w1.ctypes.data_as(ctypes.c_void_p),
                               e2.ctypes.data_as(ctypes.c_void_p), w2.ctypes.data_as(ctypes.c_void_p)))
    return e1, w1, e2, w2


def tet_points(Q: int):
    """(eta1, w1, eta2, w2, eta3, w3) of the library's collapsed tetrahedron
    quadrature."""
    import numpy as np
    arrs = [np.zeros(Q), np.zeros(Q)] + [np.zeros(Q - 1) for _ in range(4)]
    _check(lib().nk_tet_points(Q, *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs]))
    return tuple(arrs)


def basis_tables(P: int, Q: int):
    """Host 1-D tables of the library: GLL x, w and B[Q, P+1], DB[Q, P+1]."""
    x = np.zeros(Q)
    w = np.zeros(Q)
    B = np.zeros((Q, P + 1))
    D = np.zeros((Q, P + 1))
    c = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    _check(lib().nk_basis_tables(P, Q, c(x), c(w), c(B), c(D)))
    return x, w, B, D


# ------------------------------------------------------------------ spaces

class Space:
    """A collection of same-shape elements (one or several orders)."""

    def __init__(self, handle, dim, groups):
        self.handle = ctypes.c_void_p(handle)
        self.dim = dim
        self.groups = groups            # list of (P, Q, nelem)

    @classmethod
    def create(cls, dim: int, P: int, Q: int, jac, kappa=None):
        import torch
        nelem = int(jac.shape[0]) if jac is not None else 0
        h = ctypes.c_void_p()
        _check(lib().nk_space_create(ctypes.byref(h), dim, nelem, P, Q,
                                     _ptr(jac, torch.float64, "jac"),
                                     _ptr(kappa, torch.float64, "kappa"), _stream()))
        return cls(h.value, dim, [(P, Q, nelem)])

    @classmethod
    def create_varp(cls, dim: int, Ps: Sequence[int], Qs: Sequence[int], jacs, kappas=None):
        import torch
        ng = len(Ps)
        Pa = (ctypes.c_int * ng)(*Ps)
        Qa = (ctypes.c_int * ng)(*Qs)
        ne = (ctypes.c_int64 * ng)(*[int(j.shape[0]) for j in jacs])
        ja = (ctypes.c_void_p * ng)(*[_ptr(j, torch.float64, "jac").value for j in jacs])
        ka = None
        if kappas is not None:
            ka = (ctypes.c_void_p * ng)(*[(_ptr(k, torch.float64, "kappa").value if k is not None else None)
                                          for k in kappas])
        h = ctypes.c_void_p()
        _check(lib().nk_space_create_varp(ctypes.byref(h), dim, ng, Pa, Qa, ne, ja, ka, _stream()))
        return cls(h.value, dim, [(P, Q, int(n)) for P, Q, n in zip(Ps, Qs, ne)])

    @classmethod
    def create_tri(cls, P: int, Q: int, jac, kappa=None):
        """Collapsed-coordinate triangles: jac [E, 2, 2, Q(Q-1)] FP64 on the GPU."""
        import torch
        E = int(jac.shape[0]) if jac.dim() > 1 else jac.numel() // (4 * Q * (Q - 1))
        h = ctypes.c_void_p()
        _check(lib().nk_space_create_tri(ctypes.byref(h), E, P, Q, _ptr(jac, torch.float64, "jac"),
                                         _ptr(kappa, torch.float64, "kappa"), _stream()))
        return cls(h.value, 2, [(P, Q, E)])

    @classmethod
    def create_tet(cls, P: int, Q: int, jac, kappa=None):
        """Collapsed-coordinate tetrahedra: jac [E, 3, 3, Q(Q-1)^2] FP64 on the GPU."""
        import torch
        E = int(jac.shape[0]) if jac.dim() > 1 else jac.numel() // (9 * Q * (Q - 1) ** 2)
        h = ctypes.c_void_p()
        _check(lib().nk_space_create_tet(ctypes.byref(h), E, P, Q, _ptr(jac, torch.float64, "jac"),
                                         _ptr(kappa, torch.float64, "kappa"), _stream()))
        return cls(h.value, 3, [(P, Q, E)])

    @classmethod
    def create_prism(cls, P: int, Q: int, jac, kappa=None):
        """Prisms (collapsed triangle x line): jac [E, 3, 3, Q^2 (Q-1)] FP64 on the GPU."""
        import torch
        E = int(jac.shape[0]) if jac.dim() > 1 else jac.numel() // (9 * Q * Q * (Q - 1))
        h = ctypes.c_void_p()
        _check(lib().nk_space_create_prism(ctypes.byref(h), E, P, Q, _ptr(jac, torch.float64, "jac"),
                                           _ptr(kappa, torch.float64, "kappa"), _stream()))
        return cls(h.value, 3, [(P, Q, E)])

    @classmethod
    def create_pyr(cls, P: int, Q: int, jac, kappa=None):
        """Pyramids: jac [E, 3, 3, Q^2 (Q-1)] FP64 on the GPU."""
        import torch
        E = int(jac.shape[0]) if jac.dim() > 1 else jac.numel() // (9 * Q * Q * (Q - 1))
        h = ctypes.c_void_p()
        _check(lib().nk_space_create_pyr(ctypes.byref(h), E, P, Q, _ptr(jac, torch.float64, "jac"),
                                         _ptr(kappa, torch.float64, "kappa"), _stream()))
        return cls(h.value, 3, [(P, Q, E)])

    STRATEGIES = {0: "persistent", 1: "persistent_2bpc", 2: "concurrent", 3: "sequential"}

    def set_strategy(self, dtype, strategy: int):
        _check(lib().nk_space_set_strategy(self.handle, dtype, int(strategy)))

    def get_strategy(self, dtype) -> int:
        return int(lib().nk_space_get_strategy(self.handle, dtype))

    def sizes(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().nk_space_sizes(self.handle, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def destroy(self):
        if self.handle:
            _check(lib().nk_space_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().nk_space_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def _out(t, like_numel, dtype, device):
    import torch
    return torch.empty(like_numel, dtype=dtype, device=device) if t is None else t


def bwd_trans(space: Space, coeffs, phys=None, dtype=F64):
    """phys = BwdTrans(coeffs) over all elements."""
    _, nc, npnt = space.sizes()
    td = _tdtype(dtype)
    phys = _out(phys, npnt, td, coeffs.device)
    _check(lib().nk_bwd_trans(space.handle, dtype, _ptr(coeffs, td, "coeffs"),
                              _ptr(phys, td, "phys"), _stream()))
    return phys


def iprod_wrt_base(space: Space, phys, coeffs=None, dtype=F64):
    _, nc, npnt = space.sizes()
    td = _tdtype(dtype)
    coeffs = _out(coeffs, nc, td, phys.device)
    _check(lib().nk_iprod_wrt_base(space.handle, dtype, _ptr(phys, td, "phys"),
                                   _ptr(coeffs, td, "coeffs"), _stream()))
    return coeffs


def phys_deriv(space: Space, phys, deriv=None, dtype=F64):
    """deriv[e, c, q] = d u / d x_c at the quadrature points (flat [E*d*Q^d])."""
    _, _, npnt = space.sizes()
    td = _tdtype(dtype)
    deriv = _out(deriv, npnt * space.dim, td, phys.device)
    _check(lib().nk_phys_deriv(space.handle, dtype, _ptr(phys, td, "phys"),
                               _ptr(deriv, td, "deriv"), _stream()))
    return deriv


def iprod_wrt_deriv_base(space: Space, f, coeffs=None, dtype=F64):
    """coeffs = IProductWRTDerivBase(f) for a vector field f [E][d][Q^d]."""
    _, nc, _ = space.sizes()
    td = _tdtype(dtype)
    coeffs = _out(coeffs, nc, td, f.device)
    _check(lib().nk_iprod_wrt_deriv_base(space.handle, dtype, _ptr(f, td, "f"),
                                         _ptr(coeffs, td, "coeffs"), _stream()))
    return coeffs


def fwd_trans(space: Space, phys, coeffs=None, dtype=F64):
    """coeffs = FwdTrans(phys): per-element L2 projection."""
    _, nc, _ = space.sizes()
    td = _tdtype(dtype)
    coeffs = _out(coeffs, nc, td, phys.device)
    _check(lib().nk_fwd_trans(space.handle, dtype, _ptr(phys, td, "phys"),
                              _ptr(coeffs, td, "coeffs"), _stream()))
    return coeffs


def solve_batched(systems, bs, xs=None, rtol: float = 1e-10, maxit: int = 20000, mode=SOLVE_F64,
                  raise_on_fail: bool = True):
    """nk_cg_solve_batched: separately created systems solved in one call.
    Returns ([x_k], [SolveInfo dict per system])."""
    import torch
    n = len(systems)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    handles = (ctypes.c_void_p * n)(*[s.handle for s in systems])
    bp = (ctypes.c_void_p * n)(*[_ptr(b, torch.float64, "b") for b in bs])
    xp = (ctypes.c_void_p * n)(*[_ptr(x, torch.float64, "x") for x in xs])
    infos = (SolveInfo * n)()
    st = lib().nk_cg_solve_batched(handles, n, int(mode), bp, xp, float(rtol), int(maxit), infos,
                                   _stream())
    if raise_on_fail:
        _check(st)
    return xs, [i.as_dict() for i in infos]


def filtered_fwd_trans(space: Space, system, phys, rtol: float = 1e-12, mode=SOLVE_F64):
    """The modified forward transform of Eq. (3): global C0 coefficients of
    u** with u** - alpha^2 lap u** = u*, du**/dn = 0, for point values u*
    (phys, [E][Q^d]).  The space must carry kappa = alpha^2 and the system
    lambda = 1 and no Dirichlet DOFs; the right-hand side is the assembled
    IProductWRTBase of u*.  Returns (coefficients, [SolveInfo dicts])."""
    b = system.assemble(iprod_wrt_base(space, phys))
    return system.solve(b, rtol=rtol, mode=mode)


def helmholtz(space: Space, x, y=None, lam=None, lam0: float = 1.0, dtype=F64):
    """y = (L + lambda M) x, elementwise (local), matrix-free."""
    import torch
    _, nc, _ = space.sizes()
    td = _tdtype(dtype)
    y = _out(y, nc, td, x.device)
    _check(lib().nk_helmholtz(space.handle, dtype, _ptr(lam, torch.float64, "lambda"), float(lam0),
                              _ptr(x, td, "x"), _ptr(y, td, "y"), _stream()))
    return y


def helmholtz_weak_rhs(space: Space, u, du, y=None, lam=None, lam0: float = 1.0):
    import torch
    _, nc, _ = space.sizes()
    y = _out(y, nc, torch.float64, u.device)
    _check(lib().nk_helmholtz_weak_rhs(space.handle, _ptr(lam, torch.float64, "lambda"), float(lam0),
                                       _ptr(u, torch.float64, "u"), _ptr(du, torch.float64, "du"),
                                       _ptr(y, torch.float64, "y"), _stream()))
    return y


def param_grad(space: Space, z_loc, u_loc, dkappa=None, dlambda=None):
    import torch
    ne, nc, npnt = space.sizes()
    dkappa = _out(dkappa, npnt, torch.float64, z_loc.device)
    dlambda = _out(dlambda, ne, torch.float64, z_loc.device)
    _check(lib().nk_helmholtz_param_grad(space.handle, _ptr(z_loc, torch.float64, "z_loc"),
                                         _ptr(u_loc, torch.float64, "u_loc"),
                                         _ptr(dkappa, torch.float64, "dkappa"),
                                         _ptr(dlambda, torch.float64, "dlambda"), _stream()))
    return dkappa, dlambda


def autotune(space: Space, op_mask: int = 0b111):
    _check(lib().nk_autotune(space.handle, int(op_mask), _stream()))


def tile_config(op: int, dim: int, P: int, dtype=F64) -> str:
    return lib().nk_tile_config(op, dim, P, dtype).decode()


def tile_count(op: int, dim: int, P: int) -> int:
    return int(lib().nk_tile_count(op, dim, P))


def set_tile_config(op: int, dim: int, P: int, dtype, tile: int):
    _check(lib().nk_set_tile_config(op, dim, P, dtype, tile))


# ----------------------------------------------------------------- systems

class System:
    """Assembled C0 system (one, or several independent ones batched)."""

    def __init__(self, handle, space, nglobal, nsys):
        self.handle = ctypes.c_void_p(handle)
        self.space = space
        self.nglobal = nglobal
        self.nsys = nsys

    @classmethod
    def create(cls, space: Space, nglobal: int, l2g, dirichlet, lam=None, lam0: float = 1.0, sign=None):
        """sign: optional int8 device tensor of +-1 per local mode (orientation)."""
        import torch
        h = ctypes.c_void_p()
        if sign is None:
            _check(lib().nk_system_create(ctypes.byref(h), space.handle, int(nglobal),
                                          _ptr(l2g, torch.int32, "l2g"), _ptr(dirichlet, torch.uint8, "dirichlet"),
                                          _ptr(lam, torch.float64, "lambda"), float(lam0), _stream()))
        else:
            _check(lib().nk_system_create_signed(ctypes.byref(h), space.handle, int(nglobal),
                                                 _ptr(l2g, torch.int32, "l2g"), _ptr(sign, torch.int8, "sign"),
                                                 _ptr(dirichlet, torch.uint8, "dirichlet"),
                                                 _ptr(lam, torch.float64, "lambda"), float(lam0), _stream()))
        return cls(h.value, space, int(nglobal), 1)

    @classmethod
    def create_batched(cls, space: Space, elem_off: Sequence[int], dof_off: Sequence[int], l2g, dirichlet,
                       lam=None, lam0: float = 1.0):
        import torch
        ns = len(elem_off) - 1
        eo = (ctypes.c_int64 * (ns + 1))(*[int(v) for v in elem_off])
        do = (ctypes.c_int64 * (ns + 1))(*[int(v) for v in dof_off])
        h = ctypes.c_void_p()
        _check(lib().nk_system_create_batched(ctypes.byref(h), space.handle, ns, eo, do,
                                              _ptr(l2g, torch.int32, "l2g"),
                                              _ptr(dirichlet, torch.uint8, "dirichlet"),
                                              _ptr(lam, torch.float64, "lambda"), float(lam0), _stream()))
        return cls(h.value, space, int(dof_off[-1]), ns)

    def apply(self, x, y=None, dtype=F64):
        td = _tdtype(dtype)
        y = _out(y, self.nglobal, td, x.device)
        _check(lib().nk_system_apply(self.handle, dtype, _ptr(x, td, "x"), _ptr(y, td, "y"), _stream()))
        return y

    def apply_noalloc(self, x, y, dtype=F64):
        """nk_system_apply_noalloc: y must be given (the call allocates nothing)."""
        td = _tdtype(dtype)
        _check(lib().nk_system_apply_noalloc(self.handle, dtype, _ptr(x, td, "x"), _ptr(y, td, "y"),
                                             _stream()))
        return y

    def assemble(self, y_loc, b=None):
        import torch
        b = _out(b, self.nglobal, torch.float64, y_loc.device)
        _check(lib().nk_assemble(self.handle, _ptr(y_loc, torch.float64, "y_loc"),
                                 _ptr(b, torch.float64, "b"), _stream()))
        return b

    def gather(self, x, x_loc=None):
        import torch
        _, nc, _ = self.space.sizes()
        x_loc = _out(x_loc, nc, torch.float64, x.device)
        _check(lib().nk_gather(self.handle, _ptr(x, torch.float64, "x"),
                               _ptr(x_loc, torch.float64, "x_loc"), _stream()))
        return x_loc

    def diagonal(self, d=None):
        import torch
        d = _out(d, self.nglobal, torch.float64, "cuda")
        _check(lib().nk_system_diagonal(self.handle, _ptr(d, torch.float64, "diag"), _stream()))
        return d

    def solve(self, b, x=None, rtol: float = 1e-10, maxit: int = 20000, mode=SOLVE_F64,
              raise_on_fail: bool = True):
        """Jacobi-PCG solve; returns (x, [SolveInfo dicts])."""
        import torch
        if x is None:
            x = torch.zeros_like(b)
        infos = (SolveInfo * self.nsys)()
        st = lib().nk_cg_solve(self.handle, int(mode), _ptr(b, torch.float64, "b"),
                               _ptr(x, torch.float64, "x"), float(rtol), int(maxit), infos, _stream())
        if raise_on_fail:
            _check(st)
        return x, [i.as_dict() for i in infos]

    def condense(self, with_map: bool = True, with_diag: bool = False):
        """nk_system_condense: builds the statically condensed boundary system
        (once); returns (nboundary, bmap int32 device tensor or None), plus
        diag(S) (FP64 device tensor) with with_diag."""
        import torch
        nb = ctypes.c_int64(0)
        _check(lib().nk_system_condense(self.handle, ctypes.byref(nb), None, None, _stream()))
        bmap = diag = None
        if with_map or with_diag:
            n = max(nb.value, 1)
            bmap = torch.empty(n, dtype=torch.int32, device="cuda") if with_map else None
            diag = torch.empty(n, dtype=torch.float64, device="cuda") if with_diag else None
            _check(lib().nk_system_condense(self.handle, ctypes.byref(nb), _ptr(bmap, torch.int32, "bmap"),
                                            _ptr(diag, torch.float64, "bdiag"), _stream()))
            bmap = bmap[:nb.value] if bmap is not None else None
            diag = diag[:nb.value] if diag is not None else None
        return (nb.value, bmap, diag) if with_diag else (nb.value, bmap)

    def condensed_apply(self, xb, yb=None):
        """nk_condensed_apply: yb = S xb over the boundary numbering."""
        import torch
        yb = _out(yb, xb.numel(), torch.float64, xb.device)
        _check(lib().nk_condensed_apply(self.handle, _ptr(xb, torch.float64, "xb"),
                                        _ptr(yb, torch.float64, "yb"), _stream()))
        return yb

    def destroy(self):
        if self.handle:
            _check(lib().nk_system_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            if self.handle:
                lib().nk_system_destroy(self.handle)
                self.handle = None
        except Exception:
            pass
