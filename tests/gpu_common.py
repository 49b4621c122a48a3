"""Shared helpers of the GPU parity tests (imported by tests only).

Each side evaluates the shared analytic geometry at its own quadrature
points: the GPU library's GLL points (nk_basis_tables) for the device inputs,
the oracle's for the oracle inputs.  Seeded data come from `workloads`.
"""
import numpy as np

import oracle
import workloads as W

FP64_RTOL = 1e-12     # relative 2-norm over the whole output
FP32_RTOL = 2e-6      # stated FP32 bound (checked per result)


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def nk():
    from paper_1906_03489_amd import nk as m
    return m


def lib_points(P, Q):
    return nk().basis_tables(P, Q)[0]


def jacobians(shape, P, amp, nelem=None):
    """(J for the GPU, J for the oracle, lattice) on the lattice `shape`."""
    Q = P + 2
    lat = W.lattice(shape)
    Jg = W.element_jacobians(lib_points(P, Q), lat, amp)
    Jo = W.element_jacobians(oracle.gll(Q)[0], lat, amp)
    if nelem is not None:
        Jg, Jo = Jg[:nelem], Jo[:nelem]
    return np.ascontiguousarray(Jg), np.ascontiguousarray(Jo), lat


def to_dev(a, dtype=None):
    torch = torch_cuda()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def rel_err(y, ref):
    y = np.asarray(y, np.float64).ravel()
    ref = np.asarray(ref, np.float64).ravel()
    n = np.linalg.norm(ref)
    return np.linalg.norm(y - ref) / (n if n > 0 else 1.0)


def assert_close(y, ref, rtol, what=""):
    e = rel_err(y, ref)
    assert e <= rtol, f"{what}: relative error {e:.3e} > {rtol:.1e}"
    # elementwise: no single entry may be off by more than 100 x rtol of the max
    d = np.abs(np.asarray(y, np.float64).ravel() - np.asarray(ref, np.float64).ravel()).max()
    m = np.abs(np.asarray(ref)).max()
    assert d <= 100 * rtol * max(m, 1e-300), f"{what}: max abs diff {d:.3e} vs max {m:.3e}"
    return e


U64 = 2.0 ** -53


def residual_allowance(mats, l2g, nglobal, dirichlet, x, b):
    """Rounding scale of one FP64 evaluation of ||b - A x|| / ||b||.

    Each entry of A x is a sum of k products (k = local modes per element
    times the elements meeting at a vertex, 8); its rounding error is about
    sqrt(k) u (|A| |x|)_i at most in the probabilistic model (u = 2^-53), so
    two independent evaluations (the library's and the oracle's) of the
    relative residual differ by at most 2 sqrt(k) u |||A||x|||_2 / ||b||_2.
    The library's NK_OK guarantees its own value <= rtol; the oracle's may
    exceed rtol by this much and no more."""
    from oracle.assembly import MaskedOperator
    k = max(np.shape(H)[1] for H in mats) * 8
    absA = MaskedOperator([np.abs(H) for H in mats], l2g, nglobal, dirichlet)
    return 2.0 * np.sqrt(k) * U64 * np.linalg.norm(absA(np.abs(x))) / np.linalg.norm(b)


def assert_true_residual(info, rtol, A, mats, l2g, nglobal, dirichlet, x, b, what=""):
    """NK_OK, the library's true residual <= rtol exactly, and the oracle's
    own residual of x <= rtol up to the rounding of one evaluation."""
    assert info["status"] == 0, f"{what}: status {info['status']}"
    assert info["rel_resid"] <= rtol, f"{what}: library residual {info['rel_resid']:.3e} > {rtol:.1e}"
    res = np.linalg.norm(b - A(x)) / np.linalg.norm(b)
    allow = residual_allowance(mats, l2g, nglobal, dirichlet, x, b)
    assert res <= rtol + allow, f"{what}: oracle residual {res:.3e} > {rtol:.1e} + {allow:.1e}"
    return res
