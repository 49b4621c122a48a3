"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, validates arguments before touching a device, and its host
basis tables agree with the oracle's.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nk.h")


def _lib():
    from paper_1906_03489_amd import nk
    return nk, nk.lib()


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nk_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_and_library_exports_everything():
    nk, L = _lib()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(nk.EXPORTS) == names


def test_version_and_device_count_never_fail():
    _, L = _lib()
    assert L.nk_version() == 10000
    assert L.nk_device_count() >= 0


@pytest.mark.parametrize("P", [1, 2, 4, 6, 8, 10])
def test_library_basis_tables_match_oracle(P):
    nk, _ = _lib()
    Q = P + 2
    x, w, B, D = nk.basis_tables(P, Q)
    xo, wo = oracle.gll(Q)
    Bo, Do = oracle.modified_basis(P, xo)
    np.testing.assert_allclose(x, xo, atol=5e-15)
    np.testing.assert_allclose(w, wo, atol=5e-15)
    np.testing.assert_allclose(B, Bo, atol=5e-15)
    np.testing.assert_allclose(D, Do, atol=1e-13)


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_library_tables_have_the_reflection_symmetry_of_the_even_odd_kernels(P):
    """The hexahedral kernels read only the rows of the first ceil(Q/2) points
    and rebuild the others from the reflection x -> -x: the GLL points are
    symmetric, phi_p(-x) = s_p phi_{p*}(x) with p* swapping the vertex modes and
    s_p = -1 for even interior modes, and phi_p'(-x) = -s_p phi_{p*}'(x).  Then
    the even-odd split c -> (c_0 + c_P, c_1, c_3, ...), (c_0 - c_P, c_2, ...) with
    the members (1/2, phi_1, ...) and (-x/2, phi_2, ...) gives u(x_i) = E + O and
    u(x_{Q-1-i}) = E - O (derivatives likewise), which is checked here against
    the full tables on random coefficients."""
    nk, _ = _lib()
    Q, N = P + 2, P + 1
    x, _, B, D = nk.basis_tables(P, Q)
    np.testing.assert_allclose(x[::-1], -x, atol=1e-15)
    star = [N - 1] + list(range(1, N - 1)) + [0]
    sgn = np.array([1.0] + [(-1.0 if p % 2 == 0 else 1.0) for p in range(1, N - 1)] + [1.0])
    np.testing.assert_allclose(B[::-1], B[:, star] * sgn, atol=1e-14)
    np.testing.assert_allclose(D[::-1], -D[:, star] * sgn, atol=1e-12)
    c = np.random.default_rng(P).uniform(-1, 1, N)
    ce = np.r_[c[0] + c[P], c[1:P:2]]
    co = np.r_[c[0] - c[P], c[2:P:2]]
    H = (Q + 1) // 2
    for i in range(H):
        e = 0.5 * ce[0] + B[i, 1:P:2] @ ce[1:]
        o = -0.5 * x[i] * co[0] + B[i, 2:P:2] @ co[1:]
        ed = -0.5 * co[0] + D[i, 2:P:2] @ co[1:]
        od = D[i, 1:P:2] @ ce[1:]
        u, du = B @ c, D @ c
        assert abs(e + o - u[i]) < 1e-13 and abs(e - o - u[Q - 1 - i]) < 1e-13
        assert abs(ed + od - du[i]) < 1e-12 and abs(ed - od - du[Q - 1 - i]) < 1e-12


def test_invalid_arguments_rejected_before_device_work():
    nk, L = _lib()
    h = ctypes.c_void_p()
    assert L.nk_basis_tables(0, 2, None, None, None, None) == nk.NK_EINVAL
    assert L.nk_basis_tables(3, 3, None, None, None, None) == nk.NK_EINVAL
    assert L.nk_space_create(None, 3, 1, 2, 4, None, None, None) == nk.NK_EINVAL
    assert L.nk_space_create(ctypes.byref(h), 4, 1, 2, 4, None, None, None) == nk.NK_EINVAL
    assert L.nk_space_create(ctypes.byref(h), 3, -1, 2, 4, None, None, None) == nk.NK_EINVAL
    assert L.nk_space_create(ctypes.byref(h), 3, 1, 2, 4, None, None, None) == nk.NK_EINVAL
    assert b"jac" in L.nk_last_error()
    assert L.nk_space_create(ctypes.byref(h), 3, 1, 11, 13, ctypes.c_void_p(8), None, None) == nk.NK_EUNSUPPORTED
    assert L.nk_space_create(ctypes.byref(h), 3, 1, 6, 9, ctypes.c_void_p(8), None, None) == nk.NK_EUNSUPPORTED
    for f in ("nk_bwd_trans", "nk_iprod_wrt_base", "nk_phys_deriv", "nk_iprod_wrt_deriv_base",
              "nk_fwd_trans"):
        assert getattr(L, f)(None, 0, None, None, None) == nk.NK_EINVAL
    assert L.nk_helmholtz(None, 0, None, 1.0, None, None, None) == nk.NK_EINVAL
    assert L.nk_system_create(ctypes.byref(h), None, 5, None, None, None, 1.0, None) == nk.NK_EINVAL
    assert L.nk_cg_solve(None, 0, None, None, 1e-10, 10, None, None) == nk.NK_EINVAL
    assert L.nk_cg_solve(None, nk.SOLVE_CONDENSED, None, None, 1e-10, 10, None, None) == nk.NK_EINVAL
    nb = ctypes.c_int64(0)
    assert L.nk_system_condense(None, ctypes.byref(nb), None, None, None) == nk.NK_EINVAL
    assert L.nk_condensed_apply(None, None, None, None) == nk.NK_EINVAL
    assert L.nk_space_destroy(None) == nk.NK_EINVAL
    assert L.nk_system_destroy(None) == nk.NK_EINVAL
    assert L.nk_set_tile_config(2, 3, 6, 0, 99) == nk.NK_EINVAL
    assert L.nk_set_tile_config(9, 3, 6, 0, 0) == nk.NK_EINVAL
    # three vector tiles, each also in its lean and deep forms, all with the paired and the
    # point-by-point I stage, + the matrix-core variant
    assert L.nk_tile_count(2, 3, 6) == 19
    assert L.nk_set_tile_config(2, 3, 6, 0, 9) == nk.NK_OK
    assert L.nk_tile_config(2, 3, 6, 0).decode() == "epb1_thr64_pt"
    assert L.nk_set_tile_config(2, 3, 6, 0, 0) == nk.NK_OK
    # P = 8: two tiles x three forms x two I-stage forms (Q = 10 > 8: no matrix-core variant)
    assert L.nk_tile_count(2, 3, 8) == 12
    assert L.nk_tile_count(0, 3, 6) == 3      # BwdTrans: no lean form
    assert L.nk_tile_config(2, 3, 6, 0).decode().startswith("epb")


def test_no_device_reports_edevice():
    nk, L = _lib()
    if L.nk_device_count() > 0:
        pytest.skip("a device is present")
    h = ctypes.c_void_p()
    assert L.nk_space_create(ctypes.byref(h), 3, 1, 2, 4, ctypes.c_void_p(8), None, None) == nk.NK_EDEVICE
    assert b"device" in L.nk_last_error()


@pytest.mark.parametrize("Q", [3, 6, 12])
def test_library_triangle_quadrature_matches_oracle(Q):
    """The library's collapsed-triangle points and weights (Newton GLL, Radau
    weights by exactness) against the oracle's (scipy Jacobi roots, moments)."""
    import numpy as np
    from oracle import collapsed as C
    import oracle
    nk, L = _lib()
    e1, w1, e2, w2 = nk.tri_points(Q)
    x, w = oracle.gll(Q)
    np.testing.assert_allclose(e1, x, atol=1e-15)
    np.testing.assert_allclose(w1, w, atol=1e-15)
    xr, wr = C.gauss_radau_jacobi(Q - 1, 1.0, 0.0)
    np.testing.assert_allclose(e2, xr, atol=1e-14)
    np.testing.assert_allclose(w2, wr, atol=1e-13)
    assert L.nk_tri_points(2, None, None, None, None) == nk.NK_EINVAL


@pytest.mark.parametrize("Q", [3, 4, 7, 12])
def test_library_tetrahedron_quadrature_matches_oracle(Q):
    """The library's collapsed-tetrahedron rule (Golub-Welsch roots of
    P^{2,1}, Newton-polished, weights by exactness) against the oracle's
    (scipy Jacobi roots, Gauss-Jacobi moments)."""
    import numpy as np
    from oracle import collapsed as C
    nk, L = _lib()
    e1, w1, e2, w2, e3, w3 = nk.tet_points(Q)
    t1, tw1, t2, tw2 = nk.tri_points(Q)
    np.testing.assert_array_equal(e1, t1)
    np.testing.assert_array_equal(e2, t2)
    xr, wr = C.gauss_radau_jacobi(Q - 1, 2.0, 0.0)
    np.testing.assert_allclose(e3, xr, atol=1e-14)
    np.testing.assert_allclose(w3, wr, atol=1e-13)
    assert L.nk_tet_points(2, None, None, None, None, None, None) == nk.NK_EINVAL
