"""The allocation-free assembled operator (nk_system_apply_noalloc) against
nk_system_apply, through the C ABI: two calls in a row, the second on a
smaller system, in FP64 and FP32; device memory unchanged across calls; a
system whose staging does not fit the static array is rejected."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.assembly import MaskedOperator
from gpu_common import FP32_RTOL, FP64_RTOL, assert_close, jacobians, nk, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _system(shape, P, lam_seed, amp=W.WARP_AMPLITUDE):
    m = nk()
    Q = P + 2
    Jg, Jo, lat = jacobians(shape, P, amp)
    lam = np.random.default_rng(lam_seed).uniform(0.5, 2.0, lat.nelem)
    l2g, ng, dm = W.lattice_l2g(shape, P)
    space = m.Space.create(3, P, Q, to_dev(Jg))
    sysm = m.System.create(space, ng, to_dev(l2g), to_dev(dm), lam=to_dev(lam))
    return dict(space=space, sys=sysm, ng=ng, l2g=l2g, dm=dm, Jo=Jo, lam=lam, P=P, Q=Q)


def test_noalloc_apply_matches_apply_on_two_calls():
    torch = torch_cuda()
    m = nk()
    big = _system((4, 3, 3), 5, 21)
    small = _system((2, 2, 2), 3, 22)
    cases = []
    for k, c in enumerate((big, small)):
        x = np.random.default_rng(30 + k).uniform(-1, 1, c["ng"])
        ref = c["sys"].apply(to_dev(x)).cpu().numpy()
        ops = oracle.ElementOps(3, c["P"], c["Q"], c["Jo"], lam=c["lam"])
        oref = MaskedOperator(oracle.helmholtz_matrices(ops), c["l2g"], c["ng"], c["dm"])(x)
        ref32 = c["sys"].apply(to_dev(x, torch.float32), dtype=m.F32).double().cpu().numpy()
        cases.append((c, x, ref, oref, ref32))
    outs = [(torch.empty(c["ng"], dtype=torch.float64, device="cuda"),
             torch.empty(c["ng"], dtype=torch.float32, device="cuda"),
             to_dev(x), to_dev(x, torch.float32)) for c, x, *_ in cases]
    torch.cuda.synchronize()
    for rep in range(2):
        free0 = torch.cuda.mem_get_info()[0]
        # the big system first, then the smaller one: the second call must not
        # see anything the first left in the shared staging
        for (c, x, ref, oref, ref32), (y64, y32, x64, x32) in zip(cases, outs):
            y64.fill_(np.nan)
            y32.fill_(np.nan)
            c["sys"].apply_noalloc(x64, y64)
            c["sys"].apply_noalloc(x32, y32, dtype=m.F32)
            torch.cuda.synchronize()
            got = y64.cpu().numpy()
            assert_close(got, ref, FP64_RTOL, f"noalloc f64 n={c['ng']} rep={rep}")
            assert_close(got, oref, FP64_RTOL, f"noalloc f64 vs oracle n={c['ng']}")
            assert_close(y32.double().cpu().numpy(), ref32, FP32_RTOL, f"noalloc f32 n={c['ng']}")
        if rep == 1:
            # after the first round every kernel is loaded: later calls take
            # no device memory
            assert torch.cuda.mem_get_info()[0] == free0


def test_noalloc_apply_rejects_oversize_and_fits_fp32():
    """21^3 hexes at P = 8: 4 826 809 DOFs.  Two padded FP64 vectors exceed
    the 64 MiB static staging (rejected before any device work); two FP32
    vectors fit, and match nk_system_apply."""
    torch = torch_cuda()
    m = nk()
    c = _system((21, 21, 21), 8, 23, amp=0.0)
    x = np.random.default_rng(40).uniform(-1, 1, c["ng"])
    y64 = torch.zeros(c["ng"], dtype=torch.float64, device="cuda")
    with pytest.raises(m.NkError) as ei:
        c["sys"].apply_noalloc(to_dev(x), y64)
    assert ei.value.status == m.NK_EINVAL and "static scratch" in str(ei.value)
    assert float(y64.abs().max()) == 0.0
    x32 = to_dev(x, torch.float32)
    ref32 = c["sys"].apply(x32, dtype=m.F32).double().cpu().numpy()
    y32 = torch.empty(c["ng"], dtype=torch.float32, device="cuda")
    c["sys"].apply_noalloc(x32, y32, dtype=m.F32)
    torch.cuda.synchronize()
    assert_close(y32.double().cpu().numpy(), ref32, FP32_RTOL, "noalloc f32 21^3 P=8")
