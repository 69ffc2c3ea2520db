"""cpr_rk3_step_static (the entry point that allocates nothing) against
cpr_rk3_step on a context, through the C ABI: bit-identical states on two
calls in a row, the second with a smaller input, and its error paths."""

from ctypes import byref, c_void_p

import numpy as np
import pytest

import inputs
from oracle import cpr
from tests.gpu_util import dev, host, say, torch

pytestmark = pytest.mark.gpu


def _lib():
    from paper_1709_01619_amd import _lib as L
    return L, L.load()


def _state(P, nx, ny, seed):
    g = cpr.Grid(P=P, nx=nx, ny=ny)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    q[0] += inputs.gaussian_perturbation(q[0].shape, 1e-3, seed)
    return q


def _step_ctx(L, lib, cfg, q0, dt):
    """cpr_rk3_step on a context made from cfg (the allocating path)."""
    t = torch()
    ctx = c_void_p()
    stream = t.cuda.current_stream().cuda_stream
    L.check(lib.cpr_init(byref(cfg), c_void_p(stream), byref(ctx)), what="cpr_init")
    try:
        q = dev(q0)
        L.check(lib.cpr_rk3_step(ctx, c_void_p(q.data_ptr()), dt, 0), ctx, "cpr_rk3_step")
        L.check(lib.cpr_sync(ctx), ctx, "cpr_sync")
        return host(q)
    finally:
        lib.cpr_destroy(ctx)


def _step_static(L, lib, cfg, q0, dt, flag):
    t = torch()
    q = dev(q0)
    stream = t.cuda.current_stream().cuda_stream
    st = lib.cpr_rk3_step_static(byref(cfg), c_void_p(stream), c_void_p(q.data_ptr()), dt,
                                 c_void_p(flag.data_ptr()) if flag is not None else c_void_p(0))
    L.check(st, what="cpr_rk3_step_static: " + lib.cpr_last_error(None).decode())
    t.cuda.synchronize()
    return host(q)


@pytest.mark.parametrize("precision", ["fp64", "fp32_bulk"])
def test_static_step_matches_context_step_twice(precision):
    L, lib = _lib()
    t = torch()
    prec = L.CPR_FP64 if precision == "fp64" else L.CPR_FP32_BULK
    flag = t.zeros(1, dtype=t.int32, device="cuda")
    # first call: P=3 on 40 x 36 elements (ragged tiles); second: P=2 on 13 x 9
    cases = [(3, 40, 36, 0, 2e-3), (2, 13, 9, 1, 5e-3)]
    for P, nx, ny, seed, dt in cases:
        say("static step", precision, P, nx, ny)
        cfg = L.make_config(P, nx, ny, precision=prec)
        q0 = _state(P, nx, ny, seed)
        ref = _step_ctx(L, lib, cfg, q0, dt)
        got = _step_static(L, lib, cfg, q0, dt, flag)
        assert np.array_equal(got, ref), (P, nx, ny, float(np.max(np.abs(got - ref))))
        assert int(flag.item()) == 0
        # and the flag-less form, whose flag word lives in the static array
        got2 = _step_static(L, lib, cfg, q0, dt, None)
        assert np.array_equal(got2, ref)


def test_static_step_chain_scheme_matches_context_step():
    L, lib = _lib()
    say("static step chain scheme")
    cfg = L.make_config(3, 24, 17, scheme=L.CPR_SCHEME_GLL_CHAIN)
    g = cpr.Grid(P=3, nx=24, ny=17, scheme="gll_chain")
    x, y = g.coords()
    q0 = inputs.Vortex().conserved(x, y)
    ref = _step_ctx(L, lib, cfg, q0, 3e-3)
    got = _step_static(L, lib, cfg, q0, 3e-3, None)
    assert np.array_equal(got, ref)


def test_static_step_at_the_size_limit():
    """The largest state the static array serves (P=3 on 256 x 256, 2^22
    values) advances exactly as the context path does."""
    L, lib = _lib()
    say("static step at the 2^22-value limit")
    cfg = L.make_config(3, 256, 256)
    q0 = _state(3, 256, 256, 3)
    ref = _step_ctx(L, lib, cfg, q0, 1e-3)
    got = _step_static(L, lib, cfg, q0, 1e-3, None)
    assert np.array_equal(got, ref)


def test_static_step_rejects_what_it_does_not_serve():
    L, lib = _lib()
    t = torch()
    say("static step error paths")
    q = t.zeros(4, dtype=t.float64, device="cuda")
    qp = c_void_p(q.data_ptr())
    big = L.make_config(4, 512, 512)  # 26.2M values > 2^22
    assert lib.cpr_rk3_step_static(byref(big), None, qp, 1e-3, None) == L.CPR_EUNSUPPORTED
    assert b"static scratch limit" in lib.cpr_last_error(None)
    lim = L.make_config(2, 8, 8, limiter=L.CPR_LIM_TVB_CHAR)
    assert lib.cpr_rk3_step_static(byref(lim), None, qp, 1e-3, None) == L.CPR_EUNSUPPORTED
    ok = L.make_config(2, 8, 8)
    assert lib.cpr_rk3_step_static(byref(ok), None, qp, 0.0, None) == L.CPR_EINVAL
    assert lib.cpr_rk3_step_static(byref(ok), None, None, 1e-3, None) == L.CPR_EINVAL
    bad = L.make_config(2, 8, 8, gamma=1.0)
    assert lib.cpr_rk3_step_static(byref(bad), None, qp, 1e-3, None) == L.CPR_EINVAL


def test_static_step_flags_nonphysical_state():
    L, lib = _lib()
    t = torch()
    say("static step non-physical flag")
    cfg = L.make_config(2, 8, 8)
    q0 = _state(2, 8, 8, 0)
    q0[0, 3, 4, 1, 1] = -1.0
    flag = t.zeros(1, dtype=t.int32, device="cuda")
    _step_static(L, lib, cfg, q0, 1e-3, flag)
    assert int(flag.item()) == 1
