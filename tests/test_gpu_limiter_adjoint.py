"""GPU parity of the limiter and of the discrete adjoint against the oracle.

Limiter: the troubled-element test compares floating-point numbers, so an
element whose oracle margin (distance of the deciding quantity from its
threshold) is below 1e-9 relative may legitimately flip; such elements are
excluded, all others must agree exactly in their flag and to 1e-13 in
their values. Adjoint: FP64, 1e-12 relative to the largest entry."""

import numpy as np
import pytest

import inputs
from oracle import adjoint, cpr, euler, limiter
from tests.gpu_util import dev, host, make_solver, rel_err, say, torch

pytestmark = pytest.mark.gpu


def _blurred_riemann(g, width=0.03):
    x, y = g.coords()
    sx = 0.5 * (1 + np.tanh((x - 0.5) / width))
    sy = 0.5 * (1 + np.tanh((y - 0.5) / width))
    S = inputs.RIEMANN_QUADRANTS
    prim = [(S["NE"][k] * sx * sy + S["NW"][k] * (1 - sx) * sy + S["SW"][k] * (1 - sx) * (1 - sy)
             + S["SE"][k] * sx * (1 - sy)) for k in range(4)]
    return inputs.conserved_from_primitive(*prim)


def _margins(q, g, M):
    """Smallest relative distance, per element, of any quantity the
    troubled test compares from the value that would flip it."""
    qbar = cpr.element_means(q, g)
    qW, qE, qS, qN = limiter.face_means(q, g)
    out = np.full(qbar.shape[1:], np.inf)
    for axis, (lo, hi, h) in enumerate(((qW, qE, g.dx), (qS, qN, g.dy))):
        nlo, nhi = limiter._neighbour_means(qbar, g, axis)
        R, L = euler.eigenvectors(qbar, g.gamma, axis)
        ch = lambda v: np.einsum("abJI,bJI->aJI", L, v)
        up, um, dp, dm = ch(hi - qbar), ch(qbar - lo), ch(nhi - qbar), ch(qbar - nlo)
        bound = M * h * h
        scale = np.maximum.reduce([np.abs(up), np.abs(um), np.abs(dp), np.abs(dm),
                                   np.full_like(up, bound)]) + 1e-300
        for a in (up, um):
            for m in (np.abs(np.abs(a) - bound), np.abs(np.abs(a) - np.abs(dp)),
                      np.abs(np.abs(a) - np.abs(dm)), np.abs(a), np.abs(dp), np.abs(dm)):
                out = np.minimum(out, np.min(m / scale, axis=0))
    return out


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
def test_limiter_matches_oracle(P, bc):
    g = cpr.Grid(P=P, nx=21, ny=19, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=bc)
    q = _blurred_riemann(g)
    say("limiter", P, bc)
    M = 10.0
    ql, flags = limiter.limit(q, g, M=M, return_flags=True)
    s = make_solver(g, limiter=True, tvb_m=M)
    qd = dev(q)
    fd = torch().zeros((g.ny, g.nx), dtype=torch().int32, device="cuda")
    n = s.limit(qd, flags=fd, count=True)
    fg = host(fd).astype(bool)
    safe = _margins(q, g, M) > 1e-9
    assert flags.any()
    assert np.array_equal(fg[safe], flags[safe])
    assert n == int(fg.sum())
    qg = host(qd)
    both = safe & (fg == flags)
    assert np.max(np.abs(qg[:, both] - ql[:, both])) <= 1e-13 * max(1.0, np.max(np.abs(ql)))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["transmissive", "periodic"])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 17), (23, 1), (37, 11)])
def test_limiter_matches_oracle_degenerate_meshes(P, bc, nx, ny):
    """The limiter on a single element, a single column, a single row (each
    element its own neighbour across the periodic or transmissive boundary)
    and 37x11 elements (the limiter runs two lanes per element, 128 elements
    per workgroup: three full workgroups and a ragged fourth). The same bar
    as above: flags agree outside the decision margin, values to 1e-13 where
    the flags agree."""
    g = cpr.Grid(P=P, nx=nx, ny=ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc=bc)
    q = _blurred_riemann(g)
    say("limiter degenerate mesh", P, bc, nx, ny)
    M = 10.0
    ql, flags = limiter.limit(q, g, M=M, return_flags=True)
    s = make_solver(g, limiter=True, tvb_m=M)
    qd = dev(q)
    fd = torch().zeros((g.ny, g.nx), dtype=torch().int32, device="cuda")
    n = s.limit(qd, flags=fd, count=True)
    fg = host(fd).astype(bool)
    safe = _margins(q, g, M) > 1e-9
    assert np.array_equal(fg[safe], flags[safe])
    assert n == int(fg.sum())
    qg = host(qd)
    agree = fg == flags
    assert np.max(np.abs(qg[:, agree] - ql[:, agree])) <= 1e-13 * max(1.0, np.max(np.abs(ql)))


def test_limited_rk3_riemann_steps_match_oracle():
    """Four-quadrant Riemann data on a 48x48 P=2 transmissive mesh, limiter
    after every stage: three steps at the oracle's CFL 0.1 dt. Stage inputs
    are identical between the two sides as long as no flag flips, which the
    margins of this smooth-enough case avoid."""
    g = cpr.Grid(P=2, nx=48, ny=48, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive")
    x, y = g.coords()
    q = inputs.riemann_quadrants(x, y)
    say("limited rk3 riemann")
    flagged = [0]

    def lim(z):
        out, fl = limiter.limit(z, g, M=10.0, return_flags=True)
        flagged[0] += int(fl.sum())
        return out

    s = make_solver(g, limiter=True, tvb_m=10.0)
    qo = lim(q)
    qd = dev(q)
    s.limit(qd)
    assert rel_err(host(qd), qo) <= 1e-13
    for _ in range(3):
        dt = cpr.cfl_dt(qo, g, 0.1)
        qo = cpr.rk3_step(qo, dt, g, limit=lim)
        s.step(qd, dt, limit=True)
    assert rel_err(host(qd), qo) <= 1e-11
    # the running total counts every pass: the initial one and 3 per step
    assert flagged[0] > 0
    assert s.troubled_total() == flagged[0]
    assert s.troubled_total(reset=True) == flagged[0]
    assert s.troubled_total() == 0
    # diagonal symmetry of the GPU result
    qg = host(qd)
    qt = qg[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
    assert np.max(np.abs(qt - qg)) <= 1e-12


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("mesh", [(1, 1), (3, 5), (9, 8), (13, 11)], ids=lambda m: f"{m[0]}x{m[1]}")
def test_residual_vjp_matches_oracle(mesh, P, bc):
    nx, ny = mesh
    g = cpr.Grid(P=P, nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.5, bc=bc)
    q = inputs.random_state((ny, nx, P + 1, P + 1), seed=2000 + P + nx)
    v = np.random.default_rng(3000 + P).standard_normal(g.shape)
    say("vjp", P, nx, ny, bc)
    ref = adjoint.residual_vjp(q, v, g)
    s = make_solver(g)
    out = host(s.residual_vjp(dev(q), dev(v)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("P", [2, 3])
def test_adjoint_step_matches_oracle(P):
    g = cpr.Grid(P=P, nx=10, ny=9)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    lam = np.random.default_rng(4000 + P).standard_normal(g.shape)
    say("adjoint step", P)
    dt = 0.01
    ref = adjoint.rk3_adjoint_step(q, dt, lam, g)
    s = make_solver(g)
    out = host(s.adjoint_step(dev(q), dt, dev(lam)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    # in place (lam_n aliases lam_np1)
    ld = dev(lam)
    s.adjoint_step(dev(q), dt, ld, out=ld)
    assert np.max(np.abs(host(ld) - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
@pytest.mark.parametrize("mesh", [(200, 176), (199, 170)], ids=lambda m: f"{m[0]}x{m[1]}")
def test_residual_vjp_p4_large_meshes(mesh, bc):
    """P=4 in float64 (the split-layout transpose) on 550 tiles, more than
    the chip holds at once: nx even copies 16 bytes per lane into LDS, nx
    odd 4 bytes and leaves a ragged tile column."""
    nx, ny = mesh
    g = cpr.Grid(P=4, nx=nx, ny=ny, x0=0.0, x1=2.0, y0=0.0, y1=1.5, bc=bc)
    q = inputs.random_state((ny, nx, 5, 5), seed=6000 + nx)
    v = np.random.default_rng(6100 + ny).standard_normal(g.shape)
    say("vjp p4 large mesh", nx, ny, bc)
    ref = adjoint.residual_vjp(q, v, g)
    s = make_solver(g)
    out = host(s.residual_vjp(dev(q), dev(v)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("nx", [130, 131])
def test_adjoint_step_p4_large_meshes(nx):
    """The three transposes of an adjoint step at P=4 on 289 tiles, the last
    one with its two extra terms, also in place. A random state:
    on the vortex's far field the two Rusanov speeds of a face agree to
    about 1e-13, where the tie rule's threshold decides by rounding."""
    g = cpr.Grid(P=4, nx=nx, ny=130, x0=0.0, x1=2.0, y0=0.0, y1=1.5)
    q = inputs.random_state((130, nx, 5, 5), seed=6300 + nx)
    lam = np.random.default_rng(6200 + nx).standard_normal(g.shape)
    say("adjoint step p4 large mesh", nx)
    dt = 1e-4
    ref = adjoint.rk3_adjoint_step(q, dt, lam, g)
    s = make_solver(g)
    out = host(s.adjoint_step(dev(q), dt, dev(lam)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))
    ld = dev(lam)
    s.adjoint_step(dev(q), dt, ld, out=ld)
    assert np.max(np.abs(host(ld) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_rollout_gradient_matches_oracle_and_fd():
    """Rollout with checkpointing (every 3 of 8 steps) on a perturbed P=3
    vortex: the gradient of 1/2 ||rho(T) - rho_exact||^2_w equals the
    oracle's stored-state adjoint and central differences on 4 directions."""
    from paper_1709_01619_amd import Rollout
    t = torch()
    g = cpr.Grid(P=3, nx=8, ny=8)
    x, y = g.coords()
    V = inputs.Vortex()
    q0 = V.conserved(x, y)
    q0[0] += inputs.gaussian_perturbation(q0[0].shape, 1e-3, 0)
    dt, n = 0.02, 8
    rho_ex = V.conserved(x, y, dt * n)[0]
    say("rollout gradient")
    J_o, g_o = adjoint.gradient(q0, dt, n, g, rho_ex)
    s = make_solver(g)
    W = s.quad_weights()
    q0d = dev(q0).requires_grad_(True)
    qT = Rollout.apply(q0d, s, dt, n, 3)
    J = 0.5 * ((qT[0] - dev(rho_ex)) ** 2 * W).sum()
    J.backward()
    gg = host(q0d.grad)
    assert abs(J.item() - J_o) <= 1e-12 * J_o
    assert np.max(np.abs(gg - g_o)) <= 1e-11 * np.max(np.abs(g_o))
    for d in inputs.random_directions(g.shape, [1000, 1001, 1002, 1003]):
        h = 1e-6 * np.max(np.abs(q0)) / np.max(np.abs(d))
        Jp = adjoint.misfit(cpr.run(q0 + h * d, g, dt, n), rho_ex, g)
        Jm = adjoint.misfit(cpr.run(q0 - h * d, g, dt, n), rho_ex, g)
        fd = (Jp - Jm) / (2 * h)
        ad = float(np.sum(gg * d))
        assert abs(fd - ad) <= 1e-6 * abs(ad)


def test_adjoint_rejected_with_limiter():
    from paper_1709_01619_amd import _lib
    g = cpr.Grid(P=2, nx=4, ny=4)
    s = make_solver(g, limiter=True)
    q = dev(inputs.random_state((4, 4, 3, 3), seed=1))
    with pytest.raises(_lib.CprError) as ei:
        s.adjoint_step(q, 0.01, q.clone())
    assert ei.value.status == _lib.CPR_EUNSUPPORTED


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("mesh", [(8, 8), (10, 9)], ids=lambda m: f"{m[0]}x{m[1]}")
def test_residual_vjp_symmetric_vortex_ties(mesh, P):
    """The unperturbed vortex centred on an element face makes the two
    one-sided Rusanov speeds tie exactly (in exact arithmetic) along its
    centre lines while the face states differ; both sides use the mean of
    the two gradients there, so the result does not depend on rounding."""
    nx, ny = mesh
    g = cpr.Grid(P=P, nx=nx, ny=ny)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    v = np.random.default_rng(7).standard_normal(g.shape)
    say("vjp symmetric vortex", P, nx, ny)
    ref = adjoint.residual_vjp(q, v, g)
    s = make_solver(g)
    out = host(s.residual_vjp(dev(q), dev(v)))
    assert np.max(np.abs(out - ref)) <= 1e-12 * np.max(np.abs(ref))


def _vjp_fp32_scale(q, v, g):
    """Size of the terms the float32 transpose is formed from:
    (2/h)(||D||_1 + 2||g'||_inf) max||A(q)||_inf max|v|, with A the flux
    Jacobians and a Rusanov wave-speed bound added to their norm."""
    from oracle import tables
    T = tables.get(g.P)
    normD = np.max(np.sum(np.abs(T.D), axis=0))
    normg = max(np.max(np.abs(T.gLp)), np.max(np.abs(T.gRp)))
    A = max(np.max(np.sum(np.abs(euler.flux_jacobian(q, g.gamma, ax)), axis=s))
            for ax in (0, 1) for s in (0, 1))
    lam = np.max(euler.max_wave_speed(q, g.gamma))
    return 2.0 / min(g.dx, g.dy) * (normD + 2 * normg) * (A + 2 * lam) * np.max(np.abs(v))


@pytest.mark.parametrize("P", [1, 2, 3, 4])
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_residual_vjp_fp32_bulk(P, bc):
    """FP32-bulk transpose against the oracle's float64 one: the difference
    is float32 rounding of the line algebra, bounded by 64 units of 2^-24
    on the scale of the terms it is formed from."""
    g = cpr.Grid(P=P, nx=9, ny=8, x0=0.0, x1=2.0, y0=0.0, y1=1.5, bc=bc)
    q = inputs.random_state((8, 9, P + 1, P + 1), seed=5000 + P)
    v = np.random.default_rng(5100 + P).standard_normal(g.shape)
    say("vjp fp32_bulk", P, bc)
    ref = adjoint.residual_vjp(q, v, g)
    s = make_solver(g, precision="fp32_bulk")
    out = host(s.residual_vjp(dev(q), dev(v)))
    err = np.max(np.abs(out - ref))
    scale = _vjp_fp32_scale(q, v, g)
    print(f"fp32_bulk vjp P={P} {bc}: max err {err:.3e} = {err / np.max(np.abs(ref)):.2e} "
          f"of max|ref|, bound {64 * 2.0 ** -24 * scale:.3e}")
    assert err <= 64 * 2.0 ** -24 * scale


@pytest.mark.parametrize("P", [2, 3, 4])
def test_adjoint_step_fp32_bulk(P, monkeypatch):
    """FP32-bulk adjoint step (float32 transposes, float64 combinations with
    v, x and y) against the oracle's float64 transposes taken at the same
    stage states (the context's own, from cpr_rk3_step_stages, so that the
    float32 forward error of the recomputed states is not part of the
    comparison; cpr_adjoint_step recomputes exactly these, bit for bit).
    Each transpose J(q_s)^T lam_s enters scaled by at most dt, and an error
    in lam2 or lam1 reaches lam_n with a weight of at most 1 + dt |J|; the
    bound is twice the sum over the three transposes of dt 64 2^-24 times
    their term scale. The symmetric vortex has exact ties of the two Rusanov
    speeds along its centre lines; the float32 transpose recognises ties to
    2^-17 relative (above the rounding of its speeds), so the oracle is run
    with that threshold here, which makes both take the same subgradient."""
    monkeypatch.setattr(adjoint, "TIE_REL", 2.0 ** -17)
    t = torch()
    g = cpr.Grid(P=P, nx=10, ny=9)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    lam = np.random.default_rng(6600 + P).standard_normal(g.shape)
    dt = 0.01
    say("adjoint step fp32_bulk", P)
    s = make_solver(g, precision="fp32_bulk")
    qd = dev(q)
    q1d, q2d = t.empty_like(qd), t.empty_like(qd)
    s.step_stages(qd, dt, q1d, q2d, out=t.empty_like(qd))
    out = host(s.adjoint_step_stages(qd, q1d, q2d, dt, dev(lam)))
    assert np.array_equal(out, host(s.adjoint_step(qd, dt, dev(lam))))
    q1, q2 = host(q1d), host(q2d)
    lam2 = (2.0 / 3.0) * (lam + dt * adjoint.residual_vjp(q2, lam, g))
    lam1 = 0.25 * (lam2 + dt * adjoint.residual_vjp(q1, lam2, g))
    ref = lam1 + dt * adjoint.residual_vjp(q, lam1, g) + lam / 3.0 + 0.75 * lam2
    err = np.max(np.abs(out - ref))
    scale = sum(_vjp_fp32_scale(qs, ls, g) for qs, ls in ((q2, lam), (q1, lam2), (q, lam1)))
    bound = 2 * dt * 64 * 2.0 ** -24 * scale
    print(f"fp32_bulk adjoint step P={P}: max err {err:.3e}, bound {bound:.3e}")
    assert err <= bound
    # against the unmodified oracle (ties to 1e-12): the difference adds the
    # tie rule's own effect, 1/2 |jump| |grad lam_L - grad lam_R| per face on
    # the faces whose speeds differ by less than 2^-17 but more than 1e-12;
    # that term is measured as the difference of the oracle under the two
    # thresholds
    monkeypatch.setattr(adjoint, "TIE_REL", 1e-12)
    lam2 = (2.0 / 3.0) * (lam + dt * adjoint.residual_vjp(q2, lam, g))
    lam1 = 0.25 * (lam2 + dt * adjoint.residual_vjp(q1, lam2, g))
    ref12 = lam1 + dt * adjoint.residual_vjp(q, lam1, g) + lam / 3.0 + 0.75 * lam2
    tie = np.max(np.abs(ref - ref12))
    err12 = np.max(np.abs(out - ref12))
    print(f"fp32_bulk adjoint step P={P} vs the 1e-12 tie rule: max err {err12:.3e} "
          f"({err12 / np.max(np.abs(ref12)):.2e} relative), tie-rule term {tie:.3e}")
    assert err12 <= bound + tie


def test_rollout_gradient_fp32_bulk():
    """FP32-bulk rollout gradient (float32 residual and transposes, float64
    state and lam) against the oracle's float64 gradient on the perturbed
    P=3 vortex of test_rollout_gradient_matches_oracle_and_fd."""
    from paper_1709_01619_amd import Rollout
    g = cpr.Grid(P=3, nx=8, ny=8)
    x, y = g.coords()
    V = inputs.Vortex()
    q0 = V.conserved(x, y)
    q0[0] += inputs.gaussian_perturbation(q0[0].shape, 1e-3, 0)
    dt, n = 0.02, 8
    rho_ex = V.conserved(x, y, dt * n)[0]
    say("rollout gradient fp32_bulk")
    J_o, g_o = adjoint.gradient(q0, dt, n, g, rho_ex)
    s = make_solver(g, precision="fp32_bulk")
    W = s.quad_weights()
    q0d = dev(q0).requires_grad_(True)
    qT = Rollout.apply(q0d, s, dt, n, 3)
    J = 0.5 * ((qT[0] - dev(rho_ex)) ** 2 * W).sum()
    J.backward()
    gg = host(q0d.grad)
    rel = np.max(np.abs(gg - g_o)) / np.max(np.abs(g_o))
    print(f"fp32_bulk rollout gradient: misfit rel err {abs(J.item() - J_o) / J_o:.2e}, "
          f"gradient rel err {rel:.2e}")
    assert rel <= 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32_bulk"])
@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("nx", [13, 14])
def test_residual_vjp_misaligned_matches_aligned(nx, P, prec):
    """A cotangent 8 bytes past a 16-byte boundary takes the transpose
    kernel's 8-byte copies; aligned states move pairs (P >= 2, and for odd
    points per element only when nx is even). Same bits either way."""
    t = torch()
    g = cpr.Grid(P=P, nx=nx, ny=9, x0=0.0, x1=2.0, y0=0.0, y1=1.5)
    q = inputs.random_state((9, nx, P + 1, P + 1), seed=5100 + P)
    v = np.random.default_rng(5200 + P).standard_normal(g.shape)
    say("vjp misaligned", P, nx, prec)
    s = make_solver(g, precision=prec)
    qd = dev(q)
    va = dev(v)
    buf = t.empty(v.size + 1, dtype=t.float64, device="cuda")
    vm = buf[1:].view(v.shape)
    vm.copy_(va)
    assert vm.data_ptr() % 16 == 8
    oa = host(s.residual_vjp(qd, va))
    om = host(s.residual_vjp(qd, vm))
    assert np.array_equal(oa, om)
    if prec == "fp64":
        ref = adjoint.residual_vjp(q, v, g)
        assert np.max(np.abs(oa - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("scheme", ["gl_lp", "gll_chain", "gll_lp"])
def test_step_and_adjoint_with_stage_states(P, scheme):
    """cpr_rk3_step_stages returns the oracle's stage states and the same
    step as cpr_rk3_step, in place or out of place; cpr_adjoint_step_stages
    given them equals cpr_adjoint_step bit for bit; aliasing is rejected."""
    from paper_1709_01619_amd import _lib
    t = torch()
    g = cpr.Grid(P=P, nx=10, ny=9, scheme=scheme)
    x, y = g.coords()
    q = inputs.Vortex().conserved(x, y)
    lam = np.random.default_rng(6000 + P).standard_normal(g.shape)
    say("stage states", P, scheme)
    dt = 0.01
    s = make_solver(g)
    qa, qb = dev(q), dev(q)
    q1, q2 = t.empty_like(qa), t.empty_like(qa)
    s.step(qa, dt)
    q0 = dev(q)
    qo = t.empty_like(qa)
    s.step_stages(q0, dt, q1, q2, out=qo)          # out of place: q_n is kept
    assert t.equal(qo, qa) and t.equal(q0, dev(q))
    s.step_stages(qb, dt, q1, q2)
    assert t.equal(qa, qb)
    _, o1, o2, _ = cpr.rk3_stages(q, dt, g)
    assert rel_err(host(q1), o1) <= 1e-12 and rel_err(host(q2), o2) <= 1e-12
    ref = host(s.adjoint_step(dev(q), dt, dev(lam)))
    out = host(s.adjoint_step_stages(dev(q), q1, q2, dt, dev(lam)))
    assert np.array_equal(out, ref)
    ld = dev(lam)
    s.adjoint_step_stages(dev(q), q1, q2, dt, ld, out=ld)     # lam_n may alias lam_np1
    assert np.array_equal(host(ld), ref)
    with pytest.raises(_lib.CprError) as ei:
        s.step_stages(qb, dt, q1, q1)
    assert ei.value.status == _lib.CPR_EINVAL
    with pytest.raises(_lib.CprError) as ei:
        s.step_stages(qb, dt, q1, q2, out=q2)
    assert ei.value.status == _lib.CPR_EINVAL
    with pytest.raises(_lib.CprError) as ei:
        s.adjoint_step_stages(qb, q1, q2, dt, dev(lam), out=q1)
    assert ei.value.status == _lib.CPR_EINVAL
