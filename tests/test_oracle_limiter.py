"""Pins for the oracle's TVB characteristic limiter: minmod algebra, mean
preservation, idempotence, no-op limits (M -> infinity, linear data in the
interior), detection at a jump, one-dimensional data, the diagonal
symmetry of the four-quadrant Riemann problem, and hand-computed values of
the troubled flags and limited slopes (a contact and an acoustic case)."""

import numpy as np
import pytest

import inputs
from oracle import cpr, limiter


def test_minmod_values():
    a = np.array([1.0, -2.0, 3.0, 0.0, 2.0])
    b = np.array([2.0, -1.0, -1.0, 1.0, 0.5])
    c = np.array([0.5, -3.0, 2.0, 1.0, 4.0])
    np.testing.assert_array_equal(limiter.minmod(a, b, c), [0.5, -1.0, 0.0, 0.0, 0.5])
    np.testing.assert_array_equal(limiter.tvb_minmod(a, b, c, 1.5), [1.0, -1.0, 0.0, 0.0, 0.5])


def _riemann_grid(n, P=2):
    return cpr.Grid(P=P, nx=n, ny=n, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="transmissive")


def _smoothed_riemann(g):
    """Quadrant data blurred with tanh fronts so several elements are
    partially limited, evaluated at the oracle's own points."""
    x, y = g.coords()
    sx = 0.5 * (1 + np.tanh((x - 0.5) / 0.03))
    sy = 0.5 * (1 + np.tanh((y - 0.5) / 0.03))
    S = inputs.RIEMANN_QUADRANTS
    prim = [(S["NE"][k] * sx * sy + S["NW"][k] * (1 - sx) * sy + S["SW"][k] * (1 - sx) * (1 - sy)
             + S["SE"][k] * sx * (1 - sy)) for k in range(4)]
    return inputs.conserved_from_primitive(*prim)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_mean_preserved_and_idempotent(P):
    g = _riemann_grid(12, P)
    q = _smoothed_riemann(g)
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    assert flags.any() and not flags.all()
    np.testing.assert_allclose(cpr.element_means(ql, g), cpr.element_means(q, g), atol=1e-14)
    # untouched elements are bitwise unchanged
    np.testing.assert_array_equal(ql[:, ~flags], q[:, ~flags])
    # limited elements are linear: second differences along i vanish for P >= 2
    if P >= 2:
        d2 = ql[..., 2:] - 2 * ql[..., 1:-1] + ql[..., :-2]
        T = g.tables()
        h = np.diff(T.xi)
        # nodes are not equispaced: check linearity through divided differences
        s1 = (ql[..., 1:] - ql[..., :-1]) / h
        assert np.max(np.abs(np.diff(s1, axis=-1)[:, flags])) < 1e-12
        del d2
    ql2, flags2 = limiter.limit(ql, g, M=10.0, return_flags=True)
    assert not flags2.any()
    np.testing.assert_array_equal(ql2, ql)


def test_large_m_is_noop():
    g = _riemann_grid(10)
    q = _smoothed_riemann(g)
    ql, flags = limiter.limit(q, g, M=1e30, return_flags=True)
    assert not flags.any()
    np.testing.assert_array_equal(ql, q)


def test_linear_data_untouched_in_interior():
    """Globally linear conserved data: the face deviations are exactly half
    the neighbour differences, so the TVB minmod returns them and interior
    elements pass. M = 1 keeps the TVB bound M h^2 below the deviations of
    the non-constant components (so the minmod branch is exercised) but far
    above roundoff in the components whose slope is zero."""
    g = _riemann_grid(8)
    x, y = g.coords()
    q = np.stack([1.0 + 0.3 * x + 0.2 * y, 0.1 * (1.0 + 0.3 * x + 0.2 * y),
                  -0.2 + 0.1 * x, 2.5 + 0.2 * x - 0.3 * y])
    ql, flags = limiter.limit(q, g, M=1.0, return_flags=True)
    assert not flags[1:-1, 1:-1].any()
    np.testing.assert_array_equal(ql[:, 1:-1, 1:-1], q[:, 1:-1, 1:-1])
    # a pure minmod (M = 0) would flag on roundoff-level zero slopes
    _, flags0 = limiter.limit(q, g, M=0.0, return_flags=True)
    assert flags0[1:-1, 1:-1].any()


def test_jump_is_detected():
    g = _riemann_grid(16)
    x, y = g.coords()
    q = inputs.riemann_quadrants(x, y)
    # shift the split off the element faces so the jump sits inside elements
    q = inputs.riemann_quadrants(x, y, split=(0.53, 0.53))
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    cols = np.where(flags.any(axis=0))[0]
    assert 8 in cols
    # far-field elements inside a quadrant (constant data) are not flagged
    assert not flags[2, 2] and not flags[13, 13]


def test_y_independent_data_keeps_zero_y_slope():
    g = cpr.Grid(P=2, nx=12, ny=4, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc="periodic")
    x, y = g.coords()
    rho = 1.0 + 0.5 * (x > 0.52) + 0.1 * np.sin(2 * np.pi * x)
    q = inputs.conserved_from_primitive(rho, 0.2 + 0 * x, 0 * x, 1.0 + 0 * x)
    ql, flags = limiter.limit(q, g, M=10.0, return_flags=True)
    assert flags.any()
    np.testing.assert_allclose(ql, np.broadcast_to(ql[:, :1, :, :1, :], ql.shape), atol=1e-14)


def test_riemann_diagonal_symmetry_one_limited_step():
    g = _riemann_grid(16)
    x, y = g.coords()
    q = inputs.riemann_quadrants(x, y)
    lim = lambda s: limiter.limit(s, g, M=10.0)
    q = lim(q)
    dt = cpr.cfl_dt(q, g, 0.1)
    q1 = cpr.rk3_step(q, dt, g, limit=lim)
    qt = q1[[0, 2, 1, 3]].transpose(0, 2, 1, 4, 3)
    np.testing.assert_allclose(qt, q1, atol=1e-12)


# ---- value pins of the limited reconstruction (Section 2.6, eq. limu, in
# its TVB characteristic form). Every expected number below is worked out by
# hand from chosen element means and in-element polynomials; on a mesh of
# unit elements (h = 1) the slope minmod((q_E - q_W)/h, D+/h, D-/h) of the
# characteristic fields reduces to plain numbers. P = 2 represents the
# quadratic profiles exactly, so element means and face means are exact.

GAMMA = 1.4


def _row_grid(nx, P=2):
    # unit elements: dx = dy = 1; one element row, transmissive
    return cpr.Grid(P=P, nx=nx, ny=1, x0=0.0, x1=float(nx), y0=0.0, y1=1.0, bc="transmissive")


def _profile(g, mean, sigma, kappa):
    """Per element I: mean[I] + sigma[I] (x - x_I) + kappa[I] ((x - x_I)^2 - 1/12),
    whose element mean is mean[I] (the quadratic term integrates to zero over a
    unit element) and whose face values give (f_E - f_W)/h = sigma[I]."""
    x, _ = g.coords()
    xc = np.arange(g.nx) + 0.5
    xo = x - xc[None, :, None, None]
    m = np.asarray(mean)[None, :, None, None]
    s = np.asarray(sigma)[None, :, None, None]
    k = np.asarray(kappa)[None, :, None, None]
    return m + s * xo + k * (xo * xo - 1.0 / 12.0), xo


def test_limited_slope_values_contact():
    """A y-independent contact: rho varies, u = 0.2, v = 0, p = 1. The jumps
    are multiples of the entropy eigenvector (1, u, 0, u^2/2), so after the
    characteristic step the limited x-slope is s_rho (1, u, 0, u^2/2) with
    s_rho = minmod(sigma, D+rho, D-rho). Element by element (h = 1, M h^2 =
    1e-9, far below every deviation used and far above rounding):
      I  mean  sigma kappa  D-    D+    u+ = s/2+k/6, u- = s/2-k/6   troubled  s_rho
      0  1.0   0     0      0     0     0, 0                         no        -
      1  1.0   0.5   0      0     1.0   0.25 > minmod -> 0           yes       minmod(0.5,1.0,0)=0
      2  2.0   1.2   0      1.0   0.4   0.6 > 0.4                    yes       minmod(1.2,0.4,1.0)=0.4
      3  2.4   0.3   1.2    0.4   0.6   0.35, -0.05 (sign)           yes       minmod(0.3,0.6,0.4)=0.3
      4  3.0  -0.2   0      0.6  -0.1   -0.1, sign mismatch          yes       minmod(-0.2,-0.1,0.6)=0
      5  2.9   0     0     -0.1   0     0, 0                         no        -
    Element 3 has the first argument as the smallest: dropping it (eq. limu's
    two-argument form) gives 0.4, doubling it gives 0.4; element 2's slope
    comes from D+."""
    g = _row_grid(6)
    rho, xo = _profile(g, [1.0, 1.0, 2.0, 2.4, 3.0, 2.9], [0.0, 0.5, 1.2, 0.3, -0.2, 0.0],
                       [0.0, 0.0, 0.0, 1.2, 0.0, 0.0])
    u = 0.2
    q = inputs.conserved_from_primitive(rho, u + 0 * rho, 0 * rho, 1.0 + 0 * rho, GAMMA)
    ql, flags = limiter.limit(q, g, M=1e-9, return_flags=True)
    np.testing.assert_array_equal(flags[0], [False, True, True, True, True, False])
    means = np.array([1.0, 1.0, 2.0, 2.4, 3.0, 2.9])[None, :, None, None]
    s_rho = np.array([0.0, 0.0, 0.4, 0.3, 0.0, 0.0])[None, :, None, None]
    rho_lim = means + s_rho * xo
    expect = np.stack([rho_lim, u * rho_lim, 0 * rho_lim,
                       1.0 / (GAMMA - 1.0) + 0.5 * u * u * rho_lim])
    tr = flags[0]
    np.testing.assert_allclose(ql[:, :, tr], expect[:, :, tr], rtol=0, atol=2e-14)
    np.testing.assert_array_equal(ql[:, :, ~tr], q[:, :, ~tr])


def _acoustic_vectors():
    """Right eigenvectors of the x flux Jacobian at Q = (rho 1, u 0.5, v 0,
    p 1/1.4), where c = 1 and H = c^2/(g-1) + u^2/2 = 2.625:
    r+ = (1, u + c, 0, H + u c) = (1, 1.5, 0, 3.125) and
    r- = (1, u - c, 0, H - u c) = (1, -0.5, 0, 2.125)."""
    Q = np.array([1.0, 0.5, 0.0, (1.0 / 1.4) / 0.4 + 0.125])
    rp = np.array([1.0, 1.5, 0.0, 3.125])
    rm = np.array([1.0, -0.5, 0.0, 2.125])
    return Q, rp, rm


def test_acoustic_vectors_are_eigenvectors():
    """The hand values of r+ and r- are eigenvectors of the x flux Jacobian
    at Q (complex-step Jacobian of the x flux (m, m^2/rho + p, m v, (e + p) u),
    written out here), eigenvalues u + c = 1.5 and u - c = -0.5."""
    Q, rp, rm = _acoustic_vectors()

    def fx(z):
        rho, m, n, e = z
        p = (GAMMA - 1.0) * (e - 0.5 * (m * m + n * n) / rho)
        return np.array([m, m * m / rho + p, m * n / rho, (e + p) * m / rho])

    J = np.zeros((4, 4))
    for m in range(4):
        z = Q.astype(complex)
        z[m] += 1e-30j
        J[:, m] = np.imag(fx(z)) / 1e-30
    np.testing.assert_allclose(J @ rp, 1.5 * rp, atol=1e-14)
    np.testing.assert_allclose(J @ rm, -0.5 * rm, atol=1e-14)


def test_limited_slope_values_acoustic():
    """Acoustic content in both families at the middle element (I = 1) of a
    three-element row, all relative to Q = its mean:
      q_E - q_W = 0.15 r+ + 0.10 r-      (sigma of each family)
      D+ = mean(2) - Q = 0.25 r+ + 0.05 r-
      D- = Q - mean(0) = 0.20 r+ + 0.15 r-
    plus a quadratic 1.5 ((x - x_I)^2 - 1/12) r+ that makes the face
    deviation of the + family 0.15/2 + 1.5/6 = 0.325 > 0.20, so the element is
    troubled. With the eigenvectors taken at the mean Q the families separate:
    s = minmod(0.15, 0.25, 0.20) r+ + minmod(0.10, 0.05, 0.15) r-
      = 0.15 r+ + 0.05 r- = (0.2, 0.2, 0, 0.575).
    Eigenvectors taken at a face state instead mix the families and change
    both minmods."""
    Q, rp, rm = _acoustic_vectors()
    g = _row_grid(3)
    x, _ = g.coords()
    xo = x - (np.arange(3) + 0.5)[None, :, None, None]
    mid = xo[0, 1]                       # x - x_I at the middle element's points
    plus = 0.15 * mid + 1.5 * (mid * mid - 1.0 / 12.0)
    q = np.empty((4, 1, 3) + mid.shape)
    q[:, 0, 1] = Q[:, None, None] + plus[None] * rp[:, None, None] + (0.10 * mid)[None] * rm[:, None, None]
    q[:, 0, 0] = (Q - 0.20 * rp - 0.15 * rm)[:, None, None]
    q[:, 0, 2] = (Q + 0.25 * rp + 0.05 * rm)[:, None, None]
    ql, flags = limiter.limit(q, g, M=1e-9, return_flags=True)
    assert flags[0, 1]
    s = np.array([0.2, 0.2, 0.0, 0.575])
    np.testing.assert_allclose(0.15 * rp + 0.05 * rm, s, atol=1e-15)   # the hand sum
    expect = Q[:, None, None] + s[:, None, None] * mid[None]
    np.testing.assert_allclose(ql[:, 0, 1], expect, rtol=0, atol=2e-14)
    np.testing.assert_allclose(cpr.element_means(ql, g)[:, 0, 1], Q, atol=1e-15)
