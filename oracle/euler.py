"""2D Euler physics for the oracle (Section 2: state, flux and ideal-gas EOS
equations; Section 4: the Rusanov interface flux used for every method).

All functions take a leading variable axis of length 4 holding the conserved
state q = (rho, rho u, rho v, e) and broadcast over the remaining axes. They
accept complex arrays for complex-step differentiation: |.| and max are taken
with their real-part branch (abs_r, where(real(a) >= real(b))), which equals
the ordinary value for real input.
"""

from __future__ import annotations

import numpy as np


def abs_r(x):
    """|x| for real x; x*sign(Re x) for complex x (branch fixed by Re)."""
    if np.iscomplexobj(x):
        return x * np.where(x.real >= 0.0, 1.0, -1.0)
    return np.abs(x)


def max_r(a, b):
    """max(a, b) choosing by real part; ties take a (the '-' / left side)."""
    return np.where(np.real(a) >= np.real(b), a, b)


def pressure(q, gamma):
    """p = (gamma-1)(e - rho (u^2+v^2)/2)."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    return (gamma - 1.0) * (e - 0.5 * (mx * mx + my * my) / rho)


def flux_x(q, gamma):
    """f(q) = (rho u, p + rho u^2, rho u v, u (e + p))."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    p = pressure(q, gamma)
    return np.stack([mx, mx * u + p, my * u, u * (e + p)])


def flux_y(q, gamma):
    """g(q) = (rho v, rho u v, p + rho v^2, v (e + p))."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    p = pressure(q, gamma)
    return np.stack([my, mx * v, my * v + p, v * (e + p)])


def sound_speed(q, gamma):
    return np.sqrt(gamma * pressure(q, gamma) / q[0])


def normal_wave_speed(q, gamma, axis):
    """|u_n| + c with u_n = u (axis 0, x-faces) or v (axis 1, y-faces)."""
    un = q[1 + axis] / q[0]
    return abs_r(un) + sound_speed(q, gamma)


def max_wave_speed(q, gamma):
    """sqrt(u^2+v^2) + c, the speed in the CFL condition (Section 4)."""
    u = q[1] / q[0]
    v = q[2] / q[0]
    return np.sqrt(u * u + v * v) + sound_speed(q, gamma)


def rusanov(qL, qR, gamma, axis):
    """Rusanov (local Lax-Friedrichs) flux across a face with normal +x
    (axis 0) or +y (axis 1): 1/2 (F(qL) + F(qR)) - 1/2 lam (qR - qL), with
    lam = max(|u_n|+c) over the two sides."""
    F = flux_x if axis == 0 else flux_y
    lam = max_r(normal_wave_speed(qL, gamma, axis), normal_wave_speed(qR, gamma, axis))
    return 0.5 * (F(qL, gamma) + F(qR, gamma)) - 0.5 * lam * (qR - qL)


def flux_jacobian(q, gamma, axis):
    """A = df/dq (axis 0) or B = dg/dq (axis 1), shape (4, 4, ...), written out
    from the flux formulas with u, v, H = (e+p)/rho, phi = (gamma-1)(u^2+v^2)/2."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    p = pressure(q, gamma)
    H = (e + p) / rho
    gm = gamma - 1.0
    phi = 0.5 * gm * (u * u + v * v)
    z = 0.0 * u
    o = z + 1.0
    if axis == 0:
        rows = [
            [z, o, z, z],
            [phi - u * u, (3.0 - gamma) * u, -gm * v, z + gm],
            [-u * v, v, u, z],
            [u * (phi - H), H - gm * u * u, -gm * u * v, gamma * u],
        ]
    else:
        rows = [
            [z, z, o, z],
            [-u * v, v, u, z],
            [phi - v * v, -gm * u, (3.0 - gamma) * v, z + gm],
            [v * (phi - H), -gm * u * v, H - gm * v * v, gamma * v],
        ]
    return np.array([[np.asarray(c) for c in r] for r in rows])


def eigenvectors(q, gamma, axis):
    """Right and left eigenvector matrices (R, L), each (4, 4, ...), of the
    flux Jacobian in direction axis at state q; L = R^-1. Columns of R are
    ordered by eigenvalue u_n - c, u_n, u_n (shear), u_n + c."""
    rho, mx, my, e = q[0], q[1], q[2], q[3]
    u = mx / rho
    v = my / rho
    p = pressure(q, gamma)
    c = np.sqrt(gamma * p / rho)
    H = (e + p) / rho
    ke = 0.5 * (u * u + v * v)
    gm = gamma - 1.0
    b1 = gm / (c * c)
    b2 = ke * b1
    z = 0.0 * u
    o = z + 1.0
    if axis == 0:
        un, ut = u, v
    else:
        un, ut = v, u
    # R in the (rho, m_n, m_t, e) ordering, then mapped to (rho, mx, my, e)
    Rn = [
        [o, o, z, o],
        [un - c, un, z, un + c],
        [ut, ut, o, ut],
        [H - un * c, ke, ut, H + un * c],
    ]
    Ln = [
        [0.5 * (b2 + un / c), -0.5 * (b1 * un + 1.0 / c), -0.5 * b1 * ut, 0.5 * b1],
        [1.0 - b2, b1 * un, b1 * ut, -b1],
        [-ut, z, o, z],
        [0.5 * (b2 - un / c), -0.5 * (b1 * un - 1.0 / c), -0.5 * b1 * ut, 0.5 * b1],
    ]
    R = np.array([[np.asarray(x) for x in r] for r in Rn])
    L = np.array([[np.asarray(x) for x in r] for r in Ln])
    if axis == 1:
        # the normal momentum is my (row/col 2), the tangential one mx (row/col 1)
        perm = [0, 2, 1, 3]
        R = R[perm, :]
        L = L[:, perm]
    return R, L
