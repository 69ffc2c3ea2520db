"""Brute-force CPR residual at 50 digits with mpmath, written directly from
the definitions (no tables): Gauss-Legendre nodes as roots of L_{P+1} (or
Gauss-Lobatto nodes: -1, +1 and the roots of L_P') found by mpmath, Lagrange
polynomials as products, Radau correction polynomials from mpmath's Legendre
functions, and derivatives by mpmath's numerical differentiation: of the
corrected flux polynomial (schemes gl_lp on Gauss points and gll_lp on
Lobatto points), or, for the chain rule (scheme gll_chain), of the solution
polynomial, pushed through the flux as a directional derivative
d/ds F(q + s dq) at s = 0. Used only to pin the oracle on tiny meshes; it
shares nothing with the oracle."""

import mpmath as mp


def gl_nodes(n):
    xs = []
    for k in range(n):
        x0 = mp.cos(mp.pi * (k + mp.mpf(3) / 4) / (n + mp.mpf(1) / 2))
        xs.append(mp.findroot(lambda x: mp.legendre(n, x), x0))
    return sorted(xs)


def gll_nodes(n):
    P = n - 1

    def dL(x):
        return mp.diff(lambda t: mp.legendre(P, t), x)

    xs = [mp.mpf(-1), mp.mpf(1)]
    for k in range(1, P):
        x0 = -mp.cos(mp.pi * k / P)
        xs.append(mp.findroot(dL, x0))
    return sorted(xs)


def lagrange(nodes, l, x):
    out = mp.mpf(1)
    for m, xm in enumerate(nodes):
        if m != l:
            out *= (x - xm) / (nodes[l] - xm)
    return out


def pressure(q, g):
    return (g - 1) * (q[3] - (q[1] ** 2 + q[2] ** 2) / (2 * q[0]))


def flux(q, g, axis):
    p = pressure(q, g)
    un = q[1 + axis] / q[0]
    out = [q[1 + axis], q[1] * un, q[2] * un, un * (q[3] + p)]
    out[1 + axis] += p
    return out


def speed(q, g, axis):
    return abs(q[1 + axis] / q[0]) + mp.sqrt(g * pressure(q, g) / q[0])


def rusanov(qL, qR, g, axis):
    lam = max(speed(qL, g, axis), speed(qR, g, axis))
    fL, fR = flux(qL, g, axis), flux(qR, g, axis)
    return [(fL[k] + fR[k]) / 2 - lam * (qR[k] - qL[k]) / 2 for k in range(4)]


def residual(q, P, nx, ny, x0, x1, y0, y1, bc, gamma, dps=50, scheme="gl_lp"):
    """q: nested sequence q[k][J][I][j][i] of floats. Returns the same
    nesting of mpf residuals."""
    mp.mp.dps = dps
    g = mp.mpf(gamma)
    n1 = P + 1
    nodes = gl_nodes(n1) if scheme == "gl_lp" else gll_nodes(n1)
    dx = (mp.mpf(x1) - mp.mpf(x0)) / nx
    dy = (mp.mpf(y1) - mp.mpf(y0)) / ny

    def L(n, x):
        return mp.legendre(n, x)

    sgn = (-1) ** (P + 1)

    def gL(x):
        return sgn * (L(P + 1, x) - L(P, x)) / 2

    def gR(x):
        return (L(P + 1, x) + L(P, x)) / 2

    Q = [[[[[mp.mpf(float(q[k][J][I][j][i])) for i in range(n1)] for j in range(n1)]
           for I in range(nx)] for J in range(ny)] for k in range(4)]

    def point(J, I, j, i):
        return [Q[k][J][I][j][i] for k in range(4)]

    def line(J, I, c, axis):
        """The n1 states along the line through element (J, I): row j=c
        (axis 0) or column i=c (axis 1)."""
        if axis == 0:
            return [point(J, I, c, i) for i in range(n1)]
        return [point(J, I, j, c) for j in range(n1)]

    def extrap(pts, x):
        return [sum(pts[l][k] * lagrange(nodes, l, x) for l in range(n1)) for k in range(4)]

    def neighbour(J, I, axis, side):
        if axis == 0:
            I2 = I + side
            if 0 <= I2 < nx:
                return (J, I2)
            return (J, I2 % nx) if bc == "periodic" else None
        J2 = J + side
        if 0 <= J2 < ny:
            return (J2, I)
        return (J2 % ny, I) if bc == "periodic" else None

    R = [[[[[mp.mpf(0)] * n1 for _ in range(n1)] for _ in range(nx)] for _ in range(ny)]
         for _ in range(4)]
    for J in range(ny):
        for I in range(nx):
            for axis, h in ((0, dx), (1, dy)):
                for c in range(n1):
                    pts = line(J, I, c, axis)
                    fl = [flux(p, g, axis) for p in pts]
                    own_lo = extrap(pts, -1)
                    own_hi = extrap(pts, 1)
                    nb = neighbour(J, I, axis, -1)
                    lo_out = own_lo if nb is None else extrap(line(nb[0], nb[1], c, axis), 1)
                    nb = neighbour(J, I, axis, +1)
                    hi_out = own_hi if nb is None else extrap(line(nb[0], nb[1], c, axis), -1)
                    F_lo = rusanov(lo_out, own_lo, g, axis)
                    F_hi = rusanov(own_hi, hi_out, g, axis)
                    for k in range(4):
                        fk = [fl[l][k] for l in range(n1)]

                        def fpoly(x, fk=fk):
                            return sum(fk[l] * lagrange(nodes, l, x) for l in range(n1))

                        jl = F_lo[k] - fpoly(mp.mpf(-1))
                        jh = F_hi[k] - fpoly(mp.mpf(1))

                        def corrected(x, fpoly=fpoly, jl=jl, jh=jh):
                            return fpoly(x) + jl * gL(x) + jh * gR(x)

                        for a in range(n1):
                            if scheme == "gll_chain":
                                qa = pts[a]
                                dq = [mp.diff(lambda x, m=m: extrap(pts, x)[m], nodes[a])
                                      for m in range(4)]
                                dF = mp.diff(lambda s, k=k: flux([qa[m] + s * dq[m]
                                                                  for m in range(4)], g, axis)[k], 0)
                                d = (dF + jl * mp.diff(gL, nodes[a])
                                     + jh * mp.diff(gR, nodes[a]))
                            else:
                                d = mp.diff(corrected, nodes[a])
                            if axis == 0:
                                R[k][J][I][c][a] -= 2 * d / h
                            else:
                                R[k][J][I][a][c] -= 2 * d / h
    return R
