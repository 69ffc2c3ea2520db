"""One-dimensional CPR tables on the reference interval [-1, 1] (oracle).

Section 2.2 of the paper builds the CPR scheme from (i) a nodal polynomial
of degree P per element stored at solution points, (ii) a derivative of the
flux polynomial at those points, and (iii) a correction polynomial built from
Radau polynomials that lifts the interface flux jump (the DG-equivalent
choice). Tensor products of these 1D tables give the 2D quad element.

Two point sets. Gauss-Legendre nodes ("gl", the default): the flux points
on the element faces are not solution points, so face values are
extrapolated from the nodal polynomial. Gauss-Lobatto-Legendre nodes ("gll",
the paper's own choice in Section 2.2): the end points are solution points,
so the face value of a line is its end value and no interpolation is needed.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from numpy.polynomial import legendre as npleg


@dataclass(frozen=True)
class Tables:
    P: int
    xi: np.ndarray      # (n1,) solution points, ascending
    w: np.ndarray       # (n1,) quadrature weights, sum 2
    D: np.ndarray       # (n1, n1) D[i, l] = l_l'(xi_i)
    em: np.ndarray      # (n1,) l_l(-1)
    ep: np.ndarray      # (n1,) l_l(+1)
    gLp: np.ndarray     # (n1,) g_L'(xi_i), left-face correction
    gRp: np.ndarray     # (n1,) g_R'(xi_i), right-face correction

    @property
    def n1(self) -> int:
        return self.P + 1


def lagrange_eval(xi: np.ndarray, x) -> np.ndarray:
    """L[a, l] = l_l(x_a): the Lagrange basis on nodes xi evaluated at x,
    written out as the product over the other nodes."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(xi)
    out = np.ones((len(x), n))
    for l in range(n):
        for m in range(n):
            if m != l:
                out[:, l] *= (x - xi[m]) / (xi[l] - xi[m])
    return out


def lagrange_deriv(xi: np.ndarray, x) -> np.ndarray:
    """L'[a, l] = l_l'(x_a) by the product rule over the factors of l_l."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(xi)
    out = np.zeros((len(x), n))
    for l in range(n):
        for m in range(n):
            if m == l:
                continue
            term = np.full(len(x), 1.0 / (xi[l] - xi[m]))
            for r in range(n):
                if r != l and r != m:
                    term *= (x - xi[r]) / (xi[l] - xi[r])
            out[:, l] += term
    return out


def radau_left_coeffs(P: int) -> np.ndarray:
    """Legendre-series coefficients of g_L, the right Radau polynomial of
    degree P+1: g_L = (-1)^(P+1)/2 (L_{P+1} - L_P). It is 1 at -1 and 0 at +1
    (Section 2.2 uses Radau polynomials to place the correction in the DG
    framework)."""
    c = np.zeros(P + 2)
    s = 0.5 * (-1.0) ** (P + 1)
    c[P + 1] = s
    c[P] = -s
    return c


def radau_right_coeffs(P: int) -> np.ndarray:
    """g_R(x) = g_L(-x) = (L_{P+1} + L_P)/2: 0 at -1 and 1 at +1."""
    c = np.zeros(P + 2)
    c[P + 1] = 0.5
    c[P] = 0.5
    return c


def lobatto_nodes_weights(P: int):
    """Gauss-Lobatto-Legendre rule with P+1 points: -1, the P-1 roots of
    L_P', +1; weights 2 / (P (P+1) L_P(x)^2) (exact to degree 2P-1)."""
    cP = np.zeros(P + 1)
    cP[P] = 1.0
    inner = npleg.legroots(npleg.legder(cP)) if P >= 2 else np.zeros(0)
    xi = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    LP = npleg.legval(xi, cP)
    w = 2.0 / (P * (P + 1) * LP * LP)
    return xi, w


def build(P: int, points: str = "gl") -> Tables:
    if not (1 <= P <= 8):
        raise ValueError(f"P must be in [1, 8], got {P}")
    n1 = P + 1
    if points == "gl":
        xi, w = npleg.leggauss(n1)
    elif points == "gll":
        xi, w = lobatto_nodes_weights(P)
    else:
        raise ValueError(f"unknown point set {points}")
    D = lagrange_deriv(xi, xi)
    em = lagrange_eval(xi, -1.0)[0]
    ep = lagrange_eval(xi, 1.0)[0]
    gLp = npleg.legval(xi, npleg.legder(radau_left_coeffs(P)))
    gRp = npleg.legval(xi, npleg.legder(radau_right_coeffs(P)))
    return Tables(P=P, xi=xi, w=w, D=D, em=em, ep=ep, gLp=gLp, gRp=gRp)


_CACHE: dict = {}


def get(P: int, points: str = "gl") -> Tables:
    if (P, points) not in _CACHE:
        _CACHE[(P, points)] = build(P, points)
    return _CACHE[(P, points)]
