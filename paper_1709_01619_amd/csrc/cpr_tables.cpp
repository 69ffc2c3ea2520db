// Host construction of the 1D CPR tables for degree P (Section 2.2 of
// arXiv:1709.01619: nodal solution polynomial of degree P, derivative
// matrix, Radau correction in the DG-equivalent form), on one of two point
// sets.
//
//  * Gauss-Legendre nodes by Newton's method on the Legendre three-term
//    recurrence, weights 2 / ((1 - x^2) L'_{n}(x)^2).
//  * Gauss-Lobatto-Legendre nodes (the paper's CPR points, Fig. 1(b)): -1,
//    +1 and the roots of L_P', found by Newton's method with L_P'' from
//    Legendre's equation; weights 2 / (P (P+1) L_P(x)^2).
//  * Lagrange derivative matrix and face-extrapolation rows by the
//    barycentric formulas (diagonal of D from the zero row sum); on the
//    Lobatto points the face rows are unit vectors, the end points being
//    solution points.
//  * Radau correction derivatives at the nodes. Gauss points: from the DG
//    equivalence of the Radau lift, gL'(xi_i) = -l_i(-1) / w_i (the rule
//    integrates gL' l_i exactly). Lobatto points: that rule is not exact for
//    degree 2P, so gL' = (-1)^(P+1)/2 (L_{P+1}' - L_P') is evaluated
//    directly, with the derivative recurrence L_{k+1}' = L_{k-1}' +
//    (2k+1) L_k, which holds at the end points too.
#include <cmath>

#include "cpr_internal.h"

namespace cpr {

static void legendre_and_derivative(int n, double x, double* Ln, double* dLn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *Ln = 1.0;
    *dLn = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *Ln = p1;
  *dLn = n * (x * p1 - p0) / (x * x - 1.0);
}

// L_n and L_n' at any x in [-1, 1], end points included.
static void legendre_pair(int n, double x, double* Ln, double* dLn) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) {
    *Ln = 1.0;
    *dLn = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    const double d2 = d0 + (2.0 * k + 1.0) * p1;
    p0 = p1;
    p1 = p2;
    d0 = d1;
    d1 = d2;
  }
  *Ln = p1;
  *dLn = d1;
}

static void gauss_nodes(int n, Tables1D* T) {
  for (int k = 0; k < n; ++k) {
    // k-th root from the top, then stored in ascending order
    double x = std::cos(M_PI * (k + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double L, dL;
      legendre_and_derivative(n, x, &L, &dL);
      double dx = L / dL;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    double L, dL;
    legendre_and_derivative(n, x, &L, &dL);
    T->xi[n - 1 - k] = x;
    T->w[n - 1 - k] = 2.0 / ((1.0 - x * x) * dL * dL);
  }
}

static void lobatto_nodes(int P, Tables1D* T) {
  const int n = P + 1;
  const double pp1 = P * (P + 1.0);
  T->xi[0] = -1.0;
  T->xi[P] = 1.0;
  for (int k = 1; k < P; ++k) {
    // k-th interior root in ascending order, from the Chebyshev-Lobatto guess
    double x = -std::cos(M_PI * k / P);
    for (int it = 0; it < 100; ++it) {
      double L, dL;
      legendre_pair(P, x, &L, &dL);
      // (1 - x^2) L'' = 2 x L' - P (P+1) L
      const double d2L = (2.0 * x * dL - pp1 * L) / (1.0 - x * x);
      const double dx = dL / d2L;
      x -= dx;
      if (std::fabs(dx) < 1e-17) break;
    }
    T->xi[k] = x;
  }
  for (int k = 0; k < n; ++k) {
    double L, dL;
    legendre_pair(P, T->xi[k], &L, &dL);
    T->w[k] = 2.0 / (pp1 * L * L);
  }
}

bool build_tables(int P, int points, Tables1D* T) {
  if (P < 1 || P > kMaxP) return false;
  if (points != kGauss && points != kLobatto) return false;
  const int n = P + 1;
  T->P = P;
  T->points = points;
  if (points == kGauss)
    gauss_nodes(n, T);
  else
    lobatto_nodes(P, T);
  // symmetrise (the rule is symmetric; removes one-ulp asymmetries)
  for (int k = 0; k < n / 2; ++k) {
    double a = 0.5 * (T->xi[n - 1 - k] - T->xi[k]);
    T->xi[k] = -a;
    T->xi[n - 1 - k] = a;
    double wa = 0.5 * (T->w[k] + T->w[n - 1 - k]);
    T->w[k] = T->w[n - 1 - k] = wa;
  }
  if (n % 2 == 1) T->xi[n / 2] = 0.0;

  double bw[kMaxP + 1];
  for (int l = 0; l < n; ++l) {
    double prod = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != l) prod *= (T->xi[l] - T->xi[m]);
    bw[l] = 1.0 / prod;
  }
  for (int i = 0; i < n; ++i) {
    double diag = 0.0;
    for (int l = 0; l < n; ++l) {
      if (l == i) continue;
      double d = (bw[l] / bw[i]) / (T->xi[i] - T->xi[l]);
      T->D[i][l] = d;
      diag -= d;
    }
    T->D[i][i] = diag;
  }
  if (points == kLobatto)
    for (int l = 0; l < n; ++l) {
      T->em[l] = l == 0 ? 1.0 : 0.0;
      T->ep[l] = l == n - 1 ? 1.0 : 0.0;
    }
  for (int side = 0; side < 2 && points == kGauss; ++side) {
    const double x = side == 0 ? -1.0 : 1.0;
    double den = 0.0;
    for (int m = 0; m < n; ++m) den += bw[m] / (x - T->xi[m]);
    for (int l = 0; l < n; ++l) {
      double v = (bw[l] / (x - T->xi[l])) / den;
      if (side == 0)
        T->em[l] = v;
      else
        T->ep[l] = v;
    }
  }
  // the nodes are symmetric, so D[n-1-i][n-1-l] = -D[i][l],
  // l_l(+1) = l_{n-1-l}(-1) and gR'(xi_i) = -gL'(xi_{n-1-i}); rounding in the
  // formulas above can break these by an ulp, so the upper half is set from
  // the lower half (the kernels rely on the identities holding exactly)
  for (int i = 0; i < n; ++i) {
    const int mi = n - 1 - i;
    for (int l = 0; l < n; ++l) {
      const int ml = n - 1 - l;
      if (i > mi) T->D[i][l] = -T->D[mi][ml];
      else if (i == mi) T->D[i][l] = l < ml ? T->D[i][l] : l > ml ? -T->D[i][ml] : 0.0;
    }
    T->ep[i] = T->em[mi];
  }
  const double sgn = (P % 2 == 1) ? 0.5 : -0.5;  // (-1)^(P+1) / 2
  for (int i = 0; i < n; ++i) {
    if (points == kGauss) {
      T->gLp[i] = -T->em[i] / T->w[i];
    } else {
      double L, dP, dP1;
      legendre_pair(P, T->xi[i], &L, &dP);
      legendre_pair(P + 1, T->xi[i], &L, &dP1);
      T->gLp[i] = sgn * (dP1 - dP);
    }
  }
  for (int i = 0; i < n; ++i) T->gRp[i] = -T->gLp[n - 1 - i];
  return true;
}

}  // namespace cpr
