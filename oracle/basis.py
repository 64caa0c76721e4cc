"""1D reference element of the staggered spectral DG scheme (test infrastructure only).

Follows Section 2.1 ("Numerical method") of Fambri & Dumbser, arXiv:1602.05806:
  * the basis phi_l is the Lagrange interpolation polynomial through the N+1 Gauss-Legendre
    points of [0,1], so the element mass matrix is diagonal (text after eq. pDGpoly);
  * the main-cell basis omega and the dual-cell basis psi are the same phi on shifted cells;
  * the 1D matrices M, R~, L~, R-bar, L-bar are defined by the integrals of eq. (matrices);
  * the pressure blocks R, L, C of eq. (pSyst) are built from them;
  * the L2-projection matrices M^L, M^R of eq. (l2forward).

Every integral is evaluated with an (N+3)-point Gauss-Legendre rule on [0,1]. The integrands
have polynomial degree at most 2N, so this rule (exact to degree 2N+5) is exact up to rounding.
"""
import numpy as np
from numpy.polynomial.legendre import leggauss


def gauss_legendre_01(n):
    """Nodes xi_l and weights w_l of the n-point Gauss-Legendre rule mapped to [0,1] (sum w = 1)."""
    x, w = leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, p, s):
    """phi_p(s): Lagrange polynomial through `nodes`, equal to 1 at nodes[p] (product formula)."""
    s = np.asarray(s, dtype=np.float64)
    v = np.ones_like(s)
    for q, xq in enumerate(nodes):
        if q != p:
            v = v * (s - xq) / (nodes[p] - xq)
    return v


def lagrange_deriv(nodes, p, s):
    """phi_p'(s), by differentiating the product formula term by term."""
    s = np.asarray(s, dtype=np.float64)
    total = np.zeros_like(s)
    for r, xr in enumerate(nodes):
        if r == p:
            continue
        term = np.ones_like(s) / (nodes[p] - xr)
        for q, xq in enumerate(nodes):
            if q != p and q != r:
                term = term * (s - xq) / (nodes[p] - xq)
        total = total + term
    return total


class Tables:
    """All 1D matrices of degree N, FP64.

    Attributes (each (N+1)x(N+1) unless stated):
      xi, w   GL nodes and weights on [0,1] (vectors)
      M       mass matrix, int phi_p phi_q = diag(w)                         eq. (matrices)
      Rt, Lt  R~ and L~ of eq. (matrices): the weak pressure gradient from the
              two main cells overlapping a dual cell, including the pressure jump of
              eq. (pressurejump)
      Rb, Lb  R-bar and L-bar of eq. (matrices): the weak divergence on a main cell
      Cblk    C = R-bar M^-1 L~ + L-bar M^-1 R~                                eq. (pSyst)
      Rblk    R = -R-bar M^-1 R~  (couples cell i to cell i+1)                 eq. (pSyst)
      Lblk    L = -L-bar M^-1 L~  (couples cell i to cell i-1)                 eq. (pSyst)
      ML, MR  L2 projection matrices M^L, M^R                                  eq. (l2forward)
      phi0, phi1   phi_p(0) and phi_p(1) (face extrapolation vectors)
      dphi    dphi[k, m] = phi_k'(xi_m)
      dphi0, dphi1 phi_p'(0) and phi_p'(1) (face derivative vectors)
    """

    def __init__(self, N):
        if N < 0:
            raise ValueError("degree N must be >= 0")
        self.N = N
        n = N + 1
        self.n = n
        xi, w = gauss_legendre_01(n)
        self.xi, self.w = xi, w
        qx, qw = gauss_legendre_01(N + 3)

        def phi(p, s):
            return lagrange(xi, p, s)

        def dphi(p, s):
            return lagrange_deriv(xi, p, s)

        M = np.zeros((n, n))
        Rt = np.zeros((n, n))
        Lt = np.zeros((n, n))
        Rb = np.zeros((n, n))
        Lb = np.zeros((n, n))
        ML = np.zeros((n, n))
        MR = np.zeros((n, n))
        for p in range(n):
            for q in range(n):
                M[p, q] = np.sum(qw * phi(p, qx) * phi(q, qx))
                # eq. (matrices), R~: jump at the dual-cell midpoint + right half of the dual cell
                Rt[p, q] = phi(p, 0.5) * phi(q, 0.0) + 0.5 * np.sum(
                    qw * phi(p, 0.5 + qx / 2) * dphi(q, qx / 2))
                # eq. (matrices), L~: jump + left half of the dual cell
                Lt[p, q] = phi(p, 0.5) * phi(q, 1.0) - 0.5 * np.sum(
                    qw * phi(p, qx / 2) * dphi(q, 0.5 + qx / 2))
                # eq. (matrices), R-bar and L-bar (main-cell divergence)
                Rb[p, q] = phi(p, 1.0) * phi(q, 0.5) - 0.5 * np.sum(
                    qw * dphi(p, 0.5 + qx / 2) * phi(q, qx / 2))
                Lb[p, q] = phi(p, 0.0) * phi(q, 0.5) + 0.5 * np.sum(
                    qw * dphi(p, qx / 2) * phi(q, 0.5 + qx / 2))
                # eq. (l2forward)
                ML[p, q] = 0.5 * np.sum(qw * phi(p, qx / 2) * phi(q, 0.5 + qx / 2))
                MR[p, q] = 0.5 * np.sum(qw * phi(p, 0.5 + qx / 2) * phi(q, qx / 2))
        self.M, self.Rt, self.Lt, self.Rb, self.Lb = M, Rt, Lt, Rb, Lb
        self.ML, self.MR = ML, MR
        Minv = np.diag(1.0 / w)
        # eq. (pSyst): the three blocks of the 1D pressure operator
        self.Cblk = Rb @ Minv @ Lt + Lb @ Minv @ Rt
        self.Rblk = -(Rb @ Minv @ Rt)
        self.Lblk = -(Lb @ Minv @ Lt)
        self.phi0 = np.array([phi(p, 0.0) for p in range(n)], dtype=np.float64)
        self.phi1 = np.array([phi(p, 1.0) for p in range(n)], dtype=np.float64)
        self.dphi = np.array([[dphi(k, xi[m]) for m in range(n)] for k in range(n)],
                             dtype=np.float64)
        self.dphi0 = np.array([dphi(p, 0.0) for p in range(n)], dtype=np.float64)
        self.dphi1 = np.array([dphi(p, 1.0) for p in range(n)], dtype=np.float64)


_cache = {}


def tables(N):
    """Cached Tables(N)."""
    if N not in _cache:
        _cache[N] = Tables(N)
    return _cache[N]
