"""1D tables for the interpolation-histopolation (IH) basis.  Test infrastructure.

Section 2.1: the reference interval is split at the p+1 Gauss-Lobatto points
xi_0 = 0 < xi_1 < ... < xi_p = 1.  The RT degrees of freedom are normal fluxes
through sub-element faces (1D: point values -> Lagrange interpolation l_i at
the xi_i) and the L2 degrees of freedom are integrals over sub-element volumes
(1D: histopolation h_j with  int_{xi_k}^{xi_{k+1}} h_j = delta_jk).

Gauss-Legendre points are used for quadrature and, with p points, for the
nodal basis in which the local CG for the L2 mass inverse runs (Section 2.5).
All points live on [0, 1].
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_lobatto_points(p):
    """The p+1 Gauss-Lobatto points on [0,1]: the end points and the roots of
    P_p' (derivative of the Legendre polynomial of degree p), mapped from
    [-1,1].  Section 2.1 (sub-element vertices)."""
    if p < 1:
        raise ValueError("p >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    inner = npleg.Legendre.basis(p).deriv().roots()
    inner = np.sort(np.real(inner))
    x = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (x + 1.0)


def gauss_legendre(n):
    """n-point Gauss-Legendre rule on [0,1] (points, weights)."""
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange(nodes, x):
    """Matrix L[m, i] = l_i(x_m), the Lagrange polynomial through ``nodes``
    that is 1 at nodes[i] and 0 at the others (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.ones((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                out[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return out


def lagrange_deriv(nodes, x):
    """Matrix dL[m, i] = l_i'(x_m) by the product rule on the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    out = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for k in range(n):
                if k != i and k != m:
                    term *= (x - nodes[k]) / (nodes[i] - nodes[k])
            out[:, i] += term
    return out


def histopolation_coefficients(nodes):
    """Coefficients of the histopolation polynomials h_0..h_{p-1} (degree p-1)
    in the monomial basis of t = 2x - 1.

    Defined directly by the L2 degrees of freedom (Section 2.1): the integral
    of h_j over the k-th sub-interval [nodes[k], nodes[k+1]] is delta_jk.  The
    p x p moment system  A c_j = e_j  with
    A[k, m] = int_{nodes[k]}^{nodes[k+1]} t^m dx  is solved column by column.
    Returns C with h_j(x) = sum_m C[m, j] t^m.
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    p = len(nodes) - 1
    t = 2.0 * nodes - 1.0
    A = np.zeros((p, p))
    for k in range(p):
        for m in range(p):
            # dx = dt / 2
            A[k, m] = (t[k + 1] ** (m + 1) - t[k] ** (m + 1)) / (2.0 * (m + 1))
    return np.linalg.solve(A, np.eye(p))


def histopolation(nodes, x):
    """Matrix H[m, j] = h_j(x_m) for the histopolation basis on ``nodes``."""
    C = histopolation_coefficients(nodes)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = 2.0 * x - 1.0
    p = C.shape[0]
    V = np.stack([t ** m for m in range(p)], axis=1)  # [len(x), p]
    return V @ C


class Tables1D:
    """All 1D data for degree p with an n_q-point Gauss-Legendre rule.

    Attributes
    ----------
    xi : Gauss-Lobatto points (p+1)
    xq, wq : quadrature points / weights (n_q)
    L : l_i(xq_a)   [n_q, p+1]     (interpolation, RT normal direction)
    dL : l_i'(xq_a) [n_q, p+1]
    H : h_j(xq_a)   [n_q, p]       (histopolation, RT tangential dirs and L2)
    """

    def __init__(self, p, nq=None):
        self.p = p
        self.nq = p + 1 if nq is None else nq
        self.xi = gauss_lobatto_points(p)
        self.xq, self.wq = gauss_legendre(self.nq)
        self.L = lagrange(self.xi, self.xq)
        self.dL = lagrange_deriv(self.xi, self.xq)
        self.H = histopolation(self.xi, self.xq)
