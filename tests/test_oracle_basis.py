"""Pins of the oracle's 1D tables and reference element against closed forms,
library quadrature and the defining degrees of freedom (Section 2.1)."""
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import basis, element


@pytest.mark.parametrize("p,expected", [
    (1, [0.0, 1.0]),
    (2, [0.0, 0.5, 1.0]),
    (3, [0.0, (1 - 1 / np.sqrt(5)) / 2, (1 + 1 / np.sqrt(5)) / 2, 1.0]),
    (4, [0.0, (1 - np.sqrt(3 / 7)) / 2, 0.5, (1 + np.sqrt(3 / 7)) / 2, 1.0]),
])
def test_gauss_lobatto_closed_forms(p, expected):
    assert np.allclose(basis.gauss_lobatto_points(p), expected, atol=1e-15, rtol=0)


def test_gauss_legendre_closed_forms():
    x, w = basis.gauss_legendre(2)
    assert np.allclose(x, [(1 - 1 / np.sqrt(3)) / 2, (1 + 1 / np.sqrt(3)) / 2], atol=1e-15)
    assert np.allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = basis.gauss_legendre(3)
    assert np.allclose(x, [(1 - np.sqrt(0.6)) / 2, 0.5, (1 + np.sqrt(0.6)) / 2], atol=1e-15)
    assert np.allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 10))
def test_gauss_legendre_exact_monomials(n):
    x, w = basis.gauss_legendre(n)
    for k in range(2 * n):
        assert abs(w @ x ** k - 1.0 / (k + 1)) < 1e-14


@pytest.mark.parametrize("p", range(1, 9))
def test_lagrange_and_histopolation_dofs(p):
    xi = basis.gauss_lobatto_points(p)
    # interpolation: l_i(xi_k) = delta_ik
    assert np.allclose(basis.lagrange(xi, xi), np.eye(p + 1), atol=1e-12)
    # histopolation: int over sub-interval k of h_j = delta_jk (adaptive library quadrature)
    I = np.zeros((p, p))
    for j in range(p):
        for k in range(p):
            I[k, j] = quad(lambda t: basis.histopolation(xi, t)[0, j], xi[k], xi[k + 1], epsabs=1e-14)[0]
    assert np.allclose(I, np.eye(p), atol=1e-11)


@pytest.mark.parametrize("p", range(1, 9))
def test_derivative_of_interpolant_is_histopolant(p):
    """l_i' = h_{i-1} - h_i: the 1D identity behind the +-1 divergence."""
    xi = basis.gauss_lobatto_points(p)
    t = np.linspace(0, 1, 37)
    dl = basis.lagrange_deriv(xi, t)
    # independent derivative check of l_i' by central differences
    eps = 1e-6
    fd = (basis.lagrange(xi, t + eps) - basis.lagrange(xi, t - eps)) / (2 * eps)
    assert np.allclose(dl, fd, atol=1e-6 * max(1, abs(dl).max()))
    H = basis.histopolation(xi, t)
    Hp = np.concatenate([np.zeros((len(t), 1)), H, np.zeros((len(t), 1))], axis=1)
    for i in range(p + 1):
        assert np.allclose(dl[:, i], Hp[:, i] - Hp[:, i + 1], atol=1e-10 * max(1, abs(dl).max()))


@pytest.mark.parametrize("p", range(1, 6))
def test_rt_reference_reproduces_its_space(p):
    """A random field of Q_{p,p-1,p-1} x Q_{p-1,p,p-1} x Q_{p-1,p-1,p} equals
    the combination of basis functions weighted by its sub-face fluxes."""
    rng = np.random.default_rng(p)
    degs = [(p, p - 1, p - 1), (p - 1, p, p - 1), (p - 1, p - 1, p)]
    coef = [rng.standard_normal(tuple(d + 1 for d in dd)) for dd in degs]

    def field(X):
        out = np.zeros((X.shape[0], 3))
        for c in range(3):
            C = coef[c]
            for a in range(C.shape[0]):
                for b in range(C.shape[1]):
                    for g in range(C.shape[2]):
                        out[:, c] += C[a, b, g] * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** g
        return out

    xi = basis.gauss_lobatto_points(p)
    xg, wg = basis.gauss_legendre(p + 2)
    dofs = []
    for c, shp in enumerate(element.rt_shapes(p)):
        t1, t2 = [d for d in range(3) if d != c]
        for k in range(shp[2]):
            for j in range(shp[1]):
                for i in range(shp[0]):
                    idx = [i, j, k]
                    # face at xi[idx[c]] in direction c; sub-rectangle in the others
                    a1, b1 = xi[idx[t1]], xi[idx[t1] + 1]
                    a2, b2 = xi[idx[t2]], xi[idx[t2] + 1]
                    s1 = a1 + (b1 - a1) * xg
                    s2 = a2 + (b2 - a2) * xg
                    S1, S2 = np.meshgrid(s1, s2, indexing='ij')
                    W = np.outer(wg, wg) * (b1 - a1) * (b2 - a2)
                    X = np.zeros((S1.size, 3))
                    X[:, c] = xi[idx[c]]
                    X[:, t1] = S1.ravel()
                    X[:, t2] = S2.ravel()
                    dofs.append((W.ravel() * field(X)[:, c]).sum())
    dofs = np.array(dofs)
    Xt = rng.uniform(0, 1, size=(25, 3))
    phi, _ = element.rt_reference(p, Xt)
    assert np.allclose(np.einsum('nar,a->nr', phi, dofs), field(Xt), atol=1e-11)


@pytest.mark.parametrize("p", range(1, 6))
def test_l2_reference_reproduces_its_space(p):
    rng = np.random.default_rng(10 + p)
    C = rng.standard_normal((p, p, p))

    def f(X):
        out = np.zeros(X.shape[0])
        for a in range(p):
            for b in range(p):
                for c in range(p):
                    out += C[a, b, c] * X[:, 0] ** a * X[:, 1] ** b * X[:, 2] ** c
        return out

    xi = basis.gauss_lobatto_points(p)
    xg, wg = basis.gauss_legendre(p + 1)
    dofs = np.zeros(p ** 3)
    for c in range(p):
        for b in range(p):
            for a in range(p):
                lo = np.array([xi[a], xi[b], xi[c]])
                hi = np.array([xi[a + 1], xi[b + 1], xi[c + 1]])
                X = element.tensor_points(xg)
                X = lo + X * (hi - lo)
                w = element.tensor_weights(wg) * np.prod(hi - lo)
                dofs[a + p * (b + p * c)] = w @ f(X)
    Xt = rng.uniform(0, 1, size=(20, 3))
    assert np.allclose(element.l2_reference(p, Xt) @ dofs, f(Xt), atol=1e-11)
