"""Pins of the oracle's learned-diagonal path: the spread gradient against
central differences, symmetry of the target on a cube, descent and the
constraint of the projected gradient, the generalized eigenproblem against
the library solver, the network's backpropagation against central
differences, the corrected diagonal at zero scalings, and the feature map on
transformed elements."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assemble, element, learned, precond
from paper_2304_12387_amd import inputs


def _cube():
    V = np.zeros((1, 2, 2, 2, 3))
    for dz in range(2):
        for dy in range(2):
            for dx in range(2):
                V[0, dz, dy, dx] = (dx, dy, dz)
    return V


def _distorted(seed=3, aspect=3.0, shear=0.4):
    rng = np.random.default_rng(seed)
    V = _cube()
    V[..., 0] *= aspect
    V[..., 0] += shear * V[..., 1]
    V[..., 1] += 0.3 * shear * V[..., 2]
    return V + rng.uniform(-0.08, 0.08, V.shape)


def test_dof_weights_structure():
    for p in (1, 2, 3):
        A = learned.dof_weights(p)
        assert A.shape == (element.n_rt(p), 6)
        assert np.allclose(A.sum(axis=1), 1.0)
        # exactly one component pair is active per dof, dofs on the lower face
        # (xi = 0) carry theta_{2c} only
        nc = p * p * (p + 1)
        for c in range(3):
            blk = A[c * nc:(c + 1) * nc]
            other = [k for k in range(6) if k // 2 != c]
            assert np.all(blk[:, other] == 0.0)
        assert np.all(A[0] == [1, 0, 0, 0, 0, 0])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_spread_gradient_central_differences(p):
    V = _distorted()
    Me = element.element_matrices(p, V)['M'][0]
    A = learned.dof_weights(p)
    m = np.diag(Me).copy()
    theta = np.array([0.1, -0.2, 0.05, 0.15, -0.1, 0.0])
    f, g = learned.spread_gradient(Me, m, A, theta)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fd = (learned.spread(Me, m, A, theta + e) - learned.spread(Me, m, A, theta - e)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j]))


def test_generalized_eigenproblem_matches_library():
    p = 2
    V = _distorted()
    Me = element.element_matrices(p, V)['M'][0]
    A = learned.dof_weights(p)
    theta = np.array([0.2, -0.1, 0.0, 0.1, -0.3, 0.1])
    lo, hi = learned.pencil_extremes(Me, np.diag(Me), A, theta, vectors=False)
    lam = sla.eigh(Me, np.diag(np.diag(Me) * np.exp(A @ theta)), eigvals_only=True)
    assert abs(lo - lam[0]) <= 1e-12 * lam[-1] and abs(hi - lam[-1]) <= 1e-12 * lam[-1]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_target_on_cube_is_zero(p):
    """By the cube's symmetries the spread is stationary at theta = 0."""
    th, lam = learned.element_targets(_cube(), p)
    assert np.abs(th).max() <= 1e-12
    # and its value is the extreme eigenvalues of the Jacobi-scaled mass
    Me = element.element_matrices(p, _cube())['M'][0]
    d = 1.0 / np.sqrt(np.diag(Me))
    ev = np.linalg.eigvalsh(Me * d[:, None] * d[None, :])
    assert np.allclose(lam[0], [ev[0], ev[-1]], rtol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_target_descends_on_the_constraint(p):
    V = _distorted(seed=p)
    Me = element.element_matrices(p, V)['M'][0]
    th, f0, f = learned.element_target(Me, p)
    assert abs(th.sum()) <= 1e-12
    assert f <= f0
    # first-order optimality on the constraint (or the step budget ran out)
    A = learned.dof_weights(p)
    _, g = learned.spread_gradient(Me, np.diag(Me), A, th)
    pg = g - g.mean()
    assert np.linalg.norm(pg) <= 1e-2 or f < f0 - 1e-6


def test_backprop_central_differences():
    rng = np.random.default_rng(5)
    params = learned.init_params(seed=2)
    X = rng.standard_normal((7, learned.N_IN))
    Y = rng.uniform(-2.0, 2.0, (7, learned.N_OUT))
    loss, grads = learned.loss_and_grad(params, X, Y)
    h = 1e-6
    for k, P in enumerate(params):
        flat = P.reshape(-1)
        picks = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for idx in picks:
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = learned.loss_and_grad(params, X, Y)
            flat[idx] = old - h
            lm, _ = learned.loss_and_grad(params, X, Y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            gk = grads[k].reshape(-1)[idx]
            assert abs(fd - gk) <= 1e-6 * max(1e-3, abs(gk)), (k, idx, fd, gk)


def test_gelu_exact():
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    Phi = 0.5 * (1.0 + np.array([math.erf(v / math.sqrt(2)) for v in x]))
    assert np.allclose(learned.gelu(x), x * Phi, rtol=1e-15, atol=1e-300)
    assert learned.gelu(np.array([0.0]))[0] == 0.0


def test_adam_first_step_is_lr_sign():
    params = [np.array([1.0, -2.0, 3.0])]
    grads = [np.array([0.5, -1e-3, 0.0])]
    st = learned.adam_state(params)
    learned.adam_step(params, grads, st, lr=0.1)
    # bias-corrected first step is lr * g / (|g| + eps)
    assert np.allclose(params[0], [0.9, -1.9, 3.0], atol=1e-6)


def test_features_invariance():
    """Offsets are translation and scale invariant; p and the coefficients
    enter as ln alpha, ln beta, p / 6."""
    V = _distorted()
    x = learned.features(V, np.array([2.0]), np.array([0.5]), 3)
    x2 = learned.features(3.7 * V + np.array([1.0, -2.0, 5.0]), np.array([2.0]), np.array([0.5]), 3)
    assert np.allclose(x, x2, rtol=0, atol=1e-13)
    assert np.allclose(x[0, 24:], [math.log(2.0), math.log(0.5), 0.5])
    # cube: offsets are +-1/2 (mean edge length 1)
    xc = learned.features(_cube(), np.array([1.0]), np.array([1.0]), 6)
    assert np.allclose(np.abs(xc[0, :24]), 0.5) and xc[0, 26] == 1.0


def test_learned_diag_at_zero_is_plain_diag():
    cfg = inputs.graddiv_jittered(2, 2)
    m = assemble.Mesh(2, 2, 2, 2, cfg['vertices'])
    prob = assemble.Problem(m, 0, cfg['c_mass'], cfg['c_22'], ess_sides=5)
    d0 = learned.learned_diag(prob, np.zeros((m.ne, 6)))
    assert np.allclose(d0, precond.diag_M(prob), rtol=1e-14)
    # a uniform scaling of every dof of one element scales its share only
    th = np.zeros((m.ne, 6))
    th[3] = math.log(2.0)
    d1 = learned.learned_diag(prob, th)
    share = np.zeros(m.n_u)
    np.add.at(share, prob.l2g[3], np.diag(prob.Me[3]))
    share[prob.ess] = 0.0
    assert np.allclose(d1 - d0, share, rtol=1e-13, atol=1e-14 * d0.max())
