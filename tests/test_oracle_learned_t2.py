"""Pins of the second learned target (oracle.learned.saddle_*): the spread of
the element's own saddle-point pencil (A_e, B_e(theta)), which depends on
alpha and beta (a per-element correction of M~ = diag(M) of Section 2.3 and
of the Schur approximation S~ built from it).

* The pencil at theta = 0 is the assembled operator of a one-element mesh
  (oracle.assemble) with the block preconditioner diag(M~, S~) of
  oracle.precond: the same eigenvalues.
* With the exact blocks (M and the exact Schur complement) the eigenvalues
  lie in the intervals of Prop. 1 (golden fixture of Section 2.2).
* The gradient of f2 against central differences, on a distorted element.
* The descent lowers f2 and a common scaling of the six factors is not
  neutral (f2 changes with it)."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import assemble, element, learned, precond
from paper_2304_12387_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), 'golden', 'propositions.json')))


def _element(p, seed):
    V, pp, alpha, beta = inputs.training_elements(40, seed)
    k = int(np.nonzero(pp == p)[0][0]) if np.any(pp == p) else 0
    return V[k:k + 1], float(alpha[k]), float(beta[k])


def _blocks(p, seed):
    V, alpha, beta = _element(p, seed)
    mats = element.element_matrices(p, V)
    D = element.reference_divergence(p)
    A, m, ct = learned.saddle_blocks(mats['M'][0], mats['W'][0], D, alpha, beta)
    return V, alpha, beta, mats, D, A, m, ct


@pytest.mark.parametrize("p", [1, 2, 3])
def test_pencil_at_zero_is_the_assembled_one_element_problem(p):
    V, alpha, beta, mats, D, A, m, ct = _blocks(p, 3)
    lam, _, _, _ = learned.saddle_pencil(A, m, ct, D, learned.dof_weights(p), np.zeros(6))
    # the same element as a 1 x 1 x 1 mesh, natural boundary conditions
    verts = np.stack([V[0, dz, dy, dx] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)])
    mesh = assemble.Mesh(1, 1, 1, p, verts)
    prob = assemble.Problem(mesh, 0, np.array([beta]), np.array([alpha]), 0)
    Ag = prob.block_matrix().toarray()
    S = precond.schur_by_formula(prob).toarray()
    Bg = sla.block_diag(np.diag(precond.diag_M(prob)), S)
    lg = sla.eigh(Ag, Bg, eigvals_only=True)
    assert np.allclose(np.sort(lam), np.sort(lg), rtol=1e-9, atol=1e-12 * np.abs(lg).max())


@pytest.mark.parametrize("p", [1, 2, 3])
def test_exact_blocks_satisfy_prop1(p):
    V, alpha, beta, mats, D, A, m, ct = _blocks(p, 4)
    M = beta * mats['M'][0]
    C = (1.0 / alpha) * np.linalg.inv(mats['W'][0])
    S = C + D @ np.linalg.solve(M, D.T)
    lam, _, _, _ = learned.saddle_pencil(A, m, ct, D, learned.dof_weights(p), np.zeros(6), exact=(M, S))
    lo, hi = (1 - np.sqrt(5)) / 2, (1 + np.sqrt(5)) / 2
    neg, pos = lam[lam < 0], lam[lam > 0]
    tol = 1e-9
    assert neg.min() >= -1 - tol and neg.max() <= lo + tol
    assert pos.min() >= 1 - tol and pos.max() <= hi + tol
    assert abs(lam).max() / abs(lam).min() <= GOLD['prop_diag_precond']['kappa_bound'] + 1e-3


@pytest.mark.parametrize("p", [2, 3])
def test_gradient_against_central_differences(p):
    V, alpha, beta, mats, D, A, m, ct = _blocks(p, 5)
    Aw = learned.dof_weights(p)
    theta = np.random.default_rng(p).uniform(-0.3, 0.3, 6)
    f, g = learned.saddle_spread_gradient(A, m, ct, D, Aw, theta)
    h = 1e-6
    for j in range(6):
        e = np.zeros(6)
        e[j] = h
        fp, _ = learned.saddle_spread_gradient(A, m, ct, D, Aw, theta + e)
        fm, _ = learned.saddle_spread_gradient(A, m, ct, D, Aw, theta - e)
        assert abs((fp - fm) / (2 * h) - g[j]) <= 1e-5 * max(1.0, abs(g[j])), (j, (fp - fm) / (2 * h), g[j])


def test_descent_and_common_scaling():
    V, alpha, beta, mats, D, A, m, ct = _blocks(2, 6)
    Aw = learned.dof_weights(2)
    f0, _ = learned.saddle_spread_gradient(A, m, ct, D, Aw, np.zeros(6))
    f1, _ = learned.saddle_spread_gradient(A, m, ct, D, Aw, np.full(6, 0.5))
    assert abs(f1 - f0) > 1e-6
    th, fa, fb = learned.saddle_target(A, m, ct, D, 2, max_steps=10)
    assert abs(fa - f0) < 1e-12 and fb <= fa
