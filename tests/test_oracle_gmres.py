"""Pins of the oracle's GMRES and block-triangular preconditioner (the remark
on block-triangular preconditioners in Section 2.2).

* With exact blocks, A P^{-1} is unit lower triangular: every eigenvalue is 1,
  (A P^{-1} - I)^2 = 0, and GMRES converges in at most two iterations;
* GMRES solves to the sparse direct solution with the practical (M~, AMG)
  triangular preconditioner, restarted or not;
* GMRES without a preconditioner on a diagonal matrix with k distinct
  eigenvalues converges in k iterations (Krylov dimension)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import assemble, gmres
from paper_2304_12387_amd import inputs


def _problem(problem, p, ess, gamma=False, n=(2, 2, 1), seed=2):
    nx, ny, nz = n
    V = inputs.jittered_vertices(nx, ny, nz, 0.1, seed)
    m = assemble.Mesh(nx, ny, nz, p, V)
    rng = np.random.default_rng(seed)
    cm = inputs.loguniform(m.ne, 0.1, 10.0, rng)
    c22 = inputs.loguniform(m.ne, 0.1, 10.0, rng) if (problem == 0 or gamma) else None
    return assemble.Problem(m, problem, cm, c22, ess_sides=ess)


@pytest.mark.parametrize("problem,p,ess,gamma", [(0, 1, 0, False), (0, 2, 5, False), (1, 2, 63, True)],
                         ids=['graddiv_p1', 'graddiv_p2_ess', 'darcy_gamma_p2_flux'])
def test_exact_blocks_give_unit_spectrum_and_two_iterations(problem, p, ess, gamma):
    prob = _problem(problem, p, ess, gamma)
    P = gmres.TriangularPreconditioner(prob, schur='exact_blocks')
    A = prob.block_matrix().toarray()
    n = A.shape[0]
    Pinv = np.column_stack([P(e) for e in np.eye(n)])
    T = A @ Pinv
    E = T - np.eye(n)
    assert np.abs(E @ E).max() <= 1e-10 * max(1.0, np.abs(E).max())
    assert np.abs(np.linalg.eigvals(T) - 1.0).max() <= 1e-4   # defective: eigenvalue errors ~ sqrt(eps)
    b = np.random.default_rng(3).uniform(-1, 1, n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    x, it, info = gmres.gmres(prob.apply, P, b, tol=1e-12)
    assert it <= 2 and info['converged']
    assert np.linalg.norm(b - prob.apply(x)) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("restart", [30, 4])
def test_practical_preconditioner_solves(restart):
    prob = _problem(0, 2, 5, n=(3, 3, 2))
    P = gmres.TriangularPreconditioner(prob, amg_kwargs=dict(max_coarse=20))
    b = np.random.default_rng(4).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    x, it, info = gmres.gmres(prob.apply, P, b, tol=1e-10, restart=restart)
    assert info['converged']
    xd = spla.spsolve(prob.block_matrix().tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_krylov_dimension_bound():
    d = np.repeat([1.0, 2.0, 5.0, 7.5], 6)
    A = sp.diags(d)
    b = np.random.default_rng(5).uniform(-1, 1, d.size)
    x, it, info = gmres.gmres(lambda v: A @ v, lambda v: v, b, tol=1e-12)
    assert it == 4 and np.allclose(x, b / d, rtol=1e-10)
