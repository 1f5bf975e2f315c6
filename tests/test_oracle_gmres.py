"""Pins of the oracle's GMRES and block-triangular preconditioner (the remark
on block-triangular preconditioners in Section 2.2).

* With exact blocks, A P^{-1} is unit lower triangular: every eigenvalue is 1,
  (A P^{-1} - I)^2 = 0, and GMRES converges in at most two iterations;
* GMRES solves to the sparse direct solution with the practical (M~, AMG)
  triangular preconditioner, restarted or not;
* GMRES without a preconditioner on a diagonal matrix with k distinct
  eigenvalues converges in k iterations (Krylov dimension);
* each residual GMRES reports is the least-squares minimum over its Krylov
  space (Saad and Schultz's defining property), recomputed by brute force from
  an explicit Krylov basis and a QR projection, both for the first cycle and
  across a restart."""
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


def _min_residuals(AP, r0, k):
    """min over y in K_j(AP, r0) of ||r0 - AP y|| / ||r0|| for j = 1..k, from
    an explicit (column-normalised) Krylov basis and a QR projection."""
    cols, out = [], []
    v = r0 / np.linalg.norm(r0)
    for _ in range(k):
        cols.append(v)
        W = np.column_stack([AP(c) for c in cols])
        Q, _ = np.linalg.qr(W)
        res = r0 - Q @ (Q.T @ r0)
        out.append(np.linalg.norm(res) / np.linalg.norm(r0))
        v = AP(v)
        v = v / np.linalg.norm(v)
    return np.array(out)


def test_residuals_are_the_krylov_least_squares_minima():
    prob = _problem(0, 2, 5, n=(2, 2, 2), seed=7)
    P = gmres.TriangularPreconditioner(prob, amg_kwargs=dict(max_coarse=20))
    b = np.random.default_rng(8).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    AP = lambda v: prob.apply(P(v))
    k = 8
    # one cycle: GMRES(k) from x0 = 0 against the minima over K_j(AP, b)
    _, _, info = gmres.gmres(prob.apply, P, b, tol=1e-30, restart=k, maxiter=k)
    ref = _min_residuals(AP, b, k)
    assert np.allclose(info['res'][1:k + 1], ref, rtol=1e-8, atol=0), (info['res'][1:k + 1], ref)
    # a restart: the second cycle minimises over K_j(AP, r_k) with r_k the
    # residual of the first cycle's iterate
    x1, _, _ = gmres.gmres(prob.apply, P, b, tol=1e-30, restart=k, maxiter=k)
    r1 = b - prob.apply(x1)
    _, _, info2 = gmres.gmres(prob.apply, P, b, tol=1e-30, restart=k, maxiter=2 * k)
    ref2 = _min_residuals(AP, r1, 4) * np.linalg.norm(r1) / np.linalg.norm(b)
    assert np.allclose(info2['res'][k + 1:k + 5], ref2, rtol=1e-7, atol=0), (info2['res'][k + 1:k + 5], ref2)
    # the residuals never increase
    assert np.all(np.diff(info2['res']) <= 1e-12)
