"""Pins of the oracle MINRES and of the whole discretisation: iterates equal a
library MINRES, the solution equals a direct solve, exact blocks converge in
three steps, and the manufactured Darcy problem converges at the rates of
mixed finite element theory."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import assemble, precond, minres, manufactured
from paper_2304_12387_amd import inputs


def make(n=2, p=2, problem=0, ess=0, seed=1):
    cfg = inputs.graddiv_jittered(n, p, seed_mesh=seed, seed_coef=seed + 10)
    m = assemble.Mesh(n, n, n, p, cfg['vertices'])
    c22 = cfg['c_22'] if problem == 0 else None
    return assemble.Problem(m, problem, cfg['c_mass'], c22, ess_sides=ess)


@pytest.mark.parametrize("problem", [0, 1])
def test_iterates_equal_library_minres(problem):
    prob = make(problem=problem)
    P = precond.BlockPreconditioner(prob)
    b = inputs.graddiv_rhs(prob.mesh.n_u, prob.mesh.n_q)
    if problem == 1:
        b[prob.mesh.n_u:] = np.random.default_rng(0).standard_normal(prob.mesh.n_q)
    A = prob.block_matrix()
    Mop = spla.LinearOperator(A.shape, matvec=P)
    for k in (1, 2, 5, 12):
        xs, _ = spla.minres(A, b, M=Mop, maxiter=k, rtol=1e-300)
        xo, it, _ = minres.minres(prob.apply, P, b, tol=0.0, maxiter=k)
        assert it == k
        assert np.linalg.norm(xs - xo) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("problem,ess", [(0, 0), (1, 0), (0, 63)])
def test_solution_matches_direct_solve(problem, ess):
    prob = make(n=3, p=2, problem=problem, ess=ess)
    P = precond.BlockPreconditioner(prob)
    b = inputs.graddiv_rhs(prob.mesh.n_u, prob.mesh.n_q)
    x, it, info = minres.minres(prob.apply, P, b, tol=1e-12)
    assert info['converged']
    eta = np.array(info['eta'])
    assert np.all(np.diff(eta) <= 1e-12 * eta[0])     # |eta| never increases
    A = prob.block_matrix()
    xd = spla.spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


@pytest.mark.parametrize("tau,expected", [(1.0, 3), (2.0, 3)])
def test_exact_blocks_three_eigenvalues_three_steps(tau, expected):
    """C = 0 with exact blocks: B^{-1}A has three distinct eigenvalues
    (Prop. 1 and 2), so MINRES terminates in at most three steps."""
    prob = make(n=2, p=2, problem=1)
    A = prob.block_matrix().toarray()
    nu = prob.mesh.n_u
    M = A[:nu, :nu]
    Dm = A[nu:, :nu]
    S = Dm @ np.linalg.solve(M, Dm.T)
    Binv = lambda r: np.concatenate([np.linalg.solve(tau * M, r[:nu]), np.linalg.solve(S, r[nu:])])
    b = np.random.default_rng(4).standard_normal(prob.mesh.n)
    x, it, info = minres.minres(lambda v: A @ v, Binv, b, tol=1e-12)
    assert it <= expected
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


def test_singular_schur_pure_flux_problem():
    """All boundary faces essential and gamma = 0: the pressure is fixed up to
    a constant; with a compatible right-hand side MINRES with the
    constant-removing AMG preconditioner converges (Section 4.2)."""
    prob = make(n=3, p=2, problem=1, ess=63)
    P = precond.BlockPreconditioner(prob)
    assert P.singular
    rng = np.random.default_rng(8)
    b = np.zeros(prob.mesh.n)
    b[:prob.mesh.n_u] = rng.uniform(-1, 1, prob.mesh.n_u)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    x, it, info = minres.minres(prob.apply, P, b, tol=1e-10)
    assert info['converged']
    r = b - prob.block_matrix() @ x
    assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("p", [1, 2])
def test_manufactured_darcy_rates(p):
    """||u - u_h|| and ||p - p_h|| are O(h^p); ||Pi_W p - p_h|| is at least
    O(h^{p+1}) on Cartesian meshes (standard mixed finite element theory)."""
    errs = []
    hs = []
    for n in (2, 4, 8):
        m = assemble.Mesh(n, n, n, p, inputs.box_vertices(n, n, n))
        prob = assemble.Problem(m, assemble.DARCY, np.ones(n ** 3), None)
        b = manufactured.darcy_rhs(prob)
        sol = spla.spsolve(prob.block_matrix().tocsc(), b)
        errs.append(manufactured.darcy_errors(prob, sol))
        hs.append(1.0 / n)
    for key, order in (('u', p), ('p', p), ('proj_p', p + 1)):
        e = np.array([d[key] for d in errs])
        slope = np.log(e[-2] / e[-1]) / np.log(hs[-2] / hs[-1])
        assert slope >= order - 0.2, (key, slope)


def test_cfg1_minres_matches_direct_and_manufactured_error():
    cfg = inputs.darcy_cube_4()
    m = assemble.Mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    prob = assemble.Problem(m, cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
    b = manufactured.darcy_rhs(prob)
    P = precond.BlockPreconditioner(prob)
    x, it, info = minres.minres(prob.apply, P, b, tol=cfg['tol'])
    xd = spla.spsolve(prob.block_matrix().tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
    e1 = manufactured.darcy_errors(prob, x)
    e2 = manufactured.darcy_errors(prob, xd)
    for k in e1:
        assert abs(e1[k] - e2[k]) <= 1e-8 * e2[k]


def _tensor_vertices(xs, ys, zs):
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing='ij')
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_layered_darcy_flux_boundary_reproduces_constant_flow(p):
    """Darcy with gamma = 0, every boundary face essential with the flux of
    u = (1, 0, 0) (the layered-reservoir boundary condition), on a
    non-uniform tensor grid.  With constant permeability the exact velocity is
    the constant (1, 0, 0), which RT_p reproduces, so the discrete u must be
    its flux interpolant on every face (interior ones included): this pins the
    flux reading of the dofs, the lifting and the singular Schur block."""
    xs = np.array([0.0, 20.0, 50.0, 60.0])
    ys = np.array([0.0, 10.0, 25.0, 30.0, 40.0])
    zs = np.array([0.0, 2.0, 5.0])
    m = assemble.Mesh(3, 4, 2, p, _tensor_vertices(xs, ys, zs))
    k = 3.7
    prob = assemble.Problem(m, assemble.DARCY, np.full(m.ne, k), None, ess_sides=63)
    ubc = assemble.constant_field_fluxes(m, (1.0, 0.0, 0.0))
    b = prob.lift_essential(np.zeros(m.n), ubc)
    # compatibility: the net boundary flux is zero
    assert abs(b[m.n_u:].sum()) <= 1e-10 * np.abs(b).max()
    P = precond.BlockPreconditioner(prob)
    assert P.singular
    x, it, info = minres.minres(prob.apply, P, b, tol=1e-12)
    assert info['converged']
    assert np.abs(x[:m.n_u] - ubc).max() <= 1e-9 * np.abs(ubc).max()
    # a second field: the flux of (0, 0, 1) is |cell| in z-sub-face units
    fz = assemble.constant_field_fluxes(m, (0.0, 0.0, 1.0))
    assert abs(fz[m.nface[0] + m.nface[1]:].reshape(-1, 4 * p, 3 * p)[0].sum() - 60.0 * 40.0) <= 1e-9


def test_layered_darcy_mass_conservation():
    """Variable permeability (a small layered field): D u = 0, so the flux
    through every refined x-plane equals the inflow Ly Lz."""
    cfg = inputs.darcy_layered(4, 5, 3, 2, seed=3)
    m = assemble.Mesh(4, 5, 3, 2, cfg['vertices'])
    prob = assemble.Problem(m, assemble.DARCY, cfg['c_mass'], None, ess_sides=63)
    ubc = assemble.constant_field_fluxes(m, (1.0, 0.0, 0.0))
    b = prob.lift_essential(np.zeros(m.n), ubc)
    P = precond.BlockPreconditioner(prob)
    x, it, info = minres.minres(prob.apply, P, b, tol=1e-12)
    assert info['converged']
    ux = x[:m.nface[0]].reshape(3 * 2, 5 * 2, 4 * 2 + 1)
    plane = ux.sum(axis=(0, 1))
    assert np.abs(plane - 5 * 10.0 * 3 * 2.0).max() <= 1e-8 * 100.0
