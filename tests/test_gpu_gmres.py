"""GPU block-triangular preconditioner and GMRES against the oracle (the
remark on block-triangular preconditioners, Section 2.2): P^{-1} r element by
element with the same AMG hierarchy, GMRES iterations and solution, restarts,
and the comparison with block-diagonal MINRES on the same system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_helpers import gpu_context, make_case, oracle_problem, rel, to_dev, torch_cuda
from oracle import gmres, minres, precond

pytestmark = pytest.mark.gpu

CASES = [(4, 3, 3, 2, 0, 5, False), (3, 3, 2, 3, 1, 63, False), (3, 2, 2, 2, 1, 21, True)]
IDS = ['graddiv_p2_ess', 'darcy_p3_all_flux', 'darcy_gamma_p2']


@pytest.mark.parametrize("c", CASES, ids=IDS)
def test_tri_precond_matches_oracle(c):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = make_case(*c[:4], problem=c[4], ess=c[5], gamma=c[6])
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True, params=hdivsp.precond_params(max_coarse=40))
    P = gmres.TriangularPreconditioner(prob, amg_kwargs=dict(max_coarse=40))
    r = np.random.default_rng(2).uniform(-1, 1, prob.mesh.n)
    z = torch.full((prob.mesh.n,), np.nan, dtype=torch.float64, device='cuda')
    ctx.apply_tri_precond(to_dev(r), z)
    assert rel(z.cpu().numpy(), P(r)) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("c", CASES, ids=IDS)
def test_gmres_matches_oracle(c):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = make_case(*c[:4], problem=c[4], ess=c[5], gamma=c[6])
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True, params=hdivsp.precond_params(max_coarse=40))
    P = gmres.TriangularPreconditioner(prob, amg_kwargs=dict(max_coarse=40))
    b = np.random.default_rng(3).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    if precond.schur_is_singular(prob):
        b[prob.mesh.n_u:] -= b[prob.mesh.n_u:].mean()
    _, ito, _ = gmres.gmres(prob.apply, P, b, tol=1e-10, restart=30)
    x = torch.zeros(prob.mesh.n, dtype=torch.float64, device='cuda')
    info = ctx.gmres_solve(to_dev(b), x, tol=1e-10, max_it=500, restart=30)
    xb = torch.zeros_like(x)
    im = ctx.minres_solve(to_dev(b), xb, hdivsp.solve_params(tol=1e-10, max_it=3000))
    print('gmres gpu', info, 'oracle', ito, 'minres', im['iterations'], flush=True)
    assert info['status'] == 0 and info['true_rel_res'] <= 1e-10
    assert abs(info['iterations'] - ito) <= 2
    A = prob.block_matrix()
    if precond.schur_is_singular(prob):
        xs = x.cpu().numpy()
        assert np.linalg.norm(b - A @ xs) <= 1e-9 * np.linalg.norm(b)
    else:
        assert rel(x.cpu().numpy(), spla.spsolve(A.tocsc(), b)) <= 1e-8
    ctx.close()


def test_gmres_restarts_and_initial_guess():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = make_case(4, 3, 3, 2, problem=0, ess=5)
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True, params=hdivsp.precond_params(max_coarse=40))
    b = np.random.default_rng(4).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    x = torch.zeros(prob.mesh.n, dtype=torch.float64, device='cuda')
    info = ctx.gmres_solve(to_dev(b), x, tol=1e-10, max_it=2000, restart=4)
    print('gmres(4)', info, flush=True)
    assert info['status'] == 0 and info['outer'] > 1 and info['true_rel_res'] <= 1e-10
    xd = spla.spsolve(prob.block_matrix().tocsc(), b)
    assert rel(x.cpu().numpy(), xd) <= 1e-8
    # the solution as initial guess: converged without an Arnoldi step
    info2 = ctx.gmres_solve(to_dev(b), x, tol=1e-8, max_it=10, restart=4)
    assert info2['status'] == 0 and info2['iterations'] == 0
    # the iteration limit is reported, not an error
    x.zero_()
    info3 = ctx.gmres_solve(to_dev(b), x, tol=1e-14, max_it=3, restart=30)
    assert info3['status'] == hdivsp.HD_NOT_CONVERGED and info3['iterations'] == 3
    ctx.close()
