"""Several right-hand sides in one call (vectors stored one after the other):
every right-hand side must give what the oracle gives for it alone, and the
solver must treat each as an independent MINRES recurrence (same iteration
count as a single-right-hand-side solve, own stop test)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from gpu_helpers import gpu_context, make_case, oracle_problem, rel, to_dev, torch_cuda
from oracle import precond
from paper_2304_12387_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("c", [(3, 2, 2, 2, 0, 0), (5, 4, 3, 3, 1, 63), (2, 2, 2, 5, 0, 0)],
                         ids=['n3x2x2_p2_graddiv', 'n5x4x3_p3_darcy_ess', 'n2x2x2_p5_graddiv'])
def test_apply_several_rhs(c):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case', c, flush=True)
    case = make_case(*c[:4], problem=c[4], ess=c[5])
    prob = oracle_problem(case)
    ctx = gpu_context(case)
    n, nq = prob.mesh.n, prob.mesh.n_q
    R = 3
    X = np.random.default_rng(7).uniform(-1, 1, (R, n))
    xd = to_dev(X.reshape(-1))
    yd = torch.empty_like(xd)
    ctx.apply_block_op(xd, yd, nrhs=R)
    y32 = torch.empty_like(xd.float())
    ctx.apply_block_op(xd.float(), y32, prec=hdivsp.HD_F32, nrhs=R)
    torch.cuda.synchronize()
    Y = yd.cpu().numpy().reshape(R, n)
    Y32 = y32.double().cpu().numpy().reshape(R, n)
    for r in range(R):
        ref = prob.apply(X[r])
        assert rel(Y[r], ref) <= 1e-12
        assert rel(Y32[r], ref) <= 1e-5
        # the same as the single-vector call
        y1 = torch.empty(n, dtype=torch.float64, device='cuda')
        ctx.apply_block_op(xd[r * n:(r + 1) * n].contiguous(), y1)
        torch.cuda.synchronize()
        assert rel(Y[r], y1.cpu().numpy()) <= 1e-15
    # (2,2) block C for several L2 vectors
    Q = np.random.default_rng(8).uniform(-1, 1, (2, nq))
    qd = torch.empty(2 * nq, dtype=torch.float64, device='cuda')
    ctx.apply_mass_inverse(to_dev(Q.reshape(-1)), qd, nrhs=2)
    torch.cuda.synchronize()
    Qo = qd.cpu().numpy().reshape(2, nq)
    for r in range(2):
        assert rel(Qo[r], prob.C @ Q[r]) <= 1e-12
    ctx.close()


def test_large_mesh_several_rhs_equal_single_calls():
    """On a mesh of 4,096 element groups per colour (the multi-RHS block
    mapping walks each XCD's chunk of groups once per right-hand side) every
    right-hand side equals its single-vector call bit for bit (FP64 and
    FP32)."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    n1 = 32
    cfg = inputs.graddiv_jittered(n1, 2)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(n1, n1, n1, 2, cfg['vertices'])
    ctx.setup_coeffs(0, cfg['c_mass'], cfg['c_22'], 0)
    nu, nq = ctx.sizes()
    n = nu + nq
    R = 3
    X = torch.from_numpy(np.random.default_rng(8).uniform(-1, 1, R * n)).cuda()
    for prec, dt in ((hdivsp.HD_F64, torch.float64), (hdivsp.HD_F32, torch.float32)):
        x = X.to(dt)
        y = torch.empty_like(x)
        ctx.apply_block_op(x, y, prec=prec, nrhs=R)
        for r in range(R):
            y1 = torch.empty(n, dtype=dt, device='cuda')
            ctx.apply_block_op(x[r * n:(r + 1) * n].contiguous(), y1, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(y[r * n:(r + 1) * n], y1)
    ctx.close()


def test_precond_several_rhs():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = make_case(4, 3, 3, 2, problem=0)
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True, params=hdivsp.precond_params(max_coarse=40))
    P = precond.BlockPreconditioner(prob, amg_kwargs=dict(max_coarse=40))
    n = prob.mesh.n
    R = np.random.default_rng(3).uniform(-1, 1, (2, n))
    zd = torch.empty(2 * n, dtype=torch.float64, device='cuda')
    ctx.apply_precond(to_dev(R.reshape(-1)), zd, nrhs=2)
    torch.cuda.synchronize()
    Z = zd.cpu().numpy().reshape(2, n)
    for r in range(2):
        assert rel(Z[r], P(R[r])) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("mode", ['plain', 'stop_true', 'mixed'])
def test_minres_several_rhs(mode):
    """Three right-hand sides, one of them zero: each converges to the direct
    solution, with the iteration count of its own single solve; the zero one
    stops at once with x = 0."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('mode', mode, flush=True)
    case = make_case(4, 3, 3, 2, problem=0)
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True, params=hdivsp.precond_params(max_coarse=40))
    n, nu, nq = prob.mesh.n, prob.mesh.n_u, prob.mesh.n_q
    B = np.stack([inputs.graddiv_rhs(nu, nq, seed=31),
                  np.zeros(n),
                  np.random.default_rng(32).uniform(-1, 1, n)])
    if mode == 'plain':
        prm = hdivsp.solve_params(tol=1e-10, max_it=2000)
    elif mode == 'stop_true':
        prm = hdivsp.solve_params(tol=1e-8, max_it=2000, stop_true=1)
    else:
        prm = hdivsp.solve_params(tol=1e-8, max_it=2000, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5)
    bd = to_dev(B.reshape(-1))
    xd = torch.zeros_like(bd)
    infos = ctx.minres_solve(bd, xd, prm, nrhs=3)
    X = xd.cpu().numpy().reshape(3, n)
    A = prob.block_matrix().tocsc()
    print('infos', infos, flush=True)
    for r in range(3):
        inf = infos[r]
        assert inf['status'] == 0
        if r == 1:
            assert inf['iterations'] == 0 and np.all(X[r] == 0.0)
            continue
        x1 = torch.zeros(n, dtype=torch.float64, device='cuda')
        single = ctx.minres_solve(to_dev(B[r]), x1, prm)
        assert inf['iterations'] == single['iterations']
        assert rel(X[r], x1.cpu().numpy()) <= 1e-13
        xdir = spla.spsolve(A, B[r])
        if mode == 'plain':
            assert rel(X[r], xdir) <= 1e-7
        else:
            assert np.linalg.norm(B[r] - A @ X[r]) <= 1e-8 * np.linalg.norm(B[r]) * 1.0001
            assert inf['true_rel_res'] <= 1e-8
    ctx.close()
