"""Darcy with gamma varying inside the elements (Section 2.4, the general
(2,2) block W^{-1} W_gamma W^{-1}): the GPU block apply (local CG and, for
p <= 2, explicit element inverses), S~ with C~ = diag(W)^{-1} diag(W_gamma)
diag(W)^{-1} and MINRES against the oracle; a constant field against the
piecewise-constant gamma; the call-order and argument errors."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gpu_helpers import c_block_errors, make_case, rel, to_dev, torch_cuda
from oracle import assemble, minres, precond
from paper_2304_12387_amd import inputs

pytestmark = pytest.mark.gpu


def _case(nx, ny, nz, p, ess, seed=21):
    c = make_case(nx, ny, nz, p, problem=1, ess=ess)
    c['gamma_v'] = inputs.gamma_vertex_field(nx, ny, nz, seed)
    return c


def _oracle(c):
    m = assemble.Mesh(c['nx'], c['ny'], c['nz'], c['p'], c['vertices'])
    return assemble.Problem(m, assemble.DARCY, c['c_mass'], ess_sides=c['ess_sides'], gamma_vertices=c['gamma_v'])


def _context(c, local=None):
    from paper_2304_12387_amd import hdivsp
    ctx = hdivsp.Context(0)
    if local is not None:
        ctx.set_local_solver(local)
    ctx.setup_mesh(c['nx'], c['ny'], c['nz'], c['p'], c['vertices'])
    ctx.setup_coeffs(1, c['c_mass'], None, c['ess_sides'])
    ctx.set_gamma_field(c['gamma_v'])
    return ctx


def _apply(ctx, x, prec=0):
    torch = torch_cuda()
    xd = to_dev(x) if prec == 0 else to_dev(x).float()
    yd = torch.full_like(xd, np.nan)
    ctx.apply_block_op(xd, yd, prec=prec)
    torch.cuda.synchronize()
    return yd.double().cpu().numpy()


@pytest.mark.parametrize("c", [(3, 2, 2, 1, 0), (2, 3, 2, 2, 21), (3, 2, 2, 3, 0), (2, 2, 2, 4, 63)],
                         ids=['p1', 'p2_ess', 'p3', 'p4_all_flux'])
def test_apply_matches_oracle(c):
    from paper_2304_12387_amd import hdivsp
    case = _case(*c)
    prob = _oracle(case)
    x = np.random.default_rng(5).uniform(-1, 1, prob.mesh.n)
    ref = prob.apply(x)
    modes = [hdivsp.HD_LOCAL_AUTO] + ([hdivsp.HD_LOCAL_CG] if case['p'] <= 2 else [])
    for mode in modes:
        ctx = _context(case, mode)
        y = _apply(ctx, x)
        assert rel(y, ref) <= 1e-12, (mode, rel(y, ref))
        assert rel(_apply(ctx, x, prec=1), ref) <= 1e-5
        # W^{-1} W_gamma W^{-1} alone (u = 0)
        e64, e32 = c_block_errors(ctx, prob.apply, prob.mesh.n_u, prob.mesh.n)
        print('C block', mode, e64, e32, flush=True)
        assert e64 <= 1e-12 and e32 <= 1e-5, (mode, e64, e32)
        ctx.close()


def test_constant_field_equals_piecewise_constant_gamma():
    case = _case(3, 2, 2, 2, 0)
    case['gamma_v'] = np.full_like(case['gamma_v'], 1.75)
    x = np.random.default_rng(6).uniform(-1, 1, 10 ** 5)
    ctx = _context(case)
    n = sum(ctx.sizes())
    y_field = _apply(ctx, x[:n])
    ctx.close()
    from gpu_helpers import gpu_context
    c2 = dict(case)
    c2['c_22'] = np.full(case['nx'] * case['ny'] * case['nz'], 1.75)
    ctx = gpu_context(c2)
    y_pc = _apply(ctx, x[:n])
    ctx.close()
    assert rel(y_field, y_pc) <= 1e-13


def test_schur_and_minres_match_oracle():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = _case(4, 3, 3, 2, 5)
    prob = _oracle(case)
    ctx = _context(case)
    ctx.build_precond(hdivsp.precond_params(max_coarse=40))
    rp, ci, v = ctx.get_schur()
    S = sp.csr_matrix((v, ci, rp), shape=(prob.mesh.n_q, prob.mesh.n_q))
    So = precond.schur_by_formula(prob)
    assert np.array_equal(S.indptr, So.indptr) and np.array_equal(S.indices, So.indices)
    assert np.max(np.abs(S.data - So.data) / np.abs(So.data)) <= 1e-13
    b = np.random.default_rng(9).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    P = precond.BlockPreconditioner(prob, amg_kwargs=dict(max_coarse=40))
    _, ito, _ = minres.minres(prob.apply, P, b, tol=1e-10)
    xd = torch.zeros(prob.mesh.n, dtype=torch.float64, device='cuda')
    info = ctx.minres_solve(to_dev(b), xd, hdivsp.solve_params(tol=1e-10, max_it=3000))
    print('gamma field MINRES gpu', info, 'oracle', ito, flush=True)
    assert info['status'] == 0 and abs(info['iterations'] - ito) <= 2
    xdir = spla.spsolve(prob.block_matrix().tocsc(), b)
    assert rel(xd.cpu().numpy(), xdir) <= 1e-8
    ctx.close()


def test_call_order_and_argument_errors():
    from paper_2304_12387_amd import hdivsp
    from gpu_helpers import gpu_context
    case = make_case(2, 2, 2, 2, problem=0)
    ctx = gpu_context(case)
    nv = 27
    with pytest.raises(hdivsp.HdError) as e:
        ctx.set_gamma_field(np.ones(nv))          # grad-div coefficients
    assert e.value.code == hdivsp.HD_ERR_STATE
    ctx.close()
    case = _case(2, 2, 2, 2, 0)
    ctx = _context(case)
    for bad, code in ((-np.ones(nv), hdivsp.HD_ERR_ARG), (np.zeros(nv), hdivsp.HD_ERR_ARG),
                      (np.full(nv, np.nan), hdivsp.HD_ERR_NONFINITE)):
        with pytest.raises(hdivsp.HdError) as e:
            ctx.set_gamma_field(bad)
        assert e.value.code == code
    torch = torch_cuda()
    y = torch.empty(ctx.sizes()[1], dtype=torch.float64, device='cuda')
    with pytest.raises(hdivsp.HdError) as e:
        ctx.apply_mass_inverse(y.clone(), y)
    assert e.value.code == hdivsp.HD_ERR_STATE
    ctx.close()


@pytest.mark.parametrize("mode", ['mixed', 'prec32'])
def test_reduced_precision_solves_with_gamma_field(mode):
    """The FP32 applies and V-cycles of the mixed and FP32-preconditioner
    solvers use the same gamma-field block; both reach the FP64 true
    residual."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    case = _case(4, 3, 3, 3, 5)
    prob = _oracle(case)
    ctx = _context(case)
    ctx.build_precond(hdivsp.precond_params(max_coarse=40))
    b = np.random.default_rng(12).uniform(-1, 1, prob.mesh.n)
    b[:prob.mesh.n_u][prob.ess] = 0.0
    md = hdivsp.HD_MODE_MIXED if mode == 'mixed' else hdivsp.HD_MODE_PREC32
    x = torch.zeros(prob.mesh.n, dtype=torch.float64, device='cuda')
    info = ctx.minres_solve(to_dev(b), x, hdivsp.solve_params(tol=1e-9, max_it=5000, mode=md, stop_true=1))
    print(mode, info, flush=True)
    assert info['status'] == 0 and info['true_rel_res'] <= 1e-9
    xdir = spla.spsolve(prob.block_matrix().tocsc(), b)
    assert rel(x.cpu().numpy(), xdir) <= 1e-7
    ctx.close()
