"""GPU parity of the block apply, the L2 mass inverse, the diagonals and the
approximate Schur complement against the oracle (element by element on the
same seeded inputs)."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from gpu_helpers import c_block_errors, gpu_context, m_block_errors, make_case, oracle_problem, rel, to_dev, torch_cuda
from oracle import assemble, precond

pytestmark = pytest.mark.gpu

CASES = [
    # (nx, ny, nz, p, problem, ess, gamma)
    (3, 2, 2, 1, 0, 0, False),
    (3, 2, 2, 2, 0, 0, False),
    (3, 2, 2, 3, 0, 0, False),
    (2, 2, 3, 4, 0, 0, False),
    (2, 2, 1, 5, 0, 0, False),
    (2, 1, 1, 6, 0, 0, False),
    (3, 3, 2, 2, 1, 0, False),
    (3, 2, 2, 3, 1, 0, True),
    (3, 2, 2, 2, 1, 63, False),
    (2, 3, 2, 3, 0, 21, False),
]


def _id(c):
    return 'n%dx%dx%d_p%d_pb%d_ess%d%s' % (c[0], c[1], c[2], c[3], c[4], c[5], '_gamma' if c[6] else '')


@pytest.mark.parametrize("c", CASES, ids=[_id(c) for c in CASES])
def test_block_apply_f64_and_f32(c):
    torch = torch_cuda()
    print('case', _id(c), flush=True)
    case = make_case(*c[:4], problem=c[4], ess=c[5], gamma=c[6])
    prob = oracle_problem(case)
    ctx = gpu_context(case)
    nu, nq = ctx.sizes()
    assert (nu, nq) == (prob.mesh.n_u, prob.mesh.n_q)
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, nu + nq)
    y_ref = prob.apply(x)
    xd = to_dev(x)
    yd = torch.full_like(xd, np.nan)
    ctx.apply_block_op(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    assert np.isfinite(y).all()
    assert rel(y, y_ref) <= 1e-12, rel(y, y_ref)
    x32 = xd.float()
    y32 = torch.full_like(x32, np.nan)
    ctx.apply_block_op(x32, y32, prec=1)
    torch.cuda.synchronize()
    y32 = y32.double().cpu().numpy()
    assert rel(y32, y_ref) <= 1e-5, rel(y32, y_ref)
    # a second application into the same (dirty) output gives the same result
    ctx.apply_block_op(xd, yd)
    torch.cuda.synchronize()
    assert np.array_equal(yd.cpu().numpy(), y)
    # each block row on its own, and the (2,2) block alone
    assert rel(y[:nu], y_ref[:nu]) <= 1e-12 and rel(y[nu:], y_ref[nu:]) <= 1e-12
    e64, e32 = c_block_errors(ctx, prob.apply, nu, nu + nq)
    print('C block', e64, e32, flush=True)
    assert e64 <= 1e-12 and e32 <= 1e-5, (e64, e32)
    e64, e32 = m_block_errors(ctx, prob.apply, nu, nu + nq)
    print('M block', e64, e32, flush=True)
    assert e64 <= 1e-12 and e32 <= 1e-5, (e64, e32)
    ctx.close()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_mass_inverse(p):
    torch = torch_cuda()
    case = make_case(2, 2, 2, p, problem=0)
    prob = oracle_problem(case)
    ctx = gpu_context(case)
    x = np.random.default_rng(p).uniform(-1, 1, prob.mesh.n_q)
    y = torch.empty(prob.mesh.n_q, dtype=torch.float64, device='cuda')
    ctx.apply_mass_inverse(to_dev(x), y)
    assert rel(y.cpu().numpy(), prob.C @ x) <= 1e-12
    ctx.apply_l2_mass_inverse(to_dev(x), y)
    assert rel(y.cpu().numpy(), sp.linalg.spsolve(prob.W.tocsc(), x)) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("c", CASES, ids=[_id(c) for c in CASES])
def test_diagonals_and_schur(c):
    torch = torch_cuda()
    case = make_case(*c[:4], problem=c[4], ess=c[5], gamma=c[6])
    prob = oracle_problem(case)
    ctx = gpu_context(case, precond=True)
    m, w = ctx.get_diagonals()
    m = m.cpu().numpy()
    w = w.cpu().numpy()
    mo = precond.diag_M(prob)
    wo = precond.diag_W(prob)
    assert np.max(np.abs(m - mo) / np.abs(mo)) <= 1e-13
    assert np.max(np.abs(w - wo) / np.abs(wo)) <= 1e-13
    rp, ci, v = ctx.get_schur()
    S = sp.csr_matrix((v, ci, rp), shape=(prob.mesh.n_q, prob.mesh.n_q))
    So = precond.schur_by_formula(prob)
    assert np.array_equal(S.indptr, So.indptr) and np.array_equal(S.indices, So.indices)
    assert np.max(np.abs(S.data - So.data) / np.abs(So.data)) <= 1e-13
    assert (S != S.T).nnz == 0
    ctx.close()


def test_full_size_graddiv_32_p4_sampled_rows_and_symmetry():
    """grad-div 32^3, p = 4 (the benchmark workload): rows of selected
    elements against the oracle's element matrices, and symmetry of the
    operator <A x, z> = <x, A z> at full size."""
    torch = torch_cuda()
    from paper_2304_12387_amd import inputs
    cfg = inputs.graddiv_32()
    print('full size', cfg['name'], flush=True)
    ctx = gpu_context(cfg)
    nu, nq = ctx.sizes()
    assert (nu, nq) == (6340608, 2097152)
    x = inputs.uniform_vector(nu + nq, 32)
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    ctx.apply_block_op(xd, yd)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    mesh = assemble.Mesh(32, 32, 32, 4, cfg['vertices'])
    elems = np.array([0, 1, 31, 32 * 32 - 1, 16 + 32 * (16 + 32 * 16), 32 ** 3 - 1, 12345, 30000])
    qr, yq, ur, yu = assemble.apply_element_rows(mesh, 0, cfg['c_mass'], cfg['c_22'], 0, x, elems)
    assert rel(y[qr], yq) <= 1e-12
    assert rel(y[ur], yu) <= 1e-12
    # the (2,2) block alone: with u = 0 the L2 rows are -C q~, which is far
    # smaller than D u on random inputs
    xc = x.copy()
    xc[:nu] = 0.0
    ycd = torch.empty_like(xd)
    ctx.apply_block_op(to_dev(xc), ycd)
    torch.cuda.synchronize()
    qc, yqc, _, _ = assemble.apply_element_rows(mesh, 0, cfg['c_mass'], cfg['c_22'], 0, xc, elems)
    print('C block rows', rel(ycd.cpu().numpy()[qc], yqc), flush=True)
    assert rel(ycd.cpu().numpy()[qc], yqc) <= 1e-12
    # the (1,1) block alone: with q~ = 0 the RT rows are M u
    xm = x.copy()
    xm[nu:] = 0.0
    ctx.apply_block_op(to_dev(xm), ycd)
    torch.cuda.synchronize()
    _, _, um, yum = assemble.apply_element_rows(mesh, 0, cfg['c_mass'], cfg['c_22'], 0, xm, elems)
    print('M block rows', rel(ycd.cpu().numpy()[um], yum), flush=True)
    assert rel(ycd.cpu().numpy()[um], yum) <= 1e-12
    del ycd
    z = to_dev(inputs.uniform_vector(nu + nq, 33))
    az = torch.empty_like(z)
    ctx.apply_block_op(z, az)
    lhs = torch.dot(yd, z).item()
    rhs = torch.dot(xd, az).item()
    assert abs(lhs - rhs) <= 1e-12 * (torch.linalg.norm(yd) * torch.linalg.norm(z)).item()
    ctx.close()
