"""The radiation-diffusion time step on the GPU (Section 4.3: SDIRK3 of
Alexander (1977), per-dof Newton for the exchange with the flux lagged, the
Darcy-type system for (E, F) by block-preconditioned MINRES) against the
oracle (oracle.raddiff, direct Darcy solves): the sub-cell volumes (<= 1e-13),
D F against the oracle's D of Algorithm 1 on structured and unstructured
meshes (<= 1e-13), whole steps on distorted meshes (e and E within 1e-8 of
the oracle, F within 1e-7), conservation of the total energy, the radiative
equilibrium as a steady state, an unstructured mesh against the same mesh
given as a structured grid, and the call-order and argument errors."""
import numpy as np
import pytest

from gpu_helpers import rel, to_dev, torch_cuda
from oracle import assemble, raddiff, unstructured as un
from paper_2304_12387_amd import inputs

pytestmark = pytest.mark.gpu


def _params(hdivsp, **kw):
    base = dict(rho=1.0, cv=1.0, c=1.0, a=1.0, sigma=1.0, dt=0.01, tol_outer=1e-11, lin_tol=1e-11)
    base.update(kw)
    return hdivsp.rd_params(**base)


def _initial(rd_or_vol, seed):
    vol = rd_or_vol.vol if hasattr(rd_or_vol, 'vol') else rd_or_vol
    rng = np.random.default_rng(seed)
    T = 1.0 + 0.5 * rng.random(vol.size)
    e = T * vol
    E = (0.6 * T) ** 4 * vol
    return e, E


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_subcell_volumes(p):
    torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case subcell volumes p', p, flush=True)
    V = inputs.jittered_vertices(3, 2, 2, 0.15, 7)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(3, 2, 2, p, V)
    vol = ctx.subcell_volumes().cpu().numpy()
    ref = raddiff.subcell_volumes(assemble.Mesh(3, 2, 2, p, V))
    assert rel(vol, ref) <= 1e-13
    assert abs(vol.sum() - ref.sum()) <= 1e-13 * ref.sum()
    ctx.close()


@pytest.mark.parametrize("p", [1, 2, 4])
def test_divergence_structured(p):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case divergence structured p', p, flush=True)
    V = inputs.jittered_vertices(3, 2, 4, 0.1, 8)
    m = assemble.Mesh(3, 2, 4, p, V)
    D = assemble.divergence_algorithm1(m)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(3, 2, 4, p, V)
    F = inputs.uniform_vector(m.n_u, 9)
    q = torch.empty(m.n_q, dtype=torch.float64, device='cuda')
    ctx.apply_divergence(to_dev(F), q)
    assert rel(q.cpu().numpy(), D @ F) <= 1e-13
    ctx.close()


@pytest.mark.parametrize("p", [1, 3])
def test_divergence_unstructured(p):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case divergence unstructured p', p, flush=True)
    V = inputs.jittered_vertices(3, 3, 2, 0.1, 4)
    Vv, el = inputs.from_structured(3, 3, 2, V)
    V2, el2, _ = inputs.scramble(Vv, el, 5)
    m = un.HexMesh(V2, el2, p)
    D = un.divergence_algorithm1(m)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh_unstructured(V2, el2, p)
    F = inputs.uniform_vector(m.n_u, 10)
    q = torch.empty(m.n_q, dtype=torch.float64, device='cuda')
    ctx.apply_divergence(to_dev(F), q)
    assert rel(q.cpu().numpy(), D @ F) <= 1e-13
    ctx.close()


STEP_CASES = [(2, 1, 1.0, 1.0, 0.02, 0), (3, 2, 1.0, 1.0, 0.01, 0), (2, 3, 1.0, 10.0, 0.005, 0),
              (2, 4, 2.0, 3.0, 0.01, 0), (3, 2, 1.0, 2.0, 0.01, 2), (3, 3, 1.0, 2.0, 0.01, 1)]


@pytest.mark.parametrize("case", STEP_CASES, ids=['n%d_p%d_c%g_s%g' % c[:4] + ['', '_mixed', '_prec32'][c[5]]
                                                 for c in STEP_CASES])
def test_step_matches_oracle(case):
    """lin_mode 2 = HD_MODE_PREC32 (the FP32 Schur V-cycle inside the FP64
    MINRES) and 1 = HD_MODE_MIXED (FP64 refinement around FP32 MINRES) reach
    the same states as the FP64 solves."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    n, p, c, sigma, dt, mode = case
    print('case rd step', case, flush=True)
    V = inputs.jittered_vertices(n, n, n, 0.15, 3)
    rd = raddiff.RadDiff(n, n, n, p, V, rho=1.3, cv=0.8, c=c, a=0.7, sigma=sigma)
    e, E = _initial(rd, 11)
    F = np.zeros(rd.mesh.n_u)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(n, n, n, p, V)
    ctx.rd_setup(_params(hdivsp, rho=1.3, cv=0.8, c=c, a=0.7, sigma=sigma, dt=dt, lin_mode=mode))
    ge, gE, gF = to_dev(e), to_dev(E), to_dev(F)
    for step in range(2):
        e, E, F, outers = rd.step(e, E, F, dt, tol_outer=1e-12)
        info = ctx.rd_step(ge, gE, gF)
        print('step', step, 'oracle outers', outers, 'gpu', info, flush=True)
        assert info['status'] == 0
        assert rel(ge.cpu().numpy(), e) <= 1e-8
        assert rel(gE.cpu().numpy(), E) <= 1e-8
        assert rel(gF.cpu().numpy(), F) <= 1e-7
        assert all(abs(a - b) <= 3 for a, b in zip(info['outer'], outers))
    ctx.close()


def test_energy_conserved_and_equilibrium_steady():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case rd conservation', flush=True)
    n, p = 4, 3
    V = inputs.jittered_vertices(n, n, n, 0.15, 5)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(n, n, n, p, V)
    ctx.rd_setup(_params(hdivsp, sigma=5.0, dt=0.02))
    vol = ctx.subcell_volumes().cpu().numpy()
    e, E = _initial(vol, 12)
    ge, gE = to_dev(e), to_dev(E)
    gF = torch.zeros(ctx.sizes()[0], dtype=torch.float64, device='cuda')
    tot0 = e.sum() + E.sum()
    for _ in range(3):
        info = ctx.rd_step(ge, gE, gF)
        assert info['status'] == 0
    tot = float(ge.sum() + gE.sum())
    assert abs(tot - tot0) <= 1e-9 * tot0
    ctx.close()

    # radiative equilibrium on a box mesh (the constants are in the space)
    print('case rd equilibrium', flush=True)
    Vb = inputs.box_vertices(3, 3, 3, 1.0, 0.7, 1.3)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(3, 3, 3, 2, Vb)
    rho, cv, a, T = 1.2, 2.0, 0.5, 1.3
    ctx.rd_setup(_params(hdivsp, rho=rho, cv=cv, a=a, sigma=3.0, dt=0.05))
    vol = ctx.subcell_volumes()
    ge = rho * cv * T * vol
    gE = a * T ** 4 * vol
    e0, E0 = ge.clone(), gE.clone()
    gF = torch.zeros(ctx.sizes()[0], dtype=torch.float64, device='cuda')
    info = ctx.rd_step(ge, gE, gF)
    assert info['status'] == 0
    assert rel(ge.cpu().numpy(), e0.cpu().numpy()) <= 1e-11
    assert rel(gE.cpu().numpy(), E0.cpu().numpy()) <= 1e-10
    assert float(gF.abs().max()) <= 1e-10 * float(gE.abs().max())
    ctx.close()


def test_unstructured_equals_structured():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case rd unstructured', flush=True)
    n, p = 3, 2
    V = inputs.jittered_vertices(n, n, n, 0.12, 6)
    Vv, el = inputs.from_structured(n, n, n, V)
    out = []
    for kind in ('structured', 'unstructured'):
        ctx = hdivsp.Context(0)
        if kind == 'structured':
            ctx.setup_mesh(n, n, n, p, V)
        else:
            ctx.setup_mesh_unstructured(Vv, el, p)
        ctx.rd_setup(_params(hdivsp, sigma=2.0, dt=0.01))
        vol = ctx.subcell_volumes().cpu().numpy()
        e, E = _initial(vol, 13)
        ge, gE = to_dev(e), to_dev(E)
        gF = torch.zeros(ctx.sizes()[0], dtype=torch.float64, device='cuda')
        for _ in range(2):
            assert ctx.rd_step(ge, gE, gF)['status'] == 0
        out.append((vol, ge.cpu().numpy(), gE.cpu().numpy()))
        ctx.close()
    assert rel(out[1][0], out[0][0]) <= 1e-14
    assert rel(out[1][1], out[0][1]) <= 1e-9
    assert rel(out[1][2], out[0][2]) <= 1e-9


def test_errors():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case rd errors', flush=True)
    ctx = hdivsp.Context(0)
    with pytest.raises(hdivsp.HdError) as ei:
        ctx.rd_setup(_params(hdivsp))
    assert ei.value.code == hdivsp.HD_ERR_STATE
    ctx.setup_mesh(2, 2, 2, 2, inputs.box_vertices(2, 2, 2))
    nu, nq = ctx.sizes()
    x = torch.ones(nq, dtype=torch.float64, device='cuda')
    y = torch.ones(nq, dtype=torch.float64, device='cuda')
    F = torch.zeros(nu, dtype=torch.float64, device='cuda')
    with pytest.raises(hdivsp.HdError) as ei:
        ctx.rd_step(x, y, F)
    assert ei.value.code == hdivsp.HD_ERR_STATE
    for bad in (dict(dt=0.0), dict(sigma=-1.0), dict(max_outer=0), dict(lin_mode=7), dict(c=float('nan'))):
        with pytest.raises(hdivsp.HdError) as ei:
            ctx.rd_setup(_params(hdivsp, **bad))
        assert ei.value.code == hdivsp.HD_ERR_ARG
    ctx.rd_setup(_params(hdivsp))
    rc = ctx.lib.hd_rd_step(ctx.h, hdivsp._ptr(x), hdivsp._ptr(x), hdivsp._ptr(F), None)
    assert rc == hdivsp.HD_ERR_ARG
    # a Newton iteration held to one step below an unreachable tolerance
    # fails in every dof: an error, and the caller's state is left as it was
    ctx.rd_setup(_params(hdivsp, newton_max_it=1, newton_tol=1e-300))
    vol = ctx.subcell_volumes()
    e0 = (1.0 + vol / vol.max()) * vol
    E0 = 0.3 * vol
    ge, gE, gF = e0.clone(), E0.clone(), F.clone()
    with pytest.raises(hdivsp.HdError) as ei:
        ctx.rd_step(ge, gE, gF)
    assert ei.value.code == hdivsp.HD_ERR_NONFINITE
    assert torch.equal(ge, e0) and torch.equal(gE, E0) and torch.equal(gF, F)
    # a new mesh drops the time-stepping state
    ctx.setup_mesh(2, 2, 2, 1, inputs.box_vertices(2, 2, 2))
    nu, nq = ctx.sizes()
    with pytest.raises(hdivsp.HdError) as ei:
        ctx.rd_step(x[:nq].clone(), y[:nq].clone(), torch.zeros(nu, dtype=torch.float64, device='cuda'))
    assert ei.value.code == hdivsp.HD_ERR_STATE
    ctx.close()
