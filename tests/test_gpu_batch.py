"""Batches of independent instances of different sizes and degrees: the
batched (persistent, work-queue) apply in every launch variant against each
instance's oracle operator, and the batched MINRES against each instance's
solo solve (same iterations, same solution) and against the oracle."""
import numpy as np
import pytest

from gpu_helpers import gpu_context, oracle_problem, rel, to_dev, torch_cuda
from oracle import minres, precond
from paper_2304_12387_amd import inputs

pytestmark = pytest.mark.gpu


def _instances():
    # every degree 1..6, sizes with odd and even extents (ragged colour groups)
    I = inputs.batch_instances(n_inst=6, seed=7, nmin=2, nmax=4)
    for k, d in enumerate(I):
        d['p'] = k + 1
    I[2]['ess_sides'] = 63
    return I


@pytest.mark.parametrize("launch", [(0, 2048, 1), (0, 7, 3), (1, 1024, 1), (1, 5, 2), (2, 1, 1)],
                         ids=['one_launch', 'one_launch_small_grid', 'per_degree', 'per_degree_small_grid',
                              'per_instance'])
def test_batch_apply_matches_each_instance(launch):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = _instances()
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    ctx.batch_set_launch(*launch)
    off = ctx.batch_offsets
    x = np.random.default_rng(3).uniform(-1, 1, int(off[-1]))
    xd = to_dev(x)
    yd = torch.empty_like(xd)
    ctx.batch_apply(xd, yd)
    y32 = torch.empty_like(xd.float())
    ctx.batch_apply(xd.float(), y32, prec=hdivsp.HD_F32)
    torch.cuda.synchronize()
    y = yd.cpu().numpy()
    y32 = y32.double().cpu().numpy()
    for i, d in enumerate(I):
        prob = oracle_problem(d)
        seg = slice(off[i], off[i + 1])
        ref = prob.apply(x[seg])
        assert rel(y[seg], ref) <= 1e-12, i
        assert rel(y32[seg], ref) <= 1e-5, i
    ctx.close()


def test_batch_tuner_keeps_results():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = _instances()
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    off = ctx.batch_offsets
    x = to_dev(np.random.default_rng(4).uniform(-1, 1, int(off[-1])))
    y0 = torch.empty_like(x)
    ctx.batch_apply(x, y0)
    cfg = ctx.batch_tune()
    print('tuned', cfg, flush=True)
    assert cfg['mode'] in (0, 1, 2) and cfg['grid'] > 0 and cfg['tile_groups'] >= 1 and cfg['ms'] > 0
    y1 = torch.empty_like(x)
    ctx.batch_apply(x, y1)
    torch.cuda.synchronize()
    assert rel(y1.cpu().numpy(), y0.cpu().numpy()) <= 1e-15
    ctx.close()


def test_batch_launch_modes_agree_on_box_instances():
    """Instances on box grids (every element a parallelepiped): the
    persistent work-queue launch and each instance's own launch give the same
    result bit for bit (the instances' own launches keep the point-by-point
    factors of the work queue), and match the oracle."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = inputs.batch_instances(n_inst=3, seed=41, nmin=2, nmax=4, pmin=1, pmax=3)
    for d in I[:2]:
        d['vertices'] = inputs.box_vertices(d['nx'], d['ny'], d['nz'])
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    off = ctx.batch_offsets
    x = np.random.default_rng(5).uniform(-1, 1, int(off[-1]))
    xd = to_dev(x)
    ys = []
    for launch in (0, 2):
        ctx.batch_set_launch(launch, 2048, 1)
        y = torch.full_like(xd, np.nan)
        ctx.batch_apply(xd, y)
        torch.cuda.synchronize()
        ys.append(y)
    assert torch.equal(ys[0], ys[1])
    y = ys[0].cpu().numpy()
    for i, d in enumerate(I):
        seg = slice(off[i], off[i + 1])
        assert rel(y[seg], oracle_problem(d).apply(x[seg])) <= 1e-12, i
    ctx.close()


@pytest.mark.parametrize("mode", ['plain', 'prec32'])
def test_batch_minres_matches_solo_solves(mode):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = inputs.batch_instances(n_inst=4, seed=9, nmin=2, nmax=4, pmin=1, pmax=3)
    I[1]['ess_sides'] = 5
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    pp = hdivsp.precond_params(max_coarse=40)
    ctx.batch_build_precond(pp)
    off = ctx.batch_offsets
    b = np.random.default_rng(11).uniform(-1, 1, int(off[-1]))
    for i, d in enumerate(I):
        if d['ess_sides']:
            prob = oracle_problem(d)
            b[off[i]:off[i] + prob.mesh.n_u][prob.ess] = 0.0
    md = hdivsp.HD_MODE_PLAIN64 if mode == 'plain' else hdivsp.HD_MODE_PREC32
    sp = hdivsp.solve_params(tol=1e-10, max_it=3000, mode=md)
    bd = to_dev(b)
    xd = torch.zeros_like(bd)
    infos = ctx.batch_minres_solve(bd, xd, sp)
    x = xd.cpu().numpy()
    print(mode, [(f['iterations'], f['true_rel_res']) for f in infos], flush=True)
    for i, d in enumerate(I):
        seg = slice(off[i], off[i + 1])
        solo = gpu_context(d, precond=True, params=pp)
        xs = torch.zeros(int(off[i + 1] - off[i]), dtype=torch.float64, device='cuda')
        inf = solo.minres_solve(to_dev(b[seg]), xs, sp)
        solo.close()
        assert infos[i]['status'] == 0
        assert infos[i]['iterations'] == inf['iterations'], (i, infos[i], inf)
        assert rel(x[seg], xs.cpu().numpy()) <= 1e-10
        if mode == 'plain' and i == 0:
            prob = oracle_problem(d)
            P = precond.BlockPreconditioner(prob, amg_kwargs=dict(max_coarse=40))
            _, ito, _ = minres.minres(prob.apply, P, b[seg], tol=1e-10)
            assert abs(infos[i]['iterations'] - ito) <= 2
    ctx.close()


def test_batch_mixed_refinement_meets_the_fp64_tolerance():
    """HD_MODE_MIXED on a batch: each instance reaches the FP64 tolerance on
    its own true residual and its solution matches the oracle's direct solve
    of the same system; the inner iterations per instance stay within a few
    of the solo mixed solve (the batched and solo FP32 operators round
    alike up to the summation order)."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    import scipy.sparse.linalg as spla
    I = inputs.batch_instances(n_inst=4, seed=13, nmin=2, nmax=4, pmin=1, pmax=3)
    I[2]['ess_sides'] = 21
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    pp = hdivsp.precond_params(max_coarse=40)
    ctx.batch_build_precond(pp)
    off = ctx.batch_offsets
    b = np.random.default_rng(5).uniform(-1, 1, int(off[-1]))
    probs = []
    for i, d in enumerate(I):
        prob = oracle_problem(d)
        probs.append(prob)
        if d['ess_sides']:
            b[off[i]:off[i] + prob.mesh.n_u][prob.ess] = 0.0
    # instance 3 starts converged: its right-hand side is zero
    b[off[3]:off[4]] = 0.0
    sp = hdivsp.solve_params(tol=1e-10, max_it=3000, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5)
    bd = to_dev(b)
    xd = torch.full_like(bd, np.nan)
    infos = ctx.batch_minres_solve(bd, xd, sp)
    x = xd.cpu().numpy()
    print('mixed', [(f['iterations'], f['outer'], f['true_rel_res']) for f in infos], flush=True)
    for i, d in enumerate(I):
        seg = slice(off[i], off[i + 1])
        assert infos[i]['status'] == 0, (i, infos[i])
        if i == 3:
            assert infos[i]['iterations'] == 0 and np.all(x[seg] == 0.0)
            continue
        assert infos[i]['true_rel_res'] <= 1e-10 and infos[i]['outer'] >= 2
        # kappa_2(A) <= 1e5 for these instances, so a true relative residual
        # of 1e-10 bounds the relative error by 1e-5
        ref = spla.spsolve(probs[i].block_matrix().tocsc(), b[seg])
        assert rel(x[seg], ref) <= 1e-5, (i, rel(x[seg], ref))
        solo = gpu_context(d, precond=True, params=pp)
        xs = torch.zeros(int(off[i + 1] - off[i]), dtype=torch.float64, device='cuda')
        inf = solo.minres_solve(to_dev(b[seg]), xs, sp)
        solo.close()
        assert inf['status'] == 0 and inf['outer'] == infos[i]['outer'], (i, inf, infos[i])
        assert abs(inf['iterations'] - infos[i]['iterations']) <= 2 * inf['outer'], (i, inf, infos[i])
    ctx.close()


def test_batch_mixed_rejects_bad_refinement_parameters():
    from paper_2304_12387_amd import hdivsp
    I = inputs.batch_instances(n_inst=2, seed=3, nmin=2, nmax=2, pmin=1, pmax=2)
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    ctx.batch_build_precond(hdivsp.precond_params(max_coarse=40))
    torch = torch_cuda()
    n = int(ctx.batch_offsets[-1])
    bd = torch.ones(n, dtype=torch.float64, device='cuda')
    xd = torch.zeros_like(bd)
    for bad in (dict(inner_tol=0.0), dict(max_outer=0)):
        with pytest.raises(hdivsp.HdError) as e:
            ctx.batch_minres_solve(bd, xd, hdivsp.solve_params(mode=hdivsp.HD_MODE_MIXED, **bad))
        assert e.value.code == hdivsp.HD_ERR_ARG
    ctx.close()


@pytest.mark.parametrize("launch", [0, 2], ids=['persistent', 'per_instance'])
@pytest.mark.parametrize("mode", ['plain', 'prec32', 'mixed'])
def test_batch_graph_replays_match_eager_launches(mode, launch):
    """The batched recurrence replays each poll period as a HIP graph; with
    graphs off the same kernels run eagerly.  In both launch modes of the
    apply (persistent work queue, each instance's own launch) every mode
    gives the same iterations and the same solution bit for bit, over two
    solves in a row (each solve replays its graph several times)."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = inputs.batch_instances(n_inst=3, seed=17, nmin=2, nmax=4, pmin=1, pmax=3)
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    ctx.batch_set_launch(launch, 2048, 1)
    ctx.batch_build_precond(hdivsp.precond_params(max_coarse=40))
    n = int(ctx.batch_offsets[-1])
    b = to_dev(np.random.default_rng(23).uniform(-1, 1, n))
    md = {'plain': hdivsp.HD_MODE_PLAIN64, 'prec32': hdivsp.HD_MODE_PREC32, 'mixed': hdivsp.HD_MODE_MIXED}[mode]
    out = []
    for use_graph in (0, 1, 1):
        x = torch.full_like(b, np.nan)
        sp = hdivsp.solve_params(tol=1e-10, max_it=3000, mode=md, use_graph=use_graph, check_every=4)
        infos = ctx.batch_minres_solve(b, x, sp)
        torch.cuda.synchronize()
        assert all(f['status'] == 0 for f in infos), infos
        out.append(([f['iterations'] for f in infos], x.cpu().numpy()))
    print(mode, out[0][0], flush=True)
    for its, x in out[1:]:
        assert its == out[0][0]
        assert np.array_equal(x, out[0][1])
    ctx.close()


@pytest.mark.parametrize("mode", ['plain', 'prec32', 'mixed'])
def test_batch_shared_vcycle_equals_own_cycles(mode):
    """The levels >= 1 of all instances' V-cycles in shared launches (one per
    operation and level; FP64 in PLAIN64, FP32 in PREC32 and inside MIXED) give the
    iterations and the solution of every instance's own V-cycle launches bit
    for bit, with graphs and eagerly; hierarchies of different depths (every
    instance but the last has at least two levels)."""
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    I = inputs.batch_instances(n_inst=5, seed=29, nmin=3, nmax=6, pmin=2, pmax=4)
    I[1]['ess_sides'] = 21
    # and one instance whose hierarchy is a single (dense) level: it keeps its
    # own V-cycle launches beside the shared ones
    I.append(inputs.batch_instances(n_inst=1, seed=30, nmin=2, nmax=2, pmin=1, pmax=1)[0])
    ctx = hdivsp.Context(0)
    ctx.setup_batch(0, I)
    ctx.batch_build_precond(hdivsp.precond_params(max_coarse=40))
    n = int(ctx.batch_offsets[-1])
    b = to_dev(np.random.default_rng(31).uniform(-1, 1, n))
    md = {'plain': hdivsp.HD_MODE_PLAIN64, 'prec32': hdivsp.HD_MODE_PREC32, 'mixed': hdivsp.HD_MODE_MIXED}[mode]
    out = {}
    for shared in (1, 0):
        ctx.batch_set_vcycle(shared)
        for use_graph in (1, 0):
            x = torch.full_like(b, np.nan)
            sp = hdivsp.solve_params(tol=1e-10, max_it=3000, mode=md, use_graph=use_graph, check_every=4)
            infos = ctx.batch_minres_solve(b, x, sp)
            torch.cuda.synchronize()
            assert all(f['status'] == 0 for f in infos), infos
            out[(shared, use_graph)] = ([f['iterations'] for f in infos], x.cpu().numpy())
    print(mode, out[(1, 1)][0], flush=True)
    ref_its, ref_x = out[(0, 0)]
    for key, (its, x) in out.items():
        assert its == ref_its, key
        assert np.array_equal(x, ref_x), key
    with pytest.raises(hdivsp.HdError) as ei:
        ctx.batch_set_vcycle(2)
    assert ei.value.code == hdivsp.HD_ERR_ARG
    ctx.close()
