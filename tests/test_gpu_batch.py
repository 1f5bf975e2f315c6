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


@pytest.mark.parametrize("launch", [(0, 2048, 1), (0, 7, 3), (1, 1024, 1), (1, 5, 2)],
                         ids=['one_launch', 'one_launch_small_grid', 'per_degree', 'per_degree_small_grid'])
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
    assert cfg['mode'] in (0, 1) and cfg['grid'] > 0 and cfg['tile_groups'] >= 1 and cfg['ms'] > 0
    y1 = torch.empty_like(x)
    ctx.batch_apply(x, y1)
    torch.cuda.synchronize()
    assert rel(y1.cpu().numpy(), y0.cpu().numpy()) <= 1e-15
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
