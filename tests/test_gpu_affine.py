"""The block apply on meshes of parallelepipeds, where the trilinear map of
every element is affine and J^T J / det J is formed once per element (the
operator of eq. transformed-saddle-point, Section 3, unchanged): FP64 within
1e-12 and FP32 within 1e-5 of the oracle's assembled operator, grad-div and
Darcy, with and without essential sides, p = 1..6, on a box grid and on a
sheared one (J constant but not diagonal), both local solvers of the (2,2)
block at p <= 2; and the detection on box, sheared and jittered meshes."""
import numpy as np
import pytest

from gpu_helpers import oracle_problem, rel, to_dev, torch_cuda
from paper_2304_12387_amd import inputs

pytestmark = pytest.mark.gpu

# a constant linear map with positive determinant and all entries non-zero
SHEAR = np.array([[1.0, 0.3, -0.2], [0.1, 0.8, 0.25], [-0.15, 0.2, 1.1]])


def vertices(nx, ny, nz, kind):
    V = inputs.box_vertices(nx, ny, nz, 1.0, 0.8, 1.2)
    if kind == 'sheared':
        V = V @ SHEAR.T + np.array([0.5, -0.25, 2.0])
    elif kind == 'jittered':
        V = inputs.jittered_vertices(nx, ny, nz, 0.1, 5)
    return V


def case(nx, ny, nz, p, problem, ess, kind, seed=3):
    rng = np.random.default_rng(seed)
    ne = nx * ny * nz
    c_mass = inputs.loguniform(ne, 1e-2, 1e2, rng)
    c22 = inputs.loguniform(ne, 1e-2, 1e2, rng) if problem == 0 else None
    return dict(nx=nx, ny=ny, nz=nz, p=p, problem=problem, vertices=vertices(nx, ny, nz, kind), c_mass=c_mass,
                c_22=c22, ess_sides=ess)


CASES = [
    # (nx, ny, nz, p, problem, ess)
    (3, 2, 2, 1, 0, 0),
    (3, 2, 2, 2, 1, 0),
    (3, 2, 2, 2, 0, 63),
    (3, 2, 2, 3, 0, 21),
    (2, 2, 2, 4, 0, 0),
    (2, 2, 1, 5, 1, 63),
    (2, 1, 1, 6, 0, 0),
]


def _id(c, kind):
    return '%s_n%dx%dx%d_p%d_pb%d_ess%d' % ((kind,) + c)


PARAMS = [(c, k) for k in ('box', 'sheared') for c in CASES]


@pytest.mark.parametrize("c,kind", PARAMS, ids=[_id(c, k) for c, k in PARAMS])
def test_affine_apply_matches_oracle(c, kind):
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    print('case', _id(c, kind), flush=True)
    cs = case(*c, kind)
    prob = oracle_problem(cs)
    ctx = hdivsp.Context(0)
    ctx.setup_mesh(cs['nx'], cs['ny'], cs['nz'], cs['p'], cs['vertices'])
    assert ctx.mesh_affine()
    ctx.setup_coeffs(cs['problem'], cs['c_mass'], cs['c_22'], cs['ess_sides'])
    nu, nq = ctx.sizes()
    x = np.random.default_rng(11).uniform(-1, 1, nu + nq)
    y_ref = prob.apply(x)
    xd = to_dev(x)
    solvers = [hdivsp.HD_LOCAL_CG, hdivsp.HD_LOCAL_EXPLICIT] if cs['p'] <= 2 and cs['problem'] == 0 else [None]
    for solver in solvers:
        if solver is not None:
            ctx.set_local_solver(solver)
        yd = torch.full_like(xd, np.nan)
        ctx.apply_block_op(xd, yd)
        torch.cuda.synchronize()
        y = yd.cpu().numpy()
        assert np.isfinite(y).all()
        assert rel(y, y_ref) <= 1e-12, (solver, rel(y, y_ref))
        y32 = torch.full_like(xd.float(), np.nan)
        ctx.apply_block_op(xd.float(), y32, prec=1)
        torch.cuda.synchronize()
        assert rel(y32.double().cpu().numpy(), y_ref) <= 1e-5, solver
    ctx.close()


def test_affine_detection():
    """Box and sheared grids are affine; a jittered grid, and a box grid with
    one vertex moved by 1e-9 of the cell, are not."""
    from paper_2304_12387_amd import hdivsp
    ctx = hdivsp.Context(0)
    for kind, want in (('box', True), ('sheared', True), ('jittered', False)):
        ctx.setup_mesh(3, 2, 2, 2, vertices(3, 2, 2, kind))
        assert ctx.mesh_affine() == want, kind
    V = vertices(3, 2, 2, 'box')
    V[1 + 4 * (1 + 3 * 1), 0] += 1e-9   # vertex (1, 1, 1), interior
    ctx.setup_mesh(3, 2, 2, 2, V)
    assert not ctx.mesh_affine()
    ctx.close()
