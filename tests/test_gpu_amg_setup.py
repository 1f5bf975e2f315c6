"""The AMG hierarchy built on the GPU (hd_build_precond) against the
library's host builder of the same algorithm (hd_host_amg_build) on the same
S~ (Section 2.3, eq. approx-schur-entries; Prop. 5): every level matrix and
every prolongator equal bit for bit (the device code orders its sums and
products like the host code), and against the oracle's hierarchy to 1e-12;
also on meshes large enough that rows of the Galerkin products overflow the
kernels' LDS buffers, and with a singular S~."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_helpers import gpu_context, make_case, oracle_problem, torch_cuda
from oracle import precond

pytestmark = pytest.mark.gpu

CASES = [
    # (nx, ny, nz, p, problem, ess, max_coarse, check the oracle)
    (4, 3, 3, 2, 0, 0, 40, True),
    (3, 3, 3, 3, 1, 63, 20, True),       # Darcy, gamma = 0, all sides essential: singular S~
    (12, 12, 12, 2, 0, 0, 64, False),
    (8, 8, 8, 4, 0, 5, 100, False),
    (16, 14, 12, 3, 1, 0, 1024, False),
]


def _id(c):
    return 'n%dx%dx%d_p%d_pb%d_ess%d_mc%d' % c[:7]


@pytest.mark.parametrize("c", CASES, ids=[_id(c) for c in CASES])
def test_gpu_hierarchy_equals_host_builder(c):
    torch_cuda()
    from paper_2304_12387_amd import hdivsp
    nx, ny, nz, p, problem, ess, mc, with_oracle = c
    print('case', _id(c), flush=True)
    case = make_case(nx, ny, nz, p, problem=problem, ess=ess, gamma=False)
    params = hdivsp.precond_params(max_coarse=mc)
    ctx = gpu_context(case, precond=True, params=params)
    rp, ci, v = ctx.get_schur()
    singular = problem == 1 and case['c_22'] is None and ess == 63
    levels, prolongs = hdivsp.host_amg(rp, ci, v, singular=singular, params=params)
    L = ctx.amg_nlevels()
    print('levels', L, [lv[0][0] for lv in levels], flush=True)
    assert L == len(levels) and L >= 2
    for l in range(L):
        grp, gci, gv = ctx.get_amg_level(l)
        _, hrp, hci, hv = levels[l]
        assert np.array_equal(grp, hrp) and np.array_equal(gci, hci), l
        assert np.array_equal(gv, hv), (l, np.abs(gv - hv).max())
    for l in range(L - 1):
        shape, grp, gci, gv = ctx.get_amg_prolongator(l)
        hshape, hrp, hci, hv = prolongs[l]
        assert shape == hshape
        assert np.array_equal(grp, hrp) and np.array_equal(gci, hci), l
        assert np.array_equal(gv, hv), (l, np.abs(gv - hv).max())
    if with_oracle:
        prob = oracle_problem(case)
        P = precond.BlockPreconditioner(prob, amg_kwargs=dict(max_coarse=mc))
        assert P.amg.nlevels == L
        for l in range(L):
            grp, gci, gv = ctx.get_amg_level(l)
            A = sp.csr_matrix((gv, gci, grp), shape=P.amg.A[l].shape)
            assert abs((A - P.amg.A[l]).toarray()).max() <= 1e-12 * abs(P.amg.A[l]).max()
        for l in range(L - 1):
            shape, grp, gci, gv = ctx.get_amg_prolongator(l)
            Pg = sp.csr_matrix((gv, gci, grp), shape=shape)
            assert abs((Pg - P.amg.P[l]).toarray()).max() <= 1e-12
    ctx.close()
