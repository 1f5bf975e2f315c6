"""The allocation-free entry point hd_apply_tri_precond_noalloc, called
through the C ABI, against hd_apply_tri_precond on the same inputs: two
calls in a row on one device, the second on a smaller problem (the fixed
device array keeps the first call's contents), the singular Schur case
(pure flux boundary, gamma = 0), and the size and call-order errors."""
import ctypes

import numpy as np
import pytest

from gpu_helpers import gpu_context, make_case, rel, to_dev, torch_cuda

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(ctx, seed):
    torch = torch_cuda()
    nu, nq = ctx.sizes()
    r = to_dev(np.random.default_rng(seed).uniform(-1.0, 1.0, nu + nq))
    z_ref = torch.full_like(r, float('nan'))
    z_na = torch.full_like(r, float('nan'))
    ctx.apply_tri_precond(r, z_ref)
    rc = ctx.lib.hd_apply_tri_precond_noalloc(ctx.h, _ptr(r), _ptr(z_na))
    assert rc == 0, ctx.lib.hd_last_error(ctx.h)
    torch.cuda.synchronize()
    a, b = z_na.cpu().numpy(), z_ref.cpu().numpy()
    assert np.isfinite(a).all()
    return a, b


def test_noalloc_matches_allocating_entry_point():
    from paper_2304_12387_amd import hdivsp
    big = make_case(6, 5, 4, 3, problem=0, seed=3)
    small = make_case(3, 3, 2, 2, problem=1, ess=63, seed=4)    # gamma = 0, all sides essential: singular S~
    ctx_big = gpu_context(big, precond=True, params=hdivsp.precond_params(max_coarse=40))
    ctx_small = gpu_context(small, precond=True, params=hdivsp.precond_params(max_coarse=8))
    print('noalloc call 1: 6x5x4 p3 grad-div', flush=True)
    a1, b1 = _both(ctx_big, 1)
    print('noalloc call 2: 3x3x2 p2 Darcy, singular', flush=True)
    a2, b2 = _both(ctx_small, 2)
    print('differences', rel(a1, b1), rel(a2, b2), flush=True)
    # same kernels and fixed reduction order: equal to FP64 round-off
    assert rel(a1, b1) <= 1e-14 and rel(a2, b2) <= 1e-14
    # and the larger problem again after the smaller one
    a3, b3 = _both(ctx_big, 3)
    assert rel(a3, b3) <= 1e-14
    ctx_big.close()
    ctx_small.close()


def test_noalloc_errors():
    torch = torch_cuda()
    from paper_2304_12387_amd import hdivsp
    lib = hdivsp.load()
    case = make_case(2, 2, 2, 2, problem=0, seed=5)
    ctx = gpu_context(case)      # no preconditioner yet
    nu, nq = ctx.sizes()
    r = torch.zeros(nu + nq, dtype=torch.float64, device='cuda')
    z = torch.zeros_like(r)
    assert lib.hd_apply_tri_precond_noalloc(ctx.h, _ptr(r), _ptr(z)) == hdivsp.HD_ERR_STATE
    ctx.build_precond(hdivsp.precond_params(max_coarse=8))
    assert lib.hd_apply_tri_precond_noalloc(ctx.h, _ptr(r), _ptr(r)) == hdivsp.HD_ERR_ARG
    assert lib.hd_apply_tri_precond_noalloc(ctx.h, None, _ptr(z)) == hdivsp.HD_ERR_ARG
    ctx.close()
    # n_q = 43^3 * 6^3 = 17,173,512 > 2^24: rejected before any kernel
    from paper_2304_12387_amd import inputs
    n = 43
    big = hdivsp.Context(0)
    big.setup_mesh(n, n, n, 6, inputs.box_vertices(n, n, n))
    assert big.sizes()[1] > 1 << 24
    rc = lib.hd_apply_tri_precond_noalloc(big.h, _ptr(r), _ptr(z))
    assert rc == hdivsp.HD_ERR_ARG and b'exceeds' in lib.hd_last_error(big.h)
    big.close()
