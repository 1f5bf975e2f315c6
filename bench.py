"""Benchmark: GDOF/s of the matrix-free RT_p block apply and MINRES
time-to-1e-8, plain FP64 vs mixed precision, on one MI355X.

Workload: grad-div on the unit cube, 32^3 hexahedra with vertices jittered by
+-10% h, RT order p = 4 (n_u = 6,340,608, n_q = 2,097,152), alpha and beta per
element log-uniform in [1e-2, 1e2]; right-hand side b_u ~ U[-1, 1], b_q = 0.
Synthetic seeded inputs; setup (geometry, diagonals, S~, AMG) runs before the
timed region and is reported separately.

One step = NAPPLY back-to-back FP64 block applies (HIP events on the
library's stream bracket them), one plain FP64 MINRES solve to a relative
residual of 1e-8 and one mixed-precision solve to the same true FP64
residual.  `value` is the apply throughput over the timed region:
(n_u + n_q) * applies / apply time.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s of matrix-free RT_p block apply; MINRES time-to-1e-8 plain vs mixed"
NAPPLY = 20
HBM_PEAK_GBS = 8000.0


def cpu_baseline(cfg, n_dofs, budget_s=15.0):
    """The oracle's element-by-element FP64 apply (element matrices by
    quadrature, dense element products) on host cores, on a bounded sample of
    elements of the same workload, scaled to GDOF/s by the per-element share
    of the global dofs."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import assemble
    from paper_2304_12387_amd import inputs

    mesh = assemble.Mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    x = inputs.uniform_vector(mesh.n, 32)
    rng = np.random.default_rng(0)
    done = 0
    t_total = 0.0
    with threadpool_limits(1):
        while t_total < budget_s:
            elems = rng.choice(mesh.ne, 32, replace=False)
            t0 = time.perf_counter()
            assemble.apply_element_rows(mesh, cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'], x, elems)
            t_total += time.perf_counter() - t0
            done += len(elems)
    per_elem = n_dofs / mesh.ne
    return {"value": done * per_elem / t_total / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random elements of the same workload, element-by-element FP64 apply "
                      f"(oracle element matrices), {t_total:.1f} s on 1 host thread, scaled by "
                      f"{per_elem:.1f} dofs per element"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--no-cpu', action='store_true')
    ap.add_argument('--n', type=int, default=32)
    ap.add_argument('--p', type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU path is a "
              f"design, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2304_12387_amd import hdivsp, inputs

    torch.cuda.init()
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.graddiv_jittered(args.n, args.p)
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.build_precond()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    nu, nq = ctx.sizes()
    N = nu + nq
    ne = cfg['nx'] * cfg['ny'] * cfg['nz']
    q3 = (cfg['p'] + 1) ** 3
    bytes_per_apply = 16 * N + 8 * 7 * q3 * ne + 16 * ne

    x = torch.from_numpy(inputs.uniform_vector(N, 32)).to(dev)
    y = torch.empty_like(x)
    x32 = x.float()
    y32 = torch.empty_like(x32)
    b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 22)).to(dev)
    sol = torch.zeros_like(b)
    p_plain = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    p_mixed = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def step(record):
        ev0.record(stream)
        for _ in range(NAPPLY):
            ctx.apply_block_op(x, y)
        ev1.record(stream)
        ip = ctx.minres_solve(b, sol, p_plain)
        im = ctx.minres_solve(b, sol, p_mixed)
        torch.cuda.synchronize()
        if record is not None:
            record['apply_ms'].append(ev0.elapsed_time(ev1))
            record['plain'].append(ip)
            record['mixed'].append(im)

    for _ in range(args.warmup):
        step(None)
    # FP32 apply throughput (outside the timed region)
    ctx.apply_block_op(x32, y32, prec=hdivsp.HD_F32)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(NAPPLY):
        ctx.apply_block_op(x32, y32, prec=hdivsp.HD_F32)
    ev1.record(stream)
    torch.cuda.synchronize()
    f32_ms = ev0.elapsed_time(ev1) / NAPPLY

    rec = {'apply_ms': [], 'plain': [], 'mixed': []}
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    te = time.perf_counter()

    apply_ms = sum(rec['apply_ms']) / (NAPPLY * args.steps)
    value = N / (apply_ms * 1e-3) / 1e9
    achieved = bytes_per_apply / (apply_ms * 1e-3) / 1e9
    med = lambda v: float(np.median(v))
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round((te - ts) * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"graddiv_jittered_{args.n}^3_p{args.p}", "nx": args.n, "p": args.p,
                   "n_u": nu, "n_q": nq, "coefficients": "alpha, beta log-uniform [1e-2, 1e2] per element",
                   "tol": 1e-8, "applies_per_step": NAPPLY},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": f"block_apply_kernel<{args.p},double>",
                     "bytes_per_launch": bytes_per_apply, "avg_launch_ms": round(apply_ms, 5)},
        "apply_f32_gdofs": round(N / (f32_ms * 1e-3) / 1e9, 3),
        "minres": {
            "plain_f64": {"time_to_1e-8_s": round(med([r['time_s'] for r in rec['plain']]), 4),
                          "iterations": rec['plain'][-1]['iterations'],
                          "true_rel_res": rec['plain'][-1]['true_rel_res']},
            "mixed": {"time_to_1e-8_s": round(med([r['time_s'] for r in rec['mixed']]), 4),
                      "iterations": rec['mixed'][-1]['iterations'], "outer": rec['mixed'][-1]['outer'],
                      "true_rel_res": rec['mixed'][-1]['true_rel_res']},
        },
        "setup_s": {"mesh_coeffs": round(t1 - t0, 3), "precond": round(t2 - t1, 3)},
        "amg_levels": ctx.amg_nlevels(),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, N)
    ctx.close()
    print(json.dumps(out))


if __name__ == '__main__':
    main()
