"""Benchmark: GDOF/s of the matrix-free RT_p block apply and MINRES
time-to-1e-8, plain FP64 vs mixed precision, on one MI355X.

Default workload (`--workload graddiv32`): grad-div on the unit cube, 32^3
hexahedra with vertices jittered by +-10% h, RT order p = 4 (n_u = 6,340,608,
n_q = 2,097,152), alpha and beta per element log-uniform in [1e-2, 1e2];
right-hand side b_u ~ U[-1, 1], b_q = 0.  Synthetic seeded inputs; setup
(geometry, diagonals, S~, AMG) runs before the timed region and is reported
separately.

One step = NAPPLY back-to-back FP64 block applies (HIP events on the
library's stream bracket them), one plain FP64 MINRES solve to a true
relative residual of 1e-8 and one mixed-precision solve to the same true FP64
residual.  `value` is the apply throughput over the timed region:
(n_u + n_q) * applies / apply time; the applies reuse one input vector,
whose x and y (135 MB) the 256 MB memory-side cache can hold between applies,
and `apply_f64_gdofs_rotating_inputs` reports the same operator applied to
four alternating input/output pairs beside it.  `roofline.achieved` divides the
fixed-layout byte count of one launch (x and y, seven stored geometric
factors per quadrature point, two coefficients per element; half of the
elements per launch) by the event-timed launch; the kernel computes the
factors from the element vertices, so its measured HBM traffic
(`roofline.traffic`, from the committed counter summary) is lower.

Other workloads (`--workload`, one JSON line each, no CPU baseline):
  darcy_layered  60 x 220 x 85 cells, p = 2, layered log-normal permeability,
                 flux boundary condition: FP64 MINRES with the FP64 and with
                 the FP32 Schur V-cycle, and the mixed-precision solve, time
                 to a true residual of 1e-8.
  batch32        32 independent grad-div instances (n^3, n in 8..40, p in
                 1..6): batched apply in the autotuned launch mode (persistent
                 work queue, or each instance's own launch), FP64 and FP32.
  multirhs64     grad-div 64^3, p = 3, 16 right-hand sides: FP32 apply with the
                 right-hand sides interleaved ([dof][16]), beside the same
                 vectors stored one after the other.
  batch32_solve  the 32 instances of batch32 by one batched MINRES to a true
                 residual of 1e-8 (PLAIN64 and MIXED), per-instance iterations.
  batch_solve8   8 independent grad-div instances (n^3, n in 8..20, p in
                 1..4): one batched MINRES to a true residual of 1e-8 in each
                 mode, against the instances solved one after the other.
  local_inverse  grad-div on a 96^3 refined grid at p = 1, 2, 3: FP64 apply with
                 explicit element inverses of W_e (p <= 2) against the local CG.
  darcy_gamma32  Darcy on the jittered 32^3 p = 4 mesh with gamma varying inside
                 the elements: MINRES to 1e-8 and the apply beside the
                 piecewise-constant gamma.
  gmres32        the default system by GMRES(30) and GMRES(60) with the
                 block-triangular preconditioner, and by MINRES.
  distorted48    grad-div 48^3, p = 4 on a graded, sheared mesh: MINRES with
                 the plain and with the learned (1,1) diagonal (network
                 trained on GPU-generated targets first).
  unstructured32 the default system given as an unstructured mesh (turned
                 elements, renumbered vertices; grid and random element
                 order) beside the structured path: apply and MINRES.
  raddiff        grey nonlinear radiation diffusion, 96^3 hexahedra, p = 4
                 (--rd-n to change n): SDIRK3 steps of dt = h, each stage an
                 outer iteration of per-dof Newton solves and Darcy MINRES
                 solves; time per step, MINRES iterations per solve.
`cpu_baseline`: the CPU oracle on a bounded sample of the same workload (grad-div
on a jittered 6^3 mesh, p = 4, same coefficient distribution): its assembled
CSR apply on one host thread (GDOF/s, assembly excluded) and its MINRES with
the oracle's AMG, with the host CPU model and core count.

`--pmc-run` runs two FP64 applies of the default workload and an elementwise
kernel that reads and writes 1 GiB each (for counter collection under
rocprofv3 and its calibration; prints nothing else).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload NAME]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDOF/s of matrix-free RT_p block apply; MINRES time-to-1e-8 plain vs mixed"
NAPPLY = 20
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, 'profiles', 'block_apply_graddiv32_p4_traffic.json')
KERNEL_SOURCES = ['paper_2304_12387_amd/csrc/apply.hip', 'paper_2304_12387_amd/csrc/pencil.hpp',
                  'paper_2304_12387_amd/csrc/kernels_common.hpp', 'paper_2304_12387_amd/csrc/hd_internal.hpp']


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), 'rb') as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when it is missing or the kernel sources changed since."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get('kernel_source_sha256') != kernel_source_hash():
        return None
    return t.get('hbm_bytes_per_launch')


def cpu_baseline(n_sub=6, p=4, apply_s=3.0):
    """The CPU oracle on a bounded sample of the same workload: grad-div on a
    jittered n_sub^3 unit-cube mesh at degree p with the same coefficient
    distribution, assembled into CSR matrices by the oracle; then the
    assembled FP64 apply y = A x repeated for about apply_s seconds (GDOF/s,
    assembly excluded) and the oracle's MINRES with its smoothed-aggregation
    AMG preconditioner to |eta| <= 1e-9 (time and true relative residual,
    preconditioner setup reported separately).  The apply is timed on one
    thread and on all host cores available to the process (at most 16): the
    oracle's own CSR blocks split into row ranges, one per thread, which
    computes every row exactly as the one-thread apply does (scipy's sparse
    products release the interpreter lock).  The MINRES runs on one thread."""
    import platform
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import assemble, minres, precond
    from paper_2304_12387_amd import inputs

    cfg = inputs.graddiv_jittered(n_sub, p)
    cpu = platform.processor() or 'unknown'
    try:
        with open('/proc/cpuinfo') as fh:
            for line in fh:
                if line.startswith('model name'):
                    cpu = line.split(':', 1)[1].strip()
                    break
    except OSError:
        pass
    with threadpool_limits(1):
        t0 = time.perf_counter()
        mesh = assemble.Mesh(n_sub, n_sub, n_sub, p, cfg['vertices'])
        prob = assemble.Problem(mesh, cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
        t_asm = time.perf_counter() - t0
        x = inputs.uniform_vector(mesh.n, 32)
        k = 0
        ta = time.perf_counter()
        while time.perf_counter() - ta < apply_s:
            prob.apply(x)
            k += 1
        t_apply = (time.perf_counter() - ta) / k
        ncpu, t_all, k_all = apply_all_cores(prob, x, apply_s)
        t1 = time.perf_counter()
        P = precond.BlockPreconditioner(prob)
        t_prec = time.perf_counter() - t1
        b = inputs.graddiv_rhs(mesh.n_u, mesh.n_q, 22)
        t2 = time.perf_counter()
        xs, it, _ = minres.minres(prob.apply, P, b, tol=1e-9)
        t_solve = time.perf_counter() - t2
        rr = float(np.linalg.norm(b - prob.apply(xs)) / np.linalg.norm(b))
    mem_gb = None
    try:
        with open('/proc/meminfo') as fh:
            for line in fh:
                if line.startswith('MemTotal'):
                    mem_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except (OSError, ValueError):
        pass
    return {"value": mesh.n / t_all / 1e9, "unit": "GDOF/s", "cores": ncpu, "kind": "oracle",
            "sample": f"grad-div {n_sub}^3 jittered, p = {p} ({mesh.n} dofs), coefficients as in the workload: "
                      f"oracle's assembled-CSR FP64 apply (plain, unoptimised), {k_all} applies of "
                      f"{t_all * 1e3:.2f} ms on {ncpu} threads (row ranges of its CSR blocks) and {k} of "
                      f"{t_apply * 1e3:.1f} ms on 1 thread (assembly {t_asm:.1f} s excluded)",
            "value_1_core": mesh.n / t_apply / 1e9,
            "minres_s": round(t_solve, 3), "minres_iterations": it, "minres_true_rel_res": rr,
            "minres_stop": "|eta| <= 1e-9 |eta_0|", "amg_setup_s": round(t_prec, 3),
            "host_cpu": cpu, "host_nproc": os.cpu_count(), "host_mem_gb": mem_gb}


def apply_all_cores(prob, x, apply_s):
    """The oracle's apply y = [M D^T; D -C] x on all host cores available to
    the process (at most 16), its CSR blocks split into one row range per
    thread; checked equal to the one-thread apply.  Returns (threads, seconds
    per apply, applies timed)."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    ncpu = max(1, min(ncpu, 16))
    nu = prob.mesh.n_u
    xu = np.asarray(x[:nu], dtype=np.float64).copy()
    xu[prob.ess] = 0.0
    xq = np.asarray(x[nu:], dtype=np.float64)
    Dt = prob.D.T.tocsr()
    tasks = []
    for rows, top in ((nu, True), (prob.mesh.n_q, False)):
        cuts = np.linspace(0, rows, ncpu + 1).astype(int)
        for i in range(ncpu):
            a, b = int(cuts[i]), int(cuts[i + 1])
            if top:
                tasks.append((a, (prob.M[a:b], Dt[a:b])))
            else:
                tasks.append((nu + a, (prob.D[a:b], prob.C[a:b])))
    y = np.empty(prob.mesh.n)

    def run(task):
        off, (A, B) = task
        if off < nu:
            v = A @ xu + B @ xq
        else:
            v = A @ xu - B @ xq
        y[off:off + v.shape[0]] = v

    with ThreadPoolExecutor(ncpu) as pool:
        def apply():
            list(pool.map(run, tasks))
            y[:nu][prob.ess] = np.asarray(x[:nu])[prob.ess]
        apply()
        if not np.array_equal(y, prob.apply(x)):
            raise RuntimeError("threaded oracle apply differs from the one-thread apply")
        k = 0
        ta = time.perf_counter()
        while time.perf_counter() - ta < apply_s:
            apply()
            k += 1
        t = (time.perf_counter() - ta) / k
    return ncpu, t, k


def base_line(metric, value, unit, args, ms_per_step, config, higher=True, dtype="f64"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def time_applies(torch, stream, fn, n):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / n


def run_default(args, torch, hdivsp, inputs):
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.graddiv_jittered(args.n, args.p)
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nu, nq = ctx.sizes()
    N = nu + nq
    x = torch.from_numpy(inputs.uniform_vector(N, 32)).to(dev)
    y = torch.empty_like(x)
    if args.pmc_run:
        ctx.apply_block_op(x, y)
        ctx.apply_block_op(x, y)
        # counter calibration: an elementwise kernel that reads 1 GiB and
        # writes 1 GiB (a plain copy would go to the DMA engines)
        a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
        a.fill_(1.0)
        bcopy = torch.empty_like(a)
        torch.mul(a, 2.0, out=bcopy)
        torch.cuda.synchronize()
        ctx.close()
        return None
    ctx.build_precond()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ne = cfg['nx'] * cfg['ny'] * cfg['nz']
    q3 = (cfg['p'] + 1) ** 3
    bytes_per_apply = 16 * N + 8 * 7 * q3 * ne + 16 * ne
    x32 = x.float()
    y32 = torch.empty_like(x32)
    b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 22)).to(dev)
    sol = torch.zeros_like(b)
    p_plain = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    p_mixed = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def step(record):
        # one untimed apply ahead of the start event keeps the queue busy, so
        # that the events time the applies and not the host's first launch
        # after the previous step's synchronisation
        ctx.apply_block_op(x, y)
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
    rec = {'apply_ms': [], 'plain': [], 'mixed': []}
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    te = time.perf_counter()
    # FP32 apply throughput (after the timed region)
    f32_ms = time_applies(torch, stream, lambda: ctx.apply_block_op(x32, y32, prec=hdivsp.HD_F32), NAPPLY)
    # FP64 applies rotating over four input/output pairs (4 x 135 MB, more
    # than the 256 MB memory-side cache holds), after the timed region: the
    # same operator without cache reuse between consecutive applies
    xs = [x] + [torch.from_numpy(inputs.uniform_vector(N, 33 + k)).to(dev) for k in range(3)]
    ys = [torch.empty_like(x) for _ in range(4)]
    cnt = [0]

    def rotating():
        k = cnt[0] % 4
        cnt[0] += 1
        ctx.apply_block_op(xs[k], ys[k])
    rot_ms = time_applies(torch, stream, rotating, NAPPLY)
    del xs, ys

    apply_ms = sum(rec['apply_ms']) / (NAPPLY * args.steps)
    value = N / (apply_ms * 1e-3) / 1e9
    launch_ms = apply_ms / 2.0            # two launches (colours) per apply
    bytes_per_launch = bytes_per_apply / 2.0
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    med = lambda v: float(np.median(v))
    out = base_line(METRIC, round(value, 3), "GDOF/s", args, round((te - ts) * 1e3 / args.steps, 3),
                    {"workload": f"graddiv_jittered_{args.n}^3_p{args.p}", "nx": args.n, "p": args.p,
                     "n_u": nu, "n_q": nq, "coefficients": "alpha, beta log-uniform [1e-2, 1e2] per element",
                     "tol": 1e-8, "applies_per_step": NAPPLY})
    traffic = measured_traffic() if (args.n, args.p) == (32, 4) else None
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                       "kernel": f"block_apply_kernel<{args.p},double,true,false,false>",
                       "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": round(launch_ms, 5),
                       "launches_per_apply": 2}
    out["apply_f32_gdofs"] = round(N / (f32_ms * 1e-3) / 1e9, 3)
    out["apply_f64_gdofs_rotating_inputs"] = round(N / (rot_ms * 1e-3) / 1e9, 3)
    out["minres"] = {
        "plain_f64": {"time_to_1e-8_s": round(med([r['time_s'] for r in rec['plain']]), 4),
                      "iterations": rec['plain'][-1]['iterations'],
                      "true_rel_res": rec['plain'][-1]['true_rel_res']},
        "mixed": {"time_to_1e-8_s": round(med([r['time_s'] for r in rec['mixed']]), 4),
                  "iterations": rec['mixed'][-1]['iterations'], "outer": rec['mixed'][-1]['outer'],
                  "true_rel_res": rec['mixed'][-1]['true_rel_res']},
    }
    out["setup_s"] = {"mesh_coeffs": round(t1 - t0, 3), "precond": round(t2 - t1, 3)}
    out["amg_levels"] = ctx.amg_nlevels()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    ctx.close()
    return out


def run_darcy_layered(args, torch, hdivsp, inputs):
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.darcy_layered()
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], None, cfg['ess_sides'])
    ctx.build_precond()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nu, nq = ctx.sizes()
    b = torch.zeros(nu + nq, dtype=torch.float64, device=dev)
    ctx.lift_essential(ctx.constant_flux((1.0, 0.0, 0.0)), b)
    res = {}
    ts = time.perf_counter()
    for name, mode in (('plain_f64', hdivsp.HD_MODE_PLAIN64), ('prec32', hdivsp.HD_MODE_PREC32),
                       ('mixed', hdivsp.HD_MODE_MIXED)):
        times = []
        for _ in range(args.warmup + args.steps):
            x = torch.zeros_like(b)
            info = ctx.minres_solve(b, x, hdivsp.solve_params(tol=1e-8, mode=mode, stop_true=1, max_it=5000))
            times.append(info['time_s'])
        res[name] = {"time_to_1e-8_s": round(float(np.median(times[args.warmup:])), 4),
                     "iterations": info['iterations'], "true_rel_res": info['true_rel_res']}
        if mode == hdivsp.HD_MODE_MIXED:
            res[name]["outer"] = info.get('outer')
    te = time.perf_counter()
    x = torch.from_numpy(inputs.uniform_vector(nu + nq, 32)).to(dev)
    y = torch.empty_like(x)
    ms = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y), NAPPLY)
    out = base_line("MINRES time-to-1e-8 (s) of layered Darcy, FP32 Schur V-cycle in FP64 MINRES",
                    res['prec32']['time_to_1e-8_s'], "s", args,
                    round((te - ts) * 1e3 / (3 * (args.warmup + args.steps)), 3),
                    {"workload": "darcy_layered_60x220x85_p2", "n_u": nu, "n_q": nq,
                     "bc": "u.n = (1,0,0).n on the whole boundary"}, higher=False)
    out["minres"] = res
    out["apply_f64_gdofs"] = round((nu + nq) / (ms * 1e-3) / 1e9, 3)
    out["setup_s"] = round(t1 - t0, 3)
    out["amg_levels"] = ctx.amg_nlevels()
    ctx.close()
    return out


def run_batch32(args, torch, hdivsp, inputs):
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    inst = inputs.batch_instances()
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_batch(0, inst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    N = int(ctx.batch_offsets[-1])
    res = {}
    ts = time.perf_counter()
    for name, prec, dt in (('f64', hdivsp.HD_F64, torch.float64), ('f32', hdivsp.HD_F32, torch.float32)):
        tuned = ctx.batch_tune(prec)
        x = torch.rand(N, dtype=dt, device=dev)
        y = torch.empty_like(x)
        ms = time_applies(torch, stream, lambda: ctx.batch_apply(x, y, prec=prec), max(args.steps, 3))
        res[name] = {"gdofs": round(N / (ms * 1e-3) / 1e9, 3), "ms_per_apply": round(ms, 4), "tuned": tuned}
        # the best persistent work-queue launch (modes 0 and 1) beside the tuned one
        best = None
        for mode in (0, 1):
            for grid in (1024, 2048, 4096):
                for tg in (1, 2):
                    ctx.batch_set_launch(mode, grid, tg)
                    msp = time_applies(torch, stream, lambda: ctx.batch_apply(x, y, prec=prec), 3)
                    if best is None or msp < best[0]:
                        best = (msp, mode, grid, tg)
        res[name]["best_persistent"] = {"gdofs": round(N / (best[0] * 1e-3) / 1e9, 3), "mode": best[1],
                                        "grid": best[2], "tile_groups": best[3]}
        ctx.batch_set_launch(tuned['mode'], tuned['grid'], tuned['tile_groups'])
        del x, y
    te = time.perf_counter()
    out = base_line("GDOF/s of the batched block apply (32 instances, autotuned launch)",
                    res['f64']['gdofs'], "GDOF/s", args, round((te - ts) * 1e3, 3),
                    {"workload": "batch_32_graddiv_instances_n8-40_p1-6", "total_dofs": N,
                     "instances": [f"{d['nx']}^3 p{d['p']}" for d in inst]})
    out["batch"] = res
    out["setup_s"] = round(t1 - t0, 3)
    ctx.close()
    return out


def run_multirhs64(args, torch, hdivsp, inputs):
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.graddiv_jittered(64, 3, seed_mesh=4, seed_coef=14)
    ctx = hdivsp.Context(0, stream)
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
    nu, nq = ctx.sizes()
    N = nu + nq
    R = 16
    x = torch.rand(N * R, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    ts = time.perf_counter()
    # right-hand sides interleaved ([dof][16]): the timed configuration
    msil = time_applies(torch, stream, lambda: ctx.apply_block_op_interleaved(x, y, R, prec=hdivsp.HD_F32),
                        max(args.steps, 3))
    te = time.perf_counter()
    # the same 16 vectors stored one after the other, and one vector alone
    ms16 = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y, prec=hdivsp.HD_F32, nrhs=R),
                        max(args.steps, 3))
    ms1 = time_applies(torch, stream, lambda: ctx.apply_block_op(x[:N], y[:N], prec=hdivsp.HD_F32), NAPPLY)
    out = base_line("GDOF/s of the FP32 block apply with 16 right-hand sides", round(N * R / (msil * 1e-3) / 1e9, 3),
                    "GDOF/s", args, round((te - ts) * 1e3, 3),
                    {"workload": "graddiv_jittered_64^3_p3_x16rhs", "n_u": nu, "n_q": nq, "nrhs": R,
                     "layout": "interleaved [dof][nrhs]"}, dtype="f32")
    out["rhs_major_f32_gdofs"] = round(N * R / (ms16 * 1e-3) / 1e9, 3)
    out["single_rhs_f32_gdofs"] = round(N / (ms1 * 1e-3) / 1e9, 3)
    out["ms_per_apply"] = {"interleaved": round(msil, 4), "rhs_major": round(ms16, 4), "single": round(ms1, 4)}
    ctx.close()
    return out


def run_local_inverse(args, torch, hdivsp, inputs):
    """FP64 grad-div apply on the same 96^3 refined grid at p = 1, 2, 3
    (96, 48, 32 elements per side): explicit element inverses of W_e against
    the local CG in the (2,2) block (explicit only for p <= 2)."""
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    rows = {}
    ts = time.perf_counter()
    for p in (1, 2, 3):
        cfg = inputs.graddiv_jittered(96 // p, p)
        ctx = hdivsp.Context(0, stream)
        ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
        ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
        nu, nq = ctx.sizes()
        N = nu + nq
        x = torch.from_numpy(inputs.uniform_vector(N, 32)).to(dev)
        y = torch.empty_like(x)
        row = {"n": cfg['nx'], "dofs": N}
        modes = [('cg', hdivsp.HD_LOCAL_CG)] + ([('explicit', hdivsp.HD_LOCAL_EXPLICIT)] if p <= 2 else [])
        for name, mode in modes:
            ctx.set_local_solver(mode)
            ms = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y), NAPPLY)
            row[name + "_gdofs"] = round(N / (ms * 1e-3) / 1e9, 3)
            row[name + "_us_per_apply"] = round(ms * 1e3, 1)
        if p <= 2:
            row["explicit_speedup"] = round(row["cg_us_per_apply"] / row["explicit_us_per_apply"], 3)
        rows[f"p{p}"] = row
        del x, y
        ctx.close()
    te = time.perf_counter()
    out = base_line("GDOF/s of the FP64 grad-div apply at p = 2 with explicit element inverses (local CG beside it)",
                    rows['p2']['explicit_gdofs'], "GDOF/s", args, round((te - ts) * 1e3, 3),
                    {"workload": "graddiv_jittered_96^3_subvolumes_p1-3", "refined_grid": 96})
    out["local_inverse"] = rows
    return out


def run_darcy_gamma32(args, torch, hdivsp, inputs):
    """Darcy on the jittered 32^3 p = 4 mesh with gamma varying inside the
    elements (smooth log-normal vertex field): the full (2,2) block
    W^-1 W_gamma W^-1; apply throughput beside the same mesh with the
    element-mean piecewise-constant gamma (one W^-1 per apply), and MINRES to
    a true relative residual of 1e-8."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    n, p = 32, 4
    cfg = inputs.graddiv_jittered(n, p)
    gv = inputs.gamma_vertex_field(n, n, n, 31)
    ne = n ** 3
    # element means of the vertex values (the piecewise-constant comparison)
    G = gv.reshape(n + 1, n + 1, n + 1)
    gmean = sum(G[dz:dz + n, dy:dy + n, dx:dx + n] for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)).ravel() / 8
    ctx = hdivsp.Context(0, stream)
    ctx.setup_mesh(n, n, n, p, cfg['vertices'])
    nu, nq = ctx.sizes()
    N = nu + nq
    x = torch.from_numpy(inputs.uniform_vector(N, 32)).to(dev)
    y = torch.empty_like(x)
    ctx.setup_coeffs(1, cfg['c_mass'], gmean, 0)
    ms_pc = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y), NAPPLY)
    ctx.setup_coeffs(1, cfg['c_mass'], None, 0)
    ctx.set_gamma_field(gv)
    ms_field = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y), NAPPLY)
    t0 = time.perf_counter()
    ctx.build_precond()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 22)).to(dev)
    sol = torch.zeros_like(b)
    sp_ = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    for _ in range(args.warmup):
        sol.zero_()
        ctx.minres_solve(b, sol, sp_)
    times, info = [], None
    ts = time.perf_counter()
    for _ in range(args.steps):
        sol.zero_()
        torch.cuda.synchronize()
        info = ctx.minres_solve(b, sol, sp_)
        times.append(info['time_s'])
    te = time.perf_counter()
    value = float(np.median(times))
    out = base_line("MINRES time-to-1e-8 (s) of Darcy with gamma varying inside the elements", round(value, 4), "s",
                    args, round((te - ts) * 1e3 / args.steps, 3),
                    {"workload": "darcy_gamma_field_jittered_32^3_p4", "n_u": nu, "n_q": nq,
                     "gamma": "exp of a smooth Gaussian vertex field, sigma 1, correlation 2 vertices"},
                    higher=False)
    out["minres"] = {"iterations": info['iterations'], "true_rel_res": info['true_rel_res'], "status": info['status']}
    out["apply_f64_gdofs"] = {"gamma_field": round(N / (ms_field * 1e-3) / 1e9, 3),
                              "piecewise_constant_gamma": round(N / (ms_pc * 1e-3) / 1e9, 3)}
    out["setup_s"] = round(t1 - t0, 3)
    ctx.close()
    return out


def run_batch_solve8(args, torch, hdivsp, inputs):
    """Eight independent grad-div instances solved to a true relative residual
    of 1e-8 by one batched MINRES (one recurrence per instance, one batched
    apply per iteration, in the launch configuration the tuner picks for
    FP64) in each mode, and one after the other by solo solves in PLAIN64
    mode."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    inst = inputs.batch_instances(n_inst=8, seed=4, nmin=8, nmax=20, pmin=1, pmax=4)
    t0 = time.perf_counter()
    ctx = hdivsp.Context(0, stream)
    ctx.setup_batch(0, inst)
    ctx.batch_build_precond(hdivsp.precond_params())
    tuned = ctx.batch_tune(hdivsp.HD_F64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    off = ctx.batch_offsets
    N = int(off[-1])
    b_host = np.random.default_rng(40).uniform(-1.0, 1.0, N)
    b = torch.from_numpy(b_host).to(dev)
    x = torch.zeros_like(b)
    modes = (('plain', hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)),
             ('prec32', hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PREC32, stop_true=1)),
             ('mixed', hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5)))
    res = {}
    ts = time.perf_counter()
    for name, prm in modes:
        runs = []
        for rep in range(args.warmup + args.steps):
            x.zero_()
            torch.cuda.synchronize()
            infos = ctx.batch_minres_solve(b, x, prm)
            if rep >= args.warmup:
                runs.append(infos)
        res[name] = {"time_to_1e-8_s": round(float(np.median([r[0]['time_s'] for r in runs])), 4),
                     "iterations": [f['iterations'] for f in runs[-1]],
                     "worst_true_rel_res": max(f['true_rel_res'] for f in runs[-1]),
                     "status": [f['status'] for f in runs[-1]]}
    te = time.perf_counter()
    # the same PLAIN64 solve with every instance's V-cycle launched on its own
    ctx.batch_set_vcycle(0)
    tso = []
    for rep in range(args.warmup + args.steps):
        x.zero_()
        torch.cuda.synchronize()
        infos = ctx.batch_minres_solve(b, x, modes[0][1])
        if rep >= args.warmup:
            tso.append(infos[0]['time_s'])
    ctx.batch_set_vcycle(1)
    res["plain_own_vcycles"] = {"time_to_1e-8_s": round(float(np.median(tso)), 4),
                                "iterations": [f['iterations'] for f in infos]}
    ctx.close()
    solo_t, solo_it = 0.0, []
    pm = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    for i, d in enumerate(inst):
        s = hdivsp.Context(0, stream)
        s.setup_mesh(d['nx'], d['ny'], d['nz'], d['p'], d['vertices'])
        s.setup_coeffs(d['problem'], d['c_mass'], d['c_22'], d['ess_sides'])
        s.build_precond(hdivsp.precond_params())
        bi = b[int(off[i]):int(off[i + 1])].contiguous()
        xi = torch.zeros_like(bi)
        ts_i = []
        for rep in range(args.warmup + args.steps):
            xi.zero_()
            torch.cuda.synchronize()
            info = s.minres_solve(bi, xi, pm)
            if rep >= args.warmup:
                ts_i.append(info['time_s'])
        solo_t += float(np.median(ts_i))
        solo_it.append(info['iterations'])
        s.close()
    res["solo_plain_sum"] = {"time_to_1e-8_s": round(solo_t, 4), "iterations": solo_it}
    out = base_line("time-to-1e-8 (s) of one batched MINRES over 8 grad-div instances (PLAIN64)",
                    res["plain"]["time_to_1e-8_s"], "s", args, round((te - ts) * 1e3 / args.steps, 3),
                    {"workload": "batch_8_graddiv_instances_n8-20_p1-4", "total_dofs": N,
                     "instances": [f"{d['nx']}^3 p{d['p']}" for d in inst]}, higher=False)
    out["solvers"] = res
    out["batch_launch"] = tuned
    out["setup_s"] = round(t1 - t0, 3)
    return out


def run_gmres32(args, torch, hdivsp, inputs):
    """The default grad-div system (32^3, p = 4) solved to a true relative
    residual of 1e-8 by GMRES(m) with the block-triangular preconditioner
    (m = 30 and 60) and, beside it, by block-diagonal MINRES."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.graddiv_jittered(args.n, args.p)
    ctx = hdivsp.Context(0, stream)
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])
    ctx.build_precond()
    nu, nq = ctx.sizes()
    b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 22)).to(dev)
    x = torch.zeros_like(b)
    res = {}
    ts = time.perf_counter()
    for m in (30, 60):
        runs = []
        for rep in range(args.warmup + args.steps):
            x.zero_()
            torch.cuda.synchronize()
            info = ctx.gmres_solve(b, x, tol=1e-8, max_it=2000, restart=m)
            if rep >= args.warmup:
                runs.append(info)
        res[f"gmres{m}"] = {"time_to_1e-8_s": round(float(np.median([r['time_s'] for r in runs])), 4),
                            "iterations": runs[-1]['iterations'], "restarts": runs[-1]['outer'],
                            "true_rel_res": runs[-1]['true_rel_res'], "status": runs[-1]['status']}
    pm = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    runs = []
    for rep in range(args.warmup + args.steps):
        x.zero_()
        torch.cuda.synchronize()
        info = ctx.minres_solve(b, x, pm)
        if rep >= args.warmup:
            runs.append(info)
    res["minres"] = {"time_to_1e-8_s": round(float(np.median([r['time_s'] for r in runs])), 4),
                     "iterations": runs[-1]['iterations'], "true_rel_res": runs[-1]['true_rel_res']}
    te = time.perf_counter()
    out = base_line("time-to-1e-8 (s) of block-triangular GMRES(30) on grad-div 32^3 p = 4 (MINRES beside it)",
                    res["gmres30"]["time_to_1e-8_s"], "s", args, round((te - ts) * 1e3 / args.steps, 3),
                    {"workload": f"graddiv_jittered_{args.n}^3_p{args.p}", "n_u": nu, "n_q": nq}, higher=False)
    out["solvers"] = res
    ctx.close()
    return out


def run_distorted48(args, torch, hdivsp, inputs):
    """The learned (1,1) diagonal on the distorted 48^3, p = 4 grad-div mesh:
    the network is trained on 200,000 seeded single elements (targets
    generated on the GPU), then MINRES to a true relative residual of 1e-8
    with the plain diag(M) and with the learned diagonal, each in PLAIN64 and
    MIXED mode; the metric is learned + MIXED against plain PLAIN64."""
    from paper_2304_12387_amd import learned as driver
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    cfg = inputs.graddiv_distorted(48, 4)
    ctx = hdivsp.Context(0, stream)
    ctx.setup_mesh(cfg['nx'], cfg['ny'], cfg['nz'], cfg['p'], cfg['vertices'])
    ctx.setup_coeffs(cfg['problem'], cfg['c_mass'], cfg['c_22'], cfg['ess_sides'])

    def progress(msg):
        print(f'distorted48 {msg} ({time.perf_counter() - t0:.1f} s)', file=sys.stderr, flush=True)

    n_train = 200000
    t0 = time.perf_counter()
    hist = driver.train(ctx, n=n_train, seed=50, max_steps=10, epochs=20, batch=256, lr=2e-3, progress=progress)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    progress('trained')
    nu, nq = ctx.sizes()
    b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 25)).to(dev)
    # the targets themselves for the mesh's own elements (what the network
    # would have to predict exactly): element vertices gathered from the grid
    import numpy as np
    n = cfg['nx']
    Vg = np.asarray(cfg['vertices']).reshape(n + 1, n + 1, n + 1, 3)
    Ve = np.stack([np.stack([np.stack([Vg[dz:dz + n, dy:dy + n, dx:dx + n] for dx in (0, 1)], axis=3)
                             for dy in (0, 1)], axis=3) for dz in (0, 1)], axis=3)   # [z, y, x, dz, dy, dx, 3]
    Ve = np.ascontiguousarray(Ve.reshape(n ** 3, 2, 2, 2, 3))
    t0 = time.perf_counter()
    th_mesh, _, spr_mesh = ctx.learned_targets(cfg['p'], torch.from_numpy(Ve).to(dev), 10)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    ctx.set_diag_scalings(th_mesh)
    res = {}
    ts = time.perf_counter()
    modes = (('plain64', hdivsp.HD_MODE_PLAIN64), ('mixed', hdivsp.HD_MODE_MIXED))
    for name, flag in (('plain', 0), ('learned', 1), ('mesh_targets', 2)):
        t0 = time.perf_counter()
        rc = ctx.build_precond(hdivsp.precond_params(learned=flag))
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        for mname, mode in modes:
            if name == 'mesh_targets' and mode != hdivsp.HD_MODE_PLAIN64:
                continue
            x = torch.zeros_like(b)
            prm = hdivsp.solve_params(tol=1e-8, stop_true=1, max_it=5000, mode=mode, inner_tol=1e-5)
            times = []
            for _ in range(3):
                x.zero_()
                torch.cuda.synchronize()
                info = ctx.minres_solve(b, x, prm)
                times.append(info['time_s'])
            res[f'{name}_{mname}'] = {"time_to_1e-8_s": round(float(np.median(times)), 4),
                                      "iterations": info['iterations'], "outer": info.get('outer'),
                                      "true_rel_res": info['true_rel_res'], "precond_setup_s": round(tb, 3),
                                      "status": rc}
            progress(f'{name} {mname}: {res[f"{name}_{mname}"]["time_to_1e-8_s"]} s, {info["iterations"]} it')
    te = time.perf_counter()
    lm, pp = res['learned_mixed'], res['plain_plain64']
    out = base_line("MINRES time-to-1e-8 (s), learned (1,1) diagonal + mixed precision",
                    lm['time_to_1e-8_s'], "s", args, round((te - ts) * 1e3, 3),
                    {"workload": "graddiv_distorted_48^3_p4", "n_u": nu, "n_q": nq,
                     "compared_with": "plain diag(M), PLAIN64"}, higher=False)
    out["speedup_vs_plain64"] = round(pp['time_to_1e-8_s'] / lm['time_to_1e-8_s'], 3)
    out["minres"] = res
    out["training"] = {"elements": hist['n_train'] + hist['n_val'], "seconds": round(t_train, 2),
                       "final_train_loss": float(hist['train_loss'][-1]),
                       "final_val_loss": float(hist['val_loss'][-1]),
                       "mean_spread_plain": hist['spread0'], "mean_spread_targets": hist['spread_opt']}
    sm = spr_mesh.cpu().numpy()
    out["mesh_targets"] = {"seconds": round(t_targets, 2), "mean_spread_plain": float(sm[:, 0].mean()),
                           "mean_spread_targets": float(sm[:, 1].mean())}
    ctx.close()
    return out


def run_batch32_solve(args, torch, hdivsp, inputs):
    """The 32 independent grad-div instances of the batched apply solved by
    one batched MINRES to a true relative residual of 1e-8 (PLAIN64, then
    MIXED): per-instance iterations and residuals, the batched set-up (the
    instances' AMG hierarchies built on the GPU) timed separately."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    inst = inputs.batch_instances()
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_batch(0, inst)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.batch_build_precond(hdivsp.precond_params())
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tuned = ctx.batch_tune(hdivsp.HD_F64)
    off = ctx.batch_offsets
    N = int(off[-1])
    b = torch.from_numpy(np.random.default_rng(41).uniform(-1.0, 1.0, N)).to(dev)
    x = torch.zeros_like(b)
    res = {}
    ts = time.perf_counter()
    for name, prm in (('plain', hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)),
                      ('mixed', hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_MIXED, inner_tol=1e-5))):
        x.zero_()
        torch.cuda.synchronize()
        infos = ctx.batch_minres_solve(b, x, prm)
        res[name] = {"time_to_1e-8_s": round(infos[0]['time_s'], 4),
                     "iterations": [f['iterations'] for f in infos],
                     "worst_true_rel_res": max(f['true_rel_res'] for f in infos),
                     "status": [f['status'] for f in infos]}
        print(f"batch32 {name}: {res[name]['time_to_1e-8_s']} s", file=sys.stderr, flush=True)
    te = time.perf_counter()
    ctx.batch_set_vcycle(0)
    x.zero_()
    torch.cuda.synchronize()
    infos = ctx.batch_minres_solve(b, x, hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1))
    ctx.batch_set_vcycle(1)
    res["plain_own_vcycles"] = {"time_to_1e-8_s": round(infos[0]['time_s'], 4)}
    print(f"batch32 plain, own V-cycles: {res['plain_own_vcycles']['time_to_1e-8_s']} s", file=sys.stderr, flush=True)
    # the same instances solved one after the other (PLAIN64, each in its own
    # context; one untimed solve first)
    solo_t, solo_it = 0.0, []
    pm = hdivsp.solve_params(tol=1e-8, mode=hdivsp.HD_MODE_PLAIN64, stop_true=1)
    for i, d in enumerate(inst):
        s = hdivsp.Context(0, stream)
        s.setup_mesh(d['nx'], d['ny'], d['nz'], d['p'], d['vertices'])
        s.setup_coeffs(0, d['c_mass'], d['c_22'], d['ess_sides'])
        s.build_precond(hdivsp.precond_params())
        bi = b[int(off[i]):int(off[i + 1])].contiguous()
        xi = torch.zeros_like(bi)
        for rep in range(2):
            xi.zero_()
            torch.cuda.synchronize()
            info = s.minres_solve(bi, xi, pm)
        solo_t += info['time_s']
        solo_it.append(info['iterations'])
        s.close()
    res["solo_plain_sum"] = {"time_to_1e-8_s": round(solo_t, 4), "iterations": solo_it}
    print(f"batch32 solo sum: {round(solo_t, 4)} s", file=sys.stderr, flush=True)
    out = base_line("time-to-1e-8 (s) of one batched MINRES over 32 grad-div instances (PLAIN64)",
                    res['plain']['time_to_1e-8_s'], "s", args, round((te - ts) * 1e3, 3),
                    {"workload": "batch_32_graddiv_instances_n8-40_p1-6", "total_dofs": N,
                     "instances": [f"{d['nx']}^3 p{d['p']}" for d in inst]}, higher=False)
    out["solvers"] = res
    out["batch_launch"] = tuned
    out["setup_s"] = {"mesh_coeffs": round(t1 - t0, 3), "precond": round(t2 - t1, 3)}
    ctx.close()
    return out


def run_unstructured32(args, torch, hdivsp, inputs):
    """The default grad-div system (jittered 32^3, p = 4) given as an
    unstructured hexahedral mesh (element-to-vertex array, index-array gather
    and FP64 atomic face sums): once in the grid's element order with the
    vertices renumbered and every element turned by a random rotation of the
    reference cube, once with the elements in random order as well; beside it
    the structured path on the same mesh.  FP64 and FP32 apply throughput and
    MINRES to a true relative residual of 1e-8 (PLAIN64 and MIXED)."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    n, p = 32, 4
    cfg = inputs.graddiv_jittered(n, p)
    Vv, el = inputs.from_structured(n, n, n, cfg['vertices'])
    res = {}
    for kind in ('structured', 'unstructured_grid_order', 'unstructured_random_order'):
        ctx = hdivsp.Context(0, stream)
        cm, c22 = cfg['c_mass'], cfg['c_22']
        t0 = time.perf_counter()
        if kind == 'structured':
            ctx.setup_mesh(n, n, n, p, cfg['vertices'])
        else:
            V2, el2, eperm = inputs.scramble(Vv, el, 7)
            if kind == 'unstructured_grid_order':
                # undo the element permutation: element k is grid element k again
                inv = np.empty_like(eperm)
                inv[eperm] = np.arange(eperm.size)
                el2 = el2[inv]
            else:
                cm, c22 = cm[eperm], c22[eperm]
            ctx.setup_mesh_unstructured(V2, el2, p)
        ctx.setup_coeffs(0, cm, c22, 0)
        torch.cuda.synchronize()
        t_mesh = time.perf_counter() - t0
        nu, nq = ctx.sizes()
        N = nu + nq
        x = torch.from_numpy(inputs.uniform_vector(N, 32)).to(dev)
        y = torch.empty_like(x)
        ms64 = time_applies(torch, stream, lambda: ctx.apply_block_op(x, y), NAPPLY)
        x32 = x.float()
        y32 = torch.empty_like(x32)
        ms32 = time_applies(torch, stream, lambda: ctx.apply_block_op(x32, y32, prec=hdivsp.HD_F32), NAPPLY)
        t0 = time.perf_counter()
        ctx.build_precond()
        torch.cuda.synchronize()
        t_prec = time.perf_counter() - t0
        b = torch.from_numpy(inputs.graddiv_rhs(nu, nq, 22)).to(dev)
        sol = torch.zeros_like(b)
        r = {"setup_mesh_coeffs_s": round(t_mesh, 3), "precond_setup_s": round(t_prec, 3),
             "apply_f64_gdofs": round(N / (ms64 * 1e-3) / 1e9, 3), "apply_f32_gdofs": round(N / (ms32 * 1e-3) / 1e9, 3)}
        for mode, name in ((hdivsp.HD_MODE_PLAIN64, 'plain'), (hdivsp.HD_MODE_MIXED, 'mixed')):
            ts, info = [], None
            for _ in range(args.warmup + args.steps):
                sol.zero_()
                info = ctx.minres_solve(b, sol, hdivsp.solve_params(tol=1e-8, mode=mode, stop_true=1))
                ts.append(info['time_s'])
            r[name] = {"time_to_1e-8_s": round(float(np.median(ts[args.warmup:])), 4), "iterations": info['iterations'],
                       "true_rel_res": info['true_rel_res']}
        print(f"unstructured32 {kind}: {r}", file=sys.stderr, flush=True)
        res[kind] = r
        ctx.close()
    u = res['unstructured_grid_order']
    out = base_line("GDOF/s of the FP64 block apply on an unstructured hexahedral mesh", u['apply_f64_gdofs'], "GDOF/s",
                    args, round(1e3 * u['plain']['time_to_1e-8_s'], 3), {"workload": "graddiv_jittered_32^3_p4_as_unstructured_mesh", "n_u": nu, "n_q": nq})
    out["results"] = res
    return out


def run_raddiff(args, torch, hdivsp, inputs):
    """Grey nonlinear radiation diffusion (Section 4.3) at the size of the
    paper's run: 96^3 hexahedra, p = 4 (1.7e8 RT and 5.7e7 L2 unknowns), on a
    jittered unit cube with a Gaussian hot spot and the radiation out of
    equilibrium (Q = S = 0, F . n = 0); SDIRK3 steps of dt = h with c = sigma
    = rho = C_v = a = 1, outer tolerance 1e-12 relative, Newton 1e-8, each
    Darcy MINRES 1e-8 relative to its warm-started initial residual."""
    import numpy as np
    dev = torch.device('cuda', 0)
    stream = torch.cuda.current_stream(dev)
    n, p = args.rd_n, 4
    st = inputs.raddiff_hotspot(n)
    ctx = hdivsp.Context(0, stream)
    t0 = time.perf_counter()
    ctx.setup_mesh(n, n, n, p, st['vertices'])
    prm = hdivsp.rd_params(rho=1.0, cv=1.0, c=1.0, a=1.0, sigma=1.0, dt=1.0 / n, tol_outer=1e-12, newton_tol=1e-8,
                           lin_tol=1e-8, lin_mode=hdivsp.HD_MODE_PLAIN64)
    ctx.rd_setup(prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nu, nq = ctx.sizes()
    print(f"raddiff set-up {t1 - t0:.1f} s (n_u {nu}, n_q {nq})", file=sys.stderr, flush=True)
    vol = ctx.subcell_volumes()
    rep = p ** 3
    Tm = torch.from_numpy(st['T_mat']).to(dev).repeat_interleave(rep)
    Tr = torch.from_numpy(st['T_rad']).to(dev).repeat_interleave(rep)
    e = Tm * vol
    E = Tr ** 4 * vol
    del Tm, Tr
    e_init, E_init = e.clone(), E.clone()
    F = torch.zeros(nu, dtype=torch.float64, device=dev)
    energy0 = float(e.sum() + E.sum())

    def run_steps(tag):
        infos = []
        for k in range(args.warmup + args.steps):
            info = ctx.rd_step(e, E, F)
            print(f"raddiff {tag} step {k}: {info['time_s']:.3f} s, outer {info['outer']}, "
                  f"{info['linear_iterations']} MINRES it in {info['linear_solves']} solves", file=sys.stderr,
                  flush=True)
            if k >= args.warmup:
                infos.append(info)
        return infos

    infos = run_steps('PLAIN64')
    energy = float(e.sum() + E.sum())
    t_step = [i['time_s'] for i in infos]
    value = float(np.median(t_step))
    nsolve = sum(i['linear_solves'] for i in infos)
    nit = sum(i['linear_iterations'] for i in infos)
    out = base_line("time per SDIRK3 step (s) of grey nonlinear radiation diffusion", round(value, 4), "s", args,
                    round(1e3 * sum(t_step) / len(t_step), 3),
                    {"workload": f"raddiff_hotspot_jittered_{n}^3_p{p}", "n_u": nu, "n_q": nq, "dt": 1.0 / n,
                     "tolerances": {"outer": 1e-12, "newton": 1e-8, "minres": 1e-8}}, higher=False)
    out["steps_detail"] = infos
    out["minres_iterations_per_solve"] = round(nit / max(nsolve, 1), 1)
    out["outer_per_stage"] = round(sum(sum(i['outer']) for i in infos) / (3 * len(infos)), 2)
    out["newton_max_iterations"] = max(i['newton_max_it'] for i in infos)
    out["linear_solver_share"] = round(sum(i['linear_time_s'] for i in infos) / max(sum(t_step), 1e-30), 3)
    out["relative_energy_change"] = (energy - energy0) / energy0
    out["setup_s"] = round(t1 - t0, 3)
    # the same steps with the Schur-block V-cycle in FP32 inside the FP64
    # MINRES (HD_MODE_MIXED stops on the true residual, a stricter test than
    # the warm-started |eta| of the other modes: 4.4x the iterations at 32^3)
    for tag, mode in (('prec32', hdivsp.HD_MODE_PREC32),):
        prm.lin_mode = mode
        ctx.rd_setup(prm)
        e.copy_(e_init)
        E.copy_(E_init)
        F.zero_()
        iv = run_steps(tag.upper())
        nsv = sum(i['linear_solves'] for i in iv)
        out[tag] = {"time_per_step_s": round(float(np.median([i['time_s'] for i in iv])), 4),
                    "minres_iterations_per_solve": round(sum(i['linear_iterations'] for i in iv) / max(nsv, 1), 1),
                    "outer_per_stage": round(sum(sum(i['outer']) for i in iv) / (3 * len(iv)), 2),
                    "relative_energy_change": (float(e.sum() + E.sum()) - energy0) / energy0}
    ctx.close()
    return out


WORKLOADS = {'graddiv32': run_default, 'darcy_layered': run_darcy_layered, 'batch32': run_batch32,
             'multirhs64': run_multirhs64, 'distorted48': run_distorted48, 'local_inverse': run_local_inverse,
             'darcy_gamma32': run_darcy_gamma32, 'gmres32': run_gmres32, 'batch_solve8': run_batch_solve8,
             'batch32_solve': run_batch32_solve, 'raddiff': run_raddiff, 'unstructured32': run_unstructured32}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=3)
    ap.add_argument('--warmup', type=int, default=1)
    ap.add_argument('--no-cpu', action='store_true')
    ap.add_argument('--n', type=int, default=32)
    ap.add_argument('--p', type=int, default=4)
    ap.add_argument('--rd-n', type=int, default=96, help='elements per direction of the raddiff workload')
    ap.add_argument('--workload', default='graddiv32', choices=sorted(WORKLOADS))
    ap.add_argument('--pmc-run', action='store_true')
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the multi-GPU path is a "
              f"design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2304_12387_amd import hdivsp, inputs

    torch.cuda.init()
    fn = run_default if args.pmc_run else WORKLOADS[args.workload]
    out = fn(args, torch, hdivsp, inputs)
    if out is not None:
        print(json.dumps(out))


if __name__ == '__main__':
    main()
