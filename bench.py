#!/usr/bin/env python3
"""Benchmark: GMRES solves/sec at rtol 1e-6 for the one-level overlapping Schwarz (AS / ORAS)
preconditioned GMRES solve of the lowest-order Nedelec discretisation of
curl curl E - (k^2 + i xi) E = J on one MI355X.

One step = the whole path for one batch of synthetic input: box mesh and edge numbering,
partition with overlap, and for every (preconditioner, xi) instance of the batch: Galerkin
assembly, local problems + reverse Cuthill-McKee + batched factorisation, right-preconditioned
GMRES to rtol 1e-6 (true residual).  Right-hand sides are seeded per-DOF complex Gaussians,
already resident in HBM when the timed region starts.

Prints one JSON line.  Only one GPU is supported: --gpus N > 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# HBM bytes per forward-sweep launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs of the same
# command (FETCH_SIZE scaled by 2.0, WRITE_SIZE by 1.0: what the counters read for a 1 GiB
# device copy), averaged over the launches; summaries in profiles/.  Valid for the sweep kernel
# as it is now; None where not measured.
SWEEP_TRAFFIC = {("scale", "c128"): 58.85e9, ("scale", "c64"): 29.51e9, ("apply", "c128"): 65.82e9,
                 ("order2", "c128"): 12.55e9, ("batching", "c64"): 251.87e9}
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3


def factor_line(env_flops, tile_flops, seconds, precision):
    """The factorisation against its matrix-core roofline.  achieved_env: envelope LDL^T flops
    (8 sum_i w_i^2 / 2) per second; achieved_executed: the flops of the tiles the blocked
    factorisation runs, per second; mfma_util = achieved_executed / peak, the fraction of the
    matrix cores' peak rate the factorisation sustains over its whole duration (diagonal tiles,
    launches and stream hand-offs included).  A rocprofv3 counter run of the same workload
    (SQ_INSTS_VALU_MFMA_MOPS_F64 x 512) counts the same executed flops; its summary gives the
    per-kernel matrix-core busy fraction."""
    peak = FP64_PEAK_TFS if precision == "c128" else FP32_PEAK_TFS
    ex = tile_flops / seconds / 1e12 if seconds > 0 else 0.0
    return {"bound": "mfma", "achieved_env": env_flops / seconds / 1e12 if seconds > 0 else 0.0,
            "achieved_executed": ex, "peak": peak, "unit": "TFLOP/s", "mfma_util": ex / peak,
            "executed_tflop": tile_flops / 1e12, "seconds_total": seconds}


def instances(name):
    """(kind, xi exponent, rhs seed) of one batch."""
    if name == "scale":
        return [(kind, e, s) for kind in ("oras", "as") for s, e in enumerate((1.0, 1.5, 2.0))]
    if name == "scale-oras":
        return [("oras", e, s) for s, e in enumerate((1.0, 1.5, 2.0))]
    if name == "scale-xi0":  # here the exponent gives xi_prec; the problem has xi_prob = 0
        return [("oras", 1.0, 0), ("as", 1.0, 1)]
    if name == "small":
        return [("oras", 2.0, 0)]
    if name == "order2":  # xi_prob = xi_prec = k^2, then xi_prob = 0 with xi_prec = k
        return [("oras", 2.0, 0), ("oras", 1.0, 1)]
    if name == "scale-xi00":  # no absorption anywhere (exponent None: xi_prec = 0 too)
        return [("oras", None, 0)]
    raise SystemExit("unknown workload " + name)


def xi_prob_zero(name, idx):
    """Whether instance idx solves the problem without absorption (xi_prob = 0)."""
    return name in ("scale-xi0", "scale-xi00") or (name == "order2" and idx == 1)


def workload_desc(name):
    from mx_inputs import config_order2, config_scale, config_small
    if name == "order2":
        w = config_order2()
        return w, {"workload": "unit cube 24^3 cubes x 6 tets, second-order Nedelec elements "
                               "(542,736 complex DOFs), k=12, 4x4x4 subdomains, 1-layer overlap, "
                               "ORAS two-level hybrid with the coarse mesh of 4^3 cubes: xi_prob = "
                               "xi_prec = k^2, then ImpHRAS with xi_prob = 0, xi_prec = k; "
                               "GMRES(100) rtol 1e-6, complex128, seeded random complex Gaussian J",
                   "instances": len(instances(name))}
    if name == "scale-xi00":
        w = config_scale()
        return w, {"workload": "unit cube 64^3 cubes x 6 tets (1,872,064 complex DOFs), k=16, "
                               "no absorption anywhere (xi_prob = xi_prec = 0, as in Table "
                               "tab:EpsPrec0), 4x4x4 subdomains, 2-layer overlap, ORAS, GMRES(100) "
                               "rtol 1e-6, complex128, seeded random complex Gaussian J",
                   "instances": len(instances(name))}
    if name == "scale-xi0":
        w = config_scale()
        return w, {"workload": "unit cube 64^3 cubes x 6 tets (1,872,064 complex DOFs), k=16, "
                               "xi_prob = 0 (no absorption) preconditioned with xi_prec = k, "
                               "4x4x4 subdomains, 2-layer overlap, ORAS and AS, GMRES(100) rtol "
                               "1e-6, complex128, seeded random complex Gaussian J",
                   "instances": len(instances(name))}
    if name.startswith("scale"):
        w = config_scale()
        return w, {"workload": "unit cube 64^3 cubes x 6 tets (1,872,064 complex DOFs), k=16, "
                               "xi in {k, k^1.5, k^2}, 4x4x4 subdomains, 2-layer overlap, "
                               + ("ORAS and AS" if name == "scale" else "ORAS")
                               + ", GMRES(100) rtol 1e-6, complex128, seeded random complex "
                                 "Gaussian J", "instances": len(instances(name))}
    w = config_small()
    return w, {"workload": "unit cube 8^3 cubes x 6 tets, k=4, xi=k^2, 2x2x2 subdomains, ORAS, "
                           "GMRES(50), complex128", "instances": 1}


def cpu_baseline_small(w):
    """The oracle (NumPy/SciPy FP64, one thread) on the whole 8^3 case, end to end (mesh,
    assembly, partition, local factorisations, GMRES), repeated for about ten seconds.  Also
    returns the oracle's solution, against which every timed GPU solve is compared."""
    from threadpoolctl import threadpool_limits

    from oracle import dd, fem, gmres
    from oracle.mesh import Mesh as OMesh
    n, t0 = 0, time.perf_counter()
    with threadpool_limits(1):
        while n == 0 or time.perf_counter() - t0 < 10.0:
            m = OMesh(*w.n, *w.lengths)
            A = fem.assemble(m, w.k, w.xi)
            part = dd.Partition(m, *w.parts, w.layers)
            B = dd.Schwarz(part, A, dd.ORAS, w.k, w.xi)
            f = fem.load_vector(m, fem.gaussian_source(w.center, w.pol, w.sigma))
            res = gmres.gmres(A, f, B, restart=w.restart, rtol=w.rtol)
            n += 1
    el = time.perf_counter() - t0
    return {"value": n / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": "the whole 8^3 ORAS case solved by the oracle %d times in %.1f s (%d GMRES "
                      "iterations each)" % (n, el, res.iters)}, res.x


def cpu_baseline(total_iters, n_inst):
    """The oracle (NumPy/SciPy FP64) on a bounded sample of the same workload, its local problems
    on a pool of host worker processes (one per core, up to 16; the paper's one subdomain per
    core, Sec. 6.1):
    * global mesh + assembly + partition on the 32^3 box (1/8 of the 64^3 volume; scaled x8),
      one thread;
    * four ORAS local problems of each subdomain class (corner, edge, face, interior; 16 in
      all), taken from the 48^3 box cut into 3x3x3 boxes of 16^3 cubes with 2 layers, whose
      subdomains have exactly the shapes of the 64^3 benchmark's classes: assembled here, then
      factored (SuperLU) and solved once each, all concurrently on the pool.
    Estimated seconds per solve = 8 T_global + sum_c n_c (T_local_c + T_lu_c) / W
    + iterations * sum_c n_c T_solve_c / W, with the class counts n_c = 8, 24, 24, 8 of the
    64^3 partition, W workers and the GPU run's mean iteration count; solves/s is its inverse."""
    from threadpoolctl import threadpool_limits
    import numpy as np

    from mx_inputs import random_rhs
    from oracle import dd, fem, pool
    from oracle.mesh import Mesh as OMesh
    k, xi = 16.0, 16.0
    with threadpool_limits(1):
        t0 = time.perf_counter()
        m = OMesh(32, 32, 32)
        fem.assemble(m, k, xi)
        dd.Partition(m, 2, 2, 2, 2)
        t_global = time.perf_counter() - t0
        m48 = OMesh(48, 48, 48)
        part = dd.Partition(m48, 3, 3, 3, 2)
        classes = {"corner": 0, "edge": 1, "face": 4, "interior": 13}  # boxes of the 3x3x3 cut
        counts = {"corner": 8, "edge": 24, "face": 24, "interior": 8}  # in the 4x4x4 cut of 64^3
        tasks, names, t_loc = [], [], {}
        for name, l in classes.items():
            t1 = time.perf_counter()
            Al = dd.local_matrix(part, None, dd.ORAS, k, xi, l)
            t_loc[name] = time.perf_counter() - t1
            r = random_rhs(Al.shape[0], l)
            for _ in range(4):
                tasks.append((Al, r))
                names.append(name)
    W = min(pool.default_workers(), len(tasks))
    t2 = time.perf_counter()
    res = pool.solve_many(tasks, workers=W)
    t_pool = time.perf_counter() - t2
    t_lu = {c: np.mean([r[1] for r, nm in zip(res, names) if nm == c]) for c in classes}
    t_sv = {c: np.mean([r[2] for r, nm in zip(res, names) if nm == c]) for c in classes}
    iters = total_iters / max(n_inst, 1)
    per_solve = (8 * t_global + sum(counts[c] * (t_loc[c] + t_lu[c]) for c in classes) / W
                 + iters * sum(counts[c] * t_sv[c] for c in classes) / W)
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": W, "kind": "oracle",
            "host": {"cpu": model, "nproc": os.cpu_count(), "workers": W, "blas_threads": 1},
            "sample": "oracle global mesh+assembly+partition of the 32^3 box (x8, one thread); "
                      "16 ORAS local problems, 4 of each subdomain class (16^3-cube boxes with 2 "
                      "layers), assembled, factored (SuperLU) and solved on %d worker processes "
                      "at once (%.1f s wall), scaled to the 8/24/24/8 class counts of the 64^3 "
                      "partition over %d workers; GMRES iterations from the GPU run; per-solve "
                      "estimate %.0f s (global %.2f s, LU per class %s s, solve per class %s s)"
                      % (W, t_pool, W, per_solve, t_global,
                         "/".join("%.1f" % t_lu[c] for c in classes),
                         "/".join("%.3f" % t_sv[c] for c in classes))}


def cpu_baseline_order2(total_iters, n_inst):
    """The oracle (NumPy/SciPy FP64) on a bounded sample of the order-2 workload (24^3 cubes,
    4x4x4 subdomains, 1 layer, k = 12):
    * the order-2 space and global assembly of the whole box, one thread;
    * the ORAS local problems of one subdomain of each class (corner, edge, face, interior),
      assembled by the oracle, then factored (SuperLU) and solved once each on a pool of worker
      processes.
    Estimated seconds per solve = T_global + sum_c n_c (T_local_c + T_lu_c) / W
    + iterations * sum_c n_c T_solve_c / W, with the class counts n_c = 8, 24, 24, 8 and the GPU
    run's mean iteration count (the coarse level's solves, on 604 coarse DOFs, are left out)."""
    from threadpoolctl import threadpool_limits

    import numpy as np

    from mx_inputs import config_order2, random_rhs
    from oracle import dd, order2, pool
    from oracle.mesh import Mesh as OMesh
    w = config_order2()
    classes = {"corner": 0, "edge": 1, "face": 5, "interior": 21}
    counts = {"corner": 8, "edge": 24, "face": 24, "interior": 8}
    with threadpool_limits(1):
        t0 = time.perf_counter()
        om = OMesh(*w.n, *w.lengths)
        S = order2.Space(om)
        order2.assemble(S, w.k, w.xi)
        part = dd.Partition(om, *w.parts, w.layers)
        p2 = order2.Partition(S, part)
        t_global = time.perf_counter() - t0
        tasks, t_loc = [], {}
        for name, l in classes.items():
            t1 = time.perf_counter()
            Al = order2.local_matrix(p2, None, dd.ORAS, w.k, w.xi, l)
            t_loc[name] = time.perf_counter() - t1
            tasks.append((Al, random_rhs(Al.shape[0], l)))
    W = min(pool.default_workers(), 16)
    t2 = time.perf_counter()
    res = pool.solve_many(tasks, workers=W)
    t_pool = time.perf_counter() - t2
    t_lu = {c: r[1] for c, r in zip(classes, res)}
    t_sv = {c: r[2] for c, r in zip(classes, res)}
    iters = total_iters / max(n_inst, 1)
    per_solve = (t_global + sum(counts[c] * (t_loc[c] + t_lu[c]) for c in classes) / W
                 + iters * sum(counts[c] * t_sv[c] for c in classes) / W)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": W, "kind": "oracle",
            "sample": "oracle order-2 space and assembly of the whole 24^3 box (%.1f s, one thread); "
                      "ORAS local problems of one subdomain per class (corner, edge, face, interior), "
                      "assembled, factored (SuperLU) and solved on a pool (%.1f s wall); scaled to "
                      "the 8/24/24/8 class counts over %d workers with the GPU run's mean of %.0f "
                      "iterations: per-solve estimate %.1f s" % (t_global, t_pool, W, iters, per_solve)}


def cpu_baseline_batching(w, iters, n_sample=8, seed=11):
    """The oracle (NumPy/SciPy FP64) on a bounded sample of the 96x96x192 jittered-box problem:
    * n_sample subdomains drawn at random (seeded) from the 432: each one's ORAS local problem is
      assembled by the oracle on the sub-box around it (its box of cubes extended by the overlap
      layers, clipped to the domain, cut so that the subdomain is one box of that partition).  The
      layers only reach that far, and impedance on the sub-box boundary has the interface
      coefficient k, so this local matrix is the whole problem's (up to numbering).  The sample is
      factored (SuperLU) and solved once on a pool of worker processes;
    * the oracle's global mesh + assembly + partition, timed on a 32^3 box and scaled by the
      tetrahedron count (x54).
    Estimated seconds per solve = 54 T_global + 432 mean(T_local + T_lu) / W
    + iterations * 432 mean(T_solve) / W, with W workers and the GPU run's iteration count."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from mx_inputs import random_rhs
    from oracle import dd, fem, pool
    from oracle.mesh import Mesh as OMesh
    px, py, pz = w.parts
    nsub = px * py * pz
    rng = np.random.default_rng(seed)
    sample = sorted(rng.choice(nsub, n_sample, replace=False).tolist())
    tasks, t_loc, sizes = [], [], []
    with threadpool_limits(1):
        t0 = time.perf_counter()
        m32 = OMesh(32, 32, 32)
        fem.assemble(m32, w.k, w.xi)
        dd.Partition(m32, 2, 2, 2, w.layers)
        t_global = time.perf_counter() - t0
        for l in sample:
            t1 = time.perf_counter()
            _, part, lr, _, _, _ = dd.sub_box(w.n, w.lengths, w.parts, w.layers, w.cuts, l)
            Al = dd.local_matrix(part, None, dd.ORAS, w.k, w.xi, lr)
            t_loc.append(time.perf_counter() - t1)
            sizes.append(Al.shape[0])
            tasks.append((Al, random_rhs(Al.shape[0], l)))
    W = min(pool.default_workers(), len(tasks))
    t2 = time.perf_counter()
    res = pool.solve_many(tasks, workers=W)
    t_pool = time.perf_counter() - t2
    m_lu = float(np.mean([r[1] for r in res]))
    m_sv = float(np.mean([r[2] for r in res]))
    m_loc = float(np.mean(t_loc))
    per_solve = 54 * t_global + nsub * (m_loc + m_lu) / W + iters * nsub * m_sv / W
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": W, "kind": "oracle",
            "sample": "%d random subdomains of the 432 (n = %d .. %d), ORAS local problems "
                      "assembled on their sub-boxes, factored (SuperLU) and solved on %d worker "
                      "processes at once (%.1f s wall); global mesh+assembly+partition timed on "
                      "32^3 (%.2f s, x54); scaled to 432 subdomains over %d workers with the GPU "
                      "run's %d iterations: per-solve estimate %.0f s (mean LU %.1f s, mean solve "
                      "%.3f s)" % (len(tasks), min(sizes), max(sizes), W, t_pool, t_global, W,
                                   iters, per_solve, m_lu, m_sv)}


def run_batching(args):
    """The whole 96x96x192 jittered-box problem (12.5 M DOFs, 6x6x12 subdomains, ORAS, complex64
    factors) on one GPU: mesh, assembly, partition, preconditioner setup (factorised in subdomain
    groups that fit next to the trimmed factors) and FGMRES(50) to rtol 1e-6 with complex64 SpMV
    values.  The Gaussian source is resident in HBM before timing."""
    import torch

    from mx_inputs import config_batching
    from paper_1711_03789_amd import mx
    w = config_batching(0)
    ctx = mx.Context(0)
    mesh0 = mx.Mesh(*w.n, *w.lengths)
    E = mesh0.n_edge
    f = torch.from_numpy(mesh0.rhs_gaussian(w.center, w.pol, w.sigma)).cuda()
    del mesh0
    x = torch.zeros_like(f)
    torch.cuda.synchronize()

    def solve(record):
        t0 = time.perf_counter()
        mesh = mx.Mesh(*w.n, *w.lengths)
        A = mx.Matrix(ctx, mesh, w.k, w.xi)
        part = mx.Partition(mesh, *w.parts, w.layers, *w.cuts)
        t1 = time.perf_counter()
        P = mx.Precond(ctx, A, mesh, part, "oras", precision="c64")
        t2 = time.perf_counter()
        if record:
            P.sweep_timing(True)
        x.zero_()
        st = mx.gmres(ctx, A, P, f, x, restart=50, rtol=1e-6, max_iters=args.max_iters,
                      flexible=True, spmv_c64=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        tm = P.sweep_timing(False) if record else None
        inf = P.info()
        del P, A, part, mesh
        return (t0, t1, t2, t3), st, inf, tm

    for _ in range(args.warmup):
        solve(False)
    (t0, t1, t2, t3), st, inf, (nl, fms, bms) = solve(True)
    elapsed = t3 - t0
    sb = inf["sweep_bytes"]
    ach = sb / (fms / nl * 1e-3) / 1e9
    out = {
        "metric": "GMRES solves/sec at rtol 1e-6", "value": 1.0 / elapsed if st["converged"] else 0.0,
        "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "complex64 factors + FP64 FGMRES", "data": "synthetic",
        "config": {"workload": "box [0,1]x[0,1]x[0,2], 96x96x192 cubes x 6 tets (%d DOFs), k=xi=24, "
                               "6x6x12 subdomains with +-20%% jittered cut planes, 2-layer overlap, "
                               "ORAS, complex64 factors, FGMRES(50) rtol 1e-6, Gaussian source" % E,
                   "subdomains": inf["n_sub"], "factor_groups": inf["factor_groups"]},
        "iters": st["iters"], "relres_true": st["relres_true"],
        "roofline": {"bound": "hbm", "kernel": "k_sweep<float, true> (forward block sweep)",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": SWEEP_TRAFFIC.get(("batching", "c64")), "launches": nl,
                     "avg_launch_ms": fms / nl,
                     "bytes_per_launch": sb,
                     "backward": {"avg_launch_ms": bms / nl, "achieved": sb / (bms / nl * 1e-3) / 1e9}},
        "factor": {"bound": "mfma", "achieved_env": inf["env_flops"] / inf["t_factor"] / 1e12,
                   "achieved_executed": inf["tile_flops"] / inf["t_factor"] / 1e12,
                   "peak": FP32_PEAK_TFS, "unit": "TFLOP/s", "seconds": inf["t_factor"],
                   "tile_pool_bytes": inf["factor_bytes"], "pack_bytes": inf["pack_bytes"]},
        "phase_seconds": {"mesh_assemble_partition": t1 - t0, "precond_total": t2 - t1,
                          "precond_host": inf["t_host_setup"], "upload": inf["t_upload"],
                          "factor": inf["t_factor"], "pack": inf["t_pack"], "fgmres": t3 - t2},
        "local": {"n_local_total": inf["n_local_total"], "max_local": inf["max_local"],
                  "tiles": inf["tiles"], "max_blocks": inf["max_blocks"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batching(w, st["iters"])
    return out


def run_apply(args):
    """Schwarz-apply HBM GB/s on the 64^3 problem (ORAS, xi = k^2, resident factors): one plain
    device copy of known size first (the calibration kernel for HBM byte counters), then
    `reps` timed applications.  B_apply counts the envelope factor read twice, the local vectors
    and the gathers."""
    import torch

    from mx_inputs import config_scale, random_rhs
    from paper_1711_03789_amd import mx
    w = config_scale()
    ctx = mx.Context(0)
    mesh = mx.Mesh(*w.n, *w.lengths)
    part = mx.Partition(mesh, *w.parts, w.layers)
    A = mx.Matrix(ctx, mesh, w.k, w.k ** 2)
    P = mx.Precond(ctx, A, mesh, part, "oras", precision=args.precision)
    inf = P.info()
    E = mesh.n_edge
    # calibration: copy of 2 GiB (1 GiB read + 1 GiB written)
    src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    dst.copy_(src)
    torch.cuda.synchronize()
    t_copy = time.perf_counter() - c0
    del src, dst
    v = torch.from_numpy(random_rhs(E, 0)).cuda()
    z = torch.zeros_like(v)
    P.apply(v, z)
    torch.cuda.synchronize()
    P.sweep_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.reps):
        P.apply(v, z)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    nl, fms, bms = P.sweep_timing(False)
    P.check()
    sb = inf["sweep_bytes"]
    t_app = (t1 - t0) / args.reps
    ach = sb / (fms / nl * 1e-3) / 1e9
    return {
        "metric": "Schwarz-apply HBM GB/s", "value": inf["apply_bytes"] / t_app / 1e9, "unit": "GB/s",
        "n_gpus": 1, "steps": args.reps, "warmup": 1, "ms_per_step": t_app * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "complex128 (fp64)" if args.precision == "c128" else "complex64 factors (fp32)",
        "data": "synthetic: seeded per-DOF complex Gaussian vector",
        "config": {"workload": "unit cube 64^3 cubes x 6 tets (1,872,064 complex DOFs), k=16, "
                               "xi=k^2, 4x4x4 subdomains, 2-layer overlap, ORAS, resident factors, "
                               "one Schwarz application per step"},
        "roofline": {"bound": "hbm", "kernel": "k_sweep<T, true> (forward block sweep)",
                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                     "traffic": SWEEP_TRAFFIC.get(("apply", args.precision)), "launches": nl,
                     "avg_launch_ms": fms / nl, "bytes_per_launch": sb,
                     "stored_factor_over_envelope": inf["pack_bytes"] / (inf["env_entries"] *
                                                                        (16 if args.precision == "c128" else 8)),
                     "backward": {"avg_launch_ms": bms / nl, "achieved": sb / (bms / nl * 1e-3) / 1e9}},
        "apply_bytes": inf["apply_bytes"], "pack_bytes": inf["pack_bytes"],
        "calibration_copy": {"bytes_read": 1 << 30, "bytes_written": 1 << 30, "seconds": t_copy},
    }


def run_serving(args):
    """Continuous-batching server: seeded Poisson arrivals of unit-cube requests (k ~ U[4,16],
    xi in {k, k^2}, n = ceil(k^1.5)+4 cubes per side, p = clamp(ceil(n/17),2,4) subdomains per
    side, Gaussian sources), mixed-precision ORAS FGMRES(50) rtol 1e-6, admission by exact HBM
    footprint.  Arrivals at a fixed rate (--rate, default 1.5/s; with --rate 0, 0.6 x the
    throughput of a closed-loop calibration run, all calibration requests submitted at once).
    Reports throughput and p50/p99 latency (arrival to result), and any request that failed or
    did not converge."""
    import numpy as np

    from mx_inputs import serving_requests
    from paper_1711_03789_amd import mx
    srv = mx.Server(slots=args.slots, precision="c64", restart=50, flexible=True, rtol=1e-6,
                    batch_applies=not args.no_batch, batch_window_us=args.batch_window)
    calib = None
    rate = args.rate
    if rate <= 0:
        creqs = serving_requests(args.calib_requests, 1.0, args.seed + 1000)
        c0 = time.perf_counter()
        ts = [srv.submit(r["n"], r["p"], r["k"], r["xi"], r["center"], r["pol"], 0.1) for r in creqs]
        for t in ts:
            srv.wait(t, 600.0)
            srv.release(t)
        sat = len(creqs) / (time.perf_counter() - c0)
        rate = 0.6 * sat
        calib = {"requests": len(creqs), "saturated_solves_per_s": sat, "rate": rate}
    reqs = serving_requests(args.requests, rate, args.seed)
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        wait = r["arrival"] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        tickets.append((r, srv.submit(r["n"], r["p"], r["k"], r["xi"], r["center"], r["pol"], 0.1)))
        if len(tickets) % 100 == 0:
            print("submitted %d/%d" % (len(tickets), len(reqs)), file=sys.stderr, flush=True)
    # a seeded sample of the small requests is solved again by the oracle after the run
    small = [i for i, (r, _) in enumerate(tickets) if r["n"] <= 16]
    sample = set(np.random.default_rng(args.seed + 7).permutation(small)[:4].tolist()) if small else set()
    served = {}
    res = []
    for i, (r, t) in enumerate(tickets):
        out = srv.wait(t, 600.0)
        res.append(out)
        if i in sample and out["status"] == 0:
            served[i] = srv.solution(t, out["n_dof"])
        srv.release(t)
        if len(res) % 100 == 0:  # progress for long runs (stderr; stdout carries one JSON line)
            print("served %d/%d" % (len(res), len(tickets)), file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    st = srv.stats()
    srv.close()
    lat = np.array([x["t_total"] for x in res])
    ok = all(x["status"] == 0 and x["converged"] for x in res)
    failed = [{"request": i, "n": r["n"], "p": r["p"], "k": r["k"], "xi": r["xi"],
               "status": x["status"], "converged": x["converged"], "iters": x["iters"],
               "relres": x["relres_true"], "error": x.get("error", "")}
              for i, ((r, _), x) in enumerate(zip(tickets, res))
              if x["status"] != 0 or not x["converged"]]
    line = {
        "metric": "p50/p99 solve latency", "value": float(np.percentile(lat, 50)), "unit": "s",
        "n_gpus": 1, "steps": len(res), "warmup": 0, "ms_per_step": (t1 - t0) / len(res) * 1e3,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "complex64 factors + FP64 FGMRES", "data": "synthetic",
        "config": {"workload": "serving: %d requests, Poisson arrivals at %.2f/s, unit cube, "
                               "k~U[4,16], xi in {k,k^2}, n=ceil(k^1.5)+4, p=clamp(ceil(n/17),2,4), "
                               "ORAS FGMRES(50) rtol 1e-6, %d slots, %s" % (
                                   len(res), rate, args.slots,
                                   "preconditioner applications of co-resident requests batched"
                                   if not args.no_batch else "applications on each request's stream")},
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "throughput_solves_per_s": len(res) / (t1 - t0), "all_converged": ok,
        "mean_iters": float(np.mean([x["iters"] for x in res])),
        "mean_queue_s": float(np.mean([x["t_queue"] for x in res])),
        "calibration": calib,
        "server": st,
        "failed": failed[:20],
    }
    if not args.no_cpu_baseline and served:
        line["cpu_baseline"], line["error_vs_oracle"] = cpu_baseline_serving(
            [(tickets[i][0], served[i]) for i in sorted(served)], layers=2, restart=50)
    return line


def cpu_baseline_serving(sample, layers, restart):
    """The oracle (NumPy/SciPy FP64, one thread) on a seeded sample of the served requests (at most
    four with n <= 16 cubes per side), each solved end to end (mesh, assembly, load, partition,
    ORAS local factorisations, GMRES(restart) to rtol 1e-6); returns the oracle's solves/s and the
    relative L2 error of each served (mixed-precision) solution against the oracle's."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dd, fem, gmres
    from oracle.mesh import Mesh as OMesh
    errs, t = [], 0.0
    with threadpool_limits(1):
        for r, x in sample:
            t0 = time.perf_counter()
            m = OMesh(r["n"], r["n"], r["n"])
            A = fem.assemble(m, r["k"], r["xi"])
            f = fem.load_vector(m, fem.gaussian_source(r["center"], r["pol"], 0.1))
            part = dd.Partition(m, r["p"], r["p"], r["p"], layers)
            B = dd.Schwarz(part, A, dd.ORAS, r["k"], r["xi"])
            xo = gmres.gmres(A, f, B, restart=restart, rtol=1e-6).x
            t += time.perf_counter() - t0
            errs.append(float(np.linalg.norm(x - xo) / np.linalg.norm(xo)))
    desc = ", ".join("n=%d p=%d k=%.2f xi=%.2f" % (r["n"], r["p"], r["k"], r["xi"]) for r, _ in sample)
    return ({"value": len(sample) / t, "unit": "solves/s", "cores": 1, "kind": "oracle",
             "sample": "%d served requests (%s) solved again end to end by the oracle in %.1f s"
                       % (len(sample), desc, t)},
            {"per_solve": errs, "per_solve_max": max(errs), "solves": len(errs),
             "norm": "relative L2 against the FP64 oracle's solution of the same request at rtol "
                     "1e-6", "target": 1e-5})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="scale")
    ap.add_argument("--max-iters", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="c128", choices=["c128", "c64"],
                    help="c64: complex64 factors and SpMV values inside FP64 flexible GMRES")
    ap.add_argument("--reps", type=int, default=10, help="applications timed (batching)")
    ap.add_argument("--requests", type=int, default=120, help="serving: number of requests")
    ap.add_argument("--rate", type=float, default=1.5,
                    help="serving: arrivals per second (0 = 0.6 x a closed-loop calibration's "
                         "throughput)")
    ap.add_argument("--calib-requests", type=int, default=24, help="serving: calibration requests")
    ap.add_argument("--slots", type=int, default=4, help="serving: requests in flight")
    ap.add_argument("--batch-window", type=int, default=0,
                    help="serving: microseconds the batcher waits for co-resident requests' "
                         "applications (0: the library's default)")
    ap.add_argument("--no-batch", action="store_true",
                    help="serving: each request's applications on its own stream (no batching)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--coarse-cubes", type=int, default=0,
                    help="two-level with a coarse box mesh of C^3 cubes, nested or not (R^0 by a "
                         "Gauss rule of --nq points per fine edge)")
    ap.add_argument("--nq", type=int, default=12, help="quadrature points per fine edge")
    ap.add_argument("--x0", default="zero", choices=["zero", "random"],
                    help="initial guess: zero, or a seeded random vector as in the paper's runs "
                         "(GMRES then stops on the residual relative to b - A x0)")
    ap.add_argument("--coarse", type=int, default=0,
                    help="two-level: coarse mesh with this many times fewer cubes per axis (0: one-level)")
    ap.add_argument("--combine", default="hybrid", choices=["additive", "hybrid", "deflation"],
                    help="two-level form (eq:defAS / eq:RAS2, eq:HRAS, eq:ADEF1ras)")
    ap.add_argument("--tune", action="store_true",
                    help="before timing, pick the factorisation launch shape (mx_precond_tune_factor) "
                         "and the sweep grid (mx_precond_autotune) on the first instance")
    ap.add_argument("--graph", action="store_true",
                    help="replay each Arnoldi step from a captured HIP graph (the sweeps are then "
                         "not timed one by one, so no roofline figure)")
    ap.add_argument("--rhs", type=int, default=1,
                    help="right-hand sides solved per preconditioner setup (factors resident)")
    ap.add_argument("--weighted", action="store_true",
                    help="weighted GMRES in the D_k = K + k^2 M inner product (Sec. 5.2, eq:ip)")
    ap.add_argument("--overlap-factor", type=int, default=0, choices=[0, 1],
                    help="1: the next instance's factorisation also runs on the second host "
                         "thread (its own non-blocking stream), overlapping the current GMRES")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world > 1:
        print("bench.py measures one MI355X: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from mx_inputs import random_rhs
    from paper_1711_03789_amd import mx

    if args.workload == "batching":
        print(json.dumps(run_batching(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serving(args)), flush=True)
        return
    if args.workload == "apply":
        print(json.dumps(run_apply(args)), flush=True)
        return
    w, cfg = workload_desc(args.workload)
    inst = instances(args.workload)
    mixed = args.precision == "c64"
    if mixed:
        cfg["workload"] = cfg["workload"].replace(
            "GMRES(", "FGMRES(").replace("complex128", "complex64 factors and SpMV values, FP64 "
                                                      "Krylov vectors")
    if args.weighted:
        cfg["workload"] += "; weighted GMRES in the D_k = K + k^2 M inner product"
    if args.rhs > 1:
        cfg["workload"] += "; %d right-hand sides per preconditioner setup" % args.rhs
    if args.graph:
        cfg["workload"] += "; Arnoldi steps replayed from HIP graphs"
    order = 2 if args.workload == "order2" else 1
    box = None
    if args.coarse_cubes:
        if args.coarse or order == 2 or args.overlap_factor:
            raise SystemExit("--coarse-cubes is not combined with --coarse, --overlap-factor or "
                             "the order-2 workload")
        box = (args.coarse_cubes,) * 3
        cfg["workload"] += ("; two-level (%s) with a coarse mesh of %d^3 cubes, R^0 by a %d-point "
                            "Gauss rule per fine edge" % (args.combine, args.coarse_cubes, args.nq))
    if order == 2 and not args.coarse:
        args.coarse, args.combine = 6, "hybrid"
    elif args.coarse:
        if args.overlap_factor:
            raise SystemExit("--coarse is not combined with --overlap-factor")
        if order == 1:
            cfg["workload"] += ("; two-level (%s) with a nested coarse mesh of %s cubes"
                                % (args.combine, "x".join(str(v // args.coarse) for v in w.n)))
    ctx = mx.Context(0)
    n = w.n
    # inputs resident in HBM before the timed region
    mesh0 = mx.Mesh(*n, *w.lengths)
    E = mesh0.n_edge if order == 1 else mesh0.order2()["n_dof"]  # DOFs of the space
    del mesh0
    rhs = {s: torch.from_numpy(random_rhs(E, s)).cuda() for _, _, s in inst}
    # further right-hand sides of each instance when several are solved per setup
    rhs_more = {s: [torch.from_numpy(random_rhs(E, 1000 + 100 * s + q)).cuda()
                    for q in range(1, args.rhs)] for _, _, s in inst}
    if args.workload == "small":
        m0 = mx.Mesh(*n, *w.lengths)
        rhs[0] = torch.from_numpy(m0.rhs_gaussian(w.center, w.pol, w.sigma)).cuda()
    x = torch.zeros(E, dtype=torch.complex128, device="cuda")
    x0 = torch.from_numpy(random_rhs(E, 777)).cuda() if args.x0 == "random" else None
    if x0 is not None:
        cfg["workload"] += "; seeded random initial guess"
    torch.cuda.synchronize()

    refs = {}
    tuned = {"schedule": "auto", "width": 0, "sweep_grid": 0}
    if args.tune:  # untimed: a property of the mesh, partition and precision, reused by every solve
        kind0, e0, _ = inst[0]
        m0 = mx.Mesh(*n, *w.lengths)
        p0 = mx.Partition(m0, *w.parts, w.layers)
        A0 = mx.Matrix(ctx, m0, w.k, 0.0 if e0 is None else w.k ** e0, order=order)
        sch, wid, best, each = mx.tune_factor(ctx, A0, m0, p0, kind0, precision=args.precision)
        P0 = mx.Precond(ctx, A0, m0, p0, kind0, precision=args.precision, schedule=sch, width=wid)
        grid, ms = P0.autotune()
        del P0, A0, p0, m0
        tuned = {"schedule": sch, "width": wid, "sweep_grid": grid, "factor_ms_each": each,
                 "candidates": "one stream; look-ahead widths 1, 2, 3, 4", "apply_ms": ms}

    # The host half of the next instance's setup (assembly and its upload, local problems, RCM,
    # tile layout) runs on a second host thread while the device factors and solves the current
    # one; every kernel stays on this thread, in order.  At most two instances are alive at once.
    ctx_host = mx.Context(0)
    fstream = torch.cuda.Stream() if args.overlap_factor else None  # default priority


    def prepare(mesh, part, kind, e, idx):
        # the preconditioner's absorption (exponent None: none); also the problem's unless
        # xi_prob = 0
        xi = 0.0 if e is None else w.k ** e
        zero = xi_prob_zero(args.workload, idx)
        t0 = time.perf_counter()
        A = mx.Matrix(None, mesh, w.k, 0.0 if zero else xi, order=order)
        A_prec = mx.Matrix(None, mesh, w.k, xi, order=order) if zero and xi != 0 else A  # host only
        A.upload(ctx_host)  # its own stream: overlaps the device work of the current instance
        t1 = time.perf_counter()
        P = mx.Precond(ctx_host, A_prec, mesh, part, kind, xi_prec=xi, precision=args.precision,
                       plan_only=True, schedule=tuned["schedule"], width=tuned["width"],
                       sweep_grid=tuned["sweep_grid"])
        P.stage(ctx_host)  # host-to-device copies, also overlapping the current instance
        A_c = None
        if args.coarse or box:  # host half of the coarse level (R^0, A^0, plan of its
            # factorisation), built from the matrix the preconditioner is for (at xi_prec)
            A_c = A_prec
            if A_c is not A:
                A_c.upload(ctx_host)
            P.plan_coarse(A_c, mesh, args.coarse, args.combine, box=box, nq=args.nq)
        del A_prec
        if fstream is not None:
            P.materialize(ctx_host, fstream)  # returns once its factor tiles are complete
        t2 = time.perf_counter()
        return A, A_c, P, xi, zero, t1 - t0, t2 - t1

    def step(record):
        from concurrent.futures import ThreadPoolExecutor
        t = time.perf_counter()
        mesh = mx.Mesh(*n, *w.lengths)
        part = mx.Partition(mesh, *w.parts, w.layers)
        D = mx.Matrix.weight(ctx, mesh, w.k) if args.weighted else None
        t_topo = time.perf_counter() - t
        rec = []
        with ThreadPoolExecutor(max_workers=1) as ex:
            fut = ex.submit(prepare, mesh, part, inst[0][0], inst[0][1], 0)
            for idx, (kind, e, seed) in enumerate(inst):
                A, A_c, P, xi, zero, t_asm, t_pre = fut.result()
                if idx + 1 < len(inst):
                    fut = ex.submit(prepare, mesh, part, inst[idx + 1][0], inst[idx + 1][1], idx + 1)
                if fstream is None:
                    P.materialize(ctx)
                t_coarse = 0.0
                if args.coarse or box:
                    tc = time.perf_counter()
                    P.add_coarse(ctx, A_c, mesh, args.coarse, args.combine, box=box, nq=args.nq)
                    t_coarse = time.perf_counter() - tc
                t2 = time.perf_counter()
                timed = record and not args.graph
                if timed:
                    P.sweep_timing(True)
                for q, bq in enumerate([rhs[seed]] + rhs_more[seed]):
                    if x0 is None:
                        x.zero_()
                    else:
                        x.copy_(x0)
                    st = mx.gmres(ctx, A, P, bq, x, restart=w.restart, rtol=w.rtol,
                                  max_iters=args.max_iters, flexible=mixed, spmv_c64=mixed, weight=D,
                                  graph=args.graph)
                    if q == 0:
                        st0 = st
                        if record and mixed and "x_mixed" not in refs:
                            refs["x_mixed"] = (kind, e, seed, x.clone())
                        if record and args.workload == "small":
                            refs.setdefault("x_small", []).append(x.clone())
                    elif not st["converged"]:
                        st0 = st
                st = st0
                t3 = time.perf_counter()
                r = {"kind": kind, "xi": 0.0 if zero else xi, "xi_prec": xi,
                     "iters": st["iters"], "converged": st["converged"],
                     "relres": st["relres_true"], "t_assemble": t_asm, "t_precond_plan": t_pre,
                     "t_gmres": t3 - t2, "t_coarse": t_coarse}
                inf = P.info()
                r.update({"t_precond_host": inf["t_host_setup"], "t_upload": inf["t_upload"],
                          "t_factor": inf["t_factor"], "env_flops": inf["env_flops"],
                          "tile_flops": inf["tile_flops"], "sweep_bytes": inf["sweep_bytes"],
                          "apply_bytes": inf["apply_bytes"], "factor_bytes": inf["factor_bytes"],
                          "pack_bytes": inf["pack_bytes"], "env_bytes": inf["env_entries"] *
                          (16 if args.precision == "c128" else 8)})
                if timed:
                    r["sweep_launches"], r["fwd_ms"], r["bwd_ms"] = P.sweep_timing(False)
                else:
                    r["sweep_launches"], r["fwd_ms"], r["bwd_ms"] = 0, 0.0, 0.0
                rec.append(r)
                del P, A, A_c
        return t_topo, rec

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    recs = []
    for _ in range(args.steps):
        recs.append(step(True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_solves = args.steps * len(inst) * args.rhs
    all_r = [r for _, rr in recs for r in rr]
    converged = all(r["converged"] for r in all_r)
    launches = sum(r["sweep_launches"] for r in all_r)
    fwd_ms = sum(r["fwd_ms"] for r in all_r)
    bwd_ms = sum(r["bwd_ms"] for r in all_r)
    sweep_bytes = sum(r["sweep_launches"] * r["sweep_bytes"] for r in all_r)
    achieved = sweep_bytes / (fwd_ms * 1e-3) / 1e9 if fwd_ms > 0 else 0.0
    achieved_bwd = sweep_bytes / (bwd_ms * 1e-3) / 1e9 if bwd_ms > 0 else 0.0
    t_factor = sum(r["t_factor"] for r in all_r)
    t_gmres = sum(r["t_gmres"] for r in all_r)
    out = {
        "metric": "GMRES solves/sec at rtol 1e-6",
        "value": n_solves / elapsed if converged else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "complex128 (fp64)",
        "data": "synthetic: seeded per-DOF complex Gaussian right-hand sides",
        "config": cfg,
        "roofline": {"bound": "hbm", "kernel": "k_sweep<T, true> (forward block sweep of the "
                                                "Schwarz application; the backward launch is "
                                                "reported beside it)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": SWEEP_TRAFFIC.get((args.workload, args.precision)),
                     "launches": launches, "avg_launch_ms": fwd_ms / max(launches, 1),
                     "bytes_per_launch_avg": sweep_bytes / max(launches, 1),
                     "stored_factor_over_envelope": sum(r["pack_bytes"] for r in all_r) /
                     max(sum(r["env_bytes"] for r in all_r), 1),
                     "backward": {"achieved": achieved_bwd, "frac": achieved_bwd / HBM_PEAK_GBS,
                                  "avg_launch_ms": bwd_ms / max(launches, 1)}},
        "factor": factor_line(sum(r["env_flops"] for r in all_r), sum(r["tile_flops"] for r in all_r),
                              t_factor, args.precision),
        "solve_phase_solves_per_s": n_solves / t_gmres if converged and t_gmres > 0 else 0.0,
        "phase_seconds_per_step": {
            "mesh_partition": sum(t for t, _ in recs) / args.steps,
            "assemble": sum(r["t_assemble"] for r in all_r) / args.steps,
            "precond_host": sum(r["t_precond_host"] for r in all_r) / args.steps,
            "precond_upload": sum(r["t_upload"] for r in all_r) / args.steps,
            "factor": t_factor / args.steps,
            "gmres": t_gmres / args.steps,
            "note": "assemble and precond_host of the next instance run on a second host thread "
                    "while the device factors and solves the current one" +
                    ("; the next instance's factorisation too, on its own stream (factor times "
                     "then include contention with the current GMRES)" if fstream is not None
                     else "")},
        "solves": [{k: r[k] for k in ("kind", "xi", "xi_prec", "iters", "converged", "relres",
                                      "t_gmres", "t_factor", "t_coarse")} for r in recs[0][1]],
        "all_converged": converged,
    }
    if args.tune:
        out["tuned"] = tuned
    if mixed and "x_mixed" in refs:
        # accuracy of the mixed path against the complex128 path on the first instance
        kind, e, seed, xm = refs["x_mixed"]
        mesh = mx.Mesh(*n, *w.lengths)
        part = mx.Partition(mesh, *w.parts, w.layers)
        zero = xi_prob_zero(args.workload, 0)
        xe = 0.0 if e is None else w.k ** e
        A = mx.Matrix(ctx, mesh, w.k, 0.0 if zero else xe, order=order)
        A_prec = mx.Matrix(None, mesh, w.k, xe, order=order) if zero and xe != 0 else A
        P = mx.Precond(ctx, A_prec, mesh, part, kind, xi_prec=xe, precision="c128")
        if x0 is None:
            x.zero_()
        else:
            x.copy_(x0)
        st = mx.gmres(ctx, A, P, rhs[seed], x, restart=w.restart, rtol=w.rtol,
                      max_iters=args.max_iters)
        out["mixed_vs_c128"] = {"instance": [kind, xe], "c128_iters": st["iters"],
                                "rel_l2_diff": float(torch.linalg.norm(xm - x) / torch.linalg.norm(x))}
        out["dtype"] = "complex64 factors + FP64 FGMRES"
        del P, A
    if order == 2:
        out["order"] = 2
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_order2(sum(r["iters"] for r in recs[0][1]), len(inst))
    elif not args.no_cpu_baseline:
        if args.workload == "small":
            out["cpu_baseline"], x_or = cpu_baseline_small(w)
            xo = torch.from_numpy(x_or).cuda()
            errs = [float(torch.linalg.norm(xs - xo) / torch.linalg.norm(xo)) for xs in refs["x_small"]]
            out["error_vs_oracle"] = {"per_solve_max": max(errs), "per_solve_mean": sum(errs) / len(errs),
                                      "solves": len(errs), "norm": "relative L2 against the FP64 "
                                      "oracle's solution of the same problem at rtol 1e-6",
                                      "target": 1e-5 if mixed else 1e-8}
        else:
            out["cpu_baseline"] = cpu_baseline(sum(r["iters"] for r in recs[0][1]), len(inst))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
