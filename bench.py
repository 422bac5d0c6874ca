#!/usr/bin/env python3
"""Throughput benchmark of the rsolve solver on one MI355X.

Default workload (c4): Q3 finite elements on a 512 x 512 mesh (n = 2,362,369,
nnz = 58,789,033), rotating velocity 2 pi (-(y - 1/2), x - 1/2), eps = 1e-4,
dt = 5e-3, backward Euler with Picard linearisation.  `warmup + steps`
consecutive time steps are generated on the GPU (the trajectory is advanced
with an FP64 solve to 1e-10) and kept resident in HBM; then the timed region
runs the recycled mixed-precision solver (float32 Arnoldi cycles inside
float64 iterative refinement, GMRES(50), k = 16, s = 32, ell = 1, right
Jacobi) to 1e-8 relative residual on the `steps` systems, one solve plus one
recycle update per step.  Plain FP64 GMRES(50) with right Jacobi runs on the
same systems as the comparison, and two attribution legs (plain GMRES in the same
mixed precision; the recycled method in FP64) split the speed-up between recycling
and FP32.  The update (Algorithm 1) is timed on its own, per-kernel-class rooflines
come from sampled HIP-event stamps, and the oracle's first time steps give the
CPU baseline and the per-solve difference from the oracle.  Prints one JSON line.

python bench.py [--steps K] [--warmup W] [--workload c4|c3|c2|c1] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # name: (problem, solver config, tol, description)
    "c4": ("C3", dict(restart_m=50, recycle_k=16, snapshots_s=32, svd_interval=1, precond="jacobi",
                      precision="fp32_ir", inner_tol=1e-5), 1e-8,
           "Q3 512x512 Burgers-Picard sequence (n=2362369, nnz=58789033), recycled mixed GMRES(50) "
           "k=16 s=32 ell=1 right Jacobi, FP32 Arnoldi + FP64 refinement, tol 1e-8"),
    "c3": ("C3", dict(restart_m=50, recycle_k=16, snapshots_s=32, svd_interval=1, precond="jacobi",
                      precision="fp64"), 1e-10,
           "Q3 512x512 Burgers-Picard sequence, recycled FP64 GMRES(50) k=16 s=32 ell=1 right Jacobi, tol 1e-10"),
    "c2": ("C2", dict(restart_m=30, recycle_k=10, snapshots_s=20, svd_interval=1, precond="jacobi",
                      precision="fp64"), 1e-10,
           "Q2 256x256 Burgers-Picard sequence (n=263169), recycled FP64 GMRES(30) k=10 s=20 right Jacobi, "
           "tol 1e-10"),
    "c1": ("C1", dict(restart_m=30, recycle_k=5, snapshots_s=10, svd_interval=1, precond="none",
                      precision="fp64"), 1e-8,
           "Q1 32x32 Burgers-Picard sequence (n=1089), recycled FP64 GMRES(30) k=5 s=10, tol 1e-8"),
}


# batched workloads: many independent sequences of one small configuration, one launch per time step
BATCH_WORKLOADS = {
    "c1b": ("C1", 256, dict(restart_m=30, recycle_k=5, snapshots_s=10, svd_interval=1, precond="none",
                            precision="fp64"), 1e-8,
            "256 independent Q1 32x32 Burgers-Picard sequences (n=1089, nnz=8409 each; bump centres from seeds "
            "0..255), recycled FP64 GMRES(30) k=5 s=10 ell=1, tol 1e-8, all sequences' solves of a time step in "
            "one batched launch (one workgroup per sequence), then one batched recycle update"),
}


SERVE_WORKLOADS = {
    "c5": ("independent time-stepping sequences arriving as a Poisson process (200/s); per sequence Q1-Q3 "
           "(uniform), mesh 64^2-384^2 in steps of 32 (n 4,225-1,329,409), eps log-uniform in [1e-4, 1e-1], "
           "10-60 steps, dt 5e-3, beta (1, 0.5), bump centre seeded; GMRES(30) right Jacobi tol 1e-8; recycled "
           "mixed: k=10 s=20 ell=1, FP32 Arnoldi + FP64 refinement (one-block sizes batched in FP64); plain: "
           "FP64 GMRES(30); served by the rsolve server (HBM-pool admission, continuous batching of small "
           "sequences, large sequences overlapped on worker streams)"),
}


# the paper's own experiments (section 6.1, Tables 2-4): vortex field, random low-mode forcing, zero
# initial value, dt = 0.5, tol 1e-8; right Jacobi stands in for the paper's SSOR
PAPER_WORKLOADS = {
    # name: (description, generator problem; a dict is keyed by nu)
    "paper_q1": ("first-order elements on a 64x64 grid (n=4225, nnz=35225)", "PAPER_Q1"),
    "paper_sem23": ("2x2 Legendre spectral elements of order 23 (n=2209, nnz=1117433, 506 per row)", "PAPER_SEM23"),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def generate(prob, nsteps, dev):
    """Systems of `nsteps` consecutive time steps, resident on the device."""
    import torch

    from paper_1807_09467_amd import rsolve
    from paper_1807_09467_amd import workload as WL
    t0 = time.time()
    asm = WL.Assembler(prob)
    gasm = WL.GpuAssembler(asm, dev)
    log(f"pattern n={asm.pat.n} nnz={asm.pat.nnz} ready in {time.time() - t0:.1f}s")
    u0 = torch.from_numpy(WL.initial_condition(prob, 0)).to(dev)
    traj = rsolve.Sequence(asm.pat.n, asm.pat.nnz, device=dev, restart_m=50, recycle_k=16, snapshots_s=32,
                           precond="jacobi")
    systems = []
    u = u0
    for i in range(nsteps):
        vals, b = gasm.system(u)
        systems.append((vals, b))
        x, st, status = traj.solve(gasm.row_ptr, gasm.col_idx, vals, b, x0=u, tol=1e-10, same_pattern=i > 0)
        if status != 0:
            raise RuntimeError(f"trajectory solve failed at step {i}: {status}")
        traj.update()
        u = x.clone()
        log(f"generated step {i + 1}/{nsteps} ({st['iterations']} its)")
    traj.close()
    torch.cuda.synchronize()
    log(f"generation done in {time.time() - t0:.1f}s")
    return asm, gasm, u0, systems


class HostSystems:
    """The pattern of a host-assembled sequence on the device (what run_solver needs of an assembler)."""

    def __init__(self, asm, dev):
        import torch
        self.asm = asm
        self.row_ptr = torch.from_numpy(asm.pat.row_ptr).to(dev)
        self.col_idx = torch.from_numpy(asm.pat.col_idx).to(dev)


def generate_host(prob, nsteps, dev, seed=0):
    """Systems of the paper's experiments, assembled on the host (vortex field, forcing drawn per step);
    the trajectory is advanced by the GPU solver (plain FP64 GMRES(50), right Jacobi, tol 1e-12) and the
    systems are kept resident on the device."""
    import torch

    from paper_1807_09467_amd import rsolve
    from paper_1807_09467_amd import workload as WL
    t0 = time.time()
    asm = WL.Assembler(prob)
    hs = HostSystems(asm, dev)
    pat = asm.pat
    coeffs = WL.forcing_coefficients(seed, nsteps) if prob.forcing else [None] * nsteps
    traj = rsolve.Sequence(pat.n, pat.nnz, device=dev, restart_m=50, method="plain", precond="jacobi")
    u = WL.initial_condition(prob, seed)
    u0 = torch.from_numpy(u).to(dev)
    ud = u0
    systems = []
    for i in range(nsteps):
        vals, b = asm.system(u, coeffs[i])
        vt, bt = torch.from_numpy(vals).to(dev), torch.from_numpy(b).to(dev)
        systems.append((vt, bt))
        x, st, status = traj.solve(hs.row_ptr, hs.col_idx, vt, bt, x0=ud, tol=1e-12, same_pattern=i > 0)
        if status != 0:
            raise RuntimeError(f"trajectory solve failed at step {i}: {status}")
        ud = x.clone()
        u = ud.cpu().numpy()
        if (i + 1) % 100 == 0 or i + 1 == nsteps:
            log(f"generated step {i + 1}/{nsteps} ({st['iterations']} its), {time.time() - t0:.1f}s")
    traj.close()
    torch.cuda.synchronize()
    return asm, hs, u0, systems


def bench_paper_table(args, dev):
    """The paper's timing protocol (Tables 3 and 4) on its own workload: no recycling against a recycle
    space of dimension 20 taken from the SVD of the last L solutions every L steps, L = 20, 40, 60,
    for the augmented orthogonal row (the paper's timed method) and the augmented oblique row; GMRES(30),
    tol 1e-8, every step timed. With --guess-table, Table 2's comparison of extrapolation and projection
    guesses instead. One JSON line."""
    from paper_1807_09467_amd import workload as WL
    desc, pname = PAPER_WORKLOADS[args.workload]
    prob = getattr(WL, pname)
    prob = prob[args.nu] if isinstance(prob, dict) else prob
    nsteps = args.table_steps
    tol = 1e-8
    pdesc = "right multicolour SSOR (omega 1)" if args.precond == "ssor" else "right Jacobi"
    desc = (f"paper experiment (section 6.1): {desc}, nu={prob.eps:g}, dt={prob.dt:g}, projected vortex field, "
            f"random low-mode forcing, zero start, {nsteps} steps, GMRES(30) {pdesc}, tol 1e-8, Arnoldi {args.ortho}")
    asm, hs, u0, systems = generate_host(prob, nsteps, dev)
    base = dict(restart_m=30, precond=args.precond, precision="fp64", ortho=args.ortho)
    if args.guess_table:
        a = argparse.Namespace(**vars(args))
        a.warmup, a.steps = 0, nsteps
        return bench_guess_table(a, hs, u0, systems, tol, base, desc, dev)
    # Table 3's 'aug 80' row needs a ring of 80 solutions, above the library's 64
    runs = [("no aug", dict(method="plain"))]
    for L in (20, 40, 60):
        for meth in ("aug_ortho", "aug_oblique"):
            runs.append((f"{meth} {L}", dict(method=meth, recycle_k=20, snapshots_s=L, svd_interval=L)))
    rows = []
    for label, over in runs:
        c = dict(base)
        c.update(over)
        r = run_solver(hs, u0, systems, 0, nsteps, tol, c, dev, label=label, quiet=True)
        its = np.array(r["its"], dtype=float)
        est = np.array(r["est"], dtype=float)
        rows.append({"method": label, "avg_iterations": float(its.mean()), "dev": float(its.std()),
                     # the count of a solver that stops once its (projected) residual estimate meets tol
                     "avg_iterations_estimate_met": float(est.mean()) if np.all(est >= 0) else None,
                     "avg_cycles": float(np.mean(r["cycles"])), "solver_wall_s": r["elapsed"],
                     "solves_per_s": nsteps / r["elapsed"], "max_rel_residual": float(np.max(r["rel"]))})
        log(f"{label}: {its.mean():.2f} +- {its.std():.2f} its ({est.mean():.2f} to the estimate), "
            f"{r['elapsed']:.2f} s")
        del r
    out = {"metric": "solver wall time over the sequence", "unit": "s", "n_gpus": 1, "steps": nsteps,
           "warmup": 0, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": args.workload, "description": desc}, "rows": rows}
    print(json.dumps(out), flush=True)


class Roctx:
    """roctx range around the timed region (a no-op unless a profiler records marker traces)."""

    def __init__(self, on):
        self.lib = None
        if on:
            import ctypes
            for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so", "libroctx64.so"):
                try:
                    self.lib = ctypes.CDLL(name)
                    break
                except OSError:
                    continue
            if self.lib is None:
                log("roctx library not found: no marker range")

    def push(self, name):
        if self.lib is not None:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib is not None:
            self.lib.roctxRangePop()


def run_solver(gasm, u0, systems, warmup, steps, tol, cfg, dev, profile=False, label="", graphs=False,
               profile_kinds=None, quiet=False, roctx=None, profile_stride=4):
    """One pass over the sequence: warmup untimed solves, then `steps` timed solve+update steps.
    The recycle update (Algorithm 1) is synchronous, so the host clock around it is its duration."""
    import torch

    from paper_1807_09467_amd import rsolve
    from paper_1807_09467_amd import autotune
    pat = gasm.asm.pat
    seq = rsolve.Sequence(pat.n, pat.nnz, device=dev, **cfg)
    # SpMV shape: timed on the first system before anything else (not part of the timed region); an
    # SSOR sequence takes the CSR product of the caller's values and its default shape
    shape = seq.spmv_shape()
    if cfg.get("precond") != "ssor":
        shape, _, _ = autotune.tune_sequence(seq, gasm.row_ptr, gasm.col_idx, systems[0][0], cache_path=None,
                                             reps=10)
        log(f"{label} SpMV shape: {shape['format']}, {shape['lanes_per_row']} lanes/row, {shape['vec']} "
            f"entries/lane, remap {shape['xcd_remap']}: {shape['us']:.1f} us (default {shape['default_us']:.1f} us)")
    seq.graphs(graphs)
    x_prev = u0
    lat, its, cyc, keff, rel, upd, est = [], [], [], [], [], [], []
    xs = []
    t_start = None
    for i, (vals, b) in enumerate(systems[: warmup + steps]):
        if i == warmup:
            torch.cuda.synchronize()
            if profile:
                # every fourth step by default: the events' own queue work stays off most steps, and
                # the sampled steps cover every stage of a cycle
                seq.profile(True, kinds=profile_kinds, stride=profile_stride)
            if roctx is not None:
                roctx.push(f"timed {label}")
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        x, st, status = seq.solve(gasm.row_ptr, gasm.col_idx, vals, b, x0=x_prev, tol=tol, same_pattern=i > 0)
        if status != 0:
            raise RuntimeError(f"{label}: solve {i} returned {status}")
        tu = time.perf_counter()
        seq.update()
        t1 = time.perf_counter()
        if i >= warmup:
            upd.append((t1 - tu) * 1e3)
            lat.append((t1 - t0) * 1e3)
            its.append(st["iterations"])
            cyc.append(st["cycles"])
            est.append(st["its_estimate_met"])
            keff.append(st["k_eff"])
            rel.append(st["rel_res_true"])
        xs.append(x)
        x_prev = x
        if not quiet or (i + 1) % 100 == 0:
            log(f"{label} step {i + 1}/{warmup + steps}: {st['iterations']} its, {st['cycles']} cycles, "
                f"k_eff {st['k_eff']}, {1e3 * (t1 - t0):.2f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    if roctx is not None:
        roctx.pop()
    prof = seq.profile_read() if profile else []
    seq.close()
    return dict(elapsed=elapsed, lat=lat, its=its, cycles=cyc, k_eff=keff, rel=rel, upd=upd, prof=prof, xs=xs, est=est,
                shape=shape)


# rocprofv3 counter summaries of the headline run's kernels: kernel class -> (summary, the sources the
# kernel is built from); a summary's figure counts only while those sources are unchanged
TRAFFIC = {
    "spmv_arnoldi": ("k_spmv_bc_f32-q3_512x512_recycled_mixed-hbm_traffic.md",
                     ["paper_1807_09467_amd/csrc/spmv_banded.hpp", "paper_1807_09467_amd/csrc/spmv_classes.hpp",
                      "paper_1807_09467_amd/csrc/common.hpp"]),
    "dots2": ("k_dots2_f32-q3_512x512_recycled_mixed-hbm_traffic.md",
              ["paper_1807_09467_amd/csrc/k_krylov.hip", "paper_1807_09467_amd/csrc/common.hpp"]),
    "dcgs2_update": ("k_dcgs2_update_f32-q3_512x512_recycled_mixed-hbm_traffic.md",
                     ["paper_1807_09467_amd/csrc/k_krylov.hip", "paper_1807_09467_amd/csrc/common.hpp"]),
}


def measured_traffic(kernel, alg_bytes):
    """HBM bytes per launch of `kernel` from its committed rocprofv3 counter summary, or None when
    there is none or the kernel's sources have changed since the counters were taken.  A summary
    of a kernel whose launches differ in width (the sweeps, whose columns grow with the Arnoldi
    step) gives the measured traffic as a multiple of the algorithmic bytes of the same launches,
    applied here to `alg_bytes`, the algorithmic bytes per launch of this run."""
    import hashlib
    import re
    if kernel not in TRAFFIC:
        return None
    summary, sources = TRAFFIC[kernel]
    try:
        text = open(os.path.join(ROOT, "profiles", summary)).read()
    except OSError:
        return None
    m = re.search(r"^traffic_bytes_per_launch=(\d+)(?: traffic_per_algorithmic=([0-9.]+))? kernel=(\S+) "
                  r"sources_sha256=([0-9a-f]{64})$", text, re.M)
    if not m or m.group(3) != kernel:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != m.group(4):
        return None
    return float(m.group(2)) * alg_bytes if m.group(2) else float(m.group(1))


def generate_batched(prob, nseq, nsteps, dev):
    """`nsteps` systems of `nseq` independent sequences (seeds 0..nseq-1), resident on the device; the
    trajectories advance with batched FP64 solves to 1e-10."""
    import torch

    from paper_1807_09467_amd import rsolve
    from paper_1807_09467_amd import workload as WL
    t0 = time.time()
    asm = WL.Assembler(prob)
    gasm = WL.GpuAssembler(asm, dev)
    pat = asm.pat
    trajs = [rsolve.Sequence(pat.n, pat.nnz, device=dev, restart_m=30, method="plain") for _ in range(nseq)]
    u0s = [torch.from_numpy(WL.initial_condition(prob, q)).to(dev) for q in range(nseq)]
    us = list(u0s)
    systems = [[None] * nsteps for _ in range(nseq)]
    for i in range(nsteps):
        jobs = []
        for q in range(nseq):
            vals, b = gasm.system(us[q])
            systems[q][i] = (vals, b)
            jobs.append(dict(seq=trajs[q], row_ptr=gasm.row_ptr, col_idx=gasm.col_idx, val=vals, b=b, x0=us[q],
                             tol=1e-10, same_pattern=i > 0))
        us = [r[0] for r in rsolve.solve_batch(jobs)]
        log(f"generated step {i + 1}/{nsteps} of {nseq} sequences")
    for t in trajs:
        t.close()
    torch.cuda.synchronize()
    log(f"generation done in {time.time() - t0:.1f}s")
    return asm, gasm, u0s, systems


def run_batched(gasm, u0s, systems, warmup, steps, tol, cfg, dev, mode, label=""):
    """All sequences advance one time step per round: `mode` "batch" = one rsolve_solve_batch plus one
    rsolve_update_recycle_batch per round; "sequential" = rsolve_solve + rsolve_update_recycle per sequence."""
    import torch

    from paper_1807_09467_amd import rsolve
    pat = gasm.asm.pat
    nseq = len(systems)
    seqs = [rsolve.Sequence(pat.n, pat.nnz, device=dev, **cfg) for _ in range(nseq)]
    plan = rsolve.BatchPlan(seqs, [gasm.row_ptr] * nseq, [gasm.col_idx] * nseq, tol=tol) if mode == "batch" else None
    if plan is not None:
        # the inputs of every round are resident before timing: their addresses are taken once
        vptr = [plan.pointers([systems[q][i][0] for q in range(nseq)]) for i in range(warmup + steps)]
        bptr = [plan.pointers([systems[q][i][1] for q in range(nseq)]) for i in range(warmup + steps)]
    x_prev = list(u0s)
    lat, its, rel = [], [], []
    t_start = None
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t_start = time.perf_counter()
        t0 = time.perf_counter()
        if mode == "batch":
            outs = plan.solve(vptr[i], bptr[i], x_prev if i == 0 else "previous", same_pattern=i > 0,
                              nnz=pat.nnz)
            plan.update()
            t1 = time.perf_counter()
            step_lat = [(t1 - t0) * 1e3] * nseq
            v = plan.view
            res = [(outs[q], {"iterations": int(v["iterations"][q]), "rel_res_true": float(v["rel_res_true"][q])},
                    int(v["status"][q])) for q in range(nseq)]
        else:
            res, step_lat = [], []
            for q in range(nseq):
                ta = time.perf_counter()
                res.append(seqs[q].solve(gasm.row_ptr, gasm.col_idx, systems[q][i][0], systems[q][i][1],
                                         x0=x_prev[q], tol=tol, same_pattern=i > 0))
                seqs[q].update()
                step_lat.append((time.perf_counter() - ta) * 1e3)
            t1 = time.perf_counter()
        for q, (x, st, status) in enumerate(res):
            if status != 0:
                raise RuntimeError(f"{label}: sequence {q} step {i} returned {status}")
            if i >= warmup:
                its.append(st["iterations"])
                rel.append(st["rel_res_true"])
        if i >= warmup:
            lat.extend(step_lat)
        x_prev = [r[0] for r in res]
        log(f"{label} round {i + 1}/{warmup + steps}: {nseq} solves in {1e3 * (t1 - t0):.2f} ms, "
            f"mean {np.mean([r[1]['iterations'] for r in res]):.1f} its")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    xs = [x.clone() for x in x_prev]
    del plan
    for sq in seqs:
        sq.close()
    return dict(elapsed=elapsed, lat=lat, its=its, rel=rel, xs=xs, cycles=[0], solves=nseq * steps)


def bench_batched(args):
    import torch

    from paper_1807_09467_amd import workload as WL
    dev = torch.device("cuda:0")
    pname, nseq, cfg, tol, desc = BATCH_WORKLOADS[args.workload]
    if args.batch_size is not None:
        desc = desc.replace(f"{nseq} independent", f"{args.batch_size} independent")
        nseq = args.batch_size
    prob = getattr(WL, pname)
    nsteps = args.warmup + args.steps
    asm, gasm, u0s, systems = generate_batched(prob, nseq, nsteps, dev)
    main = run_batched(gasm, u0s, systems, args.warmup, args.steps, tol, cfg, dev, "batch", "recycled-batched")
    plain_cfg = dict(restart_m=cfg["restart_m"], precond=cfg["precond"], method="plain", precision="fp64")
    plain = run_batched(gasm, u0s, systems, args.warmup, args.steps, tol, plain_cfg, dev, "batch", "plain-batched")
    seqr = run_batched(gasm, u0s, systems, args.warmup, args.steps, tol, cfg, dev, "sequential",
                       "recycled-multikernel")

    def summ(r):
        lat = np.array(r["lat"])
        return {"solves_per_s": r["solves"] / r["elapsed"], "ms_per_round": 1e3 * r["elapsed"] / args.steps,
                "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
                "avg_iterations": float(np.mean(r["its"])), "max_rel_residual": float(np.max(r["rel"]))}

    m, pl, sq = summ(main), summ(plain), summ(seqr)
    diffs = [float(torch.linalg.norm(a - b) / torch.linalg.norm(b)) for a, b in zip(main["xs"], plain["xs"])]
    pl["max_rel_diff_vs_recycled"] = max(diffs)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_small(prob, asm, cfg, tol)
    out = {
        "metric": f"linear solves/sec at {tol:g} rel. residual",
        "value": round(m["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_per_round"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": asm.pat.n, "nnz": asm.pat.nnz, "sequences": nseq,
                   "steps_generated": nsteps, "parallelism": "single GPU"},
        "latency_ms": m["latency_ms"],
        "avg_iterations": m["avg_iterations"],
        "max_rel_residual": m["max_rel_residual"],
        "plain_fp64_batched": pl,
        "recycled_multikernel_sequential": sq,
        "speedup_vs_plain_fp64": m["solves_per_s"] / pl["solves_per_s"],
        "roofline": None,
        "roofline_note": "latency-bound: each sequence's working set (< 1 MB) stays in the caches",
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def bench_serving(args):
    import torch

    from paper_1807_09467_amd import serve
    dev = torch.device("cuda:0")
    specs = serve.serving_specs(args.sequences, rate=200.0, seed=0)
    warm = serve.serving_specs(max(args.warmup, 0), rate=200.0, seed=12345)
    cache = serve.AssemblerCache(dev)
    t_setup = cache.prepare(specs + warm, log)
    log(f"generator set-up (patterns, GPU assemblers) {t_setup:.1f}s for {len(cache.base)} (degree, mesh) pairs")
    pool = int(args.pool_gb * 2 ** 30)
    mixed_cfg = dict(restart_m=30, recycle_k=10, snapshots_s=20, svd_interval=1, precond="jacobi",
                     precision="fp32_ir", inner_tol=1e-5, ortho=args.ortho)
    plain_cfg = dict(restart_m=30, precond="jacobi", method="plain", precision="fp64", ortho=args.ortho)
    runs = {}
    for name, cfg in (("recycled_mixed", mixed_cfg), ("plain_fp64", plain_cfg)):
        if warm:
            serve.run_serving(warm, cfg, 1e-8, dev, pool, large_workers=args.workers, cache=cache)
        _, summ, _ = serve.run_serving(specs, cfg, 1e-8, dev, pool, large_workers=args.workers, cache=cache,
                                       log=log)
        log(f"{name}: {summ['solves']} solves in {summ['elapsed_s']:.2f}s = {summ['solves_per_s']:.1f}/s, "
            f"p50 {summ['latency_ms']['p50']:.2f} ms p99 {summ['latency_ms']['p99']:.2f} ms")
        runs[name] = summ
    m, pl = runs["recycled_mixed"], runs["plain_fp64"]
    out = {
        "metric": "linear solves/sec at 1e-8 rel. residual (recycled mixed vs plain FP64); p50/p99",
        "value": round(m["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": m["solves"],
        "warmup": len(warm),
        "ms_per_step": round(1e3 * m["elapsed_s"] / m["solves"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": SERVE_WORKLOADS["c5"] + ("; Arnoldi CGS2 with delayed reorthogonalisation on the "
                                                         "multi-kernel path" if args.ortho == "dcgs2" else ""),
                   "sequences": len(specs), "solves": m["solves"],
                   "pool_gib": args.pool_gb, "large_workers": args.workers, "parallelism": "single GPU"},
        "latency_ms": m["latency_ms"],
        "recycled_mixed": m,
        "plain_fp64": pl,
        "speedup_vs_plain_fp64": m["solves_per_s"] / pl["solves_per_s"],
        "roofline": None,
        "roofline_note": "mixed sizes and overlapping sequences; per-kernel rooflines are measured on the "
                         "single-sequence workloads",
        "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def cpu_baseline_small(prob, asm_host, cfg, tol):
    """Oracle (recycled FP64 GMRES, the workload's configuration) over the first 10 steps of one sequence."""
    from threadpoolctl import threadpool_info

    from oracle import rgmres as O
    from paper_1807_09467_amd import workload as WL
    ocfg = O.Config(restart_m=cfg["restart_m"], recycle_k=cfg["recycle_k"], snapshots_s=cfg["snapshots_s"],
                    svd_interval=cfg["svd_interval"], method=O.AUG_OBLIQUE, precond=O.PRECOND_NONE)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    nseq, nst = 16, 20
    runs = [WL.march(prob, nst, q, asm=asm_host)[1] for q in range(nseq)]
    t0 = time.perf_counter()
    for q, systems in enumerate(runs):
        st = O.RecycleState(asm_host.pat.n, ocfg)
        x = WL.initial_condition(prob, q)
        for vals, b in systems:
            res = O.solve(asm_host.csr(vals), b, x, tol, ocfg, st.W)
            st.update(res.x)
            x = res.x
    dt = time.perf_counter() - t0
    return {"value": nseq * nst / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{nseq} of the sequences x {nst} steps, each solve followed by its recycle update "
                      f"({nseq * nst} solves in {dt:.2f} s); scipy CSR matvec on 1 thread, OpenBLAS on {threads}"}


def summarize(r, steps):
    lat = np.array(r["lat"])
    out = {
        "solves_per_s": steps / r["elapsed"],
        "ms_per_solve": 1e3 * r["elapsed"] / steps,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "avg_iterations": float(np.mean(r["its"])),
        "avg_cycles": float(np.mean(r["cycles"])),
        "max_rel_residual": float(np.max(r["rel"])),
    }
    if r.get("upd"):
        # Algorithm 1 (ring push, TSQR, SVD, new W) against the whole solve + update step
        out["update_ms"] = float(np.mean(r["upd"]))
        out["update_share"] = float(np.sum(r["upd"]) / np.sum(r["lat"]))
    return out


def bench_guess_table(args, gasm, u0, systems, tol, cfg, desc, dev):
    """Extrapolation against projection initial guesses (section 4, the comparison of Table 2): for
    s = 2, 3, 4, extrapolation of order s from the last s solutions and the projection guess onto
    the span of the last s solutions (recycle space of k = s singular vectors, which spans them),
    each followed by plain GMRES; average and standard deviation of the Arnoldi steps per solve
    over the timed steps, and the solve rate.  One JSON line."""
    rows = []
    for sdim in (2, 3, 4):
        row = {"s": sdim}
        for tag, over in (("ext", dict(method=f"guess_extrap{sdim}", recycle_k=0, snapshots_s=sdim)),
                          ("proj", dict(method="guess_project", recycle_k=sdim, snapshots_s=sdim))):
            c = dict(cfg)
            c.update(over)
            r = run_solver(gasm, u0, systems, args.warmup, args.steps, tol, c, dev, label=f"{tag} s={sdim}",
                           graphs=args.graphs)
            its = np.array(r["its"], dtype=float)
            row[f"{tag}_av"] = float(its.mean())
            row[f"{tag}_dev"] = float(its.std())
            row[f"{tag}_solves_per_s"] = args.steps / r["elapsed"]
            row[f"{tag}_max_rel_residual"] = float(np.max(r["rel"]))
            del r
        rows.append(row)
        log(f"s={sdim}: ext {row['ext_av']:.2f} +- {row['ext_dev']:.2f} its, proj {row['proj_av']:.2f} +- "
            f"{row['proj_dev']:.2f} its")
    out = {"metric": "arnoldi_steps_per_solve", "unit": "steps", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": False, "data": "synthetic",
           "config": {"workload": args.workload, "description": desc + ", initial-guess comparison"},
           "rows": rows}
    print(json.dumps(out), flush=True)


def stream_triad(dev, n=1 << 27, reps=20):
    """The library's streaming reference kernel (a = b + s c, 24 n bytes a launch) timed with HIP
    events: the HBM rate a plain stream reaches on this device, beside the 8 TB/s peak the
    rooflines are quoted against."""
    import torch

    from paper_1807_09467_amd import rsolve
    a = torch.empty(n, dtype=torch.float64, device=dev)
    b = torch.ones(n, dtype=torch.float64, device=dev)
    c = torch.ones(n, dtype=torch.float64, device=dev)
    stm = torch.cuda.current_stream(dev)
    for _ in range(2):
        rsolve.triad(a, b, c, 0.5, stream=stm)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stm)
    for _ in range(reps):
        rsolve.triad(a, b, c, 0.5, stream=stm)
    e1.record(stm)
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / reps
    gbs = 24.0 * n / (us * 1e-6) / 1e9
    del a, b, c
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "bytes_per_launch": 24 * n,
            "us_per_launch": round(us, 2), "kernel": "k_triad (rsolve_triad), float64, 16-byte accesses"}


def cpu_baseline(prob, asm_host, tol, cfg, steps=3):
    """The oracle on the host cores: its own recycled solves of the first `steps` time steps of the
    same sequence (same restart, recycle dimension, snapshots, Jacobi and tolerance; Algorithm 1 update
    after each), each system assembled from the oracle's previous solution (assembly not timed).
    Returns the baseline entry and the steps' systems, starting guesses and oracle solutions."""
    from threadpoolctl import threadpool_info

    from oracle import rgmres as O
    from paper_1807_09467_amd import workload as WL
    ocfg = O.Config(restart_m=cfg["restart_m"], recycle_k=cfg.get("recycle_k", 0),
                    snapshots_s=cfg.get("snapshots_s", 0), svd_interval=cfg.get("svd_interval", 1),
                    method=O.AUG_OBLIQUE if cfg.get("recycle_k", 0) else O.PLAIN,
                    precond=O.PRECOND_JACOBI if cfg.get("precond") == "jacobi" else O.PRECOND_NONE)
    state = O.RecycleState(asm_host.pat.n, ocfg)
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    u = WL.initial_condition(prob, 0)
    dt, its, keff, records = 0.0, [], [], []
    for _ in range(steps):
        vals, b = asm_host.system(u)
        A = asm_host.csr(vals)
        t0 = time.perf_counter()
        res = O.solve(A, b, u, tol, ocfg, state.W, state.ring)
        state.update(res.x)
        dt += time.perf_counter() - t0
        its.append(res.iterations)
        keff.append(res.k_eff)
        records.append((vals, b, u, res.x))
        u = res.x
        log(f"oracle step {len(its)}/{steps}: {res.iterations} its, k_eff {res.k_eff}, {dt:.1f} s so far")
    entry = {"value": steps / dt, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
             "sample": f"the oracle's own recycled FP64 solves of time steps 1-{steps} of the same sequence "
                       f"(GMRES({cfg['restart_m']}), k={cfg.get('recycle_k', 0)}, s={cfg.get('snapshots_s', 0)}, "
                       f"right Jacobi, tol {tol:g}, Algorithm 1 update after each; {its} its, k_eff {keff}, "
                       f"{dt:.1f} s); scipy CSR matvec on 1 thread, OpenBLAS on {threads}"}
    return entry, records


def gpu_vs_oracle(records, asm_host, tol, cfg, shape, dev):
    """The timed configuration (same solver settings and SpMV shape) on the oracle's own systems, each
    started from the oracle's previous solution: per-solve difference from the oracle's solution
    (relative 2-norm and largest entry), both solved to the same tolerance."""
    import torch

    from paper_1807_09467_amd import rsolve
    pat = asm_host.pat
    rp = torch.from_numpy(pat.row_ptr).to(dev)
    ci = torch.from_numpy(pat.col_idx).to(dev)
    seq = rsolve.Sequence(pat.n, pat.nnz, device=dev, **cfg)
    seq.set_spmv_shape(shape["lanes_per_row"], shape["vec"], shape["xcd_remap"], shape["format"])
    rel, ent = [], []
    for i, (vals, b, u, xo) in enumerate(records):
        x, st, status = seq.solve(rp, ci, torch.from_numpy(vals).to(dev), torch.from_numpy(b).to(dev),
                                  x0=torch.from_numpy(u).to(dev), tol=tol, same_pattern=i > 0)
        if status != 0:
            raise RuntimeError(f"solve of the oracle's step {i + 1} returned {status}")
        seq.update()
        xg = x.cpu().numpy()
        rel.append(float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)))
        ent.append(float(np.abs(xg - xo).max() / np.abs(xo).max()))
    seq.close()
    return {"steps": list(range(1, len(records) + 1)), "rel": rel, "max_entry_rel": ent, "tol": tol,
            "note": "the timed configuration on the oracle's systems (time steps assembled from the oracle's "
                    "solutions), started from the oracle's previous solution; both stop at the same relative "
                    "residual, so they may differ by up to cond(A) tol"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4",
                    choices=sorted(WORKLOADS) + sorted(BATCH_WORKLOADS) + sorted(SERVE_WORKLOADS)
                    + sorted(PAPER_WORKLOADS))
    ap.add_argument("--sequences", type=int, default=512, help="serving workload: sequences to replay")
    ap.add_argument("--batch-size", type=int, default=None,
                    help="batched workload: sequences per batched launch (default: the workload's 256)")
    ap.add_argument("--pool-gb", type=float, default=96.0, help="serving workload: the server's HBM pool")
    ap.add_argument("--workers", type=int, default=4, help="serving workload: large-sequence worker streams")
    ap.add_argument("--nu", type=float, default=1e-2, choices=[1e-1, 1e-2, 1e-3],
                    help="paper workloads: the diffusion coefficient of the first-order case")
    ap.add_argument("--table-steps", type=int, default=1000, help="paper workloads: time steps of the sequence")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="override the FP32 cycle reduction factor of the mixed-precision workload")
    ap.add_argument("--method", choices=["aug_oblique", "defl_oblique", "aug_ortho", "defl_ortho", "guess_project",
                                         "guess_extrap2", "guess_extrap3", "guess_extrap4", "aug_ls", "defl_ls"],
                    default=None,
                    help="method of the recycled run (default: the workload's, augmented oblique); the "
                         "extrapolation guesses keep a ring of `order` solutions and no recycle space")
    ap.add_argument("--precond", choices=["jacobi", "ssor"], default="jacobi",
                    help="paper workloads: the preconditioner (multicolour SSOR stands in for the paper's SSOR)")
    ap.add_argument("--guess-table", action="store_true",
                    help="instead of the headline line: extrapolation of order s against the projection guess "
                         "onto the s previous solutions (k = s), s = 2, 3, 4, on the workload's sequence")
    ap.add_argument("--select", choices=["largest", "smallest"], default=None,
                    help="singular modes kept in the recycle space (default: largest, Algorithm 1)")
    ap.add_argument("--ortho", choices=["cgs2", "dcgs2"], default="dcgs2",
                    help="Arnoldi orthogonalisation of the multi-kernel solver (both runs): classical "
                         "Gram-Schmidt twice, or the same with the second pass delayed into the next step")
    ap.add_argument("--graphs", action="store_true",
                    help="replay the Arnoldi steps as captured hipGraphs (needs --no-profile to take effect)")
    ap.add_argument("--profile-kinds", default="all",
                    help="kernel kinds timed with HIP events (every fourth Arnoldi step) in the timed run: comma "
                         "list of spmv_arnoldi, dots, update_dots, update_norm, or 'all'")
    ap.add_argument("--profile-stride", type=int, default=4,
                    help="time every s-th Arnoldi step of a cycle (1 = all, for counter runs)")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the attribution legs (plain GMRES in mixed precision, recycled FP64)")
    ap.add_argument("--roctx", action="store_true",
                    help="mark each timed region with a roctx range (for rocprofv3 --marker-trace)")
    ap.add_argument("--oracle-steps", type=int, default=4,
                    help="time steps the oracle solves for the CPU baseline (about 25 s of host work at the default)")
    ap.add_argument("--no-profile", action="store_true",
                    help="run the timed solves without per-kernel event timing (roofline then null)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy (reference for memory-traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the solver path runs on a single device; see the design notes for how it would shard)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import __graft_entry__  # noqa: F401  (path setup)
    from paper_1807_09467_amd import rsolve
    from paper_1807_09467_amd import workload as WL
    rsolve.load()
    if args.workload in BATCH_WORKLOADS:
        return bench_batched(args)
    if args.workload in SERVE_WORKLOADS:
        return bench_serving(args)
    dev = torch.device("cuda:0")
    if args.workload in PAPER_WORKLOADS:
        return bench_paper_table(args, dev)
    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    pname, cfg, tol, desc = WORKLOADS[args.workload]
    cfg = dict(cfg)
    if args.inner_tol is not None and cfg.get("precision") == "fp32_ir":
        cfg["inner_tol"] = args.inner_tol
        desc = desc + f", inner_tol {args.inner_tol:g}"
    cfg["ortho"] = args.ortho
    desc = desc + (", Arnoldi CGS2 with delayed reorthogonalisation" if args.ortho == "dcgs2" else ", Arnoldi CGS2")
    if args.method:
        cfg["method"] = args.method
        desc = desc + f", method {args.method}"
        if args.method.startswith("guess_extrap"):
            cfg["recycle_k"], cfg["snapshots_s"] = 0, int(args.method[-1])
    if args.select:
        cfg["select"] = args.select
        desc = desc + f", {args.select} singular modes"
    prob = getattr(WL, pname)
    nsteps = args.warmup + args.steps
    asm, gasm, u0, systems = generate(prob, nsteps, dev)

    if args.guess_table:
        return bench_guess_table(args, gasm, u0, systems, tol, cfg, desc, dev)
    kinds = None if args.profile_kinds == "all" else [k for k in args.profile_kinds.split(",") if k]
    roctx = Roctx(args.roctx)
    main_run = run_solver(gasm, u0, systems, args.warmup, args.steps, tol, cfg, dev, profile=not args.no_profile,
                          label="recycled", graphs=args.graphs, profile_kinds=kinds, roctx=roctx,
                          profile_stride=args.profile_stride)
    main_sum = summarize(main_run, args.steps)

    def leg(over, label):
        c = dict(cfg)
        c.update(over)
        r = run_solver(gasm, u0, systems, args.warmup, args.steps, tol, c, dev, label=label, graphs=args.graphs,
                       roctx=roctx)
        sm = summarize(r, args.steps)
        sm["max_rel_diff_vs_recycled"] = max(float(torch.linalg.norm(a - b) / torch.linalg.norm(b))
                                             for a, b in zip(main_run["xs"][args.warmup:], r["xs"][args.warmup:]))
        return sm

    plain_sum = None
    if not args.no_plain:
        # the same systems, solved twice: both answers meet the tolerance, so they agree to kappa * tol
        plain_sum = leg(dict(method="plain", recycle_k=0, snapshots_s=0, precision="fp64"), "plain-fp64")
    legs = {}
    if not args.no_legs and args.workload == "c4":
        # attribution: recycling without FP32 and FP32 without recycling, on the same systems
        legs["plain_mixed"] = leg(dict(method="plain", recycle_k=0, snapshots_s=0), "plain-mixed")
        legs["recycled_fp64"] = leg(dict(precision="fp64"), "recycled-fp64")

    # roofline per kernel class (HIP events around sampled launches inside the library); the dominant
    # class is the one with the most time
    prof = main_run["prof"]
    wsz = 4.0 if cfg.get("precision") == "fp32_ir" else 8.0
    classes = {}
    for e in prof:
        c = classes.setdefault(e["kernel"], {"kernel": e["kernel"], "launches": 0, "ms": 0.0, "bytes": 0.0})
        c["launches"] += e["launches"]
        c["ms"] += e["ms"]
        c["bytes"] += e["bytes"]
    rooflines = []
    for c in classes.values():
        avg_us = 1e3 * c["ms"] / c["launches"]
        alg = c["bytes"] / c["launches"]
        achieved = alg / (avg_us * 1e-6) / 1e9
        r = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": c["kernel"],
             "algorithmic_bytes_per_launch": round(alg), "avg_launch_us": round(avg_us, 2),
             "launches": c["launches"], "ms_sampled": round(c["ms"], 3)}
        if c["kernel"] == "spmv_arnoldi":
            # the storage format's bytes (values, chunk offsets, 16-bit list starts, x read, y written);
            # the CSR figure (w + 4) nnz + 4 (n + 1) + 2 w n of the same product is reported beside it
            nn, nz = float(asm.pat.n), float(asm.pat.nnz)
            csr = (wsz + 4.0) * nz + 4.0 * (nn + 1.0) + 2.0 * wsz * nn
            r["algorithmic_bytes"] = "w nnz + 4 (n + 1) + 2 n + 2 w n (banded copy with shared offset lists)"
            r["csr_equivalent_bytes_per_launch"] = round(csr)
            r["csr_equivalent_gbs"] = round(csr / (avg_us * 1e-6) / 1e9, 1)
        elif c["kernel"] in ("dots2", "dots"):
            r["algorithmic_bytes"] = "(columns swept + 1) w n per launch (basis, recycle columns, vectors)"
        elif c["kernel"] in ("dcgs2_update", "update_dots"):
            r["algorithmic_bytes"] = "(j + k + 4) w n per launch (basis, A W columns, candidate in and out)"
        tr = measured_traffic(c["kernel"], alg) if pname == "C3" and cfg.get("precision") == "fp32_ir" else None
        if tr is not None:
            r["traffic"] = tr
            r["traffic_unit"] = "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)"
            r["traffic_gbs"] = round(tr / (avg_us * 1e-6) / 1e9, 1)
        rooflines.append(r)
    rooflines.sort(key=lambda r: -r["ms_sampled"])
    roofline = rooflines[0] if rooflines else None
    for e in prof:
        e["avg_us"] = 1e3 * e["ms"] / e["launches"]
        e["gb_per_s"] = e["bytes"] / (e["ms"] * 1e-3) / 1e9

    triad = stream_triad(dev)
    log(f"stream triad: {triad['gbs']:.0f} GB/s ({triad['frac_of_peak']:.3f} of {HBM_PEAK_GBS:.0f})")

    cpu = None
    err = None
    if not args.no_cpu_baseline and pname == "C3":
        log("timing the oracle on the host")
        cpu, records = cpu_baseline(prob, asm, tol, cfg, steps=args.oracle_steps)
        err = gpu_vs_oracle(records, asm, tol, cfg, main_run["shape"], dev)
        log(f"GPU vs oracle on the oracle's steps: rel {err['rel']}")
        del records

    vs = None
    out = {
        "metric": "linear solves/sec at 1e-8 rel. residual (recycled mixed vs plain FP64); p50/p99"
        if args.workload == "c4" else f"linear solves/sec at {tol:g} rel. residual",
        "value": round(main_sum["solves_per_s"], 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_sum["ms_per_solve"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": vs,
        "dtype": "f32+f64" if cfg.get("precision") == "fp32_ir" else "f64",
        "data": "synthetic",
        "config": {"workload": desc, "n": asm.pat.n, "nnz": asm.pat.nnz, "steps_generated": nsteps,
                   "parallelism": "single GPU", "graphs": bool(args.graphs and args.no_profile),
                   "spmv_shape": {k: (round(v, 2) if isinstance(v, float) else v)
                                  for k, v in main_run["shape"].items()}},
        "latency_ms": main_sum["latency_ms"],
        "avg_iterations": main_sum["avg_iterations"],
        "avg_cycles": main_sum["avg_cycles"],
        "max_rel_residual": main_sum["max_rel_residual"],
        "update_ms": main_sum.get("update_ms"),
        "update_share": main_sum.get("update_share"),
        "plain_fp64": plain_sum,
        "speedup_vs_plain_fp64": (main_sum["solves_per_s"] / plain_sum["solves_per_s"]) if plain_sum else None,
        "attribution": {name: v for name, v in legs.items()} or None,
        "roofline": roofline,
        "rooflines": rooflines,
        "kernels": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in e.items()} for e in prof],
        "err_vs_oracle": err,
        "stream_triad": triad,
        "cpu_baseline": cpu,
    }
    if legs and plain_sum:
        pm, rf = legs.get("plain_mixed"), legs.get("recycled_fp64")
        out["attribution"]["speedup_recycling_in_mixed"] = main_sum["solves_per_s"] / pm["solves_per_s"]
        out["attribution"]["speedup_fp32_without_recycling"] = pm["solves_per_s"] / plain_sum["solves_per_s"]
        out["attribution"]["speedup_recycling_in_fp64"] = rf["solves_per_s"] / plain_sum["solves_per_s"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
