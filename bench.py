#!/usr/bin/env python
"""Benchmark of the multigrid solve path: DOF/s to 1e-10 relative residual.

One step = the two systems of the 3D single-level workload solved from
x0 = 0 to ||r||_inf <= 1e-10 ||r0||_inf: the fourth-order Helmholtz system
(I - cL) u = f with c = 0.5 nu k, nu = 1e-4, k = h, homogeneous Dirichlet
conditions, and the pure-Neumann Poisson system L q = f, on 256^3 cells of
[0,1]^3.  Right-hand sides are closed-form cell averages of
sin(2 pi x) sin(2 pi y) sin(2 pi z) through (I - cL) and of
cos(2 pi x) cos(2 pi y) cos(2 pi z) through L, plus seeded N(0, 1e-3^2)
noise (the Poisson one made mean-free).  DOF per step = 2 * 256^3.

Prints one JSON line.  --workload c1 runs the 2D 128^2 workload instead;
--workload c4 the batch of 1024 independent 2D boxes; --workload imex one
IMEX time step of the four-way vortex flow on a periodic 1024^2 level;
--workload regrid one regridding of that flow's two-level hierarchy into
three levels, with its data migration.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "imex", "regrid"])
    p.add_argument("--bottom", default="exact", choices=["exact", "ilu_gmres"],
                   help="single-level workloads: coarsest-depth solver (the paper's ILU(0)-GMRES, or the exact "
                        "dense inverse)")
    p.add_argument("--bottom-iters", type=int, default=5, help="GMRES steps per bottom solve (--bottom ilu_gmres)")
    p.add_argument("--ratio", type=int, default=2, choices=[2, 4],
                   help="two-level AMR workload: refinement ratio (4: the same patches at h = 1/1024)")
    p.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    p.add_argument("--smoother", default="rb", choices=["jacobi", "rb"])
    p.add_argument("--n", type=int, default=0, help="cells per direction (default: the workload's)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-timing", action="store_true", help="skip the per-kernel event timing")
    p.add_argument("--no-autotune", action="store_true", help="keep the default tile march length")
    p.add_argument("--march", type=int, default=0,
                   help="single-level workloads: this tile march length instead of the autotuner's choice")
    p.add_argument("--nu", default=None,
                   help="pre,post smoothing steps of the V-cycle (default: 1,3 for the 3D single level, "
                        "whose 1e-10 solve it reaches fastest of V(0..2, 1..4), and for the IMEX step; "
                        "2,2 otherwise)")
    p.add_argument("--no-split", action="store_true",
                   help="3D mixed precision: keep the finest depth in interleaved storage during post-smoothing")
    p.add_argument("--no-tail", action="store_true",
                   help="mixed precision: launch every operation of the coarse depths instead of running the "
                        "coarse tail of the V-cycle in one workgroup")
    p.add_argument("--no-graph", action="store_true",
                   help="launch every kernel of a cycle directly instead of replaying its HIP graph")
    p.add_argument("--plain", action="store_true",
                   help="batched workload: the plain FP64 solver (every box solved on its own, its kernels "
                        "launched directly, no graph) instead of the batched solve")
    p.add_argument("--omega-rb", default="1.0,1.3",
                   help="single-level workloads: red-black relaxation factor of the Helmholtz and the Poisson "
                        "solve (1: plain red-black; 1.3 takes the Neumann Poisson solve from 13 to 8 V(1,3) cycles "
                        "in 3D)")
    p.add_argument("--bottom-cells", type=int, default=512,
                   help="single-level workloads: exact bottom solve once a depth has at most this many cells "
                        "(0: coarsen as far as the layout allows)")
    p.add_argument("--no-fp64", action="store_true",
                   help="single-level workloads: skip timing the plain FP64 solver on the same systems")
    p.add_argument("--no-oracle-residual", action="store_true",
                   help="single-level workloads: skip the oracle's residual of the timed solutions")
    p.add_argument("--cpu-workers", type=int, default=0,
                   help="worker processes of the CPU baseline (default: the host's cores, at most 16)")
    p.add_argument("--copy-probe", action="store_true",
                   help="first run a plain 256 MiB device copy three times (the reference kernel that "
                        "calibrates the HBM byte counters)")
    return p.parse_args()


def copy_probe():
    """Three launches of a plain device-to-device copy of 2^25 doubles
    (256 MiB read + 256 MiB written per launch)."""
    import torch
    src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def measured_traffic(name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary profiles/<name>: FETCH_SIZE and WRITE_SIZE (KiB per dispatch),
    each scaled by the factor that the same counter shows for the plain copy
    kernel.  None when the summary is missing or was taken on a different
    kernels.hip (its sha256 is recorded in the summary)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith(("#", " ")):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    src = os.path.join(ROOT, "paper_2506_02663_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if kv.get("kernels_hip_sha256") != sha:
        return None
    try:
        fetch = float(kv["fetch_kib_per_launch"]) * float(kv["fetch_factor"])
        write = float(kv["write_kib_per_launch"]) * float(kv["write_factor"])
    except (KeyError, ValueError):
        return None
    return (fetch + write) * 1024.0


# ---------------------------------------------------------------------------
# workloads (inputs only; every solve step runs in the HIP library)
def single_level_problems(dim, n, nu):
    from paper_2506_02663_amd import workloads as W
    h = 1.0 / n
    c = 0.5 * nu * h
    shape = (n,) * dim
    helm = (1.0 + dim * 4 * math.pi ** 2 * c) * W.sinprod_avg(shape, h) + W.noise(shape, 0)
    pois = -dim * 4 * math.pi ** 2 * W.cosprod_avg(shape, h) + W.noise(shape, 1)
    pois -= pois.mean()
    return h, c, [("helmholtz", "D", helm), ("poisson", "N", pois)]


def host_info():
    """CPU model and core counts of the host running the benchmark."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_available": avail}


def floor_tol(op, f, tol):
    """Absolute stopping term of a solve: at a relative tolerance of 1e-12 the
    Neumann Poisson system stops at its FP64 rounding floor, 2e-12 ||f||."""
    return 2e-12 * float(abs(f).max()) if op == "poisson" and tol <= 1e-12 else 0.0


def _oracle_sample(dim, n, nu, smoother, nu1, nu2, bottom_cells, omega_rb, tol, keep):
    """One run of the oracle on the sample (both systems); returns the DOF
    solved and, if keep, the solutions as interior arrays."""
    from oracle import mg
    from oracle.level import Level
    h, c, probs = single_level_problems(dim, n, nu)
    dof, sols = 0, {}
    for op, bc, f in probs:
        lev = Level((n,) * dim, h, [((0,) * dim, (n - 1,) * dim)], {(d, s): bc for d in range(dim) for s in (0, 1)})
        fa = lev.zeros()
        fa[lev.inner] = f
        x, st = mg.solve(lev, fa, op, c, tol_rel=tol, tol_abs=floor_tol(op, f, tol), max_cycles=100,
                         smoother=smoother, nu1=nu1, nu2=nu2, bottom_cells=bottom_cells,
                         omega_rb=(omega_rb or {}).get(op, 1.0))
        assert st["converged"]
        dof += lev.ncells
        if keep:
            sols[op] = x[lev.inner].copy()
    return dof, sols


def cpu_baseline(dim, n, nu, smoother, nu1=2, nu2=2, bottom_cells=0, omega_rb=None, tol=1e-10, workers=None):
    """The FP64 oracle on a bounded sample of the same workload (same recipe,
    same smoother, relaxation, V-cycle, bottom size and tolerance, smaller
    grid), timed on the host: one copy of the sample per worker process, all
    running at once (each single-threaded numpy), value = all DOF solved /
    wall time.  Runs before the GPU is touched.  Returns the baseline record
    and the oracle's solutions of the sample (for the error of the GPU
    solutions)."""
    from concurrent.futures import ProcessPoolExecutor
    info = host_info()
    workers = workers or max(1, min(16, info["cores_available"] or 1))
    args = (dim, n, nu, smoother, nu1, nu2, bottom_cells, omega_rb, tol)
    t0 = time.perf_counter()
    if workers == 1:
        res = [_oracle_sample(*args, True)]
    else:
        with ProcessPoolExecutor(max_workers=workers) as ex:
            futs = [ex.submit(_oracle_sample, *args, k == 0) for k in range(workers)]
            res = [f.result() for f in futs]
    dt = time.perf_counter() - t0
    dof = sum(r[0] for r in res)
    base = {"value": dof / dt, "unit": "DOF/s", "cores": workers, "kind": "oracle",
            "sample": f"{dim}D {n}^{dim}: Helmholtz (Dirichlet) + Neumann Poisson solves to {tol:g}, "
                      f"same recipe, smoother ({smoother}, omega_rb {omega_rb}), V({nu1},{nu2}) and bottom size "
                      f"({bottom_cells}) as the timed workload; {workers} copies at once, one per worker process "
                      f"(single-threaded numpy each), {dt:.1f} s wall",
            **info}
    return base, res[0][1]


def oracle_residual(dim, n, op, bc, c, f, x):
    """||f' - A x||_inf / ||f'||_inf with A the oracle's operator (numpy, FP64)
    and f' the RHS after the oracle's solvability shift: how well the GPU
    solution x (interior array) satisfies the discrete system, judged by an
    implementation that shares no code with the GPU path."""
    import numpy as np

    from oracle import mg
    from oracle.level import Level
    lev = Level((n,) * dim, 1.0 / n, [((0,) * dim, (n - 1,) * dim)], {(d, s): bc for d in range(dim) for s in (0, 1)})
    fa = lev.zeros()
    fa[lev.inner] = f
    sing = lev.singular_components(op)
    if sing:
        fa, _ = mg.solvability_shift(lev, fa, None, sing)
    xa = lev.zeros()
    xa[lev.inner] = x
    r = fa - lev.apply(xa, op, c)
    return float(np.abs(r[lev.mask]).max() / np.abs(fa[lev.mask]).max())


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        dim, n, nu = 3, args.n or 256, 1e-4
        sample = (3, 64, 1e-4)
        tol = 1e-10  # the metric's tolerance
    elif args.workload == "c1":
        dim, n, nu = 2, args.n or 128, 1e-3
        sample = (2, 64, 1e-3)
        tol = 1e-12  # the 2D single-level configuration's own tolerance
    elif args.workload == "c2":
        return bench_amr(args)
    elif args.workload == "imex":
        return bench_imex(args)
    elif args.workload == "regrid":
        return bench_regrid(args)
    else:
        return bench_batched(args)

    nu1, nu2 = map(int, (args.nu or ("1,3" if dim == 3 else "2,2")).split(","))
    base, oracle_sols = None, None
    if not args.no_cpu_baseline:
        # before the GPU is touched: worker processes of single-threaded numpy
        w_rb = dict(zip(("helmholtz", "poisson"), map(float, args.omega_rb.split(","))))
        base, oracle_sols = cpu_baseline(*sample, args.smoother, nu1, nu2, args.bottom_cells,
                                         w_rb if args.smoother == "rb" else None, tol, args.cpu_workers)

    import torch
    if args.copy_probe:
        copy_probe()

    from paper_2506_02663_amd import amg as A

    h, c, probs = single_level_problems(dim, n, nu)
    prec = A.MIXED if args.precision == "mixed" else A.FP64
    sm = A.SMOOTH_JACOBI if args.smoother == "jacobi" else A.SMOOTH_RB
    w_rb = dict(zip(("helmholtz", "poisson"), map(float, args.omega_rb.split(","))))
    # the 2D workload's 1e-12 lies at the FP64 rounding floor of its Neumann
    # Poisson system (the residual of the exact solution rounds to 1-1.6e-12
    # ||f|| at its largest cell): that solve stops at the floor, 2e-12 ||f||
    tol_abs = {op: floor_tol(op, f, tol) for op, _, f in probs}
    opts = {op: A.default_opts(precision=prec, smoother=sm, tol_rel=tol, tol_abs=tol_abs[op], max_cycles=100,
                               nu1=nu1, nu2=nu2, use_graph=0 if args.no_graph else 1, omega_rb=w_rb[op])
            for op in ("helmholtz", "poisson")}
    systems = []
    march = None
    rhs = {op: (bc, f) for op, bc, f in probs}
    for op, bc, f in probs:
        H = A.Hierarchy(dim, (n,) * dim, h, 1)
        H.set_level_boxes(0, [((0,) * dim, (n - 1,) * dim)])
        for d in range(dim):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.DIRICHLET if bc == "D" else A.NEUMANN)
        H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
        if args.no_split:  # before the autotuner, which times the sweep the solves will run
            H.set_tuning(A.TUNE_SPLIT_RB, 0)
        if args.no_tail:
            H.set_tuning(A.TUNE_TAIL, 0)
        if args.march:
            march = args.march
            H.set_tuning(A.TUNE_MARCH2 if dim == 2 else A.TUNE_MARCH3, march)
        elif not args.no_autotune:
            # tile march length of the finest sweep, timed once (setup, untimed)
            if march is None:
                march, _ = H.autotune(0, A.F32 if prec == A.MIXED else A.F64, sm)
            H.set_tuning(A.TUNE_MARCH2 if dim == 2 else A.TUNE_MARCH3, march)
        if args.bottom_cells:
            H.set_bottom_cells(args.bottom_cells)
        if args.bottom == "ilu_gmres":
            H.set_bottom_solver(A.BOTTOM_ILU_GMRES, args.bottom_iters)
        H.finalize()
        fd = torch.tensor(H.pack(0, 0, lambda i, b: f), device="cuda")
        x = torch.zeros_like(fd)
        systems.append((op, H, x, fd))
    del probs
    dof_step = len(systems) * n ** dim

    cycles = {}

    def step(op_opts=opts, cyc=cycles):
        for op, H, x, fd in systems:
            x.zero_()
            st = H.solve(0, x, fd, None, op_opts[op])
            if st["status"] != 0 or not st["converged"]:
                raise RuntimeError(f"{op} solve did not converge: {st}")
            cyc[op] = st["cycles"]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = dt * 1e3 / args.steps
    timed_ms = None
    if not args.no_timing:
        # second pass of the same steps with HIP events around every launch of
        # the finest-depth kernels (direct launches on the solve's stream)
        for _, H, _, _ in systems:
            H.timing(True)
            for k in range(A.T_KINDS):
                H.timing_read(k, reset=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        timed_ms = (time.perf_counter() - t1) * 1e3 / args.steps
        for _, H, _, _ in systems:
            H.timing(False)

    out = {
        "metric": "MG solve DOF/s to 1e-10 rel. residual, FP32-refined vs FP64; % HBM peak",
        "value": dof_step * args.steps / dt,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-in-f64" if prec == A.MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": f"{dim}D single level {n}^{dim}, Helmholtz (Dirichlet, nu={nu}) + Neumann Poisson",
                   "cells": n ** dim, "dof_per_step": dof_step, "tol_rel": tol,
                   "cycles": cycles, "smoother": args.smoother, "precision": args.precision,
                   "graph": not args.no_graph, "vcycle": f"V({nu1},{nu2})",
                   "omega_rb": w_rb if args.smoother == "rb" else None, "march": march, "bottom_cells": args.bottom_cells,
                   "bottom": args.bottom if args.bottom == "exact" else f"ilu_gmres({args.bottom_iters})",
                   "depths": systems[0][1].level_info(0).depths,
                   "split_storage": bool(systems[0][1].level_info(0).split_rb) and prec == A.MIXED and
                   args.smoother == "rb",
                   "tail_depth": systems[0][1].level_info(0).tail_depth if prec == A.MIXED else -1},
    }
    if not args.no_timing:
        # dominant kernel: the smoothing half-sweep on the finest depth (in
        # colour-split storage where the solves use it)
        split_on = out["config"]["split_storage"]
        kinds = {}
        for _, H, _, _ in systems:
            for k, name in enumerate(("sweep", "fill", "resid_restrict", "prolong", "residual64", "sweep_split")):
                c_, t_ = H.timing_read(k, reset=False)
                a = kinds.setdefault(name, [0, 0.0])
                a[0] += c_
                a[1] += t_
        cnt, tot = kinds["sweep_split" if split_on else "sweep"]
        avg_s = tot / cnt / 1e3
        word = 4 if prec == A.MIXED else 8
        if args.smoother == "jacobi":
            bytes_launch = 3 * word * n ** dim          # read u, read f, write u_new
        else:
            # one half-sweep: read u, read f on one colour, write that colour
            bytes_launch = 2 * word * n ** dim
        traffic = None
        if dim == 3 and n == 256 and word == 4:
            traffic = measured_traffic(f"{args.smoother}_sweep{'_split' if split_on else ''}_fp32_256cubed_counters.txt")
        # `achieved` is taken from the launches inside the timed solves (the
        # event pass); for reference, the same kernel launched 50 times back
        # to back by the library (amg_time_sweep, HIP events on its stream
        # around the batch), where its arrays stay in the caches between
        # launches
        _, H0, x0, f0 = systems[0]
        dt_ = torch.float32 if word == 4 else torch.float64
        u_ = (f0 * 1e-3).to(dt_)
        f_ = f0.to(dt_)
        t_ = torch.zeros_like(u_)
        H0.time_sweep(0, u_, f_, t_, smoother=sm, n=4)  # warm
        bcnt = 50
        bavg_s = H0.time_sweep(0, u_, f_, t_, smoother=sm, n=bcnt) / 1e3
        del u_, f_, t_
        ach = bytes_launch / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": f"{args.smoother} {'half-' if args.smoother == 'rb' else ''}sweep, finest depth, "
                                     f"{'FP32' if word == 4 else 'FP64'}"
                                     f"{', colour-split storage' if split_on else ''}",
                           "avg_us": avg_s * 1e6, "launches": cnt, "bytes_per_launch": bytes_launch,
                           "avg_us_back_to_back": bavg_s * 1e6, "launches_back_to_back": bcnt}
        out["kernel_ms_per_step"] = {k: v[1] / args.steps for k, v in kinds.items()}
        out["ms_per_step_event_pass"] = timed_ms
    # accuracy of the timed solutions: the oracle's operator applied to them
    # (an implementation sharing no code with the GPU path)
    if not args.no_oracle_residual:
        res = {}
        for op, H, x, fd in systems:
            bc, f = rhs[op]
            xs = H.unpack(0, 0, x.cpu().numpy())[0]
            res[op] = oracle_residual(dim, n, op, bc, c, f, xs)
        out["oracle_residual_of_timed_solution"] = res
    # accuracy against the oracle's solution: the sample the CPU baseline
    # solved, solved again on the GPU with the timed configuration
    if oracle_sols is not None:
        out["err_vs_oracle"] = sample_error(A, sample, sm, nu1, nu2, args.bottom_cells, w_rb, prec, tol, oracle_sols)
    # the plain FP64 solver on the same systems: the same V-cycle, smoother,
    # factors and tolerance in FP64, every kernel launched directly (no
    # graph); and the same with graph replay
    if prec == A.MIXED and not args.no_fp64:
        fp = {}
        for graph in (0, 1):
            o64 = {op: A.default_opts(precision=A.FP64, smoother=sm, tol_rel=tol, tol_abs=tol_abs[op], max_cycles=100,
                                      nu1=nu1, nu2=nu2, use_graph=graph, omega_rb=w_rb[op])
                   for op in ("helmholtz", "poisson")}
            cyc64 = {}
            for _ in range(args.warmup):
                step(o64, cyc64)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            for _ in range(args.steps):
                step(o64, cyc64)
            torch.cuda.synchronize()
            fp["ms_per_step_graph" if graph else "ms_per_step_plain"] = (time.perf_counter() - t2) * 1e3 / args.steps
            fp["cycles"] = cyc64
        fp["value_plain"] = dof_step / fp["ms_per_step_plain"] * 1e3
        fp["mixed_speedup_vs_plain"] = fp["ms_per_step_plain"] / ms
        fp["mixed_speedup_vs_fp64_graph"] = fp["ms_per_step_graph"] / ms
        out["fp64"] = fp
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def sample_error(A, sample, sm, nu1, nu2, bottom_cells, w_rb, prec, tol, oracle_sols):
    """Max relative difference between the GPU solutions of the CPU
    baseline's sample (same configuration as the timed solves) and the
    oracle's (both mean-free on the pure-Neumann system)."""
    import numpy as np
    import torch
    dim, n, nu = sample
    h, c, probs = single_level_problems(dim, n, nu)
    err = {}
    for op, bc, f in probs:
        H = A.Hierarchy(dim, (n,) * dim, h, 1)
        H.set_level_boxes(0, [((0,) * dim, (n - 1,) * dim)])
        for d in range(dim):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.DIRICHLET if bc == "D" else A.NEUMANN)
        H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
        if bottom_cells:
            H.set_bottom_cells(bottom_cells)
        H.finalize()
        fd = torch.tensor(H.pack(0, 0, lambda i, b: f), device="cuda")
        x = torch.zeros_like(fd)
        st = H.solve(0, x, fd, None, A.default_opts(precision=prec, smoother=sm, tol_rel=tol,
                                                    tol_abs=floor_tol(op, f, tol), max_cycles=100,
                                                    nu1=nu1, nu2=nu2, omega_rb=w_rb[op]))
        if st["status"] != 0:
            raise RuntimeError(f"sample {op} solve failed: {st}")
        got = H.unpack(0, 0, x.cpu().numpy())[0]
        want = oracle_sols[op]
        if op == "poisson":
            got, want = got - got.mean(), want - want.mean()
        err[op] = float(np.abs(got - want).max() / np.abs(want).max())
    err["sample"] = f"{dim}D {n}^{dim}, the CPU baseline's sample"
    return err


def bench_amr(args):
    """Two-level AMR workload: level 0 = 256^2 cells on [0,1]^2, level 1 = the
    56 boxes of 32^2 cells (h = 1/512) tiling two disks.  One step = the
    composite Helmholtz solve (Dirichlet, c = 0.5 nu k, nu = 1e-3, k = 1/256)
    and the composite pure-Neumann Poisson solve, each from 0 to 1e-10;
    DOF = valid cells of the composite (108,544) per solve."""
    from paper_2506_02663_amd import workloads as W
    ratio = args.ratio
    boxes = W.amr_two_level_boxes(ratio)
    c = 0.5e-3 / 256
    base = None
    if not args.no_cpu_baseline:
        from oracle import amr
        t0 = time.perf_counter()
        OH = amr.Hierarchy((256, 256), 1.0 / 256, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=ratio)
        F = []
        for l, lev in enumerate(OH.levels):
            f = lev.zeros()
            f[lev.inner] = W.single_level_rhs(lev.shape, lev.h, "helmholtz", c, seed=l)
            F.append(f)
        _, st = amr.composite_solve(OH, F, "helmholtz", c, None, tol_rel=1e-10, smoother=args.smoother)
        dt = time.perf_counter() - t0
        nvalid = sum(int(v.sum()) for v in OH.valid)
        base = {"value": nvalid / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle",
                "sample": f"the composite Helmholtz solve of the workload (one of its two solves), {dt:.1f} s"}
    import torch

    from paper_2506_02663_amd import amg as A
    prec = A.MIXED if args.precision == "mixed" else A.FP64
    sm = A.SMOOTH_JACOBI if args.smoother == "jacobi" else A.SMOOTH_RB
    w_rb = dict(zip(("helmholtz", "poisson"), map(float, args.omega_rb.split(","))))
    opts = {op: A.default_opts(precision=prec, smoother=sm, tol_rel=1e-10, max_cycles=100,
                               use_graph=0 if args.no_graph else 1, omega_rb=w_rb[op])
            for op in ("helmholtz", "poisson")}
    systems = []
    for op, bc in (("helmholtz", "D"), ("poisson", "N")):
        H = A.Hierarchy(2, (256, 256), 1.0 / 256, 2, ratio=ratio)
        for l, bl in enumerate(boxes):
            H.set_level_boxes(l, bl)
        H.set_cf_mode(1, A.CF_INTERP)
        for d in range(2):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.DIRICHLET if bc == "D" else A.NEUMANN)
        H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c if op == "helmholtz" else 0.0)
        if args.no_tail:
            H.set_tuning(A.TUNE_TAIL, 0)
        H.finalize()
        fs = []
        for l in range(2):
            n = 256 * ratio ** l
            f = W.single_level_rhs((n, n), 1.0 / n, op, c if op == "helmholtz" else 0.0, seed=l)
            fs.append(torch.tensor(H.pack(l, 0, lambda i, b, f=f: f[b["lo"][0]:b["hi"][0] + 1,
                                                                    b["lo"][1]:b["hi"][1] + 1]), device="cuda"))
        xs = [torch.zeros_like(f) for f in fs]
        systems.append((op, H, xs, fs))
    nfine = sum((hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) for lo, hi in boxes[1])
    nvalid = 256 * 256 - nfine // ratio ** 2 + nfine
    cycles = {}

    def step():
        for op, H, xs, fs in systems:
            for x in xs:
                x.zero_()
            st = H.solve_composite(xs, fs, None, opts[op])
            if st["status"] != 0 or not st["converged"]:
                raise RuntimeError(f"{op} composite solve did not converge: {st}")
            cycles[op] = st["cycles"]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {
        "metric": "MG solve DOF/s to 1e-10 rel. residual, FP32-refined vs FP64; % HBM peak",
        "value": 2 * nvalid * args.steps / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-in-f64" if prec == A.MIXED else "f64", "data": "synthetic",
        "config": {"workload": f"2D two-level AMR 256^2 + {len(boxes[1])} boxes of {16 * ratio}^2 (ratio {ratio}), "
                               "composite Helmholtz + composite Neumann Poisson", "dof_per_step": 2 * nvalid,
                   "tol_rel": 1e-10,
                   "cycles": cycles, "smoother": args.smoother, "precision": args.precision,
                   "omega_rb": w_rb if args.smoother == "rb" else None},
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def bench_imex(args):
    """The IMEX time step of eq. GePUP-IMEX on one periodic level: the
    four-way vortex merging of Section 7.3 (periodic unit square, Re = 1000,
    i.e. nu = 1e-3, Courant number 0.5) on n^2 cells, n = 1024 by default.
    One step = 6 pressure solves, 10 Helmholtz solves and 6 projections
    (tol_rel 1e-10, mixed precision unless --precision fp64); value = cell
    updates per second (n^2 / step time)."""
    import numpy as np
    import torch

    from paper_2506_02663_amd import amg as A
    from paper_2506_02663_amd import workloads as W
    n = args.n or 1024
    nu, cr = 1e-3, 0.5
    u, v = W.four_vortex_velocity(n)
    h = 1.0 / n
    dt = cr * h / max(np.abs(u).max(), np.abs(v).max())
    base = None
    if not args.no_cpu_baseline:
        from oracle import imex
        from oracle.level import Level
        m = 64
        lev = Level((m, m), 1.0 / m, [((0, 0), (m - 1, m - 1))], {(d, s): "P" for d in range(2) for s in (0, 1)})
        us_, vs_ = W.four_vortex_velocity(m)
        U = [lev.zeros(), lev.zeros()]
        U[0][lev.inner], U[1][lev.inner] = us_, vs_
        t0 = time.perf_counter()
        imex.imex_step(lev, U, cr / m / max(np.abs(us_).max(), np.abs(vs_).max()), nu, tol_rel=1e-10)
        el = time.perf_counter() - t0
        base = {"value": m * m / el, "unit": "cell updates/s", "cores": 1, "kind": "oracle",
                "sample": f"one IMEX step of the same flow on 64^2 cells, {el:.1f} s"}
    prec = A.MIXED if args.precision == "mixed" else A.FP64
    sm = A.SMOOTH_JACOBI if args.smoother == "jacobi" else A.SMOOTH_RB
    # the velocity's Helmholtz systems with plain red-black, the pressure and
    # projection systems over-relaxed
    w_rb = dict(zip(("helmholtz", "poisson"), map(float, args.omega_rb.split(","))))
    nu1, nu2 = map(int, (args.nu or "1,3").split(","))
    opts = A.default_opts(precision=prec, smoother=sm, tol_rel=1e-10, max_cycles=100, nu1=nu1, nu2=nu2,
                          use_graph=0 if args.no_graph else 1, omega_rb=w_rb["helmholtz"])
    opts_p = A.default_opts(precision=prec, smoother=sm, tol_rel=1e-10, max_cycles=100, nu1=nu1, nu2=nu2,
                            use_graph=0 if args.no_graph else 1, omega_rb=w_rb["poisson"])
    hs = []
    for op in (A.HELMHOLTZ, A.POISSON):
        H = A.Hierarchy(2, (n, n), h, 1)
        H.set_level_boxes(0, [((0, 0), (n - 1, n - 1))])
        for d in range(2):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.PERIODIC)
        H.set_operator(op, dt * nu / 4 if op == A.HELMHOLTZ else 0.0)
        if args.bottom_cells:
            H.set_bottom_cells(args.bottom_cells)
        if args.no_tail:
            H.set_tuning(A.TUNE_TAIL, 0)
        H.finalize()
        hs.append(H)
    Hv, Hp = hs
    u0 = [torch.tensor(Hv.pack(0, 0, lambda i, b, a=a: a), device="cuda") for a in (u, v)]
    us = [t.clone() for t in u0]
    stats = {}

    def step():
        for t, t0_ in zip(us, u0):
            t.copy_(t0_)
        st = A.imex_step(Hv, Hp, dt, nu, us, None, opts, opts_p)
        if st["status"] != 0 or not st["converged"]:
            raise RuntimeError(f"IMEX step failed: {st}")
        stats.update(st)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {
        "metric": "IMEX step cell updates/s (eq. GePUP-IMEX, ARK4(3)6L[2]SA, solves to 1e-10)",
        "value": n * n * args.steps / el, "unit": "cell updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32-in-f64" if prec == A.MIXED else "f64", "data": "synthetic",
        "config": {"workload": f"four-way vortex merging, periodic {n}^2, Re 1000, Cr 0.5, one IMEX step",
                   "dt": dt, "solves": stats.get("solves"), "cycles": stats.get("cycles"),
                   "max_cycles": stats.get("max_cycles"), "precision": args.precision, "smoother": args.smoother,
                   "vcycle": f"V({nu1},{nu2})", "omega_rb": w_rb},
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def _regrid_hier(A, n, h, boxes):
    H = A.Hierarchy(2, (n, n), h, len(boxes))
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.PERIODIC)
    H.set_operator(A.POISSON, 0.0)
    H.finalize()
    return H


def bench_regrid(args):
    """Regridding and data migration (Section 5.4, RDM-1..4) of the four-way
    vortex flow (Section 7.3) on the periodic unit square: level 0 = n^2
    cells (n = 512 by default), level 1 from a first regrid of the initial
    velocity (vorticity threshold 20, ratio 2).  One step regrids that
    two-level hierarchy into three levels: vorticity tags of levels 0 and 1
    on the GPU, their copy to the host, the clustering and RDM-3 boxes, the
    new hierarchy's planning and finalize, and the migration of both
    velocity components.  value = cells of the new hierarchy per second."""
    import numpy as np
    import torch

    from paper_2506_02663_amd import amg as A
    from paper_2506_02663_amd import workloads as W
    n, eps, r = args.n or 512, 20.0, 2
    h = 1.0 / n
    base = None
    if not args.no_cpu_baseline:
        from oracle import amr, regrid
        from oracle.level import PAD
        m = 128
        bc = {(d, s): "P" for d in range(2) for s in (0, 1)}
        O0 = amr.Hierarchy((m, m), 1.0 / m, [[((0, 0), (m - 1, m - 1))]], bc)
        us_, vs_ = W.four_vortex_velocity(m)
        U = [[O0.levels[0].zeros()], [O0.levels[0].zeros()]]
        U[0][0][PAD:-PAD, PAD:-PAD], U[1][0][PAD:-PAD, PAD:-PAD] = us_, vs_
        nb = regrid.new_boxes([(m, m)], regrid.tag_vorticity(O0, U, eps), r)
        O1 = amr.Hierarchy((m, m), 1.0 / m, [[((0, 0), (m - 1, m - 1))], nb[0]], bc)
        U1 = [regrid.migrate(O0, O1, U[d]) for d in range(2)]
        t0 = time.perf_counter()
        tags = regrid.tag_vorticity(O1, U1, eps)
        nb = regrid.new_boxes([lev.shape for lev in O1.levels], tags, r)
        O2 = amr.Hierarchy((m, m), 1.0 / m, [[((0, 0), (m - 1, m - 1))]] + [b for b in nb if b], bc)
        U2 = [regrid.migrate(O1, O2, U1[d]) for d in range(2)]
        el = time.perf_counter() - t0
        cells = sum(lev.ncells for lev in O2.levels)
        base = {"value": cells / el, "unit": "new-hierarchy cells/s", "cores": 1, "kind": "oracle",
                "sample": f"the same regrid of the flow at level-0 size 128^2 ({cells} new cells), {el:.2f} s"}
        del U2
    u, v = W.four_vortex_velocity(n)
    full = [((0, 0), (n - 1, n - 1))]
    H0 = _regrid_hier(A, n, h, [full])
    u0 = [torch.tensor(H0.pack(0, 0, lambda i, b, a=a: a), device="cuda") for a in (u, v)]

    def tags_of(H, us):
        nl = len(us)
        t = [torch.zeros((n * r ** l) ** 2, dtype=torch.uint8, device="cuda") for l in range(nl)]
        A.tag_vorticity(H, [list(x) for x in us], eps, t)
        return [x.cpu().numpy().reshape((n * r ** l,) * 2).T.astype(bool) for l, x in enumerate(t)]

    def regrid_once(H, us):
        """-> (new hierarchy, its boxes per level, migrated velocity [l][d],
        phase times)"""
        t0 = time.perf_counter()
        tags = tags_of(H, us)
        t1 = time.perf_counter()
        boxes = [full] + [b for b in A.regrid_boxes((n, n), r, tags) if b]
        t2 = time.perf_counter()
        Hn = _regrid_hier(A, n, h, boxes)
        t3 = time.perf_counter()
        new = [[torch.zeros(Hn.depth_size(l, 0)[0], dtype=torch.float64, device="cuda") for _ in range(2)]
               for l in range(len(boxes))]
        for d in range(2):
            A.migrate(H, Hn, [us[l][d] for l in range(len(us))], [new[l][d] for l in range(len(boxes))])
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ph = dict(tags_ms=(t1 - t0) * 1e3, boxes_ms=(t2 - t1) * 1e3, finalize_ms=(t3 - t2) * 1e3,
                  migrate_ms=(t4 - t3) * 1e3)
        return Hn, boxes, new, ph

    H1, boxes1, us1, _ = regrid_once(H0, [u0])
    phases, Hs = [], []
    for i in range(args.warmup + args.steps):
        if i == args.warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        Hn, boxes, new, ph = regrid_once(H1, us1)
        if i >= args.warmup:
            phases.append(ph)
        Hs.append(Hn)
        if len(Hs) > 1:
            Hs.pop(0).close()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    cells = sum(int(np.prod([hi[d] - lo[d] + 1 for d in range(2)])) for bl in boxes for lo, hi in bl)
    avg = {k: round(sum(p[k] for p in phases) / len(phases), 3) for k in phases[0]}
    out = {
        "metric": "regrid throughput: cells of the new hierarchy per second (Section 5.4, RDM-1..4 + migration)",
        "value": cells * args.steps / el, "unit": "new-hierarchy cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"four-way vortex flow, periodic {n}^2 base, ratio {r}, vorticity >= {eps}: "
                               f"{len(boxes1)} levels -> {len(boxes)} levels",
                   "new_cells": cells, "boxes_per_level": [len(bl) for bl in boxes], "phases_ms": avg},
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def bench_batched_plain(args, sides, fs, h, c, base):
    """The plain FP64 solver on the batched workload: each box solved on its
    own (one hierarchy per box size, reused for the boxes of that size), FP64
    throughout, every kernel launched directly (no graph), the same smoother
    and V(2,2) to 1e-10.  One step = all 1024 solves."""
    import torch

    from paper_2506_02663_amd import amg as A
    sm = A.SMOOTH_JACOBI if args.smoother == "jacobi" else A.SMOOTH_RB
    opts = A.default_opts(precision=A.FP64, smoother=sm, tol_rel=1e-10, max_cycles=100, use_graph=0)
    hier = {}
    for s in sorted(set(sides)):
        H = A.Hierarchy(2, (s, s), h, 1)
        H.set_level_boxes(0, [((0, 0), (s - 1, s - 1))])
        for d in range(2):
            for sd in (0, 1):
                H.set_physical_bc(d, sd, A.DIRICHLET)
        H.set_operator(A.HELMHOLTZ, c)
        H.finalize()
        hier[s] = H
    fds = [torch.tensor(hier[s].pack(0, 0, lambda i, b, f=fs[k]: f), device="cuda") for k, s in enumerate(sides)]
    xs = [torch.zeros_like(f) for f in fds]
    ncell = int(sum(s * s for s in sides))
    info = {"cycles": 0}

    def step():
        cyc = 0
        for k, s in enumerate(sides):
            xs[k].zero_()
            st = hier[s].solve(0, xs[k], fds[k], None, opts)
            if st["status"] != 0 or not st["converged"]:
                raise RuntimeError(f"box {k} did not converge: {st}")
            cyc = max(cyc, st["cycles"])
        info["cycles"] = cyc

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {
        "metric": "MG solve DOF/s to 1e-10 rel. residual, FP32-refined vs FP64; % HBM peak",
        "value": ncell * args.steps / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "batch of 1024 independent 2D boxes, sides 8m, m~U{2..32}, Dirichlet Helmholtz",
                   "cells": ncell, "tol_rel": 1e-10, "cycles_max": info["cycles"], "smoother": args.smoother,
                   "precision": "fp64", "solver": "plain: one box per solve, direct launches, no graph",
                   "vcycle": "V(2,2)"},
    }
    if base:
        out["cpu_baseline"] = base
    print(json.dumps(out))


def bench_batched(args):
    """1024 independent 2D boxes, sides 8m with m ~ U{2..32} (seed 0), h = 1/256,
    Dirichlet Helmholtz (I - cL) with c = 0.5 nu k, nu = 1e-3, k = h; each
    right-hand side a seeded sum of 8 sine modes.  One step = one batched
    solve of all boxes to 1e-10; DOF = all cells."""
    import numpy as np

    from paper_2506_02663_amd import workloads as W
    h = 1.0 / 256
    c = 0.5 * 1e-3 * h
    sides = W.batched_boxes(1024, seed=0)
    fs = [W.batched_rhs(s, h, seed=i) for i, s in enumerate(sides)]
    base = None
    if not args.no_cpu_baseline:
        from oracle import mg
        from oracle.level import Level
        t0 = time.perf_counter()
        dof = 0
        for i in range(0, 1024, 128):  # every 128th box: 8 boxes of the batch
            s = sides[i]
            lev = Level((s, s), h, [((0, 0), (s - 1, s - 1))], {(d, sd): "D" for d in range(2) for sd in (0, 1)})
            f = lev.zeros()
            f[lev.inner] = fs[i]
            x, st = mg.solve(lev, f, "helmholtz", c, tol_rel=1e-10, smoother=args.smoother)
            assert st["converged"]
            dof += s * s
        dt = time.perf_counter() - t0
        base = {"value": dof / dt, "unit": "DOF/s", "cores": 1, "kind": "oracle",
                "sample": f"8 boxes of the batch (every 128th, sides {[sides[i] for i in range(0, 1024, 128)]}), "
                          f"each solved to 1e-10 by the oracle, {dt:.1f} s"}
    import torch

    from paper_2506_02663_amd import amg as A
    if args.plain:
        return bench_batched_plain(args, sides, fs, h, c, base)
    prec = A.MIXED if args.precision == "mixed" else A.FP64
    sm = A.SMOOTH_JACOBI if args.smoother == "jacobi" else A.SMOOTH_RB
    opts = A.default_opts(precision=prec, smoother=sm, tol_rel=1e-10, max_cycles=100,
                          use_graph=0 if args.no_graph else 1)
    H = A.Hierarchy(2, (256, 256), h, 1)
    boxes, x0 = [], 0
    for s in sides:
        boxes.append(((x0, 0), (x0 + s - 1, s - 1)))
        x0 += s
    H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(2):
        for sd in (0, 1):
            H.set_physical_bc(d, sd, A.DIRICHLET)
    H.set_operator(A.HELMHOLTZ, c)
    if args.no_split:
        H.set_tuning(A.TUNE_SPLIT_RB, 0)
    if args.no_tail:
        H.set_tuning(A.TUNE_TAIL, 0)
    t0 = time.perf_counter()
    if args.march:
        march = args.march
    elif not args.no_autotune:
        # tile march length of the finest sweep, timed on copies of the layout
        march, _ = H.autotune(0, A.F32 if prec == A.MIXED else A.F64, sm)
    else:
        march = None
    if march:
        H.set_tuning(A.TUNE_MARCH2, march)
    H.finalize()
    setup_s = time.perf_counter() - t0
    split_on = bool(H.level_info(0).split_rb) and args.precision == "mixed" and args.smoother == "rb"
    fd = torch.tensor(H.pack(0, 0, lambda i, b: fs[i]), device="cuda")
    x = torch.zeros_like(fd)
    ncell = int(sum(s * s for s in sides))
    info = {}

    def step():
        x.zero_()
        st = H.solve(0, x, fd, None, opts)
        if st["status"] != 0 or not st["converged"]:
            raise RuntimeError(f"batched solve did not converge: {st}")
        info["cycles"] = st["cycles"]

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {
        "metric": "MG solve DOF/s to 1e-10 rel. residual, FP32-refined vs FP64; % HBM peak",
        "value": ncell * args.steps / dt, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-in-f64" if prec == A.MIXED else "f64", "data": "synthetic",
        "config": {"workload": "batch of 1024 independent 2D boxes, sides 8m, m~U{2..32}, Dirichlet Helmholtz",
                   "cells": ncell, "tol_rel": 1e-10, "cycles": info["cycles"], "smoother": args.smoother,
                   "precision": args.precision, "vcycle": "V(2,2)", "setup_s": setup_s, "march": march,
                   "split_storage": split_on},
    }
    if not args.no_timing:
        # the finest sweep over all 1024 boxes, 50 launches back to back
        # between HIP events on the library's stream (amg_time_sweep)
        word = 4 if prec == A.MIXED else 8
        dt_ = torch.float32 if word == 4 else torch.float64
        u_ = (fd * 1e-3).to(dt_)
        f_ = fd.to(dt_)
        t_ = torch.zeros_like(u_)
        H.time_sweep(0, u_, f_, t_, smoother=sm, n=4)
        cnt = 50
        avg_s = H.time_sweep(0, u_, f_, t_, smoother=sm, n=cnt) / 1e3
        del u_, f_, t_
        bytes_launch = (3 if args.smoother == "jacobi" else 2) * word * ncell
        ach = bytes_launch / avg_s / 1e9
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": None,
                           "kernel": f"{args.smoother} {'half-' if args.smoother == 'rb' else ''}sweep, finest depth, all 1024 boxes in one launch"
                                     f"{', colour-split storage' if split_on else ''}",
                           "avg_us": avg_s * 1e6, "launches": cnt, "bytes_per_launch": bytes_launch}
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
