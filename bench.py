"""Benchmark: sweep cell-direction updates/s and GMRES solve time (FP64 vs mixed).

One step = one application of the reduced operator K x of the reconstructed
low-memory scheme (all four quadrant sweeps with their angular reductions, the
B_11 stencil and the combine) on the 256 x 256, S8 (40 directions) workload with
eps = 1e-3 and seeded 8 x 8 block cross sections.  value = n_cells * n_dir * steps
/ timed seconds.  After the timed steps the same workload is solved to a true FP64
relative residual of 1e-8 in FP64 mode and in mixed mode (FP32 sweeps) with
LGMRES(60 + 10) (restart cycles augmented with the last ten corrections), and the
dominant kernel (the sweep) is timed live with HIP events on its launch stream for
the roofline figure.  The CPU baseline times the CPU oracle's operator on a bounded
sample of the same recipe (see cpu_baseline.sample).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-solve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def _progress(msg):
    """One line per finished measurement on stderr (the JSON result goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--solve-max-iter", type=int, default=16000)
    ap.add_argument("--augment", type=int, default=10,
                    help="LGMRES: earlier corrections searched per restart cycle (0 = plain GMRES)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary measurements (other workloads, several sources, small solves)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 64 MiB five times (HBM counter calibration)")
    ap.add_argument("--profile-workload", type=int, default=0,
                    help="only time K x on workload 3, 4 or 5 (all its sources) for a profiler run")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32"))
    return ap.parse_args()


def profile_workload(key, prec, steps, warmup):
    """Warm-up and timed operator applications of one workload (for rocprofv3 runs)."""
    import torch
    from paper_1907_01027_amd import lmdg
    from paper_1907_01027_amd.workloads import WORKLOADS, materials
    wl = WORKLOADS[key]
    ss, sa, ep, q = materials(key)
    dim = len(wl.n)
    om, w = lmdg.lmdg_quadrature_level_symmetric(dim, wl.order)
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda:0")
    s = lmdg.Solver(wl.n, (1.0,) * dim, om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    if q.shape[0] > 1:
        lmdg.lmdg_set_sources(s.h, T(q))
    nc = int(np.prod(wl.n))
    npm = 4 if dim == 2 else 8
    x = T(np.random.default_rng(5).normal(size=q.shape[0] * npm * nc))
    y = torch.empty_like(x)
    for _ in range(warmup):
        lmdg.lmdg_apply(s.h, wl.scheme, prec, x, y)
    torch.cuda.synchronize()
    lmdg.lmdg_profile(s.h, True)
    t0 = time.perf_counter()
    for _ in range(steps):
        lmdg.lmdg_apply(s.h, wl.scheme, prec, x, y)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / steps
    ms, k = lmdg.lmdg_sweep_kernel_time(s.h)
    s.close()
    print(json.dumps({"workload": wl.name, "prec": prec, "ms_per_apply": 1e3 * el, "sweep_kernel_ms": ms / max(k, 1),
                      "updates_per_s": nc * len(w) * q.shape[0] / el}), flush=True)


def sweep_bytes_per_launch(ncell, scheme):
    """Algorithmic HBM bytes of one operator sweep launch (FP64): per quadrant each cell's
    inputs (x_0, the two slope moments of x_1, sigma_t|K|, sigma_s/eps |K|) are read once
    and its per-quadrant reductions (6 for RLMDG, 3 LMDG, 4 STD) written once."""
    n_in = 5 if scheme != "std" else 6
    n_out = {"rlmdg": 6, "lmdg": 3, "std": 4}[scheme]
    return 4 * ncell * (n_in + n_out) * 8


TRAFFIC_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "sweep_rlmdg_256_s8_traffic.json")
SWEEP_SOURCE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1907_01027_amd", "csrc", "sweep2d.hip")


def measured_traffic():
    """HBM bytes per sweep launch from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    scaled by the same counters' reading for a plain copy of known size; None when the
    counters were taken on a different sweep source."""
    import hashlib
    try:
        rec = json.load(open(TRAFFIC_FILE))
        src = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("sweep_source_sha256") != src:
        return None
    return rec["fetch_bytes_per_launch"] / rec["copy_fetch_factor"] + rec["write_bytes_per_launch"] / rec["copy_write_factor"]


def calibrate_copy():
    import torch
    n = 1 << 23
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 5}), flush=True)


def cpu_baseline(seconds):
    """Oracle reduced operator (CPU, FP64) on a 128 x 128 sample of the same recipe."""
    from oracle import schemes as S
    from oracle.dg import Mesh
    from oracle.quadrature import level_symmetric
    from paper_1907_01027_amd.workloads import materials
    n = (128, 128)
    ss, sa, ep, q = materials(2, n=n)
    om, w = level_symmetric(8, 2)
    t0 = time.perf_counter()
    prob = S.Problem(Mesh(n), om, w, ss, sa, ep, q=q[0])
    red = S.LowMemoryReduced(prob, reconstructed=True)
    setup = time.perf_counter() - t0
    x = np.random.default_rng(0).normal(size=4 * n[0] * n[1])
    k = 0
    t0 = time.perf_counter()
    while True:
        red.apply(x)
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    ups = n[0] * n[1] * len(w) * k / el
    return {"value": ups, "unit": "cell-direction updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle RLMDG reduced operator K x (sparse LU of each direction's sweep block, "
                      f"FP64) on the 128x128 S8 mesh of the same seeded recipe; {k} applications in "
                      f"{el:.1f} s after {setup:.1f} s of assembly and factorisation; single-threaded "
                      f"SciPy/NumPy (host has {os.cpu_count()} logical CPUs)"}


def _apply_rate(torch, lmdg, h, scheme, prec, x, y, ncell, ndir, n_rhs=1, reps=5):
    for _ in range(2):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    return {"ms_per_apply": 1e3 * el, "updates_per_s": ncell * ndir * n_rhs / el}


def extra_measurements(torch, lmdg, WORKLOADS, materials):
    """Secondary figures: operator throughput on the other 2D workloads (FP64 and FP32
    sweeps), eight sources swept together, the 512x512 S12 detector gradients (adjoint
    solves, FP64 vs mixed), a 1024-cell slab (operator rates and solves), FP64 vs mixed
    solves of the 20x20 S4 workload to 1e-8 and
    1e-10, and the 128^3 3D workload with eight sources (operator throughput and solves
    to 1e-8, FP64 vs mixed)."""
    from paper_1907_01027_amd.adjoint import box_detector_moments
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    res = {}
    for key in (3, 4):
        wl = WORKLOADS[key]
        ss, sa, ep, q = materials(key)
        om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
        s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
        lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
        nc = wl.n[0] * wl.n[1]
        x = T(np.random.default_rng(1).normal(size=4 * nc))
        y = torch.empty_like(x)
        res[f"{wl.n[0]}x{wl.n[1]}_S{wl.order}_{wl.scheme}"] = {
            p: _apply_rate(torch, lmdg, s.h, wl.scheme, p, x, y, nc, len(w)) for p in ("fp64", "fp32")}
        s.close()
    _progress("operator rates of the 1024^2 and 512^2 workloads done")
    # eight sources on the benchmark mesh, swept together
    wl = WORKLOADS[2]
    ss, sa, ep, q = materials(2)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    nc = wl.n[0] * wl.n[1]
    qs = np.random.default_rng(20190708).uniform(0.0, 1.0, size=(8, nc))
    lmdg.lmdg_set_sources(s.h, T(qs))
    x = T(np.random.default_rng(2).normal(size=8 * 4 * nc))
    y = torch.empty_like(x)
    res["256x256_S8_rlmdg_8_sources"] = {
        p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, nc, len(w), n_rhs=8) for p in ("fp64", "fp32")}
    s.close()
    _progress("eight-source operator rates done")
    # 512x512, S12, eps = 1e-2, LMDG: detector response and its gradients (forward and
    # adjoint solves to 1e-8 with LGMRES(60 + 10), per-quadrant recomputed fluxes)
    wl = WORKLOADS[4]
    ss, sa, ep, q = materials(4)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    lmdg.lmdg_set_augment(s.h, 10)
    nc = wl.n[0] * wl.n[1]
    lo, hi = wl.extra["detector"]
    det = T(box_detector_moments(wl.n, (1.0, 1.0), lo, hi).ravel())
    adj = {}
    g64 = None
    for mode in ("fp64", "mixed"):
        g = [torch.zeros(nc, dtype=torch.float64, device=dev) for _ in range(3)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            J, info = lmdg.lmdg_adjoint_solve(s.h, "lmdg", mode, det, 1e-8, 60, 30000, *g)
            ok = True
        except lmdg.LmdgError as e:
            J, info, ok = float("nan"), {"error": str(e)}, False
        torch.cuda.synchronize()
        e = {"wall_s": time.perf_counter() - t0, "J": J, "converged": ok,
             "iterations": info.get("iterations"), "rel_residual": info.get("rel_residual")}
        if mode == "fp64":
            g64, J64 = g, J
        elif ok and g64 is not None:
            e["J_rel_diff_vs_fp64"] = abs(J - J64) / abs(J64)
            for name, a64, a in zip(("sigma_s", "sigma_a", "q"), g64, g):
                e[f"grad_{name}_rel_diff_vs_fp64"] = float((a - a64).abs().max() / a64.abs().max())
        adj[mode] = e
    res["512x512_S12_lmdg_adjoint_gradients"] = adj
    s.close()
    del g64
    _progress("512^2 adjoint gradients done")
    # slab geometry (a handle with dim 1): 1024 cells of [0, pi], 32-point Gauss rule,
    # eps = sigma_s = sigma_a = 1, q = (4/3) sin x (cell averages), vacuum inflow, RLMDG
    ncs = 1024
    mu, gw = np.polynomial.legendre.leggauss(32)
    s = lmdg.Solver((ncs,), (np.pi,), mu[:, None], gw / 2.0)
    edges = np.linspace(0.0, np.pi, ncs + 1)
    qs = 4.0 / 3.0 * (np.cos(edges[:-1]) - np.cos(edges[1:])) / (edges[1] - edges[0])
    one = np.ones(ncs)
    lmdg.lmdg_set_materials(s.h, T(one), T(one), T(one), T(qs))
    x = T(np.random.default_rng(4).normal(size=4 * ncs))
    y = torch.empty_like(x)
    slab = {p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, ncs, 32) for p in ("fp64", "fp32")}
    phi64 = None
    for mode in ("fp64", "mixed"):
        xs = torch.zeros(4 * ncs, dtype=torch.float64, device=dev)
        phi = torch.zeros_like(xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = lmdg.lmdg_solve(s.h, "rlmdg", mode, 1e-8, 30, 2000, xs, phi, raise_on_nonconvergence=False)
        torch.cuda.synchronize()
        e = {"wall_ms": 1e3 * (time.perf_counter() - t0), "iterations": info["iterations"],
             "converged": info["converged"], "rel_residual": info["rel_residual"]}
        rows = phi.reshape(4, ncs)[:2]  # the slab moments (1, xi)
        if mode == "fp64":
            phi64 = rows.clone()
        else:
            e["phi_rel_diff_vs_fp64"] = float((rows - phi64).abs().max() / phi64.abs().max())
        slab[f"solve_{mode}_tol1e-8"] = e
    res["slab_1024_G32_rlmdg"] = slab
    s.close()
    _progress("slab solves done")
    # 20x20, S4, eps = 1: solve times to 1e-8 and 1e-10, FP64 vs mixed
    wl = WORKLOADS[1]
    ss, sa, ep, q = materials(1)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    nc = wl.n[0] * wl.n[1]
    xs = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    phi = torch.zeros_like(xs)
    solves = {}
    for scheme in ("std", "lmdg"):
        for tol in (1e-8, 1e-10):
            phi64 = None
            for mode in ("fp64", "mixed"):
                lmdg.lmdg_solve(s.h, scheme, mode, tol, 30, 2000, xs, phi)  # warm
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = lmdg.lmdg_solve(s.h, scheme, mode, tol, 30, 2000, xs, phi)
                torch.cuda.synchronize()
                entry = {"wall_ms": 1e3 * (time.perf_counter() - t0), "iterations": info["iterations"],
                         "ir_passes": info["ir_passes"], "rel_residual": info["rel_residual"]}
                if mode == "fp64":
                    phi64 = phi.clone()
                else:  # scalar flux of the mixed solve against the FP64 solve at the same tolerance
                    entry["phi_rel_diff_vs_fp64"] = float((phi - phi64).abs().max() / phi64.abs().max())
                solves[f"{scheme}_{mode}_tol{tol:g}"] = entry
    res["20x20_S4_eps1_solves"] = solves
    s.close()
    _progress("20^2 solves done")
    # 128^3, 3D S8 (80 directions), RLMDG, eight sources swept together; solves to 1e-8
    wl = WORKLOADS[5]
    ss, sa, ep, q = materials(5)
    om, w = lmdg.lmdg_quadrature_level_symmetric(3, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    lmdg.lmdg_set_sources(s.h, T(q))
    nc = int(np.prod(wl.n))
    nr = q.shape[0]
    x = T(np.random.default_rng(3).normal(size=nr * 8 * nc))
    y = torch.empty_like(x)
    entry = {p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, nc, len(w), n_rhs=nr, reps=3) for p in ("fp64", "fp32")}
    del x, y
    # The residual norm constrains the slope moments only weakly here, so two solutions
    # at tol 1e-8 differ at the 1e-3 level in them; a second FP64 solve with another
    # restart length shows the size of that tolerance-level difference beside the mixed one.
    phi64 = None
    for name, mode, restart in (("solve_fp64_tol1e-8", "fp64", 30), ("solve_fp64_restart20_tol1e-8", "fp64", 20),
                                ("solve_mixed_tol1e-8", "mixed", 30)):
        xs = torch.zeros(nr * 8 * nc, dtype=torch.float64, device=dev)
        phi = torch.zeros_like(xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = lmdg.lmdg_solve(s.h, "rlmdg", mode, 1e-8, restart, 400, xs, phi, raise_on_nonconvergence=False)
        torch.cuda.synchronize()
        e = {"wall_s": time.perf_counter() - t0, "restart": restart, "iterations": info["iterations"],
             "ir_passes": info["ir_passes"], "converged": info["converged"], "rel_residual": info["rel_residual"]}
        del xs
        _progress(f"128^3 {name} done ({info['iterations']} applications)")
        if phi64 is None:
            phi64 = phi
        else:
            pr = phi.reshape(nr, 8, nc)
            rr = phi64.reshape(nr, 8, nc)
            scale = rr.abs().amax()
            e["phi_rel_diff_vs_fp64"] = float((pr - rr).abs().amax() / scale)
            e["scalar_flux_row_rel_diff_vs_fp64"] = float((pr[:, 0] - rr[:, 0]).abs().amax() / scale)
            del phi
        entry[name] = e
    del phi64
    res["128^3_S8_rlmdg_8_sources"] = entry
    s.close()
    _progress("128^3 eight-source rates and solves done")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the library has no multi-GPU path. "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.profile_workload:
        profile_workload(args.profile_workload, args.prec, args.steps, args.warmup)
        return
    import torch
    from paper_1907_01027_amd import lmdg
    from paper_1907_01027_amd.workloads import WORKLOADS, materials

    wl = WORKLOADS[2]
    n = wl.n
    scheme = wl.scheme
    ss, sa, ep, q = materials(2)
    omega, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(a, dtype=torch.float64, device=dev)
    solver = lmdg.Solver(n, (1.0, 1.0), omega, w)
    h = solver.h
    lmdg.lmdg_set_materials(h, T(ss), T(sa), T(ep), T(q[0]))
    ncell = n[0] * n[1]
    N = 4 * ncell
    x = T(np.random.default_rng(7).normal(size=N))
    y = torch.empty(N, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        lmdg.lmdg_apply(h, scheme, "fp64", x, y)
    torch.cuda.synchronize()
    lmdg.lmdg_profile(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lmdg.lmdg_apply(h, scheme, "fp64", x, y)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lmdg.lmdg_synchronize(h)  # raises if any sweep wait of the timed launches gave up
    k_ms, k_n = lmdg.lmdg_sweep_kernel_time(h)
    lmdg.lmdg_profile(h, False)
    ms_step = 1e3 * elapsed / args.steps
    updates = ncell * len(w) * args.steps / elapsed
    sweep_ms = k_ms / max(k_n, 1)
    _progress(f"timed steps done ({args.steps} operator applications)")
    nbytes = sweep_bytes_per_launch(ncell, scheme)
    achieved = nbytes / (sweep_ms * 1e-3) / 1e9
    out = {
        "metric": "sweep cell-direction updates/s + GMRES solve time to 1e-8, FP64 vs mixed",
        "value": updates,
        "unit": "cell-direction updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256x256 unit square, S8 level-symmetric (40 directions), eps=1e-3, "
                               "sigma_s/sigma_a on 8x8 blocks U[0.5,2], q U[0,1], vacuum inflow, "
                               "low-memory DG with upwind reconstruction (RLMDG), FP64",
                   "cells": ncell, "directions": len(w), "step": "one reduced-operator application K x"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": "sweep2d_kernel<double, RLMDG>", "kernel_ms": sweep_ms,
                     "bytes_per_launch": nbytes},
    }
    if not args.no_solve:
        res = {}
        xs = torch.zeros(N, dtype=torch.float64, device=dev)
        phi = torch.zeros(N, dtype=torch.float64, device=dev)
        lmdg.lmdg_set_augment(h, args.augment)
        phi64 = None
        for mode in ("fp64", "mixed"):
            xs.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = lmdg.lmdg_solve(h, scheme, mode, 1e-8, 60, args.solve_max_iter, xs, phi,
                                   raise_on_nonconvergence=False)
            torch.cuda.synchronize()
            info["wall_s"] = time.perf_counter() - t0
            _progress(f"256^2 {mode} solve done ({info['iterations']} applications)")
            if mode == "fp64":
                phi64 = phi.clone()
            else:  # scalar flux of the mixed solve against the FP64 solve at the same tolerance
                info["phi_rel_diff_vs_fp64"] = float((phi - phi64).abs().max() / phi64.abs().max())
            res[mode] = info
        out["solve"] = {"tol": 1e-8, "restart": 60, "augment": args.augment, "max_iter": args.solve_max_iter,
                        **res}
    solver.close()
    if not args.no_extra:
        out["extra"] = extra_measurements(torch, lmdg, WORKLOADS, materials)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        _progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
