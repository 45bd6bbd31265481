"""Benchmark: sweep cell-direction updates/s and GMRES solve time (FP64 vs mixed).

One step = one application of the reduced operator K x of the reconstructed
low-memory scheme (RLMDG) on the largest workload that fits one GPU: the unit cube
with 128^3 hexahedra, 3D S8 (80 directions), eps = sigma_s = sigma_a = 1 and eight
seeded source fields swept together in one launch, with FP32 sweeps (local solves and
direction sums in single precision; moment vectors, B_11 and the combine in FP64).
A step is the sweep of all eight octants for all eight sources with their angular
reductions, then the combine.  value = n_cells * n_dir * n_sources * steps / timed
seconds.  The dominant kernel (the 3D sweep) is timed live with HIP events on its
launch stream for the roofline figure; its algorithmic bytes per launch are
O p [2 + n_rhs (n_P + n_out)] n_cells (per octant pass each cell's two material values
and its moments are read once and its reductions written once, p = 4 bytes).

Afterwards: the same workload solved to a true FP64 relative residual of 1e-8 in FP64
and mixed mode; the other workloads as secondary figures (256^2 S8 eps = 1e-3 FP64 with
its own roofline, the 1024^2 S16 multiscale workload with FP64 and mixed solves, the
512^2 S12 detector gradients, a slab, the 20^2 S4 solves); and the CPU oracle timed on
bounded samples (see cpu_baseline.sample).  The 2D low-memory solves use the two-level
preconditioner (lmdg_set_preconditioner; --precond none for plain LGMRES); the 3D and
slab solves and the 20^2 S4 solves run without it.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-solve] [--no-extra]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed) peak, TFLOP/s
# floating-point work of one 3D RLMDG cell-direction update in the FP32 sweep kernel: its
# step executes 72 FP32 VALU instructions (35 of them FMAs, counted twice) per lane
FLOPS_PER_UPDATE_RLMDG3 = 107


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
    ap.add_argument("--cpu-seconds", type=float, default=5.0)
    ap.add_argument("--solve-max-iter", type=int, default=16000)
    ap.add_argument("--cfg3-max-iter", type=int, default=3000,
                    help="operator applications allowed to each solve of the 1024^2 multiscale workload")
    ap.add_argument("--augment", type=int, default=10,
                    help="LGMRES: earlier corrections searched per restart cycle (0 = plain GMRES)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the secondary measurements (other workloads, several sources, small solves)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of 64 MiB five times (HBM counter calibration)")
    ap.add_argument("--profile-workload", type=int, default=0,
                    help="only time K x on workload 3, 4 or 5 (all its sources) for a profiler run")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32"))
    ap.add_argument("--precond", default="two-level", choices=("none", "cell", "two-level"),
                    help="preconditioner of the 2D low-memory solves (256^2, 1024^2, 512^2 adjoint)")
    ap.add_argument("--pc-cycles", type=int, default=1, help="V-cycles per preconditioner application")
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


def sweep_bytes_per_launch(ncell, scheme, dim, n_rhs, word):
    """Algorithmic HBM bytes of one sweep launch: per octant (quadrant) pass each cell's
    two material values and its n_P moments per source are read once and its n_out
    reductions per source written once, `word` bytes each:
    O word [2 + n_rhs (n_P + n_out)] n_cells, n_out = n_P (STD, LMDG) or n_P + dim (RLMDG)."""
    n_p = 2 ** dim
    n_out = n_p + dim if scheme == "rlmdg" else n_p
    return (2 ** dim) * word * (2 + n_rhs * (n_p + n_out)) * ncell


PROFILES = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles")
CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1907_01027_amd", "csrc")
TRAFFIC = {  # dominant kernel of a workload: counter record and the source it was taken on
    5: ("sweep3d_rlmdg_128_s8_8src_fp32_traffic.json", "sweep3d.hip"),
    2: ("sweep_rlmdg_256_s8_traffic.json", "sweep2d.hip"),
}


def measured_traffic(key):
    """HBM bytes per sweep launch from the committed FETCH_SIZE / WRITE_SIZE counter runs,
    scaled by the same counters' reading for a plain copy of known size; None when the
    counters were taken on a different sweep source."""
    import hashlib
    name, source = TRAFFIC[key]
    try:
        rec = json.load(open(os.path.join(PROFILES, name)))
        src = hashlib.sha256(open(os.path.join(CSRC, source), "rb").read()).hexdigest()
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
    """The CPU oracle (test infrastructure, FP64, untuned) on bounded samples.

    value: its reduced-operator rate (updates/s) on a 12^3 sample of the headline recipe
    (3D S8, RLMDG, one source at a time: the oracle has no multi-source path).  Beside
    it: the oracle's full solves of the 20^2 S4 workload (to 1e-10, both schemes), and its
    preconditioned solve of the 256^2 S8 recipe on a 128^2 sample (to 1e-8)."""
    from oracle import schemes as S
    from oracle.dg import Mesh
    from oracle.quadrature import level_symmetric
    from paper_1907_01027_amd.workloads import materials
    threads = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    n = (12, 12, 12)
    ss, sa, ep, q = materials(5, n=n)
    om, w = level_symmetric(8, 3)
    t0 = time.perf_counter()
    red = S.LowMemoryReduced(S.Problem(Mesh(n, (1.0, 1.0, 1.0)), om, w, ss, sa, ep, q=q[0]), reconstructed=True)
    setup = time.perf_counter() - t0
    x = np.random.default_rng(0).normal(size=8 * int(np.prod(n)))
    k = 0
    t0 = time.perf_counter()
    while True:
        red.apply(x)
        k += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    ups = int(np.prod(n)) * len(w) * k / el
    del red
    # 20^2, S4, eps = 1: full oracle solves (reduced route, its own GMRES) to 1e-10
    ss1, sa1, ep1, q1 = materials(1)
    om2, w2 = level_symmetric(4, 2)
    prob1 = S.Problem(Mesh((20, 20)), om2, w2, ss1, sa1, ep1, q=q1[0])
    solves = {}
    for name, make in (("std", lambda: S.StdReduced(prob1)), ("lmdg", lambda: S.LowMemoryReduced(prob1, False))):
        t0 = time.perf_counter()
        _, its = make().solve(tol=1e-10, restart=30)
        solves[f"20x20_S4_{name}_tol1e-10"] = {"wall_s": time.perf_counter() - t0, "iterations": its}
    # 256^2 recipe on a 128^2 sample: the oracle's own preconditioned solve (its direct
    # solve of the diffusion operator) to 1e-8, set-up included
    from oracle import precond as PC
    n2 = (128, 128)
    ss2, sa2, ep2, q2 = materials(2, n=n2)
    om8, w8 = level_symmetric(8, 2)
    t0 = time.perf_counter()
    red2 = S.LowMemoryReduced(S.Problem(Mesh(n2), om8, w8, ss2, sa2, ep2, q=q2[0]), reconstructed=True)
    setup2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    x2 = np.random.default_rng(1).normal(size=4 * n2[0] * n2[1])
    red2.apply(x2)
    apply128 = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, its2 = PC.solve(red2, tol=1e-8, restart=30)
    solve128 = time.perf_counter() - t0
    return {"value": ups, "unit": "cell-direction updates/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle RLMDG reduced operator K x (sparse LU of each direction's sweep block, FP64, "
                      f"one source) on a 12^3 mesh with the 3D S8 set and the headline recipe: {k} applications "
                      f"in {el:.1f} s after {setup:.1f} s of assembly and factorisation; single-threaded "
                      f"SciPy/NumPy (host has {os.cpu_count()} logical CPUs; thread settings {threads})",
            "solves": solves,
            "128x128_S8_eps1e-3_rlmdg_preconditioned_solve": {
                "wall_s": solve128, "setup_s": setup2, "iterations": its2, "apply_s": apply128,
                "note": "oracle two-level preconditioner with a direct solve of its diffusion operator, "
                        "GMRES(30) to 1e-8; the 256^2 recipe on a 128^2 mesh (sample)"}}


def _apply_rate(torch, lmdg, h, scheme, prec, x, y, ncell, ndir, n_rhs=1, reps=5):
    for _ in range(2):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    lmdg.lmdg_synchronize(h)
    return {"ms_per_apply": 1e3 * el, "updates_per_s": ncell * ndir * n_rhs / el}


def _kernel_ms(torch, lmdg, h, scheme, prec, x, y, reps):
    """Sweep-kernel time per launch from the library's HIP events (on the launch stream)."""
    lmdg.lmdg_profile(h, True)
    for _ in range(reps):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    ms, k = lmdg.lmdg_sweep_kernel_time(h)
    lmdg.lmdg_profile(h, False)
    lmdg.lmdg_synchronize(h)
    return ms / max(k, 1)


def _solve_pair(torch, lmdg, h, scheme, N, tol, restart, max_iter, dev, label, rows=None):
    """FP64 and mixed solves from x0 = 0; the mixed scalar flux against the FP64 one."""
    res, phi64 = {}, None
    for mode in ("fp64", "mixed"):
        xs = torch.zeros(N, dtype=torch.float64, device=dev)
        phi = torch.zeros_like(xs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = lmdg.lmdg_solve(h, scheme, mode, tol, restart, max_iter, xs, phi, raise_on_nonconvergence=False)
        torch.cuda.synchronize()
        info["wall_s"] = time.perf_counter() - t0
        del xs
        sel = phi if rows is None else rows(phi)
        if mode == "fp64":
            phi64 = sel.clone()
        else:
            info["phi_rel_diff_vs_fp64"] = float((sel - phi64).abs().max() / phi64.abs().max())
        res[mode] = info
        _progress(f"{label} {mode} solve done ({info['iterations']} applications, "
                  f"rel residual {info['rel_residual']:.2e})")
    return res


def extra_measurements(torch, lmdg, WORKLOADS, materials, args):
    """Secondary figures on the other workloads (see the module docstring)."""
    from paper_1907_01027_amd.adjoint import box_detector_moments
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    res = {}
    # 256x256, S8, eps = 1e-3, RLMDG, FP64: operator rate, its sweep kernel against the
    # HBM roofline, and solves to 1e-8 with LGMRES(60 + 10)
    wl = WORKLOADS[2]
    ss, sa, ep, q = materials(2)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    nc = wl.n[0] * wl.n[1]
    x = T(np.random.default_rng(7).normal(size=4 * nc))
    y = torch.empty_like(x)
    e2 = {p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, nc, len(w), reps=20) for p in ("fp64", "fp32")}
    kms = _kernel_ms(torch, lmdg, s.h, "rlmdg", "fp64", x, y, 20)
    nbytes = sweep_bytes_per_launch(nc, "rlmdg", 2, 1, 8)
    ach = nbytes / (kms * 1e-3) / 1e9
    e2["roofline_fp64"] = {"bound": "hbm", "kernel": "sweep2d_kernel<double, RLMDG>", "kernel_ms": kms,
                           "bytes_per_launch": nbytes, "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(2)}
    if not args.no_solve:
        lmdg.lmdg_set_preconditioner(s.h, args.precond, args.pc_cycles)
        e2["solve_tol1e-8"] = _solve_pair(torch, lmdg, s.h, "rlmdg", 4 * nc, 1e-8, 30, args.solve_max_iter, dev,
                                          "256^2")
        e2["solve_tol1e-8"].update({"restart": 30, "precond": args.precond, "pc_cycles": args.pc_cycles})
        if args.precond != "none":
            # the same solves without the preconditioner: LGMRES(60 + 10)
            lmdg.lmdg_set_preconditioner(s.h, "none", 1)
            lmdg.lmdg_set_augment(s.h, args.augment)
            e2["solve_tol1e-8_unpreconditioned"] = _solve_pair(torch, lmdg, s.h, "rlmdg", 4 * nc, 1e-8, 60,
                                                               args.solve_max_iter, dev, "256^2 unpreconditioned")
            e2["solve_tol1e-8_unpreconditioned"].update({"restart": 60, "augment": args.augment})
    res["256x256_S8_eps1e-3_rlmdg"] = e2
    s.close()
    del x, y
    # 1024x1024, S16, eps 1 | 1e-4, RLMDG: operator rates and solves to 1e-8 (bounded)
    wl = WORKLOADS[3]
    ss, sa, ep, q = materials(3)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    nc = wl.n[0] * wl.n[1]
    x = T(np.random.default_rng(1).normal(size=4 * nc))
    y = torch.empty_like(x)
    e3 = {p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, nc, len(w)) for p in ("fp64", "fp32")}
    del x, y
    if not args.no_solve:
        lmdg.lmdg_set_preconditioner(s.h, args.precond, args.pc_cycles)
        if args.precond == "none":
            lmdg.lmdg_set_augment(s.h, args.augment)
        restart = 30 if args.precond != "none" else 60
        e3["solve_tol1e-8"] = _solve_pair(torch, lmdg, s.h, "rlmdg", 4 * nc, 1e-8, restart, args.cfg3_max_iter,
                                          dev, "1024^2")
        e3["solve_tol1e-8"].update({"max_iter": args.cfg3_max_iter, "restart": restart, "precond": args.precond,
                                    "pc_cycles": args.pc_cycles})
    res["1024x1024_S16_multiscale_rlmdg"] = e3
    s.close()
    _progress("1024^2 workload done")
    # 512x512, S12, eps = 1e-2, LMDG: detector response and its gradients (forward and
    # adjoint solves to 1e-8 with LGMRES(60 + 10), per-quadrant recomputed fluxes)
    wl = WORKLOADS[4]
    ss, sa, ep, q = materials(4)
    om, w = lmdg.lmdg_quadrature_level_symmetric(2, wl.order)
    s = lmdg.Solver(wl.n, (1.0, 1.0), om, w)
    lmdg.lmdg_set_materials(s.h, T(ss), T(sa), T(ep), T(q[0]))
    lmdg.lmdg_set_preconditioner(s.h, args.precond, args.pc_cycles)
    adj_restart = 30 if args.precond != "none" else 60
    if args.precond == "none":
        lmdg.lmdg_set_augment(s.h, 10)
    nc = wl.n[0] * wl.n[1]
    x = T(np.random.default_rng(1).normal(size=4 * nc))
    y = torch.empty_like(x)
    e4 = {p: _apply_rate(torch, lmdg, s.h, "lmdg", p, x, y, nc, len(w)) for p in ("fp64", "fp32")}
    del x, y
    lo, hi = wl.extra["detector"]
    det = T(box_detector_moments(wl.n, (1.0, 1.0), lo, hi).ravel())
    g64 = None
    for mode in ("fp64", "mixed") if not args.no_solve else ():
        g = [torch.zeros(nc, dtype=torch.float64, device=dev) for _ in range(3)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            J, info = lmdg.lmdg_adjoint_solve(s.h, "lmdg", mode, det, 1e-8, adj_restart, 30000, *g)
            ok = True
        except lmdg.LmdgError as e:
            J, info, ok = float("nan"), {"error": str(e)}, False
        torch.cuda.synchronize()
        e = {"wall_s": time.perf_counter() - t0, "J": J, "converged": ok, "precond": args.precond,
             "restart": adj_restart, "iterations": info.get("iterations"), "rel_residual": info.get("rel_residual")}
        if mode == "fp64":
            g64, J64 = g, J
        elif ok and g64 is not None:
            e["J_rel_diff_vs_fp64"] = abs(J - J64) / abs(J64)
            for name, a64, a in zip(("sigma_s", "sigma_a", "q"), g64, g):
                e[f"grad_{name}_rel_diff_vs_fp64"] = float((a - a64).abs().max() / a64.abs().max())
        e4[f"adjoint_gradients_{mode}"] = e
    res["512x512_S12_eps1e-2_lmdg"] = e4
    s.close()
    del g64
    _progress("512^2 workload done")
    # slab geometry (a handle with dim 1): 1024 cells of [0, pi], 32-point Gauss rule,
    # eps = sigma_s = sigma_a = 1, q = (4/3) sin x (exact cell moments), vacuum inflow, RLMDG
    ncs = 1024
    mu, gw = np.polynomial.legendre.leggauss(32)
    s = lmdg.Solver((ncs,), (np.pi,), mu[:, None], gw / 2.0)
    edges = np.linspace(0.0, np.pi, ncs + 1)
    hh = edges[1] - edges[0]
    qm = np.zeros((4, ncs))
    qm[0] = 4.0 / 3.0 * (np.cos(edges[:-1]) - np.cos(edges[1:])) / hh
    # (1/h) int (4/3) sin x xi dx with xi = 2 (x - x_c) / h, in closed form
    xc = 0.5 * (edges[:-1] + edges[1:])
    qm[1] = 4.0 / 3.0 * 2.0 / hh * (np.sin(edges[1:]) - np.sin(edges[:-1])
                                    - 0.5 * hh * (np.cos(edges[1:]) + np.cos(edges[:-1]))) / hh
    one = np.ones(ncs)
    lmdg.lmdg_set_materials(s.h, T(one), T(one), T(one), T(qm[0]))
    lmdg.lmdg_set_source_moments(s.h, T(qm))
    x = T(np.random.default_rng(4).normal(size=4 * ncs))
    y = torch.empty_like(x)
    slab = {p: _apply_rate(torch, lmdg, s.h, "rlmdg", p, x, y, ncs, 32) for p in ("fp64", "fp32")}
    if not args.no_solve:
        slab["solve_tol1e-8"] = _solve_pair(torch, lmdg, s.h, "rlmdg", 4 * ncs, 1e-8, 30, 2000, dev, "slab",
                                            rows=lambda phi: phi.reshape(4, ncs)[:2])
    res["slab_1024_G32_rlmdg"] = slab
    s.close()
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
    _progress("slab and 20^2 solves done")
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

    wl = WORKLOADS[5]
    n = wl.n
    scheme = wl.scheme
    ss, sa, ep, q = materials(5)
    n_rhs = q.shape[0]
    omega, w = lmdg.lmdg_quadrature_level_symmetric(3, wl.order)
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    solver = lmdg.Solver(n, (1.0, 1.0, 1.0), omega, w)
    h = solver.h
    lmdg.lmdg_set_materials(h, T(ss), T(sa), T(ep), T(q[0]))
    lmdg.lmdg_set_sources(h, T(q))
    ncell = int(np.prod(n))
    N = 8 * ncell * n_rhs
    x = T(np.random.default_rng(7).normal(size=N))
    y = torch.empty(N, dtype=torch.float64, device=dev)
    prec = "fp32"
    for _ in range(args.warmup):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    lmdg.lmdg_profile(h, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lmdg.lmdg_apply(h, scheme, prec, x, y)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lmdg.lmdg_synchronize(h)  # raises if any sweep wait of the timed launches gave up
    k_ms, k_n = lmdg.lmdg_sweep_kernel_time(h)
    lmdg.lmdg_profile(h, False)
    ms_step = 1e3 * elapsed / args.steps
    updates = ncell * len(w) * n_rhs * args.steps / elapsed
    sweep_ms = k_ms / max(k_n, 1)
    _progress(f"timed steps done ({args.steps} operator applications)")
    nbytes = sweep_bytes_per_launch(ncell, scheme, 3, n_rhs, 4)
    achieved = nbytes / (sweep_ms * 1e-3) / 1e9
    alu_tflops = FLOPS_PER_UPDATE_RLMDG3 * ncell * len(w) * n_rhs / (sweep_ms * 1e-3) / 1e12
    del x, y
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
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "128^3 unit cube, trilinear DG, 3D S8 level-symmetric (80 directions), eps=1, "
                               "sigma_s=sigma_a=1, 8 seeded source fields U[0,1] swept together, vacuum inflow, "
                               "low-memory DG with upwind reconstruction (RLMDG); FP32 sweeps, FP64 moment vectors "
                               "and Krylov",
                   "cells": ncell, "directions": len(w), "sources": n_rhs,
                   "step": "one reduced-operator application K x for all sources"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(5),
                     "kernel": "sweep3d_kernel<float, RLMDG>", "kernel_ms": sweep_ms,
                     "bytes_per_launch": nbytes,
                     # the sweep's arithmetic against the FP32 vector peak (its step issues no
                     # packed FP32 instructions, whose rate the peak assumes)
                     "alu": {"flops_per_update": FLOPS_PER_UPDATE_RLMDG3,
                             "achieved_tflops": alu_tflops, "peak_tflops": FP32_VECTOR_PEAK_TFLOPS,
                             "frac": alu_tflops / FP32_VECTOR_PEAK_TFLOPS}},
    }
    if not args.no_solve:
        # mixed mode: four digits per inner FP32 solve (two refinement passes instead of three)
        lmdg.lmdg_set_refinement(h, 1e-4)
        out["solve"] = {"tol": 1e-8, "restart": 30, "max_iter": 400, "mixed_inner_tol": 1e-4,
                        **_solve_pair(torch, lmdg, h, scheme, N, 1e-8, 30, 400, dev, "128^3")}
    solver.close()
    if not args.no_extra:
        out["extra"] = extra_measurements(torch, lmdg, WORKLOADS, materials, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        _progress("CPU baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
