"""Benchmark: KKT solves per second to 1e-8 relative residual on one MI355X.

Workload (default): 2-D, a = 1, nx = 255 interior points per dimension
(m = 65 025), N = nt = 256 backward-Euler steps (n = 255 time blocks),
T = 1, gamma in {1e-2, 1e-6, 1e-10}, eps = sqrt(tau), smooth-plus-noise
g, f, y0 (seeded), FP64 right-preconditioned GMRES(30) with the
epsilon-circulant RBD preconditioner (time FFT + sine transforms), stopped at
||b - A x|| <= 1e-8 ||b||.  One step solves the three systems (one batched
solve with one member per gamma); inputs are resident in HBM before timing.

Prints one JSON line.  Fields beyond the common contract:
  roofline      -- the kernel family with the largest summed event time in
                   the timed region, its algorithmic bytes per launch over
                   its mean launch duration, against 8 TB/s HBM;
  precond_apply -- the same for the whole preconditioner apply (5 kernels);
  cpu_baseline  -- the FP64 oracle timed on this host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PRECOND_FAMILIES = ("time_fwd", "dst_rows", "dst_ax2", "dst_last_solve", "time_inv", "mg_smooth",
                    "mg_restrict", "mg_prolong")


# kernel sources behind each timed family (to tell whether recorded counters
# still describe the code that runs)
_TIME_SOURCES = ["precond.hip", "time_common.hpp", "time_sk.hip", "time_ip.hpp", "time_ip_fwd_f64.hip",
                 "time_ip_inv_f64.hip", "time_ip_fwd_f32.hip", "time_ip_inv_f32.hip", "time_bl.hip", "fft_lds.hpp"]
FAMILY_SOURCES = {
    "gs_update": ["krylov.hip"], "mdot": ["krylov.hip"], "combine": ["krylov.hip"],
    "kkt_apply": ["kkt.hip", "stencil.hpp", "fem.hip", "fem.hpp"], "time_fwd": _TIME_SOURCES, "time_inv": _TIME_SOURCES,
    "dst_rows": ["dst.hip", "fft_lds.hpp"], "dst_last_solve": ["dst.hip", "fft_lds.hpp"],
    "dst_ax2": ["dst.hip", "fft_lds.hpp"], "mg_smooth": ["multigrid.hip"], "mg_restrict": ["multigrid.hip"],
    "mg_prolong": ["multigrid.hip"], "ideal_step": ["ideal.hip"],
}


def recorded_traffic(workload, family):
    """HBM bytes per launch recorded by rocprofv3 FETCH_SIZE/WRITE_SIZE runs in
    profiles/kernels_<workload>.md, or None when absent or when the kernel
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"kernels_{workload}.md")
    if not os.path.exists(path) or family not in FAMILY_SOURCES:
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
    if not rec or rec.get("workload") != workload or family not in rec.get("families", {}):
        return None
    h = hashlib.sha256()
    for fn in FAMILY_SOURCES[family]:
        with open(os.path.join(ROOT, "paper_2410_22686_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    entry = rec["families"][family]
    return entry["bytes_per_launch"] if entry.get("source") == h.hexdigest()[:12] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5],
                    help="workload: 1 2d-nx31-nt32, 2 2d-nx255-nt256 (default), 3 2d-nx511-nt512-mixed, "
                         "4 2d-nx127-nt128-batch64, 5 3d-nx63-nt128-vara-mg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-seconds", type=float, default=15.0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="override the workload's preconditioner precision")
    ap.add_argument("--graph", type=int, default=None, choices=[0, 1],
                    help="capture Arnoldi chunks as HIP graphs (default: on for the batched and smallest workloads)")
    ap.add_argument("--tune", type=int, default=1, choices=[0, 1],
                    help="time the candidate preconditioner kernels at setup and keep the fastest")
    ap.add_argument("--time-cols", type=int, default=0, choices=[0, -1, -4, -8, -16, 4, 8, 16],
                    help="time-pass kernels: 0 automatic, -P two LDS buffers, +P in place (P points per block)")
    ap.add_argument("--dst-kernel", type=int, default=0, choices=[0, 1, 2, 3, 4],
                    help="sine-transform kernels: 0 automatic, 1 register, 2 LDS-staged, 3 register with wide column "
                         "tiles, 4 half-length strided transforms")
    ap.add_argument("--kkt-jchunk", type=int, default=0, help="KKT matvec kernel: > 0 levels per thread, < 0 LDS tiles of that many levels (0 automatic)")
    ap.add_argument("--krylov-blocks", type=int, default=0, help="Krylov reduction blocks per member (0 automatic)")
    ap.add_argument("--gs-update", type=int, default=0, choices=[0, 1, 2],
                    help="Gram-Schmidt update kernel: 0 automatic, 1 doubles, 2 double2 pairs")
    ap.add_argument("--mass", choices=["identity", "q1"], default="identity",
                    help="identity: finite differences (M = I); q1: bilinear/trilinear finite elements "
                         "(M != I, a = 1, sine transforms)")
    ap.add_argument("--precond", choices=["eps", "ideal"], default="eps",
                    help="eps: the epsilon-circulant preconditioner; ideal: P of eq. matrix_P (sequential in time)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain device copy of 1 GiB (reference for HBM byte counters)")
    return ap.parse_args()


def solver_options(cfg, precision=None, graph=None):
    prec = precision or cfg.precision
    if prec == "mixed" or cfg.spatial == "mg":
        opts = dict(precision=prec, spatial=cfg.spatial, side="flexible")
    else:
        opts = dict(precision="fp64", spatial="dst", side="right")
    opts["graph"] = bool(graph) if graph is not None else cfg.config_id in (1, 4)
    return opts


def cpu_baseline(cfg, iters, budget_s, mass="identity"):
    """Time the FP64 oracle on this host on a bounded sample of the workload
    and scale it to solves/s.

    Sample: the oracle's own pieces at full size for one member -- a few of
    the n per-frequency sparse LU factorisations of (lambda_k + alpha) I +
    tau K and their solves, one dense Fourier-matrix product along time, one
    sparse KKT matvec and one modified Gram-Schmidt step.  A right-
    preconditioned solve of k iterations costs k (apply + matvec) +
    sum_{j<k} (j+1) MGS steps + one final apply, with
    apply = 4 dense DFTs + 2n LU solves (the four steps of Section 2.1);
    factorisations are setup and excluded, as on the GPU."""
    import numpy as np
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    from oracle import discretize as D, precond as P

    t_start = time.perf_counter()
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = 1
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    gamma = cfg.gammas[0]
    pb = D.make_problem(cfg.dim, cfg.nx, cfg.nt, gamma, T=cfg.T, eps=cfg.eps, mass=mass)
    n, m = pb.n, pb.m
    # the sparse KKT matvec costs O(n m): time it on the same grid with 8 time
    # blocks (the oracle's assembly of the full matrix alone takes minutes)
    n_mv = min(8, n)
    pb_mv = D.make_problem(cfg.dim, cfg.nx, n_mv + 1, gamma, T=cfg.T * (n_mv + 1) / cfg.nt, eps=pb.eps, mass=mass)
    A = D.kkt_scaled(pb_mv)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(A.shape[0])
    t0 = time.perf_counter()
    reps = 0
    while True:
        A @ x
        reps += 1
        if time.perf_counter() - t0 > 0.5:
            break
    t_mv = (time.perf_counter() - t0) / reps * (n / n_mv)
    F = P.fourier_matrix(n)
    V = rng.standard_normal((n, m)) + 0j
    F.conj().T @ V  # first call pays page faults and thread start-up
    t0 = time.perf_counter()
    F.conj().T @ V
    t_dft = time.perf_counter() - t0
    lam = P.lambda_eps(n, pb.eps)
    Kc = pb.K.tocsc().astype(np.complex128)
    I = pb.Mm.tocsc().astype(np.complex128)  # M (the identity for finite differences)
    nfac, t_fac, t_lu, nlu = 0, 0.0, 0.0, 0
    rhs = rng.standard_normal(m) + 1j * rng.standard_normal(m)
    while nfac < min(64, n):  # as many as fit about 60% of the time budget
        t0 = time.perf_counter()
        lu = spla.splu(((lam[nfac] + pb.alpha) * I + pb.tau * Kc).tocsc())
        t_fac += time.perf_counter() - t0
        t0 = time.perf_counter()
        for _ in range(3):
            lu.solve(rhs)
        t_lu += time.perf_counter() - t0
        nlu += 3
        nfac += 1
        if time.perf_counter() - t_start > 0.6 * budget_s:
            break
    t_lu /= nlu
    w = rng.standard_normal(2 * n * m)
    v = rng.standard_normal(2 * n * m)
    times = []
    for _ in range(3):  # the first pass pays page faults
        t0 = time.perf_counter()
        h = np.dot(v, w)
        w = w - h * v
        times.append(time.perf_counter() - t0)
    t_mgs = min(times[1:])
    apply_s = 4 * t_dft + 2 * n * t_lu
    total = 0.0
    for k in iters:
        total += k * (apply_s + t_mv) + sum(j + 1 for j in range(k)) * t_mgs + apply_s
    solves_per_s = len(iters) / total
    return {
        "value": solves_per_s, "unit": "solves/s", "cores": int(threads), "host_cores_visible": int(cores),
        "kind": "oracle",
        "sample": (f"FP64 NumPy/SciPy oracle pieces at full size ({cfg.name}, {mass} mass matrix, one member): {nfac} of {n} "
                   f"per-frequency splu factorisations and {nlu} LU solves, one dense time-DFT product, "
                   f"sparse KKT matvecs on {n_mv} of {n} time blocks (scaled by {n}/{n_mv}), one MGS step; scaled to {len(iters)} right-preconditioned solves "
                   f"with the GPU iteration counts {list(iters)}; factorisation (setup, "
                   f"{t_fac / max(nfac, 1):.2f} s each, {n} needed) excluded"),
        "sample_wall_s": round(time.perf_counter() - t_start, 2),
        "per_apply_s": apply_s, "per_matvec_s": t_mv,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_2410_22686_amd import Solver

    cfg = W.CONFIGS[args.config]
    if args.mass == "q1" and cfg.spatial != "dst":
        print(json.dumps({"error": "--mass q1 needs a workload with sine transforms (a = 1)"}))
        sys.exit(2)
    workload = cfg.name + ("-q1" if args.mass == "q1" else "")
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    members = list(range(len(cfg.gammas)))
    print(f"# bench: {cfg.name} members={len(members)} generating inputs", file=sys.stderr, flush=True)
    g = np.empty((len(members), cfg.n, cfg.m))
    f = np.empty_like(g)
    y0 = np.empty((len(members), cfg.m))
    for b in members:
        g[b], f[b], y0[b] = W.fields(cfg, member=b)
    opts = solver_options(cfg, args.precision, args.graph)
    stream = torch.cuda.Stream(device=dev) if opts["graph"] else None
    s = Solver(cfg.dim, cfg.nx, cfg.nt, list(cfg.gammas), T=cfg.T, eps=cfg.eps,
               coeff=None if cfg.coeff == "one" else W.coeff_function(cfg.coeff),
               restart=30, maxit=300, rtol=1e-8, device=dev, stream=stream, tune=bool(args.tune),
               time_cols=args.time_cols, dst_kernel=args.dst_kernel, precond=args.precond,
               kkt_jchunk=args.kkt_jchunk, krylov_blocks=args.krylov_blocks, gs_update=args.gs_update,
               mass=args.mass, **opts)
    print(f"# bench: kernels {s.kernels}", file=sys.stderr, flush=True)
    tg = torch.tensor(g, device=dev)
    tf = torch.tensor(f, device=dev)
    ty0 = torch.tensor(y0, device=dev)
    del g, f
    torch.cuda.synchronize()
    b = s.rhs(tg, tf, ty0)
    torch.cuda.synchronize()
    print("# bench: warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        x, infos, _ = s.solve(b)
    torch.cuda.synchronize()
    print("# bench: timed steps", file=sys.stderr, flush=True)
    # with graphs the timed region runs the captured chunks untouched and the
    # per-kernel table comes from one extra eager solve afterwards
    if not opts["graph"]:
        s.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, infos, _ = s.solve(b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if opts["graph"]:
        s.timing_enable(True)
        s.solve(b)
        torch.cuda.synchronize()
    stats = s.timing_read()
    s.timing_enable(False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    solves = len(members) * args.steps
    value = solves / elapsed
    ok = all(i.converged and i.relres_true <= 1e-8 * 1.0001 for i in infos)

    dom_name, dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    dom_ms_per_launch = dom["ms"] / dom["launches"]
    dom_bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = dom_bytes_per_launch / (dom_ms_per_launch * 1e-3) / 1e9
    traffic = recorded_traffic(workload, dom_name)
    roofline = {"bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_unit": "bytes/launch",
                "bytes_per_launch": dom_bytes_per_launch, "ms_per_launch": dom_ms_per_launch,
                "launches": dom["launches"]}
    pre = {k: v for k, v in stats.items() if k in PRECOND_FAMILIES}
    pre_ms = sum(v["ms"] for v in pre.values())
    pre_bytes = sum(v["bytes"] for v in pre.values())
    applies = max(v["launches"] for k, v in pre.items() if k == "time_fwd") if "time_fwd" in pre else 0
    precond = None
    if pre_ms > 0 and "time_fwd" in pre:
        csz = 16.0 if opts["precision"] == "fp64" else 8.0
        per_member = 8.0 * 2 * cfg.n * cfg.m + csz * 2 * (cfg.n // 2 + 1) * cfg.m
        member_applies = pre["time_fwd"]["bytes"] / per_member
        precond = {"achieved_pass_bytes_GBs": round(pre_bytes / (pre_ms * 1e-3) / 1e9, 1),
                   "frac": round(pre_bytes / (pre_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "member_applies": round(member_applies, 2),
                   "ms_per_member_apply": pre_ms / member_applies,
                   "compulsory_GBs": round(32.0 * cfg.n * cfg.m * member_applies / (pre_ms * 1e-3) / 1e9, 1),
                   "pass_bytes_per_member_apply": pre_bytes / member_applies}
    kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3),
                   "GBs": round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1]["ms"])}
    iters = [i.iters for i in infos]
    out = {
        "metric": "KKT solves/s to 1e-8 rel. residual (FP64, eps-circulant RBD-preconditioned GMRES)",
        "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if opts["precision"] == "fp64" else "f64+f32",
        "data": "synthetic (seeded smooth sine products + N(0,1e-2) noise)",
        "config": {"workload": workload, "mass": args.mass, "dim": cfg.dim, "nx": cfg.nx, "nt": cfg.nt, "T": cfg.T,
                   "gammas": list(cfg.gammas), "eps": "sqrt(tau)" if cfg.eps is None else cfg.eps,
                   "precision": opts["precision"], "spatial": opts["spatial"], "krylov": f"{opts['side']} GMRES(30)",
                   "graph": opts["graph"], "preconditioner": args.precond,
                   "rtol": 1e-8, "batch": len(members), "global_batch": len(members)},
        "iters": iters, "relres_true": [i.relres_true for i in infos], "converged": ok,
        "kernel_table_source": "eager solve after the timed region" if opts["graph"] else "timed region",
        "roofline": roofline, "precond_apply": precond, "kernel_choice": s.kernels, "kernels": kernels,
    }
    if not args.no_cpu_baseline and cfg.spatial == "mg":
        out["cpu_baseline"] = {"value": None, "note": "the oracle's multigrid path is timed only for the DST workloads"}
    elif not args.no_cpu_baseline:
        print("# bench: cpu baseline", file=sys.stderr, flush=True)
        try:
            out["cpu_baseline"] = cpu_baseline(cfg, iters, args.cpu_sample_seconds, args.mass)
        except Exception as e:  # pragma: no cover
            out["cpu_baseline"] = {"error": repr(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
