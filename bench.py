"""Benchmark: cell-updates/s per RK stage of the GRMHD finite-volume step.

Workload: the 3D relativistic magnetised blast wave at 256^3 (FP64, SSPRK3,
MC + HLLE, CFL 0.4), inputs resident in HBM before the timed region.  One
"step" is the whole hot path: CFL time step + three RK stages, each stage
= stage kernel (reconstruction, fluxes, sources, RK combine) + primitive
recovery + ghost fill.

Prints one JSON line (see the design doc for the roofline figures' derivation).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s per RK stage, FP64 256^3; p50/p99 latency, batched vs plain"
HBM_PEAK_GBS = 8000.0
# Algorithmic HBM bytes of the stage kernel per interior cell: reads prim (8),
# metric (5), q_n (8), q_s (8, stages after the first), writes q_out (8).
STAGE_BYTES = {0: 29 * 8, 1: 37 * 8, 2: 37 * 8}


def kernel_traffic():
    """HBM bytes per stage launch from the committed rocprofv3 counters, if
    the kernel sources are unchanged since they were taken (else None)."""
    import glob
    import hashlib

    path = os.path.join(ROOT, "profiles", "k_stage_blast3d_256_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2012_07322_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    if h.hexdigest() != rec.get("source_sha256"):
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n, slab, seed=0):
    """The oracle, as it is, on a slab of the same workload (n x n x slab
    cells through the blast centre, real neighbouring data in the z ghosts),
    one full SSPRK3 step on one host core."""
    import numpy as np

    import oracle
    import workloads as W

    p, _, _ = W.blast_wave_3d(n, seed=seed)
    k0 = n // 2 - slab // 2
    ps = dict(p)
    ps["n"] = [n, n, slab]
    ps["xmin"] = [p["xmin"][0], p["xmin"][1], p["xmin"][2] + k0 * p["dx"][2]]
    ps["bc"] = [list(p["bc"][0]), list(p["bc"][1]), [W.NONE, W.NONE]]
    # same cells as the full workload: pressure and field from the slab's
    # coordinates, density noise keyed by the full grid's global cell index
    pr = W.blast_prim(ps, seed=seed)
    g = W.ghosts(ps)
    kk = (np.arange(-g[2], slab + g[2]) + k0)[:, None, None]
    jj = (np.arange(-g[1], n + g[1]) % n)[None, :, None]
    ii = (np.arange(-g[0], n + g[0]) % n)[None, None, :]
    gidx = (ii + n * (jj + n * kk)).astype(np.int64)
    pr[0] = 0.01 * (1.0 + 1e-4 * W.uniform(seed, gidx))
    met = W.flat_metric(ps)
    oracle.fill_ghosts(ps, pr)
    q = oracle.prim2con(ps, pr, met)
    t0 = time.perf_counter()
    steps, _, _ = oracle.evolve(ps, q, pr, met, 0.4, 0.0, 1e30, nsteps=1)
    el = time.perf_counter() - t0
    cells = n * n * slab
    return {"value": cells * 3 * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"one SSPRK3 step (3 stages + CFL) of a {n}x{n}x{slab} slab through the blast centre, "
                      f"{el:.1f} s on 1 host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cfl", type=float, default=0.4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-slab", type=int, default=32)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is a design note, "
              f"not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    if args.calibrate_copy:
        nb = args.calibrate_copy << 20
        a = torch.ones(nb // 8, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nb, "copies": 3}), flush=True)
        return

    n = args.n
    log(f"[bench] building {n}^3 blast wave inputs")
    p, pr, met = W.blast_wave_3d(n, seed=args.seed)
    dev = torch.device("cuda:0")
    g = gmu.Grid(p)
    prim = torch.from_numpy(pr).to(dev)
    metric = torch.from_numpy(met).to(dev)
    del pr, met
    g.fill_ghosts(prim)
    qn = g.prim2con(prim, metric)
    g.c2p(qn, metric, prim)
    g.fill_ghosts(prim)
    qs = torch.zeros_like(qn)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    nf = torch.zeros(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        g.step(qn, qs, prim, metric, args.cfl, 1e30, t, dt, None, nf)
    torch.cuda.synchronize()
    g.profile(True, max_launches=16 * args.steps + 64)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.step(qn, qs, prim, metric, args.cfl, 1e30, t, dt, None, nf)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    prof = g.profile_read()
    g.profile(False)
    nfatal = int(nf.item())
    t_sim = float(t.item())
    log(f"[bench] timed {args.steps} steps: {ms:.2f} ms (wall {wall:.3f} s), t={t_sim:.6e}, nfatal={nfatal}")
    cells = n ** 3
    stages = 3 * args.steps
    value = cells * stages / (ms * 1e-3)
    st_ms, st_cnt = prof["stage"]
    bytes_total = cells * sum(STAGE_BYTES[s] for s in range(3)) * args.steps
    achieved = bytes_total / (st_ms * 1e-3) / 1e9 if st_ms > 0 else None
    traffic = kernel_traffic() if n == 256 else None
    breakdown = {k: {"ms_avg": (v[0] / v[1] if v[1] else None), "launches": v[1]} for k, v in prof.items()}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"blast3d_{n}", "cells": cells, "grid": [n, n, n], "ghosts": 2,
                   "stages_per_step": 3, "integrator": "SSPRK3", "recon": "MC", "riemann": "HLLE",
                   "cfl": args.cfl, "gamma": 4.0 / 3.0, "seed": args.seed},
        "roofline": {"bound": "hbm", "kernel": "k_stage", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": (achieved / HBM_PEAK_GBS if achieved else None), "traffic": traffic,
                     "bytes_per_cell_step": sum(STAGE_BYTES.values()), "stage_ms_avg": st_ms / max(st_cnt, 1)},
        "breakdown": breakdown,
        "nfatal": nfatal,
    }
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on a {n}x{n}x{args.cpu_slab} slab")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_slab, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
