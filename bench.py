"""Benchmark: cell-updates/s per RK stage of the GRMHD finite-volume step.

Workload: the 3D relativistic magnetised blast wave at 256^3 (FP64, SSPRK3,
MC + HLLE, CFL 0.4), inputs resident in HBM before the timed region.  One
"step" is the whole hot path: CFL time step + three RK stages, each stage
= stage kernel (reconstruction, fluxes, sources, RK combine) + primitive
recovery + ghost fill.  The timed steps are one gmunu_steps call (the CFL
maxima of each step after the first come from the previous step's last
recovery).

Prints one JSON line; the roofline object prices the stage kernel's
algorithmic bytes (ALG_BYTES) against the HBM peak.
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
FP64_PEAK_TFLOPS = 78.6
# Algorithmic HBM bytes of one RK stage per interior cell (the unavoidable
# traffic of a stage that keeps no primitives in memory): stage 1 reads q_n
# (8 doubles) and the metric (5) and writes q_1 (8); stages 2 and 3 also read
# q_n: 168, 232, 232 B, 211 B per cell-stage on average.  The roofline
# fraction of the stage kernel and of the whole step use these.
ALG_BYTES = {0: 21 * 8, 1: 29 * 8, 2: 29 * 8}
# The bytes this design's stage kernel itself must move per interior cell:
# it reads the primitives (8) that the separate recovery kernel wrote, the
# metric (5), q_n (8), q_s (8, stages after the first), and writes q_out (8).
STAGE_BYTES = {0: 29 * 8, 1: 37 * 8, 2: 37 * 8}


STAGE_SOURCES = ("paper_2012_07322_amd/csrc/gmunu.hip", "paper_2012_07322_amd/csrc/gmunu_tile.hpp",
                 "paper_2012_07322_amd/csrc/gmunu_dev.hpp", "paper_2012_07322_amd/csrc/gmunu_host.hpp",
                 "include/gmunu.h")


def stage_source_hash():
    """SHA-256 over the code (comments and blank space removed) of the
    sources the single-grid stage kernel is built from."""
    import hashlib
    import re

    h = hashlib.sha256()
    for f in STAGE_SOURCES:
        txt = open(os.path.join(ROOT, f)).read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", " ", txt)
        h.update(" ".join(txt.split()).encode())
    return h.hexdigest()


def kernel_counters():
    """The committed rocprofv3 counter record of the stage kernel on this
    workload (HBM bytes per launch, FP64 instruction counts), if the kernel
    sources are unchanged since it was taken (else None)."""

    path = os.path.join(ROOT, "profiles", "k_stage_blast3d_256_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if stage_source_hash() != rec.get("source_sha256"):
        return None
    return rec


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
    cells = n * n * slab
    sample = f"one SSPRK3 step (3 stages + CFL) of a {n}x{n}x{slab} slab through the blast centre"
    res = {}
    # the oracle as it is, single threaded; then the same source built with
    # OpenMP over its per-cell loops on every host core
    for omp in (False, True):
        oracle.use_openmp(omp)
        nth = oracle.threads()
        prc = pr.copy()
        q = oracle.prim2con(ps, prc, met)
        t0 = time.perf_counter()
        steps, _, _ = oracle.evolve(ps, q, prc, met, 0.4, 0.0, 1e30, nsteps=1)
        el = time.perf_counter() - t0
        res[omp] = {"value": cells * 3 * steps / el, "unit": "cell-updates/s", "cores": nth, "kind": "oracle",
                    "sample": f"{sample}, {el:.2f} s on {nth} host thread{'s' if nth > 1 else ''}"}
    oracle.use_openmp(False)
    out = dict(res[True])
    out["host_cpus"] = os.cpu_count()
    out["single_core"] = res[False]
    return out


def bench_star(nr=256, nth=128, steps=1000, cfl=0.4):
    """The static magnetised TOV star on a 2D spherical (r, theta) grid,
    Cowling (frozen metric), SSPRK3 steps: cell-updates/s per stage, the
    rest-mass drift, the angular momentum sum, recovery flags at the end."""
    import numpy as np
    import torch

    import oracle
    import paper_2012_07322_amd as gmu
    import workloads as W

    p, pr, met = W.magnetised_star_2d(nr, nth)
    dev = torch.device("cuda:0")
    g = gmu.Grid(p)
    prim = torch.from_numpy(pr).to(dev)
    metric = torch.from_numpy(met).to(dev)
    g.fill_ghosts(prim)
    qn = g.prim2con(prim, metric)
    g.c2p(qn, metric, prim)
    g.fill_ghosts(prim)
    qs = torch.zeros_like(qn)
    t = torch.zeros(1, dtype=torch.float64, device=dev)
    dt = torch.zeros_like(t)
    nf = torch.zeros(1, dtype=torch.int32, device=dev)
    fl = torch.zeros(g.shape, dtype=torch.uint8, device=dev)
    dV = oracle.interior(p, oracle.cell_volumes(p))
    q0 = oracle.interior(p, qn.cpu().numpy())
    m0 = float((q0[0] * dV).sum())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.step(qn, qs, prim, metric, cfl, 1e30, t, dt, fl, nf)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    q1 = oracle.interior(p, qn.cpu().numpy())
    f1 = oracle.interior(p, fl.cpu().numpy())
    m1 = float((q1[0] * dV).sum())
    cells = nr * nth
    flags = {name: int(((f1 & bit) != 0).sum()) for name, bit in
             (("atmo", 1), ("eps_clamp", 2), ("v_clamp", 4), ("fatal", 8 | 16 | 32 | 64))}
    g.close()
    return {"workload": f"magnetised TOV star, spherical {nr}x{nth}, Cowling", "steps": steps,
            "ms_per_step": ms / steps, "cell_updates_per_s": cells * 3 * steps / (ms * 1e-3),
            "t_end": float(t.item()), "rest_mass_drift": (m1 - m0) / m0,
            "angular_momentum_sum": float((q1[3] * dV).sum()), "flags_last_stage": flags,
            "nfatal": int(nf.item())}


def bench_fused(n=256, steps=10, cfl=0.4, seed=0):
    """The primitive recovery as its own kernel after each stage (what
    gmunu_step does) against the recovery done by the stage kernel itself
    in its epilogue (gmunu_rk_stage with separate input and output
    primitives, ping-ponged): per-kernel times and whole steps, same steps
    from the same initial data, results compared bit for bit."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    dev = torch.device("cuda:0")
    p, pr, met = W.blast_wave_3d(n, seed=seed)
    g = gmu.Grid(p)
    metric = torch.from_numpy(met).to(dev)
    res = {}
    finals = []
    for fused in (False, True):
        prim = torch.from_numpy(pr).to(dev)
        g.fill_ghosts(prim)
        qn = g.prim2con(prim, metric)
        g.c2p(qn, metric, prim)
        g.fill_ghosts(prim)
        qs = torch.zeros_like(qn)
        other = prim.clone() if fused else None  # edge ghosts (never filled) as in prim
        t = torch.zeros(1, dtype=torch.float64, device=dev)
        dt = torch.zeros_like(t)

        def one(prim, other):
            if not fused:
                g.step(qn, qs, prim, metric, cfl, 1e30, t, dt)
                return prim, other
            g.cfl_dt(prim, metric, cfl, 1e30, t, dt)
            g.rk_stage(0, dt, qn, qs, qs, prim, other, metric)
            g.rk_stage(1, dt, qn, qs, qs, other, prim, metric)
            g.rk_stage(2, dt, qn, qs, qn, prim, other, metric)
            t.add_(dt)
            return other, prim

        prim, other = one(prim, other)  # warm-up
        torch.cuda.synchronize()
        g.profile(True, max_launches=16 * steps + 16)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            prim, other = one(prim, other)
        e1.record()
        torch.cuda.synchronize()
        prof = g.profile_read()
        g.profile(False)
        res["fused" if fused else "separate"] = {
            "ms_per_step": e0.elapsed_time(e1) / steps,
            "stage_ms": prof["stage"][0] / max(prof["stage"][1], 1),
            "c2p_ms": prof["c2p"][0] / prof["c2p"][1] if prof["c2p"][1] else 0.0,
            "ghosts_ms": prof["ghosts"][0] / max(prof["ghosts"][1], 1)}
        finals.append((qn.cpu(), prim.cpu(), float(t.item())))
        del qn, qs, prim, other
        torch.cuda.empty_cache()
    g.close()
    res["bitwise_identical"] = bool(torch.equal(finals[0][0], finals[1][0]) and
                                    torch.equal(finals[0][1], finals[1][1]) and finals[0][2] == finals[1][2])
    res["step_speedup"] = res["separate"]["ms_per_step"] / res["fused"]["ms_per_step"]
    res["workload"] = f"blast3d_{n}, {steps} steps"
    return res


def bench_blocks(nblocks=3000, steps=5, cfl=0.4, seed=0, tune=True, single_n=192, classes=False):
    """Many AMR-style blocks (8^3, 16^3, 32^3 interiors, spherical and
    Cartesian, TOV-profile magnetised states), each its own simulation with
    its own time step, advanced (a) by the batched graph-captured step and
    (b) by one gmunu_step launch sequence per block; both from the same
    initial data, the results compared bit for bit."""
    import ctypes

    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    dev = torch.device("cuda:0")
    ps = W.amr_block_params(nblocks, seed=seed)
    star = W.tov_isotropic(1.28e-3)
    shapes = [gmu.state_shape(p) for p in ps]
    per = [[(8,) + s] * 6 + [(5,) + s] for s in shapes]
    ar = gmu.Arena(gmu.Arena.size_of([x for v in per for x in v]), device=dev)
    log(f"[blocks] {nblocks} blocks, {ar.buf.numel() * 8 / 2**30:.1f} GiB of state; generating")
    views = []
    for b, p in enumerate(ps):
        pr, met = W.amr_block_state(p, b, star, seed=seed)
        s = shapes[b]
        v = {k: ar.take((8,) + s) for k in ("qn_b", "qs_b", "pr_b", "qn_p", "qs_p", "pr_p")}
        v["met"] = ar.take((5,) + s)
        v["pr_b"].copy_(torch.from_numpy(pr))
        v["pr_p"].copy_(v["pr_b"])
        v["met"].copy_(torch.from_numpy(met))
        v["qs_b"].zero_()
        v["qs_p"].zero_()
        views.append(v)
    interior = sum(p["n"][0] * p["n"][1] * p["n"][2] for p in ps)
    with_ghosts = sum(s[0] * s[1] * s[2] for s in shapes)
    # (a) batched: one group per block
    B = gmu.Batch(nblocks, nblocks, 1 << 19)
    for b, p in enumerate(ps):
        v = views[b]
        B.set_block(b, p, v["qn_b"], v["qs_b"], v["pr_b"], v["met"], b)
        B.set_group(b, 0.0, 1e30)
    B.commit()
    B.init()
    tune_s = 0.0
    if tune:
        t0 = time.perf_counter()
        B.autotune()
        torch.cuda.synchronize()
        tune_s = time.perf_counter() - t0
    items, var = B.info()
    # the timed steps are one replay of a graph of `steps` steps
    # (gmunu_batch_steps: the CFL kernel in the first only); the warm-up
    # takes as many steps and captures that graph
    warmup = steps
    B.steps(cfl, steps)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    B.steps(cfl, steps)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    log(f"[blocks] batched: {ms_b / steps:.3f} ms/step (autotune {tune_s:.1f} s)")
    # (b) plain: one launch sequence per block (direct C-ABI calls)
    L = gmu.lib()
    grids = [gmu.Grid(p) for p in ps]
    tt = torch.zeros(nblocks, dtype=torch.float64, device=dev)
    dtt = torch.zeros(nblocks, dtype=torch.float64, device=dev)
    for b, g in enumerate(grids):
        v = views[b]
        g.fill_ghosts(v["pr_p"])
        q = g.prim2con(v["pr_p"], v["met"])
        v["qn_p"].copy_(q)
        g.c2p(v["qn_p"], v["met"], v["pr_p"])
        g.fill_ghosts(v["pr_p"])
    P = ctypes.c_void_p
    calls = []
    for b, g in enumerate(grids):
        v = views[b]
        calls.append((g._h, P(v["qn_p"].data_ptr()), P(v["qs_p"].data_ptr()), P(v["pr_p"].data_ptr()),
                      P(v["met"].data_ptr()), P(tt.data_ptr() + 8 * b), P(dtt.data_ptr() + 8 * b)))
    st = P(torch.cuda.current_stream().cuda_stream)

    def plain_step():
        for h, qn, qs, pr, met, tp, dtp in calls:
            rc = L.gmunu_step(h, qn, qs, pr, met, None, cfl, 1e30, tp, dtp, None, None, st)
            if rc:
                raise RuntimeError(f"gmunu_step failed ({rc})")

    for _ in range(warmup):
        plain_step()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        plain_step()
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    log(f"[blocks] plain: {ms_p / steps:.3f} ms/step")
    # identical results
    t_b, _ = B.times()
    same = bool((torch.from_numpy(t_b[:nblocks]).to(dev) == tt).all().item())
    for b, p in enumerate(ps):
        v = views[b]
        same = same and torch.equal(W.interior(p, v["qn_b"]), W.interior(p, v["qn_p"]))
        same = same and torch.equal(v["pr_b"], v["pr_p"])
    nvar = {}
    for x in var[:nblocks].tolist():
        nvar[x] = nvar.get(x, 0) + 1
    res = {
        "workload": f"amr_blocks_{nblocks}", "blocks": nblocks, "interior_cells": interior,
        "cells_with_ghosts": with_ghosts, "steps": steps, "warmup": warmup,
        "batched": {"value": interior * 3 * steps / (ms_b * 1e-3), "ms_per_step": ms_b / steps,
                    "graph": True, "autotune_s": tune_s, "tile_variants": nvar, "stage_items": int(items[0])},
        "plain": {"value": interior * 3 * steps / (ms_p * 1e-3), "ms_per_step": ms_p / steps,
                  "launches_per_step": 12 * nblocks},
        "unit": "cell-updates/s", "speedup": ms_p / ms_b, "bitwise_identical": same,
    }
    for g in grids:
        g.close()
    B.close()
    if classes:
        res["by_class"] = _blocks_by_class(ps, views, steps, cfl, tune)
    if single_n:
        res["same_physics_single_grid"] = _blocks_single_grid(ps, star, single_n, steps, cfl, dev)
        ref = res["same_physics_single_grid"]["value"]
        res["same_physics_single_grid"]["batched_over_single"] = res["batched"]["value"] / ref
        log(f"[blocks] single grid of the same physics: {ref:.3e} cell-updates/s; "
            f"batched / single = {res['batched']['value'] / ref:.3f}")
    return res


def _blocks_by_class(ps, views, steps, cfl, tune):
    """The batched rate of each (size, coordinates) class of blocks alone: a
    batch of only that class's blocks, restarted from their current state."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    out = {}
    for n in sorted({p["n"][0] for p in ps}):
        for coord, cname in ((W.CART, "cartesian"), (W.SPH, "spherical")):
            idx = [b for b, p in enumerate(ps) if p["n"][0] == n and p["coord"] == coord]
            if not idx:
                continue
            B = gmu.Batch(len(idx), len(idx), 1 << 19)
            for k, b in enumerate(idx):
                v = views[b]
                B.set_block(k, ps[b], v["qn_b"], v["qs_b"], v["pr_b"], v["met"], k)
                B.set_group(k, 0.0, 1e30)
            B.commit()
            B.init()
            if tune:
                B.autotune()
            B.steps(cfl, steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.steps(cfl, steps)
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / steps
            B.close()
            cells = sum(ps[b]["n"][0] * ps[b]["n"][1] * ps[b]["n"][2] for b in idx)
            out[f"{n}^3 {cname}"] = {"blocks": len(idx), "ms_per_step": sec * 1e3, "value": 3 * cells / sec}
            log(f"[blocks]   {n}^3 {cname}: {len(idx)} blocks, {3 * cells / sec:.3e} cell-updates/s")
    return out


def _time_single_grid(g, pr, met, cfl, steps):
    """Seconds for `steps` steps of one grid as one gmunu_steps call, after
    a warm-up run (initialisation and as many steps) outside the timing."""
    import torch

    qn, qs, _ = g.run(pr, met, cfl, 1e30, steps)
    t = torch.zeros(1, dtype=torch.float64, device=pr.device)
    dt = torch.zeros_like(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.steps(qn, qs, pr, met, cfl, 1e30, t, dt, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def _blocks_single_grid(ps, star, n, steps, cfl, dev):
    """The single-grid rate of the blocks' physics: one Cartesian and one
    spherical n^3 grid carrying the same TOV-profile state (curved metric,
    the same equation of state and atmosphere), gmunu_step per step; the
    rate for the block mix is the cell-weighted harmonic mean over the two
    coordinate systems."""
    import numpy as np
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    kw = {k: ps[0][k] for k in ("gamma", "rk", "rho_atmo", "k_atmo", "gamma_atmo", "rho_low_factor", "alpha_bh")}
    grids = {
        "cartesian": W.grid(3, W.CART, [n] * 3, [-12.8] * 3, [12.8] * 3, [[W.OUTFLOW, W.OUTFLOW]] * 3, **kw),
        "spherical": W.grid(3, W.SPH, [n] * 3, [0.5, 0.05, 0.0], [18.0, np.pi - 0.05, 2 * np.pi],
                            [[W.OUTFLOW, W.OUTFLOW]] * 3, **kw),
    }
    out = {"n": n, "steps": steps}
    for name, p in grids.items():
        pr, met = W.amr_block_state(p, 0, star)
        pr = torch.from_numpy(pr).to(dev)
        met = torch.from_numpy(met).to(dev)
        g = gmu.Grid(p)
        sec = _time_single_grid(g, pr, met, cfl, steps)
        g.close()
        out[name] = n ** 3 * 3 * steps / sec
    cells = {"cartesian": 0, "spherical": 0}
    for p in ps:
        cells["spherical" if p["coord"] == W.SPH else "cartesian"] += p["n"][0] * p["n"][1] * p["n"][2]
    tot = sum(cells.values())
    out["value"] = tot / sum(c / out[k] for k, c in cells.items() if c)
    out["unit"] = "cell-updates/s"
    return out


def bench_block_tiling(n=192, sizes=(32, 16, 8), steps=3, cfl=0.4, seed=0):
    """The same cells whole and in blocks: the blocks' TOV-profile state on
    an n^3 Cartesian and an n^3 spherical grid, advanced by gmunu_step, and
    the same domains cut into m^3 blocks (m in sizes, one group per block)
    advanced by the batched step.  Every block is a piece of the whole grid
    with its cells' own states, so the two rates differ only by what the
    blocks add (ghost layers per block, tile padding, work lists)."""
    import numpy as np
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    dev = torch.device("cuda:0")
    star = W.tov_isotropic(1.28e-3)
    kw = dict(gamma=2.0, rk=3, rho_atmo=1e-10, k_atmo=100.0, gamma_atmo=2.0, rho_low_factor=100.0, alpha_bh=1e-2)
    doms = {"cartesian": (W.CART, [-12.8] * 3, [12.8] * 3),
            "spherical": (W.SPH, [0.5, 0.05, 0.0], [18.0, np.pi - 0.05, 2 * np.pi])}
    bc = [[W.OUTFLOW, W.OUTFLOW]] * 3
    sizes = [m for m in sizes if n % m == 0]
    out = {"n": n, "steps": steps, "unit": "cell-updates/s"}
    for name, (coord, lo, hi) in doms.items():
        p = W.grid(3, coord, [n] * 3, lo, hi, bc, **kw)
        pr, met = W.amr_block_state(p, 0, star, seed=seed)
        pr = torch.from_numpy(pr).to(dev)
        met = torch.from_numpy(met).to(dev)
        g = gmu.Grid(p)
        whole = 3 * n ** 3 * steps / _time_single_grid(g, pr, met, cfl, steps)
        g.close()
        del pr, met
        res = {"single_grid": whole}
        h = [(hi[a] - lo[a]) / n for a in range(3)]
        for m in sizes:
            nb1 = n // m
            ps = []
            for k in range(nb1):
                for j in range(nb1):
                    for i in range(nb1):
                        x0 = [lo[a] + (i, j, k)[a] * m * h[a] for a in range(3)]
                        x1 = [lo[a] + ((i, j, k)[a] + 1) * m * h[a] for a in range(3)]
                        ps.append(W.grid(3, coord, [m] * 3, x0, x1, bc, **kw))
            shapes = [gmu.state_shape(q) for q in ps]
            ar = gmu.Arena(gmu.Arena.size_of([x for s in shapes for x in [(8,) + s] * 3 + [(5,) + s]]), device=dev)
            B = gmu.Batch(len(ps), len(ps), 1 << 20)
            for b, q in enumerate(ps):
                bpr, bmet = W.amr_block_state(q, b, star, seed=seed)
                s = shapes[b]
                qn, qs, prd = (ar.take((8,) + s) for _ in range(3))
                md = ar.take((5,) + s)
                prd.copy_(torch.from_numpy(bpr))
                md.copy_(torch.from_numpy(bmet))
                qs.zero_()
                B.set_block(b, q, qn, qs, prd, md, b)
                B.set_group(b, 0.0, 1e30)
            B.commit()
            B.init()
            B.autotune()
            B.steps(cfl, steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            B.steps(cfl, steps)
            torch.cuda.synchronize()
            rate = 3 * n ** 3 * steps / (time.perf_counter() - t0)
            B.close()
            del ar
            torch.cuda.empty_cache()
            res[f"{m}^3"] = {"blocks": len(ps), "value": rate, "over_single": rate / whole}
            log(f"[tiling] {name} {n}^3 as {len(ps)} blocks of {m}^3: {rate:.3e} cell-updates/s, "
                f"{rate / whole:.3f} of the whole grid ({whole:.3e})")
        out[name] = res
    return out


def _pct(xs, q):
    import numpy as np

    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _serve_cells(r, steps):
    return (r["n"] ** r["kind"]) * 3 * steps


def _drive_server(S, reqs, dev, offsets=None, concurrency=None):
    """Feed reqs to the server, inputs built on the device at arrival, and
    collect every result.  Open loop: request k arrives at start +
    offsets[k].  Closed loop: `concurrency` requests outstanding, the next
    one arriving when one completes."""
    import paper_2012_07322_amd as gmu
    import torch
    import workloads as W

    clock = gmu.Server.clock
    t0 = clock() + 0.02
    arrival, recs = {}, []
    i = 0

    def submit(k, at):
        p, pr, met, te, ms = W.serving_problem(reqs[k], dev)
        S.submit(p, pr, met, te, ms, prim_out=torch.empty_like(pr), tag=k)
        arrival[k] = at

    last_note = clock()
    while len(recs) < len(reqs):
        now = clock()
        if now - last_note > 20.0:
            log(f"[serve]   {len(recs)} of {len(reqs)} done")
            last_note = now
        if concurrency is None:
            while i < len(reqs) and t0 + offsets[i] <= now:
                submit(i, t0 + offsets[i])
                i += 1
                now = clock()
            wait = 50 if i >= len(reqs) else int(max(0.0, min(0.05, t0 + offsets[i] - clock())) * 1000)
        else:
            while i < len(reqs) and i - len(recs) < concurrency:
                submit(i, max(now, t0))
                i += 1
            wait = 50
        for r in S.poll(512, wait):
            k = r["tag"]
            if r["status"] != 0:
                raise RuntimeError(f"request {k} ended with status {r['status']}")
            recs.append({"k": k, "kind": reqs[k]["kind"], "lat": r["t_done"] - arrival[k],
                         "wait": r["t_admit"] - arrival[k], "done": r["t_done"], "steps": r["steps"],
                         "cells": _serve_cells(reqs[k], r["steps"])})
    return recs, t0


def _drive_plain(reqs, offsets, dev, cfl):
    """The plain loop: one solve at a time (gmunu_step launch sequence per
    step), in arrival order, each started no earlier than its arrival."""
    import paper_2012_07322_amd as gmu
    import torch
    import workloads as W

    clock = gmu.Server.clock
    t0 = clock() + 0.02
    recs, busy = [], 0.0
    last_note = clock()
    for k, r in enumerate(reqs):
        if clock() - last_note > 20.0:
            log(f"[serve]   plain: {k} of {len(reqs)} done")
            last_note = clock()
        arr = t0 + offsets[k]
        while clock() < arr:
            time.sleep(min(0.01, max(0.0, arr - clock())))
        s0 = clock()
        p, pr, met, te, ms = W.serving_problem(r, dev)
        g = gmu.Grid(p)
        qn, _, t = g.run(pr, met, cfl, te, ms)
        out = torch.empty_like(pr)
        out.copy_(pr)
        torch.cuda.synchronize()
        done = clock()
        g.close()
        busy += done - s0
        recs.append({"k": k, "kind": r["kind"], "lat": done - arr, "wait": s0 - arr, "done": done})
    return recs, t0, busy


def bench_serve(nreq=1000, probe=300, plain_n=300, plain_open=100, concurrency=64, load=0.8, seed=0,
                budget_gb=64.0, slots=512, spsync=2, cfl=0.4, rate=None):
    """Serving workload: independent 1D shock tubes (200-4096 cells, to
    t = 0.4) and 2D / 3D blast waves (64^2-1024^2, 32^3-128^3, 50 steps),
    Poisson arrivals.  (1) Capacity: the first `probe` requests with
    `concurrency` outstanding on the server, and the first `plain_n` one
    after another on the plain loop.  (2) Open loop at `load` x the server's
    capacity: p50 / p99 arrival-to-result latency of `nreq` requests on the
    server and of the first `plain_open` on the plain loop (same arrival
    times)."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    dev = torch.device("cuda:0")
    reqs = W.serving_requests(max(nreq, probe, plain_n, plain_open), seed=seed)
    S = gmu.Server(int(budget_gb * 2**30), max_slots=slots, cfl=cfl, steps_per_sync=spsync)
    # warm-up: one small and one large solve of each kind (graph capture)
    warm = [{"kind": k, "n": n, "seed": 7, "arrival": 0.0} for k, n in ((1, 200), (2, 64), (3, 32), (2, 512), (3, 64))]
    _drive_server(S, warm, dev, concurrency=8)

    def summary(recs, t0, busy=None):
        span = max(r["done"] for r in recs) - t0
        lat = [r["lat"] for r in recs]
        out = {"requests": len(recs), "makespan_s": span, "req_per_s": len(recs) / span,
               "p50_ms": 1e3 * _pct(lat, 50), "p99_ms": 1e3 * _pct(lat, 99), "mean_ms": 1e3 * sum(lat) / len(lat)}
        if "cells" in recs[0]:
            out["cell_updates_per_s"] = sum(r["cells"] for r in recs) / span
        if busy is not None:
            out["busy_req_per_s"] = len(recs) / busy
        out["by_dim"] = {str(d): {"n": sum(1 for r in recs if r["kind"] == d),
                                  "p50_ms": 1e3 * (_pct([r["lat"] for r in recs if r["kind"] == d], 50) or 0.0),
                                  "p99_ms": 1e3 * (_pct([r["lat"] for r in recs if r["kind"] == d], 99) or 0.0)}
                         for d in (1, 2, 3)}
        return out

    log(f"[serve] capacity: {probe} requests, {concurrency} outstanding")
    recs, t0 = _drive_server(S, reqs[:probe], dev, concurrency=concurrency)
    cap = summary(recs, t0)
    log(f"[serve]   server {cap['req_per_s']:.1f} req/s, {cap['cell_updates_per_s']:.3e} cell-updates/s")
    log(f"[serve] plain loop: first {plain_n} one after another")
    steps = {r["k"]: r["steps"] for r in recs}
    precs, pt0, pbusy = _drive_plain(reqs[:plain_n], [0.0] * plain_n, dev, cfl)
    if all(r["k"] in steps for r in precs):
        # same solves, same step counts (the results are identical)
        for r in precs:
            r["cells"] = _serve_cells(reqs[r["k"]], steps[r["k"]])
    cap_plain = summary(precs, pt0, pbusy)
    log(f"[serve]   plain {cap_plain['req_per_s']:.1f} req/s")
    if rate is None:
        rate = load * cap["req_per_s"]
    else:
        load = rate / cap["req_per_s"]
    offs = [r["arrival"] / rate for r in reqs[:nreq]]
    log(f"[serve] open loop: {nreq} requests at {rate:.1f} req/s ({load:.0%} of the server's capacity)")
    recs, t0 = _drive_server(S, reqs[:nreq], dev, offsets=offs)
    opn = summary(recs, t0)
    info = S.status()
    S.close()
    log(f"[serve]   p50 {opn['p50_ms']:.1f} ms, p99 {opn['p99_ms']:.1f} ms")
    log(f"[serve] plain loop, open loop: first {plain_open} at the same arrival times")
    precs, pt0, pbusy = _drive_plain(reqs[:plain_open], offs[:plain_open], dev, cfl)
    opn_plain = summary(precs, pt0, pbusy)
    sub = [r for r in recs if r["k"] < plain_open]
    opn_sub = {"p50_ms": 1e3 * _pct([r["lat"] for r in sub], 50), "p99_ms": 1e3 * _pct([r["lat"] for r in sub], 99)}
    log(f"[serve]   plain p50 {opn_plain['p50_ms']:.1f} ms, p99 {opn_plain['p99_ms']:.1f} ms "
        f"(server on the same requests: p50 {opn_sub['p50_ms']:.1f}, p99 {opn_sub['p99_ms']:.1f})")
    # plain capacity on exactly the requests of the server's probe
    same = min(probe, plain_n)
    return {
        "workload": "serving_poisson", "seed": seed, "budget_gib": budget_gb, "slots_per_lane": slots,
        "stream": ("the full 10,000-request stream" if nreq >= 10000 else
                   f"a sample: the first {nreq} requests of the 10,000-request stream"),
        "steps_per_sync": spsync, "cfl": cfl,
        "mix": "1D tube N in [200,4096] to t=0.4; 2D blast N^2, N in [64,1024]; 3D blast N^3, N in [32,128]; "
               "50 steps; dimension equally likely, N uniform",
        "capacity": {"server": cap, "plain": cap_plain, "same_requests": same == probe == plain_n,
                     "speedup": cap["req_per_s"] / cap_plain["req_per_s"]},
        "open_loop": {"load": load, "rate_req_per_s": rate, "server": opn, "server_first_n": opn_sub,
                      "plain_first_n": opn_plain},
        "server_info": {k: info[k] for k in ("replays", "pool_peak", "busy_s")},
    }


def bench_mg(n=256, half=200.0, vcycles=8, sweeps=10, coarse=10):
    """The metric-solver measurement of section 4: the lapse equation of a
    static TOV star on a Cartesian n^3 box [-half, half]^3, solved from the
    flat initial guess (alpha psi = 1) with V(2,2) red-black cycles.  Times
    one FAS full-multigrid cycle, V-cycles (each with its residual norm and
    host read-back), and smoothing sweeps of the finest level alone (the
    dominant kernel: algorithmic bytes per sweep 40 per cell = u read by
    both colours, f and a once, each cell written once; the timed call
    includes its one refresh of the colour-split copies of f and a)."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    log(f"[bench] multigrid: lapse equation on {n}^3")
    p, a_np = W.lapse_equation(n, half)
    p = dict(p, coarse=coarse)  # sweeps on the 2^3 coarsest level (one workgroup)
    M = gmu.Multigrid(p)
    a = torch.from_numpy(a_np).cuda()
    del a_np
    f = torch.zeros_like(a)
    u = torch.zeros_like(a)
    M.solve(u, f, a, tol=0.0, max_cycles=2)  # warm-up (code objects, caches)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    u.zero_()
    torch.cuda.synchronize()
    ev[0].record()
    h_fmg = M.solve(u, f, a, tol=0.0, max_cycles=1, fmg=True)
    ev[1].record()
    h_v = M.solve(u, f, a, tol=0.0, max_cycles=vcycles, fmg=False)
    ev[2].record()
    torch.cuda.synchronize()
    u.zero_()
    hist = M.solve(u, f, a, tol=1e-13, max_cycles=30, fmg=True)
    torch.cuda.synchronize()
    ev[3].record()
    M.smooth(u, f, a, sweeps=sweeps)
    ev[4].record()
    torch.cuda.synchronize()
    ms_fmg = ev[0].elapsed_time(ev[1])
    ms_v = ev[1].elapsed_time(ev[2]) / vcycles
    ms_sweep = ev[3].elapsed_time(ev[4]) / sweeps
    cells = n ** 3
    gbs = 40.0 * cells / (ms_sweep * 1e-3) / 1e9
    cyc = next((i for i, r in enumerate(hist) if r <= 1e-10 * hist[0]), None)
    out = {"workload": f"lapse equation of a static TOV star (K=100, Gamma=2, rho_c=1.28e-3), Cartesian {n}^3 on "
                       f"[-{half:g},{half:g}]^3, Dirichlet faces, flat initial guess",
           "levels": M.levels, "ms_per_fmg_cycle": ms_fmg, "ms_per_vcycle": ms_v,
           "residual_after_fmg": h_fmg[-1] / h_fmg[0], "vcycle_rate": (h_v[-1] / h_v[0]) ** (1.0 / vcycles),
           "residual_history": hist, "cycles_to_1e-10_relative": cyc,
           "smoother": {"ms_per_sweep": ms_sweep, "bytes_per_cell_sweep": 40, "achieved_GBps": gbs,
                        "peak_GBps": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}}
    log(f"[bench] multigrid: FMG {ms_fmg:.2f} ms, V-cycle {ms_v:.2f} ms, sweep {ms_sweep:.3f} ms ({gbs:.0f} GB/s), "
        f"{len(hist) - 1} cycles to {hist[-1]:.1e}")
    M.close()
    return out


def bench_xcfc(n=256, half=24.0, omega=0.01, sweeps=10, coarse=10):
    """The xCFC metric solve of section 2.6 (steps 1 to 6: X, psi, alpha psi,
    beta) for a uniformly rotating polytropic star on a Cartesian n^3 box,
    from the flat initial guess (psi = alpha = 1, beta = X = 0) to a residual
    of 1e-10 per equation; the conserved variables are those of the star on
    its TOV metric.  Also times sweeps of the vector smoother on the finest
    level (eight colour launches per sweep; algorithmic bytes 72 per cell:
    X read and written, f read, three components)."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    log(f"[bench] xCFC: rotating star on {n}^3")
    hp, pr, met = W.rotating_star_3d(n, half, omega)
    g = gmu.Grid(hp)
    prd = torch.from_numpy(pr).cuda()
    metd = torch.from_numpy(met).cuda()
    del pr
    q = g.prim2con(prd, metd)
    base = dict(ndim=3, coord=0, n=[n] * 3, xmin=[-half] * 3, dx=[2.0 * half / n] * 3, bc=[[0, 0]] * 3,
                coarse=coarse)
    rob = dict(base, bc=[[3, 3]] * 3)  # psi, alpha psi: u + x.grad u = 0 on the faces; X, beta: 0
    Mv = gmu.Multigrid(base)
    Mp = gmu.Multigrid(dict(rob, power=-1, power2=-7, offset=1.0))
    Ma = gmu.Multigrid(dict(rob, power=1, offset=1.0))
    X = Mv.empty(vector=True)
    flat = torch.from_numpy(W.flat_metric(hp)).cuda()
    tol = 1e-10
    metd.copy_(flat)
    gmu.xcfc_solve(Mv, Mp, Ma, hp, q, prd, metd, X, tol=tol, max_cycles=60)  # warm-up: code objects, graphs
    metd.copy_(flat)
    X.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc = gmu.xcfc_solve(Mv, Mp, Ma, hp, q, prd, metd, X, tol=tol, max_cycles=60)
    torch.cuda.synchronize()
    ms_solve = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    cyc_warm = gmu.xcfc_solve(Mv, Mp, Ma, hp, q, prd, metd, X, tol=tol, max_cycles=60)
    torch.cuda.synchronize()
    ms_warm = (time.perf_counter() - t0) * 1e3
    m = metd[:, 2:-2, 2:-2, 2:-2]
    shift = float(m[2:5].abs().max())
    f = torch.zeros_like(X)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    Mv.vsmooth(X, f, sweeps=sweeps)
    ev[1].record()
    torch.cuda.synchronize()
    ms_sweep = ev[0].elapsed_time(ev[1]) / sweeps
    gbs = 72.0 * n ** 3 / (ms_sweep * 1e-3) / 1e9
    out = {"workload": f"rotating polytropic star (K=100, Gamma=2, rho_c=1.28e-3, omega={omega:g}), Cartesian {n}^3 "
                       f"on [-{half:g},{half:g}]^3, Robin faces (psi, alpha psi) and Dirichlet faces (X, beta), flat initial guess",
           "tolerance": tol, "ms_per_solve": ms_solve, "cycles_X_psi_alphapsi_beta": list(cyc),
           "ms_per_warm_solve": ms_warm, "warm_cycles": list(cyc_warm),
           "psi_centre": float(m[0].max()), "alpha_centre": float(m[1].min()), "max_shift": shift,
           "vector_smoother": {"ms_per_sweep": ms_sweep, "bytes_per_cell_sweep": 72, "achieved_GBps": gbs,
                               "peak_GBps": HBM_PEAK_GBS, "frac": gbs / HBM_PEAK_GBS}}
    log(f"[bench] xCFC: solve {ms_solve:.1f} ms, cycles {cyc}, warm {ms_warm:.1f} ms {cyc_warm}, vector sweep "
        f"{ms_sweep:.3f} ms ({gbs:.0f} GB/s), max |beta| {shift:.2e}")
    for M in (Mv, Mp, Ma):
        M.close()
    return out


def bench_xcfc_sph(nr=640, nth=64, rmax=30.0, omega=0.02, tol=1e-6, smoother=1, sweeps=1, coarse=None):
    """The xCFC metric update (solve, then recovery on the new metric) of a
    uniformly rotating polytropic star on the layout of the paper's 2D
    rotating-star runs: spherical (r, theta) in [0, 30] x [0, pi/2] with
    640 x 64 cells, centre, polar axis and equator symmetry faces, Robin
    falloff for psi and alpha psi, X = beta = 0 at r = 30; from the flat
    metric, and again warm, to the paper's typical metric-solver tolerance
    (1e-6).  Smoother: line relaxation (1; V(1,1) cycles, 4 coarsest-level
    sweeps for psi and alpha psi, 2 for X and beta) or the paper's point
    smoother (0; V(4,4) and 50 recommended)."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    log(f"[bench] xCFC spherical: rotating star on {nr}x{nth}")
    hp, pr, met = W.rotating_star_sph2d(nr, nth, rmax, omega)
    g = gmu.Grid(hp)
    prd = torch.from_numpy(pr).cuda()
    metd = torch.from_numpy(met).cuda()
    q = g.prim2con(prd, metd)
    base = dict(ndim=2, coord=2, n=[nr, nth, 1], xmin=[0.0, 0.0, 0.0], dx=[rmax / nr, math.pi / 2 / nth, 1.0],
                pre=sweeps, post=sweeps, coarse=coarse or (4 if smoother else 50), smoother=smoother)
    # the vector equations' coarsest level (Dirichlet at r = 30) converges in fewer line sweeps
    Mv = gmu.Multigrid(dict(base, bc=[[1, 0], [1, 1], [1, 1]], coarse=coarse or (2 if smoother else 50)))
    Mp = gmu.Multigrid(dict(base, bc=[[1, 3], [1, 1], [1, 1]], power=-1, power2=-7, offset=1.0))
    Ma = gmu.Multigrid(dict(base, bc=[[1, 3], [1, 1], [1, 1]], power=1, offset=1.0))
    X = Mv.empty(vector=True)
    flat = torch.from_numpy(W.flat_metric(hp)).cuda()
    metd.copy_(flat)
    gmu.metric_update(g, Mp, Ma, q, prd, metd, mvec=Mv, X=X, tol=tol, max_cycles=2000)  # warm-up
    metd.copy_(flat)
    X.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc = gmu.metric_update(g, Mp, Ma, q, prd, metd, mvec=Mv, X=X, tol=tol, max_cycles=2000)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    cyc_w = gmu.metric_update(g, Mp, Ma, q, prd, metd, mvec=Mv, X=X, tol=tol, max_cycles=2000)
    torch.cuda.synchronize()
    ms_w = (time.perf_counter() - t0) * 1e3
    ng = hp["ng"]
    m = metd[:, 0, ng:ng + nth, ng:ng + nr]
    out = {"workload": f"uniformly rotating polytropic star (K=100, Gamma=2, rho_c=1.28e-3, omega={omega:g}), spherical "
                       f"{nr}x{nth} on [0,{rmax:g}]x[0,pi/2], centre/axis/equator symmetry, Robin falloff, flat "
                       f"initial metric",
           "smoother": "line" if smoother else "point", "sweeps": sweeps,
           "coarse_sweeps": {"vector": Mv.desc.coarse, "scalar": base["coarse"]},
           "tolerance": tol, "ms_per_update": ms, "cycles_X_psi_alphapsi_beta": list(cyc),
           "ms_per_warm_update": ms_w, "warm_cycles": list(cyc_w),
           "psi_centre": float(m[0].max()), "alpha_centre": float(m[1].min()),
           "min_beta_phi": float(m[4].min())}
    log(f"[bench] xCFC spherical: update {ms:.1f} ms, cycles {cyc}, warm {ms_w:.1f} ms {cyc_w}")
    for M in (Mv, Mp, Ma):
        M.close()
    g.close()
    return out


def bench_dynamical(n=256, half=24.0, omega=0.01, steps=100, every=50, eps=1e-3, tol=1e-6, cfl=0.4, coarse=10):
    """GRMHD evolution on a metric re-solved from the evolved matter
    (section 2.6; the Cowling approximation lifted): the rotating star of
    the xCFC leg on the same box, its xCFC metric first solved from the TOV
    metric (untimed), then `steps` SSPRK3 steps.  After each step the
    conformal-factor residual is checked, and the metric is re-solved when
    `every` steps have passed or the residual exceeds eps.  The solver
    tolerance is 1e-6, and Delta n = 50 as in the paper's typical range.
    The update is the xCFC solve, then the recovery on the new metric and
    the ghost fill.  The steps, the residual checks and the updates are
    timed separately; then the same evolution from the same state runs
    through evolve_dynamical (the steps between re-solves in device chunks)
    and is compared with the first bit for bit."""
    import torch

    import paper_2012_07322_amd as gmu
    import workloads as W

    log(f"[bench] dynamical metric: rotating star on {n}^3, {steps} steps, metric every {every}")
    hp, pr, met = W.rotating_star_3d(n, half, omega)
    g = gmu.Grid(hp)
    prd = torch.from_numpy(pr).cuda()
    metd = torch.from_numpy(met).cuda()
    del pr, met
    g.fill_ghosts(prd)
    q = g.prim2con(prd, metd)
    base = dict(ndim=3, coord=0, n=[n] * 3, xmin=[-half] * 3, dx=[2.0 * half / n] * 3, bc=[[0, 0]] * 3,
                coarse=coarse)
    rob = dict(base, bc=[[3, 3]] * 3)
    Mv = gmu.Multigrid(base)
    Mp = gmu.Multigrid(dict(rob, power=-1, power2=-7, offset=1.0))
    Ma = gmu.Multigrid(dict(rob, power=1, offset=1.0))
    X = Mv.empty(vector=True)
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    gmu.metric_update(g, Mp, Ma, q, prd, metd, mvec=Mv, X=X, nfatal=nf, tol=tol, max_cycles=200)
    qs = torch.zeros_like(q)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    # warm-up of the step and residual kernels (one step of the evolution)
    g.step(q, qs, prd, metd, cfl, 1e30, t, dt, None, nf)
    gmu.psi_residual(g, Mp, q, metd, Mv, X)
    torch.cuda.synchronize()
    start = [x.clone() for x in (q, qs, prd, metd, X, t, dt, nf)]
    t_step = t_res = t_upd = 0.0
    updates, since = [], 0
    for s in range(1, steps + 1):
        a0 = time.perf_counter()
        g.step(q, qs, prd, metd, cfl, 1e30, t, dt, None, nf)
        torch.cuda.synchronize()
        a1 = time.perf_counter()
        res = gmu.psi_residual(g, Mp, q, metd, Mv, X)
        a2 = time.perf_counter()
        t_step += a1 - a0
        t_res += a2 - a1
        since += 1
        if since >= every or res > eps:
            cyc = gmu.metric_update(g, Mp, Ma, q, prd, metd, mvec=Mv, X=X, nfatal=nf, tol=tol, max_cycles=200)
            torch.cuda.synchronize()
            t_upd += time.perf_counter() - a2
            updates.append({"after_step": s, "psi_residual": res, "cycles_X_psi_alphapsi_beta": list(cyc)})
            since = 0
    total = t_step + t_res + t_upd
    # the same evolution from the same state with the steps between
    # re-solves in device chunks (evolve_dynamical: the residual of every
    # step checked on the device, one host synchronisation per chunk)
    nfatal = int(nf.item())
    end = [x.clone() for x in (q, prd, metd, X, t)]
    for x, x0 in zip((q, qs, prd, metd, X, t, dt, nf), start):
        x.copy_(x0)
    del start
    torch.cuda.synchronize()
    a0 = time.perf_counter()
    upd_c = gmu.evolve_dynamical(g, q, qs, prd, metd, Mp, Ma, cfl, steps, every=every, eps=eps, mvec=Mv, X=X,
                                 t_dev=t, dt_dev=dt, nfatal=nf, tol=tol, max_cycles=200)
    torch.cuda.synchronize()
    total_c = time.perf_counter() - a0
    same = all(torch.equal(a, b) for a, b in zip(end, [q, prd, metd, X, t]))
    del end
    chunked = {"s_total": total_c, "updates_after_steps": upd_c,
               "same_updates": upd_c == [u["after_step"] for u in updates], "bitwise_equal": same,
               "nfatal": int(nf.item()),
               "cell_updates_per_s_with_metric": n ** 3 * 3 * steps / total_c}
    log(f"[bench] dynamical metric, device chunks: {total_c:.3f} s against {total:.3f} s per step on the host; "
        f"updates {upd_c}, bitwise equal {same}")
    out = {"workload": f"uniformly rotating polytropic star (K=100, Gamma=2, rho_c=1.28e-3, omega={omega:g}), "
                       f"Cartesian {n}^3 on [-{half:g},{half:g}]^3, xCFC metric re-solved every {every} steps or when "
                       f"the psi residual exceeds {eps:g} (tolerance {tol:g})",
           "steps": steps, "updates": updates, "ms_per_step": t_step / steps * 1e3,
           "ms_per_residual_check": t_res / steps * 1e3,
           "ms_per_metric_update": t_upd / max(len(updates), 1) * 1e3,
           "metric_share_of_time": (t_res + t_upd) / total,
           "cell_updates_per_s_with_metric": n ** 3 * 3 * steps / total, "nfatal": nfatal,
           "device_chunks": chunked}
    log(f"[bench] dynamical metric: {out['ms_per_step']:.2f} ms/step, residual check "
        f"{out['ms_per_residual_check']:.2f} ms, update {out['ms_per_metric_update']:.1f} ms, metric share "
        f"{out['metric_share_of_time']:.3f}")
    for M in (Mv, Mp, Ma):
        M.close()
    g.close()
    return out


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
    ap.add_argument("--fused-steps", type=int, default=10,
                    help="steps of the separate-vs-fused recovery comparison (0: skip)")
    ap.add_argument("--star-steps", type=int, default=1000,
                    help="steps of the 256x128 spherical star (0: skip)")
    ap.add_argument("--blocks", type=int, default=3000,
                    help="AMR-style blocks for the batched-vs-plain comparison (0: skip)")
    ap.add_argument("--block-steps", type=int, default=5)
    ap.add_argument("--block-classes", action="store_true",
                    help="also time the batch on each (size, coordinates) class of blocks alone")
    ap.add_argument("--block-tiling", type=int, default=0,
                    help="n: also compare an n^3 grid whole and cut into 32^3, 16^3, 8^3 blocks (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="open-loop requests for the serving measurement (0: skip)")
    ap.add_argument("--serve-probe", type=int, default=300)
    ap.add_argument("--serve-plain", type=int, default=300)
    ap.add_argument("--serve-plain-open", type=int, default=100)
    ap.add_argument("--serve-rate", type=float, default=None,
                    help="open-loop arrival rate in req/s (default: 80%% of the measured capacity)")
    ap.add_argument("--mg", type=int, default=256, help="multigrid grid size (0: skip)")
    ap.add_argument("--xcfc", type=int, default=256, help="xCFC metric-solve grid size (0: skip)")
    ap.add_argument("--dynamical", type=int, default=256,
                    help="grid size of the evolution with xCFC metric updates (0: skip)")
    ap.add_argument("--xcfc-sph", type=int, default=640,
                    help="radial cells of the spherical xCFC update (theta cells: a tenth; 0: skip)")
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
    if args.warmup > 0:
        g.steps(qn, qs, prim, metric, args.cfl, 1e30, t, dt, args.warmup, None, nf)
    torch.cuda.synchronize()
    g.profile(True, max_launches=16 * args.steps + 64)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    g.steps(qn, qs, prim, metric, args.cfl, 1e30, t, dt, args.steps, None, nf)
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
    alg_total = cells * sum(ALG_BYTES[s] for s in range(3)) * args.steps
    achieved = alg_total / (st_ms * 1e-3) / 1e9 if st_ms > 0 else None
    design_total = cells * sum(STAGE_BYTES[s] for s in range(3)) * args.steps
    design_gbs = design_total / (st_ms * 1e-3) / 1e9 if st_ms > 0 else None
    step_gbs = alg_total / (ms * 1e-3) / 1e9
    rec = kernel_counters() if n == 256 else None
    traffic = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"] if rec else None
    valu = None
    if rec and rec.get("fp64_flop_per_launch"):
        tf = rec["fp64_flop_per_launch"] / (st_ms / max(st_cnt, 1) * 1e-3) / 1e12
        valu = {"fp64_tflops": tf, "peak": FP64_PEAK_TFLOPS, "frac": tf / FP64_PEAK_TFLOPS,
                "valu_busy": rec.get("valu_busy"), "from": rec.get("from")}
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
                     "bytes_per_cell_stage": sum(ALG_BYTES.values()) / 3.0, "stage_ms_avg": st_ms / max(st_cnt, 1),
                     "step": {"achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS,
                              "bytes_per_cell_step": sum(ALG_BYTES.values())},
                     "design": {"bytes_per_cell_stage": sum(STAGE_BYTES.values()) / 3.0, "achieved": design_gbs,
                                "frac": (design_gbs / HBM_PEAK_GBS if design_gbs else None)},
                     "fp64_valu": valu},
        "breakdown": breakdown,
        "nfatal": nfatal,
    }
    del qn, qs, prim, metric
    g.close()
    torch.cuda.empty_cache()
    if args.fused_steps > 0:
        log(f"[bench] separate vs fused recovery, {args.fused_steps} steps")
        out["fused_c2p"] = bench_fused(n, args.fused_steps, cfl=args.cfl, seed=args.seed)
        torch.cuda.empty_cache()
    if args.star_steps > 0:
        log(f"[bench] star 256x128, {args.star_steps} steps")
        out["star2d"] = bench_star(256, 128, args.star_steps, cfl=args.cfl)
        torch.cuda.empty_cache()
    if args.blocks > 0:
        out["blocks"] = bench_blocks(args.blocks, steps=args.block_steps, cfl=args.cfl, seed=args.seed,
                                     classes=args.block_classes)
        torch.cuda.empty_cache()
    if args.block_tiling > 0:
        out["block_tiling"] = bench_block_tiling(args.block_tiling, steps=args.block_steps, cfl=args.cfl,
                                                 seed=args.seed)
        torch.cuda.empty_cache()
    if args.mg > 0:
        out["multigrid"] = bench_mg(args.mg)
        torch.cuda.empty_cache()
    if args.xcfc > 0:
        out["xcfc"] = bench_xcfc(args.xcfc)
        torch.cuda.empty_cache()
    if args.xcfc_sph > 0:
        out["xcfc_spherical"] = bench_xcfc_sph(args.xcfc_sph, max(8, args.xcfc_sph // 10))
        torch.cuda.empty_cache()
    if args.dynamical > 0:
        out["dynamical_metric"] = bench_dynamical(args.dynamical)
        torch.cuda.empty_cache()
    if args.serve_requests > 0:
        out["serving"] = bench_serve(args.serve_requests, probe=args.serve_probe, plain_n=args.serve_plain,
                                     plain_open=args.serve_plain_open, seed=args.seed, cfl=args.cfl,
                                     rate=args.serve_rate)
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on a {n}x{n}x{args.cpu_slab} slab")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_slab, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
