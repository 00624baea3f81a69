"""Request server (gmunu_server_*) on the GPU.

Each solve in the server is advanced by the same per-cell arithmetic as the
same solve advanced alone with gmunu_step, so every served result must equal
the alone result bit for bit, whatever else shares the GPU with it, however
long it waited for memory, and whether its buffers are host or device.
"""
import sys
import time

import numpy as np
import pytest
import torch

import paper_2012_07322_amd as gmu
import workloads as W

pytestmark = pytest.mark.gpu


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mix():
    # small members of each kind of the serving workload (1D tubes run to
    # t = 0.4, 2D / 3D blasts 50 steps)
    spec = [(1, 64), (2, 24), (3, 12), (1, 200), (2, 40), (3, 16), (1, 120), (2, 32), (3, 10), (1, 96),
            (2, 20), (3, 14)]
    return [{"kind": k, "n": n, "seed": 11 + i, "arrival": 0.0} for i, (k, n) in enumerate(spec)]


def alone(p, pr, met, t_end, max_steps):
    g = gmu.Grid(p)
    prim = pr.clone()
    qn, _, t = g.run(prim, met, 0.4, t_end, max_steps)
    torch.cuda.synchronize()
    return qn, prim, t


def collect(S, n, limit_s=120.0):
    got = []
    t0 = time.time()
    while len(got) < n:
        got += S.poll(64, timeout_ms=500)
        assert time.time() - t0 < limit_s, f"only {len(got)} of {n} results"
    return got


def test_served_results_equal_alone_under_memory_pressure():
    reqs = mix()
    probs = [W.serving_problem(r, "cuda") for r in reqs]
    # an arena that holds only the two largest solves at once and four slots:
    # solves queue for memory and slots, and finish in a different order
    foot = sorted(W.serving_footprint(r) for r in reqs)
    budget = foot[-1] + foot[-2] + (1 << 16)
    S = gmu.Server(budget, max_slots=4, cfl=0.4, steps_per_sync=3)
    outs = []
    for k, (p, pr, met, te, ms) in enumerate(probs):
        q_out, p_out = torch.empty_like(pr), torch.empty_like(pr)
        S.submit(p, pr, met, te, ms, q_out=q_out, prim_out=p_out, tag=k)
        outs.append((q_out, p_out))
    res = collect(S, len(reqs))
    info = S.status()
    S.close()
    note(f"  pool peak {info['pool_peak']} of {info['pool_bytes']}, replays {info['replays']}")
    assert info["error"] == 0 and info["pool_peak"] <= info["pool_bytes"]
    by_tag = {r["tag"]: r for r in res}
    for k, (p, pr, met, te, ms) in enumerate(probs):
        r = by_tag[k]
        assert r["status"] == 0 and r["nfatal"] == 0, r
        qa, pa, ta = alone(p, pr, met, te, ms)
        assert r["t"] == ta, (k, r["t"], ta)
        if ms:
            assert r["steps"] == ms
        assert torch.equal(W.interior(p, qa), W.interior(p, outs[k][0])), f"request {k}: q differs"
        assert torch.equal(pa, outs[k][1]), f"request {k}: prim differs"
    # solves overlapped on the device, and some waited for memory or a slot
    spans = [(r["t_admit"], r["t_done"]) for r in res]
    overlap = any(a0 < b1 and b0 < a1 for i, (a0, a1) in enumerate(spans) for (b0, b1) in spans[i + 1:])
    assert overlap
    assert max(r["t_admit"] - r["t_submit"] for r in res) > 0.0
    for r in res:
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]


def test_every_lane_equal_alone():
    """Solves of both integrators and of every kind of lane (1D lines, small
    multi-dimensional solves, large ones above 65 536 interior cells) in
    one server: each lane is made on its first solve, and every result
    equals the same solve advanced alone bit for bit."""
    spec = [(1, 300, 3), (1, 200, 2), (2, 40, 3), (2, 40, 2), (3, 14, 2), (2, 272, 3), (2, 264, 2),
            (3, 12, 3), (1, 513, 2)]
    probs = []
    for i, (kind, n, rk) in enumerate(spec):
        p, pr, met, te, ms = W.serving_problem({"kind": kind, "n": n, "seed": 40 + i, "arrival": 0.0}, "cuda")
        p["rk"] = rk
        if kind > 1:
            ms = 6  # the large 2D solves stay short
        probs.append((p, pr, met, te, ms))
    S = gmu.Server(1 << 30, max_slots=8, cfl=0.4, steps_per_sync=2)
    outs = []
    for k, (p, pr, met, te, ms) in enumerate(probs):
        q_out, p_out = torch.empty_like(pr), torch.empty_like(pr)
        S.submit(p, pr, met, te, ms, q_out=q_out, prim_out=p_out, tag=k)
        outs.append((q_out, p_out))
    res = collect(S, len(probs))
    info = S.status()
    S.close()
    assert info["error"] == 0
    by_tag = {r["tag"]: r for r in res}
    for k, (p, pr, met, te, ms) in enumerate(probs):
        r = by_tag[k]
        assert r["status"] == 0 and r["nfatal"] == 0, r
        qa, pa, ta = alone(p, pr, met, te, ms)
        assert r["t"] == ta, (k, r["t"], ta)
        assert torch.equal(W.interior(p, qa), W.interior(p, outs[k][0])), f"request {k}: q differs"
        assert torch.equal(pa, outs[k][1]), f"request {k}: prim differs"


def test_host_buffers_and_late_arrivals():
    # inputs and outputs in host memory; a second wave submitted while the
    # first is running joins the running batch
    reqs = mix()[:6]
    S = gmu.Server(1 << 30, max_slots=16, cfl=0.4, steps_per_sync=2)
    probs, outs = [], []
    for k, r in enumerate(reqs):
        p, pr, met, te, ms = W.serving_problem(r, "cpu")
        probs.append((p, pr, met, te, ms))
        q_out, p_out = np.empty(tuple(pr.shape)), np.empty(tuple(pr.shape))
        outs.append((q_out, p_out))
        S.submit(p, pr.numpy(), met.numpy(), te, ms, q_out=q_out, prim_out=p_out, tag=k)
        if k == 2:
            time.sleep(0.05)
    res = collect(S, len(reqs))
    S.close()
    for r in res:
        k = r["tag"]
        p, pr, met, te, ms = probs[k]
        assert r["status"] == 0
        qa, pa, ta = alone(p, pr.cuda(), met.cuda(), te, ms)
        assert r["t"] == ta
        assert np.array_equal(W.interior(p, qa.cpu().numpy()), W.interior(p, outs[k][0]))
        assert np.array_equal(pa.cpu().numpy(), outs[k][1])


def test_request_larger_than_the_arena_is_rejected():
    S = gmu.Server(8 << 20, max_slots=4)
    p, pr, met, te, ms = W.serving_problem({"kind": 3, "n": 64, "seed": 1}, "cuda")
    with pytest.raises(RuntimeError):
        S.submit(p, pr, met, te, ms)
    # a small one still runs
    p, pr, met, te, ms = W.serving_problem({"kind": 2, "n": 16, "seed": 1}, "cuda")
    S.submit(p, pr, met, te, 5)
    res = collect(S, 1)
    S.close()
    assert res[0]["status"] == 0 and res[0]["steps"] == 5


def test_bad_request_among_good_ones():
    """A request with no valid end (t_end NaN or negative with a step limit,
    or +inf with none) is refused at submit; the good requests around it
    still complete, and the server keeps taking work."""
    S = gmu.Server(1 << 28, max_slots=4, cfl=0.4, steps_per_sync=2)
    good = []
    bad = [(float("nan"), 5), (-1.0, 5), (float("inf"), 0)]
    for k, r in enumerate(mix()[:4]):
        p, pr, met, te, ms = W.serving_problem(r, "cuda")
        S.submit(p, pr, met, te, ms or 0, tag=k)
        good.append(k)
        te_bad, ms_bad = bad[k % len(bad)]
        with pytest.raises(RuntimeError):
            S.submit(p, pr, met, te_bad, ms_bad, tag=100 + k)
    res = collect(S, len(good))
    info = S.status()
    assert info["error"] == 0
    assert sorted(r["tag"] for r in res) == good
    assert all(r["status"] == 0 for r in res)
    # still taking work
    p, pr, met, _, _ = W.serving_problem({"kind": 2, "n": 16, "seed": 3}, "cuda")
    S.submit(p, pr, met, float("inf"), 3, tag=7)
    res = collect(S, 1)
    S.close()
    assert res[0]["status"] == 0 and res[0]["steps"] == 3


def test_served_results_against_the_oracle():
    """One request of each kind, served in a mix, against the CPU oracle
    advancing the same initial data: the 1D tube to t = 0.4 and the 2D and 3D
    blasts for their 50 steps.  Volume-weighted relative L1 per conserved
    variable <= 1e-9 (variables identically zero in the oracle must be zero),
    identical step counts and final times to 1e-12."""
    import oracle

    reqs = [{"kind": 1, "n": 256, "seed": 21}, {"kind": 2, "n": 48, "seed": 22}, {"kind": 3, "n": 24, "seed": 23}]
    probs = [W.serving_problem(r, "cuda") for r in reqs]
    S = gmu.Server(1 << 30, max_slots=8, cfl=0.4, steps_per_sync=2)
    outs = []
    for k, (p, pr, met, te, ms) in enumerate(probs):
        q_out = torch.empty_like(pr)
        S.submit(p, pr, met, te, ms, q_out=q_out, tag=k)
        outs.append(q_out)
    res = {r["tag"]: r for r in collect(S, len(reqs))}
    S.close()
    for k, (p, pr, met, te, ms) in enumerate(probs):
        r = res[k]
        assert r["status"] == 0 and r["nfatal"] == 0
        pro = pr.cpu().numpy().copy()
        meto = met.cpu().numpy()
        oracle.fill_ghosts(p, pro)
        qo = oracle.prim2con(p, pro, meto)
        qo, pro, _, _ = oracle.c2p(p, qo, meto)
        oracle.fill_ghosts(p, pro)
        steps, t_o, nf = oracle.evolve(p, qo, pro, meto, 0.4, 0.0, te, ms if ms else 100000)
        qg = outs[k].cpu().numpy()
        dV = oracle.interior(p, oracle.cell_volumes(p))
        A, B = oracle.interior(p, qg), oracle.interior(p, qo)
        e = []
        for v in range(8):
            den = (np.abs(B[v]) * dV).sum()
            if den == 0.0:
                assert np.all(A[v] == 0.0), (k, v)
                e.append(0.0)
            else:
                e.append((np.abs(A[v] - B[v]) * dV).sum() / den)
        note(f"  kind {reqs[k]['kind']} n {reqs[k]['n']}: steps served {r['steps']} oracle {steps}, "
             f"t {r['t']:.15g} / {t_o:.15g}, L1 rel {np.array2string(np.array(e), precision=2)}")
        assert r["steps"] == steps and nf == 0
        assert abs(r["t"] - t_o) <= 1e-12 * max(t_o, 1e-300)
        assert max(e) <= 1e-9
