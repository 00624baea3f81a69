"""Batched stage (gmunu_batch_*) on the GPU.

A block advanced inside a batch runs the single-grid per-cell arithmetic on
the same inputs, so it must equal the block advanced alone bit for bit
(whatever tile shape the autotuner picks); a group of blocks sharing one
time step is checked against the oracle advanced with that step.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2012_07322_amd as gmu
import workloads as W

pytestmark = pytest.mark.gpu

STAR = None


def star():
    global STAR
    if STAR is None:
        STAR = W.tov_isotropic(1.28e-3)
    return STAR


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def mixed_blocks(nb=12, seed=3, **kw):
    ps = W.amr_block_params(nb, seed=seed, sizes=(8, 16), **kw)
    out = []
    for b, p in enumerate(ps):
        pr, met = W.amr_block_state(p, b, star(), seed=seed)
        out.append((p, pr, met))
    return out


def blast_like_blocks():
    """1D, 2D and 3D Cartesian blocks with flat metric (serving-style mix)."""
    out = []
    p, pr, met = W.mhd_shock_tube(300)
    out.append((p, pr, met))
    p, pr, met = W.blast_wave_2d(48)
    out.append((p, pr, met))
    p, pr, met = W.blast_wave_3d(20)
    out.append((p, pr, met))
    return out


def alone(p, pr, met, nsteps, cfl=0.4, t_end=1e30):
    g = gmu.Grid(p)
    prd, metd = torch.from_numpy(pr.copy()).cuda(), torch.from_numpy(met).cuda()
    g.fill_ghosts(prd)
    qn = g.prim2con(prd, metd)
    g.c2p(qn, metd, prd)
    g.fill_ghosts(prd)
    qs = torch.zeros_like(qn)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros_like(t)
    for _ in range(nsteps):
        g.step(qn, qs, prd, metd, cfl, t_end, t, dt)
    torch.cuda.synchronize()
    return qn.cpu().numpy(), prd.cpu().numpy(), float(t.item())


def make_batch(blocks, groups, max_groups=None, t_end=1e30):
    shapes = []
    for p, _, _ in blocks:
        s = gmu.state_shape(p)
        shapes += [(8,) + s] * 3 + [(5,) + s]
    ar = gmu.Arena(gmu.Arena.size_of(shapes))
    B = gmu.Batch(len(blocks) + 2, max_groups or (max(groups) + 1), 1 << 16)
    views = []
    for slot, ((p, pr, met), grp) in enumerate(zip(blocks, groups)):
        s = gmu.state_shape(p)
        qn, qs, prim, m = ar.take((8,) + s), ar.take((8,) + s), ar.take((8,) + s), ar.take((5,) + s)
        prim.copy_(torch.from_numpy(pr))
        m.copy_(torch.from_numpy(met))
        qs.zero_()
        B.set_block(slot, p, qn, qs, prim, m, grp)
        views.append((qn, prim))
    for g in sorted(set(groups)):
        B.set_group(g, 0.0, t_end)
    B.commit()
    B.init()
    return B, views, ar


@pytest.mark.parametrize("tune,graph", [(False, True), (True, True), (True, False)])
def test_batch_equals_each_block_alone(tune, graph):
    blocks = mixed_blocks(10) + blast_like_blocks()
    groups = list(range(len(blocks)))
    B, views, _ = make_batch(blocks, groups)
    if tune:
        B.autotune()
        items, var = B.info()
        note(f"  tuned variants {var[:len(blocks)].tolist()} items {items.tolist()}")
    nst = 3
    for _ in range(nst):
        B.step(0.4, use_graph=graph)
    torch.cuda.synchronize()
    t_b, _ = B.times()
    for slot, (p, pr, met) in enumerate(blocks):
        qa, pa, ta = alone(p, pr, met, nst)
        qb, pb = views[slot][0].cpu().numpy(), views[slot][1].cpu().numpy()
        assert t_b[slot] == ta
        assert np.array_equal(W.interior(p, qa), W.interior(p, qb)), f"block {slot} q differs"
        assert np.array_equal(pa, pb), f"block {slot} prim differs"


def _tube(n, bc_lo, bc_hi):
    p, pr, met = W.mhd_shock_tube(n)
    p["bc"] = [[bc_lo, bc_hi]] + [list(b) for b in p["bc"][1:]]
    if W.PERIODIC in (bc_lo, bc_hi):
        p["bc"][0] = [W.PERIODIC, W.PERIODIC]
    return p, pr, met


def _xbc_block(n, bc_lo, bc_hi, seed=0):
    """A Cartesian block of extents n with the given x faces (outflow on the
    other axes) and a smooth state with a non-zero shift."""
    nd = len(n)
    lo, hi = [-0.4, -0.3, -0.2], [0.5, 0.6, 0.7]
    if W.PERIODIC in (bc_lo, bc_hi):
        bc_lo = bc_hi = W.PERIODIC
    bc = [[bc_lo, bc_hi]] + [[W.OUTFLOW, W.OUTFLOW]] * (nd - 1)
    hi = [hi[a] if a < nd else lo[a] + 1.0 for a in range(3)]
    p = W.grid(nd, W.CART, list(n), lo, hi, bc, gamma=5.0 / 3.0, rk=3, rho_atmo=1e-12, k_atmo=1.0,
               gamma_atmo=5.0 / 3.0)
    from test_gpu_parity import smooth_random_state

    pr, met = smooth_random_state(p, seed=seed, beta_amp=0.02)
    return p, pr, met


def test_x_ghosts_filled_by_the_recovery_equal_alone():
    """Blocks whose x-face ghosts the recovery kernel writes from the
    recovered cells (periodic, outflow and reflecting x faces, rows of at
    least ng cells: 1D lines, and 2D and 3D blocks with rows of 2, 3, 8, 24,
    255 cells and more), and blocks whose x ghosts stay with the ghost kernel
    (rows shorter than ng), all bitwise equal to the same grid advanced alone
    after several steps."""
    blocks = [_tube(300, W.OUTFLOW, W.OUTFLOW), _tube(300, W.REFLECT, W.OUTFLOW), _tube(300, W.OUTFLOW, W.REFLECT),
              _tube(512, W.PERIODIC, W.PERIODIC), _tube(257, W.OUTFLOW, W.REFLECT), _tube(257, W.PERIODIC, W.PERIODIC),
              _tube(200, W.REFLECT, W.REFLECT), _tube(64, W.OUTFLOW, W.OUTFLOW), _tube(1, W.OUTFLOW, W.OUTFLOW),
              _tube(2, W.REFLECT, W.REFLECT), _tube(3, W.PERIODIC, W.PERIODIC)]
    p2, pr2, met2 = W.blast_wave_2d(32)
    blocks.append((p2, pr2, met2))
    for k, (n, lo, hi) in enumerate([((24, 10), W.PERIODIC, W.PERIODIC), ((8, 12), W.REFLECT, W.OUTFLOW),
                                     ((2, 9), W.REFLECT, W.REFLECT), ((3, 7), W.PERIODIC, W.PERIODIC),
                                     ((1, 16), W.OUTFLOW, W.OUTFLOW), ((255, 3), W.OUTFLOW, W.REFLECT),
                                     ((8, 6, 5), W.OUTFLOW, W.REFLECT), ((24, 4, 3), W.PERIODIC, W.PERIODIC),
                                     ((2, 5, 4), W.REFLECT, W.OUTFLOW), ((1, 4, 4), W.OUTFLOW, W.OUTFLOW)]):
        blocks.append(_xbc_block(n, lo, hi, seed=k))
    blocks += mixed_blocks(4, seed=5)
    groups = list(range(len(blocks)))
    B, views, _ = make_batch(blocks, groups)
    items, _ = B.info()
    note(f"  ghost items of the step: {int(items[2])}")
    nst = 4
    for _ in range(nst):
        B.step(0.4)
    torch.cuda.synchronize()
    t_b, _ = B.times()
    for slot, (p, pr, met) in enumerate(blocks):
        qa, pa, ta = alone(p, pr, met, nst)
        qb, pb = views[slot][0].cpu().numpy(), views[slot][1].cpu().numpy()
        assert t_b[slot] == ta, slot
        assert np.array_equal(W.interior(p, qa), W.interior(p, qb)), f"block {slot} q differs"
        assert np.array_equal(pa, pb), f"block {slot} prim differs"


# every compiled tile shape of the batched stage: (ndim, reconstruction,
# (tx, ty, tz)), in the order of the library's variant table
TILES = [(3, 0, (8, 8, 3)), (3, 0, (8, 5, 5)), (3, 0, (16, 4, 3)), (3, 0, (8, 6, 4)), (2, 0, (16, 15, 1)),
         (2, 0, (32, 7, 1)), (2, 0, (8, 28, 1)), (1, 0, (255, 1, 1)), (3, 1, (8, 5, 5)), (2, 1, (16, 15, 1)),
         (1, 1, (255, 1, 1)), (3, 2, (8, 5, 5)), (2, 2, (16, 15, 1)), (1, 2, (255, 1, 1))]


@pytest.mark.parametrize("k", range(len(TILES)), ids=[f"{t[0]}d-rec{t[1]}-{'x'.join(map(str, t[2]))}" for t in TILES])
def test_every_tile_shape_equals_alone(k):
    """Each compiled tile shape pinned with gmunu_batch_set_tile (those that
    stage the metric on a one-cell halo among them) on ragged blocks of its
    dimension and reconstruction: bitwise equal to the blocks advanced
    alone after three steps."""
    from test_gpu_parity import smooth_random_state

    nd, rec, tile = TILES[k]
    shapes = {3: [(13, 11, 9), (8, 8, 8), (17, 5, 7)], 2: [(40, 33), (17, 60)], 1: [(300,), (511,)]}[nd]
    blocks = []
    for m, n in enumerate(shapes):
        lo, hi = [-0.4, -0.3, -0.2], [0.5, 0.6, 0.7]
        hi = [hi[a] if a < nd else lo[a] + 1.0 for a in range(3)]
        p = W.grid(nd, W.CART, list(n), lo, hi, [[W.OUTFLOW, W.OUTFLOW]] * nd, gamma=5.0 / 3.0, rk=3,
                   rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=5.0 / 3.0, ng=2 if rec == 0 else 3, recon=rec,
                   riemann=m % 2)
        pr, met = smooth_random_state(p, seed=m, beta_amp=0.02)
        blocks.append((p, pr, met))
    B, views, _ = make_batch(blocks, list(range(len(blocks))))
    for p, _, _ in blocks:
        B.set_tile(p, *tile)
    B.commit()
    _, var = B.info()
    assert var[:len(blocks)].tolist() == [k] * len(blocks)
    for _ in range(3):
        B.step(0.4)
    torch.cuda.synchronize()
    t_b, _ = B.times()
    for slot, (p, pr, met) in enumerate(blocks):
        qa, pa, ta = alone(p, pr, met, 3)
        qb, pb = views[slot][0].cpu().numpy(), views[slot][1].cpu().numpy()
        assert t_b[slot] == ta, slot
        assert np.array_equal(W.interior(p, qa), W.interior(p, qb)), f"block {slot} q differs"
        assert np.array_equal(pa, pb), f"block {slot} prim differs"


def test_multi_step_replay_equals_single_steps():
    """gmunu_batch_steps (several steps from one graph, the CFL maxima of
    each later step from the previous step's last recovery) equals the same
    number of gmunu_batch_step calls bit for bit, with groups that reach
    their end time or step limit inside the replay."""
    blocks = mixed_blocks(6, seed=9) + blast_like_blocks()
    groups = list(range(len(blocks)))
    outs = []
    for multi in (False, True):
        B, views, ar = make_batch(blocks, groups)
        B.set_group(1, 0.0, 1e30, max_steps=3)
        B.set_group(2, 0.0, 2e-3)
        B.commit()
        if multi:
            B.steps(0.4, 5)
            B.steps(0.4, 2)
        else:
            for _ in range(7):
                B.step(0.4)
        torch.cuda.synchronize()
        t, dt, ns, _ = B.times(with_steps=True)
        outs.append((t[:len(blocks)].copy(), ns[:len(blocks)].copy(),
                     [(v[0].cpu().numpy(), v[1].cpu().numpy()) for v in views]))
        B.close()
        del ar
    (t0, n0, s0), (t1, n1, s1) = outs
    assert np.array_equal(t0, t1) and np.array_equal(n0, n1)
    assert n0[1] == 3 and t0[2] == 2e-3
    for slot, (p, _, _) in enumerate(blocks):
        assert np.array_equal(W.interior(p, s0[slot][0]), W.interior(p, s1[slot][0])), slot
        assert np.array_equal(s0[slot][1], s1[slot][1]), slot


def test_batch_shared_dt_group_against_oracle():
    # blocks inside the star (density far above the atmosphere floor, where
    # the atmosphere threshold cannot flip between the two implementations)
    blocks = mixed_blocks(6, seed=5, r_range=(0.5, 5.0), box=2.5)
    for p, pr, _ in blocks:
        assert W.interior(p, pr)[0].min() > 1e4 * p["rho_atmo"]
    B, views, _ = make_batch(blocks, [0] * len(blocks))
    B.step(0.4)
    torch.cuda.synchronize()
    t, dt = B.times()
    dts = [oracle.cfl_dt(p, oracle.fill_ghosts(p, pr.copy()), met, 0.4) for p, pr, met in blocks]
    note(f"  shared dt {dt[0]:.15e} oracle min {min(dts):.15e}")
    assert abs(dt[0] - min(dts)) <= 1e-13 * min(dts)
    assert t[0] == dt[0]
    for slot in (0, 3, 5):
        p, pr, met = blocks[slot]
        po = pr.copy()
        oracle.fill_ghosts(p, po)
        q0 = oracle.prim2con(p, po, met)
        q0, po, _, _ = oracle.c2p(p, q0, met)
        oracle.fill_ghosts(p, po)
        qs = q0.copy()
        for s in range(3):
            oracle.rk_stage(p, s, dt[0], q0, qs, po, met)
            if s == 2:
                q0 = qs.copy()
        qb = views[slot][0].cpu().numpy()
        A, Bq = W.interior(p, qb), W.interior(p, q0)
        for v in range(8):
            den = np.abs(Bq[v]).max()
            if den > 0:
                assert np.abs(A[v] - Bq[v]).max() <= 1e-11 * den, (slot, v)



def _oracle_init(p, pr, met):
    po = pr.copy()
    oracle.fill_ghosts(p, po)
    q0 = oracle.prim2con(p, po, met)
    q0, po, _, _ = oracle.c2p(p, q0, met)
    oracle.fill_ghosts(p, po)
    return q0, po


def _l1_rel(p, a, b):
    dV = oracle.interior(p, oracle.cell_volumes(p))
    A, B = W.interior(p, a), W.interior(p, b)
    out = []
    for v in range(8):
        den = (np.abs(B[v]) * dV).sum()
        out.append((np.abs(A[v] - B[v]) * dV).sum() / den if den > 0 else np.abs(A[v]).max())
    return np.array(out)


def test_batch_multistep_against_oracle():
    """Spherical and Cartesian 8^3 / 16^3 blocks inside the star, advanced by
    the batch (a) ten steps with each block in its own group (its own dt) and
    (b) five steps as one group sharing the minimum dt, against the oracle
    advancing the same blocks (in (b) with the group's minimum of the oracle's
    per-block dt each step): final times to 1e-12, volume-weighted relative L1
    per conserved variable <= 1e-9."""
    blocks = mixed_blocks(8, seed=5, r_range=(0.5, 5.0), box=2.5)
    coords = {p["coord"] for p, _, _ in blocks}
    assert coords == {W.CART, W.SPH}, coords
    for p, pr, _ in blocks:
        assert W.interior(p, pr)[0].min() > 1e4 * p["rho_atmo"]
    # (a) own groups
    B, views, _ = make_batch(blocks, list(range(len(blocks))))
    for _ in range(10):
        B.step(0.4)
    torch.cuda.synchronize()
    t, _ = B.times()
    worst = 0.0
    for slot, (p, pr, met) in enumerate(blocks):
        q0, po = _oracle_init(p, pr, met)
        steps, to, nf = oracle.evolve(p, q0, po, met, 0.4, 0.0, 1e30, 10)
        assert steps == 10 and nf == 0
        assert abs(t[slot] - to) <= 1e-12 * to, (slot, t[slot], to)
        e = _l1_rel(p, views[slot][0].cpu().numpy(), q0)
        worst = max(worst, e.max())
        assert e.max() <= 1e-9, (slot, e)
    note(f"  own groups, 10 steps: worst L1 rel {worst:.2e}")
    # (b) one shared-dt group
    B, views, _ = make_batch(blocks, [0] * len(blocks))
    for _ in range(5):
        B.step(0.4)
    torch.cuda.synchronize()
    t, _ = B.times()
    st = [_oracle_init(p, pr, met) for p, pr, met in blocks]
    to = 0.0
    for _ in range(5):
        dtg = min(oracle.cfl_dt(p, st[b][1], met, 0.4) for b, (p, _, met) in enumerate(blocks))
        for b, (p, _, met) in enumerate(blocks):
            q0, po = st[b]
            qs = q0.copy()
            for s in range(3):
                assert oracle.rk_stage(p, s, dtg, q0, qs, po, met) == 0
            st[b] = (qs.copy(), po)
        to += dtg
    assert abs(t[0] - to) <= 1e-12 * to, (t[0], to)
    worst = 0.0
    for b, (p, _, _) in enumerate(blocks):
        e = _l1_rel(p, views[b][0].cpu().numpy(), st[b][0])
        worst = max(worst, e.max())
        assert e.max() <= 1e-9, (b, e)
    note(f"  shared dt, 5 steps: worst L1 rel {worst:.2e}")

def test_finished_group_left_untouched():
    blocks = blast_like_blocks()
    B, views, _ = make_batch(blocks, [0, 1, 2])
    B.set_group(1, 0.5, 0.5)  # block 1 has reached its end time
    B.commit()
    before = [v[0].clone() for v in views]
    B.step(0.4)
    B.step(0.4)
    torch.cuda.synchronize()
    t, dt = B.times()
    assert dt[1] == 0.0 and t[1] == 0.5
    assert torch.equal(before[1], views[1][0])
    assert not torch.equal(before[0], views[0][0])


def test_slots_change_between_graph_replays():
    blocks = blast_like_blocks()
    B, views, ar = make_batch(blocks, [0, 1, 2], max_groups=4)
    B.step(0.4)
    # replace block 1 by a new 2D blast of a different seed in group 3
    p, pr, met = W.blast_wave_2d(48, seed=9)
    s = gmu.state_shape(p)
    ar2 = gmu.Arena(gmu.Arena.size_of([(8,) + s] * 3 + [(5,) + s]))
    qn, qs, prim, m = ar2.take((8,) + s), ar2.take((8,) + s), ar2.take((8,) + s), ar2.take((5,) + s)
    prim.copy_(torch.from_numpy(pr))
    m.copy_(torch.from_numpy(met))
    B.clear_block(1)
    B.set_block(1, p, qn, qs, prim, m, 3)
    B.set_group(3, 0.0, 1e30)
    B.commit()
    B.init([1])
    B.step(0.4)
    B.step(0.4)
    torch.cuda.synchronize()
    qa, pa, ta = alone(p, pr, met, 2)
    assert np.array_equal(W.interior(p, qa), W.interior(p, qn.cpu().numpy()))
    t, _ = B.times()
    assert t[3] == ta
    # the blocks that kept running were not re-initialised: they match three
    # uninterrupted steps alone
    for slot in (0, 2):
        pb, prb, metb = blast_like_blocks()[slot]
        qa, _, _ = alone(pb, prb, metb, 3)
        assert np.array_equal(W.interior(pb, qa), W.interior(pb, views[slot][0].cpu().numpy()))


def test_group_limits_and_steps_past_the_end():
    # group 0 stops after 2 steps, group 1 at t = 0.01 (a few steps of the 1D
    # tube), group 2 after 1 step; further steps leave each group untouched
    blocks = blast_like_blocks()
    blocks = [blocks[1], blocks[0], blocks[2]]
    B2, views2, _ = make_batch(blocks, [0, 1, 2])
    B2.set_group(0, 0.0, 1e30, max_steps=2)
    B2.set_group(1, 0.0, 0.01)
    B2.set_group(2, 0.0, 1e30, max_steps=1)
    B2.commit()
    for _ in range(12):
        B2.step(0.4)
    torch.cuda.synchronize()
    t, dt, ns, nf = B2.times(with_steps=True)
    assert not nf[:3].any()
    note(f"  steps {ns[:3].tolist()} t {t[:3].tolist()}")
    assert ns[0] == 2 and ns[2] == 1 and 2 < ns[1] < 12
    assert t[1] == 0.01 and dt[1] == 0.0
    for slot, nst, t_end in ((0, 2, 1e30), (1, 12, 0.01), (2, 1, 1e30)):
        p, pr, met = blocks[slot]
        qa, pa, ta = alone(p, pr, met, nst, t_end=t_end)
        assert t[slot] == ta
        assert np.array_equal(W.interior(p, qa), W.interior(p, views2[slot][0].cpu().numpy())), slot
        assert np.array_equal(pa, views2[slot][1].cpu().numpy()), slot


def test_single_grid_step_past_end_changes_nothing():
    p, pr, met = W.mhd_shock_tube(64)
    g = gmu.Grid(p)
    prd, metd = torch.from_numpy(pr.copy()).cuda(), torch.from_numpy(met).cuda()
    g.fill_ghosts(prd)
    qn = g.prim2con(prd, metd)
    g.c2p(qn, metd, prd)
    g.fill_ghosts(prd)
    qs = torch.zeros_like(qn)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros_like(t)
    t_end = 0.05
    for _ in range(200):
        g.step(qn, qs, prd, metd, 0.4, t_end, t, dt)
        if float(t.item()) >= t_end:
            break
    assert float(t.item()) == t_end
    snap = [x.clone() for x in (qn, qs, prd, t)]
    for _ in range(3):
        g.step(qn, qs, prd, metd, 0.4, t_end, t, dt)
    torch.cuda.synchronize()
    assert float(dt.item()) == 0.0
    for a, b in zip(snap, (qn, qs, prd, t)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("beyond", ["one_ulp", "caller_t_end_below_t"])
def test_single_grid_time_beyond_end_changes_nothing(beyond):
    """A capped final step can leave t an ulp past t_end, and a caller may pass
    t_end < t: the next step's dt is 0 (never negative), so nothing changes."""
    p, pr, met = W.mhd_shock_tube(64)
    g = gmu.Grid(p)
    prd, metd = torch.from_numpy(pr.copy()).cuda(), torch.from_numpy(met).cuda()
    g.fill_ghosts(prd)
    qn = g.prim2con(prd, metd)
    g.c2p(qn, metd, prd)
    g.fill_ghosts(prd)
    qs = torch.zeros_like(qn)
    t_end = 0.05
    t0 = np.nextafter(t_end, 1.0) if beyond == "one_ulp" else 0.2
    t = torch.full((1,), t0, dtype=torch.float64, device="cuda")
    dt = torch.full_like(t, -1.0)
    snap = [x.clone() for x in (qn, qs, prd, t)]
    for _ in range(2):
        g.step(qn, qs, prd, metd, 0.4, t_end, t, dt)
    torch.cuda.synchronize()
    assert float(dt.item()) == 0.0
    for a, b in zip(snap, (qn, qs, prd, t)):
        assert torch.equal(a, b)
