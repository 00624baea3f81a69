"""GPU parity of the scheme options against the oracle: the local
Lax-Friedrichs (TVDLF) flux, MP5 and PPM reconstruction named in section 3,
and the GRHD z-scheme recovery of section 2.5.1 (its per-cell parity is in
test_gpu_parity.py)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2012_07322_amd as gmu
import workloads as W
from test_gpu_parity import evolve_gpu, evolve_oracle, l1_rel, note, rhs_check, smooth_random_state

pytestmark = pytest.mark.gpu


def test_rhs_parity_tvdlf_tube_evolved():
    p, pr, met = W.mhd_shock_tube(400)
    p["riemann"] = 1
    oracle.fill_ghosts(p, pr)
    q = oracle.prim2con(p, pr, met)
    oracle.evolve(p, q, pr, met, 0.4, 0.0, 0.4, nsteps=60)
    rhs_check(p, pr, met)


def test_rhs_parity_tvdlf_blast_3d_ragged():
    p, pr, met = W.blast_wave_3d(24)
    p["n"] = [37, 29, 19]
    p["dx"] = [1.0 / 37, 1.0 / 29, 1.0 / 19]
    p["riemann"] = 1
    pr = W.blast_prim(p, seed=3)
    met = W.flat_metric(p)
    oracle.fill_ghosts(p, pr)
    rhs_check(p, pr, met)


@pytest.mark.parametrize("coord,ndim", [(W.CYL, 2), (W.SPH, 3)])
def test_rhs_parity_tvdlf_curvilinear(coord, ndim):
    n = [11, 9, 7][:ndim]
    if coord == W.CYL:
        p = W.grid(ndim, coord, n, [0.4, -1, 0], [2.0, 1, 2 * math.pi], [[1, 1]] * ndim)
    else:
        p = W.grid(ndim, coord, n, [0.5, 0.3, 0], [2.5, math.pi - 0.3, 2 * math.pi], [[1, 1]] * ndim)
    p["riemann"] = 1
    pr, met = smooth_random_state(p, beta_amp=0.05)
    rhs_check(p, pr, met)


def test_hundred_steps_tvdlf_alfven():
    p, pr, met = W.alfven_wave(128, rk=2)
    p["riemann"] = 1
    qg, pg, tg, nfg = evolve_gpu(p, pr, met, 0.4, 1e30, 100)
    qo, po, to, nfo = evolve_oracle(p, pr, met, 0.4, 1e30, 100)
    e = l1_rel(p, qg, qo)
    note(f"  alfven tvdlf: L1 rel per var={np.array2string(e, precision=2)}")
    assert abs(tg - to) <= 1e-12 * to and nfg == nfo == 0
    assert e.max() <= 1e-9


@pytest.mark.parametrize("riemann", [0, 1])
def test_hydro_tube_with_z_scheme(riemann):
    """The relativistic shock tube of section 3.1.2 evolved to t = 0.4 with
    the z-scheme recovery, GPU vs oracle."""
    p, pr, met = W.srhd_shock_tube(400)
    p["c2p"] = 1
    p["riemann"] = riemann
    qg, pg, tg, nfg = evolve_gpu(p, pr, met, 0.4, 0.4, 2000)
    qo, po, to, nfo = evolve_oracle(p, pr, met, 0.4, 0.4, 2000)
    e = l1_rel(p, qg, qo)
    note(f"  srhd tube z-scheme riemann={riemann}: L1 rel per var={np.array2string(e, precision=2)}")
    assert tg == pytest.approx(0.4, abs=1e-14) and to == pytest.approx(0.4, abs=1e-14)
    assert nfg == nfo == 0
    assert e[[0, 1, 4]].max() <= 1e-9


def test_batch_blocks_with_scheme_options_equal_alone():
    """Blocks with TVDLF and the z-scheme in a batch equal the same blocks
    advanced alone, bit for bit."""
    blocks = []
    p, pr, met = W.srhd_shock_tube(300)
    p.update(c2p=1, riemann=1)
    blocks.append((p, pr, met))
    p, pr, met = W.blast_wave_2d(40, seed=4)
    p["riemann"] = 1
    blocks.append((p, pr, met))
    p, pr, met = W.blast_wave_3d(16, seed=4)
    p.update(c2p=1, riemann=1)
    pr[5:8] = 0.0
    blocks.append((p, pr, met))
    shapes = []
    for p, _, _ in blocks:
        s = gmu.state_shape(p)
        shapes += [(8,) + s] * 3 + [(5,) + s]
    ar = gmu.Arena(gmu.Arena.size_of(shapes))
    B = gmu.Batch(8, 8, 1 << 14)
    views = []
    for slot, (p, pr, met) in enumerate(blocks):
        s = gmu.state_shape(p)
        qn, qs, prim, m = ar.take((8,) + s), ar.take((8,) + s), ar.take((8,) + s), ar.take((5,) + s)
        prim.copy_(torch.from_numpy(pr))
        m.copy_(torch.from_numpy(met))
        qs.zero_()
        B.set_block(slot, p, qn, qs, prim, m, slot)
        B.set_group(slot, 0.0, 1e30)
        views.append((qn, prim))
    B.commit()
    B.init()
    for _ in range(4):
        B.step(0.4)
    torch.cuda.synchronize()
    for slot, (p, pr, met) in enumerate(blocks):
        qa, pa, ta, _ = evolve_gpu(p, pr, met, 0.4, 1e30, 4)
        assert np.array_equal(W.interior(p, qa), W.interior(p, views[slot][0].cpu().numpy()))
        assert np.array_equal(pa, views[slot][1].cpu().numpy())


# ----------------------------------- MP5 and PPM (3 ghost layers)

RECONS = pytest.mark.parametrize("recon", [1, 2], ids=["mp5", "ppm"])


@RECONS
def test_rhs_parity_high_order_tube_evolved(recon):
    p, pr, met = W.mhd_shock_tube(400, ng=3, recon=recon)
    oracle.fill_ghosts(p, pr)
    q = oracle.prim2con(p, pr, met)
    oracle.evolve(p, q, pr, met, 0.4, 0.0, 0.4, nsteps=60)
    rhs_check(p, pr, met)


@RECONS
def test_rhs_parity_high_order_blast_3d_ragged(recon):
    p, pr, met = W.blast_wave_3d(24, ng=3, recon=recon)
    p["n"] = [37, 29, 19]
    p["dx"] = [1.0 / 37, 1.0 / 29, 1.0 / 19]
    pr = W.blast_prim(p, seed=5)
    met = W.flat_metric(p)
    oracle.fill_ghosts(p, pr)
    rhs_check(p, pr, met)


@RECONS
@pytest.mark.parametrize("coord,ndim,riemann", [(W.CYL, 2, 0), (W.SPH, 3, 1), (W.SPH, 2, 0)])
def test_rhs_parity_high_order_curvilinear(coord, ndim, riemann, recon):
    n = [11, 9, 7][:ndim]
    if coord == W.CYL:
        p = W.grid(ndim, coord, n, [0.4, -1, 0], [2.0, 1, 2 * math.pi], [[1, 1]] * ndim, ng=3, recon=recon)
    else:
        p = W.grid(ndim, coord, n, [0.5, 0.3, 0], [2.5, math.pi - 0.3, 2 * math.pi], [[1, 1]] * ndim, ng=3,
                   recon=recon)
    p["riemann"] = riemann
    pr, met = smooth_random_state(p, beta_amp=0.05)
    rhs_check(p, pr, met)


@RECONS
def test_hundred_steps_high_order_alfven(recon):
    p, pr, met = W.alfven_wave(128, rk=3, ng=3, recon=recon)
    qg, pg, tg, nfg = evolve_gpu(p, pr, met, 0.4, 1e30, 100)
    qo, po, to, nfo = evolve_oracle(p, pr, met, 0.4, 1e30, 100)
    e = l1_rel(p, qg, qo)
    note(f"  alfven recon={recon}: L1 rel per var={np.array2string(e, precision=2)}")
    assert abs(tg - to) <= 1e-12 * to and nfg == nfo == 0
    assert e.max() <= 1e-9


@RECONS
def test_hydro_tube_high_order_tvdlf_to_t_end(recon):
    """TVDLF + MP5 (the paper's default scheme) or PPM + SSPRK3 on the
    relativistic shock tube, whose cold right state exercises the
    reconstruction's positivity fallback, GPU vs oracle to t = 0.4."""
    p, pr, met = W.srhd_shock_tube(400, ng=3, recon=recon, riemann=1)
    qg, pg, tg, nfg = evolve_gpu(p, pr, met, 0.4, 0.4, 2000)
    qo, po, to, nfo = evolve_oracle(p, pr, met, 0.4, 0.4, 2000)
    e = l1_rel(p, qg, qo)
    note(f"  srhd tube recon={recon}+tvdlf: L1 rel per var={np.array2string(e, precision=2)}")
    assert tg == pytest.approx(0.4, abs=1e-14) and nfg == nfo == 0
    assert e[[0, 1, 4]].max() <= 1e-9


def test_batch_high_order_blocks_equal_alone():
    blocks = [W.mhd_shock_tube(300, ng=3, recon=1), W.blast_wave_2d(40, seed=6, ng=3, recon=1, riemann=1),
              W.blast_wave_3d(16, seed=6, ng=3, recon=1), W.mhd_shock_tube(200, ng=3, recon=2),
              W.blast_wave_2d(32, seed=7, ng=3, recon=2, riemann=1), W.blast_wave_3d(12, seed=7, ng=3, recon=2)]
    shapes = []
    for p, _, _ in blocks:
        s = gmu.state_shape(p)
        shapes += [(8,) + s] * 3 + [(5,) + s]
    ar = gmu.Arena(gmu.Arena.size_of(shapes))
    B = gmu.Batch(8, 8, 1 << 14)
    views = []
    for slot, (p, pr, met) in enumerate(blocks):
        s = gmu.state_shape(p)
        qn, qs, prim, m = ar.take((8,) + s), ar.take((8,) + s), ar.take((8,) + s), ar.take((5,) + s)
        prim.copy_(torch.from_numpy(pr))
        m.copy_(torch.from_numpy(met))
        qs.zero_()
        B.set_block(slot, p, qn, qs, prim, m, slot)
        B.set_group(slot, 0.0, 1e30)
        views.append((qn, prim))
    B.commit()
    B.init()
    B.autotune()
    for _ in range(4):
        B.step(0.4)
    torch.cuda.synchronize()
    for slot, (p, pr, met) in enumerate(blocks):
        qa, pa, ta, _ = evolve_gpu(p, pr, met, 0.4, 1e30, 4)
        assert np.array_equal(W.interior(p, qa), W.interior(p, views[slot][0].cpu().numpy()))
        assert np.array_equal(pa, views[slot][1].cpu().numpy())
