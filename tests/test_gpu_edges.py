"""Edge cases of the GPU path against the oracle: the smallest grids (one
cell along an axis), extents one below, at and one above a tile edge (the
stage kernel's tiles are 255 cells in 1D, 16 x 15 in 2D and 16 x 4 x 3 in
3D; the batch's 3D tiles also 8 x 6 x 4, 8 x 8 x 3 and 8 x 5 x 5), several
steps on such grids, an empty batch and an idle server.

Tolerances as in test_gpu_parity: the right-hand side at 1e-12 of each
cell's error scale and 1e-12 forward error per variable; ten steps at
1e-9 volume-weighted relative L1 per conserved variable."""
import numpy as np
import pytest
import torch

import paper_2012_07322_amd as gmu
import workloads as W
from test_gpu_parity import evolve_gpu, evolve_oracle, l1_rel, rhs_check, smooth_random_state

pytestmark = pytest.mark.gpu


def _grid(n, coord=W.CART):
    nd = len(n)
    if coord == W.CART:
        lo, hi = [-0.4, -0.3, -0.2], [0.5, 0.6, 0.7]
    else:  # a spherical shell segment away from the centre and the axis
        lo, hi = [1.0, 0.6, 0.0], [2.0, 2.2, 1.5]
    hi = [hi[a] if a < nd else lo[a] + (1.0 if coord == W.CART or a < 2 else 2 * np.pi) for a in range(3)]
    return W.grid(nd, coord, list(n), lo, hi, [[W.OUTFLOW, W.OUTFLOW]] * nd, gamma=5.0 / 3.0, rk=3,
                  rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=5.0 / 3.0)


SHAPES = [(1,), (2,), (254,), (255,), (256,), (511,),
          (1, 1), (16, 15), (15, 14), (17, 16), (1, 40), (40, 1),
          (1, 1, 1), (8, 6, 4), (7, 5, 3), (9, 7, 5), (1, 6, 9), (17, 13, 2),
          (16, 4, 3), (15, 3, 2), (17, 5, 4), (32, 8, 6)]


@pytest.mark.parametrize("n", SHAPES, ids=["x".join(map(str, s)) for s in SHAPES])
def test_rhs_on_tiny_and_tile_edge_grids(n):
    p = _grid(n)
    pr, met = smooth_random_state(p, seed=len(n))
    rhs_check(p, pr, met)


@pytest.mark.parametrize("n", [(9, 7, 5), (1, 6, 9), (3, 17)], ids=["9x7x5", "1x6x9", "3x17"])
def test_rhs_on_small_spherical_grids(n):
    p = _grid(n, W.SPH)
    pr, met = smooth_random_state(p, seed=3)
    rhs_check(p, pr, met)


@pytest.mark.parametrize("n", [(1,), (3,), (256,), (9, 7, 5), (1, 1, 1)], ids=["1", "3", "256", "9x7x5", "1x1x1"])
def test_ten_steps_on_tiny_grids(n):
    p = _grid(n)
    pr, met = smooth_random_state(p, seed=5, beta_amp=0.0)
    qg, pg, tg, nfg = evolve_gpu(p, pr, met, 0.4, 1e30, 10)
    qo, po, to, nfo = evolve_oracle(p, pr, met, 0.4, 1e30, 10)
    assert nfg == nfo == 0
    assert abs(tg - to) <= 1e-12 * to
    assert l1_rel(p, qg, qo).max() <= 1e-9


def test_empty_batch_steps_and_reports_nothing():
    """A batch with no blocks commits, initialises and steps (with and
    without the captured graph) without error; its groups keep t = 0 and
    dt = 0."""
    B = gmu.Batch(4, 4, 1024)
    try:
        B.commit()
        B.init()
        B.step(0.4, use_graph=False)
        B.step(0.4)
        B.step(0.4)
        torch.cuda.synchronize()
        t, dt = B.times()
        assert np.all(t[:4] == 0.0) and np.all(dt[:4] == 0.0)
        items, var = B.info()
        assert items.tolist() == [0, 0, 0] and np.all(var[:4] == -1)
    finally:
        B.close()


def test_idle_server_starts_and_stops():
    S = gmu.Server(1 << 24, max_slots=4, cfl=0.4)
    try:
        info = S.status()
        assert info["submitted"] == 0 and info["resident"] == 0 and info["error"] == 0
        assert S.poll(8, 10) == []
    finally:
        S.close()
