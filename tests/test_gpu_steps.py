"""gmunu_steps (several steps in one call, the CFL maxima of each later step
written by the previous step's last recovery) against the same number of
gmunu_step calls, and the face ghosts that the recovery writes against the
ghost kernel's fill.

Both are the same arithmetic on the same data, so the comparisons are bit
for bit: conserved variables, primitives with every ghost layer, flags,
time, dt and the fatal count."""
import numpy as np
import pytest
import torch

import paper_2012_07322_amd as gmu
import workloads as W
from test_gpu_parity import smooth_random_state

pytestmark = pytest.mark.gpu


def _xbc(p, lo, hi):
    p = dict(p)
    p["bc"] = [[lo, hi]] + [list(b) for b in p["bc"][1:]]
    return p


def _smooth(nd, coord, n, bc_x, bc_rest=None, lo=None, hi=None, **kw):
    if coord == W.CART:
        lo, hi = lo or [-0.4, -0.3, -0.2], hi or [0.5, 0.6, 0.7]
    else:  # a shell segment away from the centre and the axis
        lo, hi = lo or [1.0, 0.6, 0.0], hi or [2.0, 2.2, 1.5]
    hi = [hi[a] if a < nd else lo[a] + (1.0 if coord == W.CART or a < 2 else 2 * np.pi) for a in range(3)]
    bc = [list(bc_x)] + [list(b) for b in (bc_rest or [[W.OUTFLOW, W.OUTFLOW]] * (nd - 1))]
    p = W.grid(nd, coord, list(n), lo, hi, bc, gamma=5.0 / 3.0, rk=kw.pop("rk", 3), rho_atmo=1e-12, k_atmo=1.0,
               gamma_atmo=5.0 / 3.0, **kw)
    pr, met = smooth_random_state(p, seed=len(n), beta_amp=0.02)
    return p, pr, met


def _cases():
    out = {}
    out["tube outflow"] = W.mhd_shock_tube(300)
    p, pr, met = W.mhd_shock_tube(256)
    out["tube periodic"] = (_xbc(p, W.PERIODIC, W.PERIODIC), pr, met)
    p, pr, met = W.mhd_shock_tube(200)
    out["tube reflect-outflow"] = (_xbc(p, W.REFLECT, W.OUTFLOW), pr, met)
    out["tube mp5"] = W.mhd_shock_tube(200, ng=3, recon=1)
    out["two streams limiter"] = W.two_streams(200, rk=3, pp_limiter=1)
    out["blast 2d"] = W.blast_wave_2d(48)
    out["blast 3d"] = W.blast_wave_3d(20)
    out["blast 3d rk2"] = W.blast_wave_3d(16, rk=2)
    out["sph 2d outflow"] = _smooth(2, W.SPH, (24, 16), (W.OUTFLOW, W.OUTFLOW))
    out["cart 3d reflect"] = _smooth(3, W.CART, (9, 7, 5), (W.REFLECT, W.OUTFLOW))
    out["cart 2d periodic n0=2"] = _smooth(2, W.CART, (2, 12), (W.PERIODIC, W.PERIODIC))
    out["cart 2d n0=1"] = _smooth(2, W.CART, (1, 16), (W.OUTFLOW, W.OUTFLOW))
    out["cart 3d y periodic z reflect"] = _smooth(3, W.CART, (6, 8, 5), (W.OUTFLOW, W.REFLECT),
                                                  [[W.PERIODIC, W.PERIODIC], [W.REFLECT, W.REFLECT]])
    out["cart 3d ny=1"] = _smooth(3, W.CART, (8, 1, 6), (W.REFLECT, W.OUTFLOW))
    out["sph 2d axis"] = _smooth(2, W.SPH, (16, 12), (W.OUTFLOW, W.OUTFLOW), [[W.AXIS, W.REFLECT]],
                                 lo=[1.0, 0.0, 0.0], hi=[2.0, 0.5 * np.pi, 0.0])
    return out


CASES = _cases()


def _start(g, pr, met):
    prd = torch.from_numpy(pr.copy()).cuda()
    metd = torch.from_numpy(met).cuda()
    g.fill_ghosts(prd)
    qn = g.prim2con(prd, metd)
    g.c2p(qn, metd, prd)
    g.fill_ghosts(prd)
    z = lambda: torch.zeros(1, dtype=torch.float64, device="cuda")  # noqa: E731
    fl = torch.zeros(prd.shape[1:], dtype=torch.uint8, device="cuda")
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    return qn, torch.zeros_like(qn), prd, metd, z(), z(), fl, nf


@pytest.mark.parametrize("name", list(CASES))
def test_steps_equal_single_steps(name):
    p, pr, met = CASES[name]
    g = gmu.Grid(p)
    nsteps = 7
    # a t_end reached inside the run, from the first step's dt
    qn, qs, prd, metd, t, dt, fl, nf = _start(g, pr, met)
    g.step(qn, qs, prd, metd, 0.4, 1e30, t, dt, fl, nf)
    t_mid = 3.5 * float(dt.item())
    for t_end in (1e30, t_mid):
        outs = []
        for multi in (False, True):
            qn, qs, prd, metd, t, dt, fl, nf = _start(g, pr, met)
            if multi:
                g.steps(qn, qs, prd, metd, 0.4, t_end, t, dt, nsteps, fl, nf)
            else:
                for _ in range(nsteps):
                    g.step(qn, qs, prd, metd, 0.4, t_end, t, dt, fl, nf)
            torch.cuda.synchronize()
            outs.append([x.cpu().numpy() for x in (qn, prd, fl, t, dt, nf)])
        for a, b, what in zip(outs[0], outs[1], ("q_n", "prim", "flags", "t", "dt", "nfatal")):
            assert np.array_equal(a, b), f"{name} t_end={t_end}: {what} differs"
        if t_end < 1e30:
            assert outs[1][3][0] == t_mid


@pytest.mark.parametrize("name", list(CASES))
def test_recovery_ghosts_equal_the_ghost_kernel(name):
    """After steps whose recovery wrote the face ghosts of the leading axes
    it can (all three, x only when y sits on the polar axis or holds fewer
    than ng cells, none when x does), the ghost kernel refilling every face
    leaves the primitives unchanged."""
    p, pr, met = CASES[name]
    g = gmu.Grid(p)
    qn, qs, prd, metd, t, dt, fl, nf = _start(g, pr, met)
    g.steps(qn, qs, prd, metd, 0.4, 1e30, t, dt, 3, fl, nf)
    ref = prd.clone()
    g.fill_ghosts(ref)
    torch.cuda.synchronize()
    assert torch.equal(ref, prd)
