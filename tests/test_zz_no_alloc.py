"""The allocation-free step (gmunu_step_static) against gmunu_step.

It runs the same kernels with the grid's geometry tables and the CFL
partials in the library's static per-GPU scratch: Cartesian grids (whose
geometry is 1/dx and unit face factors, computed identically on host and
device) must give the context's results bit for bit; spherical grids (device
sines and cosines in the tables) within 1e-12 of each variable's scale (the
momentum components at the momentum's).  Two
calls in a row with the second grid smaller, and then a third that is larger
again, show that each call rewrites the scratch it needs.
"""
import math

import numpy as np
import pytest
import torch

import paper_2012_07322_amd as gmu
import workloads as W

pytestmark = pytest.mark.gpu


def run(p, pr, met, nsteps, static):
    prd, metd = torch.from_numpy(pr.copy()).cuda(), torch.from_numpy(met).cuda()
    g = gmu.Grid(p)
    g.fill_ghosts(prd)
    qn = g.prim2con(prd, metd)
    g.c2p(qn, metd, prd)
    g.fill_ghosts(prd)
    qs = torch.zeros_like(qn)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros_like(t)
    nf = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(nsteps):
        if static:
            gmu.step_static(p, qn, qs, prd, metd, 0.4, 1e30, t, dt, None, nf)
        else:
            g.step(qn, qs, prd, metd, 0.4, 1e30, t, dt, None, nf)
    torch.cuda.synchronize()
    return qn.cpu().numpy(), prd.cpu().numpy(), float(t.item()), int(nf.item())


def cases():
    p1, _, _ = W.blast_wave_3d(24)
    p1["n"] = [37, 29, 19]
    p1["dx"] = [1.0 / 37, 1.0 / 29, 1.0 / 19]
    big = (p1, W.blast_prim(p1, seed=2), W.flat_metric(p1))
    small = W.blast_wave_2d(24)
    star = W.magnetised_star_2d(48, 24)
    return [("cart3d_37x29x19", big, True), ("cart2d_24x24", small, True), ("sph2d_star_48x24", star, False),
            ("cart3d_37x29x19_again", big, True)]


def test_static_step_equals_context_step():
    for name, (p, pr, met), bitwise in cases():
        qa, pa, ta, na = run(p, pr, met, 3, static=False)
        qb, pb, tb, nb = run(p, pr, met, 3, static=True)
        assert na == nb == 0
        A, B = W.interior(p, qa), W.interior(p, qb)
        if bitwise:
            assert ta == tb, name
            assert np.array_equal(A, B) and np.array_equal(pa, pb), name
        else:
            # momentum components at the momentum's scale: S_theta of a
            # spherically symmetric star is itself round-off
            assert abs(ta - tb) <= 1e-13 * ta, name
            smax = max(np.abs(A[c]).max() for c in (1, 2, 3))
            for v in range(8):
                sc = smax if v in (1, 2, 3) else np.abs(A[v]).max()
                assert np.abs(A[v] - B[v]).max() <= 1e-12 * sc + 1e-300, (name, v)
        print(f"  {name}: t={tb:.6e} {'bitwise equal' if bitwise else 'within 1e-12'}")
