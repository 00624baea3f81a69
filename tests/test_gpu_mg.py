"""GPU multigrid (gmunu_mg_*, through the C ABI) against the multigrid
oracle, element by element on the same inputs.

Tolerances (FP64 on both sides, different operation order):
  ghost fill          bit-exact (Dirichlet, Neumann, periodic); 1e-15
                      relative for the Robin factor (one rounding apart)
  operator, one sweep 1e-12 of the largest |L(u)| (or |u|)
  restriction, Kwak   1e-14 absolute on O(1) data
  solve, cleaning     1e-10 of the solution's largest magnitude (both
                      sides converge to the same discrete solution; the
                      difference is the tolerance over the operator's
                      smallest eigenvalue), residual histories to 1e-6
                      relative while above 1e-5 (below, rounding of the
                      O(1/h^2) operator dominates the difference)
"""
import math
import sys

import numpy as np
import pytest
import torch

import paper_2012_07322_amd as gmu
from oracle import mg

pytestmark = pytest.mark.gpu

CART, CYL, SPH = mg.CART, mg.CYL, mg.SPH
D, N, PER, ROB = mg.DIRICHLET, mg.NEUMANN, mg.PERIODIC, mg.ROBIN


def note(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def prob(ndim, coord, n, xmin, xmax, bc, **kw):
    n = list(n) + [1] * (3 - len(n))
    xmin, xmax = list(xmin) + [0] * (3 - len(xmin)), list(xmax) + [1] * (3 - len(xmax))
    dx = [(xmax[a] - xmin[a]) / n[a] for a in range(3)]
    bc = list(bc) + [[N, N]] * (3 - len(bc))
    p = dict(ndim=ndim, coord=coord, n=n, xmin=xmin, dx=dx, bc=bc)
    p.update(kw)
    return p


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = {
    "cart3d": prob(3, CART, (16, 8, 8), (0, 0, 0), (1, 0.5, 0.5), [[D, N], [PER, PER], [D, D]]),
    "cyl2d": prob(2, CYL, (16, 16), (0.0, -1), (2.0, 1), [[N, D], [D, N]]),
    "cyl3d": prob(3, CYL, (8, 8, 16), (0.5, -1, 0), (2.5, 1, 2 * math.pi), [[D, ROB], [N, D], [PER, PER]]),
    "sph2d": prob(2, SPH, (16, 16), (0.0, 0.0), (4.0, math.pi), [[N, ROB], [N, N]]),
    "sph3d": prob(3, SPH, (8, 8, 8), (0.5, 0.3, 0.0), (2.5, math.pi - 0.3, 2 * math.pi),
                  [[D, ROB], [N, D], [PER, PER]]),
    "sph1d": prob(1, SPH, (32,), (0.0,), (4.0,), [[N, ROB]]),
}


def random_field(p, seed, vector=False):
    rng = np.random.default_rng(seed)
    shp = ((3,) if vector else ()) + mg.shape(p)
    return rng.uniform(-1, 1, shp)


@pytest.mark.parametrize("case", sorted(CASES))
def test_ghost_fill_and_operator_parity(case):
    p = CASES[case]
    M = gmu.Multigrid(p)
    assert M.levels == mg.make_desc(p).levels
    u = random_field(p, 1)
    ug = dev(u)
    M.fill_ghosts(ug)
    uo = mg.fill_ghosts(p, u.copy())
    g = host(ug)
    robin = any(ROB in p["bc"][a] for a in range(3))
    if robin:
        np.testing.assert_allclose(g, uo, rtol=1e-15, atol=0)
    else:
        assert np.array_equal(g, uo)
    a = random_field(p, 2) * 0.1
    for power, offset in ((0, 0.0), (1, 0.5), (-1, 3.0)):
        q = dict(p, power=power, offset=offset)
        Mq = gmu.Multigrid(q)
        Lg = mg.interior(q, host(Mq.apply(dev(uo), dev(a))))
        Lo = mg.interior(q, mg.apply(q, uo, a))
        assert np.abs(Lg - Lo).max() <= 1e-12 * np.abs(Lo).max(), (power, np.abs(Lg - Lo).max())


@pytest.mark.parametrize("case", ["cart3d", "sph2d", "cyl3d"])
def test_smoothing_sweep_parity(case):
    p = dict(CASES[case], power=-1, offset=2.0)
    M = gmu.Multigrid(p)
    u, f, a = random_field(p, 3), random_field(p, 4), random_field(p, 5) * 0.1
    ug = dev(u)
    M.smooth(ug, dev(f), dev(a), sweeps=2)
    uo = mg.smooth(p, u.copy(), f, a, sweeps=2)
    g = host(ug)
    assert np.abs(g - uo).max() <= 1e-12 * np.abs(uo).max()


@pytest.mark.parametrize("case", sorted(CASES))
def test_transfer_operator_parity(case):
    p = CASES[case]
    M = gmu.Multigrid(p)
    top = M.levels - 1
    fine = random_field(p, 6)
    cg = host(M.restrict(top, dev(fine)))
    co = mg.restrict(p, top, fine)
    assert np.abs(cg - co).max() <= 1e-14
    c = np.random.default_rng(7).uniform(-1, 1, mg.shape(p, top - 1))
    fg = host(M.prolong(top, dev(c)))
    fo = mg.prolong(p, top, c)
    assert np.abs(mg.interior(p, fg) - mg.interior(p, fo)).max() <= 1e-14


SOLVES = {
    "cart2d": (prob(2, CART, (32, 32), (0, 0), (1, 1), [[D, D], [N, D]]), {}),
    "cyl2d": (prob(2, CYL, (32, 32), (0.0, -1), (2.0, 1), [[N, D], [D, D]]), {}),
    "sph2d_robin": (prob(2, SPH, (32, 16), (0.0, 0.0), (8.0, math.pi), [[N, ROB], [N, N]], pre=4, post=4), {}),
    "cart3d": (prob(3, CART, (32, 32, 32), (0, 0, 0), (1, 1, 1), [[D, D]] * 3), {}),
    "psi_sph2d": (prob(2, SPH, (32, 16), (0.0, 0.0), (8.0, math.pi), [[N, ROB], [N, N]], power=-1, offset=1.0,
                       pre=4, post=4), {"a": True}),
    "alpha_cart3d": (prob(3, CART, (32, 32, 32), (-1, -1, -1), (1, 1, 1), [[D, D]] * 3, power=1, offset=1.0),
                     {"a": True}),
}


def solve_problem(p, with_a):
    x, y, z = mg.centres(p)
    if p["coord"] == SPH:
        f = np.exp(-x * x) * (1 + 0.3 * np.cos(y) ** 2)
    else:
        f = np.exp(-((x - 0.4) ** 2 + (y - 0.2) ** 2 + (z - 0.1) ** 2) * 8)
    if with_a:
        a = -2 * math.pi * 0.05 * f if p["power"] == -1 else 2 * math.pi * 0.05 * f
        return np.zeros_like(f) if p["power"] == -1 else 0.1 * f, a
    return f - 0.2, None


@pytest.mark.parametrize("case", sorted(SOLVES))
def test_solve_parity(case):
    p, opt = SOLVES[case]
    f, a = solve_problem(p, opt.get("a", False))
    M = gmu.Multigrid(p)
    ug = torch.zeros(M.shape(), dtype=torch.float64, device="cuda")
    hist_g = M.solve(ug, dev(f), dev(a) if a is not None else None, tol=1e-11, max_cycles=100)
    uo = np.zeros(mg.shape(p))
    hist_o = mg.solve(p, uo, np.ascontiguousarray(f), np.ascontiguousarray(a) if a is not None else None, tol=1e-11,
                      max_cycles=100)
    note(f"  {case}: cycles gpu {len(hist_g) - 1} oracle {len(hist_o) - 1}, final {hist_g[-1]:.2e}")
    assert hist_g[-1] <= 1e-11 and hist_o[-1] <= 1e-11
    g = host(ug)
    scale = np.abs(mg.interior(p, uo)).max()
    assert np.abs(mg.interior(p, g) - mg.interior(p, uo)).max() <= 1e-10 * scale
    for hg, ho in zip(hist_g, hist_o):
        if ho < 1e-5:
            break
        assert abs(hg - ho) <= 1e-6 * ho, (hg, ho)


def test_cleaning_parity():
    p = prob(3, CART, (32, 32, 32), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
    x, y, z = mg.centres(p)
    s, c = np.sin, np.cos
    pi = math.pi
    q = np.stack([pi * c(pi * x) * s(pi * y) * s(pi * z) + 2 * pi * s(2 * pi * x) * c(2 * pi * y),
                  pi * s(pi * x) * c(pi * y) * s(pi * z) - 2 * pi * c(2 * pi * x) * s(2 * pi * y),
                  pi * s(pi * x) * s(pi * y) * c(pi * z)])
    q = np.ascontiguousarray(q)
    M = gmu.Multigrid(p)
    qg, phig, divg = dev(q), torch.zeros(M.shape(), dtype=torch.float64, device="cuda"), M.empty()
    hist = M.clean(qg, phig, divg, tol=1e-12, max_cycles=40)
    assert hist[-1] <= 1e-12
    div0 = mg.divergence(p, q)
    assert np.abs(mg.interior(p, host(divg)) - mg.interior(p, div0)).max() <= 1e-12 * np.abs(div0).max()
    uo = np.zeros(mg.shape(p))
    mg.solve(p, uo, np.ascontiguousarray(div0), tol=1e-12, max_cycles=40)
    mg.fill_ghosts(p, uo)
    qo = mg.subtract_gradient(p, uo, q.copy())
    qgh = host(qg)
    for i in range(3):
        assert np.abs(mg.interior(p, qgh[i]) - mg.interior(p, qo[i])).max() <= 1e-10 * np.abs(q).max()


def test_large_grid_cycle_rate_and_residual():
    """256^3 Poisson (Dirichlet box): each V(2,2)-cycle cuts the residual by
    about 10 as on small grids (a property at any size), and the solve
    reaches 1e-10 of the source scale."""
    n = 256
    p = prob(3, CART, (n, n, n), (-1, -1, -1), (1, 1, 1), [[D, D]] * 3)
    M = gmu.Multigrid(p)
    sh = M.shape()
    ax = [(torch.arange(sh[2 - a], dtype=torch.float64, device="cuda") - 0.5) * p["dx"][a] - 1 for a in range(3)]
    X = ax[0].view(1, 1, -1)
    Y = ax[1].view(1, -1, 1)
    Z = ax[2].view(-1, 1, 1)
    f = torch.exp(-8 * (X * X + Y * Y + Z * Z)).contiguous()
    u = torch.zeros(sh, dtype=torch.float64, device="cuda")
    hist = M.solve(u, f, None, tol=1e-10, max_cycles=30)
    rates = [hist[i + 1] / hist[i] for i in range(1, len(hist) - 1)]
    note(f"  256^3: {len(hist) - 1} cycles, rates {['%.3f' % r for r in rates]}")
    assert hist[-1] <= 1e-10
    assert max(rates) < 0.15


def test_invalid_descriptors_are_rejected():
    bad = [prob(2, CART, (12, 16), (0, 0), (1, 1), [[D, D], [D, D]], levels=4),   # 12 not divisible by 8
           prob(2, CART, (16, 16), (0, 0), (1, 1), [[ROB, D], [D, D]]),            # Robin in Cartesian
           prob(2, SPH, (16, 16), (0, 0), (1, 1), [[N, D], [ROB, D]]),             # Robin off axis 0
           prob(2, CART, (16, 16), (0, 0), (1, 1), [[PER, D], [D, D]]),            # one-sided periodic
           prob(2, CART, (16, 16), (0, 0), (1, 1), [[D, D], [D, D]], power=2)]
    for p in bad:
        with pytest.raises(RuntimeError):
            gmu.Multigrid(p)


# ------------------------------------------- bridge to the GRMHD state

def test_clean_state_matches_the_oracle():
    """Cleaning of q_B of a GRMHD state (q from the GPU's prim2con with a
    non-trivial conformal factor): the cleaned interior q_B equals the
    oracle's cleaning of the same field (interior q_B, ghost layer psi^6 B)."""
    import workloads as W
    n = 32
    hp = W.grid(3, W.CART, [n] * 3, [0, 0, 0], [1, 1, 1], [[W.OUTFLOW, W.OUTFLOW]] * 3, gamma=5 / 3)
    x, y, z = W.centres(hp)
    s, c, pi = np.sin, np.cos, math.pi
    pr = W.empty_prim(hp)
    pr[0] = 1.0
    pr[4] = 1.0
    pr[5] = pi * c(pi * x) * s(pi * y) * s(pi * z) + 2 * pi * s(2 * pi * x) * c(2 * pi * y)
    pr[6] = pi * s(pi * x) * c(pi * y) * s(pi * z) - 2 * pi * c(2 * pi * x) * s(2 * pi * y)
    pr[7] = pi * s(pi * x) * s(pi * y) * c(pi * z)
    met = W.flat_metric(hp)
    met[0] = 1.0 + 0.1 * s(2 * pi * x) * c(pi * y)
    g = gmu.Grid(hp)
    prd, metd = dev(pr), dev(met)
    q = g.prim2con(prd, metd)
    q0 = host(q).copy()
    mp = prob(3, CART, (n, n, n), (0, 0, 0), (1, 1, 1), [[D, D]] * 3)
    M = gmu.Multigrid(mp)
    hist = M.clean_state(hp, q, prd, metd, tol=1e-12, max_cycles=40)
    assert hist[-1] <= 1e-12
    qg = host(q)
    # oracle: the same field on the multigrid layout
    gh = 2
    sl = (slice(gh - 1, gh + n + 1),) * 3
    psi6 = met[0][sl] ** 6
    qb = np.stack([psi6 * pr[5 + i][sl] for i in range(3)])
    inner = (slice(1, -1),) * 3
    for i in range(3):
        qb[i][inner] = q0[5 + i][(slice(gh, gh + n),) * 3]
    qb = np.ascontiguousarray(qb)
    div = mg.divergence(mp, qb)
    u = np.zeros(mg.shape(mp))
    mg.solve(mp, u, np.ascontiguousarray(div), tol=1e-12, max_cycles=40)
    mg.fill_ghosts(mp, u)
    mg.subtract_gradient(mp, u, qb)
    for i in range(3):
        got = qg[5 + i][(slice(gh, gh + n),) * 3]
        assert np.abs(got - qb[i][inner]).max() <= 1e-10 * np.abs(qb).max()
    # the rest of q is untouched
    assert np.array_equal(qg[:5], q0[:5])


def test_cfc_solve_recovers_the_tov_metric():
    """The scalar CFC equations solved from the conserved variables of a
    static TOV star (built with its own metric) from a flat initial guess
    return the TOV conformal factor and lapse (TOV in isotropic coordinates
    is conformally flat), with the error falling at about second order; the
    conformal factor agrees with the oracle's solve of the same equation."""
    import workloads as W
    errs = []
    for nr, nth in ((64, 16), (128, 32)):
        hp, pr, met = W.magnetised_star_2d(nr, nth, b_peak=1e-12)
        g = gmu.Grid(hp)
        prd, metd = dev(pr), dev(met)
        g.fill_ghosts(prd)
        q = g.prim2con(prd, metd)
        exact = met.copy()
        metd[0].fill_(1.0)
        metd[1].fill_(1.0)
        mp = prob(2, SPH, (nr, nth), (0.0, 0.0), (hp["dx"][0] * nr, math.pi), [[N, ROB], [N, N]], pre=4, post=4)
        Mp = gmu.Multigrid(dict(mp, power=-1, offset=1.0))
        Ma = gmu.Multigrid(dict(mp, power=1, offset=1.0))
        cyc = gmu.cfc_solve(Mp, Ma, hp, q, prd, metd, tol=1e-12, max_cycles=200)
        m = host(metd)
        gh = hp.get("ng", 2)
        sl = (Ellipsis, slice(gh, gh + nth), slice(gh, gh + nr))
        e_psi = np.abs(m[0][sl] - exact[0][sl]).max()
        e_al = np.abs(m[1][sl] - exact[1][sl]).max()
        note(f"  TOV {nr}x{nth}: cycles {cyc}, |psi err| {e_psi:.2e}, |alpha err| {e_al:.2e}")
        errs.append((e_psi, e_al))
        # parity of the psi solve with the oracle on the same coefficient
        qh = host(q)
        a = np.zeros(mg.shape(dict(mp)))
        a[0, 1:-1, 1:-1] = -2 * math.pi * (qh[4] + qh[0])[0, gh:gh + nth, gh:gh + nr]
        uo = np.zeros(mg.shape(dict(mp)))
        po = dict(mp, power=-1, offset=1.0)
        mg.solve(po, uo, np.zeros_like(uo), np.ascontiguousarray(a), tol=1e-12, max_cycles=200)
        assert np.abs(1.0 + mg.interior(po, uo)[0] - m[0][sl][0]).max() <= 1e-9
    assert errs[1][0] < 2e-4 and errs[1][1] < 4e-4
    assert errs[0][0] / errs[1][0] > 2.5 and errs[0][1] / errs[1][1] > 2.5
