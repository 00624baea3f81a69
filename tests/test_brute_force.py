"""Brute-force evaluation of the discrete right-hand side on 8-cell grids,
in 50-digit arithmetic (mpmath), against the FP64 oracle.

The discretised equation of section 2.1: per interior cell,
    dq/dt = -(1/dV) sum_d [(F dA)_+ - (F dA)_-] + s + s_geom,
with MC-limited face values of (rho, W v^i, p, B^i), the face metric the mean
of the two adjacent centres, HLLE fluxes with the wave-speed bounds of
section 2.3, the gravitational sources of section 2.1 with centred metric
differences and K_ij from the shift (the CFC relation under maximal
slicing), and the geometric source with cell-averaged Christoffel symbols
(Appendix A).  Everything below is written independently of the oracle:
conserved variables and fluxes from the 4D stress tensor (u^mu, b^mu,
T^{mu nu} of the 4-metric), cell volumes, face areas and averaged Christoffel
symbols from their defining integrals, and every index loop written out per
cell and per face.  The grids: 1D Cartesian (8 cells), 1D spherical r (8
cells, theta and phi covering the sphere), and 3D Cartesian 2x2x2 with three
different spacings; random primitive states on every cell including the
ghosts, and a varying metric with a shift.  Agreement to 1e-13 of the
summed magnitudes of each cell's flux and source terms.
"""
import itertools
import math

import mpmath as mp
import numpy as np
import pytest

import oracle
import workloads as W

mp.mp.dps = 50
GAMMA = mp.mpf(5) / 3


def mc(a, b, c):
    dl, dr = b - a, c - b
    if dl * dr <= 0:
        return mp.mpf(0)
    m = min(abs(2 * dl), abs((dl + dr) / 2), abs(2 * dr))
    return m if (dl + dr) > 0 else -m


def ref_diag(coord, x1, x2):
    if coord == W.SPH:
        return [mp.mpf(1), x1 ** 2, (x1 * mp.sin(x2)) ** 2]
    if coord == W.CYL:
        return [mp.mpf(1), mp.mpf(1), x1 ** 2]
    return [mp.mpf(1)] * 3


def four_metric(psi, alpha, beta, ref):
    gd = [psi ** 4 * r for r in ref]
    g = mp.matrix(4, 4)
    bl = [gd[i] * beta[i] for i in range(3)]
    g[0, 0] = -alpha ** 2 + sum(bl[i] * beta[i] for i in range(3))
    for i in range(3):
        g[0, i + 1] = g[i + 1, 0] = bl[i]
        g[i + 1, i + 1] = gd[i]
    return g, gd


def state(prim, psi, alpha, beta, ref):
    """U (densitised), the three flux vectors F^a, and the stress tensor
    pieces needed by the sources, from 4D tensor algebra."""
    g, gd = four_metric(psi, alpha, beta, ref)
    gi = g ** -1
    Wv = prim[1:4]
    Wl = mp.sqrt(1 + sum(gd[i] * Wv[i] ** 2 for i in range(3)))
    v = [Wv[i] / Wl for i in range(3)]
    u = [Wl / alpha] + [Wl * (v[i] - beta[i] / alpha) for i in range(3)]
    ud = [sum(g[m, n] * u[n] for n in range(4)) for m in range(4)]
    B4 = [mp.mpf(0)] + list(prim[5:8])
    uB = sum(ud[m] * B4[m] for m in range(4))
    b = [(B4[m] + uB * u[m]) / Wl for m in range(4)]
    b2 = sum(b[m] * g[m, n] * b[n] for m in range(4) for n in range(4))
    rho, p = prim[0], prim[4]
    h = 1 + GAMMA / (GAMMA - 1) * p / rho
    T = [[(rho * h + b2) * u[m] * u[n] + (p + b2 / 2) * gi[m, n] - b[m] * b[n] for n in range(4)] for m in range(4)]
    Tmix = [[sum(T[m][l] * g[l, n] for l in range(4)) for n in range(4)] for m in range(4)]  # T^m_n
    s6 = psi ** 6
    D = rho * Wl
    U = [s6 * D] + [s6 * alpha * Tmix[0][1 + j] for j in range(3)] + [s6 * (alpha ** 2 * T[0][0] - D)] + \
        [s6 * prim[5 + j] for j in range(3)]
    F = []
    for a in range(3):
        vh = alpha * u[1 + a] / Wl
        f = [s6 * D * vh] + [s6 * alpha * Tmix[1 + a][1 + j] for j in range(3)] + \
            [s6 * (alpha ** 2 * T[0][1 + a] - D * vh)] + \
            [mp.mpf(0) if j == a else s6 * alpha * (b[1 + j] * u[1 + a] - b[1 + a] * u[1 + j]) for j in range(3)]
        F.append(f)
    # characteristic speed bounds along each axis (section 2.3)
    cs2 = GAMMA * p / (rho * h)
    ca2 = b2 / (rho * h + b2)
    a2 = cs2 + ca2 - cs2 * ca2
    v2 = sum(gd[i] * v[i] ** 2 for i in range(3))
    lam = []
    for a in range(3):
        disc = a2 * (1 - v2) * ((1 - v2 * a2) / gd[a] - (1 - a2) * v[a] ** 2)
        sq = mp.sqrt(disc) if disc > 0 else mp.mpf(0)
        lm = alpha * ((1 - a2) * v[a] - sq) / (1 - v2 * a2) - beta[a]
        lp = alpha * ((1 - a2) * v[a] + sq) / (1 - v2 * a2) - beta[a]
        lam.append((lm, lp))
    return dict(U=U, F=F, lam=lam, T=T, Tmix=Tmix, gd=gd, W=Wl)


def hlle(sl, sr, a):
    lmL, lpL = sl["lam"][a]
    lmR, lpR = sr["lam"][a]
    ap = max(mp.mpf(0), lpL, lpR)
    am = min(mp.mpf(0), lmL, lmR)
    FL, FR, UL, UR = sl["F"][a], sr["F"][a], sl["U"], sr["U"]
    if ap - am == 0:
        return [(FL[v] + FR[v]) / 2 for v in range(8)], [(abs(FL[v]) + abs(FR[v])) / 2 for v in range(8)]
    f = [(ap * FL[v] - am * FR[v] + ap * am * (UR[v] - UL[v])) / (ap - am) for v in range(8)]
    t = [(ap * abs(FL[v]) - am * abs(FR[v]) - ap * am * (abs(UR[v]) + abs(UL[v]))) / (ap - am) for v in range(8)]
    return f, t


def geometry(p):
    """Per-axis face positions, and functions giving a cell's volume, its two
    face areas along an axis, and the averaged Christoffel symbols, from their
    defining integrals (Appendix A)."""
    coord = p["coord"]
    xmin = [mp.mpf(x) for x in p["xmin"]]
    dx = [mp.mpf(x) for x in p["dx"]]

    def edges(a, i):
        return xmin[a] + i * dx[a], xmin[a] + (i + 1) * dx[a]

    def vol(i, j, k):
        (r0, r1), (t0, t1), (f0, f1) = edges(0, i), edges(1, j), edges(2, k)
        if coord == W.SPH:
            return (r1 ** 3 - r0 ** 3) / 3 * (mp.cos(t0) - mp.cos(t1)) * (f1 - f0)
        return (r1 - r0) * (t1 - t0) * (f1 - f0)

    def area(a, side, i, j, k):
        (r0, r1), (t0, t1), (f0, f1) = edges(0, i), edges(1, j), edges(2, k)
        if coord == W.SPH:
            if a == 0:
                r = r1 if side else r0
                return r * r * (mp.cos(t0) - mp.cos(t1)) * (f1 - f0)
            if a == 1:
                t = t1 if side else t0
                return (r1 ** 3 - r0 ** 3) / 3 * mp.sin(t) * (f1 - f0)
            return (r1 ** 3 - r0 ** 3) / 3 * (mp.cos(t0) - mp.cos(t1))
        return [(t1 - t0) * (f1 - f0), (r1 - r0) * (f1 - f0), (r1 - r0) * (t1 - t0)][a]

    def christoffel_avg(i, j, k):
        """<Gamma^l_ik> over the cell with the volume element r^2 sin(theta)
        (spherical), as a dict {(l, i, k): value}."""
        if coord != W.SPH:
            return {}
        (r0, r1), (t0, t1), (f0, f1) = edges(0, i), edges(1, j), edges(2, k)
        V = vol(i, j, k)

        def avg(fr, fth):  # integral of fr(r) fth(theta) r^2 sin(theta) / V
            return mp.quad(lambda r: fr(r) * r * r, [r0, r1]) * mp.quad(lambda t: fth(t) * mp.sin(t), [t0, t1]) * \
                (f1 - f0) / V
        inv_r = avg(lambda r: 1 / r, lambda t: 1)
        return {(1, 0, 1): inv_r, (1, 1, 0): inv_r, (2, 0, 2): inv_r, (2, 2, 0): inv_r,
                (0, 1, 1): avg(lambda r: -r, lambda t: 1),
                (2, 1, 2): avg(lambda r: 1, lambda t: mp.cos(t) / mp.sin(t)),
                (2, 2, 1): avg(lambda r: 1, lambda t: mp.cos(t) / mp.sin(t))}

    def centre(a, i):
        return xmin[a] + (i + mp.mpf(1) / 2) * dx[a]

    def face(a, i):
        return xmin[a] + i * dx[a]

    return vol, area, christoffel_avg, centre, face


def point_christoffel(coord, r, th):
    G = {}
    if coord == W.SPH:
        G = {(0, 1, 1): -r, (0, 2, 2): -r * mp.sin(th) ** 2, (1, 0, 1): 1 / r, (1, 1, 0): 1 / r,
             (1, 2, 2): -mp.sin(th) * mp.cos(th), (2, 0, 2): 1 / r, (2, 2, 0): 1 / r,
             (2, 1, 2): mp.cos(th) / mp.sin(th), (2, 2, 1): mp.cos(th) / mp.sin(th)}
    return G


def brute_rhs(p, prim, met):
    """dq/dt and its term-magnitude scale on every interior cell."""
    nd, coord = p["ndim"], p["coord"]
    n = p["n"]
    g = W.ghosts(p)
    vol, area, chr_avg, centre, face = geometry(p)
    dx = [mp.mpf(x) for x in p["dx"]]

    def P(v, i, j, k):
        return mp.mpf(float(prim[v, k + g[2], j + g[1], i + g[0]]))

    def M(w, i, j, k):
        return mp.mpf(float(met[w, k + g[2], j + g[1], i + g[0]]))

    out = {}
    for i, j, k in itertools.product(range(n[0]), range(n[1]), range(n[2])):
        c = (i, j, k)
        dq = [mp.mpf(0)] * 8
        scale = [mp.mpf(0)] * 8
        V = vol(i, j, k)
        for a in range(nd):
            for side in (0, 1):
                # face between cells c + (side - 1) e_a and c + side e_a
                lo = list(c)
                lo[a] += side - 1
                hi = list(c)
                hi[a] += side
                lo2, hi2 = list(lo), list(hi)
                lo2[a] -= 1
                hi2[a] += 1
                pl = [P(v, *lo) + mc(P(v, *lo2), P(v, *lo), P(v, *hi)) / 2 for v in range(8)]
                pr = [P(v, *hi) - mc(P(v, *lo), P(v, *hi), P(v, *hi2)) / 2 for v in range(8)]
                mf = [(M(w, *lo) + M(w, *hi)) / 2 for w in range(5)]
                xf = [centre(0, i), centre(1, j), centre(2, k)]
                xf[a] = face(a, c[a] + side)
                ref = ref_diag(coord, xf[0], xf[1])
                sl = state(pl, mf[0], mf[1], mf[2:5], ref)
                sr = state(pr, mf[0], mf[1], mf[2:5], ref)
                f, t = hlle(sl, sr, a)
                A = area(a, side, i, j, k)
                sgn = 1 if side else -1
                for v in range(8):
                    dq[v] -= sgn * f[v] * A / V
                    scale[v] += abs(t[v]) * A / V
        # sources at the cell centre
        x1, x2 = centre(0, i), centre(1, j)
        ref = ref_diag(coord, x1, x2)
        pc = [P(v, *c) for v in range(8)]
        psi, alpha, beta = M(0, *c), M(1, *c), [M(2 + m, *c) for m in range(3)]
        st = state(pc, psi, alpha, beta, ref)
        T, gd = st["T"], st["gd"]

        def dmet(w, a):
            if a >= nd:
                return mp.mpf(0)
            cp, cm = list(c), list(c)
            cp[a] += 1
            cm[a] -= 1
            return (M(w, *cp) - M(w, *cm)) / (2 * dx[a])
        dpsi = [dmet(0, a) for a in range(3)]
        dal = [dmet(1, a) for a in range(3)]
        Gp = point_christoffel(coord, x1, x2)
        nb = [[dmet(2 + m, a) + sum(Gp.get((m, a, l), 0) * beta[l] for l in range(3)) for m in range(3)]
              for a in range(3)]  # nb[a][m] = D^_a beta^m
        divb = nb[0][0] + nb[1][1] + nb[2][2]
        K = [[psi ** 4 / (2 * alpha) * (ref[m] * nb[a][m] + ref[a] * nb[m][a] - (mp.mpf(2) / 3 * ref[a] * divb
                                                                                   if a == m else 0))
              for m in range(3)] for a in range(3)]
        pre = alpha * psi ** 6
        T00, T0 = T[0][0], [T[0][1 + m] for m in range(3)]
        Tij = [[T[1 + a][1 + m] for m in range(3)] for a in range(3)]
        for a in range(3):
            terms = [-T00 * alpha * dal[a]]
            for m in range(3):
                T0low = T00 * gd[m] * beta[m] + T0[m] * gd[m]
                terms.append(T0low * nb[a][m])
                terms.append((T00 * beta[m] ** 2 + 2 * T0[m] * beta[m] + Tij[m][m]) * 4 * psi ** 3 * dpsi[a] * ref[m] / 2)
            dq[1 + a] += pre * sum(terms)
            scale[1 + a] += abs(pre) * sum(abs(x) for x in terms)
        terms = [T00 * K[a][m] * beta[a] * beta[m] for a in range(3) for m in range(3)]
        terms += [-T00 * beta[a] * dal[a] for a in range(3)]
        terms += [T0[a] * 2 * K[a][m] * beta[m] for a in range(3) for m in range(3)]
        terms += [-T0[a] * dal[a] for a in range(3)]
        terms += [Tij[a][m] * K[a][m] for a in range(3) for m in range(3)]
        dq[4] += pre * sum(terms)
        scale[4] += abs(pre) * sum(abs(x) for x in terms)
        # geometric source: <Gamma^l_ik> F^k_S_l with cell-centre fluxes, the
        # ignorable phi row omitted
        Ga = chr_avg(i, j, k)
        for a in range(2 if coord == W.SPH else 0):
            for (l, ii, kk), val in Ga.items():
                if ii == a:
                    term = val * st["F"][kk][1 + l]
                    dq[1 + a] += term
                    scale[1 + a] += abs(term)
        out[c] = (dq, scale)
    return out


SEEDS = {"cart1d": 11, "sph1d": 12, "cart3d_2x2x2": 13}


def random_case(name, seed):
    rng = np.random.default_rng(seed)
    if name == "cart1d":
        p = W.grid(1, W.CART, [8], [0.1, 0, 0], [0.9, 1, 1], [[W.OUTFLOW, W.OUTFLOW]])
    elif name == "sph1d":
        p = W.grid(1, W.SPH, [8], [0.5, 0, 0], [2.1, math.pi, 2 * math.pi], [[W.OUTFLOW, W.OUTFLOW]])
    else:
        p = W.grid(3, W.CART, [2, 2, 2], [0, 0, 0], [0.2, 0.26, 0.34], [[W.OUTFLOW, W.OUTFLOW]] * 3)
    shp = W.shape(p)
    pr = np.zeros((8,) + shp)
    pr[0] = rng.uniform(0.5, 2.0, shp)
    pr[4] = rng.uniform(0.2, 1.5, shp)
    x1, x2, _ = W.centres(p)
    sc = [np.ones(shp), np.ones(shp), np.ones(shp)]
    if p["coord"] == W.SPH:
        sc = [np.ones(shp), x1, x1 * np.sin(x2)]
    for a in range(3):
        pr[1 + a] = rng.uniform(-0.6, 0.6, shp) / sc[a]
        pr[5 + a] = rng.uniform(-0.8, 0.8, shp) / sc[a]
    met = np.zeros((5,) + shp)
    met[0] = 1.0 + rng.uniform(0, 0.1, shp)
    met[1] = 0.8 + rng.uniform(-0.1, 0.1, shp)
    for a in range(3):
        met[2 + a] = rng.uniform(-0.1, 0.1, shp) / sc[a]
    return p, pr, met


@pytest.mark.parametrize("name", ["cart1d", "sph1d", "cart3d_2x2x2"])
def test_rhs_equals_50_digit_brute_force(name):
    p, pr, met = random_case(name, seed=SEEDS[name])
    ref = brute_rhs(p, pr, met)
    g = W.ghosts(p)
    L = oracle.rhs(p, pr, met)
    worst = 0.0
    for (i, j, k), (dq, scale) in ref.items():
        for v in range(8):
            o = L[v, k + g[2], j + g[1], i + g[0]]
            e = abs(mp.mpf(float(o)) - dq[v]) / (scale[v] + mp.mpf("1e-300"))
            worst = max(worst, float(e))
    print(f"  {name}: {len(ref)} cells, worst |oracle - brute force| / term scale = {worst:.2e}")
    assert worst < 1e-13


# ------------------------------------------------------------ planted mistakes

MUTANTS = {
    # a transverse index of a Cartesian face area
    "cart_face_area_index": ("    if (a == 1) return d1 * d3;", "    if (a == 1) return d1 * d2;"),
    # the radial face area of the spherical grid with r instead of r^2
    "sph_radial_area_power": ("    return rf * rf * (2.0 * sin(th) * sin(0.5 * d2)) * d3;",
                              "    return rf * (2.0 * sin(th) * sin(0.5 * d2)) * d3;"),
    # the sign of the flux bracket
    "flux_bracket_sign": ("    for (int v = 0; v < NV; v++) dq[v] -= (fp[v] - fm[v]) / dV;",
                          "    for (int v = 0; v < NV; v++) dq[v] -= (fm[v] - fp[v]) / dV;"),
    # the MC limiter's central slope without the 1/2
    "mc_central_half": None,
}


def _mutant_rhs(tmp_path, name):
    import ctypes
    import os
    import subprocess

    src = open(os.path.join(os.path.dirname(oracle.__file__), "gmunu_oracle.c")).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, name
    c = tmp_path / f"{name}.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / f"{name}.so"
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", str(so), str(c), "-lm"])
    L = ctypes.CDLL(str(so))
    P = ctypes.c_void_p
    L.og_rhs.argtypes = [P, P, P, P]

    def rhs(p, prim, met):
        d = oracle.make_desc(p)
        prim, met = np.ascontiguousarray(prim), np.ascontiguousarray(met)
        out = np.zeros_like(prim)
        L.og_rhs(ctypes.byref(d), prim.ctypes.data_as(P), met.ctypes.data_as(P), out.ctypes.data_as(P))
        return out

    return rhs


def _mc_source_line():
    import os
    src = open(os.path.join(os.path.dirname(oracle.__file__), "gmunu_oracle.c")).read()
    i = src.index("static double mc_slope(")
    body = src[i:src.index("\n}\n", i)]
    line = [ln for ln in body.split("\n") if "0.5" in ln][0]
    return line, line.replace("0.5 * ", "")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistakes_fail_the_brute_force(tmp_path, name):
    if MUTANTS[name] is None:
        MUTANTS[name] = _mc_source_line()
    rhs = _mutant_rhs(tmp_path, name)
    worst = 0.0
    for case in ("cart1d", "sph1d", "cart3d_2x2x2"):
        p, pr, met = random_case(case, seed=SEEDS[case])
        ref = brute_rhs(p, pr, met)
        g = W.ghosts(p)
        L = rhs(p, pr, met)
        for (i, j, k), (dq, scale) in ref.items():
            for v in range(8):
                e = abs(mp.mpf(float(L[v, k + g[2], j + g[1], i + g[0]])) - dq[v]) / (scale[v] + mp.mpf("1e-300"))
                worst = max(worst, float(e))
    print(f"  mutant {name}: worst scaled error {worst:.2e}")
    assert worst > 1e-6
