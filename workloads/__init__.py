"""Seeded synthetic inputs for the GRMHD finite-volume step.

This module holds initial data only: grid descriptions (plain dicts), the
primitive fields (rho, W v^i, p, B^i) and the frozen metric (psi, alpha,
beta^i) of the test problems and benchmark workloads.  It holds none of the
method's arithmetic (no conserved variables, fluxes or recovery), so both the
GPU path and the CPU oracle can take their inputs from here.

Random numbers come from a counter-based generator (splitmix64 of
seed-mixed global cell indices), so a value depends only on (seed, index)
and not on array layout or blocking.
"""
from __future__ import annotations

import math

import numpy as np

CART, CYL, SPH = 0, 1, 2
PERIODIC, OUTFLOW, REFLECT, AXIS, CENTER, NONE = 0, 1, 2, 3, 4, 5

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """splitmix64 finaliser (Steele, Lea & Flood 2014) on uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed: int, idx, stream: int = 0):
    """Uniform doubles in [-1, 1) keyed by (seed, stream, idx)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = splitmix64(np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream))
        z = splitmix64(idx ^ key)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def grid(ndim, coord, n, xmin, xmax, bc, **kw):
    """Grid parameter dict.  Inactive axes: n=1 and the given extent (for an
    inactive phi the extent is 2 pi)."""
    n = list(n) + [1] * (3 - len(n))
    xmin = list(xmin)
    xmax = list(xmax)
    dx = [(xmax[a] - xmin[a]) / n[a] for a in range(3)]
    bcl = [list(b) for b in bc] + [[NONE, NONE]] * (3 - len(bc))
    p = dict(ndim=ndim, coord=coord, n=n, ng=2, xmin=xmin, dx=dx, bc=bcl)
    p.update(kw)
    return p


def ghosts(p):
    return [p.get("ng", 2) if a < p["ndim"] else 0 for a in range(3)]


def shape(p):
    g = ghosts(p)
    return tuple(p["n"][a] + 2 * g[a] for a in (2, 1, 0))


def centres(p):
    """Cell-centre coordinates (x1, x2, x3), each of shape (nt2, nt1, nt0),
    including ghost cells."""
    g = ghosts(p)
    ax = []
    for a in range(3):
        i = np.arange(-g[a], p["n"][a] + g[a])
        ax.append(p["xmin"][a] + (i + 0.5) * p["dx"][a])
    x3, x2, x1 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x1, x2, x3


def interior(p, a):
    g = ghosts(p)
    sl = tuple(slice(g[ax], g[ax] + p["n"][ax]) for ax in (2, 1, 0))
    return a[(Ellipsis,) + sl]


def global_index(p):
    """Global interior-cell index (i + n0 (j + n1 k)) of every cell, ghosts
    included (ghost indices are those of the wrapped interior cell)."""
    g = ghosts(p)
    n = p["n"]
    i = (np.arange(-g[0], n[0] + g[0]) % n[0]).astype(np.int64)
    j = (np.arange(-g[1], n[1] + g[1]) % n[1]).astype(np.int64)
    k = (np.arange(-g[2], n[2] + g[2]) % n[2]).astype(np.int64)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")
    return I + n[0] * (J + n[1] * K)


def flat_metric(p):
    m = np.zeros((5,) + shape(p))
    m[0] = 1.0
    m[1] = 1.0
    return m


def empty_prim(p):
    return np.zeros((8,) + shape(p))


# --------------------------------------------------------------- 1D problems

def mhd_shock_tube(n=400, gamma=5.0 / 3.0, rk=3, **kw):
    """Balsara-type relativistic MHD shock tube on [-0.5, 0.5] (section
    3.2.2): left (rho, p, By) = (1, 1, 1), right (0.125, 0.1, -1), Bx = 0.5."""
    p = grid(1, CART, [n], [-0.5, 0, 0], [0.5, 1, 1], [[OUTFLOW, OUTFLOW]], gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma, **kw)
    x1, _, _ = centres(p)
    left = x1 < 0.0
    pr = empty_prim(p)
    pr[0] = np.where(left, 1.0, 0.125)
    pr[4] = np.where(left, 1.0, 0.1)
    pr[5] = 0.5
    pr[6] = np.where(left, 1.0, -1.0)
    return p, pr, flat_metric(p)


def srhd_shock_tube(n=400, gamma=5.0 / 3.0, rk=3, bx=0.0, **kw):
    """Relativistic hydro shock tube on [0, 1] (section 3.1.2): left
    (rho, p, v) = (10, 40/3, 0), right (1, 0, 0), jump at x = 0.5.  A uniform
    field parallel to the flow (bx) leaves the hydrodynamics unchanged."""
    p = grid(1, CART, [n], [0, 0, 0], [1, 1, 1], [[OUTFLOW, OUTFLOW]], gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma, **kw)
    x1, _, _ = centres(p)
    left = x1 < 0.5
    pr = empty_prim(p)
    pr[0] = np.where(left, 10.0, 1.0)
    pr[4] = np.where(left, 40.0 / 3.0, 0.0)
    pr[5] = bx
    return p, pr, flat_metric(p)


def alfven_speed2(rho=1.0, pres=0.5, gamma=5.0 / 3.0, B0=1.0, A0=1.0):
    """Square of the Alfven speed of the circularly polarised wave (section
    3.2.1)."""
    h = 1.0 + gamma / (gamma - 1.0) * pres / rho
    a = 2.0 * B0 * B0 / (rho * h + B0 * B0 * (1.0 + A0 * A0))
    return a / (1.0 + math.sqrt(1.0 - (A0 * A0 * a) ** 2))


def alfven_wave(n=128, t=0.0, rk=2, gamma=5.0 / 3.0, **kw):
    """Large-amplitude circularly polarised Alfven wave on periodic [0, 1]
    (section 3.2.1), at time t (exact solution: the initial profile moved by
    v_A t along +x)."""
    p = grid(1, CART, [n], [0, 0, 0], [1, 1, 1], [[PERIODIC, PERIODIC]], gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma, **kw)
    x1, _, _ = centres(p)
    vA = math.sqrt(alfven_speed2(gamma=gamma))
    k = 2.0 * math.pi
    ph = k * (x1 - vA * t)
    A0, B0 = 1.0, 1.0
    vy = -vA * A0 * np.cos(ph)
    vz = -vA * A0 * np.sin(ph)
    W = 1.0 / np.sqrt(1.0 - vy * vy - vz * vz)
    pr = empty_prim(p)
    pr[0] = 1.0
    pr[4] = 0.5
    pr[2] = W * vy
    pr[3] = W * vz
    pr[5] = B0
    pr[6] = A0 * B0 * np.cos(ph)
    pr[7] = A0 * B0 * np.sin(ph)
    return p, pr, flat_metric(p)


def smooth_wave_2d(n=32, t=0.0, rk=2, gamma=5.0 / 3.0, A=0.2, v0=0.2, theta=math.pi / 6):
    """Two-dimensional advected sine wave on [0, 3/sqrt 2] x [0, 2] with
    N x 2N cells (section 3.1.1).  Boundary ghosts hold the exact solution
    (BC NONE: the caller refreshes them)."""
    p = grid(2, CART, [n, 2 * n], [0, 0, 0], [3.0 / math.sqrt(2.0), 2.0, 1.0], [[NONE, NONE], [NONE, NONE]],
             gamma=gamma, rk=rk, rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma)
    return p, smooth_wave_prim(p, t, A, v0, theta), flat_metric(p)


def smooth_wave_prim(p, t, A=0.2, v0=0.2, theta=math.pi / 6):
    x1, x2, _ = centres(p)
    W = 1.0 / math.sqrt(1.0 - v0 * v0)
    pr = empty_prim(p)
    ph = 2.0 * math.pi * ((x1 * math.cos(theta) + x2 * math.sin(theta)) - v0 * math.cos(theta) * t)
    pr[0] = 1.0 + A * np.sin(ph)
    pr[4] = 1.0
    pr[1] = W * v0
    return pr


def periodic_wave_3d(n=16, gamma=5.0 / 3.0, rk=3, bfield=(0.3, 0.2, 0.1), vel=(0.2, -0.1, 0.15)):
    """Smooth periodic 3D state: rho = 1 + 0.2 sin(2 pi k.x), uniform p, v, B."""
    p = grid(3, CART, [n, n, n], [0, 0, 0], [1, 1, 1], [[PERIODIC, PERIODIC]] * 3, gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma)
    x1, x2, x3 = centres(p)
    pr = empty_prim(p)
    pr[0] = 1.0 + 0.2 * np.sin(2 * math.pi * (x1 + x2 + x3))
    v2 = sum(v * v for v in vel)
    W = 1.0 / math.sqrt(1.0 - v2)
    for a in range(3):
        pr[1 + a] = W * vel[a]
        pr[5 + a] = bfield[a]
    pr[4] = 1.0
    return p, pr, flat_metric(p)


# ------------------------------------------------------------------ blast

def blast_wave_3d(n=256, seed=0, gamma=4.0 / 3.0, rk=3, **kw):
    """Relativistic magnetised blast wave in [-0.5, 0.5]^3: p = 1 inside
    r <= 0.1 and 0.01 outside, rho = 0.01 (1 + 1e-4 u) with u in [-1, 1) from
    the counter-based generator, v = 0, B = (0.1, 0, 0), Gamma = 4/3
    (a 3D variant of the cylindrical blast wave of section 3.2.3)."""
    p = grid(3, CART, [n, n, n], [-0.5] * 3, [0.5] * 3, [[OUTFLOW, OUTFLOW]] * 3, gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma, **kw)
    return p, blast_prim(p, seed), flat_metric(p)


def blast_prim(p, seed=0, r_in=0.1, p_in=1.0, p_out=0.01, rho0=0.01, bx=0.1):
    x1, x2, x3 = centres(p)
    r = np.sqrt(x1 * x1 + x2 * x2 + x3 * x3)
    u = uniform(seed, global_index(p))
    pr = empty_prim(p)
    pr[0] = rho0 * (1.0 + 1e-4 * u)
    pr[4] = np.where(r <= r_in, p_in, p_out)
    pr[5] = bx
    return pr


def blast_wave_2d(n=128, seed=0, gamma=4.0 / 3.0, rk=3, **kw):
    """2D Cartesian blast wave of the same kind as blast_wave_3d."""
    p = grid(2, CART, [n, n], [-0.5, -0.5, 0], [0.5, 0.5, 1], [[OUTFLOW, OUTFLOW]] * 2, gamma=gamma, rk=rk,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma, **kw)
    return p, blast_prim(p, seed), flat_metric(p)


# ------------------------------------------------------ near-vacuum flows

def receding_flow(coord=CART, ndim=1, n=(16, 1, 1), axis=0, centre=None, width=1, rho_low=1e-8, u=2.0,
                  gamma=5.0 / 3.0, rk=3, **kw):
    """Dense fluid (rho = p = 1) moving away along `axis` with W v = u from a
    slab of `width` near-empty static cells (rho = p = rho_low) starting at
    interior index `centre` (default the middle): the flow that opens a near
    vacuum, where the high-order Euler update of the slab goes negative.
    Domains as in uniform_state; outflow boundaries, ghosts not filled."""
    if coord == CYL:
        xmin, xmax = [0.5, -1.0, 0.0], [2.5, 1.0, 2 * math.pi]
    elif coord == SPH:
        xmin, xmax = [0.5, 0.3, 0.0], [2.5, math.pi - 0.3, 2 * math.pi]
    else:
        xmin, xmax = [0, 0, 0], [1, 1, 1]
    nn = list(n[:ndim]) + [1] * (3 - ndim)
    p = grid(ndim, coord, nn, xmin, xmax, [[OUTFLOW, OUTFLOW]] * ndim, gamma=gamma, rk=rk,
             rho_atmo=1e-20, k_atmo=1.0, gamma_atmo=gamma, **kw)
    pr = empty_prim(p)
    c0 = nn[axis] // 2 if centre is None else centre
    gi = np.arange(pr.shape[3 - axis]) - ghosts(p)[axis]
    shape_ = [1, 1, 1]
    shape_[2 - axis] = -1
    gi = gi.reshape(shape_)
    slab = (gi >= c0) & (gi < c0 + width)
    pr[0] = np.where(slab, rho_low, 1.0)
    pr[4] = np.where(slab, rho_low, 1.0)
    pr[1 + axis] = np.where(gi < c0, -u, np.where(slab, 0.0, u))
    return p, pr, flat_metric(p)


def two_streams(n=200, v=0.99, gamma=5.0 / 3.0, rk=3, **kw):
    """Periodic 1D flow on [-1/2, 1/2]: the middle half moves outwards at v
    and the outer half inwards, so a near vacuum opens at x = 0 and the
    streams collide at the periodic seam (rho = 1, p = 1e-3)."""
    p = grid(1, CART, [n], [-0.5, 0, 0], [0.5, 1, 1], [[PERIODIC, PERIODIC]], gamma=gamma, rk=rk,
             rho_atmo=1e-20, k_atmo=1.0, gamma_atmo=gamma, **kw)
    x1, _, _ = centres(p)
    pr = empty_prim(p)
    Wl = 1 / math.sqrt(1 - v * v)
    pr[0] = 1.0
    pr[4] = 1e-3
    pr[1] = Wl * v * np.sign(x1) * (np.abs(x1) < 0.25) - Wl * v * np.sign(x1) * (np.abs(x1) >= 0.25)
    return p, pr, flat_metric(p)


# ------------------------------------------------------------ uniform state

def uniform_state(coord, ndim=2, n=(16, 16, 8), rho=1.0, pres=0.3, gamma=5.0 / 3.0, bfield=(0, 0, 0)):
    """A uniform static fluid in flat space in the given coordinates (the
    state that the reference-metric form must keep static to round-off)."""
    if coord == CYL:
        xmin, xmax = [0.5, -1.0, 0.0], [2.5, 1.0, 2 * math.pi]
    elif coord == SPH:
        xmin, xmax = [0.5, 0.3, 0.0], [2.5, math.pi - 0.3, 2 * math.pi]
    else:
        xmin, xmax = [0, 0, 0], [1, 1, 1]
    nn = list(n[:ndim]) + [1] * (3 - ndim)
    if ndim < 2 and coord == SPH:
        xmin[1], xmax[1] = 0.0, math.pi
    p = grid(ndim, coord, nn, xmin, xmax, [[OUTFLOW, OUTFLOW]] * ndim, gamma=gamma, rk=3,
             rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=gamma)
    pr = empty_prim(p)
    pr[0] = rho
    pr[4] = pres
    for a in range(3):
        pr[5 + a] = bfield[a]
    return p, pr, flat_metric(p)


# ------------------------------------------------------------- random states

def random_states(n, seed=0, rho=(1e-4, 10.0), eps=(1e-4, 10.0), vmax=0.95, bmax=3.0, gamma=5.0 / 3.0):
    """n random primitive states (8, n) and a random diagonal CFC metric:
    log-uniform rho and eps, |v| <= vmax in a random direction, |B| <= bmax.
    Returns (prim, psi, alpha, ref_diag[3, n])."""
    idx = np.arange(n, dtype=np.uint64)
    u = [0.5 * (uniform(seed, idx, s) + 1.0) for s in range(12)]
    lr = np.log(rho[0]) + u[0] * (np.log(rho[1]) - np.log(rho[0]))
    le = np.log(eps[0]) + u[1] * (np.log(eps[1]) - np.log(eps[0]))
    r = np.exp(lr)
    e = np.exp(le)
    psi = 1.0 + 0.5 * u[2]
    alpha = 0.5 + 0.5 * u[3]
    ref = np.stack([np.ones(n), 0.5 + 2.0 * u[4], 0.5 + 2.0 * u[5]])
    gd = psi[None] ** 4 * ref
    # velocity: random direction in an orthonormal frame, magnitude up to vmax
    vm = vmax * u[6]
    d = np.stack([2 * u[7] - 1, 2 * u[8] - 1, 2 * u[9] - 1])
    d /= np.sqrt((d * d).sum(0))[None] + 1e-300
    vu = vm[None] * d / np.sqrt(gd)
    W = 1.0 / np.sqrt(1.0 - vm * vm)
    bm = bmax * u[10]
    db = np.stack([np.cos(7 * u[11]), np.sin(7 * u[11]) * np.cos(3 * u[10]), np.sin(3 * u[11])])
    db /= np.sqrt((db * db).sum(0))[None]
    Bu = bm[None] * db / np.sqrt(gd)
    pr = np.zeros((8, n))
    pr[0] = r
    pr[1:4] = W[None] * vu
    pr[4] = (gamma - 1.0) * r * e
    pr[5:8] = Bu
    return pr, psi, alpha, ref


# -------------------------------------------------------------- TOV star

def tov_isotropic(rho_c=1.28e-3, K=100.0, Gamma=2.0, dr=1e-3):
    """Static spherical polytropic star (TOV equations, geometrised units),
    returned on a table of isotropic radius rbar: (rbar, rho, psi, alpha) and
    the gravitational mass M, the baryon mass Mb and the isotropic surface
    radius.  Integrated in areal radius with classical RK4; outside the star
    the isotropic Schwarzschild solution is used."""
    def eos(P):
        if P <= 0.0:
            return 0.0, 0.0
        rho = (P / K) ** (1.0 / Gamma)
        return rho, rho + P / (Gamma - 1.0)

    def rhs(R, y):
        m, P, nu, lnr, mb = y
        rho, e = eos(P)
        if R == 0.0:
            return np.zeros(5)
        f = 1.0 - 2.0 * m / R
        dm = 4.0 * math.pi * R * R * e
        dnu = (m + 4.0 * math.pi * R ** 3 * P) / (R * R * f)
        dP = -(e + P) * dnu
        dlnr = 1.0 / (R * math.sqrt(f))
        dmb = 4.0 * math.pi * R * R * rho / math.sqrt(f)
        return np.array([dm, dP, dnu, dlnr, dmb])

    Pc = K * rho_c ** Gamma
    ec = rho_c + Pc / (Gamma - 1.0)
    R = dr
    # series start at small R
    m0 = 4.0 / 3.0 * math.pi * R ** 3 * ec
    y = np.array([m0, Pc, 0.0, math.log(R), 4.0 / 3.0 * math.pi * R ** 3 * rho_c])
    Rs, ys = [0.0, R], [np.array([0.0, Pc, 0.0, -np.inf, 0.0]), y.copy()]
    while True:
        h = dr
        k1 = rhs(R, y)
        k2 = rhs(R + h / 2, y + h / 2 * k1)
        k3 = rhs(R + h / 2, y + h / 2 * k2)
        k4 = rhs(R + h, y + h * k3)
        yn = y + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        if yn[1] <= 0.0 or not np.isfinite(yn[1]):
            # locate the surface by linear interpolation of P
            frac = y[1] / (y[1] - yn[1]) if yn[1] < y[1] else 1.0
            h2 = h * frac
            k1 = rhs(R, y)
            k2 = rhs(R + h2 / 2, y + h2 / 2 * k1)
            k3 = rhs(R + h2 / 2, y + h2 / 2 * k2)
            yn = y + h2 / 6 * (k1 + 2 * k2 + 2 * k3)
            yn[1] = 0.0
            R = R + h2
            Rs.append(R)
            ys.append(yn)
            break
        R += h
        y = yn
        Rs.append(R)
        ys.append(y.copy())
    Rs = np.array(Rs)
    Y = np.array(ys)
    M = Y[-1, 0]
    Rsurf = Rs[-1]
    # isotropic radius: match rbar(Rsurf) to the exterior relation
    rbar_s = 0.5 * (Rsurf - M + math.sqrt(Rsurf * Rsurf - 2.0 * M * Rsurf))
    lnr = Y[:, 3].copy()
    lnr[1:] += math.log(rbar_s) - lnr[-1]
    rbar = np.concatenate([[0.0], np.exp(lnr[1:])])
    # lapse: nu shifted so that alpha matches the exterior at the surface
    nu = Y[:, 2] + 0.5 * math.log(1.0 - 2.0 * M / Rsurf) - Y[-1, 2]
    alpha = np.exp(nu)
    psi = np.empty_like(Rs)
    psi[1:] = np.sqrt(Rs[1:] / rbar[1:])
    psi[0] = psi[1] + (psi[1] - psi[2]) * 0.0 if len(psi) > 2 else psi[1]
    # psi at the centre: limit of sqrt(R/rbar) (extrapolate quadratically)
    psi[0] = psi[1] + (psi[1] - psi[2]) * (rbar[1] - rbar[0]) / (rbar[2] - rbar[1])
    rho = np.array([eos(P)[0] for P in Y[:, 1]])
    return dict(rbar=rbar, rho=rho, psi=psi, alpha=alpha, M=M, Mb=Y[-1, 4], R_areal=Rsurf, R_iso=rbar_s,
                K=K, Gamma=Gamma)


def tov_fields(star, r):
    """rho, psi, alpha of the star at isotropic radii r (any shape)."""
    r = np.abs(np.asarray(r, dtype=np.float64))
    M = star["M"]
    inside = r <= star["R_iso"]
    rho = np.where(inside, np.interp(r, star["rbar"], star["rho"]), 0.0)
    rr = np.maximum(r, 1e-300)
    psi_out = 1.0 + M / (2.0 * rr)
    alpha_out = (1.0 - M / (2.0 * rr)) / (1.0 + M / (2.0 * rr))
    psi = np.where(inside, np.interp(r, star["rbar"], star["psi"]), psi_out)
    alpha = np.where(inside, np.interp(r, star["rbar"], star["alpha"]), alpha_out)
    return rho, psi, alpha


def lapse_equation(n=256, half=200.0, rho_c=1.28e-3, K=100.0, Gamma=2.0):
    """The lapse equation of a static TOV star in deviation form on a
    Cartesian n^3 box [-half, half]^3 (the paper's metric-solver test
    domain), as an elliptic problem L(u) = Lap(u) - a (u + 1) = 0 for
    u = alpha psi - 1 with a = 2 pi psi^4 (e + 6 p) (e = rho + p / (Gamma - 1),
    p = K rho^Gamma; U + 2S of a static fluid, with the conformal factor of
    the TOV solution).  Returns the multigrid problem dict (Dirichlet faces,
    u = 0 there) and a (one ghost layer on each axis)."""
    star = tov_isotropic(rho_c, K, Gamma)
    h = 2.0 * half / n
    x = -half + (np.arange(-1, n + 1) + 0.5) * h
    p = dict(ndim=3, coord=CART, n=[n, n, n], xmin=[-half] * 3, dx=[h] * 3, bc=[[0, 0]] * 3, power=1,
             offset=1.0)
    a = np.empty((n + 2,) * 3)
    for k in range(n + 2):  # slab by slab to bound the temporaries
        r = np.sqrt(x[k] ** 2 + x[:, None] ** 2 + x[None, :] ** 2)
        rho, psi, _ = tov_fields(star, r)
        pres = K * rho ** Gamma
        a[k] = 2.0 * math.pi * psi ** 4 * (rho + pres / (Gamma - 1.0) + 6.0 * pres)
    return p, a


def rotating_star_3d(n=256, half=24.0, omega=0.01, rho_c=1.28e-3, K=100.0, Gamma=2.0, rho_atmo=1e-10, star=None):
    """Uniformly rotating polytropic star on a Cartesian n^3 box
    [-half, half]^3 for the xCFC metric solve: the TOV profile (isotropic
    coordinates) with angular velocity omega about z inside the star
    (v^x = -omega y, v^y = omega x in the Eulerian frame, W from the TOV
    conformal factor), atmosphere outside, no field.  Returns the grid
    parameters, the primitives and the TOV metric (psi, alpha; zero shift),
    built slab by slab to bound the temporaries."""
    if star is None:
        star = tov_isotropic(rho_c, K, Gamma)
    p = grid(3, CART, [n] * 3, [-half] * 3, [half] * 3, [[OUTFLOW, OUTFLOW]] * 3, gamma=Gamma, rk=3,
             rho_atmo=rho_atmo, k_atmo=K, gamma_atmo=Gamma)
    g = ghosts(p)[0]
    h = 2.0 * half / n
    x = -half + (np.arange(-g, n + g) + 0.5) * h
    shp = shape(p)
    prim = np.zeros((8,) + shp)
    met = np.zeros((5,) + shp)
    X, Y = np.meshgrid(x, x, indexing="xy")  # [j][i]
    for k in range(shp[0]):
        r = np.sqrt(X * X + Y * Y + x[k] ** 2)
        rho, psi, alpha = tov_fields(star, r)
        inside = rho > rho_atmo
        vx, vy = np.where(inside, -omega * Y, 0.0), np.where(inside, omega * X, 0.0)
        W = 1.0 / np.sqrt(1.0 - psi ** 4 * (vx * vx + vy * vy))
        rho = np.maximum(rho, rho_atmo)
        prim[0, k] = rho
        prim[1, k] = W * vx
        prim[2, k] = W * vy
        prim[4, k] = K * rho ** Gamma
        met[0, k] = psi
        met[1, k] = alpha
    return p, prim, met


def rotating_star_sph2d(nr=640, nth=64, rmax=30.0, omega=0.02, rho_c=1.28e-3, K=100.0, Gamma=2.0, rho_atmo=1e-10,
                        star=None):
    """Uniformly rotating polytropic star on an axisymmetric, equatorially
    symmetric spherical grid (r, theta) in [0, rmax] x [0, pi/2] (the layout
    of the paper's 2D rotating-star runs): TOV profile in isotropic
    coordinates, v^phi = omega inside the star (coordinate angular
    velocity, W from the TOV conformal factor), atmosphere outside, no
    field.  Returns the grid parameters, the primitives and the TOV metric
    (zero shift)."""
    if star is None:
        star = tov_isotropic(rho_c, K, Gamma)
    p = grid(2, SPH, [nr, nth], [0.0, 0.0, 0.0], [rmax, math.pi / 2, 2 * math.pi],
             [[REFLECT, OUTFLOW], [AXIS, REFLECT]], gamma=Gamma, rk=3, rho_atmo=rho_atmo, k_atmo=K,
             gamma_atmo=Gamma)
    r, th, _ = centres(p)
    rho, psi, alpha = tov_fields(star, r)
    inside = rho > rho_atmo
    rho = np.maximum(rho, rho_atmo)
    prim = np.zeros((8,) + shape(p))
    met = np.zeros((5,) + shape(p))
    vphi = np.where(inside, omega, 0.0)
    W = 1.0 / np.sqrt(1.0 - psi ** 4 * (r * np.sin(th)) ** 2 * vphi ** 2)
    prim[0] = rho
    prim[3] = W * vphi
    prim[4] = K * rho ** Gamma
    met[0], met[1] = psi, alpha
    return p, prim, met


def magnetised_star_2d(nr=256, nth=128, rmax=20.0, rho_c=1.28e-3, K=100.0, Gamma=2.0, b_peak=1e-4,
                       rho_atmo=1e-10, star=None):
    """Static magnetised polytropic star on a frozen CFC metric in 2D
    spherical (r, theta) coordinates: TOV star in isotropic coordinates, beta
    = 0, poloidal field from A_phi = A_b varpi^2 max(p - 0.04 p_max, 0)
    (discrete curl at cell centres, A_b set so that max |B| = b_peak),
    atmosphere rho_atmo with p = K rho^Gamma outside the star."""
    if star is None:
        star = tov_isotropic(rho_c, K, Gamma)
    p = grid(2, SPH, [nr, nth], [0.0, 0.0, 0.0], [rmax, math.pi, 2 * math.pi],
             [[CENTER, OUTFLOW], [AXIS, AXIS]], gamma=Gamma, rk=3, rho_atmo=rho_atmo, k_atmo=K,
             gamma_atmo=Gamma, rho_low_factor=100.0, alpha_bh=1e-2)
    r, th, _ = centres(p)
    rho, psi, alpha = tov_fields(star, r)
    rho = np.maximum(rho, rho_atmo)
    pres = K * rho ** Gamma
    met = np.zeros((5,) + shape(p))
    met[0] = psi
    met[1] = alpha
    pr = empty_prim(p)
    pr[0] = rho
    pr[4] = pres
    B = poloidal_field(p, r, th, pres, psi, b_peak)
    pr[5] = B[0]
    pr[6] = B[1]
    return p, pr, met


def poloidal_field(p, r, th, pres, psi, b_peak):
    pmax = pres.max()
    varpi = np.abs(r * np.sin(th))
    A = varpi ** 2 * np.maximum(pres - 0.04 * pmax, 0.0)
    sqrtg = psi ** 6 * r * r * np.abs(np.sin(th))
    dAdth = np.zeros_like(A)
    dAdr = np.zeros_like(A)
    dAdth[:, 1:-1, :] = (A[:, 2:, :] - A[:, :-2, :]) / (2 * p["dx"][1])
    dAdr[:, :, 1:-1] = (A[:, :, 2:] - A[:, :, :-2]) / (2 * p["dx"][0])
    with np.errstate(divide="ignore", invalid="ignore"):
        Br = np.where(sqrtg > 0, dAdth / sqrtg, 0.0)
        Bth = np.where(sqrtg > 0, -dAdr / sqrtg, 0.0)
    gd_r = psi ** 4
    gd_th = psi ** 4 * r * r
    mag = np.sqrt(gd_r * Br * Br + gd_th * Bth * Bth)
    mi = interior(p, mag).max()
    s = b_peak / mi if mi > 0 else 0.0
    return np.stack([Br * s, Bth * s])


# ----------------------------------------------------- AMR-style block set

def amr_block_params(nblocks=3000, seed=0, sizes=(8, 16, 32), rho_atmo=1e-10, K=100.0, Gamma=2.0,
                     r_range=(0.5, 18.0), box=20.0):
    """Grid descriptions of a set of independent AMR-style blocks: interior
    size n^3 with n drawn from `sizes`, coordinates Cartesian or spherical
    50/50 (counter-based draws keyed by block index).  Spherical blocks sit at
    r0 in [0.5, 18] with d_theta = d_phi = 0.02 and dr = 0.02 r0; Cartesian
    blocks lie inside [-20, 20]^3 with dx in {0.05, 0.1, 0.2}.  Outflow ghosts."""
    idx = np.arange(nblocks, dtype=np.uint64)
    u = [0.5 * (uniform(seed, idx, 100 + s) + 1.0) for s in range(8)]
    out = []
    for b in range(nblocks):
        n = sizes[min(int(u[0][b] * len(sizes)), len(sizes) - 1)]
        sph = u[1][b] < 0.5
        if sph:
            dth = 0.02
            r0 = r_range[0] + (r_range[1] - r_range[0]) * u[2][b]
            th0 = 0.05 + (np.pi - 0.1 - n * dth) * u[3][b]
            ph0 = 2 * np.pi * u[4][b]
            dr = dth * r0
            p = grid(3, SPH, [n, n, n], [r0, th0, ph0], [r0 + n * dr, th0 + n * dth, ph0 + n * dth],
                     [[OUTFLOW, OUTFLOW]] * 3)
        else:
            dx = (0.05, 0.1, 0.2)[min(int(u[5][b] * 3), 2)]
            span = n * dx
            x0 = [-box + (2 * box - span) * u[2 + a][b] for a in range(3)]
            p = grid(3, CART, [n, n, n], x0, [x0[a] + span for a in range(3)], [[OUTFLOW, OUTFLOW]] * 3)
        p.update(gamma=Gamma, rk=3, rho_atmo=rho_atmo, k_atmo=K, gamma_atmo=Gamma, rho_low_factor=100.0,
                 alpha_bh=1e-2)
        out.append(p)
    return out


def amr_block_state(p, block_index, star, seed=0, b_peak=1e-4, v_noise=1e-3):
    """Primitives and metric of one block: the star's rho, p = K rho^Gamma,
    psi, alpha at cell centres (isotropic radius), beta = 0, a dipole-like
    field of peak b_peak weighted by rho / rho_c, and a velocity of physical
    size v_noise * u, u in [-1, 1) keyed by (seed, block, cell, component)."""
    x1, x2, x3 = centres(p)
    if p["coord"] == SPH:
        r = np.abs(x1)
        cth, sth = np.cos(x2), np.sin(x2)
        scale = [np.ones_like(r), r, r * np.abs(sth)]
    else:
        r = np.sqrt(x1 * x1 + x2 * x2 + x3 * x3)
        scale = [np.ones_like(r)] * 3
    rho, psi, alpha = tov_fields(star, r)
    rho = np.maximum(rho, p["rho_atmo"])
    pr = empty_prim(p)
    pr[0] = rho
    pr[4] = p["k_atmo"] * rho ** p["gamma"]
    f = b_peak * rho / star["rho"][0]
    if p["coord"] == SPH:
        pr[5] = f * 2.0 * cth
        pr[6] = f * sth / np.maximum(r, 1e-300)
    else:
        rr = np.maximum(r * r, 1e-300)
        pr[5] = f * 3.0 * x3 * x1 / rr
        pr[6] = f * 3.0 * x3 * x2 / rr
        pr[7] = f * (3.0 * x3 * x3 - rr) / rr
    gidx = global_index(p).astype(np.uint64) + np.uint64(block_index) * np.uint64(1 << 20)
    for a in range(3):
        pr[1 + a] = v_noise * uniform(seed, gidx, 10 + a) / np.maximum(scale[a], 1e-300)
    met = np.zeros((5,) + shape(p))
    met[0] = psi
    met[1] = alpha
    return pr, met


# ---------------------------------------------------------------- serving

SERVE_RANGES = ((200, 4096), (64, 1024), (32, 128))


def serving_requests(nreq, seed=0, ranges=SERVE_RANGES):
    """A stream of independent solves: dimension 1, 2 or 3 with equal odds,
    linear size N uniform in that dimension's range (1D shock tubes of N
    cells, 2D / 3D blast waves of N^2 / N^3 cells), an input seed, and
    arrival times of a unit-rate Poisson process (divide by the rate)."""
    idx = np.arange(nreq, dtype=np.uint64)
    u = [0.5 * (uniform(seed, idx, 300 + s) + 1.0) for s in range(3)]
    out = []
    t = 0.0
    for r in range(nreq):
        kind = 1 + min(int(u[0][r] * 3), 2)
        lo, hi = ranges[kind - 1]
        n = min(lo + int(u[1][r] * (hi - lo + 1)), hi)
        t += -math.log1p(-float(u[2][r]))
        out.append({"kind": kind, "n": n, "seed": int(seed) * 1000003 + r, "arrival": t})
    return out


def serving_problem(req, device="cpu"):
    """Grid, initial primitives, metric (torch float64 tensors on `device`)
    and stopping rule of one request.  1D: the relativistic MHD shock tube
    with its jump position moved by up to 0.1 and left / right density and
    pressure scaled by up to +-10% (seeded), run to t = 0.4.  2D / 3D: the
    magnetised blast wave with seeded 1e-4 density noise, 50 steps."""
    import torch

    kind, n, seed = req["kind"], req["n"], req["seed"]
    if kind == 1:
        p = grid(1, CART, [n], [-0.5, 0, 0], [0.5, 1, 1], [[OUTFLOW, OUTFLOW]], gamma=5.0 / 3.0, rk=3,
                 rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=5.0 / 3.0)
    elif kind == 2:
        p = grid(2, CART, [n, n], [-0.5, -0.5, 0], [0.5, 0.5, 1], [[OUTFLOW, OUTFLOW]] * 2, gamma=4.0 / 3.0, rk=3,
                 rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=4.0 / 3.0)
    else:
        p = grid(3, CART, [n, n, n], [-0.5] * 3, [0.5] * 3, [[OUTFLOW, OUTFLOW]] * 3, gamma=4.0 / 3.0, rk=3,
                 rho_atmo=1e-12, k_atmo=1.0, gamma_atmo=4.0 / 3.0)
    g = ghosts(p)
    shp = shape(p)
    ax = [p["xmin"][a] + (torch.arange(-g[a], p["n"][a] + g[a], dtype=torch.float64, device=device) + 0.5) * p["dx"][a]
          for a in range(3)]
    x1 = ax[0].view(1, 1, -1).expand(shp)
    pr = torch.zeros((8,) + shp, dtype=torch.float64, device=device)
    if kind == 1:
        v = uniform(seed, np.arange(5, dtype=np.uint64), 400)
        left = x1 < 0.1 * float(v[0])
        pr[0] = torch.where(left, 1.0 * (1 + 0.1 * float(v[1])), 0.125 * (1 + 0.1 * float(v[2])))
        pr[4] = torch.where(left, 1.0 * (1 + 0.1 * float(v[3])), 0.1 * (1 + 0.1 * float(v[4])))
        pr[5] = 0.5
        pr[6] = torch.where(left, 1.0, -1.0)
        t_end, max_steps = 0.4, 0
    else:
        x2 = ax[1].view(1, -1, 1).expand(shp)
        r2 = x1 * x1 + x2 * x2
        if kind == 3:
            x3 = ax[2].view(-1, 1, 1).expand(shp)
            r2 = r2 + x3 * x3
        gen = torch.Generator(device=device)
        gen.manual_seed(seed)
        noise = torch.rand(shp, dtype=torch.float64, device=device, generator=gen) * 2.0 - 1.0
        pr[0] = 0.01 * (1.0 + 1e-4 * noise)
        pr[4] = torch.where(r2 <= 0.01, 1.0, 0.01)
        pr[5] = 0.1
        t_end, max_steps = 1e30, 50
    met = torch.zeros((5,) + shp, dtype=torch.float64, device=device)
    met[0] = 1.0
    met[1] = 1.0
    return p, pr, met, t_end, max_steps


def serving_footprint(req):
    """Device bytes of one request's state: q_n, q_s, prim (8 doubles per
    cell each) and metric (5), ghosts included."""
    n, k = req["n"], req["kind"]
    cells = (n + 4) ** k
    return cells * 29 * 8
