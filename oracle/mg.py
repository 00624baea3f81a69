"""CPU oracle of the cell-centred multigrid solver (test infrastructure only).

Plain C, FP64 (``mg_oracle.c``), loaded through ctypes; only the tests, the
smoke check and the benchmark's CPU-baseline leg use it.  A problem is a
dict: ndim, coord (0 Cartesian, 1 cylindrical, 2 spherical), n, xmin, dx,
bc (per axis a pair of 0 Dirichlet, 1 Neumann, 2 periodic, 3 Robin
d(r u)/dr = 0), levels (0: as many as the grid allows down to two cells on
the shortest axis), pre, post, coarse (sweeps), power p, offset c and
power2 q of L(u) = Lap(u) - a (u + c)^p - a2 (u + c)^q (a, a2 optional
arrays).  The vector operator Lap X^i + (1/3) d_i d_j X^j of the xCFC shift
and vector-potential equations (Cartesian grids, and axisymmetric
cylindrical and spherical grids in orthonormal components) has its own
calls (vapply, vsmooth, vsolve).  Beside the paper's red-black point
smoother, line_smooth and vline_smooth give line-relaxation sweeps.  Arrays are numpy float64 with one ghost layer
on each active axis, shape (n2 + 2 g2, n1 + 2 g1, n0 + 2 g0); vector fields
have a leading axis of 3.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libmgoracle.so")
CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared"]

CART, CYL, SPH = 0, 1, 2
DIRICHLET, NEUMANN, PERIODIC, ROBIN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("coord", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("xmin", ctypes.c_double * 3), ("dx", ctypes.c_double * 3), ("bc", (ctypes.c_int * 2) * 3),
        ("levels", ctypes.c_int), ("pre", ctypes.c_int), ("post", ctypes.c_int), ("coarse", ctypes.c_int),
        ("power", ctypes.c_int), ("offset", ctypes.c_double), ("power2", ctypes.c_int),
        ("smoother", ctypes.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.om_desc_size.restype = I
        L.om_apply.argtypes = [P, P, P, P, P]
        L.om_fill_ghosts.argtypes = [P, I, P]
        L.om_smooth.argtypes = [P, P, P, P, P, I]
        L.om_line_smooth.argtypes = [P, P, P, P, P, I]
        L.om_vline_smooth.argtypes = [P, P, P, I]
        L.om_restrict.argtypes = [P, I, P, P]
        L.om_prolong.argtypes = [P, I, P, P]
        L.om_solve.argtypes = [P, P, P, P, P, D, I, I, P]
        L.om_solve.restype = I
        L.om_vapply.argtypes = [P, P, P]
        L.om_vsmooth.argtypes = [P, P, P, I]
        L.om_vfill_ghosts.argtypes = [P, P]
        L.om_vsolve.argtypes = [P, P, P, D, I, I, P]
        L.om_vsolve.restype = I
        L.om_xcfc_aij.argtypes = [P, P, P, P]
        L.om_xcfc_beta_rhs.argtypes = [P, P, P, P, P]
        L.om_divergence.argtypes = [P, P, P]
        L.om_subtract_gradient.argtypes = [P, P, P]
        if L.om_desc_size() != ctypes.sizeof(_Desc):
            raise RuntimeError("multigrid oracle descriptor layout mismatch")
        _lib = L
    return _lib


DEFAULTS = dict(levels=0, pre=2, post=2, coarse=50, power=0, offset=0.0, power2=0, smoother=0)


def _coarsens(p, a, L):
    """Axis a still has a valid level after L halvings: divisible, at least
    two cells, and an even count on a periodic axis (with an odd count the
    cells on either side of the wrap share a colour of the red-black and
    multi-colour orderings, which then no longer separate neighbours)."""
    n = p["n"][a] >> L
    return p["n"][a] % (1 << L) == 0 and n >= 2 and (p["bc"][a][0] != PERIODIC or n % 2 == 0)


def max_levels(p):
    """Levels down to at least two cells on every active axis (an even
    number on periodic axes)."""
    L = 1
    while all(_coarsens(p, a, L) for a in range(p["ndim"])):
        L += 1
    return L


def make_desc(p):
    q = dict(DEFAULTS)
    q.update(p)
    d = _Desc()
    d.ndim, d.coord = int(q["ndim"]), int(q["coord"])
    for a in range(3):
        d.n[a] = int(q["n"][a])
        d.xmin[a] = float(q["xmin"][a])
        d.dx[a] = float(q["dx"][a])
        d.bc[a][0], d.bc[a][1] = int(q["bc"][a][0]), int(q["bc"][a][1])
    d.levels = int(q["levels"]) or max_levels(q)
    d.pre, d.post, d.coarse, d.power = int(q["pre"]), int(q["post"]), int(q["coarse"]), int(q["power"])
    d.offset = float(q["offset"])
    d.power2 = int(q["power2"])
    d.smoother = int(q["smoother"])
    for a in range(d.ndim):
        if not _coarsens(q, a, d.levels - 1):
            raise ValueError("grid not divisible for the requested levels (even counts on periodic axes)")
        for s in (0, 1):
            if d.bc[a][s] == ROBIN and ((d.coord == SPH and a != 0) or (d.coord == CYL and a == 2)):
                raise ValueError("the Robin condition is for the outer faces in r (spherical), R and z "
                                 "(cylindrical) or x, y, z (Cartesian)")
    return d


def shape(p, level=None):
    d = make_desc(p)
    s = d.levels - 1 - (d.levels - 1 if level is None else level)
    return tuple((d.n[a] >> s) + 2 if a < d.ndim else 1 for a in (2, 1, 0))


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a):
    assert a.flags.c_contiguous and a.dtype == np.float64
    return a


def _o(a):
    return _p(_c(a)) if a is not None else None


def apply(p, u, a=None, a2=None):
    """L(u) on the interior of the finest level; u's ghosts are used as given
    (fill_ghosts applies the boundary conditions)."""
    d = make_desc(p)
    out = np.zeros_like(u)
    lib().om_apply(ctypes.byref(d), _p(_c(u)), _o(a), _o(a2), _p(out))
    return out


def fill_ghosts(p, u, level=None):
    d = make_desc(p)
    lib().om_fill_ghosts(ctypes.byref(d), d.levels - 1 if level is None else level, _p(_c(u)))
    return u


def smooth(p, u, f, a=None, sweeps=1, a2=None):
    d = make_desc(p)
    lib().om_smooth(ctypes.byref(d), _p(_c(u)), _p(_c(f)), _o(a), _o(a2), sweeps)
    return u


def line_smooth(p, u, f, a=None, sweeps=1, a2=None):
    """Alternating zebra line relaxation sweeps on the finest level (the
    alternative smoother for anisotropic cells); ghosts refreshed."""
    d = make_desc(p)
    lib().om_line_smooth(ctypes.byref(d), _p(_c(u)), _p(_c(f)), _o(a), _o(a2), sweeps)
    return u


def restrict(p, level, fine):
    d = make_desc(p)
    out = np.zeros(shape(p, level - 1))
    lib().om_restrict(ctypes.byref(d), level, _p(_c(fine)), _p(out))
    return out


def prolong(p, level, coarse):
    """Kwak prolongation; the coarse ghosts are used as given."""
    d = make_desc(p)
    out = np.zeros(shape(p, level))
    lib().om_prolong(ctypes.byref(d), level, _p(_c(coarse)), _p(out))
    return out


def solve(p, u, f, a=None, tol=1e-12, max_cycles=30, fmg=True, a2=None):
    """Solve in place; returns the residual history (max norms)."""
    d = make_desc(p)
    res = np.zeros(max_cycles + 1)
    c = lib().om_solve(ctypes.byref(d), _p(_c(u)), _p(_c(f)), _o(a), _o(a2), tol, max_cycles, 1 if fmg else 0,
                       _p(res))
    return res[:c + 1]


def _cart(d):
    """Grids the vector equations take: Cartesian, or axisymmetric
    cylindrical / spherical (at most two active axes), no Robin faces; a
    spherical grid reaching r = 0 must end at theta = pi/2 (equatorial
    symmetry: the mirror of the centre is then the cell itself)."""
    if any(d.bc[a][s] == ROBIN for a in range(3) for s in (0, 1)):
        raise ValueError("the vector equations take no Robin faces")
    if d.coord != CART and d.ndim > 2:
        raise ValueError("curvilinear vector equations are axisymmetric (at most two active axes)")
    if d.coord == SPH and abs(d.xmin[0]) < 1e-12:
        if d.ndim < 2 or abs(d.xmin[1] + d.n[1] * d.dx[1] - math.pi / 2) > 1e-12:
            raise ValueError("a spherical vector grid reaching r = 0 must end at theta = pi/2")
    return d


def vapply(p, X):
    """L(X) = Lap X + (1/3) grad div X in orthonormal components on the
    interior (X: shape (3, ...), ghosts ignored: values across the boundary
    come from the boundary rule)."""
    d = _cart(make_desc(p))
    out = np.zeros_like(X)
    lib().om_vapply(ctypes.byref(d), _p(_c(X)), _p(out))
    return out


def vfill_ghosts(p, X):
    """Face ghosts of a vector field (three components) from the vector
    boundary rule."""
    d = _cart(make_desc(p))
    lib().om_vfill_ghosts(ctypes.byref(d), _p(_c(X)))
    return X


def vsmooth(p, X, f, sweeps=1):
    d = _cart(make_desc(p))
    lib().om_vsmooth(ctypes.byref(d), _p(_c(X)), _p(_c(f)), sweeps)
    return X


def vline_smooth(p, X, f, sweeps=1):
    """Line relaxation sweeps of the vector equations (components of a line
    one after the other)."""
    d = _cart(make_desc(p))
    lib().om_vline_smooth(ctypes.byref(d), _p(_c(X)), _p(_c(f)), sweeps)
    return X


def vsolve(p, X, f, tol=1e-12, max_cycles=30, fmg=True):
    d = _cart(make_desc(p))
    res = np.zeros(max_cycles + 1)
    c = lib().om_vsolve(ctypes.byref(d), _p(_c(X)), _p(_c(f)), tol, max_cycles, 1 if fmg else 0, _p(res))
    return res[:c + 1]


def xcfc_aij(p, X):
    """A~^ij from X (six components xx, yy, zz, xy, xz, yz) and A~_ij A~^ij."""
    d = _cart(make_desc(p))
    A6 = np.zeros((6,) + X.shape[1:])
    a2 = np.zeros(X.shape[1:])
    lib().om_xcfc_aij(ctypes.byref(d), _p(_c(X)), _p(A6), _p(a2))
    return A6, a2


def xcfc_beta_rhs(p, w, S, A6):
    """16 pi w S_i + 2 A~^ij d_j w on the interior (w's ghosts as given)."""
    d = _cart(make_desc(p))
    out = np.zeros_like(S)
    lib().om_xcfc_beta_rhs(ctypes.byref(d), _p(_c(w)), _p(_c(S)), _p(_c(A6)), _p(out))
    return out


def divergence(p, q):
    d = make_desc(p)
    out = np.zeros(q.shape[1:])
    lib().om_divergence(ctypes.byref(d), _p(_c(q)), _p(out))
    return out


def subtract_gradient(p, u, q):
    d = make_desc(p)
    lib().om_subtract_gradient(ctypes.byref(d), _p(_c(u)), _p(_c(q)))
    return q


def interior(p, a):
    g = [1 if ax < p["ndim"] else 0 for ax in range(3)]
    sl = tuple(slice(g[ax], a.shape[-3 + (2 - ax)] - g[ax]) for ax in (2, 1, 0))
    return a[(Ellipsis,) + sl]


def centres(p, level=None):
    d = make_desc(p)
    s = d.levels - 1 - (d.levels - 1 if level is None else level)
    ax = []
    for a in range(3):
        g = 1 if a < d.ndim else 0
        n = (d.n[a] >> s) if a < d.ndim else 1
        h = d.dx[a] * (1 << s) if a < d.ndim else d.dx[a]
        ax.append(d.xmin[a] + (np.arange(-g, n + g) + 0.5) * h)
    x3, x2, x1 = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x1, x2, x3


def xcfc_solve(pv, ps, pa, U, S, stilde, X, u_psi, u_ap, beta, tol=1e-12, max_cycles=60):
    """The xCFC metric solve of section 2.6 on the grids of pv, ps, pa
    (Cartesian, or axisymmetric cylindrical and spherical in orthonormal
    components), steps 1 to 6
    in the paper's order, on multigrid-layout arrays:
      1. L(X)^i = 8 pi S~_i                          (vector problem pv)
      2. A~^ij from X, A2 = A~_ij A~^ij
      3. Lap(psi - 1) = -2 pi U~ / psi - (1/8) A2 psi^-7
                                 (ps: power -1, power2 -7, offset 1)
      4. S~ = stilde(psi) with the new psi
      5. Lap(alpha psi - 1) = (alpha psi) [2 pi (U~ + 2 S~) psi^-2
                                           + (7/8) A2 psi^-8]  (pa: power 1, offset 1)
      6. L(beta)^i = 16 pi w S~_i + 2 A~^ij d_j w,  w = alpha psi^-6
    U: U~; S: S~_i (shape (3, ...)); X, beta: initial guesses in, solutions
    out; u_psi = psi - 1 and u_ap = alpha psi - 1: initial guesses in,
    solutions out (ghosts filled).  Returns psi, alpha (ghosts from the
    boundary rules) and the cycles of the four solves."""
    cyc = []
    zero = np.zeros_like(U)
    cyc.append(len(vsolve(pv, X, np.ascontiguousarray(8.0 * math.pi * S), tol, max_cycles)) - 1)
    A6, A2 = xcfc_aij(pv, X)
    a = np.ascontiguousarray(-2.0 * math.pi * U)
    a2 = np.ascontiguousarray(-A2 / 8.0)
    cyc.append(len(solve(ps, u_psi, zero, a, tol, max_cycles, a2=a2)) - 1)
    fill_ghosts(ps, u_psi)
    psi = 1.0 + u_psi
    St = stilde(psi)
    a = np.ascontiguousarray(2.0 * math.pi * (U + 2.0 * St) / psi ** 2 + 7.0 / 8.0 * A2 * psi ** -8)
    cyc.append(len(solve(pa, u_ap, zero, a, tol, max_cycles)) - 1)
    fill_ghosts(pa, u_ap)
    alpha = (1.0 + u_ap) / psi
    w = np.ascontiguousarray(alpha * psi ** -6)
    cyc.append(len(vsolve(pv, beta, xcfc_beta_rhs(pv, w, S, A6), tol, max_cycles)) - 1)
    return psi, alpha, cyc


# ------------------------------------------- metric of a GRMHD state

def _layout(hp):
    """Interior slices of the GRMHD layout (ng ghost layers on active axes)."""
    g = [hp.get("ng", 2) if a < hp["ndim"] else 0 for a in range(3)]
    return tuple(slice(g[a], g[a] + hp["n"][a]) for a in (2, 1, 0))


def _to_mg(p, hp, a):
    out = np.zeros(shape(p))
    out[interior_slices(p)] = a[_layout(hp)]
    return out


def interior_slices(p):
    g = [1 if ax < p["ndim"] else 0 for ax in range(3)]
    return tuple(slice(g[ax], g[ax] + p["n"][ax]) for ax in (2, 1, 0))


def vodd(p, a, side):
    """Components (bit q) odd across the non-periodic face (a, side) for the
    vector equations: Dirichlet all; Neumann the normal one, plus phi at the
    cylindrical and polar axes and every component at the spherical centre."""
    kind = p["bc"][a][side]
    if kind == DIRICHLET:
        return 7
    odd = 1 << a
    fpos = p["xmin"][a] if side == 0 else p["xmin"][a] + p["n"][a] * p["dx"][a]
    if p["coord"] == CYL and a == 0 and abs(fpos) < 1e-12:
        odd |= 4
    if p["coord"] == SPH and a == 0 and abs(fpos) < 1e-12:
        odd = 7
    if p["coord"] == SPH and a == 1 and (abs(fpos) < 1e-12 or abs(fpos - math.pi) < 1e-12):
        odd |= 4
    return odd


def hscale(hp, c):
    """Scale factor h_c of the reference metric at the (signed) cell centres
    of the GRMHD layout: orthonormal component = h_c times the
    contravariant one, the covariant one divided by h_c."""
    g = [hp.get("ng", 2) if a < hp["ndim"] else 0 for a in range(3)]
    x = [hp["xmin"][a] + (np.arange(-g[a], hp["n"][a] + g[a]) + 0.5) * hp["dx"][a] for a in range(3)]
    x3, x2, x1 = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    if hp["coord"] == CYL and c == 2:
        return x1
    if hp["coord"] == SPH and c == 1:
        return x1
    if hp["coord"] == SPH and c == 2:
        return x1 * np.sin(x2)
    return np.ones_like(x1)


def extend(hp, p, u, comp=None):
    """A multigrid solution u (interior used) on every cell of the GRMHD
    layout of hp (ng ghost layers): each ghost layer from the boundary rule
    applied per layer, axis by axis (mirror about the face times -1 for
    Dirichlet, +1 for Neumann, r_in / r_ghost for Robin; periodic wrap).
    With comp, u is that orthonormal component of a vector field and the
    mirror takes the component's parity (vodd)."""
    ng = hp.get("ng", 2)
    nd = p["ndim"]
    v = u[interior_slices(p)]
    # cell-centre coordinates along each axis of the array as it grows
    xs = [p["xmin"][a] + (np.arange(p["n"][a]) + 0.5) * p["dx"][a] if a < nd else np.zeros(1) for a in range(3)]
    for a in range(nd):
        ax = 2 - a
        n = p["n"][a]
        idx = np.arange(-ng, n + ng)
        src = idx.copy()
        fac = np.ones(idx.size)
        sel_r = np.zeros(idx.size, bool)
        for side in (0, 1):
            sel = idx < 0 if side == 0 else idx >= n
            kind = p["bc"][a][side]
            if kind == PERIODIC:
                src[sel] = idx[sel] % n
                continue
            inn = -1 - idx[sel] if side == 0 else 2 * n - 1 - idx[sel]
            src[sel] = inn
            if comp is not None:
                if (vodd(p, a, side) >> comp) & 1:
                    fac[sel] = -1.0
            elif kind == DIRICHLET:
                fac[sel] = -1.0
            elif kind == ROBIN and p["coord"] == SPH:
                x0, h = p["xmin"][0], p["dx"][0]
                fac[sel] = (x0 + (inn + 0.5) * h) / (x0 + (idx[sel] + 0.5) * h)
            elif kind == ROBIN:
                sel_r |= sel
        shp = [1, 1, 1]
        shp[ax] = -1
        v = np.take(v, src, axis=ax) * fac.reshape(shp)
        xa = p["xmin"][a] + (idx + 0.5) * p["dx"][a]
        if sel_r.any():
            # Cartesian / cylindrical Robin: r_in / r_ghost with the other
            # coordinates of the cell as the array holds them at this stage
            # (cylindrical distance from R and z)
            X = np.meshgrid(*[xa[src + ng] if b == a else xs[b] for b in (2, 1, 0)], indexing="ij")
            G = np.meshgrid(*[xa if b == a else xs[b] for b in (2, 1, 0)], indexing="ij")
            nb = min(nd, 2) if p["coord"] == CYL else nd
            rin = np.sqrt(sum(X[2 - b] ** 2 for b in range(nb)))
            rg = np.sqrt(sum(G[2 - b] ** 2 for b in range(nb)))
            f = np.where(sel_r.reshape(shp), rin / rg, 1.0)
            v = v * f
        xs[a] = xa
    return v


def fluid_stilde_curvilinear(hp, psi, prim):
    """S~ = psi^6 (rho h W^2 v^2 + 3 p) on the GRMHD layout with
    W^2 v^2 = psi^4 gamma^_ij (W v^i)(W v^j), gamma^ the reference metric
    (Cartesian, cylindrical (R, z, phi) or spherical (r, theta, phi))."""
    g = [hp.get("ng", 2) if a < hp["ndim"] else 0 for a in range(3)]
    x = [hp["xmin"][a] + (np.arange(-g[a], hp["n"][a] + g[a]) + 0.5) * hp["dx"][a] for a in range(3)]
    x3, x2, x1 = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    one = np.ones_like(x1)
    if hp["coord"] == CYL:
        g11, g22, g33 = one, one, x1 * x1
    elif hp["coord"] == SPH:
        g11, g22, g33 = one, x1 * x1, (x1 * np.sin(x2)) ** 2
    else:
        g11, g22, g33 = one, one, one
    gam = hp["gamma"]
    rho, p = prim[0], prim[4]
    w2v2 = psi ** 4 * (g11 * prim[1] ** 2 + g22 * prim[2] ** 2 + g33 * prim[3] ** 2)
    return psi ** 6 * ((rho + gam / (gam - 1.0) * p) * w2v2 + 3.0 * p)


def stilde_fn(hp, pv, prim):
    """S~ as a function of psi on the multigrid layout of pv, for the GRMHD
    state prim: fluid_stilde_curvilinear on the interior cells, 0 on the
    multigrid ghosts."""
    L, I = _layout(hp), interior_slices(pv)

    def f(ps_):
        full = np.ones_like(prim[0])
        full[L] = ps_[I]
        out = np.zeros(shape(pv))
        out[I] = fluid_stilde_curvilinear(hp, full, prim)[L]
        return out

    return f


def metric_update(hp, ppsi, palpha, q, prim, met, tol=1e-12, max_cycles=60, pvec=None, X=None):
    """The metric of a GRMHD state re-solved from its conserved variables
    (section 2.6), then the primitives recovered on the new metric (section
    2.5): with pvec the xCFC sequence (xcfc_solve in orthonormal components:
    S~_i / h_i in, the shift's contravariant components beta / h_i out; X
    in/out), else the scalar CFC equations for psi and
    alpha psi with the shift left as it is (U~ = q_tau + q_D, S~ from the
    current primitives and the new psi).  met (psi, alpha, beta on every
    cell of the layout) is updated in place, ghost layers by the boundary
    rule of each equation applied per layer; q is corrected by the recovery.
    Returns (q, prim with its ghosts filled, flags, nfatal, cycles)."""
    import oracle as og
    L = _layout(hp)
    p0 = pvec if pvec is not None else ppsi
    U = _to_mg(p0, hp, q[4] + q[0])
    up = _to_mg(ppsi, hp, met[0] - 1.0)
    cyc = [0, 0, 0, 0]
    if pvec is not None:
        hs = [hscale(hp, c) for c in range(3)]
        S = np.ascontiguousarray(np.stack([_to_mg(pvec, hp, q[1 + c] / hs[c]) for c in range(3)]))
        beta = np.ascontiguousarray(np.stack([_to_mg(pvec, hp, met[2 + c] * hs[c]) for c in range(3)]))
        # initial guess of alpha psi from the metric as given (the converged
        # solution does not depend on it beyond the tolerance)
        ua = _to_mg(palpha, hp, met[1] * met[0] - 1.0)
        _, _, cyc = xcfc_solve(pvec, ppsi, palpha, U, S, stilde_fn(hp, pvec, prim), X, up, ua, beta, tol,
                               max_cycles)
        met[0] = 1.0 + extend(hp, ppsi, up)
        met[1] = (1.0 + extend(hp, palpha, ua)) / met[0]
        for c in range(3):
            met[2 + c] = extend(hp, pvec, beta[c], comp=c) / hs[c]
    else:
        zero = np.zeros_like(U)
        cyc[1] = len(solve(ppsi, up, zero, np.ascontiguousarray(-2.0 * math.pi * U), tol, max_cycles)) - 1
        met[0] = 1.0 + extend(hp, ppsi, up)
        St = fluid_stilde_curvilinear(hp, met[0], prim)
        a = np.zeros_like(U)
        a[interior_slices(ppsi)] = (2.0 * math.pi * (q[4] + q[0] + 2.0 * St) / met[0] ** 2)[L]
        ua = _to_mg(palpha, hp, met[1] * met[0] - 1.0)
        cyc[2] = len(solve(palpha, ua, zero, a, tol, max_cycles)) - 1
        met[1] = (1.0 + extend(hp, palpha, ua)) / met[0]
    qc, pr, flags, nf = og.c2p(hp, q, met)
    og.fill_ghosts(hp, pr)
    return qc, pr, flags, nf, cyc


def psi_residual(hp, ppsi, q, met, pvec=None, X=None):
    """max |L(psi - 1)| of the conformal-factor equation of section 2.6 with
    the metric as given (its interior) and U~ = q_tau + q_D; with pvec and X
    the A2 psi^-7 term from X."""
    U = _to_mg(ppsi, hp, q[4] + q[0])
    u = _to_mg(ppsi, hp, met[0] - 1.0)
    fill_ghosts(ppsi, u)
    a2 = None
    if pvec is not None:
        a2 = np.ascontiguousarray(-xcfc_aij(pvec, X)[1] / 8.0)
    L = apply(ppsi, u, np.ascontiguousarray(-2.0 * math.pi * U), a2)
    return float(np.abs(L[interior_slices(ppsi)]).max())
