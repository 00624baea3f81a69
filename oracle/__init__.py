"""CPU oracle of the Gmunu GRMHD finite-volume step (test infrastructure only).

Plain C, FP64 (``gmunu_oracle.c``), loaded through ctypes.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import this
package; the GPU path never does.  Grid descriptions are plain dicts (see
``workloads``); arrays are numpy float64 of shape (8, nt2, nt1, nt0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmunu_oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared"]

FLAG_ATMO, FLAG_EPS_CLAMP, FLAG_V_CLAMP = 1, 2, 4
FLAG_FATAL_RHO, FLAG_FATAL_EPS, FLAG_FATAL_V, FLAG_NOCONV = 8, 16, 32, 64


_LIB_OMP = os.path.join(_HERE, "_build", "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so (single
    threaded: the checker), and the same source with -fopenmp into
    liboracle_omp.so (its per-cell loops on all host cores: only for the
    all-cores CPU timing)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC) and \
            os.path.exists(_LIB_OMP) and os.path.getmtime(_LIB_OMP) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, out)
    return _LIB


def threads() -> int:
    """Threads of the loaded build's per-cell loops."""
    return int(lib().og_threads())


def use_openmp(on: bool):
    """Route the oracle's calls to the all-cores build (on) or back to the
    single-threaded one; results are the same (cells are independent and the
    time-step maximum is exact)."""
    global _lib, _LIB
    want = _LIB_OMP if on else os.path.join(_HERE, "_build", "liboracle.so")
    if _LIB != want:
        _LIB = want
        _lib = None


class _Desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("coord", ctypes.c_int), ("n", ctypes.c_int * 3), ("ng", ctypes.c_int),
        ("xmin", ctypes.c_double * 3), ("dx", ctypes.c_double * 3),
        ("bc", (ctypes.c_int * 2) * 3),
        ("gamma", ctypes.c_double),
        ("rho_atmo", ctypes.c_double), ("k_atmo", ctypes.c_double), ("gamma_atmo", ctypes.c_double),
        ("rho_low_factor", ctypes.c_double), ("alpha_bh", ctypes.c_double),
        ("rho_max", ctypes.c_double), ("eps_max", ctypes.c_double), ("w_max", ctypes.c_double),
        ("c2p_maxit", ctypes.c_int), ("c2p_tol", ctypes.c_double),
        ("rk", ctypes.c_int),
        ("recon", ctypes.c_int), ("riemann", ctypes.c_int), ("pp", ctypes.c_int), ("c2p", ctypes.c_int),
    ]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.og_desc_size.restype = ctypes.c_int
        L.og_threads.restype = ctypes.c_int
        L.og_ntot.restype = ctypes.c_long
        L.og_ntot.argtypes = [P]
        L.og_index.restype = ctypes.c_long
        L.og_index.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.og_prim2con.argtypes = [P, P, P, P]
        L.og_c2p.argtypes = [P, P, P, P, P]
        L.og_c2p.restype = ctypes.c_long
        L.og_fill_ghosts.argtypes = [P, P]
        L.og_rhs.argtypes = [P, P, P, P]
        L.og_rhs_cells.argtypes = [P, P, P, ctypes.c_long, P, P]
        L.og_rhs_k.argtypes = [P, P, P, P, P]
        L.og_rhs_cells_k.argtypes = [P, P, P, P, ctypes.c_long, P, P]
        L.og_rhs_scale_cells_k.argtypes = [P, P, P, P, ctypes.c_long, P, P]
        L.og_rk_stage_k.argtypes = [P, ctypes.c_int, ctypes.c_double, P, P, P, P, P, P]
        L.og_rk_stage_k.restype = ctypes.c_long
        L.og_sources_cell.argtypes = [P, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
        L.og_rhs_scale_cells.argtypes = [P, P, P, ctypes.c_long, P, P]
        L.og_cfl_dt.argtypes = [P, P, P, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.og_cfl_dt.restype = ctypes.c_double
        L.og_rk_stage.argtypes = [P, ctypes.c_int, ctypes.c_double, P, P, P, P, P]
        L.og_rk_stage.restype = ctypes.c_long
        L.og_rk_update.argtypes = [P, ctypes.c_int, ctypes.c_double, P, P, P, P]
        L.og_evolve.argtypes = [P, P, P, P, ctypes.c_double, P, ctypes.c_double, ctypes.c_long, P]
        L.og_evolve.restype = ctypes.c_long
        L.og_point_prim2con.argtypes = [ctypes.c_double, P, P, P, P]
        L.og_point_flux.argtypes = [ctypes.c_double, P, P, P, ctypes.c_int, P, P]
        L.og_c2p_point.argtypes = [P, P, ctypes.c_double, ctypes.c_double, P, P, P]
        L.og_c2p_point.restype = ctypes.c_int
        L.og_cell_geometry.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        L.og_cell_volumes.argtypes = [P, P]
        L.og_mc_faces.argtypes = [ctypes.c_int, P, P, P]
        L.og_mp5_faces.argtypes = [ctypes.c_int, P, P, P]
        L.og_ppm_faces.argtypes = [ctypes.c_int, P, P, P]
        L.og_point_hlle.argtypes = [ctypes.c_double, P, P, P, P, ctypes.c_int, P]
        L.og_point_tvdlf.argtypes = [ctypes.c_double, P, P, P, P, ctypes.c_int, P]
        if L.og_desc_size() != ctypes.sizeof(_Desc):
            raise RuntimeError("oracle descriptor layout mismatch")
        _lib = L
    return _lib


DEFAULTS = dict(ng=2, gamma=5.0 / 3.0, rho_atmo=1e-12, k_atmo=100.0, gamma_atmo=2.0,
                rho_low_factor=100.0, alpha_bh=1e-2, rho_max=float("inf"), eps_max=float("inf"),
                w_max=1e3, c2p_maxit=200, c2p_tol=1e-15, rk=3, recon=0, riemann=0, pp_limiter=0, c2p=0)


def make_desc(p: dict) -> _Desc:
    """Oracle descriptor from a plain parameter dict."""
    q = dict(DEFAULTS)
    q.update(p)
    d = _Desc()
    d.ndim, d.coord, d.ng = int(q["ndim"]), int(q["coord"]), int(q["ng"])
    for a in range(3):
        d.n[a] = int(q["n"][a])
        d.xmin[a] = float(q["xmin"][a])
        d.dx[a] = float(q["dx"][a])
        d.bc[a][0] = int(q["bc"][a][0])
        d.bc[a][1] = int(q["bc"][a][1])
    for k in ("gamma", "rho_atmo", "k_atmo", "gamma_atmo", "rho_low_factor", "alpha_bh", "rho_max",
              "eps_max", "w_max", "c2p_tol"):
        setattr(d, k, float(q[k]))
    d.c2p_maxit, d.rk = int(q["c2p_maxit"]), int(q["rk"])
    d.recon, d.riemann, d.pp, d.c2p = int(q["recon"]), int(q["riemann"]), int(q["pp_limiter"]), int(q["c2p"])
    if d.recon in (1, 2) and d.ng < 3:
        raise ValueError("MP5 and PPM need three ghost layers (ng = 3)")
    return d


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _ref(d):
    return ctypes.byref(d)


def shape(p: dict):
    d = make_desc(p)
    g = [d.ng if a < d.ndim else 0 for a in range(3)]
    return (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])


def _chk(a, nv=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


def prim2con(p, prim, metric):
    d = make_desc(p)
    prim, metric = _chk(prim), _chk(metric)
    q = np.zeros_like(prim)
    lib().og_prim2con(_ref(d), _p(prim), _p(metric), _p(q))
    return q


def c2p(p, q, metric):
    """Returns (q_corrected, prim, flags, nfatal); ghosts of prim are zero."""
    d = make_desc(p)
    q = _chk(q).copy()
    metric = _chk(metric)
    prim = np.zeros_like(q)
    flags = np.zeros(q.shape[1:], dtype=np.uint8)
    nf = lib().og_c2p(_ref(d), _p(q), _p(metric), _p(prim), _p(flags))
    return q, prim, flags, int(nf)


def fill_ghosts(p, prim):
    d = make_desc(p)
    assert prim.flags.c_contiguous and prim.dtype == np.float64
    lib().og_fill_ghosts(_ref(d), _p(prim))
    return prim


def rhs(p, prim, metric, kij=None):
    d = make_desc(p)
    prim, metric, kij = _chk(prim), _chk(metric), _kij(kij)
    out = np.zeros_like(prim)
    lib().og_rhs_k(_ref(d), _p(prim), _p(metric), None if kij is None else _p(kij), _p(out))
    return out


def _kij(kij):
    """K_ij (6 arrays xx, xy, xz, yy, yz, zz in the grid's layout) or None."""
    return None if kij is None else _chk(kij)


def rhs_cells(p, prim, metric, ijk, kij=None):
    d = make_desc(p)
    prim, metric, kij = _chk(prim), _chk(metric), _kij(kij)
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((ijk.shape[0], 8))
    lib().og_rhs_cells_k(_ref(d), _p(prim), _p(metric), None if kij is None else _p(kij), ijk.shape[0], _p(ijk),
                         _p(out))
    return out


def rhs_scale_cells(p, prim, metric, ijk, kij=None):
    d = make_desc(p)
    prim, metric, kij = _chk(prim), _chk(metric), _kij(kij)
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    out = np.zeros((ijk.shape[0], 8))
    lib().og_rhs_scale_cells_k(_ref(d), _p(prim), _p(metric), None if kij is None else _p(kij), ijk.shape[0],
                               _p(ijk), _p(out))
    return out


def sources_cell(p, prim, metric, i, j, k, kij=None):
    """(gravitational, geometric) source vectors of interior cell (i, j, k)."""
    d = make_desc(p)
    prim, metric, kij = _chk(prim), _chk(metric), _kij(kij)
    g, e = np.zeros(8), np.zeros(8)
    lib().og_sources_cell(_ref(d), _p(prim), _p(metric), None if kij is None else _p(kij), i, j, k, _p(g), _p(e))
    return g, e


def cfl_dt(p, prim, metric, cfl, t=0.0, t_end=float("inf")):
    d = make_desc(p)
    return float(lib().og_cfl_dt(_ref(d), _p(_chk(prim)), _p(_chk(metric)), cfl, t, t_end))


def rk_stage(p, stage, dt, qn, qs, prim, metric, flags=None, kij=None):
    d = make_desc(p)
    for a in (qn, qs, prim):
        assert a.flags.c_contiguous and a.dtype == np.float64
    metric, kij = _chk(metric), _kij(kij)
    fp = _p(flags) if flags is not None else None
    return int(lib().og_rk_stage_k(_ref(d), stage, dt, _p(qn), _p(qs), _p(prim), _p(metric),
                                   None if kij is None else _p(kij), fp))


def rk_update(p, stage, dt, qn, qs, prim, metric):
    """The stage's new conserved state in qs before the recovery."""
    d = make_desc(p)
    for a in (qn, qs, prim):
        assert a.flags.c_contiguous and a.dtype == np.float64
    metric = _chk(metric)
    lib().og_rk_update(_ref(d), stage, dt, _p(qn), _p(qs), _p(prim), _p(metric))


def evolve(p, q, prim, metric, cfl, t=0.0, t_end=float("inf"), nsteps=1 << 60):
    """Advance q and prim in place; returns (steps, t, nfatal)."""
    d = make_desc(p)
    for a in (q, prim):
        assert a.flags.c_contiguous and a.dtype == np.float64
    metric = _chk(metric)
    tt = ctypes.c_double(t)
    nf = ctypes.c_long(0)
    s = lib().og_evolve(_ref(d), _p(q), _p(prim), _p(metric), cfl, ctypes.byref(tt), t_end, nsteps,
                        ctypes.byref(nf))
    return int(s), tt.value, nf.value


def point_prim2con(gamma, prim8, met5, ref3):
    pr = np.ascontiguousarray(prim8, dtype=np.float64)
    m = np.ascontiguousarray(met5, dtype=np.float64)
    r = np.ascontiguousarray(ref3, dtype=np.float64)
    q = np.zeros(8)
    lib().og_point_prim2con(gamma, _p(pr), _p(m), _p(r), _p(q))
    return q


def point_flux(gamma, prim8, met5, ref3, axis):
    pr = np.ascontiguousarray(prim8, dtype=np.float64)
    m = np.ascontiguousarray(met5, dtype=np.float64)
    r = np.ascontiguousarray(ref3, dtype=np.float64)
    f = np.zeros(8)
    lam = np.zeros(2)
    lib().og_point_flux(gamma, _p(pr), _p(m), _p(r), axis, _p(f), _p(lam))
    return f, lam


def c2p_point(p, q8, psi, alpha, ref3):
    """Returns (prim8, flags, iterations)."""
    d = make_desc(p)
    q = np.ascontiguousarray(q8, dtype=np.float64)
    r = np.ascontiguousarray(ref3, dtype=np.float64)
    pr = np.zeros(8)
    it = ctypes.c_int(0)
    fl = lib().og_c2p_point(_ref(d), _p(q), psi, alpha, _p(r), _p(pr), ctypes.byref(it))
    return pr, int(fl), it.value


def cell_geometry(p, i, j, k):
    d = make_desc(p)
    out = np.zeros(12)
    lib().og_cell_geometry(_ref(d), i, j, k, _p(out))
    return out


def cell_volumes(p):
    d = make_desc(p)
    out = np.zeros(shape(p))
    lib().og_cell_volumes(_ref(d), _p(out))
    return out


def interior(p, a):
    """View of the interior cells of a (nv, nt2, nt1, nt0) or (nt2, nt1, nt0) array."""
    d = make_desc(p)
    g = [d.ng if ax < d.ndim else 0 for ax in range(3)]
    sl = (slice(g[2], g[2] + d.n[2]), slice(g[1], g[1] + d.n[1]), slice(g[0], g[0] + d.n[0]))
    return a[(Ellipsis,) + sl]


def mp5_faces(u):
    """MP5 face values on a line: (left, right) states at the n-5 faces
    between cells f and f+1, f = 2..n-4."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.shape[0]
    lo, hi = np.zeros(n - 5), np.zeros(n - 5)
    lib().og_mp5_faces(n, _p(u), _p(lo), _p(hi))
    return lo, hi


def ppm_faces(u):
    """PPM face values on a line: (left, right) states at the n-5 faces
    between cells f and f+1, f = 2..n-4."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.shape[0]
    lo, hi = np.zeros(n - 5), np.zeros(n - 5)
    lib().og_ppm_faces(n, _p(u), _p(lo), _p(hi))
    return lo, hi


def mc_faces(u):
    """MC face values on a line: (left, right) states at the n-3 faces
    between cells f and f+1, f = 1..n-3."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    n = u.shape[0]
    lo, hi = np.zeros(n - 3), np.zeros(n - 3)
    lib().og_mc_faces(n, _p(u), _p(lo), _p(hi))
    return lo, hi


def point_hlle(gamma, pl, pr, met5, ref3, axis):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (pl, pr, met5, ref3)]
    f = np.zeros(8)
    lib().og_point_hlle(gamma, _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), axis, _p(f))
    return f


def point_tvdlf(gamma, pl, pr, met5, ref3, axis):
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (pl, pr, met5, ref3)]
    f = np.zeros(8)
    lib().og_point_tvdlf(gamma, _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), axis, _p(f))
    return f
