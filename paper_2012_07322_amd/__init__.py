"""Python binding of libgmunu (the MI355X GRMHD finite-volume step).

Argument marshalling only: every step runs in the HIP kernels of
``csrc/gmunu.hip`` behind the C ABI of ``include/gmunu.h``.  PyTorch
provides device memory and the stream.  There is no CPU fallback: if the
library is not built, importing works but every call raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libgmunu.so")

CART, CYL, SPH = 0, 1, 2
PERIODIC, OUTFLOW, REFLECT, AXIS, CENTER, NONE = 0, 1, 2, 3, 4, 5
FLAG_ATMO, FLAG_EPS_CLAMP, FLAG_V_CLAMP = 1, 2, 4
FLAG_FATAL_RHO, FLAG_FATAL_EPS, FLAG_FATAL_V, FLAG_NOCONV = 8, 16, 32, 64

ERRORS = {-1: "invalid argument", -2: "null pointer", -3: "misaligned pointer", -4: "HIP error",
          -5: "out of device memory", -6: "solve stalled", -7: "server stopped"}


class GridDesc(ctypes.Structure):
    """Mirror of gmunu_grid_desc."""
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
        ("recon", ctypes.c_int), ("riemann", ctypes.c_int), ("pp_limiter", ctypes.c_int), ("c2p", ctypes.c_int),
    ]


DEFAULTS = dict(ng=2, gamma=5.0 / 3.0, rho_atmo=1e-12, k_atmo=100.0, gamma_atmo=2.0,
                rho_low_factor=100.0, alpha_bh=1e-2, rho_max=math.inf, eps_max=math.inf,
                w_max=1e3, c2p_maxit=200, c2p_tol=1e-15, rk=3, recon=0, riemann=0, pp_limiter=0, c2p=0)

_lib = None
_P = ctypes.c_void_p


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgmunu is not built ({LIB_PATH}); run paper_2012_07322_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        I, D = ctypes.c_int, ctypes.c_double
        L.gmunu_create.argtypes = [_P, ctypes.POINTER(_P)]
        L.gmunu_destroy.argtypes = [_P]
        L.gmunu_ntot.argtypes = [_P]
        L.gmunu_ntot.restype = ctypes.c_long
        L.gmunu_prim2con.argtypes = [_P, _P, _P, _P, _P]
        L.gmunu_c2p.argtypes = [_P, _P, _P, _P, _P, _P, _P]
        L.gmunu_fill_ghosts.argtypes = [_P, _P, _P]
        L.gmunu_rhs.argtypes = [_P, _P, _P, _P, _P, _P]
        L.gmunu_cfl_dt.argtypes = [_P, _P, _P, D, D, _P, _P, _P]
        L.gmunu_rk_stage.argtypes = [_P, I, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.gmunu_step.argtypes = [_P, _P, _P, _P, _P, _P, D, D, _P, _P, _P, _P, _P]
        L.gmunu_steps.argtypes = [_P, _P, _P, _P, _P, _P, D, D, _P, _P, _P, _P, I, _P]
        L.gmunu_step_static.argtypes = [_P, _P, _P, _P, _P, _P, D, D, _P, _P, _P, _P, _P]
        L.gmunu_profile.argtypes = [_P, I, I]
        L.gmunu_profile_read.argtypes = [_P, _P, _P]
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what} failed: {ERRORS.get(rc, rc)}")


def make_desc(p: dict) -> GridDesc:
    q = dict(DEFAULTS)
    q.update(p)
    d = GridDesc()
    d.ndim, d.coord, d.ng = int(q["ndim"]), int(q["coord"]), int(q["ng"])
    for a in range(3):
        d.n[a] = int(q["n"][a])
        d.xmin[a] = float(q["xmin"][a])
        d.dx[a] = float(q["dx"][a])
        d.bc[a][0] = int(q["bc"][a][0])
        d.bc[a][1] = int(q["bc"][a][1])
    for k in ("gamma", "rho_atmo", "k_atmo", "gamma_atmo", "rho_low_factor", "alpha_bh", "rho_max", "eps_max",
              "w_max", "c2p_tol"):
        setattr(d, k, float(q[k]))
    d.c2p_maxit, d.rk = int(q["c2p_maxit"]), int(q["rk"])
    d.recon, d.riemann, d.pp_limiter, d.c2p = (int(q["recon"]), int(q["riemann"]), int(q["pp_limiter"]),
                                               int(q["c2p"]))
    return d


def _ptr(t, what, dtype=torch.float64):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {dtype} tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A grid context: geometry tables and scratch on the current device."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self.desc = make_desc(params)
        h = _P()
        _check(lib().gmunu_create(ctypes.byref(self.desc), ctypes.byref(h)), "gmunu_create")
        self._h = h
        d = self.desc
        g = [d.ng if a < d.ndim else 0 for a in range(3)]
        self.shape = (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])
        self.ntot = int(lib().gmunu_ntot(h))
        self.nstages = d.rk

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, t, nv, what):
        if t is None:
            return None
        if tuple(t.shape) != (nv,) + self.shape:
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {(nv,) + self.shape}")
        return _ptr(t, what)

    def empty_state(self, nv=8, device="cuda"):
        return torch.zeros((nv,) + self.shape, dtype=torch.float64, device=device)

    def prim2con(self, prim, metric, q=None):
        q = self.empty_state() if q is None else q
        _check(lib().gmunu_prim2con(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"),
                                    self._chk(q, 8, "q"), _stream()), "gmunu_prim2con")
        return q

    def c2p(self, q, metric, prim, flags=None, nfatal=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        if flags is not None and tuple(flags.shape) != self.shape:
            raise ValueError("flags shape")
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_c2p(self._h, self._chk(q, 8, "q"), self._chk(metric, 5, "metric"),
                               self._chk(prim, 8, "prim"), fp, npn, _stream()), "gmunu_c2p")
        return prim

    def fill_ghosts(self, prim):
        _check(lib().gmunu_fill_ghosts(self._h, self._chk(prim, 8, "prim"), _stream()), "gmunu_fill_ghosts")
        return prim

    def rhs(self, prim, metric, out=None, kij=None):
        """dq/dt (gmunu_rhs); kij: optional K_ij, shape (6,) + grid shape."""
        out = self.empty_state() if out is None else out
        _check(lib().gmunu_rhs(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"),
                               self._chk(kij, 6, "kij"), self._chk(out, 8, "dqdt"), _stream()), "gmunu_rhs")
        return out

    def cfl_dt(self, prim, metric, cfl, t_end=math.inf, t_dev=None, dt_dev=None):
        dt_dev = torch.zeros(1, dtype=torch.float64, device=prim.device) if dt_dev is None else dt_dev
        _check(lib().gmunu_cfl_dt(self._h, self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"), cfl, t_end,
                                  _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), _stream()), "gmunu_cfl_dt")
        return dt_dev

    def rk_stage(self, stage, dt_dev, q_n, q_s, q_out, prim_in, prim_out, metric, flags=None, nfatal=None,
                 kij=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_rk_stage(self._h, stage, _ptr(dt_dev, "dt"), self._chk(q_n, 8, "q_n"),
                                    self._chk(q_s, 8, "q_s"), self._chk(q_out, 8, "q_out"),
                                    self._chk(prim_in, 8, "prim_in"), self._chk(prim_out, 8, "prim_out"),
                                    self._chk(metric, 5, "metric"), self._chk(kij, 6, "kij"), fp, npn, _stream()),
               "gmunu_rk_stage")

    KERNELS = ("stage", "c2p", "ghosts", "cfl", "other")

    def profile(self, enable=True, max_launches=8192):
        _check(lib().gmunu_profile(self._h, 1 if enable else 0, max_launches), "gmunu_profile")

    def profile_read(self):
        ms = (ctypes.c_double * 5)()
        cnt = (ctypes.c_long * 5)()
        _check(lib().gmunu_profile_read(self._h, ms, cnt), "gmunu_profile_read")
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNELS)}

    def step(self, q_n, q_s, prim, metric, cfl, t_end, t_dev, dt_dev, flags=None, nfatal=None, kij=None):
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_step(self._h, self._chk(q_n, 8, "q_n"), self._chk(q_s, 8, "q_s"),
                                self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"), self._chk(kij, 6, "kij"),
                                cfl, t_end, _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), fp, npn, _stream()), "gmunu_step")

    def steps(self, q_n, q_s, prim, metric, cfl, t_end, t_dev, dt_dev, nsteps, flags=None, nfatal=None, kij=None):
        """nsteps gmunu_step calls in one (gmunu_steps: the CFL kernel only in
        the first step)."""
        fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_steps(self._h, self._chk(q_n, 8, "q_n"), self._chk(q_s, 8, "q_s"),
                                 self._chk(prim, 8, "prim"), self._chk(metric, 5, "metric"), self._chk(kij, 6, "kij"),
                                 cfl, t_end, _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), fp, npn, int(nsteps), _stream()),
               "gmunu_steps")

    def run(self, prim, metric, cfl, t_end=1e30, max_steps=0, check_every=16):
        """Advance one solve on its own: ghosts of prim filled, q_n from
        prim, prim recovered, then gmunu_steps in runs of `check_every` steps
        until t reaches t_end or max_steps steps were taken (steps past t_end
        change nothing, so t is checked every `check_every` steps).  prim is
        updated in place; returns (q_n, q_s, t)."""
        if max_steps <= 0 and not (t_end < 1e300):
            raise ValueError("run needs a finite t_end or a step limit")
        self.fill_ghosts(prim)
        qn = self.prim2con(prim, metric)
        self.c2p(qn, metric, prim)
        self.fill_ghosts(prim)
        qs = torch.zeros_like(qn)
        t = torch.zeros(1, dtype=torch.float64, device=prim.device)
        dt = torch.zeros_like(t)
        L, st = lib(), _stream()
        args = (self._h, _ptr(qn, "q_n"), _ptr(qs, "q_s"), _ptr(prim, "prim"), self._chk(metric, 5, "metric"), None)
        tp, dtp = _ptr(t, "t"), _ptr(dt, "dt")
        done = 0
        while True:
            k = max_steps - done if max_steps > 0 else check_every
            if max_steps > 0 and t_end < 1e300:
                k = min(k, check_every)
            _check(L.gmunu_steps(*args, cfl, t_end, tp, dtp, None, None, k, st), "gmunu_steps")
            done += k
            if max_steps > 0 and done >= max_steps:
                break
            if float(t.item()) >= t_end:
                break
        return qn, qs, float(t.item())


def step_static(params, q_n, q_s, prim, metric, cfl, t_end, t_dev, dt_dev, flags=None, nfatal=None, kij=None):
    """One step without a context (gmunu_step_static): geometry and CFL
    partials in the library's static per-GPU scratch, nothing allocated."""
    d = make_desc(params)
    g = [d.ng if a < d.ndim else 0 for a in range(3)]
    shp = (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])

    def chk(t, nv, what):
        if t is None:
            return None
        if tuple(t.shape) != (nv,) + shp:
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {(nv,) + shp}")
        return _ptr(t, what)

    fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
    npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
    _check(lib().gmunu_step_static(ctypes.byref(d), chk(q_n, 8, "q_n"), chk(q_s, 8, "q_s"), chk(prim, 8, "prim"),
                                   chk(metric, 5, "metric"), chk(kij, 6, "kij"), cfl, t_end, _ptr(t_dev, "t"),
                                   _ptr(dt_dev, "dt"), fp, npn, _stream()), "gmunu_step_static")


# ------------------------------------------------------------------- batch

class BlockSpec(ctypes.Structure):
    """Mirror of gmunu_block."""
    _fields_ = [("desc", GridDesc), ("q_n", _P), ("q_s", _P), ("prim", _P), ("metric", _P), ("flags", _P),
                ("group", ctypes.c_int)]


def _batch_sigs(L):
    I, D = ctypes.c_int, ctypes.c_double
    L.gmunu_batch_create.argtypes = [I, I, ctypes.c_long, ctypes.POINTER(_P)]
    L.gmunu_batch_destroy.argtypes = [_P]
    L.gmunu_batch_set_block.argtypes = [_P, I, ctypes.POINTER(BlockSpec)]
    L.gmunu_batch_clear_block.argtypes = [_P, I]
    L.gmunu_batch_set_group.argtypes = [_P, I, D, D, I]
    L.gmunu_batch_commit.argtypes = [_P, _P]
    L.gmunu_batch_autotune.argtypes = [_P, _P]
    L.gmunu_batch_set_tile.argtypes = [_P, _P, I, I, I]
    L.gmunu_batch_init.argtypes = [_P, _P, I, _P]
    L.gmunu_batch_step.argtypes = [_P, D, _P, I, _P]
    L.gmunu_batch_steps.argtypes = [_P, D, I, _P, _P]
    L.gmunu_batch_times.argtypes = [_P, _P, _P, _P, _P, _P]
    L.gmunu_batch_info.argtypes = [_P, _P, _P]


def state_shape(p: dict):
    d = make_desc(p)
    g = [d.ng if a < d.ndim else 0 for a in range(3)]
    return (d.n[2] + 2 * g[2], d.n[1] + 2 * g[1], d.n[0] + 2 * g[0])


class Arena:
    """One device allocation sliced into 256-byte aligned views."""

    def __init__(self, ndoubles, device="cuda"):
        self.buf = torch.empty(int(ndoubles), dtype=torch.float64, device=device)
        self.off = 0

    @staticmethod
    def size_of(shapes):
        tot = 0
        for s in shapes:
            n = 1
            for x in s:
                n *= x
            tot += (n + 31) // 32 * 32
        return tot

    def take(self, shape):
        n = 1
        for x in shape:
            n *= x
        v = self.buf[self.off:self.off + n].view(shape)
        self.off += (n + 31) // 32 * 32
        return v


class Batch:
    """Many grids advanced together (gmunu_batch_*): blocks in slots, groups
    sharing a time step, persistent kernels, a graph-captured step."""

    def __init__(self, max_blocks, max_groups, max_items):
        L = lib()
        if not hasattr(L, "_batch_sigs_set"):
            _batch_sigs(L)
            L._batch_sigs_set = True
        h = _P()
        _check(L.gmunu_batch_create(max_blocks, max_groups, max_items, ctypes.byref(h)), "gmunu_batch_create")
        self._h = h
        self.max_blocks, self.max_groups = max_blocks, max_groups
        self.keep = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_block(self, slot, params, q_n, q_s, prim, metric, group, flags=None):
        shp = state_shape(params)
        for t, nv, nm in ((q_n, 8, "q_n"), (q_s, 8, "q_s"), (prim, 8, "prim"), (metric, 5, "metric")):
            if tuple(t.shape) != (nv,) + shp:
                raise ValueError(f"{nm} has shape {tuple(t.shape)}, expected {(nv,) + shp}")
        spec = BlockSpec()
        spec.desc = make_desc(params)
        spec.q_n, spec.q_s, spec.prim = _ptr(q_n, "q_n"), _ptr(q_s, "q_s"), _ptr(prim, "prim")
        spec.metric = _ptr(metric, "metric")
        spec.flags = _ptr(flags, "flags", torch.uint8) if flags is not None else None
        spec.group = group
        _check(lib().gmunu_batch_set_block(self._h, slot, ctypes.byref(spec)), "gmunu_batch_set_block")
        self.keep[slot] = (q_n, q_s, prim, metric, flags)

    def clear_block(self, slot):
        _check(lib().gmunu_batch_clear_block(self._h, slot), "gmunu_batch_clear_block")
        self.keep.pop(slot, None)

    def set_group(self, group, t, t_end, max_steps=0):
        _check(lib().gmunu_batch_set_group(self._h, group, t, t_end, max_steps), "gmunu_batch_set_group")

    def commit(self):
        _check(lib().gmunu_batch_commit(self._h, _stream()), "gmunu_batch_commit")

    def autotune(self):
        _check(lib().gmunu_batch_autotune(self._h, _stream()), "gmunu_batch_autotune")

    def set_tile(self, params, tx, ty, tz):
        """Pin the stage tile shape for the class of blocks of `params`
        (gmunu_batch_set_tile); applied at the next commit."""
        d = make_desc(params)
        _check(lib().gmunu_batch_set_tile(self._h, ctypes.byref(d), int(tx), int(ty), int(tz)),
               "gmunu_batch_set_tile")

    def init(self, slots=None):
        if slots is None:
            _check(lib().gmunu_batch_init(self._h, None, 0, _stream()), "gmunu_batch_init")
        else:
            arr = (ctypes.c_int * len(slots))(*slots)
            _check(lib().gmunu_batch_init(self._h, arr, len(slots), _stream()), "gmunu_batch_init")

    def step(self, cfl, nfatal=None, use_graph=True):
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_batch_step(self._h, cfl, npn, 1 if use_graph else 0, _stream()), "gmunu_batch_step")

    def steps(self, cfl, nsteps, nfatal=None):
        """nsteps steps from one captured graph (gmunu_batch_steps)."""
        npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
        _check(lib().gmunu_batch_steps(self._h, cfl, int(nsteps), npn, _stream()), "gmunu_batch_steps")

    def times(self, with_steps=False):
        """(t, dt) per group; with_steps: (t, dt, steps, fatal recoveries)."""
        import numpy as np
        t = np.zeros(self.max_groups)
        dt = np.zeros(self.max_groups)
        ns = np.zeros(self.max_groups, dtype=np.int32)
        nf = np.zeros(self.max_groups, dtype=np.uint32)
        _check(lib().gmunu_batch_times(self._h, t.ctypes.data_as(_P), dt.ctypes.data_as(_P),
                                       ns.ctypes.data_as(_P), nf.ctypes.data_as(_P), _stream()),
               "gmunu_batch_times")
        return (t, dt, ns, nf) if with_steps else (t, dt)

    def info(self):
        import numpy as np
        items = np.zeros(3, dtype=np.int64)
        var = np.zeros(self.max_blocks, dtype=np.int32)
        _check(lib().gmunu_batch_info(self._h, items.ctypes.data_as(_P), var.ctypes.data_as(_P)), "gmunu_batch_info")
        return items, var


# ------------------------------------------------------------------ server

class RequestSpec(ctypes.Structure):
    """Mirror of gmunu_request."""
    _fields_ = [("desc", GridDesc), ("prim", _P), ("metric", _P), ("t_end", ctypes.c_double),
                ("max_steps", ctypes.c_int), ("q_out", _P), ("prim_out", _P), ("tag", ctypes.c_ulonglong)]


class Result(ctypes.Structure):
    """Mirror of gmunu_result."""
    _fields_ = [("id", ctypes.c_ulonglong), ("tag", ctypes.c_ulonglong), ("status", ctypes.c_int),
                ("steps", ctypes.c_int), ("nfatal", ctypes.c_uint), ("t", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
                ("bytes", ctypes.c_size_t)]


class ServerInfo(ctypes.Structure):
    """Mirror of gmunu_server_info."""
    _fields_ = [("submitted", ctypes.c_long), ("admitted", ctypes.c_long), ("completed", ctypes.c_long),
                ("pending", ctypes.c_long), ("resident", ctypes.c_long), ("replays", ctypes.c_long),
                ("pool_bytes", ctypes.c_size_t), ("pool_used", ctypes.c_size_t), ("pool_peak", ctypes.c_size_t),
                ("busy_s", ctypes.c_double)]


def _server_sigs(L):
    I = ctypes.c_int
    L.gmunu_server_clock.argtypes = []
    L.gmunu_server_clock.restype = ctypes.c_double
    L.gmunu_server_create.argtypes = [ctypes.c_size_t, I, ctypes.c_double, I, ctypes.POINTER(_P)]
    L.gmunu_server_submit.argtypes = [_P, ctypes.POINTER(RequestSpec), ctypes.POINTER(ctypes.c_ulonglong)]
    L.gmunu_server_poll.argtypes = [_P, ctypes.POINTER(Result), I, I]
    L.gmunu_server_status.argtypes = [_P, ctypes.POINTER(ServerInfo)]
    L.gmunu_server_destroy.argtypes = [_P]


def _addr(a, what, nvars, shape):
    """Address of a float64 C-contiguous numpy array or torch tensor (host
    or device) of shape (nvars,) + shape; None passes through."""
    if a is None:
        return None
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError(f"{what} must be a contiguous float64 tensor")
        got = tuple(a.shape)
        ptr = a.data_ptr()
    else:
        import numpy as np
        if not isinstance(a, np.ndarray) or a.dtype != np.float64 or not a.flags["C_CONTIGUOUS"]:
            raise TypeError(f"{what} must be a C-contiguous float64 array")
        got = a.shape
        ptr = a.ctypes.data
    if got != (nvars,) + tuple(shape):
        raise ValueError(f"{what} has shape {got}, expected {(nvars,) + tuple(shape)}")
    return ctypes.c_void_p(ptr)


class Server:
    """Continuous-batching request server (gmunu_server_*): solves of any
    size share the GPU through one batched, graph-replayed step; each is
    admitted when its state fits the HBM budget."""

    def __init__(self, hbm_bytes, max_slots=256, cfl=0.4, steps_per_sync=2):
        L = lib()
        if not hasattr(L, "_batch_sigs_set"):
            _batch_sigs(L)
            L._batch_sigs_set = True
        if not hasattr(L, "_server_sigs_set"):
            _server_sigs(L)
            L._server_sigs_set = True
        h = _P()
        _check(L.gmunu_server_create(int(hbm_bytes), max_slots, cfl, steps_per_sync, ctypes.byref(h)),
               "gmunu_server_create")
        self._h = h
        self._keep = {}

    @staticmethod
    def clock():
        L = lib()
        if not hasattr(L, "_server_sigs_set"):
            _server_sigs(L)
            L._server_sigs_set = True
        return L.gmunu_server_clock()

    def submit(self, params, prim, metric, t_end=1e30, max_steps=0, q_out=None, prim_out=None, tag=0):
        """Queue one solve; prim / metric / outputs are numpy arrays or torch
        tensors (host or device) in the grid's layout.  Device inputs must be
        complete on the device: the current stream is synchronised first."""
        shp = state_shape(params)
        spec = RequestSpec()
        spec.desc = make_desc(params)
        spec.prim = _addr(prim, "prim", 8, shp)
        spec.metric = _addr(metric, "metric", 5, shp)
        spec.t_end = float(t_end)
        spec.max_steps = int(max_steps)
        spec.q_out = _addr(q_out, "q_out", 8, shp)
        spec.prim_out = _addr(prim_out, "prim_out", 8, shp)
        spec.tag = int(tag)
        if any(isinstance(x, torch.Tensor) and x.is_cuda for x in (prim, metric, q_out, prim_out)):
            torch.cuda.current_stream().synchronize()
        rid = ctypes.c_ulonglong()
        _check(lib().gmunu_server_submit(self._h, ctypes.byref(spec), ctypes.byref(rid)), "gmunu_server_submit")
        self._keep[rid.value] = (prim, metric, q_out, prim_out)
        return rid.value

    def poll(self, max_results=256, timeout_ms=0):
        buf = (Result * max_results)()
        n = lib().gmunu_server_poll(self._h, buf, max_results, int(timeout_ms))
        _check(n if n < 0 else 0, "gmunu_server_poll")
        out = []
        for k in range(n):
            r = buf[k]
            self._keep.pop(r.id, None)
            out.append({f: getattr(r, f) for f, _ in Result._fields_})
        return out

    def status(self):
        info = ServerInfo()
        rc = lib().gmunu_server_status(self._h, ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in ServerInfo._fields_}
        d["error"] = rc
        return d

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- multigrid

MG_DIRICHLET, MG_NEUMANN, MG_PERIODIC, MG_ROBIN = 0, 1, 2, 3


class MgDesc(ctypes.Structure):
    """Mirror of gmunu_mg_desc."""
    _fields_ = [
        ("ndim", ctypes.c_int), ("coord", ctypes.c_int), ("n", ctypes.c_int * 3),
        ("xmin", ctypes.c_double * 3), ("dx", ctypes.c_double * 3), ("bc", (ctypes.c_int * 2) * 3),
        ("levels", ctypes.c_int), ("pre", ctypes.c_int), ("post", ctypes.c_int), ("coarse", ctypes.c_int),
        ("power", ctypes.c_int), ("offset", ctypes.c_double), ("power2", ctypes.c_int),
        ("smoother", ctypes.c_int),
    ]


MG_DEFAULTS = dict(levels=0, pre=2, post=2, coarse=50, power=0, offset=0.0, power2=0, smoother=0)
MG_POINT, MG_LINE = 0, 1


def _mg_sigs(L):
    I, D = ctypes.c_int, ctypes.c_double
    L.gmunu_mg_create.argtypes = [_P, ctypes.POINTER(_P)]
    L.gmunu_mg_destroy.argtypes = [_P]
    L.gmunu_mg_levels.argtypes = [_P]
    L.gmunu_mg_size.argtypes = [_P, I]
    L.gmunu_mg_size.restype = ctypes.c_long
    L.gmunu_mg_solve.argtypes = [_P, _P, _P, _P, _P, D, I, I, _P, _P, _P]
    L.gmunu_mg_residual_norm.argtypes = [_P, _P, _P, _P, _P, _P, _P]
    L.gmunu_mg_apply.argtypes = [_P, _P, _P, _P, _P, _P]
    L.gmunu_mg_fill_ghosts.argtypes = [_P, I, _P, _P]
    L.gmunu_mg_smooth.argtypes = [_P, _P, _P, _P, _P, I, _P]
    L.gmunu_mg_restrict.argtypes = [_P, I, _P, _P, _P]
    L.gmunu_mg_prolong.argtypes = [_P, I, _P, _P, _P]
    L.gmunu_mg_divergence.argtypes = [_P, _P, _P, _P]
    L.gmunu_mg_subtract_gradient.argtypes = [_P, _P, _P, _P]
    L.gmunu_mg_clean.argtypes = [_P, _P, _P, _P, D, I, _P, _P, _P]
    L.gmunu_mg_clean_state.argtypes = [_P, _P, _P, _P, _P, D, I, _P, _P, _P]
    L.gmunu_mg_cfc_solve.argtypes = [_P, _P, _P, _P, _P, _P, D, I, _P, _P]
    L.gmunu_mg_vapply.argtypes = [_P, _P, _P, _P]
    L.gmunu_mg_vsmooth.argtypes = [_P, _P, _P, I, _P]
    L.gmunu_mg_vsolve.argtypes = [_P, _P, _P, D, I, I, _P, _P, _P]
    L.gmunu_mg_xcfc_aij.argtypes = [_P, _P, _P, _P, _P]
    L.gmunu_mg_xcfc_beta_rhs.argtypes = [_P, _P, _P, _P, _P, _P]
    L.gmunu_mg_xcfc_solve.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, D, I, _P, _P]
    L.gmunu_mg_metric_update.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, D, I, _P, _P]
    L.gmunu_mg_psi_residual.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P]
    L.gmunu_mg_dynamical_steps.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P, D, D, _P, _P, _P, _P, I, D, _P, _P,
                                           _P]


def make_mg_desc(p: dict) -> MgDesc:
    q = dict(MG_DEFAULTS)
    q.update(p)
    d = MgDesc()
    d.ndim, d.coord = int(q["ndim"]), int(q["coord"])
    for a in range(3):
        d.n[a] = int(q["n"][a])
        d.xmin[a] = float(q["xmin"][a])
        d.dx[a] = float(q["dx"][a])
        d.bc[a][0], d.bc[a][1] = int(q["bc"][a][0]), int(q["bc"][a][1])
    d.levels, d.pre, d.post, d.coarse = int(q["levels"]), int(q["pre"]), int(q["post"]), int(q["coarse"])
    d.power, d.offset, d.power2 = int(q["power"]), float(q["offset"]), int(q["power2"])
    d.smoother = int(q["smoother"])
    return d


class Multigrid:
    """Cell-centred multigrid hierarchy on the current device (gmunu_mg_*).
    Arrays are contiguous float64 device tensors of shape(level) (one ghost
    layer on each active axis); vector fields have a leading axis of 3."""

    def __init__(self, params: dict):
        L = lib()
        if not hasattr(L, "_mg_sigs_set"):
            _mg_sigs(L)
            L._mg_sigs_set = True
        self.desc = make_mg_desc(params)
        h = _P()
        _check(L.gmunu_mg_create(ctypes.byref(self.desc), ctypes.byref(h)), "gmunu_mg_create")
        self._h = h
        self.levels = int(L.gmunu_mg_levels(h))

    def close(self):
        if getattr(self, "_h", None):
            lib().gmunu_mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shape(self, level=None):
        d = self.desc
        s = 0 if level is None else self.levels - 1 - level
        return tuple((d.n[a] >> s) + 2 if a < d.ndim else 1 for a in (2, 1, 0))

    def empty(self, level=None, vector=False):
        shp = ((int(vector) if vector > 1 else 3,) if vector else ()) + self.shape(level)
        return torch.zeros(shp, dtype=torch.float64, device="cuda")

    def _chk(self, t, what, level=None, vector=False, none_ok=False):
        """vector: False (scalar), True (three components) or a component count."""
        if t is None:
            if none_ok:
                return None
            raise ValueError(f"{what} is required")
        shp = ((int(vector) if vector > 1 else 3,) if vector else ()) + self.shape(level)
        if tuple(t.shape) != shp:
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {shp}")
        return _ptr(t, what)

    def solve(self, u, f, a=None, tol=1e-12, max_cycles=30, fmg=True, a2=None):
        """Solve in place; returns the residual history (list of max norms)."""
        res = (ctypes.c_double * (max_cycles + 1))()
        cyc = ctypes.c_int(0)
        _check(lib().gmunu_mg_solve(self._h, self._chk(u, "u"), self._chk(f, "f"),
                                    self._chk(a, "a", none_ok=True), self._chk(a2, "a2", none_ok=True), float(tol),
                                    int(max_cycles), 1 if fmg else 0, res, ctypes.byref(cyc), _stream()),
               "gmunu_mg_solve")
        return [res[i] for i in range(cyc.value + 1)]

    def residual_norm(self, u, f, a=None, a2=None):
        out = ctypes.c_double(0.0)
        _check(lib().gmunu_mg_residual_norm(self._h, self._chk(u, "u"), self._chk(f, "f"),
                                            self._chk(a, "a", none_ok=True), self._chk(a2, "a2", none_ok=True),
                                            ctypes.byref(out), _stream()), "gmunu_mg_residual_norm")
        return out.value

    def apply(self, u, a=None, out=None, a2=None):
        out = self.empty() if out is None else out
        _check(lib().gmunu_mg_apply(self._h, self._chk(u, "u"), self._chk(a, "a", none_ok=True),
                                    self._chk(a2, "a2", none_ok=True), self._chk(out, "out"), _stream()),
               "gmunu_mg_apply")
        return out

    def fill_ghosts(self, u, level=None):
        lv = self.levels - 1 if level is None else level
        _check(lib().gmunu_mg_fill_ghosts(self._h, lv, self._chk(u, "u", lv), _stream()), "gmunu_mg_fill_ghosts")
        return u

    def smooth(self, u, f, a=None, sweeps=1, a2=None):
        _check(lib().gmunu_mg_smooth(self._h, self._chk(u, "u"), self._chk(f, "f"), self._chk(a, "a", none_ok=True),
                                     self._chk(a2, "a2", none_ok=True), int(sweeps), _stream()), "gmunu_mg_smooth")
        return u

    # vector equation of xCFC (Cartesian, or axisymmetric cylindrical and
    # spherical in orthonormal components): X, f of shape (3,) + shape()
    def vapply(self, X, out=None):
        out = self.empty(vector=True) if out is None else out
        _check(lib().gmunu_mg_vapply(self._h, self._chk(X, "X", vector=True), self._chk(out, "out", vector=True),
                                     _stream()), "gmunu_mg_vapply")
        return out

    def vsmooth(self, X, f, sweeps=1):
        _check(lib().gmunu_mg_vsmooth(self._h, self._chk(X, "X", vector=True), self._chk(f, "f", vector=True),
                                      int(sweeps), _stream()), "gmunu_mg_vsmooth")
        return X

    def vsolve(self, X, f, tol=1e-12, max_cycles=30, fmg=True):
        res = (ctypes.c_double * (max_cycles + 1))()
        cyc = ctypes.c_int(0)
        _check(lib().gmunu_mg_vsolve(self._h, self._chk(X, "X", vector=True), self._chk(f, "f", vector=True),
                                     float(tol), int(max_cycles), 1 if fmg else 0, res, ctypes.byref(cyc),
                                     _stream()), "gmunu_mg_vsolve")
        return [res[i] for i in range(cyc.value + 1)]

    def xcfc_aij(self, X, A6=None, A2=None):
        A6 = self.empty(vector=6) if A6 is None else A6
        A2 = self.empty() if A2 is None else A2
        _check(lib().gmunu_mg_xcfc_aij(self._h, self._chk(X, "X", vector=True), self._chk(A6, "A6", vector=6),
                                       self._chk(A2, "A2"), _stream()), "gmunu_mg_xcfc_aij")
        return A6, A2

    def xcfc_beta_rhs(self, w, S, A6, out=None):
        out = self.empty(vector=True) if out is None else out
        _check(lib().gmunu_mg_xcfc_beta_rhs(self._h, self._chk(w, "w"), self._chk(S, "S", vector=True),
                                            self._chk(A6, "A6", vector=6), self._chk(out, "out", vector=True),
                                            _stream()), "gmunu_mg_xcfc_beta_rhs")
        return out

    def restrict(self, level, fine, coarse=None):
        coarse = self.empty(level - 1) if coarse is None else coarse
        _check(lib().gmunu_mg_restrict(self._h, level, self._chk(fine, "fine", level),
                                       self._chk(coarse, "coarse", level - 1), _stream()), "gmunu_mg_restrict")
        return coarse

    def prolong(self, level, coarse, fine=None):
        fine = self.empty(level) if fine is None else fine
        _check(lib().gmunu_mg_prolong(self._h, level, self._chk(coarse, "coarse", level - 1),
                                      self._chk(fine, "fine", level), _stream()), "gmunu_mg_prolong")
        return fine

    def divergence(self, q, out=None):
        out = self.empty() if out is None else out
        _check(lib().gmunu_mg_divergence(self._h, self._chk(q, "q", vector=True), self._chk(out, "div"),
                                         _stream()), "gmunu_mg_divergence")
        return out

    def subtract_gradient(self, phi, q):
        _check(lib().gmunu_mg_subtract_gradient(self._h, self._chk(phi, "phi"), self._chk(q, "q", vector=True),
                                                _stream()), "gmunu_mg_subtract_gradient")
        return q

    def clean(self, q, phi, div=None, tol=1e-12, max_cycles=30):
        res = (ctypes.c_double * (max_cycles + 1))()
        cyc = ctypes.c_int(0)
        _check(lib().gmunu_mg_clean(self._h, self._chk(q, "q", vector=True), self._chk(phi, "phi"),
                                    self._chk(div, "div", none_ok=True), float(tol), int(max_cycles), res,
                                    ctypes.byref(cyc), _stream()), "gmunu_mg_clean")
        return [res[i] for i in range(cyc.value + 1)]

    def clean_state(self, grid_params, q, prim, metric, tol=1e-12, max_cycles=30):
        """Clean q_B of a GRMHD state (q, prim, metric: the layout of
        Grid(grid_params)) in place; returns the residual history."""
        hd = make_desc(grid_params)
        res = (ctypes.c_double * (max_cycles + 1))()
        cyc = ctypes.c_int(0)
        _check(lib().gmunu_mg_clean_state(self._h, ctypes.byref(hd), _ptr(q, "q"), _ptr(prim, "prim"),
                                          _ptr(metric, "metric"), float(tol), int(max_cycles), res,
                                          ctypes.byref(cyc), _stream()), "gmunu_mg_clean_state")
        return [res[i] for i in range(cyc.value + 1)]


def cfc_solve(mpsi, malpha, grid_params, q, prim, metric, tol=1e-12, max_cycles=60):
    """Scalar CFC metric solve (psi, then alpha) for a GRMHD state; metric is
    updated in place.  Returns the cycles of the two solves."""
    hd = make_desc(grid_params)
    cyc = (ctypes.c_int * 2)()
    _check(lib().gmunu_mg_cfc_solve(mpsi._h, malpha._h, ctypes.byref(hd), _ptr(q, "q"), _ptr(prim, "prim"),
                                    _ptr(metric, "metric"), float(tol), int(max_cycles), cyc, _stream()),
           "gmunu_mg_cfc_solve")
    return cyc[0], cyc[1]


def metric_update(grid, mpsi, malpha, q, prim, metric, mvec=None, X=None, flags=None, nfatal=None, tol=1e-12,
                  max_cycles=60):
    """Re-solve the metric of a GRMHD state from its conserved variables
    (xCFC when mvec and X are given, else the scalar CFC equations), then
    recover prim on the new metric and fill its ghosts (gmunu_mg_metric_update).
    grid: the Grid of the state.  Returns the cycles of the four solves."""
    fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
    npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
    cyc = (ctypes.c_int * 4)()
    _check(lib().gmunu_mg_metric_update(mvec._h if mvec is not None else None, mpsi._h, malpha._h, grid._h,
                                        ctypes.byref(grid.desc), grid._chk(q, 8, "q"), grid._chk(prim, 8, "prim"),
                                        grid._chk(metric, 5, "metric"),
                                        mvec._chk(X, "X", vector=True) if mvec is not None else None, fp, npn,
                                        float(tol), int(max_cycles), cyc, _stream()), "gmunu_mg_metric_update")
    return tuple(cyc[i] for i in range(4))


def psi_residual(grid, mpsi, q, metric, mvec=None, X=None):
    """max |L(psi - 1)| of the conformal-factor equation with the current
    metric and matter (gmunu_mg_psi_residual)."""
    out = ctypes.c_double(0.0)
    _check(lib().gmunu_mg_psi_residual(mvec._h if mvec is not None else None, mpsi._h, ctypes.byref(grid.desc),
                                       grid._chk(q, 8, "q"), grid._chk(metric, 5, "metric"),
                                       mvec._chk(X, "X", vector=True) if mvec is not None else None,
                                       ctypes.byref(out), _stream()), "gmunu_mg_psi_residual")
    return out.value


def dynamical_steps(grid, q_n, q_s, prim, metric, mpsi, cfl, nsteps, eps, t_dev, dt_dev, t_end=1e30, mvec=None,
                    X=None, flags=None, nfatal=None):
    """Up to nsteps steps, each followed by the conformal-factor residual on
    the device; the steps after the first one whose residual exceeds eps
    change nothing (gmunu_mg_dynamical_steps).  Returns (steps taken,
    whether the residual triggered)."""
    fp = _ptr(flags, "flags", torch.uint8) if flags is not None else None
    npn = _ptr(nfatal, "nfatal", torch.int32) if nfatal is not None else None
    done, trig = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().gmunu_mg_dynamical_steps(mvec._h if mvec is not None else None, mpsi._h, grid._h,
                                          ctypes.byref(grid.desc), grid._chk(q_n, 8, "q_n"), grid._chk(q_s, 8, "q_s"),
                                          grid._chk(prim, 8, "prim"), grid._chk(metric, 5, "metric"),
                                          mvec._chk(X, "X", vector=True) if mvec is not None else None, float(cfl),
                                          float(t_end), _ptr(t_dev, "t"), _ptr(dt_dev, "dt"), fp, npn, int(nsteps),
                                          float(eps), ctypes.byref(done), ctypes.byref(trig), _stream()),
           "gmunu_mg_dynamical_steps")
    return done.value, bool(trig.value)


def evolve_dynamical(grid, q_n, q_s, prim, metric, mpsi, malpha, cfl, steps, every=50, eps=1e-3, mvec=None, X=None,
                     t_dev=None, dt_dev=None, flags=None, nfatal=None, tol=1e-6, max_cycles=60):
    """GRMHD steps on a metric re-solved from the evolved matter (section
    2.6): after each step the metric is updated when `every` steps have
    passed since the last update or when the conformal-factor residual
    exceeds eps.  The steps between updates run in chunks on the device
    (dynamical_steps: one host synchronisation per chunk, the residual of
    every step checked there).  Returns the step numbers (1-based) after
    which it was updated."""
    dev = q_n.device
    t_dev = torch.zeros(1, dtype=torch.float64, device=dev) if t_dev is None else t_dev
    dt_dev = torch.zeros(1, dtype=torch.float64, device=dev) if dt_dev is None else dt_dev
    updates, s, since = [], 0, 0
    while s < steps:
        done, trig = dynamical_steps(grid, q_n, q_s, prim, metric, mpsi, cfl, min(steps - s, max(every, 1) - since), eps,
                                     t_dev, dt_dev, mvec=mvec, X=X, flags=flags, nfatal=nfatal)
        s += done
        since += done
        if trig or since >= every:
            metric_update(grid, mpsi, malpha, q_n, prim, metric, mvec, X, flags, nfatal, tol, max_cycles)
            updates.append(s)
            since = 0
    return updates


def xcfc_solve(mvec, mpsi, malpha, grid_params, q, prim, metric, X, tol=1e-12, max_cycles=60):
    """xCFC metric solve (X, psi, alpha, beta) for a GRMHD state on a grid
    the vector equations accept (Cartesian, axisymmetric cylindrical or
    spherical); metric and X (mvec.empty(vector=True)) are updated in
    place.  Returns the cycles of the four solves."""
    hd = make_desc(grid_params)
    cyc = (ctypes.c_int * 4)()
    _check(lib().gmunu_mg_xcfc_solve(mvec._h, mpsi._h, malpha._h, ctypes.byref(hd), _ptr(q, "q"),
                                     _ptr(prim, "prim"), _ptr(metric, "metric"),
                                     mvec._chk(X, "X", vector=True), float(tol), int(max_cycles), cyc, _stream()),
           "gmunu_mg_xcfc_solve")
    return tuple(cyc[i] for i in range(4))
