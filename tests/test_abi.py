"""CPU checks of the boundary: the C library loads, exports every symbol the
header declares, its descriptor mirror matches the header's layout, and
descriptor validation rejects bad grids before touching the device."""
import ctypes
import math
import os
import re

import pytest

import paper_2012_07322_amd as gmu
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for fn in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:int|long|void|double)\s+\**\s*(gmunu_\w+)\s*\(", txt, flags=re.M)
    return names


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    L = gmu.lib()
    for n in names:
        assert hasattr(L, n), n


def test_descriptor_layout_matches_header():
    # the struct mirrors the header field by field: 4 ints + n[3] + ... + rk
    off = {f[0]: getattr(gmu.GridDesc, f[0]).offset for f in gmu.GridDesc._fields_}
    assert off["ndim"] == 0 and off["coord"] == 4 and off["n"] == 8 and off["ng"] == 20
    assert off["xmin"] == 24 and off["dx"] == 48 and off["bc"] == 72 and off["gamma"] == 96
    assert off["recon"] == off["rk"] + 4 and ctypes.sizeof(gmu.GridDesc) == off["c2p"] + 8


@pytest.mark.parametrize("mutate", [
    lambda p: p.update(ndim=4),
    lambda p: p.update(ng=1),
    lambda p: p.update(n=[400, 2, 1]),
    lambda p: p.update(gamma=1.0),
    lambda p: p.update(rk=4),
    lambda p: p.update(bc=[[W.PERIODIC, W.OUTFLOW], [5, 5], [5, 5]]),
    lambda p: p.update(dx=[0.0, 1.0, 1.0]),
    lambda p: p.update(recon=1),  # MP5 needs three ghost layers
    lambda p: p.update(recon=2),  # so does PPM
    lambda p: p.update(recon=3, ng=3),
    lambda p: p.update(riemann=2),
    lambda p: p.update(c2p=2),
    lambda p: p.update(pp_limiter=2),
])
def test_create_rejects_invalid_descriptors(mutate):
    p, _, _ = W.mhd_shock_tube(400)
    mutate(p)
    h = ctypes.c_void_p()
    rc = gmu.lib().gmunu_create(ctypes.byref(gmu.make_desc(p)), ctypes.byref(h))
    assert rc == -1 and not h.value


def test_null_arguments_are_rejected():
    L = gmu.lib()
    assert L.gmunu_create(None, None) == -2
    assert L.gmunu_destroy(None) == -2
    assert L.gmunu_rhs(None, None, None, None, None, None) == -2
    assert L.gmunu_c2p(None, None, None, None, None, None, None) == -2


def test_binding_raises_without_device_tensors():
    with pytest.raises(TypeError):
        gmu._ptr(object(), "x")


def _c_layout(structs):
    """sizeof and field offsets of header structs, from a C program built
    with the host compiler against include/gmunu.h and gmunu_mg.h."""
    import subprocess
    import tempfile

    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "gmunu.h"', '#include "gmunu_mg.h"',
             "int main(void) {"]
    for st, fields in structs.items():
        lines.append(f'  printf("{st} size %zu\\n", sizeof({st}));')
        for f in fields:
            lines.append(f'  printf("{st} {f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "l.c"), os.path.join(d, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        out = subprocess.check_output([exe], text=True)
    res = {}
    for ln in out.splitlines():
        st, f, v = ln.split()
        res[(st, f)] = int(v)
    return res


def test_struct_mirrors_match_the_header():
    mirrors = {"gmunu_grid_desc": gmu.GridDesc, "gmunu_block": gmu.BlockSpec, "gmunu_request": gmu.RequestSpec,
               "gmunu_result": gmu.Result, "gmunu_server_info": gmu.ServerInfo, "gmunu_mg_desc": gmu.MgDesc}
    lay = _c_layout({k: [f for f, _ in v._fields_] for k, v in mirrors.items()})
    for st, cls in mirrors.items():
        assert lay[(st, "size")] == ctypes.sizeof(cls), st
        for f, _ in cls._fields_:
            assert lay[(st, f)] == getattr(cls, f).offset, (st, f)


def test_server_rejects_bad_arguments_before_touching_the_device():
    L = gmu.lib()
    gmu._server_sigs(L)
    h = ctypes.c_void_p()
    assert L.gmunu_server_create(1 << 30, 0, 0.4, 1, ctypes.byref(h)) == -1
    assert L.gmunu_server_create(1 << 30, 8, -1.0, 1, ctypes.byref(h)) == -1
    assert L.gmunu_server_create(1 << 30, 8, 0.4, 0, ctypes.byref(h)) == -1
    assert L.gmunu_server_create(1 << 30, 8, 0.4, 1, None) == -2
    assert L.gmunu_server_submit(None, None, None) == -2
    assert L.gmunu_server_poll(None, None, 0, 0) == -2
    assert L.gmunu_server_destroy(None) == -2
    assert L.gmunu_server_clock() > 0.0


def test_step_batch_and_metric_entry_points_reject_null_arguments():
    """gmunu_steps, gmunu_batch_set_tile and gmunu_mg_dynamical_steps check
    their handles and pointers before any device call."""
    L = gmu.lib()
    gmu._batch_sigs(L)
    gmu._mg_sigs(L)
    assert L.gmunu_steps(None, None, None, None, None, None, 0.4, 1e30, None, None, None, None, 1, None) == -2
    assert L.gmunu_batch_set_tile(None, None, 8, 8, 3) == -2
    n, trig = ctypes.c_int(0), ctypes.c_int(0)
    assert L.gmunu_mg_dynamical_steps(None, None, None, None, None, None, None, None, None, 0.4, 1.0, None, None,
                                      None, None, 1, 1e-3, ctypes.byref(n), ctypes.byref(trig), None) == -2


def test_range_pool_host_logic():
    """The server's arena allocator (header-only, host code) under random
    alloc / release: ranges aligned, disjoint, inside the arena, and merged
    back into one free range when everything is returned."""
    import subprocess
    import tempfile

    src = os.path.join(ROOT, "tests", "pool_check.cpp")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "pool_check")
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2012_07322_amd", "csrc"),
                               src, "-o", exe])
        out = subprocess.check_output([exe], text=True)
    assert out.strip().endswith("ok"), out


def test_multigrid_create_rejects_invalid_descriptors():
    """Validation happens before any device call."""
    L = gmu.lib()
    if not hasattr(L, "_mg_sigs_set"):
        gmu._mg_sigs(L)
        L._mg_sigs_set = True
    base = dict(ndim=2, coord=0, n=[16, 16, 1], xmin=[0, 0, 0], dx=[1 / 16, 1 / 16, 1], bc=[[0, 0]] * 3)
    bad = [dict(base, n=[12, 16, 1], levels=4),
           dict(base, coord=2, bc=[[1, 1], [3, 1], [1, 1]]), dict(base, bc=[[2, 0], [0, 0], [0, 0]]),
           dict(base, power=2), dict(base, coarse=0), dict(base, n=[16, 16, 2]), dict(base, ndim=4),
           dict(base, power2=9), dict(base, n=[12, 16, 1], bc=[[2, 2], [0, 0], [0, 0]], levels=3),
           dict(base, smoother=2), dict(base, n=[2048, 16, 1], dx=[1 / 2048, 1 / 16, 1], smoother=1)]
    for p in bad:
        h = ctypes.c_void_p()
        assert L.gmunu_mg_create(ctypes.byref(gmu.make_mg_desc(p)), ctypes.byref(h)) == -1, p
        assert not h.value


def test_static_step_rejects_what_its_scratch_cannot_hold():
    """gmunu_step_static refuses, before any device call, a grid with more
    than 8192 cells per axis (its static tables) and the limiter (which
    needs a third state)."""
    import math

    import workloads as W

    L = gmu.lib()
    buf = (ctypes.c_double * 16)()
    a = ctypes.cast(buf, ctypes.c_void_p)
    p = W.grid(1, W.CART, [8189], [0, 0, 0], [1, 1, 1], [[1, 1]])
    rc = L.gmunu_step_static(ctypes.byref(gmu.make_desc(p)), a, a, a, a, None, 0.4, 1.0, a, a, None, None, None)
    assert rc == -1
    p = W.grid(1, W.CART, [64], [0, 0, 0], [1, 1, 1], [[1, 1]], pp_limiter=1)
    rc = L.gmunu_step_static(ctypes.byref(gmu.make_desc(p)), a, a, a, a, None, 0.4, 1.0, a, a, None, None, None)
    assert rc == -1
    assert L.gmunu_step_static(None, a, a, a, a, None, 0.4, 1.0, a, a, None, None, None) == -2
