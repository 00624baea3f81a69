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
    assert ctypes.sizeof(gmu.GridDesc) == off["rk"] + 8


@pytest.mark.parametrize("mutate", [
    lambda p: p.update(ndim=4),
    lambda p: p.update(ng=1),
    lambda p: p.update(n=[400, 2, 1]),
    lambda p: p.update(gamma=1.0),
    lambda p: p.update(rk=4),
    lambda p: p.update(bc=[[W.PERIODIC, W.OUTFLOW], [5, 5], [5, 5]]),
    lambda p: p.update(dx=[0.0, 1.0, 1.0]),
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
    assert L.gmunu_rhs(None, None, None, None, None) == -2
    assert L.gmunu_c2p(None, None, None, None, None, None, None) == -2


def test_binding_raises_without_device_tensors():
    with pytest.raises(TypeError):
        gmu._ptr(object(), "x")
