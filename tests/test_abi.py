"""CPU checks of the C ABI: the library loads, exports every symbol that
include/pclb.h declares, and rejects invalid configurations before touching
the device."""
import ctypes
import os
import re

import pytest

from paper_1302_7104_amd import _native as N
from paper_1302_7104_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pclb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pclb_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(N.SYMBOLS) == declared_symbols()


def test_library_exports_every_declared_symbol():
    L = N.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def cfg(**kw):
    base = dict(n_r=64, n_theta=128, r1=1.0, r2=2.0, tau=1e-4, dt=1e-3, n_i=8, n_f=8,
                precision=64, fp64_collision=1, kernel=0, strip_chunk=0, strip_order=0,
                adjoint_tie=0.0, scheme=0, relaxation=0)
    base.update(kw)
    return N.Config(*[base[k] for k, _ in N.Config._fields_])


def test_cfl_dt_matches_workload_rule():
    c = cfg()
    dt = N.lib().pclb_cfl_dt(ctypes.byref(c), 0.3)
    assert abs(dt - W.cfl_dt(64, 128, 1.0, 2.0, 0.3)) < 1e-18
    assert N.lib().pclb_cfl_dt(ctypes.byref(cfg(r1=-1.0)), 0.3) < 0
    # a sector of one eighth: dtheta is 8 times smaller
    dt1 = N.lib().pclb_cfl_dt(ctypes.byref(cfg(n_f=1, n_theta=20)), 0.3)
    assert abs(dt1 - W.cfl_dt(64, 20, 1.0, 2.0, 0.3, nf=1)) < 1e-18
    assert N.lib().pclb_cfl_dt(ctypes.byref(cfg(n_f=0)), 0.3) < 0
    # the double and triple octagon: dtheta = 2 pi n_f / (n_i n_theta)
    for ni, nf in ((16, 16), (16, 3), (24, 24), (24, 7)):
        d = N.lib().pclb_cfl_dt(ctypes.byref(cfg(n_i=ni, n_f=nf, n_theta=40)), 0.3)
        assert abs(d - W.cfl_dt(64, 40, 1.0, 2.0, 0.3, nf=nf, ni=ni)) < 1e-18, (ni, nf)
    assert N.lib().pclb_cfl_dt(ctypes.byref(cfg(n_i=16, n_f=17)), 0.3) < 0
    assert N.lib().pclb_cfl_dt(ctypes.byref(cfg(n_i=12, n_f=8)), 0.3) < 0


@pytest.mark.parametrize("kw,code", [
    (dict(r1=0.0), -1), (dict(r2=0.5), -1), (dict(n_r=3), -1), (dict(n_theta=4), -1),
    (dict(tau=0.0), -1), (dict(dt=-1.0), -1), (dict(n_i=12), -1), (dict(n_i=32), -1),
    (dict(n_f=0), -1), (dict(n_f=9), -1), (dict(n_i=16, n_f=17), -1), (dict(n_i=24, n_f=25), -1), (dict(n_f=1, dt=2e-3), -2),
    (dict(precision=16), -1), (dict(kernel=7), -1), (dict(dt=0.01), -2),
    (dict(fp64_collision=0), -1), (dict(adjoint_tie=-1.0), -1), (dict(adjoint_tie=0.5), -1),
    (dict(scheme=4), -1), (dict(scheme=-1), -1), (dict(relaxation=2), -1),
])
def test_create_rejects_invalid_config(kw, code):
    L = N.lib()
    ctx = ctypes.c_void_p()
    rc = L.pclb_create(ctypes.byref(cfg(**kw)), ctypes.byref(ctx))
    assert rc == code
    assert not ctx.value
    assert L.pclb_last_error(None)


@pytest.mark.parametrize("field,val", [("strip_chunk", 65), ("strip_chunk", -1),
                                       ("strip_order", 3), ("strip_order", -1)])
def test_create_rejects_strip_shape_out_of_range(field, val):
    """The strip kernel holds 1/r of a chunk one row per lane: more than 64
    rows per chunk (or an unknown workgroup order) is refused at creation,
    before any device call."""
    L = N.lib()
    ctx = ctypes.c_void_p()
    rc = L.pclb_create(ctypes.byref(cfg(**{field: val})), ctypes.byref(ctx))
    assert rc == -1
    assert not ctx.value
    assert b"launch shape" in L.pclb_last_error(None)
