"""The C-ABI library loads and exports every symbol include/*.h declares, and
host-side validation rejects bad problems without touching a GPU.  CPU only:
no compute call is made."""
import ctypes as C
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2603_12550_amd", "libvds.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2603_12550_amd import build as b
        b.build()
    return C.CDLL(LIB)


def declared_functions():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w \*]*?\b(vds_\w+)\s*\(", src, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_python_binding_covers_the_header():
    from paper_2603_12550_amd import _vds
    assert set(declared_functions()) <= set(_vds.EXPORTED)


def _problem(**kw):
    from paper_2603_12550_amd import _vds
    return _vds.make_problem(**{**dict(nb=3, P=1000, h=0.4), **kw})


@pytest.mark.parametrize("bad", [dict(nb=0), dict(nb=6), dict(P=0), dict(h=0.0), dict(h=float("nan")),
                                 dict(dt=-1e-3), dict(zeta=0.0), dict(kT=-1.0),
                                 dict(potential="fene", b_max=0.0), dict(picard_max=0),
                                 dict(picard_rtol=0.0), dict(picard_batch=0), dict(picard_predictor=2)])
def test_invalid_problems_are_rejected_before_any_launch(lib, bad):
    from paper_2603_12550_amd import _vds
    pr = _problem(**bad)
    H = (C.c_double * 6)(*([1.0] * 6))
    ctx = C.c_void_p()
    st = _vds._lib.vds_create(C.byref(pr), H, None, C.byref(ctx))
    assert st == _vds.VDS_ERR_ARG
    assert not ctx.value
    assert _vds._lib.vds_last_error(None)
    assert _vds._lib.vds_workspace_bytes(C.byref(pr)) == 0


def test_valid_problem_creates_and_reports_workspace(lib):
    from paper_2603_12550_amd import _vds
    pr = _problem()
    H = (C.c_double * 3)(1.0, 1.0, 1.0)
    ctx = C.c_void_p()
    assert _vds._lib.vds_create(C.byref(pr), H, None, C.byref(ctx)) == _vds.VDS_OK
    assert _vds._lib.vds_workspace_bytes(C.byref(pr)) > 1000 * 9 * 4
    # calls before binding a workspace are call-order errors, caught on the host
    assert _vds._lib.vds_velocity(ctx, C.c_void_p(1), None, C.c_void_p(1), None) == _vds.VDS_ERR_STATE
    bad_h = (C.c_double * 3)(1.0, -1.0, 1.0)
    ctx2 = C.c_void_p()
    assert _vds._lib.vds_create(C.byref(pr), bad_h, None, C.byref(ctx2)) == _vds.VDS_ERR_ARG
    _vds._lib.vds_destroy(ctx)
