"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
entry point declared in include/abd.h, and rejects invalid model descriptions
before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1709_04145_amd import abd, build
from paper_1709_04145_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(abd.LIB_PATH):
        build.build(force=False)
    return abd.load()


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "abd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("abd_create_model", "abd_destroy_model", "abd_step", "abd_objective_grad",
                     "abd_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
        assert name in abd._PROTOS, f"binding lacks a prototype for {name}"


def _desc_c(d):
    keep = [np.ascontiguousarray(d.link_offset, dtype=np.int32), np.ascontiguousarray(d.parent, dtype=np.int32),
            np.ascontiguousarray(d.dofs_per_link, dtype=np.int32), np.ascontiguousarray(d.axis, dtype=np.float64),
            np.ascontiguousarray(d.offset, dtype=np.float64), np.ascontiguousarray(d.mass_moment, dtype=np.float64)]
    ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    cd = abd.ModelDescC(d.n_models, ip(keep[0]), ip(keep[1]), ip(keep[2]), dp(keep[3]), dp(keep[4]),
                        dp(keep[5]), (C.c_double * 3)(*d.gravity))
    return cd, keep


def _create(lib, d):
    cd, keep = _desc_c(d)
    h = C.c_void_p()
    rc = lib.abd_create_model(C.byref(cd), C.byref(h))
    return rc, lib.abd_last_error().decode()


@pytest.mark.parametrize("mutate,needle", [
    (lambda d: d.axis.__setitem__((0, 0), 2.0), "unit vector"),
    (lambda d: d.mass_moment.__setitem__((1, 9), 0.0), "mass"),
    (lambda d: d.mass_moment.__setitem__((0, 0), -5.0), "PSD"),
    (lambda d: d.parent.__setitem__(1, 3), "precede"),
    (lambda d: d.dofs_per_link.__setitem__(0, 4), "dofs_per_link"),
    (lambda d: d.offset.__setitem__((2, 1), np.nan), "offset"),
])
def test_invalid_descriptions_are_rejected_on_the_host(lib, mutate, needle):
    d = W.config_models(1)
    mutate(d)
    rc, msg = _create(lib, d)
    assert rc == abd.ABD_EINVAL
    assert needle in msg


def test_null_arguments_are_rejected(lib):
    assert lib.abd_create_model(None, None) == abd.ABD_EINVAL
    assert lib.abd_step(None, None, None, None, None, None, None) == abd.ABD_EINVAL
    assert lib.abd_objective_grad(None, None, None, None, None, None, None, None) == abd.ABD_EINVAL
