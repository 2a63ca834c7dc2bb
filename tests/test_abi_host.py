"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every symbol include/piv.h declares; piv_plan validates parameters;
entry points reject bad arguments before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2504_17987_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2504_17987_amd import build
        build.build(verbose=False)
    return _lib


def test_exports_match_header(L):
    hdr = open(os.path.join(ROOT, "include", "piv.h")).read()
    declared = set(re.findall(r"\b(piv_[a-z_]+)\s*\(", hdr))
    assert declared == set(L.EXPORTS)
    lib = L.lib()
    for name in declared:
        assert hasattr(lib, name), name


def plan(L, **kw):
    p = L.Params()
    L.lib().piv_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    h = C.c_void_p()
    s = L.lib().piv_plan(C.byref(p), C.byref(h))
    return s, h


def test_defaults_are_the_papers(L):
    p = L.Params()
    L.lib().piv_params_default(C.byref(p))
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_params.json")))
    assert p.win == g["window_px"] and p.step == g["window_px"] * (1 - g["step_over"])
    assert abs(p.uod_threshold - g["uod_threshold"]) < 1e-7
    assert abs(p.uod_epsilon - g["uod_regulariser_px"]) < 1e-7


@pytest.mark.parametrize("kw,status", [
    (dict(win=15), 1), (dict(win=4), 1), (dict(width=1020), 1), (dict(radius=0), 1),
    (dict(radius=17), 1), (dict(levels=7), 1), (dict(dtype=9), 1), (dict(win=66, step=8), 1),
    (dict(radius_coarse=30, levels=4), 1), (dict(max_batch=0), 1),
    (dict(dtype=2, bit_depth=10), 1), (dict(dtype=3, levels=3), 2), (dict(block=36), 2),
    (dict(), 0), (dict(dtype=2, bit_depth=12, win=24, step=12, width=3840, height=2160), 0),
])
def test_plan_validation(L, kw, status):
    s, h = plan(L, **kw)
    assert s == status, L.lib().piv_last_error()
    if s == 0:
        L.lib().piv_plan_destroy(h)
    else:
        assert not h.value and L.lib().piv_last_error()


def test_workspace_and_argument_errors(L):
    s, h = plan(L, max_batch=4)
    assert s == 0
    lib = L.lib()
    per = lib.piv_plan_workspace_bytes(h, 1)
    assert per > 0 and lib.piv_plan_workspace_bytes(h, 4) == 4 * per
    fake = C.c_void_p(1 << 20)   # never dereferenced: calls fail before any launch
    # no workspace bound
    assert lib.piv_predict(h, fake, fake, 1024, 1, fake, None) == L.PIV_ENOWORKSPACE
    # misaligned workspace and too small workspace
    assert lib.piv_plan_bind_workspace(h, C.c_void_p((1 << 20) + 4), per) == L.PIV_EINVAL
    assert lib.piv_plan_bind_workspace(h, fake, per - 1) == L.PIV_ENOWORKSPACE
    assert lib.piv_plan_bind_workspace(h, fake, 2 * per) == 0
    assert lib.piv_predict(h, fake, fake, 1024, 3, fake, None) == L.PIV_ENOWORKSPACE
    assert lib.piv_predict(h, fake, fake, 1024, 5, fake, None) == L.PIV_EINVAL      # n > max_batch
    assert lib.piv_correct(h, fake, fake, 1022, 1, None, fake, None, fake, None) == L.PIV_EINVAL  # pitch
    assert lib.piv_correct(h, None, fake, 1024, 1, None, fake, None, fake, None) == L.PIV_EINVAL
    assert lib.piv_correct(h, fake, fake, 1024, 1, None, None, None, fake, None) == L.PIV_EINVAL
    assert lib.piv_ssd_forward(h, fake, fake, fake, 1, fake, None) == L.PIV_EINVAL  # not an F32 plan
    assert lib.piv_status_string(3) == b"PIV_ENOWORKSPACE"
    # n = 0 is a no-op that succeeds
    assert lib.piv_vorticity(h, fake, fake, 0, None) == 0
    lib.piv_plan_destroy(h)
