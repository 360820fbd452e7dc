"""The C-ABI library loads, exports every declared entry point, and rejects
invalid arguments before touching a device (runs without a GPU)."""
import ctypes as C
import os
import re

import pytest

from paper_2002_04894_amd import fmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmm.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fmm.lib()
    names = declared()
    assert len(names) >= 14
    for nm in names:
        assert hasattr(lib, nm), nm


def _build(x=1, y=1, z=1, n=10, levels=2, theta=0.5):
    h = C.c_void_p()
    rc = fmm.lib().fmm_build(x, y, z, n, levels, theta, None, C.byref(h))
    return rc, h.value


@pytest.mark.parametrize("kw,frag", [
    (dict(x=None), "NULL"), (dict(z=None), "NULL"),
    (dict(n=0), "n must"), (dict(n=-5), "n must"), (dict(n=2 ** 31), "n must"),
    (dict(levels=-1), "levels"), (dict(levels=9), "levels"),
    (dict(theta=1.0), "theta"), (dict(theta=-0.1), "theta"), (dict(theta=float("nan")), "theta"),
])
def test_build_rejects_invalid_arguments(kw, frag):
    rc, h = _build(**kw)
    assert rc == fmm.FMM_EINVAL and h is None
    assert frag in fmm.fmm_last_error()


def test_build_rejects_null_out():
    rc = fmm.lib().fmm_build(1, 1, 1, 10, 2, 0.5, None, None)
    assert rc == fmm.FMM_EINVAL


@pytest.mark.parametrize("p,frag", [(-1, "p must"), (21, "p must")])
def test_evaluate_rejects_order(p, frag):
    rc = fmm.lib().fmm_evaluate(1, 1, 1, 1, 10, 0.5, p, 2, 1, 1, 1, 1, None)
    assert rc == fmm.FMM_EINVAL and frag in fmm.fmm_last_error()


def test_evaluate_rejects_null_outputs():
    rc = fmm.lib().fmm_evaluate(1, 1, 1, 1, 10, 0.5, 5, 2, 1, None, 1, 1, None)
    assert rc == fmm.FMM_EINVAL and "output" in fmm.fmm_last_error()
    rc = fmm.lib().fmm_evaluate(1, 1, 1, None, 10, 0.5, 5, 2, 1, 1, 1, 1, None)
    assert rc == fmm.FMM_EINVAL and "charge" in fmm.fmm_last_error()


def test_null_handle_rejected():
    L = fmm.lib()
    assert L.fmm_evaluate_tree(None, 1, 5, 1, 1, 1, 1, None) == fmm.FMM_EINVAL
    assert L.fmm_tree_perm(None, 1) == fmm.FMM_EINVAL
    assert L.fmm_tree_lists(None, 0, 0, None, None, None) == fmm.FMM_EINVAL
    assert L.fmm_free(None) == fmm.FMM_OK


def test_parts_rejected():
    # invalid handle check comes first; parts is validated on a real handle in the GPU tests
    assert fmm.lib().fmm_evaluate_tree_parts(None, 1, 5, 7, 1, 1, 1, 1, None) == fmm.FMM_EINVAL


def test_last_timings_rejects_null():
    assert fmm.lib().fmm_last_timings(None) == fmm.FMM_EINVAL


def test_bytes_estimate():
    e = fmm.fmm_bytes_estimate
    assert e(0, 2, 0.5, 5) == 0 and e(100, 9, 0.5, 5) == 0 and e(100, 2, 1.0, 5) == 0
    assert e(10 ** 6, 5, 0.5, 15) > e(10 ** 5, 5, 0.5, 15) > 0
    assert e(10 ** 6, 5, 0.5, 15) > e(10 ** 6, 5, 0.5, 8)
    assert e(10 ** 6, 5, 0.4, 15) > e(10 ** 6, 5, 0.6, 15)


def test_no_device_reports_edevice():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present; valid-argument calls need real device pointers")
    rc, h = _build()
    assert rc == fmm.FMM_EDEVICE and "device" in fmm.fmm_last_error()


def test_build_rejects_mismatched_lengths_before_the_library():
    """x, y and z of different lengths are refused in the binding, before any
    pointer reaches the library (a short y or z would be read past its end)."""
    import torch
    x = torch.zeros(10, dtype=torch.float64)
    short = torch.zeros(9, dtype=torch.float64)
    with pytest.raises(ValueError, match="same length"):
        fmm.fmm_build(x, short, x, 2, 0.5)
    with pytest.raises(ValueError, match="same length"):
        fmm.fmm_build(x, x, short, 2, 0.5)
    with pytest.raises(ValueError, match="same length"):
        fmm.fmm_build_ex(x, short, x, 2, 0.5)


def test_set_allocator_arguments():
    L = fmm.lib()
    assert L.fmm_set_allocator(fmm.ALLOC_FN(lambda n, s, u: 0), fmm.FREE_FN(), None) == fmm.FMM_EINVAL
    assert "both" in fmm.fmm_last_error()
    assert L.fmm_set_allocator(fmm.ALLOC_FN(), fmm.FREE_FN(lambda p, s, u: None), None) == fmm.FMM_EINVAL
    fmm.fmm_set_allocator(lambda n, s: 0, lambda p, s: None)
    fmm.fmm_set_allocator()  # back to the default pool
    with pytest.raises(ValueError):
        fmm.fmm_set_allocator(lambda n, s: 0)


def test_tree_bytes_rejects_null_handle():
    assert fmm.lib().fmm_tree_bytes(None, 5, 0, None, None) == fmm.FMM_EINVAL
