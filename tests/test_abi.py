"""Host-only checks of the C ABI: the library loads, exports every function
that include/ebof.h declares, and validates parameters without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2112_10591_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ebof.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ebof_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = L.load()
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.exported_symbols()) == names


def test_params_default_follow_paper_settings():
    lo = L.ebof_params_default(346, 260)
    hi = L.ebof_params_default(1280, 720)
    assert (lo.n_d, lo.n_f, lo.levels) == (1, 4, 3)
    assert (hi.n_d, hi.n_f, hi.levels) == (2, 3, 4)
    assert abs(lo.alpha - 1.08) < 1e-6 and lo.patch == 8 and lo.stride == 4
    assert L.ebof_pyramid_floats(lo) == 346 * 260 + 173 * 130 + 87 * 65
    assert L.ebof_pyramid_floats(hi) == 1_224_000


@pytest.mark.parametrize("field,value", [
    ("width", 7), ("width", 8193), ("height", 0), ("levels", 0), ("levels", 9), ("n_d", -1),
    ("n_f", 6), ("alpha", 0.0), ("alpha", float("nan")), ("alpha", 1000.0), ("patch", 16),
    ("stride", 0), ("stride", 9), ("iters", -1), ("iters", 2000), ("lambda_reg", 0.0),
    ("dt_us", 0), ("flags", 16), ("struct_size", 12)])
def test_validate_rejects(field, value):
    p = L.ebof_params_default(346, 260)
    setattr(p, field, value)
    assert L.ebof_validate(p) == L.EBOF_E_INVAL
    assert L.load().ebof_last_error(None).decode() != ""


def test_levels_must_hold_a_patch():
    p = L.ebof_params_default(346, 260, levels=7)  # 346 -> ... -> 6 px wide
    assert L.ebof_validate(p) == L.EBOF_E_INVAL
    p = L.ebof_params_default(20, 20)
    assert p.levels == 2 and L.ebof_validate(p) == L.EBOF_OK


def test_create_rejects_bad_arena():
    lib = L.load()
    h = ctypes.c_void_p()
    assert lib.ebof_create(0, None, 1 << 20, ctypes.byref(h)) == L.EBOF_E_INVAL
    assert lib.ebof_create(0, ctypes.c_void_p(0x1001), 1 << 20, ctypes.byref(h)) == L.EBOF_E_INVAL


def test_stage_calls_reject_null_context():
    lib = L.load()
    p = L.ebof_params_default(64, 64)
    assert lib.ebof_bin_events(None, ctypes.byref(p), None, None, None, 0, 0, None, None, None) == L.EBOF_E_INVAL
    assert lib.ebof_flow(None, ctypes.byref(p), None, None, None, None, None) == L.EBOF_E_INVAL


def test_set_tuning_rejects_null_context():
    lib = L.load()
    assert lib.ebof_set_tuning(None, L.EBOF_TUNE_AUTO, None) == L.EBOF_E_INVAL


def test_stream_signals_reject_null_context():
    lib = L.load()
    assert lib.ebof_stream_signal(None, 0, 1, None) == L.EBOF_E_INVAL
    assert lib.ebof_stream_wait(None, 0, 1, None) == L.EBOF_E_INVAL
    v = __import__("ctypes").c_uint32()
    assert lib.ebof_signal_read(None, 0, __import__("ctypes").byref(v)) == L.EBOF_E_INVAL
    st = __import__("ctypes").c_void_p()
    assert lib.ebof_stream_create(None, __import__("ctypes").byref(st)) == L.EBOF_E_INVAL
    assert lib.ebof_window_surface(None, None, None, None, None, 0, 0, None, None, None, None, None) == L.EBOF_E_INVAL



def test_flow_noalloc_host_checks():
    """The allocation-free flow call checks its arguments on the host, before
    any device work: NULL buffers, bad parameters, and a pyramid with more
    patches than the fixed scratch holds."""
    lib = L.load()
    p = L.ebof_params_default(346, 260)
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    assert lib.ebof_flow_noalloc(ctypes.byref(p), None, dummy, None, dummy, None) == L.EBOF_E_INVAL
    assert lib.ebof_flow_noalloc(ctypes.byref(p), dummy, dummy, None, None, None) == L.EBOF_E_INVAL
    bad = L.ebof_params_default(346, 260, stride=0)
    assert lib.ebof_flow_noalloc(ctypes.byref(bad), dummy, dummy, None, dummy, None) == L.EBOF_E_INVAL
    big = L.ebof_params_default(8192, 8192, stride=1, levels=1)
    assert lib.ebof_flow_noalloc(ctypes.byref(big), dummy, dummy, None, dummy, None) == L.EBOF_E_NOMEM
    assert "fixed scratch" in lib.ebof_last_error(None).decode()


def test_filter_params_and_state_size():
    """The flow filter's defaults follow Sec. IV-A (three layers; at 346x260
    weights 500 / 250 / 50 and 5 / 25 / 50 smoothing iterations from the
    finest layer, 500 and 20 at every layer for HD), its state holds two
    planes per layer, and bad settings are refused on the host."""
    lo = L.ebof_filter_params_default(346, 260)
    hi = L.ebof_filter_params_default(1280, 720)
    assert lo.layers == 3 and list(lo.gamma)[:3] == [500.0, 250.0, 50.0] and list(lo.smooth)[:3] == [5, 25, 50]
    assert hi.layers == 3 and list(hi.gamma)[:3] == [500.0] * 3 and list(hi.smooth)[:3] == [20] * 3
    p = L.ebof_params_default(346, 260)
    assert L.ebof_filter_state_floats(p, lo) == 2 * (346 * 260 + 173 * 130 + 87 * 65)
    lib = L.load()
    for field, value in [("layers", 0), ("layers", 4), ("gamma", 0.0), ("gamma", float("nan")),
                         ("gamma", float("inf")), ("smooth", -1), ("smooth", 1001)]:
        fp = L.ebof_filter_params_default(346, 260)
        if field == "layers":
            fp.layers = value
        else:
            getattr(fp, field)[1] = value
        assert lib.ebof_filter_state_floats(ctypes.byref(p), ctypes.byref(fp)) == -1, (field, value)
    assert lib.ebof_filter_params_default(346, 260, None) == L.EBOF_E_INVAL
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: the checks fail first
    assert lib.ebof_flow_filter(None, ctypes.byref(p), ctypes.byref(lo), dummy, dummy, None, dummy, dummy,
                                None) == L.EBOF_E_INVAL
