"""Pins of the oracle's evaluation kit (Sec. IV): the distance-surface
alternatives of the ablation study, the average endpoint error and outlier
rate, and the flow warp loss.  Values come from closed forms worked by hand
or from constants the mathematics fixes, chosen so that a dropped term, a
wrong sign or a swapped threshold fails one of them."""
import numpy as np
import pytest

import oracle


# --------------------------------------------------------------------------
# surfaces (Sec. IV-B ablations)
# --------------------------------------------------------------------------
def test_surface_linear_is_the_distance():
    D2 = np.array([0, 1, 4, 9, 2, 2**31 - 1], np.int32)
    S = oracle.surface_kind(D2, 1.08, oracle.SURFACE_LINEAR)
    assert S[:4].tolist() == [0.0, 1.0, 2.0, 3.0]
    assert S[4] == np.float32(1.4142135623730951)          # sqrt 2
    assert S[5] == np.float32(46340.950001051984)          # sqrt(2^31 - 1): the no-edge sentinel


def test_surface_bounded_saturates_at_dsat():
    """alpha = 6 / ln 255 makes d_sat = alpha ln 255 = 6 px (the paper's bound)."""
    a = 6.0 / np.log(255.0)
    D2 = np.array([0, 1, 25, 35, 36, 37, 100, 2**31 - 1], np.int32)
    S = oracle.surface_kind(D2, a, oracle.SURFACE_BOUNDED)
    assert S[:3].tolist() == [0.0, 1.0, 5.0]
    assert S[3] == np.float32(5.916079783099616)           # sqrt 35, below the bound
    assert np.all(S[4:] == 6.0)
    # at alpha = 1.08 the bound is 1.08 ln 255 = 5.984564... px
    S = oracle.surface_kind(np.array([36, 35], np.int32), 1.08, oracle.SURFACE_BOUNDED)
    assert S[0] == np.float32(5.98456462877110) and S[1] == np.float32(5.916079783099616)


def test_surface_log():
    D2 = np.array([0, 1, 9, 2**31 - 1], np.int32)
    S = oracle.surface_kind(D2, 1.08, oracle.SURFACE_LOG)
    assert S[0] == 0.0
    assert S[1] == np.float32(0.6931471805599453)          # ln 2
    assert S[2] == np.float32(1.3862943611198906)          # ln 4
    assert S[3] == np.float32(10.743802877399936)          # ln(46341.950001...)


def test_surface_kind_zero_is_equation_one_and_all_kinds_grow():
    D2 = np.arange(0, 2000, dtype=np.int32)
    assert np.array_equal(oracle.surface_kind(D2, 1.08, oracle.SURFACE_EXP), oracle.surface(D2, 1.08))
    for k in range(4):
        S = oracle.surface_kind(D2, 1.08, k)
        assert S[0] == 0.0 and np.all(np.diff(S) >= 0)


# --------------------------------------------------------------------------
# AEE and outliers
# --------------------------------------------------------------------------
def _field(H, W, a, b):
    return np.stack([np.full((H, W), a, np.float64), np.full((H, W), b, np.float64)])


def test_aee_and_outliers_closed_forms():
    H, W = 4, 5
    # |v - u| = 5 (3-4-5), above 3 px and above 5 % of |v| = 0.25
    aee, out, n = oracle.flow_errors(_field(H, W, 0, 0), _field(H, W, 3, 4))
    assert (aee, out, n) == (5.0, 1.0, 20)
    # error 3.5 px on a 100 px motion: above 3 px but within 5 % (5 px)
    aee, out, _ = oracle.flow_errors(_field(H, W, 96.5, 0), _field(H, W, 100, 0))
    assert aee == 3.5 and out == 0.0
    # error 3.5 px on a 10 px motion: both thresholds passed
    aee, out, _ = oracle.flow_errors(_field(H, W, 13.5, 0), _field(H, W, 10, 0))
    assert aee == 3.5 and out == 1.0
    # exactly 3 px is not above 3 px
    _, out, _ = oracle.flow_errors(_field(H, W, 0, 0), _field(H, W, 0, 3))
    assert out == 0.0


def test_aee_mask_selects_pixels():
    H, W = 3, 4
    u = _field(H, W, 0, 0)
    v = _field(H, W, 1, 0)
    v[0, 0, 0] = 11.0   # one far-off pixel, outside the mask
    m = np.ones((H, W), np.uint8)
    m[0, 0] = 0
    aee, out, n = oracle.flow_errors(u, v, m)
    assert (aee, out, n) == (1.0, 0.0, 11)
    aee, out, n = oracle.flow_errors(u, v)
    assert n == 12 and aee == pytest.approx(22.0 / 12.0, rel=1e-15) and out == pytest.approx(1.0 / 12.0)


# --------------------------------------------------------------------------
# flow warp loss
# --------------------------------------------------------------------------
def _track(n=8, x0=10, y0=7, dt=8000):
    """A point moving +1 px per dt/8 along x: one event at each position."""
    k = np.arange(n)
    return (np.array(x0 + k, np.uint16), np.full(n, y0, np.uint16), (k * dt // n).astype(np.int64))


def test_fwl_zero_flow_is_one():
    W, H = 40, 20
    x, y, t = _track()
    r, vc, vu = oracle.fwl(W, H, x, y, t, 0, 8000, np.zeros((2, H, W)))
    assert r == 1.0 and vc == vu


def test_fwl_true_flow_stacks_the_track():
    """With the flow (8, 0) px per window every event goes back to x0: one
    pixel holds 8 votes instead of 8 pixels holding one, so with N pixels
    FWL = (64/N - 64/N^2) / (8/N - 64/N^2) = 8 (N - 1) / (N - 8)."""
    W, H = 40, 20
    N = W * H
    x, y, t = _track()
    r, vc, vu = oracle.fwl(W, H, x, y, t, 0, 8000, _field(H, W, 8, 0))
    assert vu == pytest.approx(8 / N - 64 / N**2, rel=1e-14)
    assert vc == pytest.approx(64 / N - 64 / N**2, rel=1e-14)
    assert r == pytest.approx(8 * (N - 1) / (N - 8), rel=1e-14)
    # the flow taken the wrong way spreads the track over twice the length
    r_wrong, _, _ = oracle.fwl(W, H, x, y, t, 0, 8000, _field(H, W, -8, 0))
    assert r_wrong == pytest.approx(1.0, rel=1e-14)


def test_fwl_polarity_and_bilinear_votes():
    W, H = 40, 20
    N = W * H
    x, y, t = _track()
    pol = np.array([1, -1] * 4, np.int8)
    r, vc, vu = oracle.fwl(W, H, x, y, t, 0, 8000, _field(H, W, 8, 0), pol=pol)
    assert vc == 0.0 and vu == pytest.approx(8 / N, rel=1e-14) and r == 0.0
    # one event half-way through the window under the flow (1, 0): half a
    # vote at x - 1 and half at x
    r, vc, vu = oracle.fwl(W, H, np.array([5], np.uint16), np.array([3], np.uint16),
                           np.array([4000], np.int64), 0, 8000, _field(H, W, 1, 0))
    assert vc == pytest.approx(0.5 / N - 1 / N**2, rel=1e-14)
    assert vu == pytest.approx(1 / N - 1 / N**2, rel=1e-14)


def test_fwl_skips_events_off_the_window_or_sensor():
    W, H = 40, 20
    x, y, t = _track()
    xs = np.concatenate([x, np.array([45, 3], np.uint16)])
    ys = np.concatenate([y, np.array([2, 25], np.uint16)])
    ts = np.concatenate([t, np.array([100, 100], np.int64)])
    xs = np.concatenate([xs, np.array([3], np.uint16)])
    ys = np.concatenate([ys, np.array([3], np.uint16)])
    ts = np.concatenate([ts, np.array([8000], np.int64)])   # t0 + dt: outside the half-open window
    a = oracle.fwl(W, H, x, y, t, 0, 8000, _field(H, W, 8, 0))
    b = oracle.fwl(W, H, xs, ys, ts, 0, 8000, _field(H, W, 8, 0))
    assert a == b
