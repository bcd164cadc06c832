"""The evaluation kit of Sec. IV on the GPU against the oracle: endpoint
errors (AEE, outlier rate; per-pixel arithmetic in double without
contraction, so the outlier count is exact and the mean differs only by the
order of the sum) and the flow warp loss (fixed-point votes of 2^-32, so the
variances agree to far below 1e-9 relative)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_10591_amd import synth

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2112_10591_amd._lib")


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = L.ebof_create(arena_bytes=512 << 20)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("W,H", [(346, 260), (1280, 720), (7, 5)])
def test_flow_errors_vs_oracle(ctx, W, H):
    rng = np.random.default_rng(W)
    gt = (rng.normal(0, 4, (2, H, W))).astype(np.float32)
    fl = (gt + rng.normal(0, 2, (2, H, W)) * (rng.random((2, H, W)) < 0.3)).astype(np.float32)
    mask = (rng.random((H, W)) < 0.4).astype(np.uint8)
    for m in (None, mask):
        _say(f"flow errors {W}x{H} mask={m is not None}")
        aee, out, n = L.ebof_flow_errors(ctx, W, H, dev(fl), dev(gt), None if m is None else dev(m))
        ra, ro, rn = oracle.flow_errors(fl.astype(np.float64), gt.astype(np.float64), m)
        assert n == rn and out == ro
        assert aee == pytest.approx(ra, rel=1e-13)


def test_flow_errors_empty_mask(ctx):
    W, H = 20, 10
    z = np.zeros((2, H, W), np.float32)
    aee, out, n = L.ebof_flow_errors(ctx, W, H, dev(z), dev(z), dev(np.zeros((H, W), np.uint8)))
    assert (aee, out, n) == (0.0, 0.0, 0)


@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_fwl_vs_oracle(ctx, cfg):
    """Window k-1's events under the oracle's flow k-1 -> k (as floats),
    with and without polarity, against the oracle's FWL."""
    s = synth.c1_stream(0) if cfg == "c1" else synth.c2_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    W, H = s.W, s.H
    ev = s.window(3)
    rng = np.random.default_rng(1)
    flow = (rng.normal(0, 3, (2, H, W))).astype(np.float32)
    flow[0] += 2.5
    for pol in (None, ev["p"]):
        _say(f"fwl {cfg} polarity={pol is not None}")
        got = L.ebof_fwl(ctx, p, dev(ev["x"]), dev(ev["y"]), dev(ev["t"]), ev["t0"], dev(flow),
                         pol=None if pol is None else dev(pol))
        ref = oracle.fwl(W, H, ev["x"], ev["y"], ev["t"], ev["t0"], p.dt_us, flow.astype(np.float64), pol=pol)
        for g, r in zip(got, ref):
            assert g == pytest.approx(r, rel=1e-9, abs=1e-300)


def test_fwl_stacked_track_closed_form(ctx):
    """The oracle's closed form on the GPU: a point moving 8 px along x in a
    window, under the flow (8, 0): FWL = 8 (N - 1) / (N - 8)."""
    W, H = 40, 20
    N = W * H
    p = L.ebof_params_default(W, H, levels=1, dt_us=8000)
    k = np.arange(8)
    x, y, t = (10 + k).astype(np.uint16), np.full(8, 7, np.uint16), (k * 1000).astype(np.int64)
    flow = np.zeros((2, H, W), np.float32)
    flow[0] = 8.0
    r, vc, vu = L.ebof_fwl(ctx, p, dev(x), dev(y), dev(t), 0, dev(flow))
    assert r == pytest.approx(8 * (N - 1) / (N - 8), rel=1e-14)
