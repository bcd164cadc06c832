"""Adaptive windows on the GPU against the oracle: the window end under the
area event count rule (exact: an index), and the binning of an index range
(no time test) bit for bit, through the distance surface and pyramid."""
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
    c = L.ebof_create(arena_bytes=1 << 30)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _say(msg):
    print(msg, flush=True)


def test_window_end_random_streams(ctx):
    rng = np.random.default_rng(11)
    for trial in range(30):
        W, H = int(rng.integers(8, 400)), int(rng.integers(8, 300))
        a = int(rng.integers(4, 64))
        while ((W + a - 1) // a) * ((H + a - 1) // a) > 8192:
            a *= 2
        n = int(rng.integers(0, 60_000))
        x = rng.integers(0, W + 4, n).astype(np.uint16)
        y = rng.integers(0, H + 4, n).astype(np.uint16)
        i0 = int(rng.integers(0, n + 1))
        k = int(rng.integers(1, 400))
        want = oracle.window_end_area(W, H, x, y, i0, a, k)
        got = L.ebof_window_end(ctx, W, H, dev(x), dev(y), i0, a, k)
        assert got == (i0, want), (trial, W, H, a, n, i0, k)


def test_window_end_edge_cases(ctx):
    W, H = 64, 48
    x = np.array([70, 3, 3, 3, 40, 3], np.uint16)  # the first is off the sensor
    y = np.array([0, 2, 2, 2, 40, 2], np.uint16)
    for i0, a, k in [(0, 16, 1), (0, 16, 3), (0, 16, 5), (2, 16, 2), (6, 16, 1), (0, 64, 4), (0, 1, 2)]:
        want = oracle.window_end_area(W, H, x, y, i0, a, k)
        assert L.ebof_window_end(ctx, W, H, dev(x), dev(y), i0, a, k) == (i0, want), (i0, a, k)
    with pytest.raises(L.EbofError):
        L.ebof_window_end(ctx, 8192, 8192, dev(x), dev(y), 0, 8, 10)  # over 8192 squares


def test_window_end_stress_stream(ctx):
    """2M events of the stress workload (many chunks): ends for several
    starts, square sides and counts."""
    s = synth.c5_stream(0)
    ev = s.window(0)
    x, y = dev(ev["x"]), dev(ev["y"])
    n = len(ev["x"])
    for i0, a, k in [(0, 32, 200), (123_457, 32, 1500), (0, 128, 20_000), (1_000_000, 16, 40), (0, 2048, 1_500_000),
                     (0, 64, 10_000_000)]:
        _say(f"window end, 2M events: i0={i0} square={a} k={k}")
        want = oracle.window_end_area(s.W, s.H, ev["x"], ev["y"], i0, a, k)
        assert L.ebof_window_end(ctx, s.W, s.H, x, y, i0, a, k) == (i0, want)
    assert want == n


def test_range_binning_and_surface(ctx):
    """Consecutive adaptive windows of a 1280x720 stream: each index range
    binned without a time test, the edge image, squared distances and
    pyramid bit for bit against the oracle on the same events."""
    s = synth.c2_stream(0)
    evs = [s.window(k) for k in (0, 1)]
    x = np.concatenate([e["x"] for e in evs])
    y = np.concatenate([e["y"] for e in evs])
    t = np.concatenate([e["t"] for e in evs])
    p = L.ebof_params_default(s.W, s.H)
    W, H = s.W, s.H
    xd, yd = dev(x), dev(y)
    i0 = 0
    for w in range(3):
        rng_dev = torch.empty(2, dtype=torch.int64, device="cuda")
        L.ebof_window_end(ctx, W, H, xd, yd, i0, 32, 120, range_out=rng_dev)
        edge = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        pyr = torch.empty(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
        d2 = torch.empty(W * H, dtype=torch.int32, device="cuda")
        L.ebof_window_surface_range(ctx, p, xd, yd, rng_dev, edge, pyr, d2_out=d2)
        torch.cuda.synchronize()
        a, b = rng_dev.cpu().tolist()
        assert a == i0 and b == oracle.window_end_area(W, H, x, y, i0, 32, 120)
        _say(f"adaptive window {w}: events [{a}, {b})")
        sl = slice(a, b)
        r = oracle.window(W, H, x[sl], y[sl], np.zeros(b - a, np.int64), 0, 1, p.n_d, p.n_f,
                          float(np.float32(p.alpha)), p.levels)
        assert np.array_equal(edge.cpu().numpy().reshape(H, W), r["Edf"])
        assert np.array_equal(d2.cpu().numpy().reshape(H, W), r["D2"])
        assert np.array_equal(pyr.cpu().numpy(), r["pyr"])
        i0 = b
