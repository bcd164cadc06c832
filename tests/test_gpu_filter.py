"""GPU parity of the update-prediction flow filter (ebof_flow_filter) against
the oracle's (oracle.flow_filter), step after step so that the carried state
is checked too: every layer's state and the output flow within the flow bars
(mean endpoint error 0.01 px, and per pixel p99.9 1e-3 px), both sides
starting from their own window pyramids built from the same events (the
GPU's checked against the oracle's first).  Cases: 346x260 and 1280x720 with
Sec. IV-A's settings, an odd size with a smoothing count that is not a
multiple of the launch's eight iterations and the masked output, zero motion
(exactly zero), and the argument checks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_10591_amd import synth
from flowcheck import FLOW_MEAN, FLOW_P999, epe, ref_window, say

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


def gpu_pyramid(ctx, p, ev):
    W, H = p.width, p.height
    edge = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    pyr = torch.empty(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
    L.ebof_window_surface(ctx, p, dev(ev["x"]), dev(ev["y"]), dev(ev["t"]), ev["t0"], edge, pyr)
    return pyr, edge


def layer_view(state, W, H, l):
    return oracle.filter_layer(state, W, H, l)


def run_sequence(ctx, p, fp, wins, tag, check_mask=False):
    """Filter steps over consecutive windows on both sides, compared after
    every step."""
    W, H = p.width, p.height
    F = fp.layers
    gam = [float(fp.gamma[l]) for l in range(F)]
    smo = [int(fp.smooth[l]) for l in range(F)]
    n_state = L.ebof_filter_state_floats(p, fp)
    state = torch.zeros(n_state, dtype=torch.float32, device="cuda")
    flow = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    ost = None
    prev = None
    for k, ev in enumerate(wins):
        r = ref_window(p, ev)
        pyr, edge = gpu_pyramid(ctx, p, ev)
        torch.cuda.synchronize()
        np.testing.assert_allclose(pyr.cpu().numpy(), r["pyr"], rtol=1e-6, atol=1e-7)
        if prev is not None:
            r0, pyr0, edge0 = prev
            L.ebof_flow_filter(ctx, p, fp, pyr0, pyr, state, flow, mask=edge0 if check_mask else None)
            of, ost = oracle.flow_filter(r0["pyr"], r["pyr"], W, H, p.levels, gam, smo, ost)
            torch.cuda.synchronize()
            g = flow.cpu().numpy().reshape(2, H, W).astype(np.float64)
            gs = state.cpu().numpy().astype(np.float64)
            for l in range(F):
                e = epe(layer_view(gs, W, H, l), layer_view(ost, W, H, l))
                say(f"  {tag} step {k} layer {l}: |flow| max {np.abs(layer_view(ost, W, H, l)).max():.3f}, "
                    f"EPE vs oracle mean {e.mean():.2e} p99.9 {np.percentile(e, 99.9):.2e} max {e.max():.2e}")
                assert e.mean() <= FLOW_MEAN and np.percentile(e, 99.9) <= FLOW_P999, (tag, k, l)
            want = of
            if check_mask:
                m = r0["Edf"].astype(bool)
                want = np.where(m[None], of, 0.0)
                assert np.all(g[:, ~m] == 0.0), (tag, k)
            e = epe(g, want)
            assert e.mean() <= FLOW_MEAN and np.percentile(e, 99.9) <= FLOW_P999, (tag, k)
        prev = (r, pyr, edge)
    return ost


def test_filter_c1_sequence(ctx):
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
    fp = L.ebof_filter_params_default(s.W, s.H)
    st = run_sequence(ctx, p, fp, [s.window(k) for k in range(5)], "C1 346x260")
    assert np.abs(oracle.filter_layer(st, s.W, s.H, 0)).max() > 0.1  # it tracked some motion


def test_filter_c2_sequence(ctx):
    wins = synth.generate("c2", 0, range(3), workers=4)
    p = L.ebof_params_default(1280, 720, flags=L.EBOF_MASK_FLOW)
    fp = L.ebof_filter_params_default(1280, 720)
    run_sequence(ctx, p, fp, wins, "C2 1280x720")


def test_filter_odd_size_masked(ctx):
    """203x117, two layers of a three-level pyramid, 9 and 3 smoothing
    iterations (two launches and one), the output masked to E_df of the
    reference window."""
    s = synth.c1_stream(1)
    W, H = 203, 117
    wins = []
    for k in range(4):
        w = s.window(k)
        keep = (w["x"] < W) & (w["y"] < H)
        wins.append(dict(x=w["x"][keep], y=w["y"][keep], t=w["t"][keep], t0=w["t0"]))
    p = L.ebof_params_default(W, H, flags=L.EBOF_MASK_FLOW, levels=3)
    fp = L.ebof_filter_params_default(W, H, layers=2, gamma=[120.0, 30.0], smooth=[9, 3])
    run_sequence(ctx, p, fp, wins, "odd 203x117", check_mask=True)


def test_filter_zero_motion_is_exactly_zero(ctx):
    s = synth.c1_stream(2)
    p = L.ebof_params_default(s.W, s.H)
    fp = L.ebof_filter_params_default(s.W, s.H)
    pyr, _ = gpu_pyramid(ctx, p, s.window(0))
    state = torch.zeros(L.ebof_filter_state_floats(p, fp), dtype=torch.float32, device="cuda")
    flow = torch.full((2 * s.W * s.H,), 7.0, dtype=torch.float32, device="cuda")
    for _ in range(2):
        L.ebof_flow_filter(ctx, p, fp, pyr, pyr, state, flow)
    torch.cuda.synchronize()
    assert torch.count_nonzero(flow).item() == 0 and torch.count_nonzero(state).item() == 0


def test_filter_argument_checks(ctx):
    import ctypes
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    fp = L.ebof_filter_params_default(s.W, s.H)
    lib, h = ctx.lib, ctx.handle
    buf = torch.zeros(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
    b = ctypes.c_void_p(buf.data_ptr())
    assert lib.ebof_flow_filter(h, ctypes.byref(p), ctypes.byref(fp), b, b, None, None, b, None) == L.EBOF_E_INVAL
    assert lib.ebof_flow_filter(h, ctypes.byref(p), None, b, b, None, b, b, None) == L.EBOF_E_INVAL
    fp.layers = 4
    assert lib.ebof_flow_filter(h, ctypes.byref(p), ctypes.byref(fp), b, b, None, b, b, None) == L.EBOF_E_INVAL
    assert "layers" in lib.ebof_last_error(h).decode()


@pytest.mark.parametrize("W,H,levels,layers,smooth", [(8, 8, 1, 1, [3]), (16, 17, 2, 2, [0, 17]),
                                                       (67, 45, 3, 3, [8, 1, 16])])
def test_filter_random_state_and_images(ctx, W, H, levels, layers, smooth):
    """Random pyramids (not surfaces) and a random previous state of up to
    3 px, at the smallest sizes and smoothing counts of 0, 1, 8, 16 and 17
    (one partial launch, exactly one or two full ones, and two plus one)."""
    rng = np.random.default_rng(W * 100 + H)
    p = L.ebof_params_default(W, H, levels=levels)
    fp = L.ebof_filter_params_default(W, H, layers=layers, gamma=[40.0, 90.0, 300.0][:layers], smooth=smooth)
    P = L.ebof_pyramid_floats(p)
    pyr0 = rng.random(P).astype(np.float32)
    pyr1 = rng.random(P).astype(np.float32)
    st0 = rng.uniform(-3.0, 3.0, L.ebof_filter_state_floats(p, fp)).astype(np.float32)
    state = dev(st0)
    flow = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow_filter(ctx, p, fp, dev(pyr0), dev(pyr1), state, flow)
    of, ost = oracle.flow_filter(pyr0, pyr1, W, H, levels, [float(fp.gamma[l]) for l in range(layers)], smooth,
                                 st0.astype(np.float64))
    torch.cuda.synchronize()
    gs = state.cpu().numpy().astype(np.float64)
    for l in range(layers):
        e = epe(layer_view(gs, W, H, l), layer_view(ost, W, H, l))
        say(f"  {W}x{H} layer {l}: EPE vs oracle mean {e.mean():.2e} max {e.max():.2e}")
        assert e.mean() <= FLOW_MEAN and np.percentile(e, 99.9) <= FLOW_P999, (W, H, l)
    e = epe(flow.cpu().numpy().reshape(2, H, W).astype(np.float64), of)
    assert e.mean() <= FLOW_MEAN and np.percentile(e, 99.9) <= FLOW_P999
