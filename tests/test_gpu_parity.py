"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer stages (edge image, denoise/fill, squared distances) must be
bit-exact; the surface is compared bit-exactly too (both sides round the same
double-precision expression once); pyramid levels within 1e-6 relative; the
flow within 0.01 px mean endpoint error of the oracle and per pixel within
the bars of flowcheck.py.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2112_10591_amd import synth
from flowcheck import OracleFlow, assert_flow_matches, epe, oracle_flow, ref_window

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2112_10591_amd._lib")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = L.ebof_create(arena_bytes=1 << 30)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def gpu_window(ctx, p, ev, d2=True):
    W, H = p.width, p.height
    x, y, t = dev(ev["x"]), dev(ev["y"]), dev(ev["t"])
    edge = torch.empty(H * W, dtype=torch.uint8, device="cuda")
    pyr = torch.empty(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
    d2o = torch.empty(H * W, dtype=torch.int32, device="cuda") if d2 else None
    nd = torch.zeros(1, dtype=torch.uint64, device="cuda")
    L.ebof_bin_events(ctx, p, x, y, t, ev["t0"], edge, nd)
    L.ebof_edt_surface(ctx, p, edge, pyr, d2o)
    torch.cuda.synchronize()
    out = dict(edge=edge.cpu().numpy().reshape(H, W), pyr=pyr.cpu().numpy(), dropped=int(nd.cpu().to(torch.int64)))
    if d2:
        out["d2"] = d2o.cpu().numpy().reshape(H, W)
    out["_pyr_dev"] = pyr
    out["_edge_dev"] = edge
    return out


def check_window(g, r, p):
    assert np.array_equal(g["edge"], r["Edf"]), "edge image differs"
    assert g["dropped"] == r["dropped"]
    assert np.array_equal(g["d2"], r["D2"]), "squared distances differ"
    P0 = p.width * p.height
    assert np.array_equal(g["pyr"][:P0], r["S"].ravel()), "surface differs"
    rel = np.abs(g["pyr"].astype(np.float64) - r["pyr"]) / np.maximum(np.abs(r["pyr"]), 1e-30)
    assert rel.max() <= 1e-6, f"pyramid rel err {rel.max()}"


def random_events(W, H, n, seed, t0=0, dt=10_000, spill=0):
    rng = np.random.default_rng(seed)
    x = rng.integers(0, W + spill, n).astype(np.uint16)
    y = rng.integers(0, H + spill, n).astype(np.uint16)
    t = np.sort(rng.integers(t0 - spill * 10, t0 + dt + spill * 10, n)).astype(np.int64)
    return dict(x=x, y=y, t=t, t0=t0)


# --------------------------------------------------------------------------
# edge image, denoise/fill, EDT, surface, pyramid
# --------------------------------------------------------------------------
@pytest.mark.parametrize("W,H,n,levels", [
    (8, 8, 20, 1), (13, 9, 40, 1), (64, 64, 300, 3), (65, 130, 2000, 3), (67, 45, 900, 2),
    (346, 260, 20_000, 3), (200, 33, 3000, 2), (1280, 720, 300_000, 4), (1280, 720, 200_000, 5),
    (2048, 1100, 120_000, 8),
])
def test_window_random_events(ctx, W, H, n, levels):
    for seed, spill in [(1, 0), (2, 5)]:
        _say(f"window random W={W} H={H} n={n} seed={seed} spill={spill}")
        p = L.ebof_params_default(W, H, levels=levels)
        ev = random_events(W, H, n, seed, spill=spill)
        check_window(gpu_window(ctx, p, ev), ref_window(p, ev), p)


@pytest.mark.parametrize("n_d,n_f", [(0, 5), (1, 4), (2, 3), (0, 0), (5, 1), (3, 2), (4, 4)])
def test_denoise_fill_thresholds(ctx, n_d, n_f):
    _say(f"denoise/fill n_d={n_d} n_f={n_f}")
    p = L.ebof_params_default(150, 90, n_d=n_d, n_f=n_f, levels=2)
    ev = random_events(150, 90, 6000, 7)
    check_window(gpu_window(ctx, p, ev), ref_window(p, ev), p)


def test_empty_and_full_images(ctx):
    p = L.ebof_params_default(100, 70, n_d=0, n_f=5, levels=2)
    _say("empty window")
    ev = dict(x=np.zeros(0, np.uint16), y=np.zeros(0, np.uint16), t=np.zeros(0, np.int64), t0=0)
    g = gpu_window(ctx, p, ev)
    assert g["edge"].sum() == 0 and np.all(g["d2"] == 2**31 - 1) and np.all(g["pyr"] == 1.0)
    _say("all events outside the window")
    ev = random_events(100, 70, 500, 3, t0=50_000)
    ev["t0"] = 0
    g = gpu_window(ctx, p, ev)
    assert g["edge"].sum() == 0 and g["dropped"] == 500
    _say("every pixel an edge")
    yy, xx = np.mgrid[0:70, 0:100]
    ev = dict(x=xx.ravel().astype(np.uint16), y=yy.ravel().astype(np.uint16),
              t=np.zeros(7000, np.int64), t0=0)
    g = gpu_window(ctx, p, ev)
    assert g["edge"].all() and np.all(g["d2"] == 0) and np.all(g["pyr"][:7000] == 0.0)
    _say("single edge pixel, far corners")
    ev = dict(x=np.array([99], np.uint16), y=np.array([0], np.uint16), t=np.zeros(1, np.int64), t0=0)
    g = gpu_window(ctx, p, ev)
    check_window(g, ref_window(p, ev), p)


def test_c1_c2_windows(ctx):
    for s, k in [(synth.c1_stream(0), 0), (synth.c1_stream(0), 1), (synth.c2_stream(0), 3)]:
        _say(f"config window {s.config_id} k={k}")
        p = L.ebof_params_default(s.W, s.H)
        ev = s.window(k)
        check_window(gpu_window(ctx, p, ev), ref_window(p, ev), p)


def test_max_width_sampled(ctx):
    """8192-wide sensor (the maximum): the squared distance checked by brute
    force at sampled pixels, the edge image in full."""
    W, H = 8192, 16
    p = L.ebof_params_default(W, H, levels=1)
    ev = random_events(W, H, 50, 11)
    _say(f"max width {W}x{H}")
    g = gpu_window(ctx, p, ev)
    r = ref_window(p, ev)
    assert np.array_equal(g["edge"], r["Edf"])
    rng = np.random.default_rng(0)
    for _ in range(200):
        x, y = int(rng.integers(0, W)), int(rng.integers(0, H))
        assert g["d2"][y, x] == oracle.edt_brute_at(r["Edf"], x, y)
    assert np.array_equal(g["d2"], r["D2"])


# --------------------------------------------------------------------------
# flow
# --------------------------------------------------------------------------
def gpu_flow(ctx, p, pyr0, pyr1, mask=None):
    W, H = p.width, p.height
    f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow(ctx, p, pyr0, pyr1, f, mask=mask)
    torch.cuda.synchronize()
    return f.cpu().numpy().reshape(2, H, W).astype(np.float64)


def windows_gpu_and_oracle(ctx, p, evs):
    """Both sides from the same events: the GPU windows (checked bit for bit
    against the oracle's edge image, squared distances, surface and pyramid)
    and the oracle windows."""
    out = []
    for ev in evs:
        g = gpu_window(ctx, p, ev)
        r = ref_window(p, ev)
        check_window(g, r, p)
        out.append((g, r))
    return out


def test_flow_zero_motion_exact(ctx):
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    g = gpu_window(ctx, p, s.window(0), d2=False)
    _say("flow zero motion")
    f = gpu_flow(ctx, p, g["_pyr_dev"], g["_pyr_dev"])
    assert np.all(f == 0.0)


def test_kernel_timing_per_launch_and_span(ctx):
    """Kernel timing, with a pair per launch and with one pair around the
    launches a call makes back to back (the levels of the inverse search),
    counts every launch, reports positive times, resets on reading, and
    leaves the flow bit for bit as the untimed call's."""
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    g0 = gpu_window(ctx, p, s.window(0), d2=False)
    g1 = gpu_window(ctx, p, s.window(1), d2=False)
    want = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    _say("kernel timing: per launch, then spans")
    try:
        for span in (False, True):
            L.ebof_timing_enable(ctx, ["dis_level", "densify"], span=span)
            for _ in range(3):
                assert np.array_equal(gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"]), want)
            ms, cnt = L.ebof_timing_read(ctx, "dis_level")
            assert cnt == 3 * p.levels and ms > 0.0, (span, ms, cnt)
            ms, cnt = L.ebof_timing_read(ctx, "densify")
            assert cnt == 3 and ms > 0.0, (span, ms, cnt)
            assert L.ebof_timing_read(ctx, "dis_level") == (0.0, 0)
    finally:
        L.ebof_timing_enable(ctx, [])


@pytest.mark.parametrize("case", ["c1", "c2", "odd"])
def test_masked_flow_equals_dense_flow_masked(ctx, case):
    """With only the masked flow wanted, level 0 computes just the patches
    that hold a mask pixel (packed into the first waves of each item); the
    result must equal, bit for bit, the flow computed for every patch (the
    dense flow kept before masking) with the mask applied afterwards.  C1
    runs level 0 with 8 lanes per patch, C2 with 4, and the odd size has
    clamped border patches on both axes."""
    if case == "c2":
        W, H = 1280, 720
        evs = synth.generate("c2", 0, range(2), workers=2)
    else:
        s = synth.c1_stream(3)
        W, H = (s.W, s.H) if case == "c1" else (203, 117)
        evs = []
        for k in range(2):
            w = s.window(k)
            keep = (w["x"] < W) & (w["y"] < H)
            evs.append(dict(x=w["x"][keep], y=w["y"][keep], t=w["t"][keep], t0=w["t0"]))
    p = L.ebof_params_default(W, H, flags=L.EBOF_MASK_FLOW)
    g0 = gpu_window(ctx, p, evs[0], d2=False)
    g1 = gpu_window(ctx, p, evs[1], d2=False)
    _say(f"masked vs dense flow {case} ({W}x{H})")
    f = torch.full((2 * W * H,), 7.0, dtype=torch.float32, device="cuda")
    L.ebof_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"], f, mask=g0["_edge_dev"])
    fk = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    dense = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow_warm(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"], fk, flow_dense_out=dense, mask=g0["_edge_dev"])
    torch.cuda.synchronize()
    m = g0["_edge_dev"].cpu().numpy().reshape(H, W).astype(bool)
    f, fk, dense = (a.cpu().numpy().reshape(2, H, W) for a in (f, fk, dense))
    assert 0 < m.mean() < 0.5
    assert np.array_equal(fk, np.where(m[None], dense, 0.0))
    assert np.array_equal(f, fk)
    assert np.abs(dense[:, m]).max() > 0.1  # some motion on the mask


def test_flow_empty_windows_exact_zero(ctx):
    """A window with no events has the surface 1.0 everywhere: as the
    reference its template gradient is 0, so b = 0 and no patch moves; the
    flow is exactly 0 whatever the other window holds."""
    p = L.ebof_params_default(346, 260)
    empty = dict(x=np.zeros(0, np.uint16), y=np.zeros(0, np.uint16), t=np.zeros(0, np.int64), t0=0)
    s = synth.c1_stream(0)
    (ge, re), (g1, r1) = windows_gpu_and_oracle(ctx, p, [empty, s.window(1)])
    assert np.all(re["pyr"] == 1.0)
    _say("flow empty -> empty, empty -> C1 window")
    f = gpu_flow(ctx, p, ge["_pyr_dev"], ge["_pyr_dev"])
    assert np.all(f == 0.0)
    f = gpu_flow(ctx, p, ge["_pyr_dev"], g1["_pyr_dev"])
    assert np.all(f == 0.0)
    assert np.all(oracle_flow(p, re, r1) == 0.0)


def test_flow_c1_parity_and_known_translation(ctx):
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [s.window(0), s.window(1)])
    _say("flow C1 pair (346x260, L3)")
    f = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    assert_flow_matches(f, OracleFlow(p, r0, r1), "C1")
    m = g0["edge"][16:-16, 16:-16].astype(bool)
    assert abs(np.median(f[0][16:-16, 16:-16][m]) - 2.5) <= 0.05
    assert abs(np.median(f[1][16:-16, 16:-16][m]) + 1.5) <= 0.05


@pytest.mark.parametrize("d", [(2, -1), (-3, 2)])
def test_flow_integer_shift(ctx, d):
    """Two windows with the same sparse random events, the second shifted by
    an integer displacement (no denoise/fill): the flow recovers the shift
    away from the border, and matches the oracle."""
    H, W = 120, 160
    rng = np.random.default_rng(5)
    n = int(0.03 * W * H)
    x, y = rng.integers(0, W, n), rng.integers(0, H, n)
    x1, y1 = x + d[0], y + d[1]
    keep = (x1 >= 0) & (x1 < W) & (y1 >= 0) & (y1 < H)
    p = L.ebof_params_default(W, H, levels=3, n_d=0, n_f=5)
    ev0 = dict(x=x.astype(np.uint16), y=y.astype(np.uint16), t=np.zeros(n, np.int64), t0=0)
    ev1 = dict(x=x1[keep].astype(np.uint16), y=y1[keep].astype(np.uint16),
               t=np.zeros(int(keep.sum()), np.int64), t0=0)
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [ev0, ev1])
    _say(f"flow integer shift {d}")
    f = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    inner = (slice(12, H - 12), slice(12, W - 12))
    e = np.hypot(f[0][inner] - d[0], f[1][inner] - d[1])
    assert np.median(e) < 1e-4 and np.mean(e < 0.05) > 0.98
    assert_flow_matches(f, OracleFlow(p, r0, r1), f"shift {d}")


def test_flow_smooth_texture_damped_bias(ctx):
    """A smooth texture shifted by (2, -1) px, pyramids uploaded directly.
    At lambda = 0.3 the 16 damped steps stop short on weakly textured
    patches (the solver's bias against the true shift, a property of the
    method as configured); the GPU must reproduce the oracle's flow, bias
    included, to the per-pixel bar."""
    ndi = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(6)
    H, W, d = 120, 160, (2, -1)
    big = ndi.gaussian_filter(rng.random((H + 8, W + 8)), 2.0)
    big = (big - big.min()) / (big.max() - big.min())
    I0 = big[4:4 + H, 4:4 + W].astype(np.float32)
    I1 = big[4 - d[1]:4 - d[1] + H, 4 - d[0]:4 - d[0] + W].astype(np.float32)
    p = L.ebof_params_default(W, H, levels=3)
    pyr0, _ = oracle.pyramid(I0, 3)
    pyr1, _ = oracle.pyramid(I1, 3)
    _say("flow smooth texture, damped")
    f = gpu_flow(ctx, p, dev(pyr0), dev(pyr1))
    r = oracle.dis_flow(pyr0, pyr1, W, H, 3, lam=float(np.float32(p.lambda_reg)))
    assert_flow_matches(f, r, "smooth texture")
    inner = (slice(12, H - 12), slice(12, W - 12))
    bias = np.hypot(r[0][inner] - d[0], r[1][inner] - d[1])
    _say(f"  oracle bias to the true shift: median {np.median(bias):.2e} p90 {np.percentile(bias, 90):.2e} px")
    assert np.median(bias) < 0.05


def test_flow_c2_parity(ctx):
    s = synth.c2_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [s.window(4), s.window(5)])
    _say("flow C2 pair (1280x720, L4)")
    f = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    assert_flow_matches(f, OracleFlow(p, r0, r1), "C2")


def test_flow_c5_parity(ctx):
    """The stress workload: 1280x720, 2M events per window, 30 % noise, eight
    polygons moving up to 20 px over an expansion field, 5 levels."""
    s = synth.c5_stream(0)
    p = L.ebof_params_default(s.W, s.H, levels=5)
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [s.window(0), s.window(1)])
    _say("flow C5 pair (1280x720, L5, 2M events)")
    f = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    assert_flow_matches(f, OracleFlow(p, r0, r1), "C5")


def test_flow_mask_vs_oracle(ctx):
    """EBOF_MASK_FLOW: the flow is the oracle's on the reference window's
    edge pixels (E_df of window k-1, Sec. III-D) and exactly 0 elsewhere."""
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [s.window(0), s.window(1)])
    _say("flow masked")
    fm = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"], mask=g0["_edge_dev"])
    m = r0["Edf"].astype(bool)
    # pixels off the mask skip their sums: the same bits as masking the dense flow
    fd = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
    assert np.array_equal(fm, np.where(m[None], fd, 0.0))
    ref = OracleFlow(p, r0, r1, mask=True)
    assert np.all(fm[:, ~m] == 0.0)
    assert_flow_matches(fm, ref, "masked C1")
    assert_flow_matches(fm, ref, "masked C1, edge pixels", where=m)


def test_flow_odd_sizes_and_strides(ctx):
    for (W, H, lv, st) in [(8, 8, 1, 4), (9, 17, 1, 3), (77, 51, 3, 4), (130, 66, 2, 2), (64, 40, 2, 8),
                           (520, 400, 5, 4), (10, 10, 1, 4), (18, 26, 1, 3)]:
        _say(f"flow odd W={W} H={H} L={lv} stride={st}")
        p = L.ebof_params_default(W, H, levels=lv, stride=st, n_d=0, n_f=5)
        ev0 = random_events(W, H, max(4, W * H // 6), 21)
        ev1 = random_events(W, H, max(4, W * H // 6), 22)
        (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, [ev0, ev1])
        f = gpu_flow(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"])
        assert_flow_matches(f, OracleFlow(p, r0, r1), f"{W}x{H} L{lv} s{st}")


# --------------------------------------------------------------------------
# warm start of the coarsest level from the previous pair's flow
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_flow_warm_start_chain_vs_oracle(ctx, cfg):
    """Three consecutive windows: the pair (0, 1) cold, then (1, 2) started
    from the first pair's flow before masking (ebof_flow_warm), against the
    oracle's own chain (its cold flow fed to its warm start).  The dense copy
    equals the unmasked flow, the masked output is 0 off the reference edge
    pixels, and the warm start does change the flow."""
    s = synth.c1_stream(0) if cfg == "c1" else synth.c2_stream(0)
    p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
    W, H = s.W, s.H
    (g0, r0), (g1, r1), (g2, r2) = windows_gpu_and_oracle(ctx, p, [s.window(k) for k in (0, 1, 2)])
    _say(f"warm start chain {cfg} ({W}x{H}, L{p.levels})")
    f01 = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    d01 = torch.full((2 * W * H,), float("nan"), dtype=torch.float32, device="cuda")
    f12 = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    d12 = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    cold = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow_warm(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"], f01, flow_dense_out=d01, mask=g0["_edge_dev"])
    L.ebof_flow_warm(ctx, p, g1["_pyr_dev"], g2["_pyr_dev"], f12, flow_init=d01, flow_dense_out=d12,
                     mask=g1["_edge_dev"])
    L.ebof_flow(ctx, p, g1["_pyr_dev"], g2["_pyr_dev"], cold, mask=g1["_edge_dev"])
    torch.cuda.synchronize()
    sh = (2, H, W)
    f01, d01, f12, d12, cold = (a.cpu().numpy().reshape(sh).astype(np.float64) for a in (f01, d01, f12, d12, cold))
    o01 = OracleFlow(p, r0, r1)
    o12 = OracleFlow(p, r1, r2, prev_flow=o01.raw)
    assert_flow_matches(d01, o01, f"{cfg} pair (0,1) cold, dense")
    assert_flow_matches(d12, o12, f"{cfg} pair (1,2) warm, dense")
    m1 = r1["Edf"].astype(bool)
    assert np.array_equal(f12, np.where(m1[None], d12, 0.0))
    assert not np.array_equal(f12, cold), "the warm start changed nothing"
    o12c = oracle_flow(p, r1, r2)
    _say(f"  warm vs cold oracle flows differ at {np.mean(epe(o12.raw, o12c) > 1e-3):.1%} of pixels")


def test_flow_warm_start_constant_velocity(ctx):
    """A constant previous flow v seeds every coarsest-level patch with
    v / 2^(L-1) exactly: on a zero-motion pair (I1 = I0) whose reference is
    flat (an empty window: every gradient 0, so no step moves a patch), the
    coarsest level keeps that start and every finer level doubles it back,
    so the flow is v everywhere, exactly, on both sides."""
    p = L.ebof_params_default(200, 120, levels=3)
    W, H = 200, 120
    empty = dict(x=np.zeros(0, np.uint16), y=np.zeros(0, np.uint16), t=np.zeros(0, np.int64), t0=0)
    (g, r), = windows_gpu_and_oracle(ctx, p, [empty])
    v = (2.5, -1.5)
    prev = np.stack([np.full((H, W), v[0]), np.full((H, W), v[1])])
    f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    _say("warm start, constant velocity on a flat reference")
    L.ebof_flow_warm(ctx, p, g["_pyr_dev"], g["_pyr_dev"], f, flow_init=dev(prev.astype(np.float32)))
    torch.cuda.synchronize()
    f = f.cpu().numpy().reshape(2, H, W)
    assert np.all(f[0] == v[0]) and np.all(f[1] == v[1])
    o = oracle_flow(p, r, r, prev_flow=prev)
    assert np.all(o[0] == v[0]) and np.all(o[1] == v[1])


# --------------------------------------------------------------------------
# the distance-surface alternatives of the ablation study (Sec. IV-B)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [1, 2, 3])
def test_surface_kinds_vs_oracle(ctx, kind):
    """DS_L, DS_LB and DS_Log in place of eq. (1): the surface bit for bit
    against the oracle's formula on the same squared distances (an empty
    window included: the no-edge sentinel), the pyramid within 1e-6."""
    for W, H, n, lv in [(346, 260, 20_000, 3), (1280, 720, 300_000, 4), (100, 70, 0, 2)]:
        _say(f"surface kind {kind} {W}x{H} n={n}")
        p = L.ebof_params_default(W, H, levels=lv, surface=kind)
        ev = random_events(W, H, n, 40 + kind)
        g = gpu_window(ctx, p, ev)
        r = ref_window(p, ev)
        assert np.array_equal(g["edge"], r["Edf"]) and np.array_equal(g["d2"], r["D2"])
        S = oracle.surface_kind(r["D2"], float(np.float32(p.alpha)), kind)
        assert np.array_equal(g["pyr"][:W * H], S.ravel()), "surface differs"
        ref, _ = oracle.pyramid(S, lv)
        rel = np.abs(g["pyr"].astype(np.float64) - ref) / np.maximum(np.abs(ref), 1e-30)
        assert rel.max() <= 1e-6


def test_flow_on_bounded_surface_vs_oracle(ctx):
    """The whole path on the DS_LB surface (C1 pair): the flow against the
    oracle's flow between the oracle's DS_LB pyramids."""
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H, surface=L.EBOF_SURFACE_BOUNDED)
    rs, gs = [], []
    for k in (0, 1):
        ev = s.window(k)
        g = gpu_window(ctx, p, ev)
        r = ref_window(p, ev)
        S = oracle.surface_kind(r["D2"], float(np.float32(p.alpha)), L.EBOF_SURFACE_BOUNDED)
        r["pyr"], _ = oracle.pyramid(S, p.levels)
        assert np.array_equal(g["pyr"][:s.W * s.H], S.ravel())
        rs.append(r)
        gs.append(g)
    _say("flow on the DS_LB surface (C1)")
    f = gpu_flow(ctx, p, gs[0]["_pyr_dev"], gs[1]["_pyr_dev"])
    d_sat = float(np.float32(p.alpha)) * np.log(255.0)
    assert_flow_matches(f, OracleFlow(p, rs[0], rs[1]), "C1 DS_LB", scale=d_sat)


# --------------------------------------------------------------------------
# variational refinement of every level (the third stage of dense inverse
# search)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("cfg", ["c1", "c2", "odd"])
def test_flow_variational_refinement_vs_oracle(ctx, cfg):
    """EBOF_VAR_REFINE: every level's dense flow refined before the next
    starts from it, against the oracle's refined flow; masked output equal to
    the masked dense copy; the refinement changes the flow."""
    if cfg == "odd":
        W, H = 130, 66
        p = L.ebof_params_default(W, H, levels=2, stride=3, n_d=0, n_f=5,
                                  flags=L.EBOF_VAR_REFINE | L.EBOF_MASK_FLOW)
        evs = [random_events(W, H, W * H // 6, 31), random_events(W, H, W * H // 6, 32)]
    else:
        s = synth.c1_stream(0) if cfg == "c1" else synth.c2_stream(0)
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_VAR_REFINE | L.EBOF_MASK_FLOW)
        evs = [s.window(k) for k in (0, 1)]
    W, H = p.width, p.height
    (g0, r0), (g1, r1) = windows_gpu_and_oracle(ctx, p, evs)
    _say(f"refined flow {cfg} ({W}x{H}, L{p.levels})")
    f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    dense = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow_warm(ctx, p, g0["_pyr_dev"], g1["_pyr_dev"], f, flow_dense_out=dense, mask=g0["_edge_dev"])
    plain = L.ebof_params_default(W, H, levels=p.levels, stride=p.stride, n_d=p.n_d, n_f=p.n_f)
    fp = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    L.ebof_flow(ctx, plain, g0["_pyr_dev"], g1["_pyr_dev"], fp)
    torch.cuda.synchronize()
    f, dense, fp = (a.cpu().numpy().reshape(2, H, W).astype(np.float64) for a in (f, dense, fp))
    m = r0["Edf"].astype(bool)
    assert np.array_equal(f, np.where(m[None], dense, 0.0))
    assert_flow_matches(dense, OracleFlow(p, r0, r1), f"refined {cfg}")
    assert np.abs(dense - fp).max() > 1e-3, "the refinement changed nothing"


def test_variational_refinement_refused_outside_stage_calls(ctx):
    p = L.ebof_params_default(346, 260, flags=L.EBOF_VAR_REFINE)
    with pytest.raises(L.EbofError) as ei:
        L.ebof_stream_open(ctx, p)
    assert ei.value.code == L.EBOF_E_INVAL
