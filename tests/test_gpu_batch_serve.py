"""Batched and served forms against the single-window stage calls.

Every window's outputs must be the same alone (stage calls) and inside a
batch of windows of other streams and resolutions, in the directly launched
batch, in every replay of its captured graph, and through the serving loop
(where windows of many streams arrive interleaved and are batched as they
come).  Designed for bit-identity: the kernels do the same arithmetic for a
window whatever else shares the launch.
"""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2112_10591_amd import synth
from flowcheck import OracleFlow, assert_flow_matches, ref_window

pytestmark = pytest.mark.gpu

L = pytest.importorskip("paper_2112_10591_amd._lib")


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = L.ebof_create(arena_bytes=3 << 30)
    yield c
    torch.cuda.synchronize()
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def mixed_streams(n_low=3, n_hd=2, windows=3):
    """(params, [events per window]) for a mix of 346x260 and 1280x720 streams."""
    out = []
    for i in range(n_low + n_hd):
        s = synth.c3_streams()[i if i < n_low else 10 + i - n_low]
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        evs = []
        for k in range(windows):
            w = s.window(k)
            evs.append(dict(x=dev(w["x"]), y=dev(w["y"]), t=dev(w["t"]), t0=w["t0"]))
        out.append((p, evs))
    return out


def alone(ctx, p, evs):
    """Stage calls, one window at a time: edge, d2, pyramid and flow per window."""
    W, H = p.width, p.height
    P = L.ebof_pyramid_floats(p)
    res, prev = [], None
    for ev in evs:
        e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        d2 = torch.empty(W * H, dtype=torch.int32, device="cuda")
        pr = torch.empty(P, dtype=torch.float32, device="cuda")
        L.ebof_bin_events(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], e)
        L.ebof_edt_surface(ctx, p, e, pr, d2)
        f = None
        if prev is not None:
            f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
            L.ebof_flow(ctx, p, prev[1], pr, f, mask=prev[0])
        res.append((e, pr, d2, f))
        prev = (e, pr)
    torch.cuda.synchronize()
    return res


def test_window_surface_equals_two_stage_calls(ctx):
    """ebof_window_surface (binning, fill with the column masks formed on the
    way, distance transform, surface, pyramid in one call) gives the bits of
    ebof_bin_events followed by ebof_edt_surface, also for a window with no
    events, and counts the same dropped events."""
    for p, evs in mixed_streams(n_low=1, n_hd=1, windows=3):
        ref = alone(ctx, p, evs)
        W, H = p.width, p.height
        P = L.ebof_pyramid_floats(p)
        empty = dict(x=evs[0]["x"][:0], y=evs[0]["y"][:0], t=evs[0]["t"][:0], t0=evs[0]["t0"])
        e0 = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        pr0 = torch.empty(P, dtype=torch.float32, device="cuda")
        L.ebof_bin_events(ctx, p, empty["x"], empty["y"], empty["t"], empty["t0"], e0)
        L.ebof_edt_surface(ctx, p, e0, pr0)
        for k, ev in enumerate(evs + [empty]):
            e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
            d2 = torch.empty(W * H, dtype=torch.int32, device="cuda")
            pr = torch.empty(P, dtype=torch.float32, device="cuda")
            nd = torch.zeros(1, dtype=torch.uint64, device="cuda")
            L.ebof_window_surface(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], e, pr, d2_out=d2, n_dropped=nd)
            nd_ref = torch.zeros(1, dtype=torch.uint64, device="cuda")
            L.ebof_bin_events(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], torch.empty_like(e), n_dropped=nd_ref)
            torch.cuda.synchronize()
            assert int(nd.item()) == int(nd_ref.item()), (W, k)
            if k < len(evs):
                assert torch.equal(e, ref[k][0]) and torch.equal(d2, ref[k][2]) and torch.equal(pr, ref[k][1]), (W, k)
            else:
                assert torch.equal(e, e0) and torch.equal(pr, pr0), (W, "no events")
                assert int((d2 != 2**31 - 1).sum()) == 0
        _say(f"window_surface {W}x{H}: {len(evs) + 1} windows")


def _crop(w, W, H):
    keep = (w["x"] < W) & (w["y"] < H)
    return dict(x=dev(w["x"][keep]), y=dev(w["y"][keep]), t=dev(w["t"][keep]), t0=w["t0"])


def test_capped_row_pass_equals_column_pass(ctx):
    """A window whose squared distances are not exported and whose surface
    saturates within 64 px takes the row pass that forms capped column
    distances from the column masks itself (no column pass); with squared
    distances exported, the column pass and the exact row pass run.  Edge
    image and pyramid are bit-identical between the two and the pyramid
    equals the oracle's: 346x260 and 1280x720 streams, alpha 3.5 (the
    surface saturates 61 px out: the widest band) and 4.5 (beyond 64 px: the
    column pass again), the bounded surface DS_LB, N_d / N_f at their
    extremes, sensors of 61x23 (one chunk), 70x300 (narrower than a row
    segment, five chunks), 600x130 and the smallest ones (8x8, 9x130,
    300x9: the band wider than the image), and a window with no events."""
    cases = list(mixed_streams(n_low=2, n_hd=1, windows=2))
    s = synth.c1_stream(3)
    c1 = [s.window(k) for k in range(2)]
    for over in (dict(alpha=3.5), dict(alpha=4.5), dict(surface=L.EBOF_SURFACE_BOUNDED), dict(n_d=0, n_f=5),
                 dict(n_d=4, n_f=1)):
        cases.append((L.ebof_params_default(s.W, s.H, **over), [_crop(w, s.W, s.H) for w in c1]))
    cases.append((L.ebof_params_default(61, 23, levels=1), [_crop(c1[1], 61, 23), _crop(c1[1], 0, 0)]))
    cases.append((L.ebof_params_default(70, 300, levels=2), [_crop(c1[0], 70, 300)]))
    for (w_, h_) in ((8, 8), (9, 130), (300, 9)):
        cases.append((L.ebof_params_default(w_, h_, levels=1, n_d=0), [_crop(c1[0], w_, h_), _crop(c1[1], w_, h_)]))
    hd = synth.c3_streams()[10].window(0)
    cases.append((L.ebof_params_default(600, 130, levels=2), [_crop(hd, 600, 130)]))
    for p, evs in cases:
        W, H = p.width, p.height
        P = L.ebof_pyramid_floats(p)
        for k, ev in enumerate(evs):
            outs = []
            for with_d2 in (True, False):
                e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
                pr = torch.full((P,), float("nan"), dtype=torch.float32, device="cuda")
                d2 = torch.empty(W * H, dtype=torch.int32, device="cuda") if with_d2 else None
                L.ebof_window_surface(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], e, pr, d2_out=d2)
                outs.append((e, pr))
            torch.cuda.synchronize()
            assert torch.equal(outs[0][0], outs[1][0]), (W, H, k, "edge")
            assert torch.equal(outs[0][1].view(torch.int32), outs[1][1].view(torch.int32)), (W, H, k, "pyramid")
            if p.surface == L.EBOF_SURFACE_BOUNDED:
                continue  # (the oracle's window takes eq. 1; the bounded surface is pinned in test_gpu_parity)
            r = oracle.window(W, H, ev["x"].cpu().numpy(), ev["y"].cpu().numpy(), ev["t"].cpu().numpy(), ev["t0"],
                              p.dt_us, p.n_d, p.n_f, float(np.float32(p.alpha)), p.levels)
            assert np.array_equal(outs[1][0].cpu().numpy().reshape(H, W), r["Edf"]), (W, H, k)
            np.testing.assert_allclose(outs[1][1].cpu().numpy(), r["pyr"], rtol=1e-6, atol=1e-7)
        _say(f"capped row pass {W}x{H} (alpha {p.alpha:.2f}, surface kind {p.surface}, N_d {p.n_d}, "
             f"N_f {p.n_f}): bit-identical")


@pytest.mark.parametrize("rows", [1, 2, 4, 8])
def test_batch_capped_row_pass_equals_alone(ctx, tmp_path, rows):
    """The batched form without squared distances (capped row pass, no
    column pass) at every row count the tuner can pick: pyramids and flows
    equal the stage calls' with squared distances exported."""
    streams = mixed_streams(n_low=2, n_hd=1, windows=2)
    ref = [alone(ctx, p, evs) for p, evs in streams]
    outs = _outs_for(streams, ref, 1)
    batch = _batch_of(streams, outs, 1)
    for w in batch:
        w["d2_out"] = None
    path = tmp_path / "tune.txt"
    vals = [rows, 64] + [4] * L.EBOF_TUNE_LEVELS + [0] * L.EBOF_TUNE_STAGES
    path.write_text(L.batch_layout_key(batch) + "\t" + " ".join(map(str, vals)) + "\n")
    L.ebof_set_tuning(ctx, L.EBOF_TUNE_AUTO, str(path))
    try:
        stream = torch.cuda.Stream()
        _say(f"batch, capped row pass, rows={rows}")
        L.ebof_run_batch(ctx, batch, stream=stream)
        torch.cuda.synchronize()
        for s_ in range(len(streams)):
            r, o = ref[s_][1], outs[s_]
            assert torch.equal(o["edge"], r[0]), (rows, s_, "edge")
            assert torch.equal(o["pyr"], r[1]), (rows, s_, "pyramid")
            assert torch.equal(o["flow"], r[3]), (rows, s_, "flow")
    finally:
        L.ebof_set_tuning(ctx, L.EBOF_TUNE_AUTO, None)


def test_batch_of_consecutive_windows_of_one_camera(ctx):
    """Consecutive windows of one camera in one batch (the batched form
    along time): window k's reference pyramid and mask are window k-1's,
    produced by the same batch's preprocessing stages, which all run before
    its flow stages.  Edge images, pyramids and flows equal the stage
    calls', in two consecutive batches (graph recorded, then replayed)."""
    s = synth.c1_stream(4)
    p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
    evs = []
    for k in range(17):
        w = s.window(k)
        evs.append(dict(x=dev(w["x"]), y=dev(w["y"]), t=dev(w["t"]), t0=w["t0"]))
    ref = alone(ctx, p, evs)
    N, P = s.W * s.H, L.ebof_pyramid_floats(p)
    edge = [torch.empty(N, dtype=torch.uint8, device="cuda") for _ in range(17)]
    pyr = [torch.empty(P, dtype=torch.float32, device="cuda") for _ in range(17)]
    flow = [torch.full((2 * N,), float("nan"), dtype=torch.float32, device="cuda") for _ in range(17)]
    L.ebof_window_surface(ctx, p, evs[0]["x"], evs[0]["y"], evs[0]["t"], evs[0]["t0"], edge[0], pyr[0])
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    for k0 in (1, 9):
        batch = [dict(params=p, x=evs[k]["x"], y=evs[k]["y"], t=evs[k]["t"], t0_us=evs[k]["t0"], edge_out=edge[k],
                      pyr_out=pyr[k], pyr_prev=pyr[k - 1], mask=edge[k - 1], flow_out=flow[k])
                 for k in range(k0, k0 + 8)]
        L.ebof_run_batch(ctx, batch, stream=stream)
    torch.cuda.synchronize()
    for k in range(1, 17):
        assert torch.equal(edge[k], ref[k][0]) and torch.equal(pyr[k], ref[k][1]), k
        assert torch.equal(flow[k], ref[k][3]), k
    _say("consecutive windows of one camera: two batches of 8, bit-identical to the stage calls")


def test_pipelined_driver_equals_sequential():
    """The benchmark's pipelined plain driver (each window's surface call and
    flow on stream k mod 4, ordered by the context counters, a buffer ring of
    5 so that slots are reused while earlier flows may still read them)
    gives every window the flow of the sequential stage calls."""
    import ctypes
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    c = L.ebof_create(arena_bytes=1 << 30)
    try:
        s = synth.c1_stream(0)
        nwin, NB = 20, 5
        wins = [s.window(k) for k in range(nwin)]
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        N, P = s.W * s.H, L.ebof_pyramid_floats(p)
        evs = [dict(x=dev(w["x"]), y=dev(w["y"]), t=dev(w["t"]), t0=w["t0"]) for w in wins]
        ref = alone(c, p, evs)
        streams = [L.ebof_stream_create(c) for _ in range(4)]
        sp = [ctypes.c_void_p(st.cuda_stream) for st in streams]
        edge = [torch.empty(N, dtype=torch.uint8, device="cuda") for _ in range(NB)]
        pyr = [torch.empty(P, dtype=torch.float32, device="cuda") for _ in range(NB)]
        flows = [torch.full((2 * N,), float("nan"), dtype=torch.float32, device="cuda") for _ in range(nwin)]
        torch.cuda.synchronize()
        lib, h, vp, pp = c.lib, c.handle, ctypes.c_void_p, ctypes.byref(p)

        def pre(k, i):
            e = evs[k]
            assert lib.ebof_window_surface(h, pp, vp(e["x"].data_ptr()), vp(e["y"].data_ptr()), vp(e["t"].data_ptr()),
                                           int(e["x"].numel()), int(e["t0"]), vp(edge[k % NB].data_ptr()), None, None,
                                           vp(pyr[k % NB].data_ptr()), sp[i]) == 0

        def flw(k, i):
            b, bp = k % NB, (k - 1) % NB
            assert lib.ebof_flow(h, pp, vp(pyr[bp].data_ptr()), vp(pyr[b].data_ptr()), vp(edge[bp].data_ptr()),
                                 vp(flows[k].data_ptr()), sp[i]) == 0

        run = bench.pipelined_driver(lib, h, sp, NB, 0, pre, flw)
        run(0, nwin)
        torch.cuda.synchronize()
        for k in range(1, nwin):
            assert torch.equal(flows[k], ref[k][3]), k
        _say(f"pipelined driver: {nwin} windows, ring {NB}, 4 streams")
    finally:
        c.close()


def test_native_sequence_equals_sequential():
    """ebof_run_sequence (the pipelined plain driver issued natively: window k
    on stream k mod 4, a ring of 5 buffer slots) gives every window the flow
    of the sequential stage calls, also when a second call continues the
    sequence; and it rejects a ring no longer than the stream count and a
    reversed window range."""
    import ctypes
    c = L.ebof_create(arena_bytes=1 << 30)
    try:
        s = synth.c1_stream(0)
        nwin, NB = 20, 5
        wins = [s.window(k) for k in range(nwin)]
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        N, P = s.W * s.H, L.ebof_pyramid_floats(p)
        evs = [dict(x=dev(w["x"]), y=dev(w["y"]), t=dev(w["t"]), t0=w["t0"]) for w in wins]
        ref = alone(c, p, evs)
        streams = [L.ebof_stream_create(c) for _ in range(4)]
        ring = [dict(edge=torch.empty(N, dtype=torch.uint8, device="cuda"),
                     pyr=torch.empty(P, dtype=torch.float32, device="cuda"),
                     flow=torch.full((2 * N,), float("nan"), dtype=torch.float32, device="cuda")) for _ in range(NB)]
        torch.cuda.synchronize()
        for lo, hi in ((0, 12), (12, nwin)):
            L.Sequence(c, p, evs[lo:hi], ring, streams, slot0=8).run(lo, hi)
            torch.cuda.synchronize()
            for k in range(max(1, hi - NB), hi):
                assert torch.equal(ring[k % NB]["flow"], ref[k][3]), (lo, hi, k)
                assert torch.equal(ring[k % NB]["pyr"], ref[k][1]) and torch.equal(ring[k % NB]["edge"], ref[k][0])
        # an empty range issues nothing; a run of window 0 alone writes no flow
        L.Sequence(c, p, evs[:1], ring, streams, slot0=20).run(0, 0)
        ring[0]["flow"].fill_(float("nan"))
        L.Sequence(c, p, evs[:1], ring, streams, slot0=20).run(0, 1)
        torch.cuda.synchronize()
        assert torch.isnan(ring[0]["flow"]).all()
        assert torch.equal(ring[0]["pyr"], ref[0][1]) and torch.equal(ring[0]["edge"], ref[0][0])
        seq = L.Sequence(c, p, evs[:4], ring[:4], streams, slot0=8)
        assert c.lib.ebof_run_sequence(c.handle, ctypes.byref(p), seq.win, 20, 24, seq.ring, 4, seq.streams, 4,
                                       8) == L.EBOF_E_INVAL
        assert c.lib.ebof_run_sequence(c.handle, ctypes.byref(p), seq.win, 24, 20, seq.ring, 4, seq.streams, 3,
                                       8) == L.EBOF_E_INVAL
        assert c.lib.ebof_run_sequence(c.handle, ctypes.byref(p), seq.win, 20, 24, seq.ring, 4, seq.streams, 3,
                                       L.EBOF_SIGNAL_SLOTS - 2) == L.EBOF_E_INVAL
        _say(f"native sequence: {nwin} windows in two calls, ring {NB}, 4 streams")
    finally:
        torch.cuda.synchronize()
        c.close()


def test_stage_calls_across_stamp_wrap():
    """A stage scratch marks a window's pixels with a stamp 1..255 and clears
    its staging image when the stamp wraps: 262 windows on one stream
    (three windows in turn) give every window the edge image (and, through
    ebof_window_surface, the pyramid) of its first occurrence, also past the
    wrap, where stale marks of window 0 would land in window 256 (a
    different window)."""
    c = L.ebof_create(arena_bytes=1 << 30)
    try:
        s = synth.c1_stream(0)
        wins = [s.window(k) for k in range(3)]
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        N, P = s.W * s.H, L.ebof_pyramid_floats(p)
        evs = [dict(x=dev(w["x"]), y=dev(w["y"]), t=dev(w["t"]), t0=w["t0"]) for w in wins]
        st = [torch.cuda.Stream() for _ in range(2)]
        first = {}
        for k in range(262):
            ev = evs[k % 3]
            e1 = torch.empty(N, dtype=torch.uint8, device="cuda")
            e2 = torch.empty(N, dtype=torch.uint8, device="cuda")
            pr = torch.empty(P, dtype=torch.float32, device="cuda")
            L.ebof_bin_events(c, p, ev["x"], ev["y"], ev["t"], ev["t0"], e1, stream=st[0])
            L.ebof_window_surface(c, p, ev["x"], ev["y"], ev["t"], ev["t0"], e2, pr, stream=st[1])
            torch.cuda.synchronize()
            if k < 3:
                assert torch.equal(e1, e2)
                first[k] = (e1, pr)
            else:
                r = first[k % 3]
                assert torch.equal(e1, r[0]) and torch.equal(e2, r[0]) and torch.equal(pr, r[1]), k
        _say("stamp wrap: 262 windows, bin_events and window_surface")
    finally:
        c.close()


def test_batch_equals_alone_and_graph_replays(ctx):
    streams = mixed_streams()
    ref = [alone(ctx, p, evs) for p, evs in streams]
    outs = []
    for p, evs in streams:
        W, H = p.width, p.height
        P = L.ebof_pyramid_floats(p)
        outs.append([dict(edge=torch.empty(W * H, dtype=torch.uint8, device="cuda"),
                          d2=torch.empty(W * H, dtype=torch.int32, device="cuda"),
                          pyr=torch.empty(P, dtype=torch.float32, device="cuda"),
                          flow=torch.empty(2 * W * H, dtype=torch.float32, device="cuda"))
                     for _ in evs])
    stream = torch.cuda.Stream()
    nwin = len(streams[0][1])
    for rep in range(3):  # first pass captures the graphs, later ones replay them
        for k in range(nwin):
            batch = []
            for s, (p, evs) in enumerate(streams):
                o = outs[s][k]
                w = dict(params=p, x=evs[k]["x"], y=evs[k]["y"], t=evs[k]["t"], t0_us=evs[k]["t0"],
                         edge_out=o["edge"], d2_out=o["d2"], pyr_out=o["pyr"])
                if k > 0:
                    w.update(pyr_prev=outs[s][k - 1]["pyr"], mask=outs[s][k - 1]["edge"], flow_out=o["flow"])
                batch.append(w)
            _say(f"batch rep {rep} window {k}: {len(batch)} windows")
            L.ebof_run_batch(ctx, batch, stream=stream)
            # the program's own eager work between replays
            torch.cuda.synchronize()
        for s in range(len(streams)):
            for k in range(nwin):
                r, o = ref[s][k], outs[s][k]
                assert torch.equal(o["edge"], r[0]), (rep, s, k, "edge")
                assert torch.equal(o["pyr"], r[1]), (rep, s, k, "pyramid")
                assert torch.equal(o["d2"], r[2]), (rep, s, k, "d2")
                if k > 0:
                    assert torch.equal(o["flow"], r[3]), (rep, s, k, "flow")
        for s in range(len(streams)):  # scribble so a stale replay cannot pass
            for k in range(nwin):
                for v in outs[s][k].values():
                    v.zero_()


def _batch_of(streams, outs, k):
    batch = []
    for s, (p, evs) in enumerate(streams):
        o = outs[s]
        w = dict(params=p, x=evs[k]["x"], y=evs[k]["y"], t=evs[k]["t"], t0_us=evs[k]["t0"],
                 edge_out=o["edge"], d2_out=o["d2"], pyr_out=o["pyr"])
        if k > 0:
            w.update(pyr_prev=o["pyr_prev"], mask=o["mask"], flow_out=o["flow"])
        batch.append(w)
    return batch


def _outs_for(streams, ref, k):
    outs = []
    for s, (p, _) in enumerate(streams):
        W, H = p.width, p.height
        P = L.ebof_pyramid_floats(p)
        outs.append(dict(edge=torch.empty(W * H, dtype=torch.uint8, device="cuda"),
                         d2=torch.empty(W * H, dtype=torch.int32, device="cuda"),
                         pyr=torch.empty(P, dtype=torch.float32, device="cuda"),
                         flow=torch.empty(2 * W * H, dtype=torch.float32, device="cuda"),
                         pyr_prev=ref[s][k - 1][1], mask=ref[s][k - 1][0]))
    return outs


def _check_outs(streams, ref, outs, k, tag):
    for s in range(len(streams)):
        r, o = ref[s][k], outs[s]
        assert torch.equal(o["edge"], r[0]), (tag, s, "edge")
        assert torch.equal(o["d2"], r[2]), (tag, s, "d2")
        assert torch.equal(o["pyr"], r[1]), (tag, s, "pyramid")
        assert torch.equal(o["flow"], r[3]), (tag, s, "flow")


@pytest.mark.parametrize("rows, tile_w, lanes, grid", [(1, 256, 8, 256), (8, 128, 4, 0), (2, 64, 4, 4096),
                                                        (4, 16, 8, 0)])
def test_batch_forced_launch_shapes_equal_alone(ctx, tmp_path, rows, tile_w, lanes, grid):
    """Every tile shape and block count the tuner can pick gives the stage
    calls' results: shapes forced through the tuning cache file."""
    streams = mixed_streams(n_low=2, n_hd=1, windows=2)
    ref = [alone(ctx, p, evs) for p, evs in streams]
    outs = _outs_for(streams, ref, 1)
    batch = _batch_of(streams, outs, 1)
    path = tmp_path / "tune.txt"
    vals = [rows, tile_w] + [lanes] * L.EBOF_TUNE_LEVELS + [grid] * L.EBOF_TUNE_STAGES
    path.write_text(L.batch_layout_key(batch) + "\t" + " ".join(map(str, vals)) + "\n")
    L.ebof_set_tuning(ctx, L.EBOF_TUNE_AUTO, str(path))
    try:
        stream = torch.cuda.Stream()
        _say(f"forced shapes rows={rows} tile_w={tile_w} lanes={lanes} grid={grid}")
        L.ebof_run_batch(ctx, batch, stream=stream)
        torch.cuda.synchronize()
        _check_outs(streams, ref, outs, 1, (rows, tile_w, lanes, grid))
        # the file is unchanged: the layout was tuned already (read from it)
        assert path.read_text().count("\n") == 1
    finally:
        L.ebof_set_tuning(ctx, L.EBOF_TUNE_AUTO, None)


def test_autotune_cache_roundtrip(tmp_path):
    """A new layout is tuned once and appended to the cache; a context that
    reads the cache uses the entry (appends nothing) and gives the same
    results as the stage calls."""
    path = tmp_path / "cache.txt"
    streams = mixed_streams(n_low=1, n_hd=1, windows=2)
    for round_ in range(2):
        c = L.ebof_create(arena_bytes=1 << 30)
        try:
            L.ebof_set_tuning(c, L.EBOF_TUNE_AUTO, str(path))
            ref = [alone(c, p, evs) for p, evs in streams]
            outs = _outs_for(streams, ref, 1)
            batch = _batch_of(streams, outs, 1)
            _say(f"autotune round {round_}")
            L.ebof_run_batch(c, batch, stream=torch.cuda.Stream())
            torch.cuda.synchronize()
            _check_outs(streams, ref, outs, 1, ("autotune", round_))
            lines = path.read_text().splitlines()
            assert len(lines) == 1, lines
            key, vals = lines[0].split("\t")
            assert key == L.batch_layout_key(batch)
            v = [int(x) for x in vals.split()]
            assert len(v) == 2 + L.EBOF_TUNE_LEVELS + L.EBOF_TUNE_STAGES
            assert v[0] in (1, 2, 4, 8) and v[1] in (16, 64, 128, 256)
            assert all(x in (4, 8) for x in v[2:2 + L.EBOF_TUNE_LEVELS])
        finally:
            torch.cuda.synchronize()
            c.close()


def test_tuning_rejects_bad_cache(ctx, tmp_path):
    path = tmp_path / "bad.txt"
    path.write_text("346,260,3,4,1,0;\t4 64 1 2\n")  # too few values
    with pytest.raises(L.EbofError) as ei:
        L.ebof_set_tuning(ctx, L.EBOF_TUNE_AUTO, str(path))
    assert ei.value.code == L.EBOF_E_INVAL
    with pytest.raises(L.EbofError):
        L.ebof_set_tuning(ctx, 7, None)


def test_stage_calls_pipelined_over_streams(ctx):
    """Window k's binning and EDT on HIP stream k mod 3, the flow k-1 -> k on
    the same stream after an event on window k-1's pyramid: consecutive
    windows overlap on the device and every output equals the sequential
    stage calls'."""
    for p, evs in mixed_streams(n_low=1, n_hd=1, windows=4):
        ref = alone(ctx, p, evs)
        W, H = p.width, p.height
        P = L.ebof_pyramid_floats(p)
        sts = [torch.cuda.Stream() for _ in range(3)]
        out, ev_pre = [], []
        for k, ev in enumerate(evs):
            st = sts[k % 3]
            e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
            d2 = torch.empty(W * H, dtype=torch.int32, device="cuda")
            pr = torch.empty(P, dtype=torch.float32, device="cuda")
            L.ebof_bin_events(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], e, stream=st)
            L.ebof_edt_surface(ctx, p, e, pr, d2, stream=st)
            done = torch.cuda.Event()
            done.record(st)
            ev_pre.append(done)
            f = None
            if k > 0:
                st.wait_event(ev_pre[k - 1])
                f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
                L.ebof_flow(ctx, p, out[k - 1][1], pr, f, mask=out[k - 1][0], stream=st)
            out.append((e, pr, d2, f))
        torch.cuda.synchronize()
        _say(f"pipelined {W}x{H}: {len(evs)} windows")
        for k in range(len(evs)):
            for i, name in enumerate(("edge", "pyramid", "d2", "flow")):
                if out[k][i] is not None:
                    assert torch.equal(out[k][i], ref[k][i]), (W, k, name)


def test_stage_calls_ordered_by_stream_signals():
    """The pipelined plain form ordered by context counters instead of
    events, on context-owned streams: window k preprocessed on stream k mod 2, which then stores k+1
    into counter k mod 2; the flow k-1 -> k on flow stream k mod 2 waits for
    counter (k-1) mod 2 >= k and counter k mod 2 >= k+1.  Every output equals
    the sequential stage calls' and the counters end at the last values
    stored."""
    c = L.ebof_create(arena_bytes=1 << 30)
    try:
        with pytest.raises(L.EbofError):
            L.ebof_stream_signal(c, L.EBOF_SIGNAL_SLOTS, 1)
        with pytest.raises(L.EbofError):
            L.ebof_stream_wait(c, -1, 1)
        assert L.ebof_signal_read(c, 5) == 0
        owned = [L.ebof_stream_create(c) for _ in range(4)]  # a hardware queue each
        for p, evs in mixed_streams(n_low=1, n_hd=1, windows=5):
            ref = alone(c, p, evs)
            W, H = p.width, p.height
            P = L.ebof_pyramid_floats(p)
            pre = owned[:2]
            fl = owned[2:]
            base = max(L.ebof_signal_read(c, i) for i in range(4))
            out = []
            for k, ev in enumerate(evs):
                st = pre[k % 2]
                e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
                d2 = torch.empty(W * H, dtype=torch.int32, device="cuda")
                pr = torch.empty(P, dtype=torch.float32, device="cuda")
                L.ebof_bin_events(c, p, ev["x"], ev["y"], ev["t"], ev["t0"], e, stream=st)
                L.ebof_edt_surface(c, p, e, pr, d2, stream=st)
                L.ebof_stream_signal(c, k % 2, base + k + 1, stream=st)
                f = None
                if k > 0:
                    sf = fl[k % 2]
                    L.ebof_stream_wait(c, (k - 1) % 2, base + k, stream=sf)
                    L.ebof_stream_wait(c, k % 2, base + k + 1, stream=sf)
                    f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
                    L.ebof_flow(c, p, out[k - 1][1], pr, f, mask=out[k - 1][0], stream=sf)
                    L.ebof_stream_signal(c, 2 + k % 2, base + k + 1, stream=sf)
                out.append((e, pr, d2, f))
            torch.cuda.synchronize()
            n = len(evs)
            _say(f"signal-ordered {W}x{H}: {n} windows")
            assert L.ebof_signal_read(c, (n - 1) % 2) == base + n
            assert L.ebof_signal_read(c, 2 + (n - 1) % 2) == base + n
            for k in range(n):
                for i, name in enumerate(("edge", "pyramid", "d2", "flow")):
                    if out[k][i] is not None:
                        assert torch.equal(out[k][i], ref[k][i]), (W, k, name)
    finally:
        c.close()


def test_serving_alone_vs_mix(ctx):
    streams = mixed_streams(n_low=4, n_hd=2, windows=4)
    ref = [alone(ctx, p, evs) for p, evs in streams]
    sids = [L.ebof_stream_open(ctx, p) for p, _ in streams]
    outs = {}
    tickets = {}
    nwin = len(streams[0][1])
    # interleave the streams' windows, host events for half the streams
    for k in range(nwin):
        for s, (p, evs) in enumerate(streams):
            W, H = p.width, p.height
            f = torch.full((2 * W * H,), 7.0, dtype=torch.float32, device="cuda")
            m = torch.full((W * H,), 9, dtype=torch.uint8, device="cuda")
            ev = evs[k]
            if s % 2:
                x, y, t = ev["x"].cpu().numpy(), ev["y"].cpu().numpy(), ev["t"].cpu().numpy()
            else:
                x, y, t = ev["x"], ev["y"], ev["t"]
            tk = None
            while tk is None:
                tk = L.ebof_submit(ctx, sids[s], p, x, y, t, ev["t0"], f, m)
            tickets[(s, k)] = tk
            outs[(s, k)] = (f, m)
    _say(f"served {len(tickets)} windows")
    L.ebof_drain(ctx)
    for (s, k), tk in tickets.items():
        st, lat = L.ebof_poll(ctx, tk, with_latency=True)
        f, m = outs[(s, k)]
        assert lat > 0
        if k == 0:
            assert st == L.EBOF_NO_FLOW
            assert torch.count_nonzero(f) == 0 and torch.count_nonzero(m) == 0
        else:
            assert st == L.EBOF_OK
            assert torch.equal(f, ref[s][k][3]), (s, k, "flow")
            assert torch.equal(m, ref[s][k - 1][0]), (s, k, "mask")
    with pytest.raises(L.EbofError):
        L.ebof_poll(ctx, tickets[(0, 1)])  # already reported
    for sid in sids:
        L.ebof_stream_close(ctx, sid)


def test_serving_gap_resets_stream(ctx):
    s = synth.c1_stream(0)
    p = L.ebof_params_default(s.W, s.H)
    sid = L.ebof_stream_open(ctx, p)
    W, H = s.W, s.H
    sts = []
    for k, shift in [(0, 0), (1, 0), (2, 5 * synth.DT_US)]:  # the third window skips ahead
        w = s.window(k)
        f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
        m = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        tk = L.ebof_submit(ctx, sid, p, w["x"], w["y"], w["t"] + shift, w["t0"] + shift, f, m)
        L.ebof_drain(ctx)
        sts.append(L.ebof_poll(ctx, tk))
    assert sts == [L.EBOF_NO_FLOW, L.EBOF_OK, L.EBOF_NO_FLOW]
    L.ebof_stream_close(ctx, sid)
    with pytest.raises(L.EbofError):
        L.ebof_stream_close(ctx, sid)


def test_serving_admission_by_arena():
    """A context whose arena cannot hold a 1280x720 stream's resident state
    refuses the stream (EBOF_E_NOMEM); a window larger than the whole event
    ring can never be admitted and is refused with EBOF_E_NOMEM too (not
    EBOF_E_AGAIN, which a caller would retry for ever)."""
    c = L.ebof_create(arena_bytes=16 << 20)
    try:
        p_hd = L.ebof_params_default(1280, 720)
        with pytest.raises(L.EbofError) as ei:
            L.ebof_stream_open(c, p_hd)
        assert ei.value.code == L.EBOF_E_NOMEM
        p = L.ebof_params_default(346, 260)
        sid = L.ebof_stream_open(c, p)
        n = 1_000_000  # 12 MB of events, more than the ring of this small arena
        x = np.zeros(n, np.uint16)
        t = np.zeros(n, np.int64)
        f = torch.empty(2 * 346 * 260, dtype=torch.float32, device="cuda")
        m = torch.empty(346 * 260, dtype=torch.uint8, device="cuda")
        with pytest.raises(L.EbofError) as ei:
            L.ebof_submit(c, sid, p, x, x, t, 0, f, m)
        assert ei.value.code == L.EBOF_E_NOMEM
        L.ebof_stream_close(c, sid)
    finally:
        torch.cuda.synchronize()
        c.close()


# --------------------------------------------------------------------------
# the batched and served forms against the CPU oracle
# --------------------------------------------------------------------------
def _oracle_check(p, ev0, ev1, out0, out1, tag):
    """Window k-1 and k of one stream against the oracle: edge image,
    squared distances (when exported) and pyramid bit for bit, and the
    masked flow k-1 -> k to the flow bars."""
    W, H = p.width, p.height
    r0, r1 = ref_window(p, ev0), ref_window(p, ev1)
    for r, o, k in ((r0, out0, 0), (r1, out1, 1)):
        assert np.array_equal(o["edge"].cpu().numpy().reshape(H, W), r["Edf"]), (tag, k, "edge")
        if o.get("d2") is not None:
            assert np.array_equal(o["d2"].cpu().numpy().reshape(H, W), r["D2"]), (tag, k, "d2")
        assert np.array_equal(o["pyr"].cpu().numpy(), r["pyr"]), (tag, k, "pyramid")
    f = out1["flow"].cpu().numpy().reshape(2, H, W).astype(np.float64)
    ref = OracleFlow(p, r0, r1, mask=True)
    assert np.all(f[:, ~r0["Edf"].astype(bool)] == 0.0), tag
    assert_flow_matches(f, ref, tag)


def test_batch_c3_vs_oracle(ctx):
    """The 16-stream batch (10 x 346x260, 6 x 1280x720, lognormal event
    counts, own affine motions): two consecutive windows of every stream, one
    ebof_run_batch per window index, each window against the oracle."""
    streams = synth.c3_streams()
    ps, evs, outs = [], [], []
    for s in streams:
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        W, H, P = s.W, s.H, L.ebof_pyramid_floats(p)
        ps.append(p)
        evs.append([s.window(k) for k in (0, 1)])
        outs.append([dict(edge=torch.empty(W * H, dtype=torch.uint8, device="cuda"),
                          d2=torch.empty(W * H, dtype=torch.int32, device="cuda"),
                          pyr=torch.empty(P, dtype=torch.float32, device="cuda"),
                          flow=torch.empty(2 * W * H, dtype=torch.float32, device="cuda")) for _ in (0, 1)])
    dev_ev = [[dict(x=dev(e["x"]), y=dev(e["y"]), t=dev(e["t"]), t0=e["t0"]) for e in ev] for ev in evs]
    stream = torch.cuda.Stream()
    for k in (0, 1):
        batch = []
        for i, p in enumerate(ps):
            e, o = dev_ev[i][k], outs[i][k]
            w = dict(params=p, x=e["x"], y=e["y"], t=e["t"], t0_us=e["t0"], edge_out=o["edge"], d2_out=o["d2"],
                     pyr_out=o["pyr"])
            if k:
                w.update(pyr_prev=outs[i][0]["pyr"], mask=outs[i][0]["edge"], flow_out=o["flow"])
            batch.append(w)
        _say(f"C3 batch, window {k}: {len(batch)} windows")
        L.ebof_run_batch(ctx, batch, stream=stream)
    torch.cuda.synchronize()
    for i, p in enumerate(ps):
        _oracle_check(p, evs[i][0], evs[i][1], outs[i][0], outs[i][1], f"C3 stream {i} ({p.width}x{p.height})")


def test_serving_c4_mix_vs_oracle(ctx):
    """Six cameras of the serving workload, two per resolution class
    (346x260, 640x480, 1280x720), three windows each, submitted interleaved
    (host events for half of them) and batched as they arrive: every flow
    and mask against the oracle."""
    cams = [synth.c4_camera(c) for c in range(6)]
    nwin = 3
    ps = [L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW) for s in cams]
    evs = [[s.window(k) for k in range(nwin)] for s in cams]
    sids = [L.ebof_stream_open(ctx, p) for p in ps]
    res = {}
    for k in range(nwin):
        for c, (s, p) in enumerate(zip(cams, ps)):
            W, H = s.W, s.H
            f = torch.full((2 * W * H,), 7.0, dtype=torch.float32, device="cuda")
            m = torch.full((W * H,), 9, dtype=torch.uint8, device="cuda")
            ev = evs[c][k]
            if c % 2:
                x, y, t = ev["x"], ev["y"], ev["t"]
            else:
                x, y, t = dev(ev["x"]), dev(ev["y"]), dev(ev["t"])
            tk = None
            while tk is None:
                tk = L.ebof_submit(ctx, sids[c], p, x, y, t, ev["t0"], f, m)
            res[(c, k)] = (tk, f, m, (x, y, t))
    _say(f"C4 mix: served {len(res)} windows")
    L.ebof_drain(ctx)
    for c, (s, p) in enumerate(zip(cams, ps)):
        W, H = s.W, s.H
        refs = [ref_window(p, evs[c][k]) for k in range(nwin)]
        for k in range(nwin):
            tk, f, m, _ = res[(c, k)]
            st = L.ebof_poll(ctx, tk)
            if k == 0:
                assert st == L.EBOF_NO_FLOW
                continue
            assert st == L.EBOF_OK
            r0, r1 = refs[k - 1], refs[k]
            assert np.array_equal(m.cpu().numpy().reshape(H, W), r0["Edf"]), (c, k, "mask")
            fl = f.cpu().numpy().reshape(2, H, W).astype(np.float64)
            assert_flow_matches(fl, OracleFlow(p, r0, r1, mask=True), f"C4 camera {c} ({W}x{H}) window {k}")
    for sid in sids:
        L.ebof_stream_close(ctx, sid)


def test_serving_warm_start_vs_oracle(ctx):
    """EBOF_WARM_START through ebof_submit: three cameras (one per resolution
    class), four windows each.  The second window's flow starts cold, every
    later one from the stream's resident previous flow (kept before masking);
    each is checked against the oracle's chain fed with its own previous
    flow.  A gap in time starts the stream over (cold again)."""
    cams = [synth.c4_camera(c) for c in range(3)]
    nwin = 4
    ps = [L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW | L.EBOF_WARM_START) for s in cams]
    evs = [[s.window(k) for k in range(nwin)] for s in cams]
    sids = [L.ebof_stream_open(ctx, p) for p in ps]
    res = {}
    for k in range(nwin):
        for c, (s, p) in enumerate(zip(cams, ps)):
            W, H = s.W, s.H
            f = torch.full((2 * W * H,), 7.0, dtype=torch.float32, device="cuda")
            m = torch.full((W * H,), 9, dtype=torch.uint8, device="cuda")
            ev = evs[c][k]
            x, y, t = dev(ev["x"]), dev(ev["y"]), dev(ev["t"])
            tk = None
            while tk is None:
                tk = L.ebof_submit(ctx, sids[c], p, x, y, t, ev["t0"], f, m)
            res[(c, k)] = (tk, f, m, (x, y, t))
    _say(f"warm-started serving: {len(res)} windows")
    L.ebof_drain(ctx)
    for c, (s, p) in enumerate(zip(cams, ps)):
        W, H = s.W, s.H
        refs = [ref_window(p, evs[c][k]) for k in range(nwin)]
        prev = None
        for k in range(nwin):
            tk, f, m, _ = res[(c, k)]
            st = L.ebof_poll(ctx, tk)
            if k == 0:
                assert st == L.EBOF_NO_FLOW
                continue
            assert st == L.EBOF_OK
            r0, r1 = refs[k - 1], refs[k]
            o = OracleFlow(p, r0, r1, prev_flow=prev, mask=True)
            fl = f.cpu().numpy().reshape(2, H, W).astype(np.float64)
            assert_flow_matches(fl, o, f"warm camera {c} ({W}x{H}) window {k}")
            prev = o.raw
    # a gap in time: the stream starts over, and its next flow is cold again
    c, s, p = 0, cams[0], ps[0]
    W, H = s.W, s.H
    outs = []
    for j, k in enumerate((nwin + 3, nwin + 4)):
        ev = s.window(k)
        f = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
        m = torch.empty(W * H, dtype=torch.uint8, device="cuda")
        tk = None
        while tk is None:
            tk = L.ebof_submit(ctx, sids[c], p, dev(ev["x"]), dev(ev["y"]), dev(ev["t"]), ev["t0"], f, m)
        outs.append((tk, f, ev))
    L.ebof_drain(ctx)
    assert L.ebof_poll(ctx, outs[0][0]) == L.EBOF_NO_FLOW
    assert L.ebof_poll(ctx, outs[1][0]) == L.EBOF_OK
    r0, r1 = ref_window(p, outs[0][2]), ref_window(p, outs[1][2])
    fl = outs[1][1].cpu().numpy().reshape(2, H, W).astype(np.float64)
    assert_flow_matches(fl, OracleFlow(p, r0, r1, mask=True), "after a gap: cold")
    for sid in sids:
        L.ebof_stream_close(ctx, sid)
