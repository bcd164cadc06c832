"""The allocation-free flow call (ebof_flow_noalloc, patch displacements in a
fixed device array) against ebof_flow on the same pyramids: two calls in a
row, the second on a smaller sensor, each bit-identical to ebof_flow (same
kernels, same arithmetic)."""
import numpy as np
import pytest
import torch

from paper_2112_10591_amd import _lib as L
from paper_2112_10591_amd import synth

pytestmark = pytest.mark.gpu


def _pyramids(ctx, s, p, ks):
    out = []
    for k in ks:
        ev = s.window(k)
        e = torch.empty(p.width * p.height, dtype=torch.uint8, device="cuda")
        pr = torch.empty(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
        L.ebof_window_surface(ctx, p, torch.from_numpy(ev["x"]).cuda(), torch.from_numpy(ev["y"]).cuda(),
                              torch.from_numpy(ev["t"]).cuda(), ev["t0"], e, pr)
        out.append((pr, e))
    torch.cuda.synchronize()
    return out


def test_noalloc_flow_matches_stage_call_twice_shrinking():
    print("wip_no_alloc: C2 1280x720 then C1 346x260, masked", flush=True)
    ctx = L.ebof_create(arena_bytes=512 << 20)
    cases = [(synth.c2_stream(0), (3, 4)), (synth.c1_stream(0), (0, 1))]
    for s, ks in cases:
        p = L.ebof_params_default(s.W, s.H, flags=L.EBOF_MASK_FLOW)
        (a, ea), (b, _) = _pyramids(ctx, s, p, ks)
        N = s.W * s.H
        ref = torch.empty(2 * N, dtype=torch.float32, device="cuda")
        got = torch.full((2 * N,), float("nan"), dtype=torch.float32, device="cuda")
        L.ebof_flow(ctx, p, a, b, ref, mask=ea)
        L.ebof_flow_noalloc(p, a, b, got, mask=ea)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert np.isfinite(g).all()
        assert np.array_equal(r, g), f"{s.W}x{s.H}: {np.abs(r - g).max()} max difference"
        assert np.abs(r).max() > 0.1  # the windows move: the comparison is not of zeros
    ctx.close()
