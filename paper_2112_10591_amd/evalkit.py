"""Evaluation kit (Sec. IV) on synthetic streams with known motion: the
ablations of Sec. IV-B (no denoising/filling, and the distance surfaces
DS_L, DS_LB, DS_Log beside eq. 1) and a sensitivity sweep over N_d, N_f and
d_sat (Sec. IV, sensitivity analysis), scored by the average endpoint error
and outlier rate against the generator's motion field and by the flow warp
loss.  The paper's datasets are not available: the generator's streams stand
in for them (346x260 translating segments, 1280x720 affine scenes).

Every computation runs in the library (stage calls, ebof_flow_filter,
ebof_flow_errors, ebof_fwl); this module only chooses parameters and
averages the results.

    python -m paper_2112_10591_amd.evalkit [--pairs N] [--hd] [--sweep]
"""
from __future__ import annotations

import argparse
import math
import sys

import numpy as np
import torch

from . import _lib as L
from . import synth

BORDER = 16  # pixels from the border left out of the endpoint errors


def _window(ctx, p, ev):
    W, H = p.width, p.height
    e = torch.empty(W * H, dtype=torch.uint8, device="cuda")
    pr = torch.empty(L.ebof_pyramid_floats(p), dtype=torch.float32, device="cuda")
    dv = dict(x=torch.from_numpy(ev["x"]).cuda(), y=torch.from_numpy(ev["y"]).cuda(),
              t=torch.from_numpy(ev["t"]).cuda(), p=torch.from_numpy(ev["p"]).cuda(), t0=ev["t0"])
    L.ebof_window_surface(ctx, p, dv["x"], dv["y"], dv["t"], ev["t0"], e, pr)
    return e, pr, dv


def score(ctx, stream, p, pairs, warm=False, filt=None):
    """Mean AEE, outlier fraction (reference edge pixels away from the
    border) and FWL (the reference window's events, each voting 1: the
    generator draws polarities at random, so signed votes would cancel
    rather than sharpen) over `pairs` consecutive window pairs; warm: each
    flow starts from the previous pair's; filt: an ebof_filter_params, the
    flow then comes from the update-prediction filter (its state carried
    from pair to pair, from zero)."""
    W, H = p.width, p.height
    inner = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    inner[BORDER:H - BORDER, BORDER:W - BORDER] = 1
    flow = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    dense = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    before = torch.empty(2 * W * H, dtype=torch.float32, device="cuda")
    aee, out, fwl = [], [], []
    state = None
    if filt is not None:
        state = torch.zeros(L.ebof_filter_state_floats(p, filt), dtype=torch.float32, device="cuda")
    prev = _window(ctx, p, stream.window(0))
    for k in range(1, pairs + 1):
        cur = _window(ctx, p, stream.window(k))
        if filt is not None:
            L.ebof_flow_filter(ctx, p, filt, prev[1], cur[1], state, dense)
        else:
            init = before if (warm and k > 1) else None
            L.ebof_flow_warm(ctx, p, prev[1], cur[1], flow, flow_init=init, flow_dense_out=dense, mask=prev[0])
        gt = torch.from_numpy(stream.gt_flow(k).astype(np.float32).reshape(-1)).cuda()
        m = (prev[0].view(H, W) * inner).contiguous()
        a, o, n = L.ebof_flow_errors(ctx, W, H, dense, gt, m)
        if n:
            aee.append(a)
            out.append(o)
        ev = prev[2]
        f, _, _ = L.ebof_fwl(ctx, p, ev["x"], ev["y"], ev["t"], ev["t0"], dense)
        fwl.append(f)
        before.copy_(dense)
        prev = cur
    torch.cuda.synchronize()
    return dict(aee=float(np.mean(aee)) if aee else math.nan, outliers=float(np.mean(out)) if out else math.nan,
                fwl=float(np.mean(fwl)))


def ablations(ctx, stream, pairs):
    base = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW)
    rows = []
    p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW)
    rows.append(("proposed + warm start from the previous pair", score(ctx, stream, p, pairs, warm=True)))
    p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW | L.EBOF_VAR_REFINE)
    rows.append(("proposed + variational refinement", score(ctx, stream, p, pairs)))
    p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW)
    fp = L.ebof_filter_params_default(stream.W, stream.H)
    rows.append(("update-prediction filter in place of DIS (Sec. IV-A settings)",
                 score(ctx, stream, p, pairs, filt=fp)))
    for name, over in [("proposed (eq. 1)", {}), ("NDF: no denoising/filling", dict(n_d=0, n_f=5)),
                       ("DS_L: linear distance", dict(surface=L.EBOF_SURFACE_LINEAR)),
                       ("DS_LB: distance bounded at d_sat", dict(surface=L.EBOF_SURFACE_BOUNDED)),
                       ("DS_Log: log distance", dict(surface=L.EBOF_SURFACE_LOG))]:
        p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW, **over)
        p.levels = base.levels
        rows.append((name, score(ctx, stream, p, pairs)))
    return rows


def sweep(ctx, stream, pairs):
    rows = []
    base = L.ebof_params_default(stream.W, stream.H)
    for n_d in (0, 1, 2, 3):
        for n_f in (2, 3, 4, 5):
            p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW, n_d=n_d, n_f=n_f)
            rows.append((f"N_d={n_d} N_f={n_f} d_sat=6", score(ctx, stream, p, pairs)))
    for d_sat in (2, 4, 6, 8, 10, 12):
        a = d_sat / math.log(255.0)
        p = L.ebof_params_default(stream.W, stream.H, flags=L.EBOF_MASK_FLOW, alpha=a)
        rows.append((f"N_d={base.n_d} N_f={base.n_f} d_sat={d_sat}", score(ctx, stream, p, pairs)))
    return rows


def table(title, rows):
    out = [f"### {title}", "", "| setting | AEE (px) | outliers | FWL |", "|---|---:|---:|---:|"]
    for name, r in rows:
        out.append(f"| {name} | {r['aee']:.3f} | {100 * r['outliers']:.2f} % | {r['fwl']:.3f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=20)
    ap.add_argument("--hd", action="store_true", help="also the 1280x720 affine stream")
    ap.add_argument("--sweep", action="store_true", help="the N_d / N_f / d_sat sweep (346x260)")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        sys.exit("evalkit needs the GPU")
    ctx = L.ebof_create(arena_bytes=1 << 30)
    streams = [("346x260, 40 segments translating (+2.5, -1.5) px per window", synth.c1_stream(0))]
    if args.hd:
        streams.append(("1280x720, 300 segments + 50 ellipses under an affine walk", synth.c2_stream(0)))
    for title, s in streams:
        print(table(f"Ablations, {title}, {args.pairs} pairs", ablations(ctx, s, args.pairs)), flush=True)
    if args.sweep:
        print(table(f"Sensitivity, {streams[0][0]}, {args.pairs} pairs", sweep(ctx, streams[0][1], args.pairs)),
              flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
