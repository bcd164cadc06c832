"""Shared bars of the GPU parity tests (imported by the test modules).

Flow against the oracle: mean endpoint error <= 0.01 px over the field, and
per pixel: 99.9 % of pixels within FLOW_P999 px, every pixel within
FLOW_MAX px.  Both sides run the same damped solver (lambda = 0.3, 16
steps), so the oracle's own bias against the true motion (the contraction
lambda (H + lambda I)^-1 per step, pinned on the CPU) is not an error here:
the GPU must reproduce it.  The GPU iterates in single precision (sums of
order one, relative rounding 2^-24 per step, each step bounded by
|b| / lambda), so its displacements stay within ~1e-5 px of the oracle's.
"""
import numpy as np

import oracle

FLOW_MEAN = 0.01
FLOW_P999 = 1e-3
FLOW_MAX = 0.05


def say(msg):
    print(msg, flush=True)


def epe(a, b):
    return np.hypot(a[0] - b[0], a[1] - b[1])


def assert_flow_matches(f, r, tag, where=None):
    """GPU flow f against oracle flow r ([2, H, W]): mean and per-pixel bars
    over the pixels `where` selects (default all)."""
    e = epe(f, r)
    if where is not None:
        e = e[where]
    p999 = float(np.percentile(e, 99.9))
    say(f"  {tag}: EPE vs oracle mean {e.mean():.2e} p99.9 {p999:.2e} max {e.max():.2e} over {e.size} px")
    assert e.mean() <= FLOW_MEAN, tag
    assert p999 <= FLOW_P999, tag
    assert e.max() <= FLOW_MAX, tag


def ref_window(p, ev):
    """The oracle's window (edge image, squared distances, surface, pyramid)
    for parameters p and events ev (dict x, y, t, t0; NumPy arrays)."""
    return oracle.window(p.width, p.height, ev["x"], ev["y"], ev["t"], ev["t0"], p.dt_us, p.n_d, p.n_f,
                         float(np.float32(p.alpha)), p.levels)


def oracle_flow(p, r0, r1, prev_flow=None):
    return oracle.dis_flow(r0["pyr"], r1["pyr"], p.width, p.height, p.levels, stride=p.stride, iters=p.iters,
                           lam=float(np.float32(p.lambda_reg)), prev_flow=prev_flow)


def masked(r0, flow):
    """where(E_df of the reference window, flow, 0)."""
    return np.where(r0["Edf"].astype(bool)[None], flow, 0.0)
