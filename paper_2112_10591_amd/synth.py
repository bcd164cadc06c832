"""Seeded synthetic event streams shaped like the paper's workloads.

This module only draws inputs: it holds none of the flow method's arithmetic,
so both the GPU path and the CPU oracle can be fed from it.

A stream is a scene (line segments, ellipses, polygons) moving under a
per-window pose sequence.  Window k covers [k*dt, (k+1)*dt) microseconds; each
signal event picks a scene edge point (probability proportional to length),
a time tau ~ U[0,1) inside the window, and is placed where that point is at
time k + tau (linear interpolation between pose k and pose k+1), rounded to
the nearest pixel.  Noise events are uniform in pixels and time.  Polarity is
+-1 with probability 1/2 (the method ignores it, Sec. III-A).  Events are
sorted by time (stable).

Seeding: ``SeedSequence([config_id, stream_id], spawn_key=...)`` with key (0,)
for the scene, (k+1, 0) for the events of window k and (k+1, 1) for the pose
increment after window k, so any window can be drawn alone, in any order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DT_US = 10_000  # window length of every synthetic workload (10 ms)


def _rng(config_id, stream_id, *key):
    ss = np.random.SeedSequence([int(config_id), int(stream_id)], spawn_key=tuple(key))
    return np.random.Generator(np.random.PCG64(ss))


def _affine(lin, trans):
    m = np.zeros((2, 3))
    m[:, :2] = lin
    m[:, 2] = trans
    return m


def _compose(a, b):
    """a after b, both 2x3."""
    out = np.zeros((2, 3))
    out[:, :2] = a[:, :2] @ b[:, :2]
    out[:, 2] = a[:, :2] @ b[:, 2] + a[:, 2]
    return out


IDENTITY = _affine(np.eye(2), np.zeros(2))


def _polyline_ellipse(c, ax, ay, th, n=96):
    s = np.linspace(0.0, 2 * math.pi, n + 1)
    pts = np.stack([ax * np.cos(s), ay * np.sin(s)], 1)
    r = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
    pts = pts @ r.T + np.asarray(c)
    return np.stack([pts[:-1], pts[1:]], 1)  # (n, 2, 2) segments


def _polygon(c, radius, nv, rng):
    ang = np.sort(rng.uniform(0, 2 * math.pi, nv))
    rad = radius * rng.uniform(0.6, 1.0, nv)
    pts = np.stack([rad * np.cos(ang), rad * np.sin(ang)], 1) + np.asarray(c)
    return np.stack([pts, np.roll(pts, -1, 0)], 1)


@dataclass
class Group:
    """Edges that share one motion: segments (n,2,2) in scene coordinates."""
    segs: np.ndarray
    pose_fn: object  # k -> 2x3 pose (scene -> image) at window boundary k


@dataclass
class Stream:
    W: int
    H: int
    config_id: int
    stream_id: int
    groups: list
    n_events: object  # k -> event count of window k
    noise: float
    gt_kind: str = "affine"
    t_base: int = 0
    _cache: dict = field(default_factory=dict)

    # ------------------------------------------------------------------
    def t0(self, k):
        return self.t_base + k * DT_US

    def window(self, k):
        """Events of window k: dict x,y (uint16), t (int64 us), p (int8)."""
        key = ("win", k)
        if key in self._cache:
            return self._cache[key]
        rng = _rng(self.config_id, self.stream_id, k + 1, 0)
        n = int(self.n_events(k))
        n_sig = int(round((1.0 - self.noise) * n))
        # Only segments whose pose-k / pose-(k+1) bounding box meets the sensor
        # can produce an accepted event; sampling among them (by length) and
        # rejecting points off the sensor gives the same accepted distribution
        # as sampling among all of them.
        vis = []
        for g in self.groups:
            a, b = g.pose_fn(k), g.pose_fn(k + 1)
            ends = [g.segs[:, e] @ m[:, :2].T + m[:, 2] for m in (a, b) for e in (0, 1)]
            ex = np.stack([q[:, 0] for q in ends], 1)
            ey = np.stack([q[:, 1] for q in ends], 1)
            keep = ((ex.max(1) >= -1) & (ex.min(1) <= self.W) &
                    (ey.max(1) >= -1) & (ey.min(1) <= self.H))
            vis.append(np.nonzero(keep)[0])
        lens = [np.linalg.norm(g.segs[v, 1] - g.segs[v, 0], axis=1) for g, v in zip(self.groups, vis)]
        glen = np.array([l.sum() for l in lens])
        if glen.sum() <= 0:
            n_sig = 0
        xs, ys, ts = [], [], []
        need = n_sig
        while need > 0:
            m = int(need * 1.3) + 64
            gi = rng.choice(len(self.groups), size=m, p=glen / glen.sum())
            tau = rng.random(m)
            px = np.empty(m)
            py = np.empty(m)
            for g_idx, g in enumerate(self.groups):
                sel = np.nonzero(gi == g_idx)[0]
                if sel.size == 0:
                    continue
                p = lens[g_idx] / lens[g_idx].sum()
                si = vis[g_idx][rng.choice(len(vis[g_idx]), size=sel.size, p=p)]
                s = rng.random(sel.size)[:, None]
                pts = g.segs[si, 0] * (1 - s) + g.segs[si, 1] * s  # scene coords
                a = g.pose_fn(k)
                b = g.pose_fn(k + 1)
                pa = pts @ a[:, :2].T + a[:, 2]
                pb = pts @ b[:, :2].T + b[:, 2]
                tt = tau[sel][:, None]
                q = pa * (1 - tt) + pb * tt
                px[sel] = q[:, 0]
                py[sel] = q[:, 1]
            ix = np.floor(px + 0.5)
            iy = np.floor(py + 0.5)
            ok = (ix >= 0) & (ix < self.W) & (iy >= 0) & (iy < self.H)
            ix, iy, tau = ix[ok][:need], iy[ok][:need], tau[ok][:need]
            xs.append(ix.astype(np.uint16))
            ys.append(iy.astype(np.uint16))
            ts.append(np.floor(tau * DT_US).astype(np.int64))
            need -= ix.size
        n_noise = n - n_sig
        xs.append(rng.integers(0, self.W, n_noise).astype(np.uint16))
        ys.append(rng.integers(0, self.H, n_noise).astype(np.uint16))
        ts.append(rng.integers(0, DT_US, n_noise).astype(np.int64))
        x = np.concatenate(xs)
        y = np.concatenate(ys)
        rel = np.concatenate(ts)
        # window-relative times fit in 16 bits: NumPy's stable sort is a radix sort there
        order = np.argsort(rel.astype(np.uint16) if DT_US <= 65535 else rel, kind="stable")
        t = rel + self.t0(k)
        p = np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8)
        ev = dict(x=np.ascontiguousarray(x[order]), y=np.ascontiguousarray(y[order]),
                  t=np.ascontiguousarray(t[order]), p=p, t0=self.t0(k))
        if len(self._cache) < 8:
            self._cache[key] = ev
        return ev

    # ------------------------------------------------------------------
    def gt_flow(self, k):
        """Motion field at pixel centres from window k-1 to window k of the
        first group (the background): the map between the mid-window poses,
        x -> A(k+1/2) A(k-1/2)^-1 x - x, with A(k+1/2) = (pose k + pose k+1)/2.
        float64 [2,H,W]."""
        g = self.groups[0]
        a = 0.5 * (g.pose_fn(k - 1) + g.pose_fn(k))
        b = 0.5 * (g.pose_fn(k) + g.pose_fn(k + 1))
        ainv_lin = np.linalg.inv(a[:, :2])
        m_lin = b[:, :2] @ ainv_lin
        m_t = b[:, 2] - m_lin @ a[:, 2]
        yy, xx = np.mgrid[0:self.H, 0:self.W].astype(np.float64)
        u = m_lin[0, 0] * xx + m_lin[0, 1] * yy + m_t[0] - xx
        v = m_lin[1, 0] * xx + m_lin[1, 1] * yy + m_t[1] - yy
        return np.stack([u, v])


# ----------------------------------------------------------------------
# pose sequences
# ----------------------------------------------------------------------
def translation_pose(v):
    v = np.asarray(v, np.float64)

    def pose(k):
        return _affine(np.eye(2), v * k)
    return pose


class AffineWalk:
    """Global affine motion about the image centre, composed window after
    window.  The increment of window k has rotation rot*sin(.) degrees, zoom
    zoom*sin(.) and translation tr*sin(.) px per axis, each sine with its own
    stream-seeded amplitude (50-100 % of the maximum), period (40-120 windows)
    and phase: the motion stays within the per-window bounds, changes
    smoothly from one window to the next, and its cumulative drift stays
    bounded over long sequences."""

    def __init__(self, W, H, config_id, stream_id, rot=2.0, zoom=0.03, tr=12.0,
                 start=None):
        self.c = np.array([W / 2.0, H / 2.0])
        rng = _rng(config_id, stream_id, 0, 7)
        amp = rng.uniform(0.5, 1.0, 4) * np.array([rot, zoom, tr, tr])
        self.amp = amp
        self.period = rng.uniform(40.0, 120.0, 4)
        self.phase = rng.uniform(0.0, 2 * math.pi, 4)
        self.poses = [IDENTITY if start is None else start]

    def increment(self, k):
        v = self.amp * np.sin(2 * math.pi * k / self.period + self.phase)
        th = math.radians(v[0])
        z = 1.0 + v[1]
        lin = z * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]])
        trans = self.c - lin @ self.c + v[2:]
        return _affine(lin, trans)

    def __call__(self, k):
        while len(self.poses) <= k:
            j = len(self.poses) - 1
            self.poses.append(_compose(self.increment(j), self.poses[j]))
        return self.poses[k]


def expansion_pose(foe, eps):
    foe = np.asarray(foe, np.float64)

    def pose(k):
        s = (1.0 + eps) ** k
        return _affine(s * np.eye(2), foe - s * foe)
    return pose


# ----------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------
def random_segments_uniform(rng, W, H, n):
    """n segments with endpoints uniform in the sensor."""
    a = rng.uniform([0, 0], [W, H], (n, 2))
    b = rng.uniform([0, 0], [W, H], (n, 2))
    return np.stack([a, b], 1)


def random_canvas_scene(rng, W, H, n_seg, n_ell, canvas=3.0, len_rng=(20, 300),
                        axis_rng=(10, 80)):
    """Segments and ellipses with centres on a canvas `canvas` times the sensor,
    centred on it (so that motion keeps the view populated)."""
    lo = np.array([W, H]) * (1 - canvas) / 2
    hi = np.array([W, H]) * (1 + canvas) / 2
    c = rng.uniform(lo, hi, (n_seg, 2))
    ln = rng.uniform(*len_rng, n_seg)
    th = rng.uniform(0, math.pi, n_seg)
    d = np.stack([np.cos(th), np.sin(th)], 1) * (ln / 2)[:, None]
    segs = [np.stack([c - d, c + d], 1)]
    for _ in range(n_ell):
        ce = rng.uniform(lo, hi)
        ax, ay = rng.uniform(*axis_rng, 2)
        segs.append(_polyline_ellipse(ce, ax, ay, rng.uniform(0, math.pi)))
    return np.concatenate(segs, 0)


# ----------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------
RES = {"low": (346, 260), "vga": (640, 480), "hd": (1280, 720)}
LEVELS = {(346, 260): 3, (640, 480): 4, (1280, 720): 4}


def c1_stream(stream_id=0):
    """346x260, two 10 ms windows of 20k events, 40 segments translating by
    (+2.5, -1.5) px per window, 5 % noise."""
    W, H = RES["low"]
    rng = _rng(1, stream_id, 0)
    segs = random_segments_uniform(rng, W, H, 40)
    g = Group(segs, translation_pose((2.5, -1.5)))
    return Stream(W, H, 1, stream_id, [g], lambda k: 20_000, 0.05, "translation")


def c2_stream(stream_id=0):
    """1280x720, 300k events per window, 300 segments + 50 ellipses under a
    cumulative random affine walk, 10 % noise."""
    W, H = RES["hd"]
    rng = _rng(2, stream_id, 0)
    segs = random_canvas_scene(rng, W, H, 300, 50)
    g = Group(segs, AffineWalk(W, H, 2, stream_id))
    return Stream(W, H, 2, stream_id, [g], lambda k: 300_000, 0.10)


def _lognormal_count(config_id, stream_id, median, sigma, lo=5_000, hi=500_000):
    def n(k):
        r = _rng(config_id, stream_id, k + 1, 2)
        return int(np.clip(round(r.lognormal(math.log(median), sigma)), lo, hi))
    return n


def c3_streams():
    """16 streams: 10 at 346x260 and 6 at 1280x720, lognormal event counts
    (median 50k, sigma 1) clipped to [5k, 500k], own affine walks."""
    out = []
    for s in range(16):
        W, H = RES["low"] if s < 10 else RES["hd"]
        rng = _rng(3, s, 0)
        scale = W / 1280.0
        segs = random_canvas_scene(rng, W, H, 300 if s >= 10 else 80,
                                   50 if s >= 10 else 12,
                                   len_rng=(20 * max(scale, 0.3), 300 * max(scale, 0.3)),
                                   axis_rng=(10 * max(scale, 0.3), 80 * max(scale, 0.3)))
        g = Group(segs, AffineWalk(W, H, 3, s, tr=12.0 * max(scale, 0.3)))
        out.append(Stream(W, H, 3, s, [g], _lognormal_count(3, s, 50_000, 1.0), 0.10))
    return out


def c4_camera(c):
    """Camera c of the 64-camera serving workload: resolution by c mod 3,
    lognormal counts with median 0.25*W*H, sigma 0.5, clipped to [5k, 500k]."""
    W, H = [RES["low"], RES["vga"], RES["hd"]][c % 3]
    rng = _rng(4, c, 0)
    scale = W / 1280.0
    segs = random_canvas_scene(rng, W, H, max(60, int(300 * scale)), max(10, int(50 * scale)),
                               len_rng=(20 * max(scale, 0.3), 300 * max(scale, 0.3)),
                               axis_rng=(10 * max(scale, 0.3), 80 * max(scale, 0.3)))
    g = Group(segs, AffineWalk(W, H, 4, c, tr=12.0 * max(scale, 0.3)))
    return Stream(W, H, 4, c, [g], _lognormal_count(4, c, 0.25 * W * H, 0.5), 0.10)


def c5_stream(stream_id=0):
    """1280x720 stress: 2M events per window, 30 % noise, 8 random polygons each
    translating U[-20,20]^2 px per window over a 2 % expansion field."""
    W, H = RES["hd"]
    rng = _rng(5, stream_id, 0)
    bg = random_canvas_scene(rng, W, H, 300, 50, canvas=1.5)
    foe = np.array([W / 2.0, H / 2.0]) + rng.uniform(-40, 40, 2)
    groups = [Group(bg, expansion_pose(foe, 0.02))]
    for _ in range(8):
        c = rng.uniform([0, 0], [W, H])
        poly = _polygon(c, rng.uniform(40, 200), int(rng.integers(3, 9)), rng)
        groups.append(Group(poly, translation_pose(rng.uniform(-20, 20, 2))))
    return Stream(W, H, 5, stream_id, groups, lambda k: 2_000_000, 0.30)


# ----------------------------------------------------------------------
# parallel generation (call before the GPU is initialised: uses fork)
# ----------------------------------------------------------------------
_FACTORIES = {"c1": c1_stream, "c2": c2_stream, "c4": c4_camera, "c5": c5_stream,
              "c3": lambda i: c3_streams()[i]}


def _gen_one(args):
    name, sid, k = args
    ev = _FACTORIES[name](sid).window(k)
    return ev["x"], ev["y"], ev["t"], ev["t0"]


def generate(name, sid, ks, workers=8):
    """Windows ks of stream `sid` of workload `name` ("c1".."c5"), as a list
    of dicts x, y, t, t0 (polarity dropped), generated by `workers`
    processes."""
    return generate_jobs([(name, sid, k) for k in ks], workers)


def generate_jobs(jobs, workers=8):
    """Windows for a list of (workload, stream id, window index) jobs."""
    import concurrent.futures as cf
    import multiprocessing as mp
    jobs = list(jobs)
    if workers <= 1 or len(jobs) < 4:
        res = [_gen_one(j) for j in jobs]
    else:
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            res = list(ex.map(_gen_one, jobs, chunksize=max(1, len(jobs) // (4 * workers))))
    return [dict(x=x, y=y, t=t, t0=t0) for x, y, t, t0 in res]
