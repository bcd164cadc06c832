"""Pins of the oracle's update-prediction flow filter (the flow block Sec.
III-D selects, with the per-layer weights and smoothing iterations of Sec.
IV-A; the reading is spelled out in oracle/ebof_oracle.h).  Each pin is a
closed form worked out by hand: the one-pixel update on an intensity ramp,
the transport of a linear flow field over one and two windows, the smoothing
of an impulse and of a corner value, and the coarse layer's innovation handed
to the finer layer at its parent pixel."""
import numpy as np

import oracle

HUGE = 1e30  # a weight that leaves the prediction untouched


def flat_pyramid(levels):
    """Packed pyramid from a list of [H_l, W_l] float32 images."""
    return np.concatenate([np.asarray(a, np.float32).ravel() for a in levels])


def test_update_on_a_ramp_by_hand():
    """I0 = s x, I1 = I0 shifted right by t: at every interior pixel the
    gradient is (255 s, 0) and the residual at zero flow -255 s t, so one
    update gives u = (255 s)^2 t / ((255 s)^2 + gamma), v = 0.  Catches a
    dropped 255, a flipped residual and a misplaced weight."""
    W, H, s, t = 40, 12, 0.01, 1.5
    x = np.arange(W, dtype=np.float64)
    I0 = np.tile(s * x, (H, 1)).astype(np.float32)
    I1 = np.tile(s * (x - t), (H, 1)).astype(np.float32)
    for gamma in (5.0, 50.0):
        flow, _ = oracle.flow_filter(flat_pyramid([I0]), flat_pyramid([I1]), W, H, 1, [gamma], [0])
        g2 = (255.0 * s) ** 2
        want = g2 * t / (g2 + gamma)
        inner = flow[:, :, 1:W - 1]
        np.testing.assert_allclose(inner[0], want, rtol=1e-5)
        np.testing.assert_allclose(inner[1], 0.0, atol=1e-12)
        assert want > 0.1 * t  # the shift is to the right: u > 0


def test_constant_state_is_carried_unchanged():
    """A uniform previous flow is its own transport, the smoothing keeps it,
    and a huge weight keeps the update from moving it."""
    W, H = 33, 21
    rng = np.random.default_rng(0)
    sizes = oracle.level_sizes(W, H, 2)
    pyr0 = rng.random(sum(w * h for w, h in sizes)).astype(np.float32)
    pyr1 = rng.random(pyr0.size).astype(np.float32)
    state = np.concatenate([np.concatenate([np.full(w * h, c0 * 2.0 ** -l), np.full(w * h, c1 * 2.0 ** -l)])
                            for l, (w, h) in enumerate(sizes) for c0, c1 in [(1.25, -0.5)]])
    flow, st = oracle.flow_filter(pyr0, pyr1, W, H, 2, [HUGE, HUGE], [3, 7], state)
    np.testing.assert_allclose(flow[0], 1.25, atol=1e-12)
    np.testing.assert_allclose(flow[1], -0.5, atol=1e-12)
    np.testing.assert_allclose(st, state, atol=1e-12)


def test_transport_of_a_linear_field():
    """U = (a x, b y): the flow carried along itself is P(x, y) =
    (a (x - a x), b (y - b y)) wherever the sample stays inside the image
    (bilinear interpolation of a linear field is exact); a second window
    carries P along itself again.  Catches x + U in place of x - U and a
    swapped component."""
    W, H, a, b = 30, 20, 0.05, -0.03
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    U = np.stack([a * x, b * y])
    P = oracle.ff_transport(U)
    # rows whose sample y - b y stays inside (b < 0 pushes the last rows out)
    rows = slice(0, int((H - 1) / (1 - b)) + 1)
    np.testing.assert_allclose(P[0], a * (x - a * x), atol=1e-12)
    np.testing.assert_allclose(P[1][rows], (b * (y - b * y))[rows], atol=1e-12)
    assert abs(P[1][H - 1, 0] - b * (H - 1)) < 1e-12  # beyond it, the border row's value
    # the same through the filter (huge weight, no smoothing), twice
    zeros = np.zeros((H, W), np.float32)
    st = U.ravel().copy()
    f1, st = oracle.flow_filter(flat_pyramid([zeros]), flat_pyramid([zeros]), W, H, 1, [HUGE], [0], st)
    np.testing.assert_allclose(f1, P, atol=1e-12)
    f2, _ = oracle.flow_filter(flat_pyramid([zeros]), flat_pyramid([zeros]), W, H, 1, [HUGE], [0], st)
    ka, kb = a * (1 - a), b * (1 - b)
    rows2 = slice(0, int((H - 1) / (1 - kb)) - 1)  # (and clear of the rows clamped in the first window)
    np.testing.assert_allclose(f2[0], ka * (x - ka * x), atol=1e-12)
    np.testing.assert_allclose(f2[1][rows2], (kb * (y - kb * y))[rows2], atol=1e-12)


def test_smoothing_by_hand():
    """Five-point mean with replicated border: an interior impulse spreads as
    1/5 at its cross after one iteration, and after two as 1/5 at the centre,
    2/25 at the cross and the diagonals, 1/25 two pixels away; a corner value
    1 becomes 3/5 (its two missing neighbours are itself); both planes alike."""
    F = np.zeros((2, 9, 9))
    F[0, 4, 4] = 1.0
    F[1, 4, 4] = -2.0
    one = oracle.ff_smooth(F, 1)
    want = np.zeros((9, 9))
    want[4, 4] = want[3, 4] = want[5, 4] = want[4, 3] = want[4, 5] = 0.2
    np.testing.assert_allclose(one[0], want, atol=1e-15)
    np.testing.assert_allclose(one[1], -2.0 * want, atol=1e-15)
    two = oracle.ff_smooth(F, 2)[0]
    assert abs(two[4, 4] - 0.2) < 1e-15
    for (dy, dx), v in [((1, 0), 2 / 25), ((1, 1), 2 / 25), ((2, 0), 1 / 25), ((0, 2), 1 / 25), ((2, 1), 0.0)]:
        assert abs(two[4 + dy, 4 + dx] - v) < 1e-15, (dy, dx)
    C = np.zeros((2, 5, 6))
    C[0, 0, 0] = 1.0
    assert abs(oracle.ff_smooth(C, 1)[0, 0, 0] - 0.6) < 1e-15


def test_innovation_reaches_the_finer_layer_at_the_parent():
    """Two layers.  Layer 1 sees I0 = s X^2 and I1 = s (X - t)^2: gradient
    255 * 2 s X, residual 255 s (t^2 - 2 t X), so its update is
    D(X) = -(255 2 s X)(255 s (t^2 - 2 t X)) / ((255 2 s X)^2 + gamma_1);
    layer 0 (flat images, huge weight) then holds 2 D(floor(x / 2)).
    Catches a missing factor 2, a wrong parent pixel and swapped layer
    weights."""
    W, H, s, t, g1 = 48, 10, 1e-4, 1.0, 7.0
    (w0, h0), (w1, h1) = oracle.level_sizes(W, H, 2)
    X = np.arange(w1, dtype=np.float64)
    L1a = np.tile(s * X * X, (h1, 1))
    L1b = np.tile(s * (X - t) ** 2, (h1, 1))
    flat = np.zeros((h0, w0), np.float32)
    pyr0 = flat_pyramid([flat, L1a])
    pyr1 = flat_pyramid([flat, L1b])
    flow, st = oracle.flow_filter(pyr0, pyr1, W, H, 2, [HUGE, g1], [0, 0])
    gx = 255.0 * 2 * s * X
    D = -gx * (255.0 * s * (t * t - 2 * t * X)) / (gx * gx + g1)
    layer1 = oracle.filter_layer(st, W, H, 1)
    inner = slice(1, w1 - 1)  # the ramp's border pixels see a one-sided gradient
    np.testing.assert_allclose(layer1[0][:, inner], np.tile(D[inner], (h1, 1)), rtol=1e-4, atol=1e-9)
    x0 = np.arange(w0)
    par = x0 // 2
    ok = (par >= 1) & (par <= w1 - 2)
    np.testing.assert_allclose(flow[0][:, ok], np.tile(2 * D[par[ok]], (h0, 1)), rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(flow[1], 0.0, atol=1e-12)
    assert np.abs(D[inner]).max() > 0.05  # the pin is not vacuous


def test_zero_motion_and_first_step():
    """Identical windows from a zero state give zero flow at every layer."""
    rng = np.random.default_rng(3)
    W, H, L = 37, 29, 3
    pyr = rng.random(sum(w * h for w, h in oracle.level_sizes(W, H, L))).astype(np.float32)
    flow, st = oracle.flow_filter(pyr, pyr, W, H, L, [500.0, 250.0, 50.0], [5, 25, 50])
    assert np.all(flow == 0.0) and np.all(st == 0.0)
