"""Closed-form pins of the oracle's dense inverse search, step by step.

The paper leaves the frame-based flow open (Sec. III-D), so every DIS rule
below is a reading of ours (the readings are listed with the design notes).
Each test fixes one rule with hand-derived numbers, so that a plausible
mistake in the oracle fails it:

  densification weight 1/max(1, 255 |d|)   -- drop the 255, drop the max(1, .)
  outlier reset |u - u0| > patch size      -- other threshold, |u| instead of
                                              |u - u0|, reset to 0, max-norm
  coarse-to-fine start at the patch centre -- start at the origin, no factor 2
  cover of the clamped last patch          -- last origin not clamped / dropped
  warm start from the previous flow        -- wrong level scale or pixel
  damping lambda I                         -- the linearised contraction
                                              lambda (H + lambda I)^-1 per step
"""
import numpy as np
import pytest

import oracle


# --------------------------------------------------------------------------
# densification weight
# --------------------------------------------------------------------------
def _two_patch_case(step):
    """12x8 level, stride 4: two patches, origins x = 0 (A) and x = 4 (B),
    one patch row.  I0 = 0.5; I1 = 0.5 on columns 0..4 and 0.5 + step on
    columns 5..11 (values exact in float32).  A moves by (1, 0), B stays."""
    I0 = np.full((8, 12), 0.5, np.float32)
    I1 = I0.copy()
    I1[:, 5:] = np.float32(0.5 + step)
    pu = np.array([[[1.0, 0.0], [0.0, 0.0]]])  # [ny=1, nx=2, 2]
    return I0, I1, pu


def test_densify_weight_uses_255_scale():
    """Pixel x = 4 lies in both patches.  A samples I1(5) - I0(4) = 0.125,
    weight 1/(255 * 0.125) = 1/31.875; B samples I1(4) - I0(4) = 0, weight 1.
    U = (1/31.875 * 1 + 1 * 0) / (1/31.875 + 1) = 1/32.875.  Pixels 5..7:
    both residuals 0.125, equal weights, U = 1/2.  Pixels 0..3 only in A
    (U = 1), pixels 8..11 only in B (U = 0).  Without the 255 both weights at
    x = 4 would be 1 (U = 1/2)."""
    I0, I1, pu = _two_patch_case(0.125)
    U = oracle.densify(I0, I1, pu)
    expect_u = [1, 1, 1, 1, 1 / 32.875, 0.5, 0.5, 0.5, 0, 0, 0, 0]
    for y in range(8):
        assert np.allclose(U[0, y], expect_u, rtol=0, atol=1e-15)
    assert np.all(U[1] == 0.0)


def test_densify_weight_saturates_at_one():
    """A residual below 1/255 gives weight exactly 1 (the max(1, .)):
    step 2^-9 = 0.001953125, 255 * step = 0.498 < 1, so at x = 4 the weights
    are 1 and 1 and U = 1/2.  Without the max the weight of B (residual 0)
    would be infinite."""
    I0, I1, pu = _two_patch_case(2.0 ** -9)
    U = oracle.densify(I0, I1, pu)
    assert U[0, 3, 4] == 0.5 and U[0, 3, 5] == 0.5 and U[0, 3, 3] == 1.0 and U[0, 3, 8] == 0.0


def test_densify_cover_of_clamped_last_patch():
    """Flat images (every residual 0, every weight 1): the densified flow is
    the plain mean over the covering patches.  Patch (kx, ky) moves by
    (2^kx, 2^ky).  18 px at stride 3: origins 0, 3, 6, 9 and the clamped
    last one at 10 (not 12), covering 0..7, 3..10, 6..13, 9..16, 10..17;
    10 px at stride 4: origins 0 and 2 (not 4), covering 0..7 and 2..9.
    Means over those cover sets, worked by hand:"""
    mean_18_s3 = [1, 1, 1, 1.5, 1.5, 1.5, 7 / 3, 7 / 3, 3, 14 / 3, 7.5, 28 / 3, 28 / 3, 28 / 3, 12, 12, 12, 16]
    mean_10_s4 = [1, 1, 1.5, 1.5, 1.5, 1.5, 1.5, 1.5, 2, 2]
    for W, H, s, ex, ey in [(18, 10, 3, mean_18_s3, None), (10, 18, 4, mean_10_s4, None),
                            (18, 18, 3, mean_18_s3, mean_18_s3), (10, 10, 4, mean_10_s4, mean_10_s4)]:
        nx, ny = (W - 8 + s - 1) // s + 1, (H - 8 + s - 1) // s + 1
        pu = np.zeros((ny, nx, 2))
        pu[..., 0] = 2.0 ** np.arange(nx)[None, :]
        pu[..., 1] = 2.0 ** np.arange(ny)[:, None]
        img = np.full((H, W), 0.25, np.float32)
        U = oracle.densify(img, img, pu, stride=s)
        assert np.allclose(U[0], np.array(ex)[None, :], rtol=0, atol=1e-13), (W, H, s)
        if ey is not None:
            assert np.allclose(U[1], np.array(ey)[:, None], rtol=0, atol=1e-13), (W, H, s)


# --------------------------------------------------------------------------
# outlier reset
# --------------------------------------------------------------------------
def _x_ramp_pair(d, W=112, H=16, a=1.0 / 64):
    """I0 = 0.1 + a x, I1 = I0 shifted right by d (I1(x) = I0(x - d))."""
    x = np.arange(W, dtype=np.float64)
    I0 = np.tile(0.1 + a * x, (H, 1)).astype(np.float32)
    I1 = np.tile(0.1 + a * (x - d), (H, 1)).astype(np.float32)
    return I0, I1


def _interior_patches(pu, W, s=4, reach=16):
    """patches whose samples x + u stay inside the image for |u| <= reach"""
    nx = pu.shape[1]
    ox = np.minimum(np.arange(nx) * s, W - 8)
    keep = (ox - reach >= 0) & (ox + 7 + reach <= W - 1)
    return pu[:, keep]


def test_reset_threshold_on_ramp():
    """On a ramp along x the step is exact along x: with lambda = 1e-3 each
    step leaves lambda / (lambda + 64 a^2) = 0.06 of the error, so 16 steps
    reach the shift.  A shift of 7 px (< 8 = the patch size) is kept; a shift
    of 9 px is taken back to the start, exactly 0."""
    W = 112
    for d, expect in [(7.0, 7.0), (9.0, 0.0), (7.9, 7.9), (8.1, 0.0)]:
        I0, I1 = _x_ramp_pair(d, W)
        pu = _interior_patches(oracle.dis_level(I0, I1, lam=1e-3), W)
        assert np.allclose(pu[..., 0], expect, rtol=0, atol=1e-4), d
        assert np.all(pu[..., 1] == 0.0)
        if expect == 0.0:
            assert np.all(pu == 0.0)


def test_reset_measures_the_move_from_the_start():
    """Start at u0 = (5, 0).  Shift 9: the patch moves by 4 from its start and
    is kept (a reset judged on |u| > 8 would return it to 5).  Shift 14: it
    moves by 9 and goes back to exactly (5, 0) (not to 0)."""
    W = 112
    for d, expect in [(9.0, 9.0), (14.0, 5.0)]:
        I0, I1 = _x_ramp_pair(d, W)
        nx, ny = (W - 8 + 3) // 4 + 1, (16 - 8 + 3) // 4 + 1
        u0 = np.zeros((ny, nx, 2))
        u0[..., 0] = 5.0
        pu = _interior_patches(oracle.dis_level(I0, I1, u0=u0, lam=1e-3), W, reach=20)
        assert np.allclose(pu[..., 0], expect, rtol=0, atol=1e-4), d
        if expect == 5.0:
            assert np.all(pu[..., 0] == 5.0) and np.all(pu[..., 1] == 0.0)


def test_reset_uses_euclidean_norm():
    """A paraboloid has a full-rank Hessian, and an integer shift is a
    fixed point of the bilinear residual.  Shift (5, 5): |d| = 7.07 < 8,
    recovered.  Shift (7, 7): each component is below 8 but |d| = 9.9 > 8:
    reset to exactly 0."""
    W = H = 96
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)

    def img(x, y):
        return 1e-3 * ((x - 48.0) ** 2 + (y - 48.0) ** 2)

    for d, kept in [((5.0, 5.0), True), ((7.0, 7.0), False)]:
        I0 = img(xx, yy).astype(np.float32)
        I1 = img(xx - d[0], yy - d[1]).astype(np.float32)
        pu = oracle.dis_level(I0, I1, lam=1e-3, iters=40)
        inner = pu[5:-5, 5:-5]  # origins 20..72: samples stay inside
        if kept:
            assert np.allclose(inner[..., 0], d[0], atol=1e-3) and np.allclose(inner[..., 1], d[1], atol=1e-3)
        else:
            assert np.all(inner == 0.0)


# --------------------------------------------------------------------------
# where a patch starts
# --------------------------------------------------------------------------
def test_coarse_to_fine_start_at_patch_centre():
    """A 21x13 level at stride 4 has patch origins x = 0, 4, 8, 12, 13 (the
    last clamped) and y = 0, 4, 5.  Their centres o + 4, halved, give the
    coarser pixels x = 2, 4, 6, 8, 8 and y = 2, 4, 4.  With the coarser flow
    u(x, y) = x + 100 y, v(x, y) = 1000 + x, the start is twice that there:"""
    Wc, Hc = 11, 7
    yy, xx = np.mgrid[0:Hc, 0:Wc].astype(np.float64)
    Uc = np.stack([xx + 100 * yy, 1000 + xx])
    u0 = oracle.patch_init_coarser(21, 13, Uc)
    expect_u = [[404, 408, 412, 416, 416],
                [804, 808, 812, 816, 816],
                [804, 808, 812, 816, 816]]
    expect_v = [[2004, 2008, 2012, 2016, 2016]] * 3
    assert np.array_equal(u0[..., 0], np.array(expect_u, np.float64))
    assert np.array_equal(u0[..., 1], np.array(expect_v, np.float64))
    # a coarser field smaller than the centres reach: clamped into it
    u0 = oracle.patch_init_coarser(21, 13, Uc[:, :2, :3].copy())
    assert np.array_equal(u0[..., 0], np.array([[2 * (min(c, 2) + 100 * min(r, 1)) for c in (2, 4, 6, 8, 8)]
                                                  for r in (2, 4, 4)], np.float64))


def test_warm_start_from_previous_flow():
    """Level 2 of a 64x40 sensor is 16x10: origins x = 0, 4, 8 and y = 0, 2;
    centres 4, 8, 12 and 4, 6, times 2^2: sensor pixels x = 16, 32, 48,
    y = 16, 24.  With the previous flow u = x + 100 y, v = -y, the start is
    that there divided by 4."""
    yy, xx = np.mgrid[0:40, 0:64].astype(np.float64)
    Up = np.stack([xx + 100 * yy, -yy])
    u0 = oracle.patch_init_previous(16, 10, 2, Up)
    assert np.array_equal(u0[..., 0], np.array([[404, 408, 412], [604, 608, 612]], np.float64))
    assert np.array_equal(u0[..., 1], np.array([[-4, -4, -4], [-6, -6, -6]], np.float64))


def test_warm_start_seeds_the_coarsest_level():
    """Constant velocity: the previous pair's flow is (2.5, -1.5) everywhere.
    With a flat coarsest level (no gradient, the patches keep their start)
    the coarsest patches of the warm-started flow are exactly that flow
    scaled to the level, (2.5, -1.5) / 4 at level 2; cold, they stay 0."""
    W, H, L = 64, 48, 3
    rng = np.random.default_rng(3)
    sizes = oracle.level_sizes(W, H, L)
    lv0 = [rng.random((h, w)).astype(np.float32) for w, h in sizes]
    lv0[-1][:] = 1.0
    pyr0 = np.concatenate([a.ravel() for a in lv0])
    pyr1 = pyr0.copy()
    prev = np.stack([np.full((H, W), 2.5), np.full((H, W), -1.5)])
    npl = [oracle.patch_count(w, h) for w, h in sizes]
    _, pu = oracle.dis_flow(pyr0, pyr1, W, H, L, want_patches=True, prev_flow=prev)
    coarse = pu[sum(npl[:2]):]
    assert np.all(coarse[:, 0] == 0.625) and np.all(coarse[:, 1] == -0.375)
    _, pu = oracle.dis_flow(pyr0, pyr1, W, H, L, want_patches=True)
    assert np.all(pu[sum(npl[:2]):] == 0.0)


def test_warm_start_recovers_motion_beyond_the_cold_reach():
    """Events shifted by 20 px: the cold two-level search would need 10 px at
    the coarse level, beyond the 8-px reset, and ends far off; started from
    the previous pair's (20, 0) it recovers the shift."""
    W, H, L = 160, 96, 2
    rng = np.random.default_rng(11)
    n = int(0.03 * W * H)
    x, y = rng.integers(0, W, n), rng.integers(0, H, n)
    x1 = x + 20
    keep = x1 < W
    t = np.zeros(n, np.int64)
    a = oracle.window(W, H, x, y, t, 0, 10, 0, 5, 1.08, L)
    b = oracle.window(W, H, x1[keep], y[keep], t[keep], 0, 10, 0, 5, 1.08, L)
    inner = (slice(12, H - 12), slice(12, W - 32))
    cold = oracle.dis_flow(a["pyr"], b["pyr"], W, H, L)
    prev = np.stack([np.full((H, W), 20.0), np.zeros((H, W))])
    warm = oracle.dis_flow(a["pyr"], b["pyr"], W, H, L, prev_flow=prev)
    e_cold = np.hypot(cold[0][inner] - 20, cold[1][inner])
    e_warm = np.hypot(warm[0][inner] - 20, warm[1][inner])
    assert np.median(e_cold) > 5.0
    assert np.median(e_warm) < 1e-6 and np.mean(e_warm < 0.05) > 0.95


# --------------------------------------------------------------------------
# damping: the bias of lambda = 0.3 after 16 steps
# --------------------------------------------------------------------------
def test_damping_contraction_on_smooth_texture():
    """An integer shift d of a smooth texture is an exact fixed point of the
    bilinear residual.  Started near it, at u0 = d + e0, the damped step
    leaves e_{k+1} = lambda (H + lambda I)^-1 e_k to first order (H = sum g g^T
    of the patch), so after 16 steps the error is M^16 e0 with
    M = lambda (H + lambda I)^-1: at lambda = 0.3 weakly textured patches keep
    a visible part of their start error -- the bias of the damped solver
    that the flow tests carry (the GPU reproduces it, it is the oracle's).
    Checked per patch against the prediction from the texture's gradient."""
    ndi = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(6)
    H, W, d, lam = 72, 96, (2, -1), 0.3
    big = ndi.gaussian_filter(rng.random((H + 8, W + 8)), 2.0)
    big = (big - big.min()) / (big.max() - big.min())
    I0 = big[4:4 + H, 4:4 + W].astype(np.float32)
    I1 = big[4 - d[1]:4 - d[1] + H, 4 - d[0]:4 - d[0] + W].astype(np.float32)  # I1(x) = I0(x - d)
    nx, ny = (W - 8 + 3) // 4 + 1, (H - 8 + 3) // 4 + 1
    e0 = np.array([0.05, -0.03])
    u0 = np.tile(np.array(d, np.float64) + e0, (ny, nx, 1))
    pu = oracle.dis_level(I0, I1, u0=u0, lam=lam)
    # gradient of the template by central differences (interior patches only)
    I = I0.astype(np.float64)
    gx = np.zeros_like(I)
    gy = np.zeros_like(I)
    gx[:, 1:-1] = 0.5 * (I[:, 2:] - I[:, :-2])
    gy[1:-1, :] = 0.5 * (I[2:, :] - I[:-2, :])
    checked = 0
    worst = 0.0
    for ky in range(2, ny - 2):
        for kx in range(2, nx - 2):
            oy, ox = ky * 4, kx * 4
            px, py = gx[oy:oy + 8, ox:ox + 8].ravel(), gy[oy:oy + 8, ox:ox + 8].ravel()
            Hm = np.array([[px @ px, px @ py], [px @ py, py @ py]])
            M = lam * np.linalg.inv(Hm + lam * np.eye(2))
            pred = np.linalg.matrix_power(M, 16) @ e0
            got = pu[ky, kx] - np.array(d)
            worst = max(worst, float(np.linalg.norm(got - pred)))
            checked += 1
    assert checked > 100
    # first-order model: agreement to a small fraction of |e0| (0.058 px)
    assert worst < 0.1 * np.linalg.norm(e0), worst
    # and the bias is real: some patches keep more than a fifth of e0
    biased = [np.linalg.norm(pu[ky, kx] - np.array(d)) for ky in range(2, ny - 2) for kx in range(2, nx - 2)]
    assert max(biased) > 0.2 * np.linalg.norm(e0)
