"""Pins of the oracle's variational refinement (the third stage of dense
inverse search): exact fixed points, a two-pixel case worked by hand, the
symmetry between the axes, and the direction it moves a wrong flow."""
import numpy as np
import pytest

import oracle


def test_zero_motion_stays_zero():
    rng = np.random.default_rng(0)
    I0 = rng.random((20, 24)).astype(np.float32)
    assert np.all(oracle.var_refine(I0, I0, np.zeros((2, 20, 24))) == 0.0)


def test_swapping_the_axes_swaps_the_result():
    """Transposed images with the flow's components swapped give exactly the
    transposed, swapped result (integer flows: the warp is exact): catches a
    swapped derivative, a misplaced coupling term or a transposed index."""
    rng = np.random.default_rng(1)
    for H, W in [(20, 24), (9, 13)]:
        I0 = rng.random((H, W)).astype(np.float32)
        I1 = rng.random((H, W)).astype(np.float32)
        U = rng.integers(-2, 3, (2, H, W)).astype(np.float64)
        a = oracle.var_refine(I0, I1, U)
        b = oracle.var_refine(I0.T.copy(), I1.T.copy(), np.stack([U[1].T, U[0].T]))
        assert np.array_equal(a[0], b[1].T) and np.array_equal(a[1], b[0].T)
        assert np.abs(a - U).max() > 0.1  # and it did move


def test_two_pixels_by_hand():
    """A 2x1 image, I0 = (0.25, 0.75), I1 = (0.5, 0.5), U = 0, one fixed-point
    iteration of one SOR sweep.  On the 8-bit scale: It = (63.75, -63.75);
    the average image's x-derivative is 31.875 at both pixels (replicated
    border), every other spatial derivative is 0; Ixt = 0 - 63.75.  Data
    weight delta / sqrt(63.75^2 + 1e-6) at both pixels; gradient terms vanish
    (Ixx = Ixy = 0); smoothness weight alpha / sqrt(0 + 1e-6) = 1000 alpha.
    The red pixel (x = 0) solves (a11 + w) du0 = -b1 (its neighbour's
    increment is still 0), the black one (a11 + w) du1 = w du0 - b1(1), each
    relaxed by omega; v stays 0."""
    a, g, d, om = 20.0, 10.0, 5.0, 1.6
    I0 = np.array([[0.25, 0.75]], np.float32)
    I1 = np.array([[0.5, 0.5]], np.float32)
    out = oracle.var_refine(I0, I1, np.zeros((2, 1, 2)), outer=1, inner=1, alpha=a, gamma=g, delta=d, omega=om)
    wc = d / np.sqrt(63.75 ** 2 + 1e-6)
    a11 = wc * 31.875 * 31.875
    b1 = wc * 31.875 * 63.75
    w = a * 1000.0
    du0 = om * (-b1 / (a11 + w))
    du1 = om * ((w * du0 + b1) / (a11 + w))
    assert out[0, 0, 0] == pytest.approx(du0, rel=1e-13)
    assert out[0, 0, 1] == pytest.approx(du1, rel=1e-13)
    assert np.all(out[1] == 0.0)
    assert du0 < 0 and du1 > du0  # the smoothness pulls pixel 1 along, its own brightness change back


def test_wrong_flow_moves_towards_the_shift():
    """A smooth texture shifted by (2, -1) px, refined from the constant flow
    (2.4, -1.3): the interior error to the true shift shrinks."""
    ndi = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(6)
    H, W, dx, dy = 60, 80, 2, -1
    big = ndi.gaussian_filter(rng.random((H + 8, W + 8)), 3.0)
    big = (big - big.min()) / (big.max() - big.min())
    I0 = big[4:4 + H, 4:4 + W].astype(np.float32)
    I1 = big[4 - dy:4 - dy + H, 4 - dx:4 - dx + W].astype(np.float32)
    U = np.stack([np.full((H, W), 2.4), np.full((H, W), -1.3)])
    out = oracle.var_refine(I0, I1, U)
    inner = (slice(8, H - 8), slice(8, W - 8))
    e0 = np.hypot(U[0][inner] - dx, U[1][inner] - dy).mean()
    e1 = np.hypot(out[0][inner] - dx, out[1][inner] - dy).mean()
    assert e1 < 0.5 * e0


def test_refined_flow_zero_motion_and_levels():
    """The whole flow with refinement: zero motion gives exactly 0; without
    refinement settings it is the plain flow."""
    rng = np.random.default_rng(2)
    H, W = 64, 80
    S = rng.random((H, W)).astype(np.float32)
    pyr, _ = oracle.pyramid(S, 3)
    assert np.all(oracle.dis_flow(pyr, pyr, W, H, 3, refine={}) == 0.0)
    T = np.roll(S, 2, axis=1)
    pyr1, _ = oracle.pyramid(T, 3)
    assert np.array_equal(oracle.dis_flow(pyr, pyr1, W, H, 3), oracle.dis_flow(pyr, pyr1, W, H, 3, refine=None))
    assert not np.array_equal(oracle.dis_flow(pyr, pyr1, W, H, 3), oracle.dis_flow(pyr, pyr1, W, H, 3, refine={}))
