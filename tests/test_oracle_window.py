"""Pins of the oracle's adaptive window rule (area event count): hand-worked
event sequences whose window end follows from the definition."""
import numpy as np

import oracle


def ev(pts):
    a = np.array(pts, np.int64).reshape(-1, 2)
    return a[:, 0].astype(np.uint16), a[:, 1].astype(np.uint16)


def test_first_square_to_reach_k_ends_the_window():
    # 8x8 sensor, 4-px squares: (0,0) (1,0) / (0,1) (1,1)
    x, y = ev([(0, 0), (5, 5), (1, 1), (6, 1), (2, 3), (7, 7), (3, 0)])
    # square (0,0) gets events 0, 2, 4, 6 -> its 3rd event is event 4
    assert oracle.window_end_area(8, 8, x, y, 0, 4, 3) == 5
    # square (1,1) gets events 1 and 5: k = 2 is reached at event 5 but (0,0)
    # reaches 2 earlier, at event 2
    assert oracle.window_end_area(8, 8, x, y, 0, 4, 2) == 3
    # k = 1: the first on-sensor event ends the window
    assert oracle.window_end_area(8, 8, x, y, 0, 4, 1) == 1


def test_start_index_and_no_square_reaching_k():
    x, y = ev([(0, 0), (0, 0), (0, 0), (5, 5), (5, 6)])
    assert oracle.window_end_area(8, 8, x, y, 2, 4, 2) == 5   # from event 2: (1,1) reaches 2 at event 4
    assert oracle.window_end_area(8, 8, x, y, 3, 4, 3) == 5   # nothing reaches 3: all events
    assert oracle.window_end_area(8, 8, x, y, 5, 4, 1) == 5   # empty remainder


def test_off_sensor_events_count_for_no_square():
    x, y = ev([(9, 0), (0, 9), (1, 1), (2, 2)])
    assert oracle.window_end_area(8, 8, x, y, 0, 4, 2) == 4


def test_one_square_is_an_event_count_window():
    rng = np.random.default_rng(0)
    x = rng.integers(0, 40, 500).astype(np.uint16)
    y = rng.integers(0, 30, 500).astype(np.uint16)
    x[::7] = 60   # off the 40x30 sensor
    on = np.flatnonzero(x < 40)
    # a square covering the sensor: the window is the next 100 on-sensor events
    assert oracle.window_end_area(40, 30, x, y, 0, 64, 100) == on[99] + 1
    assert oracle.window_end_area(40, 30, x, y, 13, 64, 100) == on[np.searchsorted(on, 13) + 99] + 1


def test_brute_force_small_streams():
    """Against counting by hand over numpy: for each prefix length, the
    largest square count."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        W, H = int(rng.integers(1, 30)), int(rng.integers(1, 30))
        a = int(rng.integers(1, 12))
        n = int(rng.integers(0, 200))
        x = rng.integers(0, W + 3, n).astype(np.uint16)
        y = rng.integers(0, H + 3, n).astype(np.uint16)
        i0 = int(rng.integers(0, n + 1))
        k = int(rng.integers(1, 9))
        ax = (W + a - 1) // a
        on = (x < W) & (y < H)
        sq = (y.astype(np.int64) // a) * ax + x.astype(np.int64) // a
        want = n
        for i1 in range(i0 + 1, n + 1):
            s = sq[i0:i1][on[i0:i1]]
            if s.size and np.bincount(s).max() >= k:
                want = i1
                break
        assert oracle.window_end_area(W, H, x, y, i0, a, k) == want
