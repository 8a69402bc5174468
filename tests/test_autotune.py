"""The autotuner's decision rule (CPU): the threshold of a pass is the window before
the first sustained loss of the direct pass (two consecutive swept windows where it
is slower than the large-window pass by more than the tolerance); a single loss
within the noise does not end the direct range, and later wins do not reopen it."""
from paper_2002_09474_amd import autotune


def _rows(axis, pairs):
    return [{"axis": axis, "w": w, "direct_us": d, "large_us": l} for w, (d, l) in pairs.items()]


def test_threshold_stops_at_first_sustained_loss():
    rows = _rows("x", {2: (1.0, 2.0), 3: (1.0, 1.02), 4: (1.2, 1.0), 5: (1.2, 1.0), 6: (0.5, 1.0)})
    rows += _rows("y", {2: (3.0, 1.0), 3: (2.0, 1.0)})
    assert autotune.threshold(rows, "x") == 3  # 4 and 5 lose by 20%; 6's win does not count
    assert autotune.threshold(rows, "y") == 1  # direct loses at once
    assert autotune.threshold(rows, "x", tol=0.25) == 6


def test_a_single_loss_in_the_noise_does_not_end_the_direct_range():
    rows = _rows("x", {2: (1.05, 1.0), 3: (1.0, 1.0), 4: (1.0, 1.0), 5: (1.1, 1.0), 6: (1.0, 1.0),
                       7: (1.1, 1.0), 8: (1.1, 1.0)})
    assert autotune.threshold(rows, "x") == 6
    # a loss at the last swept window ends the range
    rows = _rows("y", {2: (1.0, 1.0), 3: (1.0, 1.0), 4: (1.2, 1.0)})
    assert autotune.threshold(rows, "y") == 3


def test_threshold_unordered_input():
    rows = _rows("x", {5: (1.0, 1.0), 2: (1.0, 1.0), 4: (1.0, 1.0), 3: (1.0, 1.0)})
    assert autotune.threshold(rows, "x") == 5


def test_unit_height_least_worst_over_windows():
    """A unit height is chosen by its worst time relative to the best height at each
    window, so one window's large loss is not hidden by small gains elsewhere."""
    res = [{"h": 8, "us": [10.0, 20.0, 30.0]},
           {"h": 16, "us": [13.0, 19.0, 28.0]},   # sum 60 (least), but 30% worse at the first
           {"h": 24, "us": [10.5, 19.5, 29.0]}]   # at most 5% worse anywhere
    assert autotune.least_worst(res, "h") == 24
    assert autotune.least_worst(res[:1], "h") == 8
