"""The autotuner's decision rule (CPU): the threshold of a pass is the largest window
up to which the direct pass is never slower than the large-window pass by more
than the tolerance; later windows do not reopen it."""
from paper_2002_09474_amd import autotune


def _rows(axis, pairs):
    return [{"axis": axis, "w": w, "direct_us": d, "large_us": l} for w, (d, l) in pairs.items()]


def test_threshold_stops_at_first_loss():
    rows = _rows("x", {2: (1.0, 2.0), 3: (1.0, 1.02), 4: (1.2, 1.0), 5: (0.5, 1.0)})
    rows += _rows("y", {2: (3.0, 1.0), 3: (1.0, 2.0)})
    assert autotune.threshold(rows, "x") == 3  # 4 loses by 20%; 5's win does not count
    assert autotune.threshold(rows, "y") == 1  # direct loses at once
    assert autotune.threshold(rows, "x", tol=0.25) == 5


def test_threshold_unordered_input():
    rows = _rows("x", {5: (1.0, 1.0), 2: (1.0, 1.0), 4: (1.0, 1.0), 3: (1.0, 1.0)})
    assert autotune.threshold(rows, "x") == 5
