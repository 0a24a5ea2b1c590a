"""CPU checks of the persistent optimiser's built-in launch table: the shape
the library picks for a batch (disk_optimize_default_tune) is the first row of
the committed table (written by the autotuner) that bounds the batch's size,
largest side and largest tap count, else 256 threads x 4; every row is a valid
launch shape; and the table covers every batch the autotuner measured."""
import os
import re

import pytest

import paper_2512_04556_amd as disk
from paper_2512_04556_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(ROOT, "paper_2512_04556_amd", "csrc", "opt_tune_table.inc")


def _rows():
    src = open(TABLE).read()
    return [tuple(int(v) for v in m) for m in re.findall(r"\{(\d+), (\d+), (\d+), (\d+), (\d+)\}", src)]


def _expected(B, side, T):
    for max_B, max_side, max_T, threads, wgs in _rows():
        if B <= max_B and side <= max_side and T <= max_T:
            return threads, wgs
    return 256, 4


def test_rows_are_valid_shapes():
    rows = _rows()
    assert len(rows) == len(autotune.BATCHES) * len(autotune.SIDES) * len(autotune.TAPS)
    for r in rows:
        assert (r[3], r[4]) in autotune.CANDIDATES, r


@pytest.mark.parametrize("B", [1, 4, 5, 16, 32, 33, 64, 200, 256, 512, 513, 1024, 2048, 2049, 4096, 100000])
def test_lookup_matches_first_row(B):
    for side in (1, 15, 31, 33, 63, 95, 127, 129, 255, 301):
        for T in (2, 48, 49, 96, 256):
            assert disk.optimize_default_tune(B, side, T) == _expected(B, side, T), (B, side, T)


def test_measured_cells_pick_their_own_row():
    """Each cell the autotuner timed (its batch size, its largest side, its
    tap bound) maps back to the row written for it."""
    rows = _rows()
    i = 0
    for B, max_B in autotune.BATCHES:
        for lo, hi in autotune.SIDES:
            for max_T, _ in autotune.TAPS:
                T = 48 if max_T == 48 else 96
                assert rows[i][:3] == (max_B, hi, max_T)
                assert disk.optimize_default_tune(B, hi, T) == (rows[i][3], rows[i][4]), (B, hi, T)
                i += 1


def test_bad_meta_is_refused():
    with pytest.raises(disk.DiskError):
        disk.optimize_default_tune(0, 31, 48)
    with pytest.raises(disk.DiskError):
        disk.optimize_default_tune(4, 31, 0)
