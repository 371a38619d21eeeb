"""Bounds of the LDS reads of the ramp and ray kernels, walked on the host
from the kernels' own layout formulas (skei_lds_read_bounds; no device).

Ramp: every window read of every thread -- including threads whose outputs
lie past the row end, which read beyond the row into the partial-sum area --
stays inside the allocation, and threads that own an output read only the
staged row, for every detector count the library accepts (2..2048).
Ray march: clamped tap positions stay inside the padded line for every image
size (2..2032).
Gathers: the fixed-point pixel positions of every 16 x 16 tile fall in
window bins 0 .. 31 (with the interpolation neighbour) for every angle of a
7- and a 360-angle table, at small and full detector counts, for image sizes
across the range (ragged tiles, powers of two and the maximum 2032)."""
import ctypes

import pytest

from paper_2411_05771_amd import capi


def bounds(kernel, size, n):
    out = (ctypes.c_longlong * n)()
    capi.call("skei_lds_read_bounds", kernel, size, out)
    return list(out)


def test_ramp_window_reads_stay_in_lds(hiplib):
    worst = None
    for nd in range(2, 2049):
        lo, hi_active, hi_any, row_end, alloc = bounds(0, nd, 5)
        assert lo >= 0, nd
        assert hi_active <= row_end, nd           # output-owning threads read the staged row only
        assert hi_any < alloc, nd                 # idle threads stay inside the allocation
        slack = alloc - 1 - hi_any
        worst = slack if worst is None else min(worst, slack)
    print(f"smallest slack below the end of the ramp's LDS allocation: {worst} doubles")


def test_ray_taps_stay_in_padded_line(hiplib):
    for n in range(2, 2033):
        lo, hi, pitch = bounds(1, n, 3)
        assert lo >= 0 and hi < pitch, n


@pytest.mark.parametrize("n", [2, 3, 15, 16, 17, 31, 33, 64, 100, 255, 256, 257, 511, 512, 1000, 1024, 2032])
def test_gather_positions_stay_in_window(hiplib, n):
    lo, hi, win = bounds(2, n, 3)
    assert lo >= 0 and hi <= win - 1, (n, lo, hi)


def test_layout_walk_rejects_bad_arguments(hiplib):
    out = (ctypes.c_longlong * 5)()
    assert capi.lib().skei_lds_read_bounds(0, 1, out) == -1
    assert capi.lib().skei_lds_read_bounds(0, 4096, out) == -4
    assert capi.lib().skei_lds_read_bounds(7, 64, out) == -1
