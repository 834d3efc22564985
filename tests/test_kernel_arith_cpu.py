"""Arithmetic shortcuts the kernels take, checked exhaustively on the CPU."""
import numpy as np


def test_fp32_row_division_exact_for_small_rectangles():
    """The expansion finds the row of pair kk in a w-wide rectangle as
    floor((kk + 1/2) * rcp(w)) in fp32 when rectangles have at most 256 x 256
    tiles.  Exact for every w <= 256 and kk < 256 w, with the hardware
    reciprocal off by up to one ulp in either direction."""
    f32 = np.float32
    for w in range(1, 257):
        kk = np.arange(256 * w, dtype=np.uint32)
        want = kk // np.uint32(w)
        r = f32(1.0) / f32(w)
        for inv in (np.nextafter(r, f32(0)), r, np.nextafter(r, f32(1))):
            got = ((kk.astype(f32) + f32(0.5)) * f32(inv)).astype(np.uint32)
            assert np.array_equal(got, want), w
