"""Pins of the oracle's window-resize scheme (Sec. III-C, Fig. 4, Table III): r_now taps per
side spread over the original radius r_orig at spacing s = r_orig / r_now, reference values
interpolated.  With s = 1 and s = 2 it is exactly the dense window and the integer dilation;
with a fractional s and a translation-only homography the per-view score is one minus
numpy's Pearson correlation of the two patches sampled by scipy's linear interpolation."""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle

from test_oracle_pins import _K, _fronto, _pose_problem, _textured


def _both(A, B, D, window, dilation=1, tap_radius=0, bilateral=False, sigma_s=4.0):
    h, w = A.shape
    return _pose_problem([A, B], [_K(w, h), _K(w, h, dcx=D)], window=window, dilation=dilation, bilateral=bilateral,
                         sigma_s=sigma_s, tap_radius=tap_radius)


@pytest.mark.parametrize("bilateral", [False, True])
@pytest.mark.parametrize("window,tap_radius,dilation", [(11, 5, 1), (21, 5, 2), (13, 3, 2)])
def test_integer_spacing_equals_the_integer_dilation(window, tap_radius, dilation, bilateral):
    """s = r_orig / r_now integer: the resize scheme samples texels exactly, bitwise the
    integer-dilation window (FP32 and FP64 modes)."""
    h, w = 44, 52
    A, B = _textured(h, w, 11), _textured(h, w, 12)
    a = _both(A, B, 3, window, tap_radius=tap_radius, bilateral=bilateral)
    b = _both(A, B, 3, window, dilation=dilation, bilateral=bilateral)
    for fp64 in (False, True):
        ca, pa, oka = oracle.eval_cost(a, _fronto(h, w), fp64=fp64)
        cb, pb, okb = oracle.eval_cost(b, _fronto(h, w), fp64=fp64)
        assert np.array_equal(ca, cb) and np.array_equal(pa, pb) and np.array_equal(oka, okb)
    assert np.array_equal(a.valid_mask(), b.valid_mask())


@pytest.mark.parametrize("window,tap_radius", [(13, 5), (15, 5), (17, 5), (19, 5)])
def test_fractional_spacing_matches_interpolated_correlation(window, tap_radius):
    """Rectified pair with integer disparity D: the warped tap of reference offset o = s k is
    the source point shifted by D, so both patches are linear interpolations at the same
    fractional offsets (scipy), and 1 - C_j is their Pearson correlation (weights off)."""
    h, w = 48, 56
    A, B = _textured(h, w, 13), _textured(h, w, 14)
    D = 3
    pb = _both(A, B, D, window, tap_radius=tap_radius)
    _, pv, ok = oracle.eval_cost(pb, _fronto(h, w), fp64=True)
    r_orig = (window - 1) // 2
    s = r_orig / tap_radius
    offs = s * np.arange(-tap_radius, tap_radius + 1)
    rng = np.random.default_rng(1)
    m = pb.valid_mask()
    assert m.sum() == (w - 2 * r_orig) * (h - 2 * r_orig)  # validity radius is r_orig
    n = 0
    for _ in range(40):
        x = int(rng.integers(r_orig, w - r_orig - D))
        y = int(rng.integers(r_orig, h - r_orig))
        yy, xx = np.meshgrid(y + offs, x + offs, indexing="ij")
        a = ndi.map_coordinates(A.astype(np.float64), [yy.ravel(), xx.ravel()], order=1)
        b = ndi.map_coordinates(B.astype(np.float64), [yy.ravel(), xx.ravel() + D], order=1)
        z = np.corrcoef(a, b)[0, 1]
        assert ok[y, x, 0]
        assert abs((1 - pv[y, x, 0]) - z) < 1e-9
        n += 1
    assert n == 40
