"""Pins of the local noise normalisation oracle (CPU only).

Sect. 4.1: the cube is divided by its noise measured in a running window
(31 px / 31 ch in the speed test of Sect. 5). The oracle measures the noise
on a grid of blocks, each in a window around the block's centre (readings
N1-N4 in oracle/nn_oracle.cpp). Each test checks it against something other
than itself: a hand-worked line (tests/golden), the independent brute force
(oracle/brute.py), the smooth-and-clip oracle's global noise (whole-cube
window), closed forms and exact floating-point invariants.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    with open(os.path.join(GOLDEN, "noise_norm_1d.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("axis", ["x", "y", "z"])
def test_hand_worked_line_on_every_axis(axis):
    g = _golden()
    v = np.array(g["values"], np.float32)
    shape = {"x": (1, 1, 7), "y": (1, 7, 1), "z": (7, 1, 1)}[axis]
    x = v.reshape(shape)
    w, step = g["window"], g["grid"]
    # the other axes are one voxel long: any window there holds that voxel
    w_xy, g_xy, w_z, g_z = (w, step, 1, 1) if axis != "z" else (1, 1, w, step)
    for case in g["cases"]:
        sig, y = oracle.normalise(x, w_xy, w_z, g_xy, g_z, case["mode"], case["range"])
        sig = sig.ravel()
        if case["mode"] == "mad":
            expect = 1.4826 * np.array(case["median_abs"])
        else:
            expect = np.sqrt(np.array(case["mean_square"]))
        np.testing.assert_allclose(sig, expect, rtol=1e-15, err_msg=f"{axis} {case}")
        blocks = [0, 0, 1, 1, 2, 2, 3]
        expect_y = np.array([np.float32(float(v[i]) / sig[blocks[i]]) for i in range(7)])
        np.testing.assert_array_equal(y.ravel(), expect_y)


def test_hand_worked_zeros_are_not_negative():
    g = _golden()
    z = g["zero_line"]
    x = np.array(z["values"], np.float32).reshape(1, 1, 7)
    sig, _ = oracle.normalise(x, g["window"], 1, g["grid"], 1, z["mode"], z["range"])
    np.testing.assert_allclose(sig.ravel(), 1.4826 * np.array(z["median_abs"]), rtol=1e-15)


def _rand_cube(rng, shape, nan_frac=0.03):
    x = rng.standard_normal(shape).astype(np.float32)
    x *= np.float32(1.0) + rng.random(shape).astype(np.float32)
    x[rng.random(shape) < nan_frac] = np.nan
    return x


@pytest.mark.parametrize("mode,rng_", [("mad", "negative"), ("mad", "all"),
                                       ("mad", "positive"), ("std", "all"),
                                       ("std", "negative")])
def test_brute_force_agrees(mode, rng_):
    rng = np.random.default_rng(hash((mode, rng_)) % 2**32)
    for shape, w_xy, w_z, g_xy, g_z in [((9, 11, 13), 5, 3, 3, 2), ((7, 6, 10), 7, 5, 4, 4),
                                        ((12, 5, 5), 3, 9, 2, 5), ((4, 9, 8), 1, 3, 1, 2),
                                        ((10, 10, 10), 31, 31, 16, 16)]:
        x = _rand_cube(rng, shape)
        sig, y = oracle.normalise(x, w_xy, w_z, g_xy, g_z, mode, rng_)
        sb, yb = brute.normalise(x, w_xy, w_z, g_xy, g_z, mode, rng_)
        assert sig.shape == sb.shape
        if mode == "mad":
            np.testing.assert_array_equal(sig, sb)
            np.testing.assert_array_equal(y, yb)
        else:   # summation order differs: FP64 rounding only
            np.testing.assert_allclose(sig, sb, rtol=1e-14)
            np.testing.assert_array_equal(np.isnan(y), np.isnan(yb))
            f = np.isfinite(y)
            np.testing.assert_allclose(y[f], yb[f], rtol=2 ** -23)


def test_whole_cube_window_is_the_global_noise():
    """A window and a block covering the whole cube reduce the normalisation
    to a division by the smooth-and-clip oracle's global noise."""
    rng = np.random.default_rng(3)
    x = _rand_cube(rng, (6, 8, 10))
    for mode, rng_ in [("mad", "negative"), ("std", "all")]:
        sig, y = oracle.normalise(x, 21, 13, 10, 6, mode, rng_)
        assert sig.shape == (1, 1, 1)
        s, _ = oracle.noise(np.where(np.isfinite(x), x, np.nan).astype(np.float64), mode, rng_)
        assert sig[0, 0, 0] == s
        with np.errstate(invalid="ignore"):
            np.testing.assert_array_equal(y, (x.astype(np.float64) / s).astype(np.float32))


def test_constant_magnitude_cube():
    """|v| = c everywhere (alternating signs): every window's MAD noise is
    1.4826 c and its RMS c, at every block, edges included."""
    c = np.float32(0.75)
    x = np.full((9, 10, 11), c, np.float32)
    x[:, :, 1::2] *= -1
    for mode, expect in [("mad", 1.4826 * 0.75), ("std", 0.75)]:
        sig, y = oracle.normalise(x, 5, 3, 3, 2, mode, "all")
        assert np.all(sig == expect), mode
        np.testing.assert_array_equal(y, (x.astype(np.float64) / expect).astype(np.float32))


def test_piecewise_sigma_field_exact_ratios():
    """Noise scaled by 8 on the right half of the field: every block whose
    window lies inside one half measures exactly that half's scale times the
    noise of the unscaled pattern, and normalises to the same values."""
    rng = np.random.default_rng(5)
    nz, ny, nx = 8, 12, 24
    pat = _rand_cube(rng, (nz, ny, nx), nan_frac=0.0)
    scale = np.where(np.arange(nx) < nx // 2, 1.0, 8.0).astype(np.float32)
    x = pat * scale[None, None, :]
    w, g = 5, 3
    for mode, rng_ in [("mad", "negative"), ("std", "all")]:
        s_pat, y_pat = oracle.normalise(pat, w, 3, g, 2, mode, rng_)
        s_x, y_x = oracle.normalise(x, w, 3, g, 2, mode, rng_)
        checked = 0
        for b in range(s_x.shape[2]):
            lo, hi = b * g, min(nx, (b + 1) * g) - 1
            c = lo + (hi - lo) // 2
            a, e = max(0, c - w // 2), min(nx - 1, c + w // 2)
            if e < nx // 2:
                k = 1.0
            elif a >= nx // 2:
                k = 8.0
            else:
                continue
            np.testing.assert_array_equal(s_x[:, :, b], k * s_pat[:, :, b])
            np.testing.assert_array_equal(y_x[:, :, lo:hi + 1], y_pat[:, :, lo:hi + 1])
            checked += 1
        assert checked >= 6


def test_power_of_two_scaling_and_sign_symmetry_exact():
    rng = np.random.default_rng(7)
    x = _rand_cube(rng, (10, 9, 14))
    s1, y1 = oracle.normalise(x, 5, 5, 3, 3, "mad", "negative")
    s4, y4 = oracle.normalise(x * np.float32(4), 5, 5, 3, 3, "mad", "negative")
    np.testing.assert_array_equal(s4, 4 * s1)
    np.testing.assert_array_equal(y4, y1)
    sp, yp = oracle.normalise(-x, 5, 5, 3, 3, "mad", "positive")
    np.testing.assert_array_equal(sp, s1)
    np.testing.assert_array_equal(yp, -y1)


def test_blanked_voxels_and_empty_windows():
    """Non-finite voxels stay NaN; a block whose window has no selected voxel
    (or zero noise) is blanked entirely."""
    x = np.ones((4, 6, 6), np.float32)        # no negative voxel at all
    x[0, 0, 0] = np.nan
    sig, y = oracle.normalise(x, 3, 3, 2, 2, "mad", "negative")
    assert np.all(np.isnan(sig)) and np.all(np.isnan(y))
    sig, y = oracle.normalise(x, 3, 3, 2, 2, "mad", "all")
    assert np.all(sig == 1.4826)
    assert np.isnan(y[0, 0, 0]) and np.isfinite(y).sum() == x.size - 1
    z = np.zeros((3, 4, 4), np.float32)       # zero noise: blanked
    sig, y = oracle.normalise(z, 3, 3, 2, 2, "std", "all")
    assert np.all(sig == 0.0) and np.all(np.isnan(y))
    # zero MAD noise with nonzero voxels in the block: blanked, not +-inf
    z[1, 1, 1] = 5.0
    z[0, 2, 3] = -2.0
    sig, y = oracle.normalise(z, 3, 3, 2, 2, "mad", "all")
    assert np.all(sig == 0.0) and np.all(np.isnan(y))


def test_bad_arguments():
    x = np.zeros((3, 3, 3), np.float32)
    for args in [(4, 3, 2, 2), (3, 2, 2, 2), (0, 3, 2, 2), (3, 3, 0, 2), (3, 3, 2, 0)]:
        with pytest.raises(ValueError):
            oracle.normalise(x, *args, "mad", "all")
