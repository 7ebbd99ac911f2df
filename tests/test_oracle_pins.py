"""Pins of the FP64 oracle against what the mathematics fixes (CPU only).

Each test checks the oracle against something other than itself: hand-worked
values (tests/golden), closed forms, reductions to library routines, exact
floating-point invariants, or the independent dense-matrix brute force.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _json(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- plan (R1)

@pytest.mark.parametrize("fwhm,expect", [(3, (3, 1)), (5, (6, 1)), (6, (3, 2)),
                                         (9, (4, 3)), (10, (5, 3)), (0, (0, 0))])
def test_plan_table(fwhm, expect):
    assert oracle.plan(fwhm) == expect


def test_plan_matches_exhaustive_search():
    for f in np.linspace(0.25, 14.0, 56):
        assert oracle.plan(float(f)) == brute.plan(float(f)), f


def test_plan_rejects_bad_fwhm():
    for f in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError):
            oracle.plan(f)


# ------------------------------------------------------- smoothing closed forms

def test_spectral_boxcar_of_delta_interior_and_edge():
    nz = 20
    for w in (3, 5, 7, 15):
        for z0 in (0, 1, nz // 2, nz - 1):
            x = np.zeros((nz, 1, 1), np.float32)
            x[z0] = 1.0
            s = oracle.smooth(x, 0.0, w)[:, 0, 0]
            h = (w - 1) // 2
            expect = np.zeros(nz)
            expect[max(0, z0 - h):min(nz, z0 + h + 1)] = 1.0 / w
            np.testing.assert_allclose(s, expect, rtol=0, atol=1e-15)


def test_spectral_identity_widths():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((9, 4, 5)).astype(np.float32)
    for w in (0, 1):
        np.testing.assert_array_equal(oracle.smooth(x, 0.0, w), x.astype(np.float64))


def test_even_width_rejected():
    x = np.zeros((5, 5, 5), np.float32)
    with pytest.raises(ValueError):
        oracle.smooth(x, 0.0, 4)


def test_cascade_of_delta_matches_hand_taps():
    for case in _json("cascade_taps.json")["cases"]:
        n_it, r = oracle.plan(case["fwhm"])
        assert (n_it, r) == (case["n_iter"], case["r"])
        L = len(case["taps"])
        nx = L + 20
        x = np.zeros((1, nx, nx), np.float32)
        c = nx // 2
        x[0, c, c] = 1.0
        s = oracle.smooth(x, case["fwhm"], 0)[0]
        h1 = np.asarray(case["taps"], np.float64) / case["denominator"]
        lo = c - (L - 1) // 2
        expect = np.zeros((nx, nx))
        expect[lo:lo + L, lo:lo + L] = np.outer(h1, h1)
        np.testing.assert_allclose(s, expect, rtol=1e-13, atol=1e-16)
        # sum 1, variance n r (r+1)/3, support 2nr+1, symmetric
        k = np.arange(L) - (L - 1) // 2
        assert math.isclose(h1.sum(), 1.0, rel_tol=1e-15)
        assert math.isclose((h1 * k * k).sum(), n_it * r * (r + 1) / 3.0, rel_tol=1e-13)
        assert L == 2 * n_it * r + 1
        np.testing.assert_array_equal(h1, h1[::-1])
        assert math.isclose((h1 ** 2).sum(), case["sum_sq_num"] / case["sum_sq_den"],
                            rel_tol=1e-13)


@pytest.mark.parametrize("fwhm", [3, 5, 6, 9, 10])
def test_cascade_interior_is_nfold_uniform(fwhm):
    n_it, r = oracle.plan(fwhm)
    h = np.ones(1)
    for _ in range(n_it):
        h = np.convolve(h, np.ones(2 * r + 1) / (2 * r + 1))
    nx = len(h) + 10
    # the row through the impulse is h(x) times the centre tap of h(y)
    x = np.zeros((1, len(h) + 2, nx), np.float32)
    cy, cx = (len(h) + 2) // 2, nx // 2
    x[0, cy, cx] = 1.0
    s = oracle.smooth(x, fwhm, 0)[0]
    row = s[cy]
    lo = cx - (len(h) - 1) // 2
    expect = np.zeros(nx)
    expect[lo:lo + len(h)] = h * h[(len(h) - 1) // 2]
    np.testing.assert_allclose(row, expect, rtol=1e-12, atol=1e-18)


def test_cascade_edge_rezeroes_each_pass():
    """At the edge each pass drops the mass that falls outside (R2)."""
    nx = 12
    x = np.zeros((1, 1, nx), np.float32)
    x[0, 0, 0] = 1.0
    s = oracle.smooth(x, 3.0, 0)[0, 0]
    # y axis of length 1: each y pass keeps 1/3 of the value (truncated window)
    n_it, r = oracle.plan(3.0)
    b = np.zeros(nx)
    b[0] = 1.0
    for _ in range(n_it):   # x passes with truncation
        b = np.array([b[max(0, i - r):i + r + 1].sum() / (2 * r + 1) for i in range(nx)])
    b *= (1.0 / (2 * r + 1)) ** n_it
    np.testing.assert_allclose(s, b, rtol=1e-13, atol=1e-18)
    # a single composite convolution with zero padding would keep more mass
    assert s.sum() < (1.0 / 3) ** n_it


def test_smoothed_noise_variance_scaling():
    """For i.i.d. N(0,1) input, interior sigma_k = sqrt(sum hx^2 sum hy^2 sum hz^2)."""
    spec = synth.CubeSpec(160, 160, 96, seed=11)
    x = synth.generate(spec)
    for fwhm, w in [(0, 7), (3, 0), (6, 3), (9, 15)]:
        n_it, r = oracle.plan(fwhm)
        h = np.ones(1)
        for _ in range(n_it):
            h = np.convolve(h, np.ones(2 * r + 1) / (2 * r + 1))
        sh2 = (h ** 2).sum()
        hz2 = 1.0 / w if w >= 3 else 1.0
        expect = math.sqrt(sh2 * sh2 * hz2)
        s = oracle.smooth(x, fwhm, w)
        m = n_it * r + 1
        mz = (w - 1) // 2 + 1 if w >= 3 else 0
        core = s[mz:x.shape[0] - mz, m:x.shape[1] - m, m:x.shape[2] - m]
        got = float(np.sqrt(np.mean(core ** 2)))
        assert abs(got / expect - 1) < 0.03, (fwhm, w, got, expect)


# --------------------------------------------------------------------- noise

def test_noise_hand_multiset():
    g = _json("noise_multiset.json")
    v = np.array([float(a) for a in g["values"]])
    for key, exp in g["expected"].items():
        mode, rng = key.split("_")
        sigma, m = oracle.noise(v, mode, rng)
        assert math.isclose(sigma, exp["sigma"], rel_tol=1e-14), key
        if mode == "mad":
            assert m == len(exp["sorted_abs"])
            assert math.isclose(sigma, 1.4826 * exp["median"], rel_tol=1e-15)
        else:
            assert m == exp["count"]
            assert math.isclose(sigma, math.sqrt(exp["sum_sq"] / exp["count"]),
                                rel_tol=1e-14)


def test_noise_empty_selection_is_enostat():
    sigma, m = oracle.noise(np.array([1.0, 2.0, np.nan]), "mad", "negative")
    assert m == 0 and math.isnan(sigma)


def test_mad_of_gaussian_sample():
    rng = np.random.default_rng(5)
    v = rng.standard_normal(2_000_001) * 2.5
    for r in ("negative", "all", "positive"):
        sigma, _ = oracle.noise(v, "mad", r)
        # E = 2.5 * 1.4826 * Phi^-1(3/4); sampling error of the median ~ 1e-3
        assert abs(sigma / (2.5 * 1.4826 * 0.6744897501960817) - 1) < 4e-3, r


def test_mad_matches_numpy_median():
    rng = np.random.default_rng(6)
    for n in (1, 2, 3, 10, 11, 1000, 1001):
        v = rng.standard_normal(n)
        v[rng.random(n) < 0.1] = np.nan
        for r in ("negative", "all", "positive"):
            sel = v[np.isfinite(v)]
            sel = sel[sel < 0] if r == "negative" else sel[sel > 0] if r == "positive" else sel
            sigma, m = oracle.noise(v, "mad", r)
            assert m == sel.size
            if sel.size:
                assert sigma == pytest.approx(1.4826 * np.median(np.abs(sel)), rel=1e-15)


def test_std_matches_numpy_rms():
    rng = np.random.default_rng(7)
    v = rng.standard_normal(100_003) * 3
    for r, sel in (("negative", v[v < 0]), ("all", v), ("positive", v[v > 0])):
        sigma, _ = oracle.noise(v, "std", r)
        assert sigma == pytest.approx(np.sqrt(np.mean(sel ** 2)), rel=1e-12)


# ------------------------------------------------------- whole-run reductions

def test_single_unsmoothed_kernel_is_threshold_finder():
    """K = 1, kernel (0, 0): S+C reduces to |x| > t sigma (Sect. 4.2)."""
    spec = synth.CubeSpec(40, 36, 30, seed=3, n_gal=2)
    x = synth.generate(spec)
    x[3] = np.nan
    fin = np.isfinite(x)
    for mode in ("std", "mad"):
        for r in ("negative", "all", "positive"):
            res = oracle.run(x, [(0.0, 0)], 3.0, mode, r, repl=2.0)
            v = x[fin].astype(np.float64)
            v = v[v < 0] if r == "negative" else v[v > 0] if r == "positive" else v
            sig = (np.sqrt(np.mean(v ** 2)) if mode == "std"
                   else 1.4826 * np.median(np.abs(v)))
            assert res.sigma[0] == pytest.approx(sig, rel=1e-12)
            with np.errstate(invalid="ignore"):
                expect = (fin & (np.abs(x.astype(np.float64)) > 3.0 * sig)).astype(np.uint8)
            np.testing.assert_array_equal(res.mask, expect)
            assert res.sigma0 == pytest.approx(sig, rel=1e-12)


def _random_case(rng, shape):
    x = rng.standard_normal(shape).astype(np.float32)
    x += (rng.random(shape) < 0.02) * 6.0 * np.sign(rng.standard_normal(shape)).astype(np.float32)
    if rng.random() < 0.5:
        x[rng.random(shape) < 0.1] = np.nan
    return x


def test_brute_force_agrees_with_oracle():
    rng = np.random.default_rng(12)
    kernels_pool = [(0.0, 0), (0.0, 3), (0.0, 5), (3.0, 0), (3.0, 3), (5.0, 1),
                    (6.0, 7), (1.0, 3)]
    n_cases = 0
    for trial in range(40):
        shape = tuple(int(v) for v in rng.integers(1, 13, size=3))
        if np.prod(shape) > 1500:
            continue
        x = _random_case(rng, shape)
        K = int(rng.integers(1, 4))
        kernels = [kernels_pool[i] for i in rng.choice(len(kernels_pool), K)]
        mode = ["std", "mad"][trial % 2]
        r = ["negative", "all", "positive"][trial % 3]
        repl = [2.0, -1.0, 1.5, 0.0][trial % 4]
        t = float(rng.uniform(1.0, 3.0))
        res = oracle.run(x, kernels, t, mode, r, repl=repl)
        bm, bs, b0 = brute.run(x, kernels, t, mode, r, repl=repl)
        if res.status != 0:
            assert np.isnan(bs).any() or np.isnan(b0)
            continue
        np.testing.assert_allclose(res.sigma, bs, rtol=1e-12)
        if repl >= 0:
            assert res.sigma0 == pytest.approx(b0, rel=1e-12)
        # identical masks unless a voxel sits on the threshold to ~1e-12
        diff = res.mask != bm
        assert diff.sum() == 0, (trial, shape, kernels, mode, r, repl)
        n_cases += 1
    assert n_cases >= 20


def test_brute_force_smoothing_values():
    rng = np.random.default_rng(13)
    for shape in [(1, 1, 1), (3, 1, 7), (5, 6, 4), (9, 8, 10), (2, 13, 3)]:
        x = _random_case(rng, shape)
        mask = (rng.random(shape) < 0.2).astype(np.uint8)
        for f, w in [(0.0, 3), (3.0, 0), (6.0, 5), (5.0, 7)]:
            a = oracle.smooth(x, f, w, mask, 2.0, 0.7)
            b = brute.smooth(x, f, w, mask, 2.0, 0.7)
            np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_replacement_keeps_sign_and_uses_sigma0():
    """Sect. 6.2.4: detected voxels become +-n sigma_0 before smoothing."""
    x = np.zeros((7, 1, 1), np.float32)
    x[2, 0, 0] = 9.0
    x[4, 0, 0] = -8.0
    mask = np.zeros(x.shape, np.uint8)
    mask[2] = mask[4] = 1
    s = oracle.smooth(x, 0.0, 1, mask, 2.0, 0.5)[:, 0, 0]
    np.testing.assert_array_equal(s, [0, 0, 1.0, 0, -1.0, 0, 0])
    s = oracle.smooth(x, 0.0, 3, mask, 2.0, 0.5)[:, 0, 0]
    np.testing.assert_allclose(s, [0, 1 / 3, 1 / 3, 0, -1 / 3, -1 / 3, 0], rtol=1e-15)
    # replacement off: raw values are smoothed
    s = oracle.smooth(x, 0.0, 1, mask, -1.0, 0.5)[:, 0, 0]
    np.testing.assert_array_equal(s, x[:, 0, 0].astype(np.float64))


def test_blanked_voxels_are_zero_in_smoothing_and_never_detected():
    x = np.ones((3, 3, 3), np.float32) * 5
    x[1, 1, 1] = np.nan
    s = oracle.smooth(x, 0.0, 3)
    assert np.isnan(s[1, 1, 1])
    # z = 0 at the cube edge: window {outside, 5, blank} -> 5 / 3
    assert s[0, 1, 1] == pytest.approx(5 / 3, rel=1e-15)
    assert s[2, 1, 1] == pytest.approx(5 / 3, rel=1e-15)
    assert s[1, 0, 0] == pytest.approx(5.0, rel=1e-15)
    res = oracle.run(x, [(0.0, 3)], 0.5, "std", "all", repl=-1)
    assert res.mask[1, 1, 1] == 0


# ---------------------------------------------------------------- invariants

def _cfg_like(seed, shape=(48, 40, 36)):
    nz, ny, nx = shape
    x = synth.generate(synth.CubeSpec(nx, ny, nz, seed=seed, radial=True,
                                      sigma_lo=0.8, sigma_hi=1.5, n_gal=3,
                                      nan_border=2))
    return x


KERNELS = [(0.0, 0), (0.0, 3), (3.0, 0), (3.0, 7), (6.0, 3)]


def test_sign_symmetry_exact():
    x = _cfg_like(21)
    a = oracle.run(x, KERNELS, 3.5, "mad", "negative")
    b = oracle.run(-x, KERNELS, 3.5, "mad", "positive")
    np.testing.assert_array_equal(a.mask, b.mask)
    np.testing.assert_array_equal(a.sigma, b.sigma)
    c = oracle.run(x, KERNELS, 3.5, "std", "all")
    d = oracle.run(-x, KERNELS, 3.5, "std", "all")
    np.testing.assert_array_equal(c.mask, d.mask)
    np.testing.assert_array_equal(c.sigma, d.sigma)


def test_power_of_two_scaling_exact():
    x = _cfg_like(22)
    a = oracle.run(x, KERNELS, 3.5, "mad", "negative")
    b = oracle.run(x * np.float32(8.0), KERNELS, 3.5, "mad", "negative")
    np.testing.assert_array_equal(a.mask, b.mask)
    np.testing.assert_array_equal(a.sigma * 8.0, b.sigma)


def test_threshold_monotone_without_replacement():
    x = _cfg_like(23)
    lo = oracle.run(x, KERNELS, 3.0, "std", "all", repl=-1)
    hi = oracle.run(x, KERNELS, 3.6, "std", "all", repl=-1)
    assert np.all(hi.mask <= lo.mask)
    np.testing.assert_array_equal(lo.sigma, hi.sigma)


def test_mask_union_and_steps_compose():
    """run() equals chaining step() with the running union."""
    x = _cfg_like(24, (30, 26, 22))
    full = oracle.run(x, KERNELS, 3.5, "mad", "negative")
    mask = np.zeros(x.shape, np.uint8)
    for k, (f, w) in enumerate(KERNELS):
        st = oracle.step(x, f, w, 3.5, "mad", "negative", mask, 2.0, full.sigma0)
        assert st.sigma == full.sigma[k]
        assert np.all(st.mask >= mask)
        mask = st.mask
    np.testing.assert_array_equal(mask, full.mask)


def test_clip_is_strict_at_exact_threshold():
    """|s| equal to t sigma is not detected (R10: 'in excess of', Sect. 4.2)."""
    x = np.full((4, 3, 5), 2.0, np.float32)
    x[::2] *= -1
    res = oracle.run(x, [(0.0, 0)], 1.0, "std", "all", repl=-1)
    assert res.sigma[0] == 2.0
    assert res.mask.sum() == 0
    res = oracle.run(x, [(0.0, 0)], 0.999, "std", "all", repl=-1)
    assert res.mask.sum() == x.size


@pytest.mark.parametrize("t", [3.5, 4.0])
@pytest.mark.parametrize("m", [1.0, 64.0])
def test_boundary_band_width_and_units(t, m):
    """The boundary band is the set of finite voxels with | |s|/sigma_k - t |
    <= 1e-5, i.e. within 1e-5 sigma_k of the threshold (the tolerance rule
    for mask parity; detection is strict, Sect. 4.2).

    Hand-built cube: every voxel is +-m (m a power of two) except a few test
    voxels at |s| = sigma (t + d) for fixed offsets d, so the MAD over all
    voxels is exactly 1.4826 m (the median of |s| is m). Each test voxel is a
    float32, within 1.6e-7 sigma of its nominal offset; the offsets keep at
    least 2e-6 sigma from the band edge, so their membership is fixed:
    |d| in {0.5e-5, 0.8e-5} inside, |d| in {1.3e-5, 2e-5} outside. m = 64
    puts sigma far from 1, so a band measured in absolute units instead of
    units of sigma_k fails too."""
    nz, ny, nx = 4, 16, 32
    x = np.full((nz, ny, nx), m, np.float32)
    x[:, :, 1::2] *= -1.0
    sigma = 1.4826 * m
    offsets = {0.5e-5: True, -0.5e-5: True, 0.8e-5: True, -0.8e-5: True,
               1.3e-5: False, -1.3e-5: False, 2e-5: False, -2e-5: False}
    spots = {}
    for i, (d, inside) in enumerate(offsets.items()):
        z, y, xx = i % nz, 3 + i, 5 + 2 * i
        sign = -1.0 if i % 3 == 0 else 1.0
        x[z, y, xx] = np.float32(sign * sigma * (t + d))
        spots[(z, y, xx)] = (d, inside)
    x[1, 0, 0] = np.nan          # blanked: never in the band, never detected
    res = oracle.run(x, [(0.0, 0)], t, "mad", "all", repl=-1)
    assert res.sigma[0] == sigma
    band = res.band.astype(bool)
    for (z, y, xx), (d, inside) in spots.items():
        assert band[z, y, xx] == inside, (d, t, m)
        assert res.mask[z, y, xx] == (1 if d > 0 else 0), (d, t, m)
    assert int(band.sum()) == sum(offsets.values())
    assert res.band_count[0] == int(band.sum())
    assert not band[1, 0, 0] and res.mask[1, 0, 0] == 0
    # the same classification through a single step
    st = oracle.step(x, 0.0, 0, t, "mad", "all")
    np.testing.assert_array_equal(st.band, res.band)
    assert st.band_count == res.band_count[0]


def test_noise_plane_subsampling_and_given_noise():
    """Noise subsampling (every s-th plane) equals the noise of the sub-array
    of those planes of the oracle's own smoothed cube; the clip covers every
    voxel. A given noise skips the measurement: the clip of step g with it.
    Stride 1 is the plain step."""
    x = _cfg_like(11)
    prev = oracle.step(x, 0.0, 0, 3.5, "mad", "negative").mask
    for f, w, stride in [(0.0, 0, 4), (3.0, 7, 3), (6.0, 3, 5)]:
        s = oracle.smooth(x, f, w, prev, 2.0, 0.9)
        sub, _ = oracle.noise(s[::stride], "mad", "negative")
        st = oracle.step(x, f, w, 3.5, "mad", "negative", prev, 2.0, 0.9, plane_stride=stride)
        assert st.sigma == sub
        fin = np.isfinite(s)
        with np.errstate(invalid="ignore"):
            expect = prev | (fin & (np.abs(s) > 3.5 * sub)).astype(np.uint8)
        np.testing.assert_array_equal(st.mask, expect)
        full = oracle.step(x, f, w, 3.5, "mad", "negative", prev, 2.0, 0.9)
        one = oracle.step(x, f, w, 3.5, "mad", "negative", prev, 2.0, 0.9, plane_stride=1)
        np.testing.assert_array_equal(one.mask, full.mask)
        assert one.sigma == full.sigma
        given = oracle.step(x, f, w, 3.5, "mad", "negative", prev, 2.0, 0.9,
                            sigma_given=full.sigma)
        np.testing.assert_array_equal(given.mask, full.mask)
        np.testing.assert_array_equal(given.band, full.band)
        assert given.sigma == full.sigma


def test_given_noise_clip_is_strict_and_banded():
    """With the noise given, the clip is still strict (|s| > t sigma_k) and the
    band still measured in units of that noise."""
    x = np.full((4, 3, 5), 2.0, np.float32)
    x[::2] *= -1
    st = oracle.step(x, 0.0, 0, 1.0, "std", "all", sigma_given=2.0)
    assert st.sigma == 2.0 and st.mask.sum() == 0 and st.band_count == x.size
    st = oracle.step(x, 0.0, 0, 0.999, "std", "all", sigma_given=2.0)
    assert st.mask.sum() == x.size and st.band_count == 0
    st = oracle.step(x * np.float32(64), 0.0, 0, 1.0 + 0.8e-5, "std", "all", sigma_given=128.0)
    assert st.band_count == x.size and st.mask.sum() == 0
    st = oracle.step(x * np.float32(64), 0.0, 0, 1.0 + 2e-5, "std", "all", sigma_given=128.0)
    assert st.band_count == 0


# ------------------------------------------ sampled Gaussian (reading G1)

def _sigma_g(fwhm):
    return fwhm / (2.0 * np.sqrt(2.0 * np.log(2.0)))


@pytest.mark.parametrize("fwhm", [0.6, 1.0, 3.0, 4.7, 5.0, 6.0, 9.0, 10.0, 13.3])
def test_gauss_taps_match_scipy_impulse_and_closed_forms(fwhm):
    """The taps are scipy.ndimage.gaussian_filter1d's response to a delta
    (truncate = 4: radius floor(4 sigma + 1/2), normalised, zero outside);
    they sum to 1, are symmetric, and their sum of squares and variance are
    those of the continuous Gaussian up to sampling and truncation."""
    from scipy.ndimage import gaussian_filter1d
    h = oracle.gauss_taps(fwhm)
    s = _sigma_g(fwhm)
    R = int(np.floor(4.0 * s + 0.5))
    assert h.size == 2 * R + 1
    d = np.zeros(2 * R + 41)
    d[R + 20] = 1.0
    ref = gaussian_filter1d(d, s, mode="constant", cval=0.0, truncate=4.0)
    np.testing.assert_allclose(h, ref[20:20 + 2 * R + 1], rtol=0, atol=1e-15)
    assert abs(h.sum() - 1.0) < 1e-14
    np.testing.assert_array_equal(h, h[::-1])
    if s >= 1.0:
        k = np.arange(-R, R + 1)
        assert abs((h * h).sum() * 2.0 * np.sqrt(np.pi) * s - 1.0) < 1e-3
        assert abs((k * k * h).sum() / (s * s) - 1.0) < 2e-3


def test_gauss_identity_for_zero_and_tiny_fwhm():
    x = np.random.default_rng(3).normal(size=(4, 9, 11)).astype(np.float32)
    for f in (0.0, 0.2):
        np.testing.assert_array_equal(oracle.gauss_taps(f), [1.0])
        np.testing.assert_array_equal(oracle.smooth(x, f, 0, kind=1), x.astype(np.float64))
    with pytest.raises(ValueError):
        oracle.gauss_taps(-1.0)


@pytest.mark.parametrize("fwhm,width", [(3.0, 0), (6.0, 7), (10.0, 3)])
def test_gauss_smoothing_matches_scipy_per_plane(fwhm, width):
    """Spatial part: scipy.ndimage.gaussian_filter over each plane (both axes,
    zero outside) of the blanked cube; spectral part: the plain boxcar; NaN
    restored at blanked voxels."""
    from scipy.ndimage import gaussian_filter, uniform_filter1d
    rng = np.random.default_rng(7)
    x = rng.normal(size=(12, 45, 38)).astype(np.float32)
    x[3, 10, 5:9] = np.nan
    x[:, 0, 0] = np.inf
    s = _sigma_g(fwhm)
    b = np.where(np.isfinite(x), x, 0.0).astype(np.float64)
    ref = np.stack([gaussian_filter(p, s, mode="constant", cval=0.0, truncate=4.0) for p in b])
    if width >= 3:
        ref = uniform_filter1d(ref, width, axis=0, mode="constant", cval=0.0)
    ref[~np.isfinite(x)] = np.nan
    g = oracle.smooth(x, fwhm, width, kind=1)
    np.testing.assert_allclose(g, ref, rtol=0, atol=1e-13, equal_nan=True)


def test_gauss_kind_in_steps_and_runs():
    """Kernel kinds mix in one run; the run equals the chained steps with the
    same kinds, and a Gaussian kernel differs from the cascade one."""
    rng = np.random.default_rng(8)
    x = rng.normal(size=(20, 30, 33)).astype(np.float32)
    kernels = [(0.0, 0), (3.0, 0, 1), (6.0, 3, 1), (6.0, 3, 0)]
    r = oracle.run(x, kernels, 3.0, "mad", "negative", 2.0)
    m = None
    for k, kern in enumerate(kernels):
        st = oracle.step(x, kern[0], kern[1], 3.0, "mad", "negative", m, 2.0, r.sigma0,
                         kind=kern[2] if len(kern) > 2 else 0)
        assert st.sigma == r.sigma[k]
        m = st.mask
    np.testing.assert_array_equal(m, r.mask)
    assert r.sigma[2] != r.sigma[3]
