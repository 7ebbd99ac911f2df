"""Pins of the parameterisation and reliability oracle (CPU only).

Eq. (4) and (5), the Gaussian-beam solid angle (Sect. 6.1.2) and the
reliability filter of Sect. 4.4 with readings P1-P7 (oracle/param.py),
checked against a hand-worked cube (tests/golden), a numerical integral of
the beam, explicit loops, and constructed parameter sets whose reliability
follows from the definition.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle

param = oracle.param_module()

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _hand():
    with open(os.path.join(GOLDEN, "param_hand.json")) as f:
        g = json.load(f)
    cube = np.array([[[np.nan if v == "nan" else v for v in row] for row in pl]
                     for pl in g["cube"]], dtype=np.float32)
    return g, cube, np.array(g["labels"], dtype=np.int32)


def test_hand_worked_parameters():
    g, cube, labels = _hand()
    p = param.parameterise(cube, labels, 3, g["channel_width"], (0, 0), g["sigma_rms"])
    for k, v in g["expect"].items():
        if k == "note":
            continue
        np.testing.assert_allclose(p[k], v, rtol=1e-15, atol=0, err_msg=k)


def test_beam_solid_angle_is_the_integral_of_the_beam():
    """Omega in pixels = the sum over pixels of a peak-1 Gaussian with the
    given FWHM (closed form pi a b / (4 ln 2))."""
    for a, b in [(5.0, 5.0), (3.0, 7.5), (10.0, 4.0)]:
        sx, sy = a / (2 * math.sqrt(2 * math.log(2))), b / (2 * math.sqrt(2 * math.log(2)))
        r = np.arange(-200, 201) / 4.0          # quarter-pixel grid
        X, Y = np.meshgrid(r, r)
        integral = np.exp(-0.5 * (X / sx) ** 2 - 0.5 * (Y / sy) ** 2).sum() / 16.0
        assert abs(param.beam_solid_angle(a, b) / integral - 1) < 1e-9
    assert param.beam_solid_angle(0, 0) == 1.0


def test_beam_enters_flux_and_uncertainty():
    g, cube, labels = _hand()
    p1 = param.parameterise(cube, labels, 3, 1.0, (0, 0), 1.0)
    om = param.beam_solid_angle(4.0, 6.0)
    p2 = param.parameterise(cube, labels, 3, 1.0, (4.0, 6.0), 1.0)
    np.testing.assert_allclose(p2["flux"], p1["flux"] / om, rtol=1e-15)
    np.testing.assert_allclose(p2["flux_err"], p1["flux_err"] / math.sqrt(om), rtol=1e-15)
    np.testing.assert_allclose(p2["snr"], p1["snr"] / math.sqrt(om), rtol=1e-14)


def _loop_params(cube, labels, n):
    out = {"count": [0] * n, "sum": [0.0] * n, "peak": [-np.inf] * n, "min": [np.inf] * n}
    nz, ny, nx = cube.shape
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                k = int(labels[z, y, x])
                v = float(cube[z, y, x])
                if k <= 0 or not math.isfinite(v):
                    continue
                out["count"][k - 1] += 1
                out["sum"][k - 1] += v
                out["peak"][k - 1] = max(out["peak"][k - 1], v)
                out["min"][k - 1] = min(out["min"][k - 1], v)
    return out


def test_sums_match_explicit_loops():
    rng = np.random.default_rng(3)
    cube = rng.standard_normal((6, 7, 8)).astype(np.float32)
    cube[rng.random(cube.shape) < 0.05] = np.nan
    labels = rng.integers(0, 6, size=cube.shape).astype(np.int32)
    p = param.parameterise(cube, labels, 5)
    ref = _loop_params(cube, labels, 5)
    np.testing.assert_array_equal(p["count"], ref["count"])
    np.testing.assert_allclose(p["sum"], ref["sum"], rtol=1e-13, atol=1e-13)
    np.testing.assert_array_equal(p["peak"], ref["peak"])
    np.testing.assert_array_equal(p["min"], ref["min"])


def _params(peak, s, mean, mn):
    n = len(s)
    return {"peak": np.array(peak, float), "sum": np.array(s, float), "mean": np.array(mean, float),
            "min": np.array(mn, float), "count": np.ones(n), "snr": np.ones(n)}


def _vec(rng, n):
    peak = 10 ** rng.uniform(0.5, 1.0, n)
    s = 10 ** rng.uniform(1.0, 2.0, n)
    mean = 10 ** rng.uniform(-0.5, 0.5, n)
    return peak, s, mean


def test_mirrored_populations_have_zero_reliability():
    """Positives that mirror the negatives exactly: the two densities are equal
    at every positive detection, so R = 0."""
    rng = np.random.default_rng(5)
    pk, s, m = _vec(rng, 12)
    p = _params(list(pk) + [0.1] * 12, list(s) + list(-s), list(m) + list(-m),
                [0.01] * 12 + list(-pk))
    R = param.reliability(p, 0.4)
    np.testing.assert_allclose(R[:12], 0.0, atol=1e-12)
    assert np.all(R[12:] == 0.0)


def test_isolated_positive_is_reliable_and_brute_force_agrees():
    rng = np.random.default_rng(6)
    pk, s, m = _vec(rng, 20)
    # 20 negatives, 5 positives among them, 1 positive far away in parameter space
    ppk, ps, pm = _vec(rng, 5)
    p = _params(list(ppk) + [1e4] + [0.1] * 20, list(ps) + [1e6] + list(-s),
                list(pm) + [1e3] + list(-m), [0.01] * 6 + list(-pk))
    R = param.reliability(p, 0.4)
    assert R[5] == 1.0
    # brute force: explicit loops, a solve instead of an inverse
    vp = np.log10(np.stack([p["peak"][:6], p["sum"][:6], p["mean"][:6]], 1))
    vn = np.log10(np.stack([-p["min"][6:], -p["sum"][6:], -p["mean"][6:]], 1))
    mu = vn.mean(0)
    C = sum(np.outer(v - mu, v - mu) for v in vn) / (len(vn) - 1) * 0.16
    for i in range(6):
        P = sum(math.exp(-0.5 * float((vp[i] - q) @ np.linalg.solve(C, vp[i] - q))) for q in vp)
        N = sum(math.exp(-0.5 * float((vp[i] - q) @ np.linalg.solve(C, vp[i] - q))) for q in vn)
        assert abs(R[i] - max(0.0, (P - N) / P)) < 1e-12


def test_few_negatives_and_kept_flag():
    p = _params([5.0, 4.0, 0.1], [50.0, 40.0, -3.0], [2.0, 1.0, -1.0], [1.0, 1.0, -2.0])
    R = param.reliability(p, 0.4)
    np.testing.assert_array_equal(R, [1.0, 1.0, 0.0])
    g, cube, labels = _hand()
    c = param.catalogue(cube, labels, 3, 1.0, (0, 0), 1.0, 0.4, 0.9, 2.8)
    # positives 1 and 3 (R = 1: one negative only); SNR 6/sqrt(3) = 3.46 and 0.5
    np.testing.assert_array_equal(c["kept"], [1, 0, 0])
    # the SNR threshold is inclusive
    c = param.catalogue(cube, labels, 3, 1.0, (0, 0), 1.0, 0.4, 0.9, float(c["snr"][0]))
    np.testing.assert_array_equal(c["kept"], [1, 0, 0])
    c = param.catalogue(cube, labels, 3, 1.0, (0, 0), 1.0, 0.4, 1.0, 0.5)
    np.testing.assert_array_equal(c["kept"], [1, 0, 1])


def test_reliability_is_zero_where_negatives_outnumber_positives():
    """A positive detection sitting on three negatives with its own parameter
    vector: P = 1 + (the others' share), N >= 3 at that point, so (P - N) / P
    < 0 and R is clipped to 0."""
    rng = np.random.default_rng(9)
    pk, s, m = _vec(rng, 10)
    peak = [pk[0]] + [0.1] * 13
    ssum = [s[0]] + [-s[0]] * 3 + list(-s)
    mean = [m[0]] + [-m[0]] * 3 + list(-m)
    mn = [0.01] + [-pk[0]] * 3 + list(-pk)
    R = param.reliability(_params(peak, ssum, mean, mn), 0.4)
    assert R[0] == 0.0


def test_voxel_subset_and_sampled_reliability_agree_with_the_whole():
    """parameterise_voxels over the labelled voxels of a cube gives what
    parameterise gives over the whole cube; reliability at sampled detections
    equals the whole-catalogue reliability there."""
    rng = np.random.default_rng(11)
    cube = rng.normal(size=(9, 10, 11)).astype(np.float32)
    cube[0, 0, :3] = np.nan
    labels = rng.integers(0, 25, size=cube.shape).astype(np.int32)
    labels[rng.random(cube.shape) < 0.5] = 0
    whole = param.parameterise(cube, labels, 20)
    idx = np.flatnonzero(labels)
    sub = param.parameterise_voxels(idx, cube.ravel()[idx], labels.ravel()[idx], cube.shape, 20)
    for k in whole:
        np.testing.assert_array_equal(sub[k], whole[k], err_msg=k)
    R = param.reliability(whole, 0.4)
    at = [0, 3, 7, 19]
    Ra = param.reliability(whole, 0.4, at)
    np.testing.assert_array_equal(Ra[at], R[at])
    assert np.isnan(np.delete(Ra, at)).all()
