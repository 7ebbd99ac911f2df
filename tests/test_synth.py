"""The seeded input generator (CPU only)."""
import numpy as np
import pytest

import synth


def test_philox_known_answers():
    # Known-answer vectors published with Philox4x32-10 (Salmon et al. 2011).
    assert synth.philox4x32_10([0, 0, 0, 0], [0, 0]) == [
        0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]
    assert synth.philox4x32_10([0xFFFFFFFF] * 4, [0xFFFFFFFF, 0xFFFFFFFF]) == [
        0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]
    assert synth.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344],
                               [0xA4093822, 0x299F31D0]) == [
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]


def test_deterministic_and_slab_consistent():
    spec = synth.CubeSpec(33, 17, 40, seed=9, radial=True, sigma_lo=0.8,
                          sigma_hi=1.5, n_gal=4, nan_border=2)
    a = synth.generate(spec)
    b = synth.generate(spec)
    np.testing.assert_array_equal(a, b)
    slab = synth.generate(spec, z0=11, z1=29)
    np.testing.assert_array_equal(slab, a[11:29])


def test_noise_statistics_and_field():
    spec = synth.CubeSpec(64, 64, 64, seed=4)
    x = synth.generate(spec).astype(np.float64)
    assert abs(x.mean()) < 0.01
    assert abs(x.std() - 1.0) < 0.01
    spec = synth.CubeSpec(101, 101, 4, seed=4, radial=True, sigma_lo=0.8, sigma_hi=1.5)
    f = synth.sigma_field(spec)
    assert f[50, 50] == pytest.approx(0.8)
    assert f[0, 0] == pytest.approx(1.5) and f[100, 100] == pytest.approx(1.5)


def test_nan_border_fraction():
    spec = synth.CubeSpec(1024, 1024, 1, seed=2, nan_border=13)
    x = synth.generate(spec)
    frac = np.isnan(x).mean()
    assert frac == pytest.approx(1 - (998 / 1024) ** 2)
    assert abs(frac - 0.0501) < 1e-3


def test_galaxies_are_positive_blobs():
    base = synth.CubeSpec(48, 48, 64, seed=5, n_gal=0)
    gal = synth.CubeSpec(48, 48, 64, seed=5, n_gal=3)
    d = synth.generate(gal).astype(np.float64) - synth.generate(base)
    assert d.min() > -1e-5
    assert d.max() > 0.4
