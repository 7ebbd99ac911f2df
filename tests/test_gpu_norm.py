"""GPU parity of the local noise normalisation (Sect. 4.1) against the FP64
oracle, through the C ABI (sofia_sc_normalise).

With MAD noise both sides select the same order statistics of the same
float32 values and compute sigma = 1.4826 x median in FP64 the same way, and
both divide in FP64 and round to float32 once: the noise grid and the
normalised cube must be equal bit for bit. With RMS noise the FP64 sums run
in another order: the grid to 1e-12 relative, the cube to 1 ulp.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def _cube(shape, seed, nan_frac=0.01, field=True):
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(shape).astype(np.float32)
    if field:    # noise level varying across the field and along z
        fx = 0.8 + 0.7 * (np.arange(nx) / max(1, nx - 1)) ** 2
        fz = 1.0 + 0.3 * np.sin(np.arange(nz) / 7.0)
        x *= (fz[:, None, None] * fx[None, None, :]).astype(np.float32)
    x[rng.random(shape) < nan_frac] = np.nan
    return x


def check(h, x, wxy, wz, gxy, gz, mode, rng_, what=""):
    sig_ref, y_ref = oracle.normalise(x, wxy, wz, gxy or (wxy + 1) // 2,
                                      gz or (wz + 1) // 2, mode, rng_)
    y, sig = h.normalise(torch.from_numpy(x).cuda(), wxy, wz, gxy, gz, mode, rng_)
    y = y.cpu().numpy()
    assert sig.shape == sig_ref.shape, what
    np.testing.assert_array_equal(np.isnan(sig), np.isnan(sig_ref), err_msg=what)
    np.testing.assert_array_equal(np.isnan(y), np.isnan(y_ref), err_msg=what)
    if mode == "mad":
        np.testing.assert_array_equal(sig, sig_ref, err_msg=what)
        np.testing.assert_array_equal(y, y_ref, err_msg=what)
    else:
        f = np.isfinite(sig_ref)
        np.testing.assert_allclose(sig[f], sig_ref[f], rtol=1e-12, err_msg=what)
        f = np.isfinite(y_ref)
        np.testing.assert_allclose(y[f], y_ref[f], rtol=2 ** -23, atol=0, err_msg=what)
    return sig


CASES = [
    # shape, window xy, window z, grid xy, grid z
    ((40, 50, 60), 31, 31, 0, 0),
    ((70, 33, 45), 7, 15, 3, 5),
    ((9, 64, 65), 15, 3, 8, 2),
    ((31, 40, 97), 33, 7, 16, 4),     # rows wider than 32 voxels
    ((5, 3, 2), 31, 31, 16, 16),      # window larger than the cube
    ((12, 1, 130), 5, 1, 2, 1),       # window 1 along z, single row
    ((1, 1, 1), 1, 1, 1, 1),
    ((20, 20, 20), 1, 1, 1, 1),       # one-voxel windows
    ((17, 29, 31), 9, 9, 0, 0),
]


@pytest.mark.parametrize("mode,rng_", [("mad", "negative"), ("mad", "all"),
                                       ("mad", "positive"), ("std", "all"),
                                       ("std", "negative")])
@pytest.mark.parametrize("case", CASES, ids=[str(c) for c in CASES])
def test_normalise_matches_oracle(h, case, mode, rng_):
    shape, wxy, wz, gxy, gz = case
    x = _cube(shape, seed=sum(shape) + wxy)
    check(h, x, wxy, wz, gxy, gz, mode, rng_, f"{case} {mode} {rng_}")


@pytest.mark.parametrize("mode,rng_", [("mad", "negative"), ("mad", "all"), ("std", "all")])
def test_normalise_large_windows_and_crowded_bins(h, mode, rng_):
    """Windows of ~1.2e5 voxels, more keys in the median's top-level bin
    than the kernel stages in LDS (it streams the window again for the lower
    levels), and values from a few levels only (long runs of equal keys
    around the median)."""
    x = _cube((40, 70, 70), seed=5)
    check(h, x, 63, 31, 32, 16, mode, rng_, "63 x 63 x 31 windows")
    rng = np.random.default_rng(6)
    q = (rng.integers(-4, 5, size=(30, 40, 50)) * 0.25).astype(np.float32)
    q[rng.random(q.shape) < 0.01] = np.nan
    check(h, q, 31, 31, 16, 16, mode, rng_, "quantised values")


def test_normalise_config2_recipe_in_place_and_grid_only(h):
    """A cube of the 1024^3 recipe (sigma 0.8-1.5 across the field, NaN
    border) at 1/64 volume: the paper's 31 px / 31 ch window; in place, and
    the grid alone."""
    wl = synth.workload("plain_256cube")
    x = synth.generate(wl.cubes[0])
    sig_ref, y_ref = oracle.normalise(x, 31, 31, 16, 16, "mad", "negative")
    xd = torch.from_numpy(x).cuda()
    y, sig = h.normalise(xd, 31, 31, 0, 0, "mad", "negative", out=xd)   # in place
    np.testing.assert_array_equal(sig, sig_ref)
    np.testing.assert_array_equal(xd.cpu().numpy(), y_ref)
    _, sig2 = h.normalise(torch.from_numpy(x).cuda(), 31, 31, 16, 16, "mad", "negative",
                          out=False)
    np.testing.assert_array_equal(sig2, sig_ref)
    fin = np.isfinite(sig_ref)
    say(f"256^3 recipe: noise grid {sig_ref.shape}, sigma {sig_ref[fin].min():.3f}.."
        f"{sig_ref[fin].max():.3f}, blanked blocks {int((~fin).sum())}")


def test_blanked_blocks(h):
    """Blocks whose window has no voxel in the range, or zero noise, are NaN."""
    x = np.abs(_cube((16, 16, 16), seed=5, nan_frac=0.0)) + np.float32(0.1)
    x[:8] *= -1                        # negative voxels only in the first planes
    sig = check(h, x, 5, 5, 4, 4, "mad", "negative", "negative half")
    assert np.isnan(sig).any() and np.isfinite(sig).any()
    z = np.zeros((8, 8, 8), np.float32)
    z[3, 3, 3] = 2.0
    check(h, z, 3, 3, 2, 2, "mad", "all", "zero noise")


def test_bad_arguments(h):
    xd = torch.zeros((8, 8, 8), device="cuda")
    for args in [(4, 3, 0, 0), (3, 4, 0, 0), (0, 3, 0, 0), (257, 3, 0, 0), (3, 3, -1, 0)]:
        with pytest.raises(sc.ScError) as e:
            h.normalise(xd, *args, "mad", "negative")
        assert e.value.code == sc.EINVAL, args
    # no window-volume limit
    h.normalise(xd, 41, 21, 0, 0, "std", "all")
    h.normalise(xd, 41, 21, 0, 0, "mad", "negative")
