"""The sampled-Gaussian spatial kernel (reading G1) on the GPU against the
oracle: smoothing values, single teacher-forced steps and GPU-forced chains
of whole runs that mix it with the cascade, through the C ABI."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_chain import forced_chain

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

# Largest |s_gpu - s_oracle| over rms(s): the x pass sums 2R + 1 FP32
# products, the y pass is accumulated in FP64 and rounded once.
SMOOTH_BAR = 3e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def radius(fwhm):
    return (oracle.gauss_taps(fwhm).size - 1) // 2


def cube(nx, ny, nz, seed, n_gal=3, border=2):
    return synth.generate(synth.CubeSpec(nx, ny, nz, seed=seed, radial=True, sigma_lo=0.8,
                                         sigma_hi=1.5, n_gal=n_gal, nan_border=border))


# FWHM 0.6 .. 14.1: radii 1 .. 24 (the largest supported)
GAUSS_FWHM = [0.6, 3.0, 5.0, 6.0, 9.0, 10.0, 12.2, 14.1]


@pytest.mark.parametrize("fwhm", GAUSS_FWHM)
@pytest.mark.parametrize("width", [0, 7])
def test_gauss_smooth_matches_oracle(h, fwhm, width):
    """Three strips (256, 256 and a ragged 18 columns) and chunk edges in y,
    with replacement, NaN voxels and an Inf column."""
    x = cube(530, 150, 9, seed=41)
    rng = np.random.default_rng(3)
    x[rng.random(x.shape) < 0.003] = np.nan
    x[:, 40, 300] = np.inf
    mask = (rng.random(x.shape) < 0.01).astype(np.uint8)
    mask[~np.isfinite(x)] = 0
    s_ref = oracle.smooth(x, fwhm, width, mask, 2.0, 0.9, kind=1)
    s_gpu = host(h.smooth(dev(x), (fwhm, width, "gauss"), replacement=2.0, sigma0=0.9,
                          mask_in=dev(mask))).astype(np.float64)
    np.testing.assert_array_equal(np.isnan(s_gpu), np.isnan(s_ref))
    fin = np.isfinite(s_ref)
    err = np.abs(s_gpu[fin] - s_ref[fin]).max() / math.sqrt(np.mean(s_ref[fin] ** 2))
    say(f"gauss smooth FWHM {fwhm} (R {radius(fwhm)}), width {width}: "
        f"max |ds| / rms(s) = {err:.3g}")
    assert err < SMOOTH_BAR


@pytest.mark.parametrize("shape", [(3, 1, 1), (2, 5, 3), (4, 40, 1), (3, 1, 300), (5, 37, 257)])
@pytest.mark.parametrize("fwhm", [3.0, 10.0])
def test_gauss_smooth_edge_shapes(h, shape, fwhm):
    """Planes narrower and shorter than the halo, single rows and columns,
    one column past a strip."""
    nz, ny, nx = shape
    x = np.random.default_rng(5).normal(size=shape).astype(np.float32)
    s_ref = oracle.smooth(x, fwhm, 0, kind=1)
    s_gpu = host(h.smooth(dev(x), (fwhm, 0, "gauss"))).astype(np.float64)
    err = np.abs(s_gpu - s_ref).max() / math.sqrt(np.mean(s_ref ** 2))
    assert err < SMOOTH_BAR, (shape, fwhm, err)


def test_gauss_rejects_too_wide_and_bad_kind(h):
    x = dev(np.zeros((2, 4, 4), np.float32))
    for k in [(14.5, 0, "gauss"), (3.0, 0, 2), (3.0, 0, -1)]:
        with pytest.raises(sc.ScError) as e:
            h.smooth(x, k)
        assert e.value.code == sc.EINVAL
    # beyond the cascade's halo limit but within the Gaussian's
    h.smooth(x, (14.0, 0, "gauss"))
    with pytest.raises(sc.ScError):
        h.smooth(x, (14.0, 0))


@pytest.mark.parametrize("kernel", [(3.0, 0), (10.0, 7), (6.0, 15)])
def test_gauss_teacher_forced_step(h, kernel):
    x = cube(300, 210, 64, seed=43, n_gal=5, border=3)
    raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
    s0, _ = oracle.noise(raw, "mad", "negative")
    m1 = oracle.step(x, 0.0, 0, 3.5, "mad", "negative").mask
    ref = oracle.step(x, kernel[0], kernel[1], 3.5, "mad", "negative", m1, 2.0, s0, kind=1)
    out, sk = h.step(dev(x), (kernel[0], kernel[1], "gauss"), 3.5, "mad", "negative", 2.0, s0,
                     mask_in=dev(m1))
    g = host(out)
    rel = abs(sk / ref.sigma - 1)
    diff = g != ref.mask
    say(f"gauss step {kernel}: sigma rel {rel:.2e}, band {ref.band_count}, "
        f"diff {int(diff.sum())}")
    assert rel <= 1e-6
    assert int((diff & (ref.band == 0)).sum()) == 0


def test_gauss_forced_chain_mixed_kinds(h):
    """A whole run whose kernel list mixes both spatial kinds, checked
    iteration by iteration from the GPU's own state."""
    x = cube(200, 170, 96, seed=45, n_gal=8, border=3)
    kernels = [(0.0, 0), (3.0, 0, "gauss"), (3.0, 7), (6.0, 3, "gauss"), (10.0, 15, "gauss"),
               (6.0, 3)]
    forced_chain(h, dev(x), x, kernels, 3.5, "mad", "negative", 2.0, what="gauss mixed")


def test_gauss_forced_chain_f16_storage(h):
    """16-bit storage: the Gaussian reads the FP16 cube; the oracle works on
    the dequantised cube in units of sigma_0."""
    from test_gpu_precision import _sigma_ok, dequantize_np, quantize_np
    x = cube(150, 130, 64, seed=47, n_gal=4, border=2)
    raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
    s0, _ = oracle.noise(raw, "mad", "negative")
    q = dequantize_np(quantize_np(x, s0, "f16"), "f16")
    kernels = [(0.0, 0), (5.0, 0, "gauss"), (9.0, 7, "gauss")]
    forced_chain(h, dev(x), x, kernels, 3.5, "mad", "negative", 2.0, what="gauss f16",
                 storage="f16", sigma0=s0, x_oracle=q,
                 sigma_ok=_sigma_ok(q, kernels, "mad", "negative", "gauss f16"))
