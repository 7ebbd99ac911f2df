"""Parity at the full benchmark size (1024^3, MAD on negative voxels, 3.5 sigma).

The whole 12-kernel oracle run at this size takes minutes, so the full-size
check is split into what the oracle computes exactly in seconds:
  * step 1 (kernel (0, 0)): sigma_1 = sigma_0 and the plain threshold mask;
  * single S+C iterations of a spectral-only and a spatial+spectral kernel,
    teacher-forced with the oracle's step-1 mask and sigma_0, in the same
    launch configuration as the benchmark;
and the whole GPU run is checked for properties that hold at any size
(mask contains the step-1 mask, blanked voxels never set, sigma_1 = sigma_0,
sign symmetry bit-exact).
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
def cfg2():
    wl = synth.workload("plain_1024cube")
    x = synth.generate(wl.cubes[0])
    raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
    s0, m = oracle.noise(raw, "mad", "negative")
    del raw
    fin = np.isfinite(x)
    ax = np.abs(x.astype(np.float64))
    with np.errstate(invalid="ignore"):
        m1 = (fin & (ax > 3.5 * s0)).astype(np.uint8)
        band1 = (fin & (np.abs(ax / s0 - 3.5) <= 1e-5)).astype(np.uint8)
    del ax
    say("full size: sigma0", s0, "selected", m, "step-1 detections", int(m1.sum()))
    return wl, x, s0, m1, band1


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def test_fullsize_first_step_exact(h, cfg2):
    wl, x, s0, m1, band1 = cfg2
    xd = torch.from_numpy(x).cuda()
    out, s1 = h.step(xd, (0.0, 0), 3.5, "mad", "negative", 2.0, s0)
    g = out.cpu().numpy()
    assert abs(s1 / s0 - 1) <= 1e-6
    diff = g != m1
    assert int((diff & (band1 == 0)).sum()) == 0


@pytest.mark.parametrize("kernel", [(0.0, 15), (6.0, 15)])
def test_fullsize_teacher_forced_step(h, cfg2, kernel):
    wl, x, s0, m1, _ = cfg2
    ref = oracle.step(x, kernel[0], kernel[1], 3.5, "mad", "negative", m1, 2.0, s0)
    xd = torch.from_numpy(x).cuda()
    out, sk = h.step(xd, kernel, 3.5, "mad", "negative", 2.0, s0,
                     mask_in=torch.from_numpy(m1).cuda())
    g = out.cpu().numpy()
    diff = g != ref.mask
    say(f"full size {kernel}: sigma gpu {sk} oracle {ref.sigma} rel {abs(sk / ref.sigma - 1):.2e}"
        f" band {ref.band_count} diff {int(diff.sum())}")
    assert abs(sk / ref.sigma - 1) <= 1e-6
    assert int((diff & (ref.band == 0)).sum()) == 0


def test_fullsize_run_properties(h, cfg2):
    wl, x, s0, m1, band1 = cfg2
    xd = torch.from_numpy(x).cuda()
    mask, noise, sigma0 = h.run(xd, wl.kernels, wl.threshold, wl.noise_mode,
                                wl.flux_range, wl.replacement)
    g = mask.cpu().numpy()
    assert abs(noise[0] / s0 - 1) <= 1e-6 and abs(sigma0 / s0 - 1) <= 1e-6
    assert g.max() == 1
    assert not g[~np.isfinite(x)].any()
    # the union contains the step-1 detections (outside the step-1 band)
    assert int(((m1 == 1) & (g == 0) & (band1 == 0)).sum()) == 0
    del mask
    neg = torch.neg(xd)
    mask2, noise2, _ = h.run(neg, wl.kernels, wl.threshold, wl.noise_mode, "positive",
                             wl.replacement)
    np.testing.assert_array_equal(noise2, noise)
    assert torch.equal(mask2.cpu(), torch.from_numpy(g))


_CUT = {}


def _gpu_state(h, xd, wl, k):
    """The GPU's mask (host copy), noise and sigma_0 after its first k
    iterations of the full-size run: the run cut to its first k kernels."""
    if k not in _CUT:
        m, n, s0 = h.run(xd, wl.kernels[:k], wl.threshold, wl.noise_mode, wl.flux_range,
                         wl.replacement)
        torch.cuda.synchronize()
        _CUT.clear()   # keep at most two 1 GiB host masks
        _CUT[k] = (m.cpu().numpy(), n, s0)
        del m
    return _CUT[k]


@pytest.fixture(scope="module")
def xd_full(cfg2):
    return torch.from_numpy(cfg2[1]).cuda()


@pytest.mark.parametrize("k", range(12))
def test_fullsize_gpu_forced_chain(h, cfg2, xd_full, k):
    """Iteration k of the whole full-size run, checked against the oracle from
    the GPU's own state after iterations 1..k-1 (its run cut to k-1 kernels)
    and the GPU's sigma_0: noise to 1e-6, mask equal outside the band. The
    twelve tests together cover the whole 12-kernel run of the benchmark."""
    wl, x, s0, m1, band1 = cfg2
    f, w = wl.kernels[k]
    prev = None
    if k:
        prev, n_prev, s0_prev = _gpu_state(h, xd_full, wl, k)
    cur, n_cur, s0_gpu = _gpu_state(h, xd_full, wl, k + 1)
    if k:
        np.testing.assert_array_equal(n_cur[:k], n_prev)
        assert s0_gpu == s0_prev
    assert abs(s0_gpu / s0 - 1) <= 1e-6
    say(f"full-size chain step {k} ({f}, {w}): oracle step ...")
    ref = oracle.step(x, f, w, wl.threshold, wl.noise_mode, wl.flux_range, prev,
                      wl.replacement, s0_gpu)
    diff = cur != ref.mask
    out = int((diff & (ref.band == 0)).sum())
    rel = abs(n_cur[k] / ref.sigma - 1)
    say(f"  sigma rel {rel:.2e}, band {ref.band_count}, diff {int(diff.sum())} "
        f"(outside the band {out}), detections {int(cur.sum())}")
    assert rel <= 1e-6
    assert out == 0


def test_fullsize_noise_normalisation_bit_exact(h, cfg2, xd_full):
    """Local noise normalisation of the 1024^3 cube with the paper's window of
    31 pixels and 31 channels (Sect. 5), MAD on negative voxels, grid 16:
    noise grid and normalised cube equal to the oracle's bit for bit. Then the
    first S+C iteration on the normalised cube against the oracle."""
    wl, x, s0, m1, band1 = cfg2
    sig_ref, y_ref = oracle.normalise(x, 31, 31, 16, 16, "mad", "negative")
    y, sig = h.normalise(xd_full, 31, 31, 16, 16, "mad", "negative")
    np.testing.assert_array_equal(sig, sig_ref)
    yh = y.cpu().numpy()
    np.testing.assert_array_equal(yh, y_ref)
    fin = np.isfinite(sig_ref)
    say(f"full-size normalisation: grid {sig.shape}, sigma {sig_ref[fin].min():.3f}.."
        f"{sig_ref[fin].max():.3f}, equal bit for bit")
    ref = oracle.step(y_ref, 0.0, 0, 3.5, "mad", "negative")
    out, s1 = h.step(y, (0.0, 0), 3.5, "mad", "negative", -1.0, float("nan"))
    g = out.cpu().numpy()
    assert abs(s1 / ref.sigma - 1) <= 1e-6
    assert int(((g != ref.mask) & (ref.band == 0)).sum()) == 0
    say(f"  first S+C step on the normalised cube: sigma {s1:.6f} (oracle {ref.sigma:.6f}), "
        f"{int(g.sum())} detections vs {int(m1.sum())} before normalisation")


def test_fullsize_linker_bit_exact(h, cfg2, xd_full):
    """The whole 12-kernel run's mask of the 1024^3 cube, linked on the GPU
    with the mock run's settings (radius 2, minimum 8 pixels / 5 channels,
    Sect. 6) and without size filter: labels, counts and boxes equal to the
    oracle's."""
    mask, _, _ = _gpu_state(h, xd_full, cfg2[0], 12)
    md = torch.from_numpy(mask).cuda()
    for filt in [(8, 5, 0, 0), (0, 0, 0, 0)]:
        lab_ref, n_ref, box_ref = oracle.link(mask, 2, 2, *filt)
        lab, n, boxes = h.link(md, 2, 2, *filt)
        assert n == n_ref
        np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref)
        np.testing.assert_array_equal(boxes, box_ref)
        say(f"full-size linker {filt}: {n} detections from {int(mask.sum())} voxels, "
            f"equal to the oracle")
        del lab, lab_ref


def test_fullsize_parameterisation_and_reliability(h, cfg2, xd_full):
    """Parameters and reliability of 24576 seeded ragged-box detections (about
    the catalogue size of the mock run, Sect. 6) in the 1024^3 cube: every
    detection's parameters against the oracle over the labelled voxels, the
    reliability and kept flag at 512 sampled positive detections (the
    oracle's densities there run over all detections)."""
    from test_gpu_param import _term_scales, compare
    param = oracle.param_module()
    wl, x, s0, m1, band1 = cfg2
    n = 24576
    labels = synth.random_labels(x.shape, n, 77)
    ld = torch.from_numpy(labels).cuda()
    g, kept = h.parameterise(xd_full, ld, n, sigma_rms=s0)
    del ld
    idx = np.flatnonzero(labels)
    lab = labels.ravel()[idx]
    del labels
    vals = x.ravel()[idx]
    p = param.parameterise_voxels(idx, vals, lab, x.shape, n, sigma_rms=s0)
    rng = np.random.default_rng(5)
    at = np.sort(rng.choice(np.flatnonzero(p["sum"] > 0), 512, replace=False))
    o = param.finish(p, at=at)
    say(f"full-size parameterisation: {n} detections over {idx.size} voxels, "
        f"{int((o['sum'] > 0).sum())} positive, {int((o['sum'] < 0).sum())} negative")
    compare(g, o, _term_scales(idx, vals, lab, x.shape, n), n, kept, at=at)
