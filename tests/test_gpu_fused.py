"""Replacement off with the pairs that share a spatial kernel fused into
shared passes (fuse_widths): against the oracle's whole run (independent
pairs when replacement is off, Sect. 6.2.4) and against the per-pair GPU
path, through the C ABI."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from gpu_chain import sc_kind

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

SIGMA_RTOL = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def cube(nx, ny, nz, seed, n_gal=6, border=3):
    return synth.generate(synth.CubeSpec(nx, ny, nz, seed=seed, radial=True, sigma_lo=0.8,
                                         sigma_hi=1.5, n_gal=n_gal, nan_border=border))


KERNELS_12 = [(float(f), w) for f in (0, 3, 6) for w in (0, 3, 7, 15)]


def against_oracle(h, x, kernels, t, rng_, what, mode="std", **kw):
    ref = oracle.run(x, [(k[0], k[1], sc_kind(k)) for k in kernels], t, mode, rng_, -1.0)
    m, noise, s0 = h.run(dev(x), kernels, t, mode, rng_, -1.0, fuse_widths=True, **kw)
    g = m.cpu().numpy()
    rel = np.abs(noise / ref.sigma - 1)
    diff = g != ref.mask
    out = int((diff & (ref.band == 0)).sum())
    say(f"{what}: sigma rel max {rel.max():.2e}, detections {int(g.sum())}, "
        f"diff {int(diff.sum())} (outside the band {out})")
    assert math.isnan(s0)
    assert np.all(rel <= SIGMA_RTOL), rel
    assert out == 0
    return g, noise


@pytest.mark.parametrize("rng_", ["all", "negative"])
def test_fused_matches_oracle_12_pairs(h, rng_):
    x = cube(200, 170, 120, seed=51)
    against_oracle(h, x, KERNELS_12, 3.5, rng_, f"fused 12 pairs {rng_}")


def test_fused_mixed_kinds_many_widths_and_order(h):
    """A spatial kernel reused out of order, both spatial kinds, and one
    source with ten widths (two fused passes of up to eight)."""
    x = cube(150, 130, 140, seed=52)
    kernels = [(3.0, 7), (0.0, 0), (6.0, 3, "gauss")] + \
              [(0.0, w) for w in (3, 5, 7, 9, 11, 13, 15, 17, 21)] + [(3.0, 0), (6.0, 31, "gauss")]
    against_oracle(h, x, kernels, 4.0, "all", "fused mixed")


def test_fused_equals_per_pair_path(h):
    x = cube(180, 160, 100, seed=53)
    xd = dev(x)
    m0, n0, _ = h.run(xd, KERNELS_12, 3.5, "std", "all", -1.0)
    m1, n1, _ = h.run(xd, KERNELS_12, 3.5, "std", "all", -1.0, fuse_widths=True)
    np.testing.assert_allclose(n1, n0, rtol=1e-12)
    diff = int((m0 != m1).sum().item())
    say(f"fused vs per pair: noise max rel {np.abs(n1 / n0 - 1).max():.2e}, mask diff {diff}")
    assert diff <= 2


def test_fused_keep_input_mask_and_subsampling(h):
    x = cube(120, 110, 96, seed=54)
    kernels = [(0.0, 0), (0.0, 7), (3.0, 3)]
    rng = np.random.default_rng(4)
    pre = (rng.random(x.shape) < 0.01).astype(np.uint8) * 5
    md = dev(pre)
    m, noise, _ = h.run(dev(x), kernels, 3.5, "std", "all", -1.0, mask=md,
                        keep_input_mask=True, fuse_widths=True)
    ref = oracle.run(x, kernels, 3.5, "std", "all", -1.0)
    g = m.cpu().numpy()
    expect = np.where(ref.mask == 1, pre | 1, pre)
    diff = g != expect
    assert int((diff & (ref.band == 0)).sum()) == 0
    # noise on every 4th plane
    m2, n2, _ = h.run(dev(x), kernels, 3.5, "std", "all", -1.0, fuse_widths=True,
                      noise_plane_stride=4)
    for k, (f, w) in enumerate(kernels):
        st = oracle.step(x, f, w, 3.5, "std", "all", None, -1.0, float("nan"), plane_stride=4)
        assert abs(n2[k] / st.sigma - 1) <= SIGMA_RTOL, k


@pytest.mark.parametrize("rng_", ["negative", "all"])
def test_fused_mad_matches_oracle_12_pairs(h, rng_):
    """MAD: per width its own sample, prediction and exact selection from the
    keys one shared selection pass captured."""
    x = cube(200, 170, 120, seed=55)
    h.profile(True)
    against_oracle(h, x, KERNELS_12, 3.5, rng_, f"fused MAD 12 pairs {rng_}", mode="mad")
    h.profile(False)
    fam = {s["name"]: s for s in h.profile_read()}
    assert "fused_select" in fam and "column_hist2" not in fam, sorted(fam)


def test_fused_mad_mixed_kinds_and_many_widths(h):
    x = cube(150, 130, 140, seed=56)
    kernels = [(3.0, 7), (0.0, 0), (6.0, 3, "gauss")] + \
              [(0.0, w) for w in (3, 5, 7, 9, 11, 13, 15, 17, 21)] + [(3.0, 0)]
    against_oracle(h, x, kernels, 3.5, "negative", "fused MAD mixed", mode="mad")


def test_fused_mad_equals_per_pair_path(h):
    x = cube(180, 160, 100, seed=57)
    xd = dev(x)
    m0, n0, _ = h.run(xd, KERNELS_12, 3.5, "mad", "negative", -1.0)
    m1, n1, _ = h.run(xd, KERNELS_12, 3.5, "mad", "negative", -1.0, fuse_widths=True)
    rel = np.abs(n1 / n0 - 1)
    diff = int((m0 != m1).sum().item())
    say(f"fused MAD vs per pair: noise max rel {rel.max():.2e}, mask diff {diff}")
    assert rel.max() <= SIGMA_RTOL
    assert diff <= 4


def test_fused_mad_falls_back_when_sample_is_unrepresentative(h):
    """Rows read by the sampling passes scaled 100x: every width's predicted
    window misses and its full histogram passes run, still exact."""
    nx, ny, nz = 256, 120, 90
    rng = np.random.default_rng(58)
    x = rng.standard_normal((nz, ny, nx)).astype(np.float32)
    x[:, ::17, :] *= 100.0
    kernels = [(0.0, 0), (0.0, 3), (0.0, 7), (3.0, 0)]
    h.profile(True)
    against_oracle(h, x, kernels, 3.5, "negative", "fused MAD fallback", mode="mad")
    h.profile(False)
    fam = {s["name"]: s for s in h.profile_read()}
    assert fam.get("column_hist2", {}).get("launches", 0) >= 1, sorted(fam)


def test_fused_mad_capture_overflow(h):
    """Most voxels share one value: the captured keys exceed a width's list
    and its full level-2 pass takes over."""
    rng = np.random.default_rng(59)
    x = np.full((128, 256, 256), -1.0, np.float32)
    noisy = rng.random(x.shape) < 0.1
    x[noisy] = rng.standard_normal(int(noisy.sum())).astype(np.float32)
    h.profile(True)
    against_oracle(h, x, [(0.0, 0), (0.0, 3)], 3.5, "negative", "fused MAD overflow",
                   mode="mad")
    h.profile(False)
    fam = {s["name"]: s for s in h.profile_read()}
    assert fam.get("column_hist2", {}).get("launches", 0) >= 1, sorted(fam)


def test_fused_rejects_what_it_does_not_cover(h):
    xd = dev(np.random.default_rng(1).normal(size=(8, 16, 16)).astype(np.float32))
    for kw in [dict(replacement=2.0), dict(storage="f16")]:
        args = dict(noise_mode="std", replacement=-1.0)
        args.update(kw)
        with pytest.raises(sc.ScError) as e:
            h.run(xd, [(0.0, 3)], 3.0, args["noise_mode"], "all", args["replacement"],
                  storage=kw.get("storage", "f32"), fuse_widths=True)
        assert e.value.code == sc.EINVAL


def test_fused_nostat(h):
    x = -np.abs(np.random.default_rng(2).normal(size=(10, 20, 20))).astype(np.float32) - 0.1
    m, noise, _ = h.run(dev(x), [(0.0, 0), (0.0, 3)], 3.0, "std", "positive", -1.0,
                        fuse_widths=True, allow_nostat=True)
    assert np.isnan(noise).all()
    assert int(m.sum().item()) == 0
