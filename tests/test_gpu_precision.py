"""16-bit noise-scaled storage (F16 / BF16) against the FP64 oracle.

Comparisons (no single pass/fail bar exists for the total error of a 16-bit
cube):
  * on the same quantised data, one step at a time: the oracle runs on
    q = RN16(x / sigma_0) (quantised here with numpy, sigma_0 from the oracle
    and handed to the GPU) in scaled units, and every GPU step starts from the
    oracle's previous mask (teacher forcing); this isolates the kernels'
    arithmetic. The mask must match outside the band, the noise to 1e-6 or,
    where that is tighter than the data allow, to the interval that the fixed
    smoothing bar (|ds| <= 3e-6 rms(s), held by the smoothing parity tests)
    allows around the oracle's own smoothed cube: an RMS moves by at most the
    bar; a median by at most the bar, plus the effect of voxels whose sign the
    bar leaves open (a value within the bar of zero may leave or join the
    negative-pixel set, which shifts the median's rank by a half). The latter
    is what a 16-bit lattice shows: a smoothed value of ~1e-9 that FP32
    cancels to exactly 0 leaves the set and moves the median by one
    order-statistic spacing (~2e-6 of the median at 1e6 voxels);
  * the same data through a whole run, every iteration checked from the
    run's own previous state (GPU-forced chain) to the same bar;
  * against the original FP32 cube: the total error (storage rounding
    included) is reported and held to loose bounds.
"""
import sys

import numpy as np
import pytest

import gpu_chain
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


def quantize_np(x, scale, storage):
    """q = RN_T(RN_f32(x * RN_f64(1/scale))), finite values saturated (numpy)."""
    inv = 1.0 / scale
    with np.errstate(over="ignore", invalid="ignore"):
        y = (x.astype(np.float64) * inv).astype(np.float32)
    fin = np.isfinite(x)
    if storage == "f16":
        big = fin & ~(np.abs(y) <= np.float32(65504.0))
        y = np.where(big, np.copysign(np.float32(65504.0), y), y).astype(np.float32)
        with np.errstate(over="ignore", invalid="ignore"):
            return y.astype(np.float16).view(np.uint16)
    bmax = np.array([0x7F7F0000], np.uint32).view(np.float32)[0]
    big = fin & ~(np.abs(y) <= bmax)
    y = np.where(big, np.copysign(bmax, y), y).astype(np.float32)
    u = y.view(np.uint32).astype(np.uint64)
    q = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)
    nan = np.isnan(y)
    q[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return q


def dequantize_np(q, storage):
    if storage == "f16":
        return q.view(np.float16).astype(np.float32)
    return (q.astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_quantize_bit_exact(h, storage):
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(1 << 18) * 3).astype(np.float32)
    x[::97] = np.nan
    x[5] = np.inf
    x[6] = -np.inf
    x[7] = 1e6           # saturates in F16
    x[8] = -3e38         # saturates in BF16 after scaling by 1/0.73
    x[9] = 0.0
    x[10] = -0.0
    x[11] = 1e-30        # F16 underflow to (signed) zero / subnormal
    scale = 0.73
    got = h.quantize(torch.from_numpy(x).cuda(), scale, storage).cpu().numpy().view(np.uint16)
    exp = quantize_np(x, scale, storage)
    gv, ev = dequantize_np(got, storage), dequantize_np(exp, storage)
    np.testing.assert_array_equal(np.isnan(gv), np.isnan(ev))
    ok = ~np.isnan(ev)
    np.testing.assert_array_equal(got[ok], exp[ok])
    assert np.isfinite(gv[7]) and np.isfinite(gv[8])


def _oracle_chain(xq, kernels, t, mode, rng_, repl, sigma0):
    """Oracle run on a cube with sigma_0 given (chained single steps)."""
    mask = np.zeros(xq.shape, np.uint8)
    band = np.zeros(xq.shape, np.uint8)
    sig = []
    for f, w in kernels:
        st = oracle.step(xq, f, w, t, mode, rng_, mask, repl, sigma0)
        sig.append(st.sigma)
        band |= st.band
        mask = st.mask
    return mask, np.array(sig), band


CASES = [
    ("plain_64x64x128", None),
    ("cfg2_like", [(float(f), w) for f in (0, 3, 6) for w in (0, 3, 7, 15)]),
    # planes several strips wide: the 16-bit loads of the interior row loop
    ("wide_620x90x40", [(0.0, 0), (3.0, 3), (4.0, 0), (6.0, 7), (5.0, 15)]),
]


def _cube(name):
    if name == "plain_64x64x128":
        wl = synth.workload(name)
        return (synth.generate(wl.cubes[0]), wl.kernels, wl.threshold, wl.noise_mode,
                wl.flux_range)
    if name == "wide_620x90x40":
        spec = synth.CubeSpec(620, 90, 40, seed=62, radial=True, sigma_lo=0.8, sigma_hi=1.5,
                              n_gal=4, nan_border=2)
        return synth.generate(spec), CASES[2][1], 3.5, "mad", "negative"
    spec = synth.CubeSpec(150, 130, 120, seed=61, radial=True, sigma_lo=0.8, sigma_hi=1.5,
                          n_gal=8, nan_border=3)
    return synth.generate(spec), CASES[1][1], 3.5, "mad", "negative"


def _same_data(case, storage):
    x, kernels, t, mode, rng_ = _cube(case)
    raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
    s0, _ = oracle.noise(raw, mode, rng_)
    q = dequantize_np(quantize_np(x, s0, storage), storage)
    return x, q, s0, kernels, t, mode, rng_


# Smoothing bar of the FP32 arithmetic, as the smoothing parity tests hold
# it: |s_gpu - s_oracle| <= SMOOTH_BAR * rms(s). A 16-bit run performs the same
# arithmetic on the stored values, which FP32 holds exactly.
SMOOTH_BAR = 3e-6


def _noise_interval(s_ref, mode, rng_):
    """Noise values consistent with the oracle's smoothed cube s_ref moved by
    at most e = SMOOTH_BAR * rms(s_ref) per voxel (oracle values and the fixed
    bar only).

    std (RMS about zero): within e. MAD: the median of |s| moves by at most e;
    voxels with |s_ref| <= e may change sign (or become 0), so for a signed
    flux range the median is also taken with all of them in the set and with
    all of them out."""
    fin = np.isfinite(s_ref)
    e = SMOOTH_BAR * float(np.sqrt(np.mean(s_ref[fin] ** 2)))
    sig, _ = oracle.noise(s_ref, mode, rng_)
    if mode == "std":
        return sig - e, sig + e
    lo = hi = sig
    amb = fin & (np.abs(s_ref) <= e)
    if rng_ != "all" and amb.any():
        sign = -1.0 if rng_ == "negative" else 1.0
        s_in = s_ref.copy()
        s_in[amb] = sign * (np.abs(s_ref[amb]) + 1e-300)
        s_out = s_ref.copy()
        s_out[amb] = np.nan
        a, _ = oracle.noise(s_in, mode, rng_)
        b, _ = oracle.noise(s_out, mode, rng_)
        lo, hi = min(sig, a, b), max(sig, a, b)
    return lo - 1.4826 * e, hi + 1.4826 * e


def _sigma_ok(q, kernels, mode, rng_, tag):
    """Noise bar of a same-data step: 1e-6 relative, or inside the interval
    the smoothing bar allows around the oracle's smoothed cube."""
    def ok(k, mask_prev, ref_sigma, gpu_sigma):
        rel = abs(gpu_sigma / ref_sigma - 1)
        if rel <= 1e-6:
            return True
        f, w = kernels[k][0], kernels[k][1]
        s_ref = oracle.smooth(q, f, w, mask_prev, 2.0, 1.0, kind=gpu_chain.sc_kind(kernels[k]))
        lo, hi = _noise_interval(s_ref, mode, rng_)
        say(f"{tag} step {k} ({f}, {w}): sigma rel {rel:.2e}, smoothing-bar interval "
            f"[{lo / ref_sigma - 1:.2e}, {hi / ref_sigma - 1:.2e}]")
        return lo <= gpu_sigma <= hi
    return ok


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_16bit_storage_same_data_teacher_forced(h, storage, case):
    x, q, s0, kernels, t, mode, rng_ = _same_data(case, storage)
    xd = torch.from_numpy(x).cuda()
    mask = np.zeros(x.shape, np.uint8)
    worst = 0.0
    ok = _sigma_ok(q, kernels, mode, rng_, f"{case} {storage} teacher-forced")
    for k, (f, w) in enumerate(kernels):
        ref = oracle.step(q, f, w, t, mode, rng_, mask, 2.0, 1.0)
        mask_d = torch.from_numpy(mask).cuda()
        out, sk = h.step_ex(xd, (f, w), t, mode, rng_, mask_in=mask_d,
                            replacement=2.0, sigma0=s0, storage=storage)
        rel = abs(sk / s0 / ref.sigma - 1)
        diff = out.cpu().numpy() != ref.mask
        say(f"{case} {storage} same-data step ({f}, {w}): sigma rel {rel:.2e}, "
            f"mask diff {int(diff.sum())} (band {ref.band_count})")
        worst = max(worst, rel)
        assert ok(k, mask, ref.sigma, sk / s0)
        assert int((diff & (ref.band == 0)).sum()) == 0
        mask = ref.mask
    say(f"{case} {storage} same-data teacher-forced: worst sigma rel {worst:.2e}")


@pytest.mark.parametrize("storage", ["f16", "bf16"])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_16bit_storage_same_data_whole_run(h, storage, case):
    """Whole 16-bit runs on the quantised data, every iteration checked against
    the oracle on the dequantised cube from the run's own previous state."""
    x, q, s0, kernels, t, mode, rng_ = _same_data(case, storage)
    xd = torch.from_numpy(x).cuda()
    full = h.run(xd, kernels, t, mode, rng_, 2.0, storage=storage, sigma0=s0)
    assert full[2] == s0
    gpu_chain.forced_chain(h, xd, x, kernels, t, mode, rng_, 2.0, what=f"{case} {storage}",
                           storage=storage, sigma0=s0, x_oracle=q, full=full,
                           sigma_ok=_sigma_ok(q, kernels, mode, rng_, f"{case} {storage}"))


@pytest.mark.parametrize("storage,sig_tol", [("f16", 2e-3), ("bf16", 2e-2)])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_16bit_storage_total_error_report(h, storage, sig_tol, case):
    x, kernels, t, mode, rng_ = _cube(case)
    ref = oracle.run(x, kernels, t, mode, rng_, 2.0)
    xd = torch.from_numpy(x).cuda()
    m32, n32, _ = h.run(xd, kernels, t, mode, rng_, 2.0)
    m16, n16, s016 = h.run(xd, kernels, t, mode, rng_, 2.0, storage=storage)
    g32, g16 = m32.cpu().numpy(), m16.cpu().numpy()
    rel = np.abs(n16 / ref.sigma - 1)
    flips = int((g16 != ref.mask).sum())
    det = int(ref.mask.sum())
    say(f"{case} {storage} vs FP64 oracle on the FP32 cube: sigma rel max {rel.max():.2e} "
        f"(per kernel {np.array2string(rel, precision=1)}), mask flips {flips} of {det} "
        f"detections; FP32 path flips {int((g32 != ref.mask).sum())}")
    assert abs(s016 / ref.sigma0 - 1) <= 1e-6     # sigma_0 is measured on FP32 data
    assert rel.max() <= sig_tol
    assert flips <= max(10, det // 20)
