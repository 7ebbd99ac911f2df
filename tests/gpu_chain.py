"""GPU-forced oracle chain: the parity check of whole S+C runs.

A whole run is a chain of iterations: iteration k smooths the cube after
replacing the voxels detected by iterations 1..k-1 (Sect. 6.2.4), measures
the noise and ORs its detections into the mask (Sect. 4.2). A legitimate
difference inside one iteration's boundary band changes what later
iterations replace, so comparing a whole GPU run with a whole oracle run
needs a guess at how far such a difference travels. Instead each iteration
of the GPU's own run is checked against the oracle given the GPU's own state:

  * the GPU's state after k iterations is the result of the same run cut to
    its first k kernels (runs are deterministic, and a run cut short performs
    the same launches as the first k iterations of the whole run: the noise
    values of every cut run must equal the whole run's bit for bit);
  * the oracle performs iteration k from that mask and the GPU's sigma_0;
  * the GPU's mask after iteration k must then equal the oracle's on every
    voxel outside the oracle's boundary band, and sigma_k must agree to 1e-6.

sigma_0 itself (measured before any detection) is compared with the oracle's
own to 1e-6. The test files import this module; nothing else does.
"""
import sys

import numpy as np

import oracle

SIGMA_RTOL = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def sc_kind(kernel) -> int:
    """Spatial kind of a kernel tuple: 0 cascade, 1 sampled Gaussian."""
    if len(kernel) < 3:
        return 0
    k = kernel[2]
    return {"cascade": 0, "gauss": 1}[k] if isinstance(k, str) else int(k)


def forced_chain(h, xd, x, kernels, t, mode, rng_, repl, what="", storage="f32",
                 sigma0=float("nan"), x_oracle=None, full=None, sigma_ok=None,
                 plane_stride=1):
    """Check every iteration of the GPU run of `kernels` on cube xd (host copy
    x) against the oracle from the GPU's own previous state.

    storage f16/bf16: x_oracle is the dequantised cube in units of the given
    sigma0; the oracle then works in those units (replacement level repl,
    sigma_0 = 1) and the GPU's noise values are divided by sigma0.
    full: the whole run's (mask tensor, noise, sigma_0) if already taken.
    sigma_ok(k, mask_prev, ref_sigma, gpu_sigma): replaces the 1e-6 noise
    bar (16-bit storage, where the test derives a bar of its own).
    plane_stride: noise subsampling, on both sides.
    Returns (largest sigma relative error, band voxels summed over steps)."""
    import torch
    q16 = storage != "f32"
    xo = x if x_oracle is None else x_oracle
    ps = plane_stride
    if full is None:
        full = h.run(xd, kernels, t, mode, rng_, repl, storage=storage, sigma0=sigma0,
                     noise_plane_stride=ps)
    fm, fn, fs0 = full
    if not q16 and repl >= 0 and np.isnan(sigma0):
        raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
        s0_ref, _ = oracle.noise(raw[::ps], mode, rng_)
        del raw
        assert abs(fs0 / s0_ref - 1) <= SIGMA_RTOL, f"{what}: sigma_0 {fs0} vs {s0_ref}"
    unit = sigma0 if q16 else 1.0
    s0_oracle = 1.0 if q16 else fs0
    prev = None
    worst, bands = 0.0, 0
    for k, kern in enumerate(kernels):
        f, w = kern[0], kern[1]
        kind = sc_kind(kern)
        if k == len(kernels) - 1:
            m_k, n_k = fm, fn
        else:
            m_k, n_k, s_k = h.run(xd, kernels[:k + 1], t, mode, rng_, repl, storage=storage,
                                  sigma0=sigma0, noise_plane_stride=ps)
            np.testing.assert_array_equal(n_k, fn[:k + 1],
                                          err_msg=f"{what}: cut run {k + 1} noise")
            assert (np.isnan(s_k) and np.isnan(fs0)) or s_k == fs0, f"{what}: cut run sigma_0"
        torch.cuda.synchronize()
        g = m_k.cpu().numpy()
        ref = oracle.step(xo, f, w, t, mode, rng_, prev, repl, s0_oracle, plane_stride=ps,
                          kind=kind)
        rel = abs(n_k[k] / unit / ref.sigma - 1)
        diff = g != ref.mask
        out = int((diff & (ref.band == 0)).sum())
        inside = int(diff.sum()) - out
        worst = max(worst, rel)
        bands += int(ref.band_count)
        if sigma_ok is None:
            assert rel <= SIGMA_RTOL, f"{what} step {k} ({f}, {w}): sigma rel {rel:.3g}"
        else:
            assert sigma_ok(k, prev, ref.sigma, n_k[k] / unit), \
                f"{what} step {k} ({f}, {w}): sigma rel {rel:.3g} outside the bar"
        assert out == 0, (f"{what} step {k} ({f}, {w}): {out} mask differences outside "
                          f"the band ({inside} inside)")
        prev = g
    say(f"{what}: GPU-forced chain of {len(kernels)} steps, worst sigma rel {worst:.2e}, "
        f"band voxels {bands}")
    return worst, bands
