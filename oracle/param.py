"""TEST INFRASTRUCTURE: FP64 NumPy oracle of SoFiA 2's source parameterisation
and reliability filter (Westmeier et al. 2021, arXiv:2106.15789).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this module. It shares no code with the GPU library.

What the paper fixes:
  * the integrated flux of a detection is F = (channel width / beam solid
    angle) x the sum of the flux densities S_i of its N voxels, Eq. (4), and
    for a Gaussian beam 4 ln(2) Omega = pi a b with a, b the beam's FWHM in
    pixels (Sect. 6.1.2);
  * its statistical uncertainty is sigma_F = sqrt(N) x channel width x
    sigma_rms / sqrt(Omega), Eq. (5), and SNR = F / sigma_F;
  * the peak flux density is the largest value inside the source mask
    (Sect. 6.2.2); parameters are measured across the 3-D mask (Sect. 4.5);
  * reliability compares the number density of detections with positive and
    negative total flux in the 3-D space of peak, summed and mean flux
    density (Sect. 4.4); detections below a reliability threshold or an
    integrated-SNR threshold are discarded; the mock run uses threshold 0.9,
    kernel scale factor 0.4 and SNR threshold 2.8 (Sect. 6).

Readings where the paper is silent (listed with reasons in the design notes):
  P1 a detection's voxels are those carrying its label; only finite values
     count (N is the number of finite voxels);
  P2 the centroid is the flux-weighted mean position (NaN for a zero sum);
  P3 Omega = 1 when no beam is given (no beam correction); sigma_rms is the
     caller's (e.g. the S+C sigma_0, or 1 after noise normalisation);
  P4 a detection is positive when its summed flux is > 0, negative when < 0;
     its parameter vector is log10 of (peak, sum, mean) for a positive one and
     of (-min, -sum, -mean) for a negative one;
  P5 densities are sums of Gaussian kernels exp(-d^T C^-1 d / 2) whose
     covariance C is the sample covariance (divisor n - 1) of the negative
     detections' parameter vectors times the scale factor squared; the
     density of positives at a positive detection includes itself;
  P6 R = max(0, (P - N) / P) for positive detections, 0 for the others; with
     fewer than three negative detections, or a singular covariance, there is
     no evidence of false positives and R = 1 for every positive detection;
  P7 a detection is kept when it is positive, R >= the reliability threshold
     and SNR >= the SNR threshold.
"""
from __future__ import annotations

import math

import numpy as np

FIELDS = ("count", "sum", "peak", "min", "mean", "x", "y", "z", "flux", "flux_err", "snr",
          "reliability", "kept")


def beam_solid_angle(a: float, b: float) -> float:
    """Omega in pixels for a Gaussian beam of FWHM a x b pixels (P3: 1 without
    a beam)."""
    if a > 0 and b > 0:
        return math.pi * a * b / (4.0 * math.log(2.0))
    return 1.0


def parameterise(cube: np.ndarray, labels: np.ndarray, n: int, channel_width: float = 1.0,
                 beam=(0.0, 0.0), sigma_rms: float = 1.0) -> dict:
    """Per-detection parameters for labels 1..n (arrays of length n)."""
    x = np.asarray(cube, dtype=np.float64).ravel()
    lab = np.asarray(labels).ravel()
    return parameterise_voxels(np.arange(x.size), x, lab, cube.shape, n, channel_width, beam,
                               sigma_rms)


def parameterise_voxels(index: np.ndarray, values: np.ndarray, labels: np.ndarray, shape,
                        n: int, channel_width: float = 1.0, beam=(0.0, 0.0),
                        sigma_rms: float = 1.0) -> dict:
    """parameterise() over a subset of a cube of the given shape (nz, ny, nx)
    that holds at least every labelled voxel: their raster indices, values and
    labels."""
    x = np.asarray(values, dtype=np.float64).ravel()
    lab = np.asarray(labels).ravel().astype(np.int64)
    ok = (lab > 0) & (lab <= n) & np.isfinite(x)
    lab, v = lab[ok], x[ok]
    idx = np.asarray(index, dtype=np.int64).ravel()[ok]
    nz, ny, nx = shape
    px, py, pz = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    count = np.bincount(lab, minlength=n + 1)[1:]
    s = np.bincount(lab, weights=v, minlength=n + 1)[1:]
    sx = np.bincount(lab, weights=v * px, minlength=n + 1)[1:]
    sy = np.bincount(lab, weights=v * py, minlength=n + 1)[1:]
    sz = np.bincount(lab, weights=v * pz, minlength=n + 1)[1:]
    peak = np.full(n, -np.inf)
    mn = np.full(n, np.inf)
    np.maximum.at(peak, lab - 1, v)
    np.minimum.at(mn, lab - 1, v)
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = s / count
        cx, cy, cz = sx / s, sy / s, sz / s
    omega = beam_solid_angle(*beam)
    flux = channel_width / omega * s
    flux_err = np.sqrt(count) * channel_width * sigma_rms / math.sqrt(omega)
    with np.errstate(invalid="ignore", divide="ignore"):
        snr = flux / flux_err
    cx = np.where(s != 0, cx, np.nan)
    cy = np.where(s != 0, cy, np.nan)
    cz = np.where(s != 0, cz, np.nan)
    return {"count": count.astype(np.int64), "sum": s, "peak": peak, "min": mn, "mean": mean,
            "x": cx, "y": cy, "z": cz, "flux": flux, "flux_err": flux_err, "snr": snr}


def _vectors(p: dict, sign: int) -> np.ndarray:
    if sign > 0:
        return np.log10(np.stack([p["peak"], p["sum"], p["mean"]], axis=1))
    return np.log10(np.stack([-p["min"], -p["sum"], -p["mean"]], axis=1))


def reliability(p: dict, scale: float = 0.4, at=None) -> np.ndarray:
    """Reliability of every detection (P4-P6). With `at` (detection indices)
    only those are evaluated, the others are NaN; the densities still sum
    over every detection."""
    s = p["sum"]
    pos, neg = s > 0, s < 0
    only = np.ones(s.size, dtype=bool)
    if at is not None:
        only[:] = False
        only[np.asarray(at, dtype=np.int64)] = True

    def result(R):
        return np.where(only, R, np.nan)

    R = np.zeros(s.size)
    if not pos.any():
        return result(R)
    vp = _vectors({k: v[pos] for k, v in p.items()}, +1)
    if neg.sum() < 3:
        R[pos] = 1.0
        return result(R)
    vn = _vectors({k: v[neg] for k, v in p.items()}, -1)
    cov = np.cov(vn.T, ddof=1) * scale * scale
    det = np.linalg.det(cov)
    if not (np.isfinite(det) and det > 0):
        R[pos] = 1.0
        return result(R)
    inv = np.linalg.inv(cov)

    def density(at, of):
        d = at[:, None, :] - of[None, :, :]
        q = np.einsum("ijk,kl,ijl->ij", d, inv, d)
        return np.exp(-0.5 * q).sum(axis=1)

    ev = pos & only
    va = _vectors({k: v[ev] for k, v in p.items()}, +1)
    P = density(va, vp)
    N = density(va, vn)
    R[ev] = np.maximum(0.0, (P - N) / P)
    return result(R)


def catalogue(cube, labels, n, channel_width=1.0, beam=(0.0, 0.0), sigma_rms=1.0,
              scale=0.4, rel_threshold=0.9, snr_threshold=2.8) -> dict:
    """Parameters, reliability and the kept flag (P7) of detections 1..n."""
    p = parameterise(cube, labels, n, channel_width, beam, sigma_rms)
    return finish(p, scale, rel_threshold, snr_threshold)


def finish(p: dict, scale=0.4, rel_threshold=0.9, snr_threshold=2.8, at=None) -> dict:
    """Adds reliability and the kept flag (P7) to parameters p (with `at`,
    only for those detections: see reliability())."""
    p["reliability"] = reliability(p, scale, at)
    with np.errstate(invalid="ignore"):
        p["kept"] = ((p["sum"] > 0) & (p["reliability"] >= rel_threshold) &
                     (p["snr"] >= snr_threshold)).astype(np.int32)
    return p
