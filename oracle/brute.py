"""TEST INFRASTRUCTURE: brute-force smooth-and-clip on tiny cubes (NumPy).

An independent formulation of the same readings as ``sc_oracle.cpp``, used
only to pin it: the whole 3-D smoothing is one explicit N x N matrix (the
Kronecker product of per-axis operators, each the matrix power of a banded
boxcar matrix, so truncation at the cube edges is built into the matrix), the
median comes from a full sort, and the cascade plan from an exhaustive
search. Nothing here is shared with the C++ oracle or the GPU library.

Sect. 4.2 (S+C: smooth on several scales, threshold against the noise of each
scale, both signs, one binary mask); Sect. 6.2.4 (replacement by +-n times the
noise, sign kept); Fig. 9 caption (Gaussian by FWHM in pixels, boxcar by
width in channels); Sect. 4.1 (MAD-based RMS).
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Tuple

import numpy as np

MAD_FACTOR = 1.4826


def plan(fwhm: float) -> Tuple[int, int]:
    """Exhaustive search over (n_iter, r) for reading R1."""
    if fwhm == 0:
        return 0, 0
    target = (fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))) ** 2
    cands = []
    for n in range(3, 7):
        for r in range(1, 200):
            var = n * r * (r + 1) / 3.0
            cands.append((abs(var - target), -n, r))
    d, mn, r = min(cands)
    return -mn, r


def boxcar_matrix(length: int, r: int) -> np.ndarray:
    """Rows: output index; 1/(2r+1) on |i-j| <= r inside the axis, 0 outside."""
    i = np.arange(length)
    band = np.abs(i[:, None] - i[None, :]) <= r
    return band.astype(np.float64) / (2 * r + 1)


def axis_operator(length: int, n_pass: int, r: int) -> np.ndarray:
    if n_pass == 0 or r == 0:
        return np.eye(length)
    return np.linalg.matrix_power(boxcar_matrix(length, r), n_pass)


def smoothing_operator(shape, fwhm: float, width: int) -> np.ndarray:
    """Dense N x N operator for the index order (z, y, x)."""
    nz, ny, nx = shape
    n_it, r = plan(fwhm)
    ax = axis_operator(nx, n_it, r)
    ay = axis_operator(ny, n_it, r)
    az = axis_operator(nz, 1, (width - 1) // 2) if width >= 3 else np.eye(nz)
    return np.kron(az, np.kron(ay, ax))


def noise(s: np.ndarray, mode: str, flux_range: str) -> float:
    v = s[np.isfinite(s)]
    if flux_range == "negative":
        v = v[v < 0]
    elif flux_range == "positive":
        v = v[v > 0]
    if v.size == 0:
        return float("nan")
    if mode == "std":
        return float(np.sqrt(np.sum(v * v) / v.size))
    a = np.sort(np.abs(v))
    m = a.size
    med = a[m // 2] if m % 2 else 0.5 * (a[m // 2 - 1] + a[m // 2])
    return float(MAD_FACTOR * med)


def smooth(cube: np.ndarray, fwhm: float, width: int,
           mask_prev: Optional[np.ndarray] = None, repl: float = -1.0,
           sigma0: float = float("nan")) -> np.ndarray:
    x = cube.astype(np.float64)
    finite = np.isfinite(x)
    y = np.where(finite, x, 0.0)
    if repl >= 0 and mask_prev is not None:
        hit = (mask_prev != 0) & finite
        y = np.where(hit, np.copysign(repl * sigma0, x), y)
    s = smoothing_operator(cube.shape, fwhm, width) @ y.ravel()
    s = s.reshape(cube.shape)
    s[~finite] = np.nan
    return s


def run(cube: np.ndarray, kernels: Sequence[Tuple[float, int]], threshold: float,
        mode: str, flux_range: str, repl: float = 2.0):
    """Returns (mask uint8, sigma per kernel, sigma0)."""
    x = cube.astype(np.float64)
    finite = np.isfinite(x)
    sigma0 = float("nan")
    if repl >= 0:
        sigma0 = noise(np.where(finite, x, np.nan), mode, flux_range)
    mask = np.zeros(cube.shape, dtype=np.uint8)
    sig = []
    for f, w in kernels:
        s = smooth(cube, f, w, mask if repl >= 0 else None, repl, sigma0)
        sk = noise(s, mode, flux_range)
        sig.append(sk)
        with np.errstate(invalid="ignore"):
            hit = finite & (np.abs(s) > threshold * sk)
        mask = mask | hit.astype(np.uint8)
    return mask, np.array(sig), sigma0


# ------------------------------------------------ local noise normalisation

def _axis_blocks(n: int, g: int, w: int):
    """Per block of one axis: (member indices, window indices). Members are
    the voxels whose index // g is the block number; the centre is the lower
    middle member; the window is every index within (w - 1) / 2 of it."""
    idx = np.arange(n)
    out = []
    for b in range(int(np.ceil(n / g))):
        members = np.flatnonzero(idx // g == b)
        centre = members[(members.size - 1) // 2]
        window = np.flatnonzero(np.abs(idx - centre) <= (w - 1) // 2)
        out.append((members, window))
    return out


def normalise(cube: np.ndarray, w_xy: int, w_z: int, g_xy: int, g_z: int, mode: str,
              flux_range: str):
    """Noise of every block's window (sort-based median) and the cube divided
    by its block's noise: (sigma [nbz][nby][nbx], float32 cube)."""
    x = cube.astype(np.float64)
    nz, ny, nx = x.shape
    bx, by, bz = _axis_blocks(nx, g_xy, w_xy), _axis_blocks(ny, g_xy, w_xy), \
        _axis_blocks(nz, g_z, w_z)
    sig = np.empty((len(bz), len(by), len(bx)))
    y = np.full(x.shape, np.nan, dtype=np.float32)
    for k, (mz, wz) in enumerate(bz):
        for j, (my, wy) in enumerate(by):
            for i, (mx, wx) in enumerate(bx):
                s = noise(x[np.ix_(wz, wy, wx)].ravel(), mode, flux_range)
                sig[k, j, i] = s
                if np.isfinite(s) and s > 0:
                    with np.errstate(invalid="ignore"):
                        y[np.ix_(mz, my, mx)] = (x[np.ix_(mz, my, mx)] / s).astype(np.float32)
    return sig, y


# ----------------------------------------------------------------- linker

def link(mask: np.ndarray, r_xy: int, r_z: int, min_xy: int = 0, min_z: int = 0,
         max_xy: int = 0, max_z: int = 0):
    """Friends-of-friends on tiny masks: every pair of detected voxels is
    tested against the ellipsoid (scaled squared distance <= 1, radius-0
    axes admit offset 0 only), the components come from scipy's
    connected_components, sizes from the voxels' coordinates, and labels are
    handed out by sorting the kept components by their smallest index."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    nz, ny, nx = mask.shape
    idx = np.flatnonzero(mask.ravel() != 0)
    z, y, x = idx // (nx * ny), (idx // nx) % ny, idx % nx
    n = idx.size
    labels = np.zeros(mask.shape, dtype=np.int32)
    if n == 0:
        return labels, 0, np.zeros((0, 7), dtype=np.int64)
    dx = x[:, None] - x[None, :]
    dy = y[:, None] - y[None, :]
    dz = z[:, None] - z[None, :]
    d = np.zeros((n, n))
    ok = np.ones((n, n), dtype=bool)
    if r_xy > 0:
        d += (dx ** 2 + dy ** 2) / float(r_xy) ** 2
    else:
        ok &= (dx == 0) & (dy == 0)
    if r_z > 0:
        d += dz ** 2 / float(r_z) ** 2
    else:
        ok &= dz == 0
    adj = ok & (d <= 1.0 + 1e-12)
    i, j = np.nonzero(adj)
    ncomp, comp = connected_components(coo_matrix((np.ones(i.size), (i, j)), shape=(n, n)),
                                       directed=False)
    kept = []
    for c in range(ncomp):
        sel = comp == c
        ex = x[sel].max() - x[sel].min() + 1
        ey = y[sel].max() - y[sel].min() + 1
        ez = z[sel].max() - z[sel].min() + 1
        keep = ex >= min_xy and ey >= min_xy and ez >= min_z
        if max_xy > 0 and (ex > max_xy or ey > max_xy):
            keep = False
        if max_z > 0 and ez > max_z:
            keep = False
        if keep:
            kept.append((idx[sel].min(), c))
    kept.sort()
    boxes = []
    flat = labels.ravel()
    for lab, (_, c) in enumerate(kept, start=1):
        sel = comp == c
        flat[idx[sel]] = lab
        boxes.append([x[sel].min(), x[sel].max(), y[sel].min(), y[sel].max(), z[sel].min(),
                      z[sel].max(), int(sel.sum())])
    return labels, len(kept), np.array(boxes, dtype=np.int64).reshape(-1, 7)
