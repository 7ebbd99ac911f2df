"""Seeded synthetic H I cubes shared by the oracle tests, GPU tests and bench.

Holds no smooth-and-clip arithmetic: it only draws noise and mock galaxies
(see ``gen.c``) and names the workload recipes. The paper's cubes (a WSRT
cube with WHISP galaxies, ASKAP Eridanus noise with galmod mocks, the
WALLABY Hydra field; Sects. 5-7) are not available, so these stand in for
them with the shapes and settings of the benchmark workloads.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
        ("seed", ctypes.c_uint64), ("cube_id", ctypes.c_uint32),
        ("field_kind", ctypes.c_int32),
        ("sigma_lo", ctypes.c_double), ("sigma_hi", ctypes.c_double),
        ("n_gal", ctypes.c_int64), ("nan_border", ctypes.c_int64),
        ("peak_lo", ctypes.c_double), ("peak_hi", ctypes.c_double),
        ("fwhm_z_lo", ctypes.c_double), ("fwhm_z_hi", ctypes.c_double),
        ("fwhm_xy_lo", ctypes.c_double), ("fwhm_xy_hi", ctypes.c_double),
        ("z0", ctypes.c_int64), ("z1", ctypes.c_int64),
    ]


def build(verbose: bool = False) -> str:
    """Compile gen.c into libsynth.so (gcc, OpenMP)."""
    import subprocess
    src = os.path.join(_HERE, "gen.c")
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", src,
           "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_cube.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        lib.synth_cube.restype = ctypes.c_int
        lib.synth_sigma_field.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        lib.synth_sigma_field.restype = ctypes.c_int
        lib.synth_philox4x32_10.argtypes = [
            ctypes.POINTER(ctypes.c_uint32), ctypes.c_uint32, ctypes.c_uint32,
            ctypes.POINTER(ctypes.c_uint32)]
        lib.synth_philox4x32_10.restype = None
        _lib = lib
    return _lib


@dataclass
class CubeSpec:
    """Recipe for one synthetic cube (float32, [nz][ny][nx])."""
    nx: int
    ny: int
    nz: int
    seed: int
    cube_id: int = 0
    radial: bool = False          # sigma grows as rho^2 from the centre
    sigma_lo: float = 1.0
    sigma_hi: float = 1.0
    n_gal: int = 0
    nan_border: int = 0
    peak: Tuple[float, float] = (0.5, 3.0)       # x local sigma
    fwhm_z: Tuple[float, float] = (5.0, 20.0)    # channels
    fwhm_xy: Tuple[float, float] = (4.0, 12.0)   # pixels

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    def _params(self, z0: int = 0, z1: int = 0) -> _Params:
        return _Params(
            self.nx, self.ny, self.nz, self.seed, self.cube_id,
            1 if self.radial else 0, self.sigma_lo, self.sigma_hi,
            self.n_gal, self.nan_border, self.peak[0], self.peak[1],
            self.fwhm_z[0], self.fwhm_z[1], self.fwhm_xy[0], self.fwhm_xy[1],
            z0, z1)


def generate(spec: CubeSpec, out: Optional[np.ndarray] = None,
             z0: int = 0, z1: int = 0) -> np.ndarray:
    """Generate the cube (or planes [z0, z1)) as float32 [nz][ny][nx]."""
    lib = _load()
    z1 = z1 or spec.nz
    shape = (z1 - z0, spec.ny, spec.nx)
    if out is None:
        out = np.empty(shape, dtype=np.float32)
    if out.shape != shape or out.dtype != np.float32 or not out.flags.c_contiguous:
        raise ValueError("out must be a C-contiguous float32 array of shape %r" % (shape,))
    p = spec._params(z0, z1)
    rc = lib.synth_cube(ctypes.byref(p), out.ctypes.data)
    if rc != 0:
        raise RuntimeError("synth_cube failed (%d)" % rc)
    return out


def sigma_field(spec: CubeSpec) -> np.ndarray:
    lib = _load()
    out = np.empty((spec.ny, spec.nx), dtype=np.float64)
    p = spec._params()
    if lib.synth_sigma_field(ctypes.byref(p), out.ctypes.data) != 0:
        raise RuntimeError("synth_sigma_field failed")
    return out


def philox4x32_10(ctr, key):
    """Raw Philox4x32-10 block (for the generator's known-answer test)."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*ctr)
    o = (ctypes.c_uint32 * 4)()
    lib.synth_philox4x32_10(c, key[0], key[1], o)
    return [int(v) for v in o]


# --------------------------------------------------------------------------
# Workload recipes. Kernel lists are (spatial FWHM px, spectral width ch),
# spatial-major, as in the paper's benchmark settings (Sect. 5).

@dataclass
class Workload:
    name: str
    cubes: List[CubeSpec]
    kernels: List[Tuple[float, int]]
    threshold: float
    noise_mode: str            # "std" | "mad"
    flux_range: str            # "negative" | "all" | "positive"
    replacement: float = 2.0   # n in +-n*sigma0 (Sect. 6.2.4); < 0 disables
    notes: str = ""


def _pairs(spatial, spectral):
    return [(float(f), int(w)) for f in spatial for w in spectral]


def batch_specs(n: int, seed: int, xy: Tuple[int, int], z: Tuple[int, int],
                sigma: Tuple[float, float] = (0.5, 2.0),
                gal_per_gvox: float = 2000.0) -> List[CubeSpec]:
    """n cubes of seeded uneven shapes: nx, ny uniform in xy, nz uniform in z
    (inclusive), one constant noise sigma per cube uniform in `sigma`, mock
    galaxies at the density of the 1024^3 workload (at least one per cube).
    Shapes and sigmas come from numpy's PCG64 stream for `seed`; the voxels
    from the cube generator with cube_id = index."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nx, ny = (int(v) for v in rng.integers(xy[0], xy[1] + 1, size=2))
        nz = int(rng.integers(z[0], z[1] + 1))
        sig = float(rng.uniform(sigma[0], sigma[1]))
        n_gal = max(1, int(round(gal_per_gvox * nx * ny * nz / float(1 << 30))))
        out.append(CubeSpec(nx, ny, nz, seed=seed, cube_id=i, sigma_lo=sig, sigma_hi=sig,
                            n_gal=n_gal))
    return out


def workload(name: str) -> Workload:
    """Named workloads (shapes and settings of the benchmark configurations)."""
    if name == "plain_64x64x128":
        return Workload(
            name, [CubeSpec(64, 64, 128, seed=1, n_gal=5)],
            _pairs([0, 3], [0, 3, 7]), 4.0, "std", "all",
            notes="i.i.d. sigma=1 noise, 5 blobs; flux range not stated -> all")
    if name == "plain_1024cube":
        return Workload(
            name, [CubeSpec(1024, 1024, 1024, seed=2, radial=True, sigma_lo=0.8,
                            sigma_hi=1.5, n_gal=2000, nan_border=13)],
            _pairs([0, 3, 6], [0, 3, 7, 15]), 3.5, "mad", "negative")
    if name == "plain_256cube":
        # Same recipe as plain_1024cube at 1/64 of the volume (galaxy density
        # kept); sized for the CPU oracle.
        return Workload(
            name, [CubeSpec(256, 256, 256, seed=2, radial=True, sigma_lo=0.8,
                            sigma_hi=1.5, n_gal=31, nan_border=4)],
            _pairs([0, 3, 6], [0, 3, 7, 15]), 3.5, "mad", "negative")
    if name == "large_2048x2048x4096":
        return Workload(
            name, [CubeSpec(2048, 2048, 4096, seed=4, radial=True, sigma_lo=0.8,
                            sigma_hi=1.5, n_gal=20000, nan_border=26)],
            _pairs([0, 3, 6, 9], [0, 3, 7, 15, 31]), 3.5, "mad", "negative",
            notes="64 GiB float32; spatially varying sigma; 26-px NaN border (5 % of voxels)")
    if name == "batch96":
        return Workload(
            name, batch_specs(96, seed=3, xy=(96, 512), z=(128, 1024)),
            _pairs([0, 3, 6], [0, 3, 7, 15]), 3.5, "mad", "negative",
            notes="96 independent cubes, spatial 96-512 px, 128-1024 channels, "
                  "sigma 0.5-2 per cube")
    if name == "batch_small":
        # Same recipe at sizes the oracle runs in seconds; ragged shapes.
        return Workload(
            name, batch_specs(7, seed=5, xy=(17, 75), z=(24, 90)),
            _pairs([0, 3, 6], [0, 3, 7, 15]), 3.5, "mad", "negative")
    if name == "paper_360x360x1464":
        return Workload(
            name, [CubeSpec(360, 360, 1464, seed=7, n_gal=40)],
            _pairs([0, 5, 10], [0, 3, 7, 15]), 3.5, "mad", "negative",
            notes="shape and kernels of the paper's laptop speed test (Sect. 5)")
    if name == "paper_1501cube":
        # 1501^3 float32 (12.6 GiB), i.i.d. noise of sigma 1 (the paper scales
        # its mock cube's noise to 1) and mock galaxies at the 1024^3 density.
        return Workload(
            name, [CubeSpec(1501, 1501, 1501, seed=8, n_gal=6300)],
            _pairs([0, 5, 10], [0, 3, 7, 15]), 3.5, "mad", "negative",
            notes="shape of the paper's 12.6 GB cube (Sects. 5 and 6)")
    raise KeyError(name)


def random_labels(shape: Tuple[int, int, int], n: int, seed: int,
                  extent_xy: Tuple[int, int] = (4, 16), extent_z: Tuple[int, int] = (3, 24),
                  fill: float = 0.85) -> np.ndarray:
    """An int32 label cube [nz][ny][nx] of n seeded detections 1..n: each is a
    box of extents uniform in extent_xy (x and y) and extent_z (z) at a
    uniform position, of which each voxel is kept with probability `fill`
    (ragged shapes). Later boxes overwrite earlier ones where they overlap, so
    some labels may end up with few or no voxels. Stands in for a linker's
    output with the size mix of detections of at least 8 px and 5 channels."""
    nz, ny, nx = shape
    rng = np.random.default_rng(seed)
    lab = np.zeros(shape, dtype=np.int32)
    for i in range(1, n + 1):
        ex = int(rng.integers(extent_xy[0], extent_xy[1] + 1))
        ey = int(rng.integers(extent_xy[0], extent_xy[1] + 1))
        ez = int(rng.integers(extent_z[0], extent_z[1] + 1))
        ex, ey, ez = min(ex, nx), min(ey, ny), min(ez, nz)
        x0 = int(rng.integers(0, nx - ex + 1))
        y0 = int(rng.integers(0, ny - ey + 1))
        z0 = int(rng.integers(0, nz - ez + 1))
        keep = rng.random((ez, ey, ex)) < fill
        view = lab[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex]
        view[keep] = i
    return lab
