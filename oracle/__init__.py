"""TEST INFRASTRUCTURE: the FP64 CPU oracle of the smooth-and-clip finder.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never calls it and it
never calls the GPU library.

``sc_oracle.cpp`` is the smooth-and-clip oracle proper (C++17, FP64, direct
summation); ``nn_oracle.cpp`` the local noise normalisation (Sect. 4.1);
``link_oracle.cpp`` the friends-of-friends linker (Sect. 4.3);
``brute.py`` is an independent dense-matrix formulation used to pin them on
tiny cubes. Citations are to Westmeier et al. 2021 (arXiv:2106.15789).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsc_oracle.so")
# Tests that plant mistakes in a copy of the oracle point this at the copy.
_LIB_OVERRIDE = os.environ.get("SC_ORACLE_LIB")
_lib = None
# The other oracle libraries: source file -> library, and the variable that
# points a planted-mistake test at its copy.
_EXTRA = {
    "nn": ("nn_oracle.cpp", "libnn_oracle.so", "NN_ORACLE_LIB"),
    "link": ("link_oracle.cpp", "liblink_oracle.so", "LINK_ORACLE_LIB"),
}
_extra_libs = {}

NOISE = {"std": 0, "mad": 1}
RANGE = {"negative": -1, "all": 0, "positive": 1}
ENOSTAT = -4

def _compile(src_name: str, lib_path: str, verbose: bool) -> None:
    import subprocess
    src = os.path.join(_HERE, src_name)
    tmp = lib_path + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib_path)


def build(verbose: bool = False) -> str:
    """Compile the oracles with g++ -O2 -fopenmp (no fast-math: IEEE FP64)."""
    _compile("sc_oracle.cpp", _LIB_PATH, verbose)
    for src, lib, _ in _EXTRA.values():
        _compile(src, os.path.join(_HERE, lib), verbose)
    return _LIB_PATH


def lib_paths() -> List[str]:
    return [_LIB_PATH] + [os.path.join(_HERE, lib) for _, lib, _ in _EXTRA.values()]


def _extra(name: str):
    """Load one of the other oracle libraries (or its planted-mistake copy)."""
    if name not in _extra_libs:
        src, lib, env = _EXTRA[name]
        path = os.environ.get(env) or os.path.join(_HERE, lib)
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
        _extra_libs[name] = _bind_extra(name, ctypes.CDLL(path))
    return _extra_libs[name]


def _bind_extra(name, lib):
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    if name == "nn":
        lib.nno_blocks.argtypes = [i64, i64]
        lib.nno_blocks.restype = i64
        lib.nno_normalise.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, i32, i32,
                                      vp, vp]
        lib.nno_normalise.restype = ctypes.c_int
    if name == "link":
        lib.lko_link.argtypes = [vp, i64, i64, i64, i32, i32, i32, i32, i32, i32, vp,
                                 ctypes.POINTER(i64), vp, i64]
        lib.lko_link.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            return _bind(ctypes.CDLL(_LIB_OVERRIDE))
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: run __graft_entry__.build() first")
        return _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(lib):
    global _lib
    i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.sco_plan.argtypes = [dbl, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.sco_smooth.argtypes = [vp, i64, i64, i64, vp, dbl, dbl, dbl, i32, vp]
    lib.sco_noise.argtypes = [vp, i64, i32, i32, ctypes.POINTER(dbl),
                              ctypes.POINTER(i64)]
    lib.sco_step.argtypes = [vp, i64, i64, i64, vp, dbl, dbl, dbl, i32, dbl,
                             i32, i32, vp, ctypes.POINTER(dbl), vp,
                             ctypes.POINTER(i64)]
    lib.sco_run.argtypes = [vp, i64, i64, i64, vp, vp, vp, i32, dbl, i32, i32,
                            dbl, vp, vp, ctypes.POINTER(dbl), vp, vp]
    lib.sco_step_sub.argtypes = [vp, i64, i64, i64, vp, dbl, dbl, dbl, i32, i32, dbl, i32,
                                 i32, i32, dbl, vp, ctypes.POINTER(dbl), vp,
                                 ctypes.POINTER(i64)]
    lib.sco_smooth_kind.argtypes = [vp, i64, i64, i64, vp, dbl, dbl, dbl, i32, i32, vp]
    lib.sco_gauss_taps.argtypes = [dbl, vp, i32, ctypes.POINTER(i32)]
    fns = [lib.sco_plan, lib.sco_smooth, lib.sco_noise, lib.sco_step, lib.sco_run,
           lib.sco_step_sub, lib.sco_smooth_kind, lib.sco_gauss_taps]
    for f in fns:
        f.restype = ctypes.c_int
    _lib = lib
    return _lib


def _cube(x: np.ndarray) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    if x.ndim != 3:
        raise ValueError("cube must be 3-D [nz][ny][nx]")
    return x


def _mask_in(m: Optional[np.ndarray], shape) -> Optional[np.ndarray]:
    if m is None:
        return None
    m = np.ascontiguousarray(m, dtype=np.uint8)
    if m.shape != shape:
        raise ValueError("mask shape mismatch")
    return m


def plan(fwhm: float) -> Tuple[int, int]:
    """(n_iter, radius) of the boxcar cascade for a spatial FWHM (reading R1)."""
    n, r = ctypes.c_int32(), ctypes.c_int32()
    if _load().sco_plan(float(fwhm), ctypes.byref(n), ctypes.byref(r)) != 0:
        raise ValueError("bad FWHM %r" % fwhm)
    return n.value, r.value


def gauss_taps(fwhm: float) -> np.ndarray:
    """Taps of the sampled, truncated, normalised Gaussian (reading G1)."""
    cap = 4096
    h = np.empty(cap, dtype=np.float64)
    n = ctypes.c_int32()
    if _load().sco_gauss_taps(float(fwhm), h.ctypes.data, cap, ctypes.byref(n)) != 0:
        raise ValueError("bad FWHM %r" % fwhm)
    return h[:n.value].copy()


def smooth(cube: np.ndarray, fwhm: float, width: int,
           mask_prev: Optional[np.ndarray] = None, repl: float = -1.0,
           sigma0: float = float("nan"), kind: int = 0) -> np.ndarray:
    """Smoothed cube s (FP64, NaN where the input is blanked); kind 0 = the
    boxcar cascade (R1), 1 = the sampled Gaussian (G1)."""
    x = _cube(cube)
    m = _mask_in(mask_prev, x.shape)
    out = np.empty(x.shape, dtype=np.float64)
    nz, ny, nx = x.shape
    rc = _load().sco_smooth_kind(x.ctypes.data, nx, ny, nz,
                                 None if m is None else m.ctypes.data,
                                 float(repl), float(sigma0), float(fwhm), int(width),
                                 int(kind), out.ctypes.data)
    if rc != 0:
        raise ValueError("sco_smooth failed (%d)" % rc)
    return out


def noise(values: np.ndarray, mode: str, flux_range: str) -> Tuple[float, int]:
    """(sigma, number of selected voxels) of an FP64 array; NaN = blanked."""
    v = np.ascontiguousarray(values, dtype=np.float64).ravel()
    s, m = ctypes.c_double(), ctypes.c_int64()
    rc = _load().sco_noise(v.ctypes.data, v.size, NOISE[mode], RANGE[flux_range],
                           ctypes.byref(s), ctypes.byref(m))
    if rc not in (0, ENOSTAT):
        raise ValueError("sco_noise failed (%d)" % rc)
    return s.value, m.value


@dataclass
class StepResult:
    mask: np.ndarray
    sigma: float
    band: np.ndarray
    band_count: int
    status: int


def step(cube: np.ndarray, fwhm: float, width: int, threshold: float,
         mode: str, flux_range: str, mask_prev: Optional[np.ndarray] = None,
         repl: float = -1.0, sigma0: float = float("nan"), plane_stride: int = 1,
         sigma_given: float = float("nan"), kind: int = 0) -> StepResult:
    """One S+C iteration (teacher-forcing unit): mask_prev OR new detections.

    plane_stride > 1 measures the noise on every plane_stride-th plane only;
    a finite sigma_given replaces the measurement (clip of a slab with the
    noise of the whole cube); kind 1 takes the sampled Gaussian (G1) as the
    spatial kernel."""
    x = _cube(cube)
    m = _mask_in(mask_prev, x.shape)
    nz, ny, nx = x.shape
    out = np.empty(x.shape, dtype=np.uint8)
    band = np.zeros(x.shape, dtype=np.uint8)
    sig, nb = ctypes.c_double(), ctypes.c_int64()
    if plane_stride != 1 or not np.isnan(sigma_given) or kind != 0:
        rc = _load().sco_step_sub(x.ctypes.data, nx, ny, nz,
                                  None if m is None else m.ctypes.data, float(repl),
                                  float(sigma0), float(fwhm), int(width), int(kind),
                                  float(threshold),
                                  NOISE[mode], RANGE[flux_range], int(plane_stride),
                                  float(sigma_given), out.ctypes.data, ctypes.byref(sig),
                                  band.ctypes.data, ctypes.byref(nb))
    else:
        rc = _load().sco_step(x.ctypes.data, nx, ny, nz,
                              None if m is None else m.ctypes.data, float(repl),
                              float(sigma0), float(fwhm), int(width), float(threshold),
                              NOISE[mode], RANGE[flux_range], out.ctypes.data,
                              ctypes.byref(sig), band.ctypes.data, ctypes.byref(nb))
    if rc not in (0, ENOSTAT):
        raise ValueError("sco_step failed (%d)" % rc)
    return StepResult(out, sig.value, band, nb.value, rc)


@dataclass
class RunResult:
    mask: np.ndarray
    sigma: np.ndarray
    sigma0: float
    band: np.ndarray
    band_count: np.ndarray
    status: int


def run(cube: np.ndarray, kernels: Sequence[Tuple[float, int]], threshold: float,
        mode: str, flux_range: str, repl: float = 2.0) -> RunResult:
    """Whole S+C run over the kernel list, in list order. A kernel is
    (FWHM, width) or (FWHM, width, kind) with kind 1 = sampled Gaussian."""
    x = _cube(cube)
    nz, ny, nx = x.shape
    K = len(kernels)
    f = np.array([k[0] for k in kernels], dtype=np.float64)
    w = np.array([k[1] for k in kernels], dtype=np.int32)
    kd = np.array([k[2] if len(k) > 2 else 0 for k in kernels], dtype=np.int32)
    mask = np.empty(x.shape, dtype=np.uint8)
    band = np.empty(x.shape, dtype=np.uint8)
    sig = np.full(K, np.nan)
    bc = np.zeros(K, dtype=np.int64)
    s0 = ctypes.c_double()
    rc = _load().sco_run(x.ctypes.data, nx, ny, nz, f.ctypes.data, w.ctypes.data,
                         kd.ctypes.data, K, float(threshold), NOISE[mode], RANGE[flux_range],
                         float(repl), mask.ctypes.data, sig.ctypes.data,
                         ctypes.byref(s0), band.ctypes.data, bc.ctypes.data)
    if rc not in (0, ENOSTAT):
        raise ValueError("sco_run failed (%d)" % rc)
    return RunResult(mask, sig, s0.value, band, bc, rc)


# ------------------------------------------------ local noise normalisation

def nn_grid(nx: int, ny: int, nz: int, g_xy: int, g_z: int) -> Tuple[int, int, int]:
    """Blocks (nbz, nby, nbx) of the noise grid (reading N1)."""
    lib = _extra("nn")
    return (int(lib.nno_blocks(nz, g_z)), int(lib.nno_blocks(ny, g_xy)),
            int(lib.nno_blocks(nx, g_xy)))


def normalise(cube: np.ndarray, w_xy: int, w_z: int, g_xy: int, g_z: int, mode: str,
              flux_range: str, want_cube: bool = True):
    """Local noise normalisation (Sect. 4.1): (sigma grid [nbz][nby][nbx]
    FP64, normalised float32 cube or None)."""
    x = _cube(cube)
    nz, ny, nx = x.shape
    sig = np.empty(nn_grid(nx, ny, nz, g_xy, g_z), dtype=np.float64)
    y = np.empty(x.shape, dtype=np.float32) if want_cube else None
    rc = _extra("nn").nno_normalise(x.ctypes.data, nx, ny, nz, int(w_xy), int(w_z),
                                    int(g_xy), int(g_z), NOISE[mode], RANGE[flux_range],
                                    sig.ctypes.data, None if y is None else y.ctypes.data)
    if rc != 0:
        raise ValueError("nno_normalise failed (%d)" % rc)
    return sig, y


# ----------------------------------------------------------------- linker

def link(mask: np.ndarray, r_xy: int, r_z: int, min_xy: int = 0, min_z: int = 0,
         max_xy: int = 0, max_z: int = 0):
    """Friends-of-friends linker (Sect. 4.3): (int32 label cube, number of
    kept detections, [n][7] int64 boxes x0, x1, y0, y1, z0, z1, voxels)."""
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    if m.ndim != 3:
        raise ValueError("mask must be 3-D [nz][ny][nx]")
    nz, ny, nx = m.shape
    labels = np.empty(m.shape, dtype=np.int32)
    n = ctypes.c_int64()
    cap = int(m.sum()) + 1
    boxes = np.empty((cap, 7), dtype=np.int64)
    rc = _extra("link").lko_link(m.ctypes.data, nx, ny, nz, int(r_xy), int(r_z), int(min_xy),
                                 int(min_z), int(max_xy), int(max_z), labels.ctypes.data,
                                 ctypes.byref(n), boxes.ctypes.data, cap)
    if rc != 0:
        raise ValueError("lko_link failed (%d)" % rc)
    return labels, n.value, boxes[:n.value].copy()


def param_module():
    """The parameterisation / reliability oracle (oracle/param.py), or the
    planted-mistake copy a test points PARAM_ORACLE_FILE at."""
    path = os.environ.get("PARAM_ORACLE_FILE")
    if not path:
        from oracle import param
        return param
    import importlib.util
    spec = importlib.util.spec_from_file_location("param_mutant", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod
