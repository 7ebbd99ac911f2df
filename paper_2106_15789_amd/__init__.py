"""MI355X smooth-and-clip (S+C) source finder: Python binding of libsofia_sc.so.

The work runs in the HIP kernels behind the C ABI of ``include/sofia_sc.h``;
this module only marshals arguments (torch tensors give device memory and
streams) and fails loudly when the library is missing. Method: SoFiA 2's S+C
finder, Westmeier et al. 2021 (arXiv:2106.15789), Sect. 4.2 and 6.2.4.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(_HERE)
LIB_PATH = os.path.join(_HERE, "libsofia_sc.so")
HEADER = os.path.join(ROOT, "include", "sofia_sc.h")
SOURCES = [os.path.join(_HERE, "csrc", n) for n in (
    "sc_kernels.hip", "sc_spatial_n3.hip", "sc_spatial_n4.hip", "sc_spatial_n5.hip",
    "sc_spatial_n6.hip", "sc_col_std.hip", "sc_col_hist.hip", "sc_col_select.hip", "sc_col_selclip.hip",
    "sc_col_clip.hip", "sc_col_write.hip", "sc_norm.hip", "sc_link.hip", "sc_param.hip",
    "sc_gauss_a.hip", "sc_gauss_b.hip", "sc_gauss_c.hip", "sc_multi.hip", "sc_api.hip")]

OK, EINVAL, ENOMEM, EDEVICE, ENOSTAT = 0, -1, -2, -3, -4
NOISE = {"std": 0, "mad": 1}
RANGE = {"negative": -1, "all": 0, "positive": 1}

# Every symbol include/sofia_sc.h declares.
EXPORTS = [
    "sofia_sc_default_options", "sofia_sc_create", "sofia_sc_destroy",
    "sofia_sc_run", "sofia_sc_run_ex", "sofia_sc_run_noalloc", "sofia_sc_run_batch",
    "sofia_sc_tune_batch", "sofia_sc_tune_run", "sofia_sc_set_shapes", "sofia_sc_get_shapes",
    "sofia_sc_step", "sofia_sc_step_ex",
    "sofia_sc_smooth",
    "sofia_sc_normalise", "sofia_sc_normalise_grid", "sofia_sc_link",
    "sofia_sc_param_defaults", "sofia_sc_parameterise", "sofia_sc_check_run",
    "sofia_sc_plan", "sofia_sc_quantize", "sofia_sc_profile", "sofia_sc_profile_read",
    "sofia_sc_last_error", "sofia_sc_strerror",
]


HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               # packed FP32 instructions stay off (see the design notes)
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile the HIP library for gfx950 (cross-compiles without a GPU).

    Each translation unit is compiled in its own hipcc process, in parallel,
    then linked into libsofia_sc.so.
    """
    import tempfile
    hipcc = "/opt/rocm/bin/hipcc"
    inc = "-I" + os.path.join(ROOT, "include")
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="sofia_sc_build_") as tmpd:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, os.path.basename(src) + ".o")
            objs.append(obj)
            cmd = [hipcc, *HIPCC_FLAGS, inc, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(subprocess.Popen(cmd))
            while sum(p.poll() is None for p in procs) >= jobs:
                procs[[p.poll() is None for p in procs].index(True)].wait()
        bad = [src for src, p in zip(SOURCES, procs) if p.wait() != 0]
        if bad:
            raise RuntimeError("hipcc failed for " + ", ".join(bad))
        tmp = LIB_PATH + ".tmp"
        cmd = [hipcc, *HIPCC_FLAGS, "-shared", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Kernel(ctypes.Structure):
    _fields_ = [("spatial_fwhm_px", ctypes.c_double),
                ("spectral_width_ch", ctypes.c_int32),
                ("spatial_kind", ctypes.c_int32)]


SPATIAL = {"cascade": 0, "gauss": 1}


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32),
                ("replacement", ctypes.c_double),
                ("sigma0", ctypes.c_double),
                ("storage", ctypes.c_int32),
                ("keep_input_mask", ctypes.c_int32),
                ("noise_plane_stride", ctypes.c_int32),
                ("fuse_widths", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


STORAGE = {"f32": 0, "f16": 1, "bf16": 2}


class BatchTuning(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("col_blocks", ctypes.c_int32),
                ("strip_rows", ctypes.c_int32), ("strip_waves", ctypes.c_int32),
                ("col_min_planes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class Cube(ctypes.Structure):
    _fields_ = [("cube", ctypes.c_void_p), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("nz", ctypes.c_int64), ("mask", ctypes.c_void_p)]


class ParamOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("channel_width", ctypes.c_double), ("beam_major_px", ctypes.c_double),
                ("beam_minor_px", ctypes.c_double), ("sigma_rms", ctypes.c_double),
                ("rel_scale", ctypes.c_double), ("rel_threshold", ctypes.c_double),
                ("snr_threshold", ctypes.c_double)]


# sofia_sc_source as a NumPy record (field names follow the parameter names
# the oracle uses: count = n_vox).
SOURCE_DTYPE = np.dtype([("count", "<i8"), ("sum", "<f8"), ("peak", "<f8"), ("min", "<f8"),
                         ("mean", "<f8"), ("x", "<f8"), ("y", "<f8"), ("z", "<f8"),
                         ("flux", "<f8"), ("flux_err", "<f8"), ("snr", "<f8"),
                         ("reliability", "<f8"), ("kept", "<i4"), ("pad", "<i4")])


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("voxels", ctypes.c_double)]


_lib = None


def load():
    """Load libsofia_sc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build(); "
            "there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, dbl, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.sofia_sc_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.sofia_sc_default_options.restype = None
    lib.sofia_sc_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.sofia_sc_destroy.argtypes = [vp]
    lib.sofia_sc_destroy.restype = None
    lib.sofia_sc_run.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(Kernel), i32,
                                 dbl, i32, i32, vp, ctypes.POINTER(dbl)]
    lib.sofia_sc_run_ex.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(Kernel), i32,
                                    dbl, i32, i32, vp, ctypes.POINTER(dbl),
                                    ctypes.POINTER(Options), ctypes.POINTER(dbl)]
    lib.sofia_sc_run_noalloc.argtypes = lib.sofia_sc_run_ex.argtypes
    lib.sofia_sc_run_batch.argtypes = [vp, ctypes.POINTER(Cube), i32, ctypes.POINTER(Kernel),
                                       i32, dbl, i32, i32, ctypes.POINTER(dbl),
                                       ctypes.POINTER(Options), ctypes.POINTER(dbl)]
    lib.sofia_sc_tune_batch.argtypes = [vp, ctypes.POINTER(Cube), i32, ctypes.POINTER(Kernel),
                                        i32, dbl, i32, i32, ctypes.POINTER(Options),
                                        ctypes.POINTER(BatchTuning)]
    lib.sofia_sc_tune_run.argtypes = [vp, vp, i64, i64, i64, ctypes.POINTER(Kernel), i32, dbl,
                                      i32, i32, vp, ctypes.POINTER(Options),
                                      ctypes.POINTER(BatchTuning)]
    lib.sofia_sc_set_shapes.argtypes = [vp, ctypes.POINTER(BatchTuning)]
    lib.sofia_sc_get_shapes.argtypes = [vp, ctypes.POINTER(BatchTuning)]
    lib.sofia_sc_step.argtypes = [vp, vp, i64, i64, i64, Kernel, dbl, i32, i32, dbl,
                                  dbl, vp, vp, ctypes.POINTER(dbl), vp]
    lib.sofia_sc_step_ex.argtypes = [vp, vp, i64, i64, i64, Kernel, dbl, i32, i32, vp, vp,
                                     ctypes.POINTER(dbl), ctypes.POINTER(Options)]
    lib.sofia_sc_smooth.argtypes = [vp, vp, i64, i64, i64, Kernel, dbl, dbl, vp, vp, vp]
    lib.sofia_sc_plan.argtypes = [dbl, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.sofia_sc_normalise.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i32, i32, i32,
                                       vp, vp, vp]
    lib.sofia_sc_link.argtypes = [vp, vp, i64, i64, i64, i32, i32, i32, i32, i32, i32, vp,
                                  ctypes.POINTER(i64), vp, i64, vp]
    lib.sofia_sc_check_run.argtypes = [i64, i64, i64, ctypes.POINTER(Kernel), i32, dbl, i32, i32,
                                       ctypes.POINTER(Options)]
    lib.sofia_sc_param_defaults.argtypes = [ctypes.POINTER(ParamOptions)]
    lib.sofia_sc_param_defaults.restype = None
    lib.sofia_sc_parameterise.argtypes = [vp, vp, vp, i64, i64, i64, i64,
                                          ctypes.POINTER(ParamOptions), vp,
                                          ctypes.POINTER(i64), vp]
    lib.sofia_sc_normalise_grid.argtypes = [i64, i64, i64, i32, i32, i32, i32,
                                            ctypes.POINTER(i64), ctypes.POINTER(i64),
                                            ctypes.POINTER(i64)]
    lib.sofia_sc_quantize.argtypes = [vp, vp, i64, dbl, i32, vp, vp]
    lib.sofia_sc_profile.argtypes = [vp, ctypes.c_int]
    lib.sofia_sc_profile_read.argtypes = [vp, ctypes.POINTER(KernelStat), i32,
                                          ctypes.POINTER(i32)]
    lib.sofia_sc_last_error.argtypes = [vp]
    lib.sofia_sc_last_error.restype = ctypes.c_char_p
    lib.sofia_sc_strerror.argtypes = [ctypes.c_int]
    lib.sofia_sc_strerror.restype = ctypes.c_char_p
    for name in ("sofia_sc_create", "sofia_sc_run", "sofia_sc_run_ex", "sofia_sc_run_noalloc",
                 "sofia_sc_run_batch",
                 "sofia_sc_tune_batch", "sofia_sc_tune_run", "sofia_sc_set_shapes",
                 "sofia_sc_get_shapes",
                 "sofia_sc_step",
                 "sofia_sc_step_ex",
                 "sofia_sc_smooth", "sofia_sc_plan", "sofia_sc_quantize", "sofia_sc_profile",
                 "sofia_sc_normalise", "sofia_sc_normalise_grid", "sofia_sc_link",
                 "sofia_sc_parameterise", "sofia_sc_check_run", "sofia_sc_profile_read"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _shapes_dict(t) -> dict:
    return {"lanes": t.lanes, "col_blocks": t.col_blocks, "strip_rows": t.strip_rows,
            "strip_waves": t.strip_waves, "col_min_planes": t.col_min_planes, "ms": t.ms}


class ScError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def plan(fwhm: float) -> Tuple[int, int]:
    """(n_iter, radius) of the spatial boxcar cascade for a FWHM."""
    n, r = ctypes.c_int32(), ctypes.c_int32()
    rc = load().sofia_sc_plan(float(fwhm), ctypes.byref(n), ctypes.byref(r))
    if rc != OK:
        raise ScError(rc, "bad spatial FWHM")
    return n.value, r.value


def _kernel(k) -> "Kernel":
    """A kernel from (FWHM, width) or (FWHM, width, kind); kind 0 / "cascade"
    = boxcar cascade, 1 / "gauss" = sampled Gaussian."""
    kind = k[2] if len(k) > 2 else 0
    kind = SPATIAL[kind] if isinstance(kind, str) else int(kind)
    return Kernel(float(k[0]), int(k[1]), kind)


def _kernels(kernels: Sequence[Tuple[float, int]]):
    arr = (Kernel * len(kernels))()
    for i, k in enumerate(kernels):
        arr[i] = _kernel(k)
    return arr


def _check_cube(cube):
    import torch
    if not (isinstance(cube, torch.Tensor) and cube.is_cuda and cube.dtype == torch.float32
            and cube.dim() == 3 and cube.is_contiguous()):
        raise ValueError("cube must be a contiguous 3-D float32 CUDA tensor [nz][ny][nx]")
    nz, ny, nx = cube.shape
    return nx, ny, nz


def _check_like(t, cube, dtype, what):
    """A caller-supplied mask/output must match the cube's shape and device."""
    import torch
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.dtype == dtype and t.is_contiguous()
            and t.shape == cube.shape and t.device == cube.device):
        raise ValueError(f"{what} must be a contiguous {dtype} tensor shaped like the cube")


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


class SofiaSC:
    """A library handle bound to one HIP device."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.h = ctypes.c_void_p()
        rc = self.lib.sofia_sc_create(ctypes.byref(self.h), int(device))
        if rc != OK:
            raise ScError(rc, "sofia_sc_create failed: " +
                          self.lib.sofia_sc_strerror(rc).decode())
        self.device = device

    def close(self):
        if self.h:
            self.lib.sofia_sc_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _raise(self, rc: int, what: str):
        msg = self.lib.sofia_sc_last_error(self.h).decode()
        raise ScError(rc, f"{what}: {msg or self.lib.sofia_sc_strerror(rc).decode()}")

    def run(self, cube, kernels, threshold: float, noise_mode: str = "mad",
            flux_range: str = "negative", replacement: float = 2.0, mask=None,
            stream=None, allow_nostat: bool = False, storage: str = "f32",
            sigma0: float = float("nan"), keep_input_mask: bool = False,
            noise_plane_stride: int = 0, fuse_widths: bool = False):
        """Whole S+C run. Returns (mask uint8 tensor, noise[K] ndarray, sigma0).

        keep_input_mask: OR the detections into the given mask instead of
        overwriting it. noise_plane_stride: measure every noise on every n-th
        plane only. fuse_widths: with replacement off and RMS noise, the pairs
        sharing a spatial kernel share their passes."""
        import torch
        nx, ny, nz = _check_cube(cube)
        _check_like(mask, cube, torch.uint8, "mask")
        if mask is None:
            mask = torch.empty(cube.shape, dtype=torch.uint8, device=cube.device)
        K = len(kernels)
        noise = (ctypes.c_double * K)()
        s0 = ctypes.c_double()
        opt = Options()
        self.lib.sofia_sc_default_options(ctypes.byref(opt))
        opt.replacement = float(replacement)
        opt.sigma0 = float(sigma0)
        opt.storage = STORAGE[storage]
        opt.keep_input_mask = 1 if keep_input_mask else 0
        opt.noise_plane_stride = int(noise_plane_stride)
        opt.fuse_widths = 1 if fuse_widths else 0
        opt.stream = _stream_ptr(stream)
        rc = self.lib.sofia_sc_run_ex(self.h, cube.data_ptr(), nx, ny, nz,
                                      _kernels(kernels), K, float(threshold),
                                      NOISE[noise_mode], RANGE[flux_range],
                                      mask.data_ptr(), noise, ctypes.byref(opt),
                                      ctypes.byref(s0))
        if rc != OK and not (allow_nostat and rc == ENOSTAT):
            self._raise(rc, "sofia_sc_run_ex")
        return mask, np.array(noise[:], dtype=np.float64), s0.value

    def run_noalloc(self, cube, kernels, threshold: float, noise_mode: str = "mad",
                    flux_range: str = "negative", replacement: float = 2.0, mask=None,
                    stream=None, allow_nostat: bool = False, storage: str = "f32",
                    sigma0: float = float("nan"), keep_input_mask: bool = False,
                    noise_plane_stride: int = 0):
        """run() through sofia_sc_run_noalloc: no device allocation by the
        library (workspace in its fixed device scratch array). The caller
        supplies the mask (and the cube): allocating them is the caller's."""
        import torch
        nx, ny, nz = _check_cube(cube)
        if mask is None:
            raise ValueError("run_noalloc: the caller supplies the mask")
        _check_like(mask, cube, torch.uint8, "mask")
        K = len(kernels)
        noise = (ctypes.c_double * K)()
        s0 = ctypes.c_double()
        opt = self._options(replacement, sigma0, storage, stream, keep_input_mask,
                            noise_plane_stride)
        rc = self.lib.sofia_sc_run_noalloc(self.h, cube.data_ptr(), nx, ny, nz,
                                           _kernels(kernels), K, float(threshold),
                                           NOISE[noise_mode], RANGE[flux_range],
                                           mask.data_ptr(), noise, ctypes.byref(opt),
                                           ctypes.byref(s0))
        if rc != OK and not (allow_nostat and rc == ENOSTAT):
            self._raise(rc, "sofia_sc_run_noalloc")
        return mask, np.array(noise[:], dtype=np.float64), s0.value

    def _batch_args(self, cubes, masks):
        import torch
        n = len(cubes)
        if masks is None:
            masks = [torch.empty(c.shape, dtype=torch.uint8, device=c.device) for c in cubes]
        if len(masks) != n:
            raise ValueError("one mask per cube")
        desc = (Cube * n)()
        for i, (c, m) in enumerate(zip(cubes, masks)):
            nx, ny, nz = _check_cube(c)
            _check_like(m, c, torch.uint8, "mask")
            desc[i].cube, desc[i].nx, desc[i].ny, desc[i].nz = c.data_ptr(), nx, ny, nz
            desc[i].mask = m.data_ptr()
        return desc, masks

    def _options(self, replacement, sigma0, storage, stream, keep_input_mask=False,
                 noise_plane_stride=0):
        opt = Options()
        self.lib.sofia_sc_default_options(ctypes.byref(opt))
        opt.replacement = float(replacement)
        opt.sigma0 = float(sigma0)
        opt.storage = STORAGE[storage]
        opt.keep_input_mask = 1 if keep_input_mask else 0
        opt.noise_plane_stride = int(noise_plane_stride)
        opt.stream = _stream_ptr(stream)
        return opt

    def tune_batch(self, cubes, kernels, threshold: float, noise_mode: str = "mad",
                   flux_range: str = "negative", replacement: float = 2.0, masks=None,
                   stream=None, storage: str = "f32", sigma0: float = float("nan")):
        """Autotune the launch shapes on this batch; returns the chosen
        {lanes, col_blocks, strip_rows, strip_waves, col_min_planes, ms}, kept
        by the handle for its later runs and batches."""
        desc, masks = self._batch_args(cubes, masks)
        opt = self._options(replacement, sigma0, storage, stream)
        best = BatchTuning()
        rc = self.lib.sofia_sc_tune_batch(self.h, desc, len(cubes), _kernels(kernels),
                                          len(kernels), float(threshold), NOISE[noise_mode],
                                          RANGE[flux_range], ctypes.byref(opt),
                                          ctypes.byref(best))
        if rc != OK and rc != ENOSTAT:
            self._raise(rc, "sofia_sc_tune_batch")   # switched off in this build
        return _shapes_dict(best)

    def tune_run(self, cube, kernels, threshold: float, noise_mode: str = "mad",
                 flux_range: str = "negative", replacement: float = 2.0, mask=None,
                 stream=None, storage: str = "f32", sigma0: float = float("nan")):
        """Autotune the launch shapes of whole runs on this cube; returns the
        chosen shapes (kept by the handle for its later calls)."""
        import torch
        nx, ny, nz = _check_cube(cube)
        _check_like(mask, cube, torch.uint8, "mask")
        if mask is None:
            mask = torch.empty(cube.shape, dtype=torch.uint8, device=cube.device)
        opt = self._options(replacement, sigma0, storage, stream)
        best = BatchTuning()
        rc = self.lib.sofia_sc_tune_run(self.h, cube.data_ptr(), nx, ny, nz, _kernels(kernels),
                                        len(kernels), float(threshold), NOISE[noise_mode],
                                        RANGE[flux_range], mask.data_ptr(), ctypes.byref(opt),
                                        ctypes.byref(best))
        if rc != OK and rc != ENOSTAT:
            self._raise(rc, "sofia_sc_tune_run")
        return _shapes_dict(best)

    def set_shapes(self, shapes=None):
        """Set the handle's launch shapes (dict as returned by tune_run), or
        the defaults for None."""
        if shapes is None:
            rc = self.lib.sofia_sc_set_shapes(self.h, None)
        else:
            t = BatchTuning()
            for k in ("lanes", "col_blocks", "strip_rows", "strip_waves", "col_min_planes"):
                setattr(t, k, int(shapes[k]))
            rc = self.lib.sofia_sc_set_shapes(self.h, ctypes.byref(t))
        if rc != OK:
            self._raise(rc, "sofia_sc_set_shapes")

    def shapes(self):
        t = BatchTuning()
        rc = self.lib.sofia_sc_get_shapes(self.h, ctypes.byref(t))
        if rc != OK:
            self._raise(rc, "sofia_sc_get_shapes")
        return _shapes_dict(t)

    def run_batch(self, cubes, kernels, threshold: float, noise_mode: str = "mad",
                  flux_range: str = "negative", replacement: float = 2.0, masks=None,
                  stream=None, allow_nostat: bool = False, storage: str = "f32",
                  sigma0: float = float("nan"), keep_input_mask: bool = False,
                  noise_plane_stride: int = 0):
        """Independent S+C runs of many cubes in one graph launch.

        Returns (list of mask tensors, noise[n_cubes, K] ndarray, sigma0[n_cubes])."""
        n = len(cubes)
        desc, masks = self._batch_args(cubes, masks)
        K = len(kernels)
        noise = (ctypes.c_double * (n * K))()
        s0 = (ctypes.c_double * n)()
        opt = self._options(replacement, sigma0, storage, stream, keep_input_mask,
                            noise_plane_stride)
        rc = self.lib.sofia_sc_run_batch(self.h, desc, n, _kernels(kernels), K,
                                         float(threshold), NOISE[noise_mode],
                                         RANGE[flux_range], noise, ctypes.byref(opt), s0)
        if rc != OK and not (allow_nostat and rc == ENOSTAT):
            self._raise(rc, "sofia_sc_run_batch")
        return (masks, np.array(noise[:], dtype=np.float64).reshape(n, K),
                np.array(s0[:], dtype=np.float64))

    def step(self, cube, kernel, threshold: float, noise_mode: str, flux_range: str,
             replacement: float = 2.0, sigma0: float = float("nan"), mask_in=None,
             mask_out=None, stream=None, allow_nostat: bool = False):
        """One S+C iteration from a given state. Returns (mask_out, noise)."""
        import torch
        nx, ny, nz = _check_cube(cube)
        _check_like(mask_in, cube, torch.uint8, "mask_in")
        _check_like(mask_out, cube, torch.uint8, "mask_out")
        if mask_out is None:
            mask_out = torch.empty(cube.shape, dtype=torch.uint8, device=cube.device)
        noise = ctypes.c_double()
        k = _kernel(kernel)
        rc = self.lib.sofia_sc_step(self.h, cube.data_ptr(), nx, ny, nz, k,
                                    float(threshold), NOISE[noise_mode],
                                    RANGE[flux_range], float(replacement), float(sigma0),
                                    None if mask_in is None else mask_in.data_ptr(),
                                    mask_out.data_ptr(), ctypes.byref(noise),
                                    _stream_ptr(stream))
        if rc != OK and not (allow_nostat and rc == ENOSTAT):
            self._raise(rc, "sofia_sc_step")
        return mask_out, noise.value

    def step_ex(self, cube, kernel, threshold: float, noise_mode: str, flux_range: str,
                mask_in=None, mask_out=None, replacement: float = 2.0,
                sigma0: float = float("nan"), storage: str = "f32", stream=None,
                allow_nostat: bool = False, noise_plane_stride: int = 0):
        """step with options (storage, noise subsampling). Returns (mask_out, noise)."""
        import torch
        nx, ny, nz = _check_cube(cube)
        _check_like(mask_in, cube, torch.uint8, "mask_in")
        _check_like(mask_out, cube, torch.uint8, "mask_out")
        if mask_out is None:
            mask_out = torch.empty(cube.shape, dtype=torch.uint8, device=cube.device)
        noise = ctypes.c_double()
        opt = Options()
        self.lib.sofia_sc_default_options(ctypes.byref(opt))
        opt.replacement = float(replacement)
        opt.sigma0 = float(sigma0)
        opt.storage = STORAGE[storage]
        opt.noise_plane_stride = int(noise_plane_stride)
        opt.stream = _stream_ptr(stream)
        k = _kernel(kernel)
        rc = self.lib.sofia_sc_step_ex(self.h, cube.data_ptr(), nx, ny, nz, k,
                                       float(threshold), NOISE[noise_mode], RANGE[flux_range],
                                       None if mask_in is None else mask_in.data_ptr(),
                                       mask_out.data_ptr(), ctypes.byref(noise),
                                       ctypes.byref(opt))
        if rc != OK and not (allow_nostat and rc == ENOSTAT):
            self._raise(rc, "sofia_sc_step_ex")
        return mask_out, noise.value

    def smooth(self, cube, kernel, replacement: float = -1.0,
               sigma0: float = float("nan"), mask_in=None, out=None, stream=None):
        """Smoothed cube s (float32, NaN at blanked voxels) of one kernel."""
        import torch
        nx, ny, nz = _check_cube(cube)
        _check_like(mask_in, cube, torch.uint8, "mask_in")
        _check_like(out, cube, torch.float32, "out")
        if out is None:
            out = torch.empty(cube.shape, dtype=torch.float32, device=cube.device)
        k = _kernel(kernel)
        rc = self.lib.sofia_sc_smooth(self.h, cube.data_ptr(), nx, ny, nz, k,
                                      float(replacement), float(sigma0),
                                      None if mask_in is None else mask_in.data_ptr(),
                                      out.data_ptr(), _stream_ptr(stream))
        if rc != OK:
            self._raise(rc, "sofia_sc_smooth")
        return out

    def normalise(self, cube, window_xy: int = 31, window_z: int = 31, grid_xy: int = 0,
                  grid_z: int = 0, noise_mode: str = "mad", flux_range: str = "negative",
                  out=None, grid: bool = True, stream=None):
        """Local noise normalisation (Sect. 4.1). Returns (normalised cube
        tensor or None, noise grid [nbz][nby][nbx] ndarray or None). out may
        be the cube itself (in place); out=False skips the division."""
        import torch
        nx, ny, nz = _check_cube(cube)
        if out is None:
            out = torch.empty_like(cube)
        elif out is not False:
            _check_like(out, cube, torch.float32, "out")
        g = None
        if grid:
            nb = [ctypes.c_int64() for _ in range(3)]
            rc = self.lib.sofia_sc_normalise_grid(nx, ny, nz, int(window_xy), int(window_z),
                                                  int(grid_xy), int(grid_z), *map(ctypes.byref, nb))
            if rc != OK:
                raise ScError(rc, "sofia_sc_normalise_grid: bad settings")
            g = np.empty((nb[2].value, nb[1].value, nb[0].value), dtype=np.float64)
        rc = self.lib.sofia_sc_normalise(self.h, cube.data_ptr(), nx, ny, nz, int(window_xy),
                                         int(window_z), int(grid_xy), int(grid_z),
                                         NOISE[noise_mode], RANGE[flux_range],
                                         None if out is False else out.data_ptr(),
                                         None if g is None else g.ctypes.data,
                                         _stream_ptr(stream))
        if rc != OK:
            self._raise(rc, "sofia_sc_normalise")
        return (None if out is False else out), g

    def link(self, mask, radius_xy: int = 2, radius_z: int = 2, min_size_xy: int = 0,
             min_size_z: int = 0, max_size_xy: int = 0, max_size_z: int = 0, labels=None,
             boxes: bool = True, stream=None):
        """Friends-of-friends linker (Sect. 4.3). Returns (int32 label tensor,
        number of kept detections, [n][7] int64 boxes or None)."""
        import torch
        if not (isinstance(mask, torch.Tensor) and mask.is_cuda and mask.dtype == torch.uint8
                and mask.dim() == 3 and mask.is_contiguous()):
            raise ValueError("mask must be a contiguous 3-D uint8 CUDA tensor [nz][ny][nx]")
        nz, ny, nx = mask.shape
        if labels is None:
            labels = torch.empty(mask.shape, dtype=torch.int32, device=mask.device)
        elif not (labels.dtype == torch.int32 and labels.is_contiguous()
                  and labels.shape == mask.shape and labels.device == mask.device):
            raise ValueError("labels must be a contiguous int32 tensor shaped like the mask")
        n = ctypes.c_int64()
        cap = 0
        out = None
        if boxes:
            cap = int(torch.count_nonzero(mask).item())
            out = np.empty((max(cap, 1), 7), dtype=np.int64)
        rc = self.lib.sofia_sc_link(self.h, mask.data_ptr(), nx, ny, nz, int(radius_xy),
                                    int(radius_z), int(min_size_xy), int(min_size_z),
                                    int(max_size_xy), int(max_size_z), labels.data_ptr(),
                                    ctypes.byref(n), None if out is None else out.ctypes.data,
                                    cap, _stream_ptr(stream))
        if rc != OK:
            self._raise(rc, "sofia_sc_link")
        return labels, n.value, (None if out is None else out[:n.value].copy())

    def parameterise(self, cube, labels, n: int, channel_width: float = 1.0,
                     beam=(0.0, 0.0), sigma_rms: float = 1.0, scale: float = 0.4,
                     rel_threshold: float = 0.9, snr_threshold: float = 2.8, out=None,
                     stream=None):
        """Parameters and reliability of detections 1..n (Sect. 4.4, 4.5).
        Returns (dict of per-detection NumPy arrays keyed like SOURCE_DTYPE's
        fields, number kept); out, if given, is a uint8 CUDA tensor of at
        least n * SOURCE_DTYPE.itemsize bytes that receives the records."""
        import torch
        if not (isinstance(cube, torch.Tensor) and cube.is_cuda and cube.dtype == torch.float32
                and cube.dim() == 3 and cube.is_contiguous()):
            raise ValueError("cube must be a contiguous 3-D float32 CUDA tensor [nz][ny][nx]")
        if not (isinstance(labels, torch.Tensor) and labels.dtype == torch.int32
                and labels.is_contiguous() and labels.shape == cube.shape
                and labels.device == cube.device):
            raise ValueError("labels must be a contiguous int32 tensor shaped like the cube")
        n = int(n)
        nz, ny, nx = cube.shape
        size = max(n, 1) * SOURCE_DTYPE.itemsize
        if out is None:
            out = torch.empty(size, dtype=torch.uint8, device=cube.device)
        elif not (out.dtype == torch.uint8 and out.is_contiguous() and out.numel() >= size
                  and out.device == cube.device):
            raise ValueError("out must be a contiguous uint8 tensor of n records")
        o = ParamOptions()
        self.lib.sofia_sc_param_defaults(ctypes.byref(o))
        o.channel_width = float(channel_width)
        o.beam_major_px, o.beam_minor_px = float(beam[0]), float(beam[1])
        o.sigma_rms = float(sigma_rms)
        o.rel_scale = float(scale)
        o.rel_threshold = float(rel_threshold)
        o.snr_threshold = float(snr_threshold)
        kept = ctypes.c_int64()
        rc = self.lib.sofia_sc_parameterise(self.h, cube.data_ptr(), labels.data_ptr(), nx, ny,
                                            nz, n, ctypes.byref(o), out.data_ptr(),
                                            ctypes.byref(kept), _stream_ptr(stream))
        if rc != OK:
            self._raise(rc, "sofia_sc_parameterise")
        rec = out[:n * SOURCE_DTYPE.itemsize].cpu().numpy().view(SOURCE_DTYPE)
        return {k: rec[k].copy() for k in SOURCE_DTYPE.names if k != "pad"}, kept.value

    def quantize(self, cube, scale: float, storage: str = "f16", out=None, stream=None):
        """The 16-bit noise-scaled copy a F16/BF16 run stores (uint16 bit patterns)."""
        import torch
        if not (isinstance(cube, torch.Tensor) and cube.is_cuda and cube.dtype == torch.float32
                and cube.is_contiguous()):
            raise ValueError("cube must be a contiguous float32 CUDA tensor")
        if out is None:
            out = torch.empty(cube.shape, dtype=torch.int16, device=cube.device)
        if not (out.dtype == torch.int16 and out.is_contiguous() and
                out.numel() == cube.numel() and out.device == cube.device):
            raise ValueError("out must be a contiguous int16 tensor of the cube's size")
        rc = self.lib.sofia_sc_quantize(self.h, cube.data_ptr(), cube.numel(), float(scale),
                                        STORAGE[storage], out.data_ptr(), _stream_ptr(stream))
        if rc != OK:
            self._raise(rc, "sofia_sc_quantize")
        return out

    def profile(self, enable: bool):
        rc = self.lib.sofia_sc_profile(self.h, 1 if enable else 0)
        if rc != OK:
            self._raise(rc, "sofia_sc_profile")

    def profile_read(self) -> List[dict]:
        cap = 32
        arr = (KernelStat * cap)()
        n = ctypes.c_int32()
        rc = self.lib.sofia_sc_profile_read(self.h, arr, cap, ctypes.byref(n))
        if rc != OK:
            self._raise(rc, "sofia_sc_profile_read")
        return [dict(name=arr[i].name.decode(), launches=arr[i].launches,
                     total_ms=arr[i].total_ms, bytes=arr[i].bytes,
                     voxels=arr[i].voxels) for i in range(min(n.value, cap))]
