"""C ABI of libsofia_sc.so on the CPU: load, exports, host-only entry points."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2106_15789_amd as sc


def _declared_functions():
    text = open(sc.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sofia_sc_\w+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = sc.load()
    declared = _declared_functions()
    assert declared == sorted(sc.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


def test_plan_matches_oracle_reading():
    for f in list(np.linspace(0.1, 13.0, 130)) + [3, 5, 6, 9, 10, 0]:
        assert sc.plan(float(f)) == oracle.plan(float(f)), f


def test_plan_rejects_bad_fwhm():
    for f in (-0.5, float("nan"), float("inf")):
        with pytest.raises(sc.ScError) as e:
            sc.plan(f)
        assert e.value.code == sc.EINVAL


def test_strerror_and_null_handle_paths():
    lib = sc.load()
    for code in (sc.OK, sc.EINVAL, sc.ENOMEM, sc.EDEVICE, sc.ENOSTAT):
        assert lib.sofia_sc_strerror(code)
    lib.sofia_sc_destroy(None)                      # NULL is a no-op
    assert lib.sofia_sc_last_error(None) == b"NULL handle"
    assert lib.sofia_sc_profile(None, 1) == sc.EINVAL
    n = ctypes.c_int32()
    assert lib.sofia_sc_profile_read(None, None, 0, ctypes.byref(n)) == sc.EINVAL
    assert lib.sofia_sc_create(None, 0) == sc.EINVAL
    noise = (ctypes.c_double * 1)()
    k = (sc.Kernel * 1)()
    assert lib.sofia_sc_run(None, None, 1, 1, 1, k, 1, 3.0, 0, 0, None, noise) == sc.EINVAL
    cubes = (sc.Cube * 1)()
    assert lib.sofia_sc_run_batch(None, cubes, 1, k, 1, 3.0, 0, 0, noise, None,
                                  None) == sc.EINVAL


def test_batch_tuning_layout_matches_header():
    """sofia_sc_batch_tuning: six int32 fields, then a double (32 bytes)."""
    assert ctypes.sizeof(sc.BatchTuning) == 32
    assert [f for f, _ in sc.BatchTuning._fields_] == ["lanes", "col_blocks", "strip_rows",
                                                       "strip_waves", "col_min_planes",
                                                       "reserved", "ms"]
    lib = sc.load()
    cubes = (sc.Cube * 1)()
    k = (sc.Kernel * 1)()
    assert lib.sofia_sc_tune_batch(None, cubes, 1, k, 1, 3.0, 0, 0, None, None) == sc.EINVAL


def test_cube_descriptor_layout_matches_header():
    """sofia_sc_cube: pointer, three int64 dimensions, pointer (40 bytes)."""
    assert ctypes.sizeof(sc.Cube) == 40
    assert [f for f, _ in sc.Cube._fields_] == ["cube", "nx", "ny", "nz", "mask"]
    text = open(sc.HEADER).read()
    body = text[text.index("typedef struct {\n    const float *cube;"):]
    body = body[:body.index("} sofia_sc_cube;")]
    assert re.findall(r"\b(cube|nx|ny|nz|mask)\b[,;]", body) == ["cube", "nx", "ny", "nz",
                                                                   "mask"]


def test_default_options():
    opt = sc.Options()
    sc.load().sofia_sc_default_options(ctypes.byref(opt))
    assert opt.struct_size == ctypes.sizeof(sc.Options)
    assert opt.replacement == 2.0
    assert opt.keep_input_mask == 0
    assert not opt.stream


def test_binding_has_no_compute_fallback():
    """The binding only marshals: it must not import the oracle or numpy math."""
    src = open(os.path.join(os.path.dirname(sc.__file__), "__init__.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_param_layouts_and_defaults():
    """sofia_sc_source: int64 count, eleven doubles, two int32 (104 bytes) in
    header order; sofia_sc_param_options: two int32, seven doubles (64 bytes);
    defaults of the mock-galaxy run (Sect. 6)."""
    assert sc.SOURCE_DTYPE.itemsize == 104
    text = open(sc.HEADER).read()
    body = text[text.index("typedef struct {\n    int64_t n_vox;"):]
    body = body[:body.index("} sofia_sc_source;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = re.findall(r"(\w+)[,;]", body)
    assert names == ["n_vox", "sum", "peak", "min", "mean", "x", "y", "z", "flux", "flux_err",
                     "snr", "reliability", "kept", "pad"]
    assert list(sc.SOURCE_DTYPE.names) == ["count"] + names[1:]
    assert ctypes.sizeof(sc.ParamOptions) == 64
    o = sc.ParamOptions()
    lib = sc.load()
    lib.sofia_sc_param_defaults(ctypes.byref(o))
    assert o.struct_size == 64
    assert (o.channel_width, o.sigma_rms, o.rel_scale, o.rel_threshold, o.snr_threshold) == \
        (1.0, 1.0, 0.4, 0.9, 2.8)
    assert (o.beam_major_px, o.beam_minor_px) == (0.0, 0.0)
    n = ctypes.c_int64(5)
    assert lib.sofia_sc_parameterise(None, None, None, 1, 1, 1, 1, ctypes.byref(o), None,
                                     ctypes.byref(n), None) == sc.EINVAL


def _check(nx, ny, nz, kernels=((0.0, 0),), t=3.0, mode=0, rng=0, **opt_fields):
    """sofia_sc_check_run: the argument checks sofia_sc_run_ex runs before any
    device work (the same code), with no handle, device or buffer."""
    lib = sc.load()
    opt = sc.Options()
    lib.sofia_sc_default_options(ctypes.byref(opt))
    for k, v in opt_fields.items():
        setattr(opt, k, v)
    return lib.sofia_sc_check_run(nx, ny, nz, sc._kernels(list(kernels)), len(kernels), t, mode,
                                  rng, ctypes.byref(opt))


def test_run_argument_checks_without_buffers():
    assert _check(64, 64, 64) == sc.OK
    assert _check(2048, 2048, 4096, [(9.0, 31), (14.0, 0, "gauss")]) == sc.OK
    assert _check(1 << 14, 1 << 14, 1 << 12) == sc.OK              # 2^40 voxels
    for dims in [(0, 4, 4), (4, 0, 4), (4, 4, 0), (-1, 4, 4),
                 (16385, 16385, 1),                                # plane above 2^28
                 (1 << 14, 1 << 14, 1 << 13)]:                     # 2^41 voxels
        assert _check(*dims) == sc.EINVAL, dims
    for kernels in [[(0.0, 4)], [(-1.0, 0)], [(40.0, 0)], [(0.0, 65)], [(float("nan"), 0)],
                    [(3.0, 0, 2)], [(14.5, 0, "gauss")], []]:
        assert _check(16, 16, 16, kernels or [(0.0, 0)] * 65) == sc.EINVAL, kernels
    for t in (0.0, -1.0, float("nan"), float("inf")):
        assert _check(16, 16, 16, t=t) == sc.EINVAL, t
    assert _check(16, 16, 16, mode=2) == sc.EINVAL
    assert _check(16, 16, 16, rng=3) == sc.EINVAL
    for fields in [dict(struct_size=8), dict(keep_input_mask=2), dict(storage=7),
                   dict(sigma0=-1.0), dict(noise_plane_stride=-1), dict(fuse_widths=2),
                   dict(fuse_widths=1),                          # replacement on
                   dict(fuse_widths=1, replacement=-1.0, storage=1)]:
        assert _check(16, 16, 16, **fields) == sc.EINVAL, fields
    assert _check(16, 16, 16, mode=1, fuse_widths=1, replacement=-1.0) == sc.OK
    assert _check(16, 16, 16, fuse_widths=1, replacement=-1.0) == sc.OK
