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
