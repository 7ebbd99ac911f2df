"""sofia_sc_run_noalloc: the whole-run entry point that allocates nothing.

Its workspace lives in the library's fixed device scratch array, so it must
give exactly what sofia_sc_run_ex gives (same launches, same arithmetic): the
masks, noise values and sigma_0 of two calls in a row, the second on a smaller
cube (the array keeps the first call's contents), are compared bit for bit
with sofia_sc_run_ex on the same inputs. Oversized cubes are refused with
EINVAL before any device work.
"""
import ctypes
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

KERNELS = [(float(f), w) for f in (0, 3, 6) for w in (0, 3, 7, 15)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _cube(nx, ny, nz, seed, n_gal, border):
    spec = synth.CubeSpec(nx, ny, nz, seed=seed, radial=True, sigma_lo=0.8, sigma_hi=1.5,
                          n_gal=n_gal, nan_border=border)
    return torch.from_numpy(synth.generate(spec)).cuda()


def _same(a, b, what):
    (ma, na, sa), (mb, nb, sb) = a, b
    torch.cuda.synchronize()
    assert torch.equal(ma, mb), f"{what}: masks differ"
    np.testing.assert_array_equal(na, nb, err_msg=f"{what}: noise")
    assert (np.isnan(sa) and np.isnan(sb)) or sa == sb, f"{what}: sigma_0"


def test_noalloc_equals_run_ex_on_two_calls_second_smaller():
    h = sc.SofiaSC(0)
    try:
        big = _cube(200, 150, 110, seed=81, n_gal=8, border=3)     # 3.3e6 voxels
        small = _cube(64, 64, 128, seed=82, n_gal=5, border=0)     # 5.2e5 voxels
        cases = [
            (big, KERNELS, 3.5, "mad", "negative", 2.0, {}),
            (small, [(0.0, 0), (0.0, 3), (0.0, 7), (3.0, 0), (3.0, 3), (3.0, 7)], 4.0, "std",
             "all", 2.0, {}),
        ]
        for i, (x, kern, t, mode, rng_, repl, kw) in enumerate(cases):
            say(f"call {i}: {tuple(x.shape)} {mode} {rng_}")
            m_ref = torch.full(x.shape, 0x55, dtype=torch.uint8, device="cuda")
            ref = h.run(x, kern, t, mode, rng_, repl, mask=m_ref, **kw)
            m = torch.full(x.shape, 0xAA, dtype=torch.uint8, device="cuda")
            got = h.run_noalloc(x, kern, t, mode, rng_, repl, mask=m, **kw)
            _same(got, ref, f"call {i}")
            say(f"  noise {np.array2string(got[1][:3], precision=4)}..., "
                f"{int(m.sum().item())} detections: equal to sofia_sc_run_ex")
        # options through the scratch path: 16-bit storage, kept input mask,
        # replacement off, after the calls above
        prior = (torch.rand(small.shape, device="cuda") < 0.05).to(torch.uint8) * 3
        for kw in ({"storage": "f16"}, {"keep_input_mask": True}, {"replacement": -1.0}):
            m_ref = prior.clone()
            ref = h.run(small, KERNELS[:6], 3.5, "mad", "negative", mask=m_ref, **kw)
            m = prior.clone()
            got = h.run_noalloc(small, KERNELS[:6], 3.5, "mad", "negative", mask=m, **kw)
            _same(got, ref, f"options {kw}")
    finally:
        h.close()


def test_noalloc_refuses_oversized_cubes():
    h = sc.SofiaSC(0)
    try:
        opt = sc.Options()
        h.lib.sofia_sc_default_options(ctypes.byref(opt))
        # more voxels than SOFIA_SC_NOALLOC_MAX_VOXELS (real buffers of that size)
        for (nx, ny, nz), kern, word in [((2049, 2048, 1), [(0.0, 0)], "MAX_VOXELS"),
                                         ((1, 1, 1 << 22), [(3.0, 0)], "workspace")]:
            x = torch.zeros((nz, ny, nx), dtype=torch.float32, device="cuda")
            m = torch.zeros((nz, ny, nx), dtype=torch.uint8, device="cuda")
            noise = (ctypes.c_double * 1)()
            rc = h.lib.sofia_sc_run_noalloc(h.h, x.data_ptr(), nx, ny, nz, sc._kernels(kern),
                                            1, 3.0, 0, 0, m.data_ptr(), noise,
                                            ctypes.byref(opt), None)
            msg = h.lib.sofia_sc_last_error(h.h).decode()
            say(f"{(nx, ny, nz)}: rc {rc}, '{msg}'")
            assert rc == sc.EINVAL and word in msg
            assert np.isnan(noise[0])
            assert int(m.sum().item()) == 0
        # the handle and the entry point still work
        x = _cube(40, 30, 20, seed=83, n_gal=1, border=0)
        ref = h.run(x, KERNELS[:4], 3.5, "mad", "negative")
        got = h.run_noalloc(x, KERNELS[:4], 3.5, "mad", "negative",
                            mask=torch.empty(x.shape, dtype=torch.uint8, device="cuda"))
        _same(got, ref, "after refusals")
    finally:
        h.close()
