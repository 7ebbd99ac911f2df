"""Parity at the plane size of the 2048 x 2048 x 4096 workload.

The whole cube (64 GiB) is beyond what the oracle can take in a test, so the
check runs on its first 96 planes (the generator gives a slab the same values
as the whole cube): the spatial kernel works on 2048 x 2048 planes exactly as
in the full-size run, and the column kernels stream the same columns. On the
slab the oracle computes, in seconds:
  * step 1 (kernel (0, 0)): sigma_1 = sigma_0 and the plain threshold mask;
  * single S+C iterations of the widest kernels of that workload, (9, 31) and
    (9, 0), and of (3, 7), teacher-forced with the step-1 mask and sigma_0.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

PLANES = 96


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def slab():
    wl = synth.workload("large_2048x2048x4096")
    spec = wl.cubes[0]
    x = synth.generate(spec, z0=0, z1=PLANES)
    raw = np.where(np.isfinite(x), x, np.nan).astype(np.float64)
    s0, m = oracle.noise(raw, "mad", "negative")
    del raw
    ax = np.abs(x.astype(np.float64))
    m1 = (ax > 3.5 * s0).astype(np.uint8)
    band1 = (np.abs(ax / s0 - 3.5) <= 1e-5).astype(np.uint8)
    del ax
    say(f"large slab {x.shape}: sigma0 {s0}, selected {m}, step-1 detections {int(m1.sum())}")
    return x, s0, m1, band1


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def test_large_plane_first_step_exact(h, slab):
    x, s0, m1, band1 = slab
    out, s1 = h.step(torch.from_numpy(x).cuda(), (0.0, 0), 3.5, "mad", "negative", 2.0, s0)
    g = out.cpu().numpy()
    assert abs(s1 / s0 - 1) <= 1e-6
    assert int(((g != m1) & (band1 == 0)).sum()) == 0


@pytest.mark.parametrize("kernel", [(9.0, 31), (9.0, 0), (3.0, 7)])
def test_large_plane_teacher_forced_step(h, slab, kernel):
    x, s0, m1, _ = slab
    ref = oracle.step(x, kernel[0], kernel[1], 3.5, "mad", "negative", m1, 2.0, s0)
    out, sk = h.step(torch.from_numpy(x).cuda(), kernel, 3.5, "mad", "negative", 2.0, s0,
                     mask_in=torch.from_numpy(m1).cuda())
    g = out.cpu().numpy()
    diff = g != ref.mask
    say(f"large plane {kernel}: sigma rel {abs(sk / ref.sigma - 1):.2e}, band "
        f"{ref.band_count}, diff {int(diff.sum())}, detections {int(ref.mask.sum())}")
    assert abs(sk / ref.sigma - 1) <= 1e-6
    assert int((diff & (ref.band == 0)).sum()) == 0
