"""GPU tests of how a run's detections reach the caller's byte mask: the
working state of a run is packed bits, and the caller's mask is written once
at the end (0/1, ORed into the caller's mask when it is kept, or, for one
step, the step's detections ORed with the incoming mask).

Checked against the FP64 oracle (masks equal outside the boundary band,
noise to 1e-6) and against the same call on an aligned mask (bit for bit)."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


def _cube(nx, ny, nz, seed):
    spec = synth.CubeSpec(nx, ny, nz, seed=seed, radial=True, sigma_lo=0.8, sigma_hi=1.5,
                          n_gal=4, nan_border=2)
    x = synth.generate(spec)
    rng = np.random.default_rng(seed)
    x[rng.random(x.shape) < 0.004] = np.nan
    return x


def _unaligned_like(shape, offset):
    """A contiguous uint8 tensor of `shape` whose data starts `offset` bytes
    into a larger allocation (not 16-byte aligned for offset % 16 != 0)."""
    n = int(np.prod(shape))
    buf = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
    return buf[offset:offset + n].view(shape)


@pytest.mark.parametrize("kernel", [(0.0, 0), (3.0, 7), (0.0, 15)])
def test_step_keeps_marks_on_blanked_voxels(h, kernel):
    """A step seeded with a mask that also marks blanked (non-finite) voxels:
    those voxels are never replaced, and the output holds the incoming marks
    ORed with the step's detections, like the oracle's step."""
    x = _cube(90, 70, 50, seed=41)
    rng = np.random.default_rng(7)
    mask = (rng.random(x.shape) < 0.02).astype(np.uint8)
    nan = ~np.isfinite(x)
    mask[nan & (rng.random(x.shape) < 0.5)] = 1           # marks on blanked voxels
    assert (mask.astype(bool) & nan).any()
    s0 = 0.9
    ref = oracle.step(x, kernel[0], kernel[1], 3.5, "mad", "negative", mask, 2.0, s0)
    out, sig = h.step(torch.from_numpy(x).cuda(), kernel, 3.5, "mad", "negative", 2.0, s0,
                      mask_in=torch.from_numpy(mask).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    assert abs(sig / ref.sigma - 1) <= 1e-6
    diff = (got != ref.mask) & (ref.band == 0)
    assert not diff.any(), f"{int(diff.sum())} mismatches outside the band"
    assert (got[mask.astype(bool)] == 1).all()
    assert got.max() <= 1
    say(f"step {kernel}: {int(got.sum())} voxels, {int((mask.astype(bool) & nan).sum())} "
        f"marks on blanked voxels kept")


@pytest.mark.parametrize("shape", [(40, 33, 65), (24, 64, 64)])
@pytest.mark.parametrize("offset", [1, 3, 16])
def test_run_into_unaligned_mask(h, shape, offset):
    """Whole runs (and keep_input_mask) into masks at odd byte offsets equal
    the same runs into aligned masks, bit for bit."""
    nz, ny, nx = shape
    x = torch.from_numpy(_cube(nx, ny, nz, seed=43 + offset)).cuda()
    kernels = [(0.0, 0), (0.0, 3), (3.0, 0), (3.0, 7)]
    ref = torch.empty(shape, dtype=torch.uint8, device="cuda")
    h.run(x, kernels, 3.5, "mad", "negative", 2.0, mask=ref)
    m = _unaligned_like(shape, offset)
    h.run(x, kernels, 3.5, "mad", "negative", 2.0, mask=m)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(m.cpu().numpy(), ref.cpu().numpy())
    # kept input mask: the run's detections ORed into bytes of other values
    rng = np.random.default_rng(offset)
    prior = rng.choice(np.array([0, 0, 0, 7, 255], np.uint8), size=shape)
    m2 = _unaligned_like(shape, offset)
    m2.copy_(torch.from_numpy(prior).cuda())
    h.run(x, kernels, 3.5, "mad", "negative", 2.0, mask=m2, keep_input_mask=True)
    torch.cuda.synchronize()
    want = prior | ref.cpu().numpy()
    np.testing.assert_array_equal(m2.cpu().numpy(), want)
    say(f"unaligned {shape} +{offset}: {int(ref.sum().item())} voxels")
