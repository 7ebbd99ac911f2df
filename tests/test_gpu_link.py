"""GPU parity of the friends-of-friends linker (Sect. 4.3) against the CPU
oracle, through the C ABI (sofia_sc_link). The labels are canonical (a
detection's number is the raster rank of its first voxel among the kept
detections), so label cubes, counts and boxes must be equal bit for bit."""
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


def check(h, mask, r_xy, r_z, filt=(0, 0, 0, 0), what=""):
    lab_ref, n_ref, box_ref = oracle.link(mask, r_xy, r_z, *filt)
    md = torch.from_numpy(np.ascontiguousarray(mask)).cuda()
    lab, n, boxes = h.link(md, r_xy, r_z, *filt)
    assert n == n_ref, f"{what}: {n} detections, oracle {n_ref}"
    np.testing.assert_array_equal(lab.cpu().numpy(), lab_ref, err_msg=what)
    np.testing.assert_array_equal(boxes, box_ref, err_msg=what)
    return n


RADII = [(1, 1), (2, 2), (2, 1), (1, 3), (0, 2), (3, 0), (4, 4), (0, 0)]


@pytest.mark.parametrize("r_xy,r_z", RADII)
def test_random_masks(h, r_xy, r_z):
    rng = np.random.default_rng(100 * r_xy + r_z)
    for shape, p in [((20, 30, 40), 0.02), ((16, 33, 65), 0.1), ((9, 70, 71), 0.3),
                     ((40, 1, 50), 0.2), ((1, 1, 300), 0.5), ((7, 9, 11), 0.9)]:
        mask = (rng.random(shape) < p).astype(np.uint8)
        for filt in [(0, 0, 0, 0), (3, 2, 0, 0), (2, 1, 10, 6)]:
            check(h, mask, r_xy, r_z, filt, f"{shape} p={p} r=({r_xy},{r_z}) filt={filt}")


def test_edge_masks(h):
    for shape in [(1, 1, 1), (3, 4, 5)]:
        check(h, np.zeros(shape, np.uint8), 2, 2, what=f"empty {shape}")
        check(h, np.ones(shape, np.uint8), 2, 2, what=f"full {shape}")
    m = np.zeros((5, 6, 7), np.uint8)
    m[2, 3, 4] = 1
    assert check(h, m, 2, 2, (1, 1, 0, 0), "single voxel") == 1
    assert check(h, m, 2, 2, (2, 1, 0, 0), "single voxel, min 2") == 0
    # mask bytes other than 1 count as detected
    rng = np.random.default_rng(9)
    m = rng.choice(np.array([0, 1, 2, 255], np.uint8), size=(10, 12, 14), p=[0.85, 0.05, 0.05, 0.05])
    check(h, m, 2, 2, what="bytes 2 and 255")


def test_sc_mask_with_the_mock_run_settings(h):
    """The S+C mask of a cube of the 1024^3 recipe (GPU run), linked with the
    settings of the paper's mock-galaxy run: radius 2, minimum 8 pixels and 5
    channels (Sect. 6); repeated runs give the same labels."""
    spec = synth.CubeSpec(300, 260, 240, seed=2, radial=True, sigma_lo=0.8, sigma_hi=1.5,
                          n_gal=30, nan_border=4)
    x = torch.from_numpy(synth.generate(spec)).cuda()
    kern = [(float(f), w) for f in (0, 3, 6) for w in (0, 3, 7, 15)]
    m, _, _ = h.run(x, kern, 3.5, "mad", "negative")
    mask = m.cpu().numpy()
    n = check(h, mask, 2, 2, (8, 5, 0, 0), "S+C mask, mock-run settings")
    n_all = check(h, mask, 2, 2, what="S+C mask, no size filter")
    lab1, _, _ = h.link(m, 2, 2, 8, 5)
    lab2, _, _ = h.link(m, 2, 2, 8, 5)
    assert torch.equal(lab1, lab2)
    say(f"S+C mask {mask.shape}: {int(mask.sum())} detected voxels, {n_all} detections, "
        f"{n} kept with min 8 px / 5 ch")


def test_bad_arguments(h):
    m = torch.zeros((4, 4, 4), dtype=torch.uint8, device="cuda")
    for args in [(-1, 2, 0, 0, 0, 0), (2, 5, 0, 0, 0, 0), (2, 2, -1, 0, 0, 0),
                 (2, 2, 0, 0, 0, -3)]:
        with pytest.raises(sc.ScError) as e:
            h.link(m, *args)
        assert e.value.code == sc.EINVAL, args
    # 2^31 voxels (real buffers): beyond the int32 forest
    big = torch.zeros((1024, 1024, 2048), dtype=torch.uint8, device="cuda")
    lab = torch.empty((1024, 1024, 2048), dtype=torch.int32, device="cuda")
    with pytest.raises(sc.ScError) as e:
        h.link(big, 2, 2, labels=lab, boxes=False)
    assert e.value.code == sc.EINVAL and "2^31" in str(e.value)
    del big, lab
    torch.cuda.empty_cache()
