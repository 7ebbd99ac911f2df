"""Pins of the friends-of-friends linker oracle (CPU only).

Sect. 4.3: detected voxels within a merging radius are linked, spatially and
spectrally, into detections with unique identifiers; size filters drop
detections that are too small or too large (radius 2 and minimum sizes of 8
pixels / 5 channels in the mock run of Sect. 6). Readings L1-L4 are stated
in oracle/link_oracle.cpp. Each test checks the oracle against something
other than itself: hand-drawn masks (tests/golden), scipy's 6-connected
labelling, the pairwise brute force of oracle/brute.py, and hand-built size
cases at the filter limits.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_hand_drawn_masks():
    with open(os.path.join(GOLDEN, "linker_hand.json")) as f:
        g = json.load(f)
    mask = np.zeros(g["shape"], np.uint8)
    for z, y, x in g["voxels"]:
        mask[z, y, x] = 1
    for case in g["cases"]:
        labels, n, boxes = oracle.link(mask, case["r_xy"], case["r_z"])
        got = [int(labels[z, y, x]) for z, y, x in g["voxels"]]
        assert got == case["labels"], case["note"]
        assert n == max(case["labels"])
        assert int((labels > 0).sum()) == len(g["voxels"])


def test_radius_one_is_six_connected_labelling():
    """r = 1 in every axis: the friends are the face neighbours, so the
    detections are scipy.ndimage.label's with its default (6-connected)
    structure, up to the numbering."""
    from scipy import ndimage
    rng = np.random.default_rng(1)
    for p in (0.1, 0.3, 0.5):
        mask = (rng.random((12, 13, 14)) < p).astype(np.uint8)
        labels, n, _ = oracle.link(mask, 1, 1)
        ref, nref = ndimage.label(mask)
        assert n == nref
        # same partition: a one-to-one map between the two labellings
        pairs = set(zip(labels[mask > 0].tolist(), ref[mask > 0].tolist()))
        assert len(pairs) == n
        # numbering in raster order of the first voxel
        first = [np.flatnonzero(labels.ravel() == k)[0] for k in range(1, n + 1)]
        assert first == sorted(first)


@pytest.mark.parametrize("r_xy,r_z", [(1, 1), (2, 2), (2, 1), (1, 3), (0, 2), (3, 0), (2, 4)])
def test_brute_force_agrees(r_xy, r_z):
    rng = np.random.default_rng(10 * r_xy + r_z)
    for shape, p in [((6, 7, 9), 0.08), ((5, 9, 8), 0.2), ((9, 5, 6), 0.35), ((1, 12, 13), 0.3)]:
        mask = (rng.random(shape) < p).astype(np.uint8)
        for filt in [(0, 0, 0, 0), (2, 2, 0, 0), (1, 1, 3, 2), (3, 1, 0, 4)]:
            got = oracle.link(mask, r_xy, r_z, *filt)
            ref = brute.link(mask, r_xy, r_z, *filt)
            np.testing.assert_array_equal(got[0], ref[0], err_msg=f"{shape} {filt}")
            assert got[1] == ref[1]
            np.testing.assert_array_equal(got[2], ref[2])


def _bar(nz, ny, nx, z0, y0, x0, ez, ey, ex, mask):
    mask[z0:z0 + ez, y0:y0 + ey, x0:x0 + ex] = 1


def test_size_filters_at_their_limits():
    """Boxes of known extents: a detection is kept when its extents along x
    and y are >= min_xy and along z >= min_z (and <= the maxima when those
    are set); one voxel less, or more, drops it."""
    mask = np.zeros((30, 40, 60), np.uint8)
    # (z0, y0, x0, ez, ey, ex): well apart from each other
    boxes = [(0, 0, 0, 5, 8, 8),     # at the minima
             (0, 0, 20, 4, 8, 8),    # one channel short
             (0, 0, 40, 5, 7, 8),    # one row short
             (0, 20, 0, 5, 8, 7),    # one column short
             (10, 20, 20, 12, 10, 9),  # larger
             (25, 20, 45, 5, 15, 8)]   # wider along y than max_xy = 12
    for b in boxes:
        _bar(30, 40, 60, *b, mask)
    labels, n, bb = oracle.link(mask, 2, 2, min_xy=8, min_z=5)
    kept = [b for b in boxes if b[3] >= 5 and b[4] >= 8 and b[5] >= 8]
    assert n == len(kept) == 3
    for (z0, y0, x0, ez, ey, ex), row in zip(sorted(kept), bb):
        assert list(row) == [x0, x0 + ex - 1, y0, y0 + ey - 1, z0, z0 + ez - 1, ez * ey * ex]
    labels, n, _ = oracle.link(mask, 2, 2, min_xy=8, min_z=5, max_xy=12, max_z=11)
    assert n == 1          # only the box at the minima: the larger one has 12 channels
    labels, n, _ = oracle.link(mask, 2, 2, min_xy=8, min_z=5, max_xy=12, max_z=12)
    assert n == 2


def test_labels_cover_only_detected_voxels_and_numbering_is_dense():
    rng = np.random.default_rng(4)
    mask = (rng.random((10, 20, 30)) < 0.15).astype(np.uint8)
    labels, n, bb = oracle.link(mask, 2, 2, min_xy=2, min_z=1)
    assert not labels[mask == 0].any()
    assert set(np.unique(labels[labels > 0]).tolist()) == set(range(1, n + 1))
    for k in range(1, n + 1):
        assert bb[k - 1][6] == int((labels == k).sum())


def test_bad_arguments():
    m = np.zeros((2, 2, 2), np.uint8)
    for args in [(-1, 1), (1, -1)]:
        with pytest.raises(ValueError):
            oracle.link(m, *args)
