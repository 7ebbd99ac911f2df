"""The launch-shape autotuner of whole runs (sofia_sc_tune_run) and the
handle's shape setters.

The tuner times candidate shapes on the caller's cube and keeps the fastest
in the handle for its later runs and batches. Launch shapes change nothing in
MAD results, so tuned runs and batches must equal the runs of a fresh handle
with default shapes bit for bit.
"""
import sys

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CANDIDATES = {"lanes": (4, 8, 16), "col_blocks": (3072, 6144, 12288),
              "strip_rows": (64, 128, 256), "strip_waves": (1, 2, 4),
              "col_min_planes": (32, 64, 128)}


def test_tune_run_picks_candidate_shapes_and_keeps_results():
    wl = synth.workload("batch_small")
    xd = [torch.from_numpy(synth.generate(c)).cuda() for c in wl.cubes]
    big = torch.from_numpy(synth.generate(synth.CubeSpec(
        300, 260, 200, seed=91, radial=True, sigma_lo=0.8, sigma_hi=1.5, n_gal=10,
        nan_border=3))).cuda()
    args = (wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range, wl.replacement)
    h0 = sc.SofiaSC(0)
    try:
        ref = [tuple(r if i else r.cpu().numpy() for i, r in enumerate(h0.run(x, *args)))
               for x in xd + [big]]
    finally:
        h0.close()
    ht = sc.SofiaSC(0)
    try:
        assert ht.shapes()["col_blocks"] == 6144
        m = torch.empty(big.shape, dtype=torch.uint8, device="cuda")
        best = ht.tune_run(big, *args, mask=m)
        say("tuned shapes:", best)
        for k, vals in CANDIDATES.items():
            assert best[k] in vals, k
        assert best["ms"] > 0
        assert ht.shapes() == best
        np.testing.assert_array_equal(m.cpu().numpy(), ref[-1][0])
        # later single runs and a batch of the tuned handle: same results
        for i, x in enumerate(xd + [big]):
            mi, ni, zi = ht.run(x, *args)
            np.testing.assert_array_equal(mi.cpu().numpy(), ref[i][0], err_msg=f"run {i}")
            np.testing.assert_array_equal(ni, ref[i][1])
            assert zi == ref[i][2]
        masks, noise, s0 = ht.run_batch(xd, *args)
        for i in range(len(xd)):
            np.testing.assert_array_equal(masks[i].cpu().numpy(), ref[i][0])
            np.testing.assert_array_equal(noise[i], ref[i][1])
        # shapes can be set and reset; values outside the candidates are refused
        ht.set_shapes(None)
        assert ht.shapes()["col_blocks"] == 6144 and ht.shapes()["strip_waves"] == 4
        bad = dict(best, strip_waves=3)
        with pytest.raises(sc.ScError) as e:
            ht.set_shapes(bad)
        assert e.value.code == sc.EINVAL
        ht.set_shapes(best)
        assert ht.shapes()["strip_rows"] == best["strip_rows"]
    finally:
        ht.close()


def test_batch_tuner_is_switched_off():
    """The graph-capturing batch tuner returns EDEVICE at once and touches
    nothing (see its declaration)."""
    wl = synth.workload("batch_small")
    xd = [torch.from_numpy(synth.generate(c)).cuda() for c in wl.cubes[:2]]
    h = sc.SofiaSC(0)
    try:
        with pytest.raises(sc.ScError) as e:
            h.tune_batch(xd, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                         wl.replacement)
        assert e.value.code == sc.EDEVICE and "switched off" in str(e.value)
    finally:
        h.close()
