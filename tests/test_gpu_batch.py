"""Batched runs (sofia_sc_run_batch): one graph launch over many cubes.

Each cube of a batch must give exactly what a single run of it gives (same
kernels and launch shapes, so bit for bit: masks, noise and sigma_0), and
therefore the oracle's result to the parity bar. The batch is captured into a
HIP graph once and replayed by identical calls: every replay is checked
against the single runs, with the program's own eager work and
synchronisations between the replays.
"""
import math
import sys

import numpy as np
import pytest

import gpu_chain
import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

SIGMA_RTOL = 1e-6


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


@pytest.fixture(scope="module")
def small():
    wl = synth.workload("batch_small")
    xs = [synth.generate(c) for c in wl.cubes]
    return wl, xs, [torch.from_numpy(x).cuda() for x in xs]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _singles(h, xd, wl, **kw):
    out = []
    for x in xd:
        m, n, s0 = h.run(x, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                         kw.get("replacement", wl.replacement), storage=kw.get("storage", "f32"))
        out.append((host(m), n, s0))
    return out


def _assert_same(batch, singles, what):
    masks, noise, s0 = batch
    for i, (m, n, z) in enumerate(singles):
        np.testing.assert_array_equal(host(masks[i]), m, err_msg=f"{what}: mask of cube {i}")
        np.testing.assert_array_equal(noise[i], n, err_msg=f"{what}: noise of cube {i}")
        assert (math.isnan(s0[i]) and math.isnan(z)) or s0[i] == z, f"{what}: sigma_0 {i}"


def test_batch_equals_single_runs_over_graph_replays(h, small):
    wl, xs, xd = small
    say("batch_small:", [(c.nx, c.ny, c.nz) for c in wl.cubes])
    ref = _singles(h, xd, wl)
    masks = [torch.full(x.shape, 7, dtype=torch.uint8, device="cuda") for x in xd]
    for rep in range(3):
        for m in masks:
            m.fill_(0xAA)               # every replay must overwrite the masks
        out = h.run_batch(xd, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                          wl.replacement, masks=masks)
        _assert_same(out, ref, f"replay {rep}")
        # eager work of the program between replays
        h.run(xd[rep], wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
              wl.replacement)
        torch.cuda.synchronize()
    say("  3 replays equal the single runs bit for bit")


def test_batch_matches_oracle(h, small):
    """Each cube's batched result equals its single run bit for bit, and every
    iteration of that run matches the oracle from the run's own state."""
    wl, xs, xd = small
    out = h.run_batch(xd, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                      wl.replacement)
    _assert_same(out, _singles(h, xd, wl), "batch vs singles")
    masks, noise, s0 = out
    for i, x in enumerate(xs):
        gpu_chain.forced_chain(h, xd[i], x, wl.kernels, wl.threshold, wl.noise_mode,
                               wl.flux_range, wl.replacement, what=f"batch cube {i} {x.shape}",
                               full=(masks[i], noise[i], s0[i]))


def test_batch_recaptures_for_new_cubes_and_settings(h, small):
    wl, xs, xd = small
    sub = [xd[5], xd[1], xd[3]]          # fewer cubes than lanes
    kernels = [(0.0, 0), (3.0, 7), (6.0, 3)]
    for args in [("std", "all", -1.0), ("mad", "all", 1.5), ("mad", "negative", 2.0)]:
        mode, rng_, repl = args
        ref = []
        for x in sub:
            m, n, z = h.run(x, kernels, 3.0, mode, rng_, repl)
            ref.append((host(m), n, z))
        out = h.run_batch(sub, kernels, 3.0, mode, rng_, repl)
        _assert_same(out, ref, f"subset {args}")
    # back to the full batch (a fresh capture again)
    out = h.run_batch(xd, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                      wl.replacement)
    _assert_same(out, _singles(h, xd, wl), "full batch again")


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_batch_16bit_storage_equals_single_runs(h, small, storage):
    wl, xs, xd = small
    out = h.run_batch(xd, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                      wl.replacement, storage=storage)
    _assert_same(out, _singles(h, xd, wl, storage=storage), storage)


def test_batch_edge_shapes(h):
    shapes = [(1, 1, 1), (3, 1, 5), (130, 2, 7), (1, 40, 33), (257, 3, 64)]
    rng = np.random.default_rng(17)
    xs = [rng.standard_normal((z, y, x)).astype(np.float32) for x, y, z in shapes]
    xs[2][:, 0, :5] = np.nan
    xd = [torch.from_numpy(x).cuda() for x in xs]
    kernels = [(0.0, 0), (3.0, 3), (0.0, 15)]
    ref = []
    for x in xd:
        m, n, z = h.run(x, kernels, 2.5, "mad", "all", 2.0)
        ref.append((host(m), n, z))
    out = h.run_batch(xd, kernels, 2.5, "mad", "all", 2.0)
    _assert_same(out, ref, "edge shapes")
    for i, x in enumerate(xs):
        gpu_chain.forced_chain(h, xd[i], x, kernels, 2.5, "mad", "all", 2.0,
                               what=f"edge cube {x.shape}",
                               full=(out[0][i], out[1][i], out[2][i]))


def test_batch_keep_input_mask_toggles_between_identical_calls(h, small):
    """Two batch calls that differ only in keep_input_mask must not replay one
    another's graph: keep = 0 overwrites the whole mask, keep = 1 ORs the
    detections into it. Checked in both orders on pre-filled masks against
    sofia_sc_run_ex of each cube alone."""
    wl, xs, xd = small
    sub = xd[:3]
    rng = np.random.default_rng(21)
    prior = [rng.choice(np.array([0, 1, 2, 6], np.uint8), size=tuple(x.shape),
                        p=[0.7, 0.1, 0.1, 0.1]) for x in sub]
    plain = [host(h.run(x, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                        wl.replacement)[0]) for x in sub]
    masks = [torch.empty(x.shape, dtype=torch.uint8, device="cuda") for x in sub]
    for order in ([False, True], [True, False], [False, True, True, False]):
        for keep in order:
            for m, p in zip(masks, prior):
                m.copy_(torch.from_numpy(p))
            h.run_batch(sub, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                        wl.replacement, masks=masks, keep_input_mask=keep)
            for i, (m, p, r) in enumerate(zip(masks, prior, plain)):
                expect = (p | r) if keep else r
                np.testing.assert_array_equal(host(m), expect,
                                              err_msg=f"order {order} keep {keep} cube {i}")
    say("keep_input_mask toggles: every call matches its own setting")


def test_batch_errors(h, small):
    wl, xs, xd = small
    m = torch.empty(xd[0].shape, dtype=torch.uint8, device="cuda")
    with pytest.raises(sc.ScError) as e:
        h.run_batch([xd[0], xd[0]], wl.kernels, 3.5, masks=[m, m])
    assert e.value.code == sc.EINVAL and "mask" in str(e.value)
    with pytest.raises(sc.ScError) as e:
        h.run_batch(xd[:2], [(0.0, 4)], 3.5)
    assert e.value.code == sc.EINVAL
    # a cube with no voxel in the range: ENOSTAT, the other cubes still filled in
    empty = torch.full((9, 8, 7), float("nan"), device="cuda")
    masks, noise, s0 = h.run_batch([xd[0], empty, xd[2]], [(0.0, 0), (3.0, 3)], 3.5,
                                   allow_nostat=True)
    assert np.all(np.isfinite(noise[0])) and np.all(np.isfinite(noise[2]))
    assert np.all(np.isnan(noise[1]))
    with pytest.raises(sc.ScError) as e:
        h.run_batch([xd[0], empty], [(0.0, 0)], 3.5)
    assert e.value.code == sc.ENOSTAT
