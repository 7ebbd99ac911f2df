"""Parity at the size of the 96-cube batch workload, in its launch configuration.

The whole batch (4.8e9 voxels) runs as one graph launch, exactly as the
benchmark times it. Checks:
  * every cube of the batch equals its own single run, bit for bit (masks,
    noise, sigma_0): the lanes, the graph and the shared workspaces change
    nothing;
  * the three smallest cubes of the batch against the FP64 oracle, step by
    step with the oracle's previous mask and sigma_0 given (teacher forcing):
    noise to 1e-6, masks equal outside the boundary band;
  * the same cubes' whole batched runs, every iteration checked against the
    oracle from the run's own previous mask and sigma_0 (a flip inside one
    iteration's band legitimately changes what later iterations replace, so
    each iteration is compared from the state the GPU actually had): noise to
    1e-6, masks equal outside the boundary band.
"""
import sys

import numpy as np
import pytest

import gpu_chain
import oracle
import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def batch():
    wl = synth.workload("batch96")
    order = sorted(range(len(wl.cubes)), key=lambda i: wl.cubes[i].n_vox)
    keep = set(order[:3])
    xs, host_x = [], {}
    for i, c in enumerate(wl.cubes):
        x = synth.generate(c)
        if i in keep:
            host_x[i] = x
        xs.append(torch.from_numpy(x).cuda())
        del x
    say(f"batch96: {len(xs)} cubes generated, smallest {[wl.cubes[i].shape for i in order[:3]]}")
    return wl, xs, host_x


@pytest.fixture(scope="module")
def h():
    handle = sc.SofiaSC(0)
    yield handle
    handle.close()


@pytest.fixture(scope="module")
def batch_result(h, batch):
    wl, xs, _ = batch
    masks, noise, s0 = h.run_batch(xs, wl.kernels, wl.threshold, wl.noise_mode,
                                   wl.flux_range, wl.replacement)
    torch.cuda.synchronize()
    return masks, noise, s0


def test_batch96_equals_single_runs(h, batch, batch_result):
    wl, xs, _ = batch
    masks, noise, s0 = batch_result
    for i, x in enumerate(xs):
        m, n, z = h.run(x, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                        wl.replacement)
        assert torch.equal(m, masks[i]), f"mask of cube {i}"
        np.testing.assert_array_equal(n, noise[i], err_msg=f"noise of cube {i}")
        assert z == s0[i], f"sigma_0 of cube {i}"
        del m
    say("batch96: all 96 cubes equal their single runs bit for bit")


def test_batch96_smallest_cubes_teacher_forced(h, batch):
    wl, xs, host_x = batch
    for i, x in sorted(host_x.items()):
        s0, _ = oracle.noise(np.where(np.isfinite(x), x, np.nan).astype(np.float64),
                             wl.noise_mode, wl.flux_range)
        mask = np.zeros(x.shape, np.uint8)
        worst, bands = 0.0, 0
        for k, (f, w) in enumerate(wl.kernels):
            ref = oracle.step(x, f, w, wl.threshold, wl.noise_mode, wl.flux_range, mask,
                              wl.replacement, s0)
            out, sk = h.step(xs[i], (f, w), wl.threshold, wl.noise_mode, wl.flux_range,
                             wl.replacement, s0,
                             mask_in=torch.from_numpy(mask).cuda() if k else None)
            g = out.cpu().numpy()
            rel = abs(sk / ref.sigma - 1)
            worst = max(worst, rel)
            bands += int(ref.band_count)
            assert rel <= 1e-6, f"cube {i} step {k}: sigma rel {rel:.3g}"
            assert int(((g != ref.mask) & (ref.band == 0)).sum()) == 0, f"cube {i} step {k}"
            mask = ref.mask
        say(f"batch96 cube {i} {x.shape} teacher-forced: worst sigma rel {worst:.2e}, "
            f"band voxels {bands}")


def test_batch96_smallest_cubes_end_to_end(h, batch, batch_result):
    """The batched runs of the smallest cubes, every iteration checked against
    the oracle from the run's own previous state (the batch equals the single
    runs bit for bit, so the cut runs are single runs)."""
    wl, xs, host_x = batch
    masks, noise, s0 = batch_result
    for i, x in sorted(host_x.items()):
        gpu_chain.forced_chain(h, xs[i], x, wl.kernels, wl.threshold, wl.noise_mode,
                               wl.flux_range, wl.replacement,
                               what=f"batch96 cube {i} {x.shape}",
                               full=(masks[i], noise[i], s0[i]))
