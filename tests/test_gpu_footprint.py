"""Device memory a handle takes for a run, against the workspace the design
budgets: three packed bit planes (blank bits and two sets of detection bits)
3N/8, P 4N (spatial kernels only), MAD capture list N/8 keys x 4 B, undecided
list N/256 x 16 B, plus a few MB of histograms, partials and state."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2106_15789_amd as sc  # noqa: E402

pytestmark = pytest.mark.gpu

MIB = 1 << 20


def _free():
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.mark.parametrize("kernels,per_voxel", [
    ([(0.0, 0), (3.0, 7), (6.0, 15)], 3 / 8 + 4 + 4 / 8 + 16 / 256),
    ([(0.0, 0), (0.0, 7), (0.0, 15)], 3 / 8 + 4 / 8 + 16 / 256),
])
def test_run_workspace_within_budget(kernels, per_voxel):
    spec = synth.CubeSpec(256, 256, 128, seed=81, n_gal=3)
    x = torch.from_numpy(synth.generate(spec)).cuda()
    m = torch.empty(x.shape, dtype=torch.uint8, device="cuda")
    warm = sc.SofiaSC(0)      # loads the code object (and its fixed device arrays)
    warm.run(x[:4, :16, :16].contiguous(), [(0.0, 0)], 3.5, "mad", "negative")
    warm.close()
    free0 = _free()
    h = sc.SofiaSC(0)
    try:
        h.run(x, kernels, 3.5, "mad", "negative", mask=m)
        used = free0 - _free()
    finally:
        h.close()
    n = x.numel()
    budget = per_voxel * n + 32 * MIB
    print(f"workspace {used / MIB:.1f} MiB for {n} voxels ({used / n:.2f} B/voxel), "
          f"budget {budget / MIB:.1f} MiB")
    assert used <= budget
    assert used >= 0.9 * per_voxel * n
    assert free0 - _free() <= 16 * MIB       # released by destroy
