"""lrx_det_window_noalloc (the library's own counters) against lrx_det_window (a caller
workspace): identical inputs in two identical walker batches give identical results, on two
calls in a row, the second with a smaller batch."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2602_05255_amd import inputs as gen  # noqa: E402
from paper_2602_05255_amd import lrx  # noqa: E402
from paper_2602_05255_amd.uneven import UnevenWalkers  # noqa: E402


def _classes(g, sizes, walkers):
    out = []
    for n, W in zip(sizes, walkers):
        phi = gen.normal(g, (2 * n, n))
        occ, emp = gen.occupancy(g, W, 2 * n, n)
        out.append({"n": n, "phi": phi, "occ": occ, "empty": emp})
    return out


def _state(uw):
    return [(p.ratio.cpu().numpy(), p.accept.cpu().numpy(), p.occ.cpu().numpy(), p.empty.cpu().numpy(),
             p.st.logabs.cpu().numpy(), p.st.inv.cpu().numpy(), p.st.slot) for p in uw.parts]


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_window_matches_workspace_window(dt):
    g = gen.generator(5100)
    k_max, ranks, steps = 4, (1, 2, 4), 9
    for call, (sizes, walkers, delays) in enumerate([((48, 100, 160), (40, 25, 12), (4, 3, 8)),
                                                    ((32, 70), (9, 5), (2, 5))]):
        say(f"noalloc window {dt} call {call}: sizes {sizes} walkers {walkers}")
        classes = _classes(g, sizes, walkers)
        draws = [gen.hop_draws_batch(g, steps, W, n, n, ranks, k_max) for n, W in zip(sizes, walkers)]
        runs = []
        for noalloc in (False, True):
            uw = UnevenWalkers(dt, classes, k_max, list(delays), steps, grid=9)
            uw.set_draws(draws)
            if noalloc:
                lrx.lrx_det_window_noalloc(uw.parts, steps, lrx.LRX_MH_DEVICE_RNG, 99, 7, uw.grid)
            else:
                lrx.lrx_det_window(uw.parts, steps, lrx.LRX_MH_DEVICE_RNG, 99, 7, uw.work, uw.grid)
            torch.cuda.synchronize()
            runs.append(_state(uw))
        for a, b in zip(*runs):
            for x, y in zip(a, b):
                if isinstance(x, np.ndarray):
                    np.testing.assert_array_equal(x, y)
                else:
                    assert x == y
        acc = sum(int(r[1].sum()) for r in runs[0])
        say(f"  identical ratios, decisions ({acc} accepted), occupancies, log|det| and inverses")
