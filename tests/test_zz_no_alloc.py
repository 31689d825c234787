"""The allocation-free totals entry point (hydro_conserved_totals_noalloc)
against hydro_conserved_totals of a handle holding the same state: two calls
in a row on one device, the second on a smaller mesh (the shared scratch
keeps the first call's partials), then a split mesh in the block layout.
Each result must be bitwise the handle's."""
import numpy as np
import pytest

from paper_2501_02317_amd import workloads as wl
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def handle_and_state(H, c, precision, steps, blocks=None):
    h = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, lo=c.lo, hi=c.hi, bc=c.bc, blocks=blocks)
    h.set_primitive(c.W)
    h.step_auto(steps)
    return h


def test_noalloc_totals_equal_handle_totals(H):
    import torch
    cases = [
        ("3-D 48x40x36 mixed, 3 steps", wl.turbulence_3d(n=(48, 40, 36), mach=1.5, seed=71), 1, 3, None),
        ("2-D 40x24 FP64, 2 steps (smaller)", wl.shear_layer_2d(nx=40, ny=24, seed=72), 0, 2, None),
        ("3-D 32x32x16 in 2x2x1 blocks FP64, 2 steps", wl.turbulence_3d(n=(32, 32, 16), mach=1.0, seed=73), 0, 2,
         (2, 2, 1)),
    ]
    for name, c, prec, steps, blocks in cases:
        say("noalloc totals", name)
        h = handle_and_state(H, c, prec, steps, blocks)
        ref = h.totals()                       # syncs the handle's stream
        U = h.state_view().contiguous()        # the handle's layout (block layout when split)
        out = torch.full((h.ncomp,), float("nan"), dtype=torch.float64, device=U.device)
        s = torch.cuda.current_stream(U.device)
        H.conserved_totals_noalloc(h.cfg, U, out, stream=s)
        s.synchronize()
        got = out.cpu().numpy()
        h.close()
        print(f"[noalloc] {name}: {got} vs {ref}", flush=True)
        assert got.shape == ref.shape
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (name, got, ref)
