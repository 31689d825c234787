"""Tile autotuner: its timing steps are ordinary steps of the run, it picks
one of the candidates, the JSON cache skips tuning, and a run that ends while
tuning is reported without changing the tile."""
import pytest

from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, gpu_mesh, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


@pytest.mark.parametrize("ndim", [2, 3])
def test_autotune_steps_are_steps_of_the_run(H, tmp_path, ndim):
    c = (wl.turbulence_3d(n=(40, 36, 28), mach=1.0, seed=23) if ndim == 3
         else wl.shear_layer_2d(96, 160, seed=4030))
    cache = str(tmp_path / "tiles.json")
    say("autotune", ndim, c.n)
    h = gpu_mesh(c, H.MIXED)
    tiles, k = h.autotune(1, cache=cache)
    cands = H.tile_candidates(ndim, c.n, H.MIXED)
    assert all(t in cands for t in tiles) and k == len(cands) + 1 and h.get_tile() == tiles
    ref = gpu_mesh(c, H.MIXED)
    ref.step_auto(k)
    assert bitwise_equal(h.get_state(), ref.get_state())
    assert h.time() == ref.time() and h.steps_done() == ref.steps_done() == k
    # a cached tile is set without steps
    h2 = gpu_mesh(c, H.MIXED)
    assert h2.autotune(1, cache=cache) == (tiles, 0)
    assert h2.get_tile() == tiles and h2.steps_done() == 0
    for x in (h, ref, h2):
        x.close()


def test_autotune_reports_a_run_that_ended(H):
    c = wl.turbulence_3d(n=(24, 20, 16), mach=1.0, seed=24)
    say("autotune end of run")
    h = gpu_mesh(c, H.FP64)
    before = h.get_tile()
    with pytest.raises(H.HydroError) as e:
        h.autotune(1, t_end=1e-9)            # reached by the first step
    assert e.value.status == H.E_STATE
    assert h.get_tile() == before and h.time() == 1e-9
    h.step_auto(2)                            # still usable
    assert h.steps_done() >= 2
    h.close()


@pytest.mark.parametrize("ndim,prec", [(3, 0), (3, 1), (2, 1)])
def test_results_bitwise_independent_of_tile(H, ndim, prec):
    """Every candidate tile (shapes, fixed and automatic chunk lengths) gives
    the same bits after several steps on a ragged mesh."""
    c = (wl.turbulence_3d(n=(72, 44, 40), mach=1.5, seed=25) if ndim == 3
         else wl.shear_layer_2d(200, 136, seed=4031))
    ref = None
    cands = H.tile_candidates(ndim, c.n, prec)
    # every candidate for both stages, then mixed pairs
    pairs = [(t, t) for t in cands] + list(zip(cands, cands[1:] + cands[:1]))
    for t1, t2 in pairs:
        say("tiles", ndim, prec, t1, t2)
        h = gpu_mesh(c, prec)
        h.set_tile(*t1, stage=1)
        h.set_tile(*t2, stage=2)
        h.step_auto(4)
        U = h.get_state()
        h.close()
        if ref is None:
            ref = U
        else:
            assert bitwise_equal(U, ref), (t1, t2)
