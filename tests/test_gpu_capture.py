"""hydro_step_auto enqueues only kernels (no host synchronisation, no
allocation, no memset), so it can be captured into a HIP graph: a single
mesh, a mesh split into blocks, and a refined mesh.  While the handle's stream
is captured, the block-stream form adds its per-group stage kernels to the
capture's graph as nodes with the group dependencies, and a refined mesh's
second stream runs on the handle's stream.  Each graph is replayed several times, with eager work and host
synchronisation between the replays, and every replay is checked bitwise
against the same steps run eagerly."""
import numpy as np
import pytest

from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def make(H, c, stream, blocks=None, refined=None, streams=False, W=None, precision=1, integrator=0):
    h = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, lo=c.lo, hi=c.hi, bc=c.bc, stream=stream,
                blocks=blocks, refined=refined, integrator=integrator)
    if streams:
        h.set_block_streams(True)
    h.set_primitive(c.W if W is None else W)
    return h


# name, blocks, refined, block streams, precision, integrator, t_end
CASES = [pytest.param("single", None, None, False, 1, 0, 0.0, id="single"),
         pytest.param("blocks", (2, 2, 2), None, False, 1, 0, 0.0, id="blocks"),
         pytest.param("block streams", (2, 2, 4), None, True, 1, 0, 0.0, id="block streams"),
         pytest.param("refined", (2, 2, 2), [0, 5], False, 1, 0, 0.0, id="refined"),
         pytest.param("fp64", None, None, False, 0, 0, 0.0, id="fp64"),
         pytest.param("van Leer", (1, 2, 2), None, False, 1, 1, 0.0, id="van Leer"),
         pytest.param("refined fp64", (2, 2, 2), [1, 2, 7], False, 0, 0, 0.0, id="refined fp64"),
         pytest.param("refined van Leer", (2, 2, 2), [0, 6], False, 1, 1, 0.0, id="refined van Leer"),
         # the end time falls inside the second replay: the step that would
         # pass it lands on it, and the third replay changes nothing
         pytest.param("to t_end", (2, 1, 1), None, False, 1, 0, 0.0135, id="to t_end")]


@pytest.mark.parametrize("name,blocks,refined,streams,precision,integrator,t_end", CASES)
def test_captured_steps_replay_like_eager_steps(H, name, blocks, refined, streams, precision, integrator,
                                                t_end):
    import torch
    c = wl.turbulence_3d(n=(32, 32, 32), mach=1.0, seed=81)
    W = None
    if refined is not None:
        leaves = H.smr_leaves(H.make_config(c.n, c.gamma, c.cfl, blocks=blocks), refined)
        W = wl.smr_field(leaves, c.n, blocks, gamma=c.gamma)
    nsteps, replays = 3, 3
    say("capture", name)
    s = torch.cuda.Stream()
    opts = dict(blocks=blocks, refined=refined, streams=streams, W=W, precision=precision, integrator=integrator)
    # eager reference: the same calls, states after each call
    ref = make(H, c, s, **opts)
    expect = []
    for _ in range(replays):
        ref.step_auto(nsteps, t_end)
        expect.append((ref.get_state(), ref.time(), ref.steps_done()))
    ref.close()
    if t_end > 0.0:
        assert expect[0][1] < t_end and expect[1][1] == t_end and expect[2][2] == expect[1][2]
    h = make(H, c, s, **opts)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        h.step_auto(nsteps, t_end)
    for r in range(replays):
        g.replay()
        # eager work of the program between replays, then a host synchronisation
        junk = torch.ones(1 << 20, device="cuda")
        junk.mul_(2.0)
        torch.cuda.synchronize()
        U, t, k = h.get_state(), h.time(), h.steps_done()
        assert k == expect[r][2] and t == expect[r][1], (name, r)
        assert bitwise_equal(U, expect[r][0]), (name, r)
    del g
    h.close()
