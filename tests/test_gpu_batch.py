"""Batched stepping of ragged meshes: identical to stepping each mesh alone,
identical with and without HIP-graph replay, and on the oracle's results."""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, oracle_mesh, rel_l1, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def member_cases():
    """(case, precision, max_steps, t_end) of a ragged mix."""
    return [
        (wl.shear_layer_2d(64, 96, seed=4010), 1, 9, 0.0),
        (wl.shear_layer_2d(192, 128, seed=4011), 1, 14, 0.0),
        (wl.shear_layer_2d(96, 96, seed=4012), 0, 14, 0.0),
        (wl.shear_layer_2d(384, 64, seed=4013), 1, 6, 0.0),
        (wl.turbulence_3d(n=(40, 24, 20), mach=1.0, seed=16), 1, 11, 0.0),
        (wl.turbulence_3d(n=(20, 20, 36), mach=1.0, seed=17), 0, 7, 0.0),
        (wl.smooth_1d(200), 0, 0, 0.015),   # reaches t_end in about 10 steps
    ]


def make(H, c, prec, stream):
    h = H.Hydro(c.n, c.gamma, c.cfl, precision=prec, lo=c.lo, hi=c.hi, bc=c.bc, stream=stream)
    h.set_primitive(c.W)
    return h


def run_batch(H, cases, nsteps, use_graph, calls=1):
    import torch
    s = torch.cuda.Stream()
    ms = []
    for c, prec, ks, te in cases:
        h = make(H, c, prec, s)
        h.set_run_limit(ks, te)
        ms.append(h)
    b = H.Batch(ms, use_graph=use_graph)
    outs = []
    for _ in range(calls):
        b.step(nsteps)
        s.synchronize()
        outs.append([h.get_state() for h in ms])
    info = b.info()
    b.close()
    times = [h.time() for h in ms]
    steps = [h.steps_done() for h in ms]
    for h in ms:
        h.close()
    return outs, times, steps, info


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "streams"])
def test_batch_equals_each_mesh_alone(H, use_graph):
    """Captured (one stream), or launched directly with the groups spread
    over the batch's streams."""
    import torch
    cases = member_cases()
    say("batch vs alone", use_graph)
    outs, times, steps, info = run_batch(H, cases, 16, use_graph=use_graph)
    assert info["groups"] >= 4 and info["graph"] == use_graph
    for (c, prec, ks, te), U, t, k in zip(cases, outs[0], times, steps):
        s = torch.cuda.Stream()
        h = make(H, c, prec, s)
        h.step_auto(ks if ks else 16, te)
        s.synchronize()
        assert bitwise_equal(h.get_state(), U), c.name
        assert h.time() == t and h.steps_done() == k
        if ks:
            assert k == ks
        else:
            assert t == te
        h.close()


def test_batch_graph_replays_match_direct_launches(H):
    """Several replays of one captured graph, with eager work and host
    synchronisation between them, each equal to direct launches."""
    cases = [(c, p, 0, 0.0) for c, p, _, _ in member_cases()[:5]]
    say("batch graph replay")
    g_outs, *_ = run_batch(H, cases, 3, use_graph=True, calls=3)
    d_outs, *_ = run_batch(H, cases, 3, use_graph=False, calls=3)
    for call in range(3):
        for a, b in zip(g_outs[call], d_outs[call]):
            assert bitwise_equal(a, b)


def test_batch_members_track_oracle(H):
    cases = [(wl.shear_layer_2d(128, 96, seed=4020, steps=12), 0, 12, 0.0),
             (wl.turbulence_3d(n=(24, 24, 24), mach=1.0, seed=18, steps=8), 1, 8, 0.0)]
    say("batch vs oracle")
    outs, times, steps, info = run_batch(H, cases, 12, use_graph=True)
    for (c, prec, ks, te), U in zip(cases, outs[0]):
        m = oracle_mesh(c)
        U_o, *_ = O.run(m, O.prim_to_cons(m, c.W), c.cfl, max_steps=ks)
        err = rel_l1(U, U_o)
        print(c.name, prec, "relL1 vs oracle", err)
        assert np.all(err <= (1e-12 if prec == 0 else 1e-5))


_subset_oracle = {}


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-3)])
def test_batch_workload_subset_tracks_oracle(H, precision, tol):
    """Sixteen meshes of the 512-mesh ragged 2-D workload (seeded choice,
    the smallest and the largest included), 20 batched steps, each member
    against the oracle.  FP64 to the 1e-12 gate; mixed to the loose bound of
    marginally resolved layers (the tanh width spans 1 to 8 cells here)."""
    full = wl.batch_sizes(512, seed=401)
    cells = [nx * ny for nx, ny in full]
    rng = np.random.default_rng(402)
    pick = {int(np.argmin(cells)), int(np.argmax(cells))}
    while len(pick) < 16:
        pick.add(int(rng.integers(len(full))))
    pick = sorted(pick)
    cases = [(wl.shear_layer_2d(*full[m], seed=4000 + m, steps=20), precision, 20, 0.0) for m in pick]
    say("batch workload subset", precision, [full[m] for m in pick])
    outs, times, steps, info = run_batch(H, cases, 20, use_graph=True)
    assert steps == [20] * 16
    worst = np.zeros(4)
    for (c, prec, ks, te), U, t in zip(cases, outs[0], times):
        key = (c.name, c.meta["seed"])
        if key not in _subset_oracle:
            m = oracle_mesh(c)
            _subset_oracle[key] = O.run(m, O.prim_to_cons(m, c.W), c.cfl, max_steps=ks)
        U_o, t_o, s_o, _ = _subset_oracle[key]
        err = rel_l1(U, U_o)
        worst = np.maximum(worst, err)
        assert np.all(err <= tol), (c.name, err)
        assert abs(t - t_o) <= (1e-14 if prec == 0 else 1e-6) * t_o
    print("worst relL1 per component", worst)


def test_batch_autotune_steps_are_steps_of_the_run(H):
    """The batch autotuner's timing steps are ordinary batched steps: tuned
    then stepped equals stepped straight through, bitwise."""
    import torch
    cases = [(c, p, 0, 0.0) for c, p, _, _ in member_cases()]
    say("batch autotune")
    s = torch.cuda.Stream()
    A = [make(H, c, p, s) for c, p, _, _ in cases]
    B = [make(H, c, p, s) for c, p, _, _ in cases]
    ba = H.Batch(A, use_graph=True)
    rule, ms = ba.autotune(2)
    k = A[0].steps_done()
    assert k == 1 + 2 * 12 and all(h.steps_done() == k for h in A)
    ba.step(5)
    bb = H.Batch(B, use_graph=True)
    bb.step(k + 5)
    s.synchronize()
    for (c, *_), ha, hb in zip(cases, A, B):
        assert bitwise_equal(ha.get_state(), hb.get_state()), c.name
        assert ha.time() == hb.time()
    print("chosen rule", rule, "ms per step", ms, ba.info())
    for x in (ba, bb):
        x.close()
    for h in A + B:
        h.close()
