"""The memory-optimised van Leer integrator (Sec. 3.3) on the GPU against
the oracle's: FP64 to the 1e-12 gate, mixed (predicted state stored in FP32)
to the 1e-5 smooth-flow gate, conservation, symmetries, batching and the
workspace it saves."""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, gpu_mesh, oracle_mesh, rel_l1, say

pytestmark = pytest.mark.gpu
VL2 = 1


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def _with_bc(c, bc):
    c.bc = bc
    return c


def run_both(H, c, precision, steps=None, t_end=None):
    m = oracle_mesh(c, VL2)
    U0 = O.prim_to_cons(m, c.W)
    steps = c.steps if steps is None else steps
    t_end = c.t_end if t_end is None else t_end
    U_o, t_o, s_o, _ = O.run(m, U0, c.cfl, max_steps=steps, t_end=t_end)
    h = gpu_mesh(c, precision, VL2)
    h.step_auto(s_o + (3 if t_end > 0 else 0), t_end)
    U = h.get_state()
    t, s = h.time(), h.steps_done()
    T, T0 = h.totals(), O.totals(m, U0)
    h.close()
    return m, U0, U_o, t_o, s_o, U, t, s, T, T0


CASES = [
    ("smooth_1d", lambda: wl.smooth_1d(256)),
    ("sod_1d", lambda: wl.sod_1d(256)),
    ("shear_layer_96x80", lambda: wl.shear_layer_2d(96, 80, seed=4001, steps=40)),
    ("turb2d_130x70_outflow", lambda: _with_bc(wl.turbulence_3d(n=(130, 70), mach=1.0, seed=3, ndim=2,
                                                                   steps=30), ((2, 2), (3, 3)))),
    ("turb3d_40x36x28", lambda: wl.turbulence_3d(n=(40, 36, 28), mach=2.0, seed=4, steps=12)),
    ("turb3d_33x20x17_mixedbc", lambda: _with_bc(wl.turbulence_3d(n=(33, 20, 17), mach=1.0, seed=5,
                                                                     steps=10), ((1, 2), (3, 3), (0, 0)))),
]
SMOOTH = [CASES[0], CASES[4], ("turb3d_72x40x36_mach1", lambda: wl.turbulence_3d(n=(72, 40, 36), mach=1.0,
                                                                                 seed=6, steps=20))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fp64_run_matches_oracle(H, name, make):
    c = make()
    say("vl2 fp64", name)
    m, U0, U_o, t_o, s_o, U, t, s, T, T0 = run_both(H, c, H.FP64)
    err = rel_l1(U, U_o)
    print(name, "relL1", err, "t", t, t_o)
    assert s == s_o and abs(t - t_o) <= 1e-14 * max(t_o, 1e-300)
    assert np.all(err <= 1e-12), err


@pytest.mark.parametrize("name,make", SMOOTH, ids=[c[0] for c in SMOOTH])
def test_mixed_run_within_smooth_gate(H, name, make):
    c = make()
    say("vl2 mixed", name)
    m, U0, U_o, t_o, s_o, U, t, s, T, T0 = run_both(H, c, H.MIXED)
    err = rel_l1(U, U_o)
    print(name, "relL1", err)
    assert s == s_o and abs(t - t_o) <= 1e-6 * t_o
    assert np.all(err <= 1e-5), err


@pytest.mark.parametrize("precision", [0, 1])
def test_periodic_conservation(H, precision):
    c = wl.turbulence_3d(n=(36, 28, 20), mach=1.5, seed=21, steps=15)
    say("vl2 conservation", precision)
    m, U0, U_o, t_o, s_o, U, t, s, T, T0 = run_both(H, c, precision)
    dV = np.prod(m.dx)
    drift = np.abs(T - T0) / (dV * np.abs(U0).reshape(m.ncomp, -1).sum(axis=1))
    print("drift", drift)
    assert np.all(drift <= 1e-12)


@pytest.mark.parametrize("precision", [0, 1])
def test_transpose_bitwise_3d(H, precision):
    c = wl.turbulence_3d(n=(24, 24, 20), mach=1.0, seed=8, steps=6)
    WT = np.swapaxes(c.W, 2, 3).copy()
    WT[[1, 2]] = WT[[2, 1]]
    say("vl2 transpose", precision)
    h = gpu_mesh(c, precision, VL2)
    h.step_auto(6)
    U = h.get_state()
    h.close()
    c.W = WT
    h = gpu_mesh(c, precision, VL2)
    h.step_auto(6)
    UT = h.get_state()
    h.close()
    back = np.swapaxes(UT, 2, 3).copy()
    back[[1, 2]] = back[[2, 1]]
    assert bitwise_equal(back, U)


def test_mixed_workspace_is_smaller(H):
    n = (64, 64, 64)
    heun = H.workspace_bytes(H.make_config(n, 5 / 3, 0.3, H.MIXED))
    vl2 = H.workspace_bytes(H.make_config(n, 5 / 3, 0.3, H.MIXED, integrator=H.VL2))
    vl2_64 = H.workspace_bytes(H.make_config(n, 5 / 3, 0.3, H.FP64, integrator=H.VL2))
    cells = 64 ** 3
    assert heun - vl2 == 5 * 4 * cells          # FP32 predicted state instead of FP64 U1
    assert vl2_64 == heun


@pytest.mark.parametrize("use_graph", [True, False], ids=["graph", "streams"])
def test_batch_members_equal_alone(H, use_graph):
    import torch
    cases = [(wl.turbulence_3d(n=(40, 24, 20), mach=1.0, seed=16), 1),
             (wl.turbulence_3d(n=(20, 20, 36), mach=1.0, seed=17), 0),
             (wl.shear_layer_2d(96, 128, seed=4012), 1)]
    say("vl2 batch")
    s = torch.cuda.Stream()
    ms = []
    for c, p in cases:
        h = H.Hydro(c.n, c.gamma, c.cfl, precision=p, lo=c.lo, hi=c.hi, bc=c.bc, stream=s, integrator=VL2)
        h.set_primitive(c.W)
        ms.append(h)
    b = H.Batch(ms, use_graph=use_graph)
    assert b.info()["groups"] == 3
    b.step(7)
    s.synchronize()
    for (c, p), h in zip(cases, ms):
        a = gpu_mesh(c, p, VL2)
        a.step_auto(7)
        assert bitwise_equal(a.get_state(), h.get_state()), c.name
        assert a.time() == h.time()
        a.close()
    b.close()
    for h in ms:
        h.close()


def test_autotune_steps_are_steps_of_the_run(H):
    c = wl.turbulence_3d(n=(40, 36, 28), mach=1.0, seed=23)
    say("vl2 autotune")
    h = gpu_mesh(c, H.MIXED, VL2)
    tiles, k = h.autotune(1)
    ref = gpu_mesh(c, H.MIXED, VL2)
    ref.step_auto(k)
    assert bitwise_equal(h.get_state(), ref.get_state())
    h.close()
    ref.close()
