"""The van Leer integrator (Sec. 3.3) on a statically refined mesh on the GPU
against the oracle's (Sec. 2.3 block tree; Sec. 3 cross-level sequence in
both stages: restriction, minmod prolongation, fine-flux average at level
jumps).

On a refined handle the predicted state is kept conserved in FP64, so the
level-jump passes serve the predictor (piecewise-constant states, half a
step) and the corrector alike.  Checked: the oracle's result to the
precision's tolerance on smooth flows and on a shock crossing level jumps,
one to three levels deep; the split and the uniform van Leer runs when
nothing or everything is refined; conservation to round-off; a uniform state
kept exactly; a run to an end time and on host-given steps."""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, say
from test_gpu_smr import smooth_state, sod_state

pytestmark = pytest.mark.gpu

P, F, OUT, R = O.BC_PERIODIC, O.BC_FREE, O.BC_OUTFLOW, O.BC_REFLECT
TOL = {0: 1e-12, 1: 1e-5}
VL2 = 1
LS = 26


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def vl2_mesh(n, gamma, bc=None):
    m = O.Mesh(n, gamma, bc=bc)
    m.integrator = O.VL2
    return m


def run_gpu(H, S, W, precision, steps, cfl, t_end=0.0):
    m = S.mesh
    h = H.Hydro(m.n, m.gamma, cfl, precision=precision, lo=m.lo, hi=m.hi, bc=m.bc, blocks=S.blocks[:m.ndim],
                refined=S.refined, integrator=VL2)
    assert tuple(h.shape) == tuple(S.shape)
    assert np.array_equal(h.leaves, S.leaves)
    h.set_primitive(W)
    h.step_auto(steps, t_end)
    out = h.get_state(), h.time(), h.steps_done(), h.totals()
    h.close()
    return out


def rel_per_comp(U, U_o, nc):
    a = U.transpose(1, 0, 2, 3, 4).reshape(nc, -1)
    b = U_o.transpose(1, 0, 2, 3, 4).reshape(nc, -1)
    return np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)


CASES = [
    ("1d", (64,), (4,), [1, 2], ((F, OUT),)),
    ("2d periodic", (64, 32), (4, 2), [1, 6], ((P, P), (P, P))),
    ("2d walls", (48, 32), (4, 4), [5, 6, 9], ((R, R), (OUT, F))),
    ("3d", (32, 32, 16), (2, 2, 2), [0, 3, 5], ((P, P), (P, P), (F, R))),
    ("3d ragged", (48, 24, 16), (3, 3, 2), [1, 4, 7, 13], ((P, P), (R, OUT), (P, P))),
    ("2d three levels", (64, 32), (4, 2), [1, 6, (1 << LS) | 3, (1 << LS) | 20], ((P, P), (P, P))),
    ("3d four levels", (32, 32, 32), (2, 2, 2), [0, (1 << LS) | 0, (2 << LS) | 0], ((P, P), (P, P), (P, P))),
]


@pytest.mark.parametrize("name,n,B,ref,bc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_matches_oracle(H, name, n, B, ref, bc, precision):
    m = vl2_mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=71)
    steps = 6
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, max_steps=steps)
    say("smr van Leer vs oracle", name, precision)
    U, t, s, T = run_gpu(H, S, W, precision, steps, 0.4)
    assert s == s_o == steps
    assert abs(t - t_o) <= (1e-14 if precision == 0 else 1e-6) * t_o
    rel = rel_per_comp(U, U_o, m.ncomp)
    print(name, precision, "leaves per level", np.bincount(S.leaves[:, 0]), "relL1", rel)
    assert np.all(rel <= TOL[precision]), rel
    T_o = S.totals(U)
    assert np.allclose(T, T_o, rtol=1e-12, atol=1e-12 * np.abs(T_o).max())


SHOCK_CASES = [
    ("1d band", (64,), (8,), [3, 4], ((F, F),), 0, 0.2),
    ("1d two levels", (64,), (8,), [3, 4, (1 << LS) | 7, (1 << LS) | 8], ((F, F),), 0, 0.2),
    ("2d partial", (64, 32), (8, 4), [3, 4, 11, 12, 20], ((F, F), (P, P)), 70, 0.0),
    ("3d partial", (32, 16, 16), (4, 2, 2), [1, 2, 5, 14], ((F, F), (R, R), (P, P)), 45, 0.0),
]


@pytest.mark.parametrize("name,n,B,ref,bc,steps,t_end", SHOCK_CASES, ids=[c[0] for c in SHOCK_CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_shock_across_level_jumps_matches_oracle(H, name, n, B, ref, bc, steps, t_end, precision):
    """Sod's shock through refined blocks: FP64 to the 1e-12 gate; mixed to
    1e-4 (a shock: not the smooth-flow bound)."""
    m = vl2_mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    W = sod_state(S)
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, max_steps=steps, t_end=t_end)
    say("smr van Leer shock vs oracle", name, precision)
    U, t, s, T = run_gpu(H, S, W, precision, steps if steps else s_o + 4, 0.4, t_end)
    assert s == s_o
    assert abs(t - t_o) <= (1e-14 if precision == 0 else 1e-6) * t_o
    rel = rel_per_comp(U, U_o, m.ncomp)
    print(name, precision, "relL1", rel, "steps", s)
    assert np.all(rel <= (1e-12 if precision == 0 else 1e-4)), rel


def to_blocks(W, B):
    nc, nz, ny, nx = W.shape
    bz, by, bx = nz // B[2], ny // B[1], nx // B[0]
    V = W.reshape(nc, B[2], bz, B[1], by, B[0], bx).transpose(1, 3, 5, 0, 2, 4, 6)
    return np.ascontiguousarray(V.reshape(B[0] * B[1] * B[2], nc, bz, by, bx))


@pytest.mark.parametrize("precision", [0, 1])
def test_nothing_refined_is_the_split_mesh(H, precision):
    """FP64: bit for bit the split van Leer run (the conserved predictor
    converts to the same primitive values the uniform path stores); mixed:
    the uniform path stores the predictor in FP32, so within the smooth-flow
    tolerance."""
    c = wl.turbulence_3d(n=(32, 32, 16), mach=1.0, seed=73)
    B = (2, 2, 2)
    say("smr van Leer nothing refined", precision)
    a = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, blocks=B, integrator=VL2)
    a.set_primitive(c.W)
    a.step_auto(5)
    Ua = to_blocks(a.get_state(), B)
    b = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, blocks=B, refined=[], integrator=VL2)
    b.set_primitive(to_blocks(c.W, B))
    b.step_auto(5)
    Ub = b.get_state()
    if precision == 0:
        assert bitwise_equal(Ub, Ua)
        assert a.time() == b.time()
    else:
        rel = rel_per_comp(Ub, Ua, 5)
        print("mixed, conserved vs FP32 predictor", rel)
        assert np.all(rel <= 1e-5), rel
        assert abs(a.time() - b.time()) <= 1e-6 * a.time()
    a.close()
    b.close()


@pytest.mark.parametrize("twice", [False, True], ids=["once", "twice"])
def test_everything_refined_is_the_finer_uniform_mesh(H, twice):
    """All blocks refined once (twice): bit for bit the uniform van Leer run
    two (four) times finer, FP64."""
    c = wl.turbulence_3d(n=(32, 32, 32), mach=1.0, seed=74)
    say("smr van Leer everything refined", "twice" if twice else "once")
    a = H.Hydro(c.n, c.gamma, c.cfl, precision=0, blocks=(4, 4, 4), integrator=VL2)
    a.set_primitive(c.W)
    a.step_auto(3)
    Ua = to_blocks(a.get_state(), (4, 4, 4))
    if twice:
        b = H.Hydro((8, 8, 8), c.gamma, c.cfl, precision=0, blocks=(1, 1, 1),
                    refined=[0] + [(1 << LS) | i for i in range(8)], integrator=VL2)
        assert np.all(b.leaves[:, 0] == 2)
    else:
        b = H.Hydro((16, 16, 16), c.gamma, c.cfl, precision=0, blocks=(2, 2, 2), refined=list(range(8)),
                    integrator=VL2)
        assert np.all(b.leaves[:, 0] == 1)
    # leaves in the order of the finest level's block grid: the 4x4x4 blocks
    b.set_primitive(to_blocks(c.W, (4, 4, 4)))
    b.step_auto(3)
    assert a.time() == b.time()
    assert bitwise_equal(b.get_state(), Ua)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_conserves_and_keeps_uniform_state(H, precision):
    n, B, ref = (32, 32, 16), (2, 2, 2), [0, 3, (1 << LS) | 0]
    m = vl2_mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    W = smooth_state(S, seed=75, amp=0.3, mach=1.0)
    say("smr van Leer conservation", precision)
    h = H.Hydro(n, m.gamma, 0.3, precision=precision, blocks=B, refined=ref, integrator=VL2)
    h.set_primitive(W)
    T0 = h.totals()
    h.step_auto(20)
    T1 = h.totals()
    U = h.get_state()
    h.close()
    scale = S.totals(np.abs(S.prim_to_cons(W)))
    print("drift", (T1 - T0) / scale)
    assert np.all(np.abs(T1 - T0) <= 1e-13 * scale)
    assert np.all(np.isfinite(U))
    Wu = np.empty(S.shape)
    Wu[:, 0], Wu[:, 1], Wu[:, 2], Wu[:, 3], Wu[:, 4] = 1.3, 0.7, -0.4, 0.2, 0.9
    h = H.Hydro(n, 1.4, 0.4, precision=precision, blocks=B, refined=ref, integrator=VL2)
    h.set_primitive(Wu)
    U0 = h.get_state()
    h.step_auto(4)
    assert bitwise_equal(h.get_state(), U0)
    h.close()


def test_run_to_end_time_and_host_dt(H):
    n, B, ref = (64, 32), (4, 2), [1, 6]
    m = vl2_mesh(n, 1.4, bc=((R, R), (P, P)))
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=76)
    U_o, t_o, s_o, dts = S.run(S.prim_to_cons(W), 0.4, max_steps=1000, t_end=0.05)
    say("smr van Leer t_end")
    U, t, s, _ = run_gpu(H, S, W, 0, 10000, 0.4, t_end=0.05)
    assert t == 0.05 and s == s_o
    assert np.abs(U - U_o).sum() / np.abs(U_o).sum() <= 1e-12
    h = H.Hydro(n, 1.4, 0.4, bc=m.bc, blocks=B, refined=ref, integrator=VL2)
    h.set_primitive(W)
    for dt in dts:
        h.step(dt)
    assert np.abs(h.get_state() - U_o).sum() / np.abs(U_o).sum() <= 1e-12
    h.close()
