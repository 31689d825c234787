"""Two-level static mesh refinement on the GPU against the oracle's
(Sec. 2.3 block tree one level deep; Sec. 3 cross-level c-boundaries:
restriction, minmod prolongation, fine-flux average at level jumps).

Both sides start from the same block-layout state; the GPU run matches the
oracle to the precision's tolerance, keeps a uniform state exactly, conserves
the totals to round-off, and reduces to the split-mesh and fine uniform runs
when nothing or everything is refined."""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl
from gpu_util import bitwise_equal, say

pytestmark = pytest.mark.gpu

P, F, OUT, R = O.BC_PERIODIC, O.BC_FREE, O.BC_OUTFLOW, O.BC_REFLECT
TOL = {0: 1e-12, 1: 1e-5}


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2501_02317_amd import hydro
    return hydro


def smooth_state(S, seed, amp=0.2, mach=0.5):
    """A smooth random state on the leaves' cell centres (periodic modes)."""
    rng = np.random.default_rng(seed)
    X = S.centres()
    nd = S.mesh.ndim
    W = np.empty(S.shape)

    def field(scale):
        f = np.zeros(X[0].shape)
        for _ in range(4):
            k = rng.integers(1, 3, size=nd)
            ph = rng.random() * 2 * np.pi
            arg = sum(2 * np.pi * k[d] * X[d] / (S.mesh.hi[d] - S.mesh.lo[d]) for d in range(nd)) + ph
            f = f + np.sin(arg)
        return scale * f / 4

    W[:, 0] = 1.0 + field(amp)
    for d in range(nd):
        W[:, 1 + d] = field(mach)
    W[:, -1] = 1.0 + field(amp)
    return W


def run_gpu(H, S, W, precision, steps, cfl, t_end=0.0):
    m = S.mesh
    h = H.Hydro(m.n, m.gamma, cfl, precision=precision, lo=m.lo, hi=m.hi, bc=m.bc, blocks=S.blocks[:m.ndim],
                refined=S.refined)
    assert tuple(h.shape) == tuple(S.shape)
    assert np.array_equal(h.leaves, S.leaves)
    h.set_primitive(W)
    h.step_auto(steps, t_end)
    out = h.get_state(), h.time(), h.steps_done(), h.totals()
    h.close()
    return out


CASES = [
    ("1d", (64,), (4,), [1, 2], ((F, OUT),)),
    ("2d periodic", (64, 32), (4, 2), [1, 6], ((P, P), (P, P))),
    ("2d walls", (48, 32), (4, 4), [5, 6, 9], ((R, R), (OUT, F))),
    ("3d", (32, 32, 16), (2, 2, 2), [0, 3, 5], ((P, P), (P, P), (F, R))),
    ("3d ragged", (48, 24, 16), (3, 3, 2), [1, 4, 7, 13], ((P, P), (R, OUT), (P, P))),
]


@pytest.mark.parametrize("name,n,B,ref,bc", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_matches_oracle(H, name, n, B, ref, bc, precision):
    m = O.Mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=61)
    steps = 6
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, max_steps=steps)
    say("smr vs oracle", name, precision)
    U, t, s, T = run_gpu(H, S, W, precision, steps, 0.4)
    assert s == s_o == steps
    assert abs(t - t_o) <= (1e-14 if precision == 0 else 1e-6) * t_o
    a = U.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    b = U_o.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    rel = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    print(name, precision, "relL1", rel)
    assert np.all(rel <= TOL[precision]), rel
    # the device totals agree with the oracle's level-weighted totals
    T_o = S.totals(U)
    assert np.allclose(T, T_o, rtol=1e-12, atol=1e-12 * np.abs(T_o).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_conservation_across_level_jumps(H, precision):
    n, B, ref = (32, 32, 16), (2, 2, 2), [0, 3, 5]
    m = O.Mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=62, amp=0.3, mach=1.0)
    say("smr conservation", precision)
    h = H.Hydro(n, m.gamma, 0.3, precision=precision, blocks=B, refined=ref)
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


@pytest.mark.parametrize("precision", [0, 1])
def test_uniform_state_exact(H, precision):
    n, B, ref = (32, 32, 16), (2, 2, 2), [1, 2, 7]
    m = O.Mesh(n, 1.4)
    S = O.SMR(m, B, ref)
    W = np.empty(S.shape)
    W[:, 0], W[:, 1], W[:, 2], W[:, 3], W[:, 4] = 1.3, 0.7, -0.4, 0.2, 0.9
    say("smr uniform", precision)
    h = H.Hydro(n, 1.4, 0.4, precision=precision, blocks=B, refined=ref)
    h.set_primitive(W)
    U0 = h.get_state()
    h.step_auto(5)
    assert bitwise_equal(h.get_state(), U0)
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_nothing_refined_is_the_split_mesh(H, precision):
    c = wl.turbulence_3d(n=(32, 32, 16), mach=1.0, seed=63)
    B = (2, 2, 2)
    say("smr nothing refined", precision)
    a = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, blocks=B)
    a.set_primitive(c.W)
    a.step_auto(5)
    Ua = a.state_view().cpu().numpy()
    b = H.Hydro(c.n, c.gamma, c.cfl, precision=precision, blocks=B, refined=[])
    m = O.Mesh(c.n, c.gamma)
    S = O.SMR(m, B, [])
    Wb = np.ascontiguousarray(c.W.reshape(5, 2, 8, 2, 16, 2, 16).transpose(1, 3, 5, 0, 2, 4, 6).reshape(S.shape))
    b.set_primitive(Wb)
    b.step_auto(5)
    Ub = b.get_state()
    assert bitwise_equal(Ub, Ua)
    assert a.time() == b.time()
    a.close()
    b.close()


def test_everything_refined_is_the_fine_mesh(H):
    """All roots refined: the uniform mesh at twice the resolution."""
    c = wl.turbulence_3d(n=(32, 32, 32), mach=1.0, seed=64)
    say("smr everything refined")
    a = H.Hydro(c.n, c.gamma, c.cfl, precision=0, blocks=(4, 4, 4))
    a.set_primitive(c.W)
    a.step_auto(4)
    Ua = a.state_view().cpu().numpy()
    b = H.Hydro((16, 16, 16), c.gamma, c.cfl, precision=0, blocks=(2, 2, 2), refined=list(range(8)))
    Wb = np.ascontiguousarray(c.W.reshape(5, 4, 8, 4, 8, 4, 8).transpose(1, 3, 5, 0, 2, 4, 6).reshape(b.shape))
    b.set_primitive(Wb)
    b.step_auto(4)
    assert a.time() == b.time()
    assert bitwise_equal(b.get_state(), Ua)
    a.close()
    b.close()


def test_run_to_end_time_and_host_dt(H):
    n, B, ref = (64, 32), (4, 2), [1, 6]
    m = O.Mesh(n, 1.4, bc=((R, R), (P, P)))
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=65)
    U_o, t_o, s_o, dts = S.run(S.prim_to_cons(W), 0.4, max_steps=1000, t_end=0.05)
    say("smr t_end")
    U, t, s, _ = run_gpu(H, S, W, 0, 10000, 0.4, t_end=0.05)
    assert t == 0.05 and s == s_o
    rel = np.abs(U - U_o).sum() / np.abs(U_o).sum()
    assert rel <= 1e-12
    # host-chosen steps: the oracle's dt sequence
    h = H.Hydro(n, 1.4, 0.4, bc=m.bc, blocks=B, refined=ref)
    h.set_primitive(W)
    for dt in dts:
        h.step(dt)
    assert np.abs(h.get_state() - U_o).sum() / np.abs(U_o).sum() <= 1e-12
    h.close()


def test_refined_handle_rejects_unsupported_calls(H):
    h = H.Hydro((32, 32), 1.4, 0.4, blocks=(2, 2), refined=[0])
    for call in (lambda: h.stage_rhs(1e-3), lambda: h.padded_primitive(), lambda: h.autotune(1),
                 lambda: h.set_block_streams(True)):
        with pytest.raises(H.HydroError):
            call()
    with pytest.raises(H.HydroError):
        H.Batch([h])
    h.close()


def test_nonphysical_state_in_a_fine_block_is_reported(H):
    n, B, ref = (32, 32, 16), (2, 2, 2), [0, 3]
    m = O.Mesh(n, 1.4)
    S = O.SMR(m, B, ref)
    W = smooth_state(S, seed=66)
    W[-1, -1, 2, 3, 4] = -1.0                       # negative pressure in the last (fine) leaf
    assert S.leaves[-1][0] == 1
    say("smr nonphysical")
    h = H.Hydro(n, 1.4, 0.4, blocks=B, refined=ref)
    h.set_primitive(W)
    with pytest.raises(H.HydroError) as e:
        h.cfl_dt()
    assert e.value.status == H.E_NONPHYSICAL
    h.close()


def sod_state(S, x0=0.3, axis=0):
    """Sod's two states (1, 0, 1) | (0.125, 0, 0.1) split at x0 along axis."""
    X = S.centres()
    W = np.zeros(S.shape)
    left = X[axis] < x0
    W[:, 0] = np.where(left, 1.0, 0.125)
    W[:, -1] = np.where(left, 1.0, 0.1)
    return W


# a shock tube along x whose shock crosses level jumps: in 1-D a refined band
# (entered and left by t = 0.2); in 2-D and 3-D refined blocks that cover only
# part of the tube's cross-section, so level jumps also run along the flow
SHOCK_CASES = [
    ("1d band", (64,), (8,), [3, 4], ((F, F),), 0, 0.2),
    ("2d partial", (64, 32), (8, 4), [3, 4, 11, 12, 20], ((F, F), (P, P)), 70, 0.0),
    ("3d partial", (32, 16, 16), (4, 2, 2), [1, 2, 5, 14], ((F, F), (R, R), (P, P)), 45, 0.0),
]


@pytest.mark.parametrize("name,n,B,ref,bc,steps,t_end", SHOCK_CASES, ids=[c[0] for c in SHOCK_CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_shock_across_level_jumps_matches_oracle(H, name, n, B, ref, bc, steps, t_end, precision):
    """The minmod-limited prolongation and the fine-flux correction acting on
    a shock: GPU against the oracle.  FP64 to the 1e-12 gate; mixed to 1e-4
    (a shock: not the smooth-flow bound)."""
    m = O.Mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    W = sod_state(S)
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, max_steps=steps, t_end=t_end)
    say("smr shock vs oracle", name, precision)
    U, t, s, T = run_gpu(H, S, W, precision, steps if steps else s_o + 4, 0.4, t_end)
    assert s == s_o
    assert abs(t - t_o) <= (1e-14 if precision == 0 else 1e-6) * t_o
    a = U.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    b = U_o.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    rel = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    print(name, precision, "relL1", rel, "steps", s)
    assert np.all(rel <= (1e-12 if precision == 0 else 1e-4)), rel


# ---- refinement deeper than one level (codes: level << 26 | index on that
# level's block grid; the library adds the balance refinement the oracle does)
LS = 26
LEVEL_CASES = [
    ("1d three levels", (64,), (4,), [1, (1 << LS) | 3], ((F, OUT),)),
    ("2d three levels", (64, 32), (4, 2), [1, 6, (1 << LS) | 3, (1 << LS) | 20], ((P, P), (P, P))),
    ("2d walls, balance added", (64, 32), (4, 2), [1, 2, 5, 6, (1 << LS) | 3, (1 << LS) | 4],
     ((R, R), (OUT, F))),
    ("3d three levels", (32, 32, 16), (2, 2, 2), [0, (1 << LS) | 0, (1 << LS) | 5], ((P, P), (P, P), (F, R))),
    ("3d four levels", (32, 32, 32), (2, 2, 2), [0, (1 << LS) | 0, (2 << LS) | 0], ((P, P), (P, P), (P, P))),
]


@pytest.mark.parametrize("name,n,B,ref,bc", LEVEL_CASES, ids=[c[0] for c in LEVEL_CASES])
@pytest.mark.parametrize("precision", [0, 1])
def test_deeper_refinement_matches_oracle(H, name, n, B, ref, bc, precision):
    m = O.Mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() >= 2
    W = smooth_state(S, seed=67)
    steps = 6
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, max_steps=steps)
    say("smr levels vs oracle", name, precision)
    U, t, s, T = run_gpu(H, S, W, precision, steps, 0.4)
    assert s == s_o == steps
    assert abs(t - t_o) <= (1e-14 if precision == 0 else 1e-6) * t_o
    a = U.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    b = U_o.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    rel = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    print(name, precision, "leaves per level", np.bincount(S.leaves[:, 0]), "relL1", rel)
    assert np.all(rel <= TOL[precision]), rel
    T_o = S.totals(U)
    assert np.allclose(T, T_o, rtol=1e-12, atol=1e-12 * np.abs(T_o).max())


@pytest.mark.parametrize("precision", [0, 1])
def test_deeper_refinement_conserves_and_keeps_uniform_state(H, precision):
    n, B, ref = (32, 32, 16), (2, 2, 2), [0, 3, (1 << LS) | 0, (1 << LS) | 27]
    m = O.Mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    W = smooth_state(S, seed=68, amp=0.3, mach=1.0)
    say("smr levels conservation", precision)
    h = H.Hydro(n, m.gamma, 0.3, precision=precision, blocks=B, refined=ref)
    h.set_primitive(W)
    T0 = h.totals()
    h.step_auto(15)
    T1 = h.totals()
    h.close()
    scale = S.totals(np.abs(S.prim_to_cons(W)))
    print("drift", (T1 - T0) / scale)
    assert np.all(np.abs(T1 - T0) <= 1e-13 * scale)
    Wu = np.empty(S.shape)
    Wu[:, 0], Wu[:, 1], Wu[:, 2], Wu[:, 3], Wu[:, 4] = 1.3, 0.7, -0.4, 0.2, 0.9
    h = H.Hydro(n, 1.4, 0.4, precision=precision, blocks=B, refined=ref)
    h.set_primitive(Wu)
    U0 = h.get_state()
    h.step_auto(4)
    assert bitwise_equal(h.get_state(), U0)
    h.close()


def test_everything_refined_twice_is_the_mesh_four_times_finer(H):
    c = wl.turbulence_3d(n=(32, 32, 32), mach=1.0, seed=69)
    say("smr everything refined twice")
    a = H.Hydro(c.n, c.gamma, c.cfl, precision=0, blocks=(4, 4, 4))
    a.set_primitive(c.W)
    a.step_auto(3)
    Ua = a.state_view().cpu().numpy()
    codes = list(range(1)) + [(1 << LS) | i for i in range(8)]
    b = H.Hydro((8, 8, 8), c.gamma, c.cfl, precision=0, blocks=(1, 1, 1), refined=codes)
    assert np.all(b.leaves[:, 0] == 2)
    Wb = np.ascontiguousarray(c.W.reshape(5, 4, 8, 4, 8, 4, 8).transpose(1, 3, 5, 0, 2, 4, 6).reshape(b.shape))
    b.set_primitive(Wb)
    b.step_auto(3)
    assert a.time() == b.time()
    assert bitwise_equal(b.get_state(), Ua)
    a.close()
    b.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_shock_across_two_levels_of_jumps_matches_oracle(H, precision):
    """Sod's shock through a band refined twice (1-D, to t = 0.2)."""
    n, B, ref, bc = (64,), (8,), [3, 4, (1 << LS) | 7, (1 << LS) | 8], ((F, F),)
    m = O.Mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    W = sod_state(S)
    U_o, t_o, s_o, _ = S.run(S.prim_to_cons(W), 0.4, t_end=0.2)
    say("smr shock two levels", precision)
    U, t, s, T = run_gpu(H, S, W, precision, s_o + 4, 0.4, 0.2)
    assert s == s_o and t == 0.2
    a = U.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    b = U_o.transpose(1, 0, 2, 3, 4).reshape(m.ncomp, -1)
    rel = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    print("shock two levels", precision, "relL1", rel, "steps", s)
    assert np.all(rel <= (1e-12 if precision == 0 else 1e-4)), rel
