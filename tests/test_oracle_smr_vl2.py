"""Pins of the oracle's van Leer integrator on a statically refined mesh
(Sec. 3.3: the half-step predictor from piecewise-constant states, then the
full step from PLM states of the predicted state; Sec. 2.3 and Sec. 3: both
stages take the cross-level ghosts and the fine-flux average at level jumps).

Pinned by what the mathematics fixes:
  * no refined block: the van Leer block-mesh run, bit for bit;
  * every block refined (once or twice): the van Leer run on the uniform mesh
    two or four times finer, bit for bit (this fixes the predictor's order
    and half step and the corrector's full step from U^n);
  * a uniform state stays uniform, bit for bit, across one and two jumps;
  * conservation to round-off with level jumps;
  * mirror symmetry to round-off;
  * a smooth wave and a shock tube: the error lies between those of the
    coarse and the fine uniform van Leer runs;
  * a planted mistake (Heun in place of van Leer for the refined run) is
    caught by the uniform-fine-mesh identity.
CPU only.
"""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl

P, F, OUT, R = O.BC_PERIODIC, O.BC_FREE, O.BC_OUTFLOW, O.BC_REFLECT
LS = 26


def code(level, index):
    return (level << LS) | index


def to_blocks(U, blocks):
    """Mesh layout (nc, nz, ny, nx) -> block layout (nblk, nc, bz, by, bx)."""
    nc, nz, ny, nx = U.shape
    B = list(blocks) + [1] * (3 - len(blocks))
    bz, by, bx = nz // B[2], ny // B[1], nx // B[0]
    V = U.reshape(nc, B[2], bz, B[1], by, B[0], bx).transpose(1, 3, 5, 0, 2, 4, 6)
    return V.reshape(B[0] * B[1] * B[2], nc, bz, by, bx).copy()


def vl2_mesh(*args, **kw):
    m = O.Mesh(*args, **kw)
    m.integrator = O.VL2
    return m


def test_no_refinement_is_the_vl2_block_run():
    c = wl.turbulence_3d(n=(16, 16, 8), mach=1.0, seed=61)
    m = vl2_mesh(c.n, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(m, c.W)
    U, t, s, dts = O.run_blocks(m, (2, 2, 1), U0, c.cfl, max_steps=4)
    S = O.SMR(m, (2, 2, 1), [])
    Us, ts, ss, dtss = S.run(to_blocks(U0, (2, 2, 1)), c.cfl, max_steps=4)
    assert t == ts and np.array_equal(dts, dtss)
    assert np.array_equal(Us, to_blocks(U, (2, 2, 1)))


def _fine_case(ndim, factor, seed):
    n = (16, 8, 8)[:ndim]
    B = (2, 2, 2)[:ndim]
    fine = tuple(factor * v for v in n)
    c = wl.turbulence_3d(n=fine, mach=1.0, seed=seed, ndim=ndim) if ndim > 1 else wl.smooth_1d(N=fine[0], seed=seed)
    return n, B, fine, c


@pytest.mark.parametrize("integ", [O.VL2, O.HEUN])
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_refining_everything_is_the_uniform_fine_vl2_run(ndim, integ):
    """The refined van Leer run equals the uniform fine van Leer run; a
    refined run with the other integrator (the planted mistake) does not."""
    n, B, fine, c = _fine_case(ndim, 2, 62)
    mf = vl2_mesh(fine, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(mf, c.W)
    U, t, s, dts = O.run(mf, U0, c.cfl, max_steps=4)
    m = O.Mesh(n, c.gamma, c.lo, c.hi, c.bc)
    m.integrator = integ
    S = O.SMR(m, B, list(range(int(np.prod(B)))))
    FB = tuple(2 * v for v in B)
    Us, ts, ss, dtss = S.run(to_blocks(U0, FB), c.cfl, max_steps=4)
    same = t == ts and np.array_equal(dts, dtss) and np.array_equal(Us, to_blocks(U, FB))
    assert same == (integ == O.VL2)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_refining_everything_twice_is_the_uniform_mesh_four_times_finer(ndim):
    n, B, fine, c = _fine_case(ndim, 4, 63)
    mf = vl2_mesh(fine, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(mf, c.W)
    U, t, s, dts = O.run(mf, U0, c.cfl, max_steps=3)
    m = vl2_mesh(n, c.gamma, c.lo, c.hi, c.bc)
    nroot = int(np.prod(B))
    ref = list(range(nroot)) + [code(1, i) for i in range(nroot * 2 ** ndim)]
    S = O.SMR(m, B, ref)
    assert np.all(S.leaves[:, 0] == 2)
    FB = tuple(4 * v for v in B)
    Us, ts, ss, dtss = S.run(to_blocks(U0, FB), c.cfl, max_steps=3)
    assert t == ts and np.array_equal(dts, dtss)
    assert np.array_equal(Us, to_blocks(U, FB))


# one level of jumps (PATTERNS of the Heun pins) and two (LEVEL_PATTERNS)
CASES = {
    "2d one jump": ((32, 16), (4, 2), [1, 6]),
    "3d one jump": ((16, 16, 8), (2, 2, 1), [0, 3]),
    "2d two jumps": ((32, 16), (4, 2), [code(0, 1), code(0, 6), code(1, 3), code(1, 20)]),
    "3d two jumps": ((16, 16, 8), (2, 2, 1), [code(0, 0), code(1, 0), code(1, 5)]),
}


@pytest.mark.parametrize("case", list(CASES))
def test_uniform_state_preserved_bitwise(case):
    n, B, ref = CASES[case]
    ndim = len(n)
    m = vl2_mesh(n, 1.4)
    S = O.SMR(m, B, ref)
    W = np.empty(S.shape)
    W[:, 0] = 1.3
    for d in range(ndim):
        W[:, 1 + d] = (0.7, -0.4, 0.2)[d]
    W[:, -1] = 0.9
    U0 = S.prim_to_cons(W)
    U, *_ = S.run(U0, 0.4, max_steps=5)
    assert np.array_equal(U, U0)


@pytest.mark.parametrize("case", list(CASES))
def test_conservation_across_level_jumps(case):
    n, B, ref = CASES[case]
    ndim = len(n)
    m = vl2_mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    rng = np.random.default_rng(64)
    X = S.centres()
    W = np.empty(S.shape)
    W[:, 0] = 1.0 + 0.2 * np.sin(2 * np.pi * X[0]) + 0.2 * rng.random(X[0].shape)
    for d in range(ndim):
        W[:, 1 + d] = 0.3 * (rng.random(X[0].shape) - 0.5)
    W[:, -1] = 1.0 + 0.1 * rng.random(X[0].shape)
    U0 = S.prim_to_cons(W)
    U, *_ = S.run(U0, 0.3, max_steps=8)
    T0, T1 = S.totals(U0), S.totals(U)
    scale = S.totals(np.abs(U0))
    assert np.all(np.abs(T1 - T0) <= 1e-14 * scale), (T1 - T0, scale)


def test_mirror_symmetry():
    """Mirror-symmetric refinement (two levels) and state in a reflecting x
    channel stay mirror-symmetric to round-off."""
    n, B = (32, 16), (4, 2)
    ref = [code(0, 1), code(0, 2), code(0, 5), code(0, 6), code(1, 3), code(1, 4)]
    m = vl2_mesh(n, 1.4, bc=((R, R), (P, P)))
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    X, Y = S.centres()
    xs = X - 0.5
    W = np.empty(S.shape)
    W[:, 0] = 1.0 + 0.3 * np.exp(-(xs * xs) * 20.0) * (1.0 + 0.2 * np.cos(2 * np.pi * Y))
    W[:, 1] = xs * (0.5 + np.cos(2 * np.pi * Y) ** 2)
    W[:, 2] = 0.1 * np.cos(2 * np.pi * Y) * (1.0 - xs * xs)
    W[:, 3] = 1.0 + 0.2 * (xs * xs)
    U, *_ = S.run(S.prim_to_cons(W), 0.4, max_steps=15)
    index = {tuple(l): i for i, l in enumerate(S.leaves)}
    for i, (L, cx, cy, cz) in enumerate(S.leaves):
        j = index[(L, B[0] * 2 ** L - 1 - cx, cy, cz)]
        mir = U[j][..., ::-1].copy()
        mir[1] = -mir[1]
        assert np.abs(mir - U[i]).max() <= 1e-13, (i, j)


def _wave_state(S, amp=1e-3, gamma=5.0 / 3.0):
    """Right-going sound wave along x: rho = 1, p = 1/gamma, so c = 1."""
    X = S.centres()
    W = np.zeros(S.shape)
    ph = 2 * np.pi * X[0]
    W[:, 0] = 1.0 + amp * np.sin(ph)
    W[:, 1] = amp * np.sin(ph)
    W[:, -1] = 1.0 / gamma + amp * np.sin(ph)
    return W


def test_smooth_wave_error_between_uniform_runs():
    gamma = 5.0 / 3.0

    def err(n, B, ref):
        m = vl2_mesh((n,), gamma)
        S = O.SMR(m, (B,), ref)
        W0 = _wave_state(S)
        U, t, s, _ = S.run(S.prim_to_cons(W0), 0.4, t_end=1.0)
        W = S.cons_to_prim(U)
        dV = (1.0 / n) / 2.0 ** S.leaves[:, 0]
        return float((np.abs(W[:, 0] - W0[:, 0]).reshape(len(S.leaves), -1).sum(axis=1) * dV).sum())

    e_coarse, e_fine = err(64, 8, []), err(128, 16, [])
    e_smr = err(64, 8, [2, 3, 4, 5])
    assert e_fine < e_smr < e_coarse, (e_fine, e_smr, e_coarse)
    e_half = err(32, 8, [2, 3, 4, 5])
    assert e_half / e_smr > 2.5, (e_half, e_smr)


def test_shock_through_refined_band_error_between_uniform_runs():
    """Sod's tube crossing a refined band and its two level jumps."""
    gamma, x0 = 1.4, 0.3
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)

    def err(n, B, ref):
        m = vl2_mesh((n,), gamma, bc=((F, F),))
        S = O.SMR(m, (B,), ref)
        X = S.centres()
        W = np.zeros(S.shape)
        lft = X[0] < x0
        W[:, 0] = np.where(lft, 1.0, 0.125)
        W[:, -1] = np.where(lft, 1.0, 0.1)
        U, t, s, _ = S.run(S.prim_to_cons(W), 0.4, t_end=0.2)
        assert t == 0.2
        W = S.cons_to_prim(U)
        ex = O.exact_sample(gamma, left, right, ((X[0] - x0) / t).ravel())[0].reshape(X[0].shape)
        dV = (1.0 / n) / 2.0 ** S.leaves[:, 0]
        return float((np.abs(W[:, 0] - ex).reshape(len(S.leaves), -1).sum(axis=1) * dV).sum())

    e_coarse, e_fine = err(64, 8, []), err(128, 16, [])
    e_band = err(64, 8, [3, 4])
    assert e_fine < e_band < e_coarse, (e_fine, e_band, e_coarse)
