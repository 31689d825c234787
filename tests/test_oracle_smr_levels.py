"""Pins of the oracle's refinement deeper than one level (the 2^d-tree of
Sec. 2.3 applied recursively, with refinement added so that face-neighbouring
blocks differ by at most one level): a block of level L is listed by the code
L * 2^26 + its index on the level-L block grid, after its parent.

Pinned by what the mathematics fixes, as for one level:
  * every block refined twice: the uniform mesh at four times the
    resolution, bit for bit;
  * a uniform state stays uniform, bit for bit, across level jumps;
  * a linear primitive field: every c-boundary ghost (same level, restricted
    or prolonged) equals the field at the ghost's centre;
  * conservation to round-off with level jumps on two levels of jumps;
  * mirror symmetry to round-off;
  * a smooth wave: the error lies between those of the coarse and the fine
    uniform meshes;
and the tree itself: the leaves of a hand-worked refinement, the balance
refinement the paper's rule adds, and refused specifications.  CPU only.
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


def all_codes(B, level):
    return [code(level, i) for i in range(int(np.prod([b << level for b in B])))]


def leaf_set(S):
    return {tuple(int(v) for v in l) for l in S.leaves}


def test_hand_worked_tree_with_balance():
    """1-D, four roots.  Refine root 1 (children 2, 3 at level 1) and its
    right child 3 (children 6, 7 at level 2).  Level-2 block 7 then touches
    root 2 across a face, two levels apart, so the balance rule refines root
    2 (children 4, 5 at level 1).  Leaves in order: roots 0 and 3, level-1
    blocks 2, 4, 5, level-2 blocks 6, 7."""
    m = O.Mesh((32,), 1.4, bc=((F, F),))
    S = O.SMR(m, (4,), [code(0, 1), code(1, 3)])
    assert [tuple(l[:2]) for l in S.leaves] == [(0, 0), (0, 3), (1, 2), (1, 4), (1, 5), (2, 6), (2, 7)]
    # without the level-1 code it is the one-level refinement
    S1 = O.SMR(m, (4,), [code(0, 1)])
    assert [tuple(l[:2]) for l in S1.leaves] == [(0, 0), (0, 2), (0, 3), (1, 2), (1, 3)]


@pytest.mark.parametrize("ndim", [2, 3])
def test_leaves_are_balanced(ndim):
    """A deep corner refinement: no two face-neighbouring leaves differ by
    more than one level, the leaves tile the domain exactly once, and the
    balance rule added blocks beyond the listed ones."""
    B = (2,) * ndim
    n = (8,) * ndim
    m = O.Mesh(n, 1.4)
    E1 = [2 * b for b in B]
    # refine root 0, its level-1 corner child 0 (the listed chain)
    S = O.SMR(m, B, [code(0, 0), code(1, 0)])
    levels = {}
    for L, *c in S.leaves:
        levels[(L, *c[:ndim])] = L
    # cover: sum of leaf volumes = 1 (in units of a root)
    vol = sum(0.5 ** (ndim * L) for L in S.leaves[:, 0])
    assert vol == np.prod(B)
    # face neighbours at the finest grid differ by at most one level
    Lmax = int(S.leaves[:, 0].max())
    fine = {}
    for L, *c in S.leaves:
        k = 2 ** (Lmax - L)
        rng = [range(c[d] * k, (c[d] + 1) * k) for d in range(ndim)]
        for x in np.stack(np.meshgrid(*rng, indexing="ij"), -1).reshape(-1, ndim):
            fine[tuple(x)] = L
    ext = [b << Lmax for b in B]
    for x, L in fine.items():
        for d in range(ndim):
            y = list(x)
            y[d] = (y[d] + 1) % ext[d]                    # periodic
            assert abs(fine[tuple(y)] - L) <= 1
    assert Lmax == 2
    listed = 1 + 2 ** ndim - 1 + 2 ** ndim            # root 0 split, child 0 split
    assert len(S.leaves) > np.prod(B) - 1 + listed - 1    # balance added blocks


@pytest.mark.parametrize("spec", [
    [code(1, 0)],                          # a level-1 block whose parent is not listed: refused
    [code(0, 0), code(1, 0), code(2, 0)],  # a level-2 block with its ancestors: leaves reach level 3
])
def test_refused_or_accepted_specs(spec):
    m = O.Mesh((32, 16), 1.4)
    if spec[-1] >> LS == 2:
        S = O.SMR(m, (4, 2), spec)
        assert S.leaves[:, 0].max() == 3
    else:
        with pytest.raises(O.OracleError):
            O.SMR(m, (4, 2), spec)


@pytest.mark.parametrize("bad", [[code(3, 0)], [code(0, 8)], [code(0, 1), code(0, 1)], [-1]])
def test_invalid_codes_rejected(bad):
    m = O.Mesh((32, 16), 1.4)
    with pytest.raises(O.OracleError):
        O.SMR(m, (4, 2), bad)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_refining_everything_twice_is_the_uniform_mesh_four_times_finer(ndim):
    n = (8, 8, 4)[:ndim]
    B = (2, 2, 1)[:ndim]
    fine = tuple(4 * v for v in n)
    c = wl.turbulence_3d(n=fine, mach=1.0, seed=57, ndim=ndim) if ndim > 1 else wl.smooth_1d(N=fine[0], seed=57)
    mf = O.Mesh(fine, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(mf, c.W)
    U, t, s, dts = O.run(mf, U0, c.cfl, max_steps=3)
    m = O.Mesh(n, c.gamma, c.lo, c.hi, c.bc)
    S = O.SMR(m, B, all_codes(B, 0) + all_codes(B, 1))
    assert np.all(S.leaves[:, 0] == 2)
    FB = tuple(4 * v for v in B)
    Us, ts, ss, dtss = S.run(to_blocks(U0, FB), c.cfl, max_steps=3)
    assert t == ts and np.array_equal(dts, dtss)
    assert np.array_equal(Us, to_blocks(U, FB))


LEVEL_PATTERNS = {
    1: ((32,), (4,), [code(0, 1), code(1, 3)]),
    2: ((32, 16), (4, 2), [code(0, 1), code(0, 6), code(1, 3), code(1, 20)]),
    3: ((16, 16, 8), (2, 2, 1), [code(0, 0), code(1, 0), code(1, 5)]),
}


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_uniform_state_preserved_bitwise_three_levels(ndim):
    n, B, ref = LEVEL_PATTERNS[ndim]
    m = O.Mesh(n, 1.4)
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    W = np.empty(S.shape)
    W[:, 0] = 1.3
    for d in range(ndim):
        W[:, 1 + d] = (0.7, -0.4, 0.2)[d]
    W[:, -1] = 0.9
    U0 = S.prim_to_cons(W)
    U, *_ = S.run(U0, 0.4, max_steps=5)
    assert np.array_equal(U, U0)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_linear_field_ghosts_exact_three_levels(ndim):
    """Every ghost across a c-boundary between leaves of levels 0, 1 and 2
    (same level, restricted, prolonged) equals the linear field at its
    centre."""
    n, B, ref = LEVEL_PATTERNS[ndim]
    hi = (2.0, 1.0, 1.0)[:ndim]
    m = O.Mesh(n, 1.4, lo=(0.0,) * ndim, hi=hi, bc=((F, F),) * ndim)
    S = O.SMR(m, B, ref)
    grads = [(0.3, -0.2, 0.1), (-0.5, 0.25, 0.4), (0.125, 0.5, -0.3), (0.2, 0.1, 0.05), (0.1, -0.1, 0.2)]
    coeffs = [(2.0 + c, grads[c][:ndim]) for c in range(ndim + 2)]
    X = S.centres()
    W = np.empty(S.shape)
    for comp, (a0, grad) in enumerate(coeffs):
        W[:, comp] = a0 + sum(g * x for g, x in zip(grad, X))
    Wp = S.ghosts(W)
    dx0 = [(m.hi[d] - m.lo[d]) / m.n[d] for d in range(ndim)]
    bn = S.bn
    at = {(int(l[0]),) + tuple(int(v) for v in l[1:1 + ndim]): i for i, l in enumerate(S.leaves)}
    checked = {"same": 0, "restricted": 0, "prolonged": 0}
    for b, (L, *cc) in enumerate(S.leaves):
        cc = [int(v) for v in cc[:ndim]]
        dx = [v / 2 ** L for v in dx0]
        for d in range(ndim):
            E = B[d] * 2 ** L
            for s in (0, 1):
                q = cc[d] + (1 if s else -1)
                if q < 0 or q >= E:
                    continue
                nb = list(cc)
                nb[d] = q
                if (L,) + tuple(nb) in at:
                    kind = "same"
                elif L > 0 and (L - 1,) + tuple(v // 2 for v in nb) in at:
                    kind = "prolonged"
                else:
                    kind = "restricted"
                for l in range(2):
                    gi = bn[d] + l if s else -1 - l
                    sl = [slice(2, 2 + bn[e]) if e < ndim else slice(0, 1) for e in range(3)]
                    sl[d] = gi + 2
                    x = [None] * ndim
                    for e in range(ndim):
                        idx = np.arange(bn[e]) if e != d else np.array([gi])
                        x[e] = m.lo[e] + (cc[e] * bn[e] + idx + 0.5) * dx[e]
                    grid = np.meshgrid(*[x[e] for e in range(ndim)], indexing="ij")
                    keep = np.ones(grid[0].shape, dtype=bool)
                    if kind == "prolonged":
                        # a coarse cell whose transverse slope, or that of a
                        # coarser ancestor its neighbours were prolonged from,
                        # comes from a p-boundary ghost: left out (within
                        # 2^(L-1) coarse cells of a mesh face)
                        for e in range(ndim):
                            if e == d:
                                continue
                            coarse = (cc[e] * bn[e] + np.arange(bn[e])) // 2
                            reach = 2 ** (L - 1)
                            edge = (coarse < reach) | (coarse >= (n[e] << (L - 1)) - reach)
                            shp = [1] * ndim
                            shp[e] = bn[e]
                            keep &= ~np.broadcast_to(edge.reshape(shp), keep.shape)
                    for comp, (a0, grad) in enumerate(coeffs):
                        exact = a0 + sum(g * xx for g, xx in zip(grad, grid))
                        got = Wp[b, comp][tuple(sl[::-1])]
                        got = np.transpose(got.reshape([bn[e] if e != d else 1 for e in range(3)][::-1]),
                                           list(range(3))[::-1]).reshape(exact.shape)
                        assert np.allclose(got[keep], exact[keep], rtol=0, atol=1e-13), (kind, b, d, s, l, comp)
                    checked[kind] += 1
    assert all(v > 0 for v in checked.values()), checked


@pytest.mark.parametrize("ndim", [2, 3])
def test_conservation_three_levels(ndim):
    n, B, ref = LEVEL_PATTERNS[ndim]
    m = O.Mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    rng = np.random.default_rng(58)
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


def test_mirror_symmetry_three_levels():
    """A refinement and a state mirror-symmetric in x, in a reflecting x
    channel, stay mirror-symmetric to round-off across two levels of jumps."""
    n, B = (32, 16), (4, 2)
    # root blocks 1, 2 (and 5, 6), and at level 1 the inner children next to
    # the centre line: 3 and 4 on row 0 of the level-1 grid (mirror pair)
    ref = [code(0, 1), code(0, 2), code(0, 5), code(0, 6), code(1, 3), code(1, 4)]
    m = O.Mesh(n, 1.4, bc=((R, R), (P, P)))
    S = O.SMR(m, B, ref)
    assert S.leaves[:, 0].max() == 2
    X, Y = S.centres()
    xs = X - 0.5
    W = np.empty(S.shape)
    W[:, 0] = 1.0 + 0.3 * np.exp(-(xs * xs) * 20.0) * (1.0 + 0.2 * np.cos(2 * np.pi * Y))
    W[:, 1] = xs * (0.5 + np.cos(2 * np.pi * Y) ** 2)
    W[:, 2] = 0.1 * np.cos(2 * np.pi * Y) * (1.0 - xs * xs)
    W[:, 3] = 1.0 + 0.2 * (xs * xs)
    U, *_ = S.run(S.prim_to_cons(W), 0.4, max_steps=12)
    index = {tuple(int(v) for v in l): i for i, l in enumerate(S.leaves)}
    for i, (L, cx, cy, cz) in enumerate(S.leaves):
        j = index[(int(L), int(B[0] * 2 ** L - 1 - cx), int(cy), int(cz))]
        mir = U[j][..., ::-1].copy()
        mir[1] = -mir[1]
        assert np.abs(mir - U[i]).max() <= 1e-13, (i, j)


def test_smooth_wave_error_between_uniform_runs_three_levels():
    """A sound wave across a band refined twice: the error after one crossing
    lies between those of the coarse and the four-times-finer uniform
    meshes, and below that of the band refined once."""
    gamma = 5.0 / 3.0

    def err(n, B, ref):
        m = O.Mesh((n,), gamma)
        S = O.SMR(m, (B,), ref)
        X = S.centres()
        W0 = np.empty(S.shape)
        ph = 2 * np.pi * X[0]
        W0[:, 0] = 1.0 + 1e-3 * np.sin(ph)
        W0[:, 1] = 1e-3 * np.sin(ph)
        W0[:, 2] = 1.0 / gamma + 1e-3 * np.sin(ph)
        U, t, s, _ = S.run(S.prim_to_cons(W0), 0.4, t_end=1.0)
        W = S.cons_to_prim(U)
        dV = (1.0 / n) / 2.0 ** S.leaves[:, 0]
        return float((np.abs(W[:, 0] - W0[:, 0]).reshape(len(S.leaves), -1).sum(axis=1) * dV).sum())

    e_coarse, e_fine = err(32, 4, []), err(128, 16, [])
    once = [code(0, 1), code(0, 2)]
    e_once = err(32, 4, once)
    e_twice = err(32, 4, once + [code(1, 3), code(1, 4)])
    assert e_fine < e_twice < e_once < e_coarse, (e_fine, e_twice, e_once, e_coarse)
