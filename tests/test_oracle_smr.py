"""Pins of the oracle's two-level static mesh refinement (the 2^d-tree of
Sec. 2.3 one level deep, cross-level c-boundaries of Sec. 3): restriction by
volume averages, minmod-limited prolongation (eq. minmod) on primitive
variables, and the fine-flux average on the coarse side of a level jump.

Pinned by what the mathematics fixes:
  * no refined block: the block-mesh run, bit for bit;
  * every block refined: the uniform mesh at twice the resolution, bit for bit;
  * a uniform state stays uniform, bit for bit, across level jumps;
  * a linear primitive field: every c-boundary ghost (same level, restricted
    or prolonged) equals the field at the ghost's centre;
  * conservation to round-off with level jumps (flux correction);
  * mirror symmetry to round-off;
  * a smooth wave: the error lies between those of the coarse and the fine
    uniform meshes.
CPU only.
"""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl

P, F, OUT, R = O.BC_PERIODIC, O.BC_FREE, O.BC_OUTFLOW, O.BC_REFLECT


def to_blocks(U, blocks):
    """Mesh layout (nc, nz, ny, nx) -> block layout (nblk, nc, bz, by, bx)."""
    nc, nz, ny, nx = U.shape
    B = list(blocks) + [1] * (3 - len(blocks))
    bz, by, bx = nz // B[2], ny // B[1], nx // B[0]
    V = U.reshape(nc, B[2], bz, B[1], by, B[0], bx).transpose(1, 3, 5, 0, 2, 4, 6)
    return V.reshape(B[0] * B[1] * B[2], nc, bz, by, bx).copy()


def test_no_refinement_is_the_block_run():
    c = wl.turbulence_3d(n=(16, 16, 8), mach=1.0, seed=51)
    m = O.Mesh(c.n, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(m, c.W)
    U, t, s, dts = O.run_blocks(m, (2, 2, 1), U0, c.cfl, max_steps=4)
    S = O.SMR(m, (2, 2, 1), [])
    Us, ts, ss, dtss = S.run(to_blocks(U0, (2, 2, 1)), c.cfl, max_steps=4)
    assert t == ts and np.array_equal(dts, dtss)
    assert np.array_equal(Us, to_blocks(U, (2, 2, 1)))


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_refining_everything_is_the_uniform_fine_mesh(ndim):
    n = (16, 8, 8)[:ndim]
    B = (2, 2, 2)[:ndim]
    fine = tuple(2 * v for v in n)
    c = wl.turbulence_3d(n=fine + (1,) * 0 if ndim == 3 else fine, mach=1.0, seed=52, ndim=ndim) \
        if ndim > 1 else wl.smooth_1d(N=fine[0], seed=52)
    mf = O.Mesh(fine, c.gamma, c.lo, c.hi, c.bc)
    U0 = O.prim_to_cons(mf, c.W)
    U, t, s, dts = O.run(mf, U0, c.cfl, max_steps=4)
    m = O.Mesh(n, c.gamma, c.lo, c.hi, c.bc)
    S = O.SMR(m, B, list(range(int(np.prod(B)))))
    assert np.all(S.leaves[:, 0] == 1)
    FB = tuple(2 * v for v in B)
    Us, ts, ss, dtss = S.run(to_blocks(U0, FB), c.cfl, max_steps=4)
    assert t == ts and np.array_equal(dts, dtss)
    assert np.array_equal(Us, to_blocks(U, FB))


PATTERNS = {
    1: ((32,), (4,), [1, 2], ((F, OUT),)),
    2: ((32, 16), (4, 2), [1, 6], ((P, P), (R, R))),
    3: ((16, 16, 8), (2, 2, 1), [0, 3], ((P, P), (P, P), (F, R))),
}


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_uniform_state_preserved_bitwise(ndim):
    n, B, ref, bc = PATTERNS[ndim]
    m = O.Mesh(n, 1.4, bc=bc)
    S = O.SMR(m, B, ref)
    W = np.empty(S.shape)
    W[:, 0] = 1.3
    for d in range(ndim):
        W[:, 1 + d] = (0.7, -0.4, 0.2)[d]
    W[:, -1] = 0.9
    U0 = S.prim_to_cons(W)
    U, *_ = S.run(U0, 0.4, max_steps=5)
    # reflecting and outflow faces change a moving uniform state near them;
    # the cells away from the mesh faces stay exactly uniform only for a
    # periodic mesh, so compare with the same mesh unrefined where needed
    if all(b == (P, P) for b in bc):
        assert np.array_equal(U, U0)
    else:
        W0 = np.empty(S.shape)
        W0[:] = W
        W0[:, 1:1 + ndim] = 0.0                       # at rest: every boundary rule keeps it
        U0 = S.prim_to_cons(W0)
        U, *_ = S.run(U0, 0.4, max_steps=5)
        assert np.array_equal(U, U0)


def _linear(S, coeffs):
    X = S.centres()
    W = np.empty(S.shape)
    for comp, (a0, grad) in enumerate(coeffs):
        W[:, comp] = a0 + sum(g * x for g, x in zip(grad, X))
    return W


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_linear_field_ghosts_exact(ndim):
    """Every ghost across a c-boundary (same level, restricted onto a coarse
    block, prolonged onto a fine one) equals the linear field at its centre."""
    n = (32, 16, 16)[:ndim]
    B = (4, 2, 2)[:ndim]
    ref = {1: [1, 2], 2: [1, 2, 5], 3: [1, 2, 5]}[ndim]
    m = O.Mesh(n, 1.4, lo=(0.0,) * ndim, hi=(2.0, 1.0, 1.0)[:ndim], bc=((F, F),) * ndim)
    S = O.SMR(m, B, ref)
    grads = [(0.3, -0.2, 0.1), (-0.5, 0.25, 0.4), (0.125, 0.5, -0.3), (0.2, 0.1, 0.05), (0.1, -0.1, 0.2)]
    coeffs = [(2.0 + c, grads[c][:ndim]) for c in range(ndim + 2)]
    W = _linear(S, coeffs)
    Wp = S.ghosts(W)
    dx0 = [(m.hi[d] - m.lo[d]) / m.n[d] for d in range(ndim)]
    bn = S.bn
    checked = {"same": 0, "restricted": 0, "prolonged": 0}
    levels = {tuple(l[1:]) + (l[0],): i for i, l in enumerate(S.leaves)}
    for b, (L, *cc) in enumerate(S.leaves):
        dx = [v / 2 ** L for v in dx0]
        for d in range(ndim):
            E = B[d] * 2 ** L
            for s in (0, 1):
                q = cc[d] + (1 if s else -1)
                if q < 0 or q >= E:
                    continue                                  # a mesh face: p-boundary rule
                nb = list(cc)
                nb[d] = q
                if tuple(nb) + (L,) in levels:
                    kind = "same"
                elif L == 1:
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
                    # a prolonged ghost whose coarse cell lies on a mesh face
                    # takes a transverse slope from a p-boundary ghost (not
                    # part of the linear field): leave those out
                    keep = np.ones(grid[0].shape, dtype=bool)
                    if kind == "prolonged":
                        for e in range(ndim):
                            if e == d:
                                continue
                            coarse = (cc[e] * bn[e] + np.arange(bn[e])) // 2
                            edge = (coarse == 0) | (coarse == n[e] - 1)
                            shp = [1] * ndim
                            shp[e] = bn[e]
                            keep &= ~np.broadcast_to(edge.reshape(shp), keep.shape)
                    for comp, (a0, grad) in enumerate(coeffs):
                        exact = a0 + sum(g * xx for g, xx in zip(grad, grid))   # axes (x, y, z)
                        got = Wp[b, comp][tuple(sl[::-1])]
                        got = np.transpose(got.reshape([bn[e] if e != d else 1 for e in range(3)][::-1]),
                                           list(range(3))[::-1]).reshape(exact.shape)
                        assert np.allclose(got[keep], exact[keep], rtol=0, atol=1e-13), (kind, b, d, s, l, comp)
                    checked[kind] += 1
    assert all(v > 0 for v in checked.values()), checked


def _wave_state(S, amp=1e-3, gamma=5.0 / 3.0):
    """Right-going sound wave along x: rho = 1, p = 1/gamma, so c = 1 and
    delta v = delta p = delta rho."""
    X = S.centres()
    W = np.empty(S.shape)
    ph = 2 * np.pi * X[0]
    W[:, 0] = 1.0 + amp * np.sin(ph)
    W[:, 1] = amp * np.sin(ph)
    for d in range(1, S.mesh.ndim):
        W[:, 1 + d] = 0.0
    W[:, -1] = 1.0 / gamma + amp * np.sin(ph)
    return W


@pytest.mark.parametrize("ndim", [2, 3])
def test_conservation_across_level_jumps(ndim):
    n, B, ref, _ = PATTERNS[ndim]
    m = O.Mesh(n, 5.0 / 3.0)
    S = O.SMR(m, B, ref)
    rng = np.random.default_rng(53)
    W = _wave_state(S, amp=0.05)
    W[:, 0] *= 1.0 + 0.2 * rng.random(W[:, 0].shape)
    W[:, 1:1 + ndim] += 0.3 * (rng.random(W[:, 1:1 + ndim].shape) - 0.5)
    U0 = S.prim_to_cons(W)
    U, *_ = S.run(U0, 0.3, max_steps=8)
    T0, T1 = S.totals(U0), S.totals(U)
    scale = np.abs(U0).reshape(U0.shape[0], U0.shape[1], -1).sum(axis=(0, 2)) / np.prod(n)
    assert np.all(np.abs(T1 - T0) <= 1e-14 * scale), (T1 - T0, scale)


def test_mirror_symmetry():
    """Mirror-symmetric refinement and state in a reflecting x channel stay
    mirror-symmetric to round-off (the HLLC arithmetic itself is not exactly
    antisymmetric under a mirror, so neither is the unrefined run; a wrong
    side or offset in a cross-level ghost would show at the 1e-3 level)."""
    n, B = (32, 16), (4, 2)
    ref = [1, 2, 5, 6]                                   # symmetric under bx -> 3 - bx
    m = O.Mesh(n, 1.4, bc=((R, R), (P, P)))
    S = O.SMR(m, B, ref)
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


def test_smooth_wave_error_between_uniform_runs():
    """A sound wave across a refined band: the error after one crossing lies
    between those of the coarse and the fine uniform meshes."""
    gamma = 5.0 / 3.0

    def err(n, B, ref):
        m = O.Mesh((n,), gamma)
        S = O.SMR(m, (B,), ref)
        W0 = _wave_state(S)
        U, t, s, _ = S.run(S.prim_to_cons(W0), 0.4, t_end=1.0)
        W = S.cons_to_prim(U)
        dV = (1.0 / n) / 2.0 ** S.leaves[:, 0]
        return float((np.abs(W[:, 0] - W0[:, 0]).reshape(len(S.leaves), -1).sum(axis=1) * dV).sum())

    e_coarse = err(64, 8, [])
    e_fine = err(128, 16, [])
    e_smr = err(64, 8, [2, 3, 4, 5])
    assert e_fine < e_smr < e_coarse, (e_fine, e_smr, e_coarse)
    # and it converges at close to second order with the base resolution
    e_half = err(32, 8, [2, 3, 4, 5])
    assert e_half / e_smr > 2.5, (e_half, e_smr)


@pytest.mark.parametrize("bad", [[8], [1, 1], [-1]])
def test_invalid_refinement_rejected(bad):
    m = O.Mesh((32, 16), 1.4)
    with pytest.raises(O.OracleError):
        O.SMR(m, (4, 2), bad)
    with pytest.raises(O.OracleError):
        O.SMR(O.Mesh((24, 16), 1.4), (4, 2), [0])     # blocks of 6 cells: fine
        O.SMR(O.Mesh((12, 16), 1.4), (4, 2), [0])     # blocks of 3 cells: odd


def _sod_state(S, x0=0.3, axis=0):
    """Sod's two states (1, 0, 1) | (0.125, 0, 0.1) split at x0 along axis."""
    X = S.centres()
    W = np.zeros(S.shape)
    left = X[axis] < x0
    W[:, 0] = np.where(left, 1.0, 0.125)
    W[:, -1] = np.where(left, 1.0, 0.1)
    return W


def test_shock_through_refined_band_error_between_uniform_runs():
    """Sod's shock tube with the refined band [0.375, 0.625) in its path: by
    t = 0.2 the shock has entered and left the band (crossing both level
    jumps, where the prolongation limiter and the flux correction act on a
    discontinuity) and the contact sits inside it.  The density's L1 error
    against the exact solution lies between those of the coarse and the fine
    uniform meshes."""
    gamma, x0 = 1.4, 0.3
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)

    def err(n, B, ref):
        m = O.Mesh((n,), gamma, bc=((F, F),))
        S = O.SMR(m, (B,), ref)
        U, t, s, _ = S.run(S.prim_to_cons(_sod_state(S, x0)), 0.4, t_end=0.2)
        assert t == 0.2
        W = S.cons_to_prim(U)
        (X,) = S.centres()
        ex = O.exact_sample(gamma, left, right, ((X - x0) / t).ravel())[0].reshape(X.shape)
        dV = (1.0 / n) / 2.0 ** S.leaves[:, 0]
        return float((np.abs(W[:, 0] - ex).reshape(len(S.leaves), -1).sum(axis=1) * dV).sum())

    e_coarse, e_fine = err(64, 8, []), err(128, 16, [])
    e_band = err(64, 8, [3, 4])
    assert e_fine < e_band < e_coarse, (e_fine, e_band, e_coarse)
    # refining the whole wave region gets close to the fine mesh
    e_wide = err(64, 8, [2, 3, 4, 5])
    assert e_wide < 1.1 * e_fine, (e_wide, e_fine)
