"""Pins of the oracle's multi-block mesh: c-boundaries between blocks of one
mesh, where each block writes its interior layers next to a shared face
straight into the neighbour's ghost zone, and the p-boundary rules
(Sec. 3.1.1) at the faces of the whole mesh.

A c-boundary copies exact values, so a uniform mesh split into blocks must
advance bit for bit like the unsplit mesh (the single-mesh oracle is pinned
on its own against closed forms, convergence and the exact Riemann
solution): a wrong neighbour, a missing or shifted ghost layer or a boundary
rule applied at an inner face changes the result.  CPU only.
"""
import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl

P, F, OUT, R = O.BC_PERIODIC, O.BC_FREE, O.BC_OUTFLOW, O.BC_REFLECT


def mesh_of(c, integrator, bc=None):
    return O.Mesh(c.n, c.gamma, c.lo, c.hi, bc if bc is not None else c.bc, integrator=integrator)


def assert_same_run(m, U0, cfl, blocks, steps):
    U, t, s, dts = O.run(m, U0, cfl, max_steps=steps)
    Ub, tb, sb, dtsb = O.run_blocks(m, blocks, U0, cfl, max_steps=steps)
    assert s == sb == steps and t == tb
    assert np.array_equal(dts, dtsb)
    assert np.array_equal(U, Ub), np.abs(U - Ub).max()
    return U


@pytest.mark.parametrize("integrator", [O.HEUN, O.VL2])
@pytest.mark.parametrize("blocks", [(2, 1, 1), (4, 1, 1), (12, 1, 1)])
def test_1d_split_matches_unsplit(integrator, blocks):
    c = wl.sod_1d(48)
    m = mesh_of(c, integrator)
    U0 = O.prim_to_cons(m, c.W)
    assert_same_run(m, U0, c.cfl, blocks, 12)


@pytest.mark.parametrize("integrator", [O.HEUN, O.VL2])
@pytest.mark.parametrize("blocks", [(2, 3, 1), (4, 1, 1), (1, 6, 1), (12, 12, 1)])
def test_2d_reflecting_box_split_matches_unsplit(integrator, blocks):
    c = wl.implosion_2d(N=24)
    m = mesh_of(c, integrator)
    U0 = O.prim_to_cons(m, c.W)
    assert_same_run(m, U0, c.cfl, blocks, 10)


@pytest.mark.parametrize("integrator", [O.HEUN, O.VL2])
@pytest.mark.parametrize("blocks", [(2, 2, 2), (3, 4, 5), (6, 1, 2), (1, 1, 5)])
def test_3d_periodic_split_matches_unsplit(integrator, blocks):
    c = wl.turbulence_3d(n=(12, 8, 10), mach=1.2, seed=31)
    m = mesh_of(c, integrator)
    U0 = O.prim_to_cons(m, c.W)
    assert_same_run(m, U0, c.cfl, blocks, 5)


@pytest.mark.parametrize("integrator", [O.HEUN, O.VL2])
def test_3d_mixed_boundaries_split_matches_unsplit(integrator):
    """Every p-boundary rule on some face of the whole mesh; periodic z."""
    c = wl.turbulence_3d(n=(12, 10, 8), mach=0.8, seed=32)
    bc = ((R, OUT), (F, R), (P, P))
    m = mesh_of(c, integrator, bc)
    U0 = O.prim_to_cons(m, c.W)
    U = None
    for blocks in [(2, 5, 2), (3, 2, 4), (6, 1, 1)]:
        Ub = assert_same_run(m, U0, c.cfl, blocks, 5)
        U = Ub if U is None else U
        assert np.array_equal(U, Ub)
    # the boundary codes matter: the periodic mesh gives another result
    Up, *_ = O.run(mesh_of(c, integrator), U0, c.cfl, max_steps=5)
    assert not np.array_equal(Up, U)


def test_run_to_end_time_matches_unsplit():
    c = wl.implosion_2d(N=16)
    m = mesh_of(c, O.HEUN)
    U0 = O.prim_to_cons(m, c.W)
    U, t, s, _ = O.run(m, U0, c.cfl, t_end=0.05)
    Ub, tb, sb, _ = O.run_blocks(m, (4, 2), U0, c.cfl, t_end=0.05)
    assert t == tb == 0.05 and s == sb and np.array_equal(U, Ub)


@pytest.mark.parametrize("blocks", [(5, 1, 1), (2, 1, 2), (0, 1, 1), (24, 1, 1)])
def test_invalid_decompositions_rejected(blocks):
    """Blocks must divide the mesh, a split axis needs two cells per block,
    and inactive axes take one block."""
    c = wl.implosion_2d(N=24)
    m = mesh_of(c, O.HEUN)
    U0 = O.prim_to_cons(m, c.W)
    with pytest.raises(O.OracleError):
        O.run_blocks(m, blocks, U0, c.cfl, max_steps=1)
