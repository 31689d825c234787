"""C ABI checks that need no GPU: the library loads, exports every function
include/hydro.h declares, and rejects invalid configurations on the host."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "hydro.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def H():
    from paper_2501_02317_amd import build
    build.build(force=False)
    from paper_2501_02317_amd import hydro
    return hydro


def test_library_exports_every_declared_symbol(H):
    names = header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(H._lib, n), n
    assert set(names) == set(H.exported_symbols())


def test_workspace_bytes_validation(H):
    ok = H.make_config((64, 32, 16), 5.0 / 3.0, 0.3)
    nb = H.workspace_bytes(ok)
    assert nb >= 2 * 5 * 64 * 32 * 16 * 8
    bad = [
        H.make_config((64,), 1.0, 0.3),                       # gamma <= 1
        H.make_config((64,), 1.4, 0.0),                       # cfl <= 0
        H.make_config((64,), 1.4, 1.5),                       # cfl > 1
        H.make_config((64,), 1.4, 0.3, precision=7),          # unknown precision
        H.make_config((0,), 1.4, 0.3),                        # empty axis
        H.make_config((1,), 1.4, 0.3),                        # periodic needs two cells
        H.make_config((8,), 1.4, 0.3, bc=((0, 1),)),          # periodic on one side only
        H.make_config((8,), 1.4, 0.3, lo=(1.0,), hi=(0.0,)),  # inverted box
    ]
    for cfg in bad:
        assert H.workspace_bytes(cfg) == 0
    cfg = H.make_config((8,), 1.4, 0.3)
    cfg.ndim = 4
    assert H.workspace_bytes(cfg) == 0
    cfg = H.make_config((8,), 1.4, 0.3)
    cfg.n[1] = 2                                              # inactive axis must be 1
    assert H.workspace_bytes(cfg) == 0


def test_create_rejects_bad_arguments_without_device(H):
    cfg = H.make_config((64,), 1.4, 0.4)
    h = C.c_void_p()
    assert H._lib.hydro_create(C.byref(cfg), None, 1 << 20, None, C.byref(h)) == H.E_INVAL
    assert H._lib.hydro_create(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(h)) == H.E_INVAL
    assert H._lib.hydro_create(C.byref(cfg), C.c_void_p(100), 1 << 20, None, C.byref(h)) == H.E_INVAL
    assert H._lib.hydro_create(None, C.c_void_p(256), 1 << 20, None, C.byref(h)) == H.E_INVAL
    assert H._lib.hydro_step(None, 1.0) == H.E_INVAL
    assert H._lib.hydro_step_auto(None, 1, 0.0) == H.E_INVAL
    assert H._lib.hydro_destroy(None) == H.E_INVAL
    assert H._lib.hydro_riemann_fluxes(3, 1, 1.4, 10, None, None, None, None) == H.E_INVAL
    assert H._lib.hydro_riemann_fluxes(0, 1, 1.4, 0, None, None, None, None) == H.OK
    assert "non-physical" in H.strerror(H.E_NONPHYSICAL)
    # the allocation-free totals refuse an invalid call before any device work
    bad = H.make_config((64,), 1.0, 0.4)
    p = C.c_void_p(256)
    assert H._lib.hydro_conserved_totals_noalloc(C.byref(cfg), None, p, None) == H.E_INVAL
    assert H._lib.hydro_conserved_totals_noalloc(C.byref(cfg), p, None, None) == H.E_INVAL
    assert H._lib.hydro_conserved_totals_noalloc(None, p, p, None) == H.E_INVAL
    assert H._lib.hydro_conserved_totals_noalloc(C.byref(bad), p, p, None) == H.E_INVAL


def test_batch_rejects_invalid_members_without_device(H):
    arr = (C.c_void_p * 2)(None, None)
    assert H._lib.hydro_batch_workspace_bytes(2, arr) == 0
    assert H._lib.hydro_batch_workspace_bytes(0, arr) == 0
    b = C.c_void_p()
    assert H._lib.hydro_batch_create(2, arr, C.c_void_p(256), 1 << 20, 1, C.byref(b)) == H.E_INVAL
    assert H._lib.hydro_batch_step(None, 1) == H.E_INVAL
    assert H._lib.hydro_batch_destroy(None) == H.E_INVAL


def test_tile_candidates(H):
    """The autotuner's candidate tiles: every one supported, none repeated,
    kz values that differ in the chunks they give."""
    c3 = H.tile_candidates(3, (256, 256, 256))
    assert len(c3) == 20 and len(set(c3)) == 20
    assert {(tx, ty) for tx, ty, _ in c3} == {(32, 8), (64, 8), (16, 16), (32, 16)}
    assert {kz for *_, kz in c3} == {0, 8, 16, 32, 64}        # 0: automatic
    # a short marching axis: kz beyond it gives the same single chunk
    assert {kz for *_, kz in H.tile_candidates(3, (64, 64, 12))} == {0, 8, 16}
    # 2-D: rows much wider than the mesh are not tried
    assert H.tile_candidates(2, (64, 512)) == [(64, 1, 0), (64, 1, 8), (64, 1, 16), (64, 1, 32),
                                               (64, 1, 64)]
    assert {tx for tx, *_ in H.tile_candidates(2, (96, 96))} == {64, 128}
    assert H.tile_candidates(1, (256,)) == [(64, 1, 1), (128, 1, 1), (256, 1, 1)]
    bad = H.make_config((0, 4), 1.4, 0.4)
    assert H._lib.hydro_tile_candidates(C.byref(bad), None, 0) == H.E_INVAL


def test_block_split_validation(H):
    """A split mesh: equal blocks dividing the mesh, two cells per block on a
    split axis, one block on inactive axes, at most 1024 blocks; the
    workspace is that of the unsplit mesh."""
    base = H.workspace_bytes(H.make_config((64, 32, 16), 1.4, 0.3))
    for blocks in [(2, 2, 2), (4, 1, 8), (32, 16, 2), (1, 1, 1), (0, 0, 0)]:
        assert H.workspace_bytes(H.make_config((64, 32, 16), 1.4, 0.3, blocks=blocks)) == base
    bad = [
        ((64, 32, 16), (3, 1, 1)),     # does not divide
        ((64, 32, 16), (64, 1, 1)),    # one cell per block
        ((64, 32, 16), (32, 32, 2)),   # 2048 blocks
        ((64, 48), (2, 2, 2)),         # inactive axis split
        ((64,), (-1,)),                # negative
    ]
    for n, blocks in bad:
        cfg = H.make_config(n, 1.4, 0.3, blocks=blocks)
        if len(blocks) > len(n):
            for d in range(3):
                cfg.blocks[d] = blocks[d]
        assert H.workspace_bytes(cfg) == 0, (n, blocks)
    # a reflecting axis split into blocks of two cells is valid
    cfg = H.make_config((8, 4), 1.4, 0.3, bc=((3, 3), (2, 1)), blocks=(4, 2))
    assert H.workspace_bytes(cfg) > 0
    assert H._lib.hydro_set_block_streams(None, 1) == H.E_INVAL


def test_refinement_validation_and_leaves(H):
    """Refinement plans on the host: leaf order (level 0 by root, then level
    1 by the level-1 grid), the workspace, and the rejected cases."""
    import numpy as np
    cfg = H.make_config((32, 16), 1.4, 0.4, blocks=(4, 2))
    L = H.smr_leaves(cfg, [1, 6])
    assert [tuple(r) for r in L[:6]] == [(0, 0, 0, 0), (0, 2, 0, 0), (0, 3, 0, 0), (0, 0, 1, 0), (0, 1, 1, 0),
                                         (0, 3, 1, 0)]
    assert len(L) == 6 + 8 and np.all(L[6:, 0] == 1)
    assert [tuple(r[1:3]) for r in L[6:]] == [(2, 0), (3, 0), (2, 1), (3, 1), (4, 2), (5, 2), (4, 3), (5, 3)]
    assert H.workspace_bytes(cfg, [1, 6]) > H.workspace_bytes(cfg, [])
    assert H.workspace_bytes(cfg, []) > 0
    bad = [
        (cfg, [8]),                                                          # no such root
        (cfg, [1, 1]),                                                       # listed twice
        (H.make_config((24, 16), 1.4, 0.4, blocks=(8, 2)), [0]),             # blocks of 3 cells
        (H.make_config((8, 16), 1.4, 0.4, blocks=(4, 2)), [0]),              # blocks of 2 cells
    ]
    for c, ref in bad:
        assert H.workspace_bytes(c, ref) == 0, ref
        with pytest.raises(H.HydroError):
            H.smr_leaves(c, ref)
    # the van Leer integrator refines the same way, in the same workspace
    # (its predicted state stays conserved FP64 on a refined handle)
    vl = H.make_config((32, 16), 1.4, 0.4, blocks=(4, 2), integrator=1)
    for prec in (0, 1):
        vp = H.make_config((64, 32), 1.4, 0.4, precision=prec, blocks=(4, 2), integrator=1)
        hp = H.make_config((64, 32), 1.4, 0.4, precision=prec, blocks=(4, 2))
        assert H.workspace_bytes(vp, [1, 6]) == H.workspace_bytes(hp, [1, 6]) > 0
    assert np.array_equal(H.smr_leaves(vl, [1, 6]), L)


def test_deeper_refinement_plans_match_the_oracle(H):
    """Refinement deeper than one level, planned on the host: the library's
    leaves (with the balance refinement it adds) equal the oracle's for the
    same codes, and the codes the oracle refuses are refused."""
    import numpy as np
    import oracle as O
    LS = 26
    cases = [
        ((32,), (4,), [1, (1 << LS) | 3], ((1, 1),)),
        ((32, 16), (4, 2), [1, 6, (1 << LS) | 3, (1 << LS) | 20], ((0, 0), (0, 0))),
        ((32, 16), (4, 2), [1, 2, 5, 6, (1 << LS) | 3, (1 << LS) | 4], ((3, 3), (0, 0))),
        ((16, 16, 8), (2, 2, 1), [0, (1 << LS) | 0, (1 << LS) | 5], ((0, 0), (0, 0), (1, 1))),
        ((16, 16, 16), (2, 2, 2), [0, (1 << LS) | 0, (2 << LS) | 0], ((0, 0), (0, 0), (0, 0))),
    ]
    for n, B, codes, bc in cases:
        cfg = H.make_config(n, 1.4, 0.4, bc=bc, blocks=B)
        got = H.smr_leaves(cfg, codes)
        want = O.SMR(O.Mesh(n, 1.4, bc=bc), B, codes).leaves
        assert np.array_equal(got, want), (n, codes)
        assert H.workspace_bytes(cfg, codes) > 0
    cfg = H.make_config((32, 16), 1.4, 0.4, blocks=(4, 2))
    for bad in ([(1 << LS) | 0], [(3 << LS) | 0], [0, (1 << LS) | 64], [-1]):
        assert H.workspace_bytes(cfg, bad) == 0, bad
        with pytest.raises(O.OracleError):
            O.SMR(O.Mesh((32, 16), 1.4), (4, 2), bad)
