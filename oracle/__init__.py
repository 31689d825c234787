"""ctypes binding of the FP64 oracle -- TEST INFRASTRUCTURE ONLY.

The oracle is the plain serial-order CPU reference of the Godunov step of
arXiv 2501.02317, Sec. 3 (see hydro_oracle.h).  Only the tests, the package
smoke check and the CPU-baseline leg of the benchmark import this module; the
GPU product path never does.

Fields are numpy float64 arrays of shape (ncomp, nz, ny, nx) (trailing unit
axes for 1-D/2-D), conserved U = (rho, m_1..m_ndim, E) or primitive
W = (rho, v_1..v_ndim, p).
"""
import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

BC_PERIODIC, BC_FREE, BC_OUTFLOW, BC_REFLECT = 0, 1, 2, 3


class _Mesh(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("gamma", C.c_double), ("bc", (C.c_int32 * 2) * 3),
                ("integrator", C.c_int32)]


HEUN, VL2 = 0, 1


@dataclass
class Mesh:
    """Uniform Cartesian mesh; n lists the active axes' cell counts (x first)."""
    n: tuple
    gamma: float
    lo: tuple = None
    hi: tuple = None
    bc: tuple = None  # per active axis: (low, high); default periodic
    integrator: int = 0  # HEUN or VL2 (Sec. 3.3), used by run()

    def __post_init__(self):
        self.n = tuple(int(v) for v in self.n)
        nd = len(self.n)
        if self.lo is None:
            self.lo = (0.0,) * nd
        if self.hi is None:
            self.hi = (1.0,) * nd
        if self.bc is None:
            self.bc = ((BC_PERIODIC, BC_PERIODIC),) * nd

    @property
    def ndim(self):
        return len(self.n)

    @property
    def ncomp(self):
        return self.ndim + 2

    @property
    def shape(self):
        """(ncomp, nz, ny, nx) of a field array."""
        n = list(self.n) + [1] * (3 - self.ndim)
        return (self.ncomp, n[2], n[1], n[0])

    @property
    def dx(self):
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] for d in range(self.ndim))

    def to_c(self):
        m = _Mesh()
        m.ndim = self.ndim
        for d in range(3):
            active = d < self.ndim
            m.n[d] = self.n[d] if active else 1
            m.lo[d] = self.lo[d] if active else 0.0
            m.hi[d] = self.hi[d] if active else 1.0
            for s in range(2):
                m.bc[d][s] = self.bc[d][s] if active else BC_PERIODIC
        m.gamma = self.gamma
        m.integrator = self.integrator
        return m


_lib = None
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of the same sources (the tests run
        # a sanitizer-instrumented build in a subprocess through it)
        path = os.environ.get("ORACLE_LIB") or _build.build(force=False)
        L = C.CDLL(path)
        mp = C.POINTER(_Mesh)
        sig = {
            "orc_ncomp": (C.c_int, [mp]),
            "orc_minmod": (C.c_double, [C.c_double, C.c_double]),
            "orc_prim_to_cons": (None, [mp, _dp, _dp]),
            "orc_cons_to_prim": (C.c_int, [mp, _dp, _dp]),
            "orc_hllc": (None, [C.c_double, C.c_int, _dp, _dp, _dp, _dp]),
            "orc_plm_face": (None, [_dp, _dp, _dp]),
            "orc_cfl_dt": (C.c_double, [mp, _dp, C.c_double]),
            "orc_fill_ghosts": (C.c_int, [mp, _dp]),
            "orc_rhs": (C.c_int, [mp, _dp, C.c_double, _dp]),
            "orc_heun_step": (C.c_int, [mp, _dp, C.c_double]),
            "orc_rhs_prim": (C.c_int, [mp, _dp, C.c_double, C.c_int, _dp]),
            "orc_vl2_step": (C.c_int, [mp, _dp, C.c_double]),
            "orc_run": (C.c_int, [mp, _dp, C.c_double, C.c_int, C.c_double, _dp,
                                  C.POINTER(C.c_int), _dp]),
            "orc_run_blocks": (C.c_int, [mp, C.POINTER(C.c_int32), _dp, C.c_double, C.c_int, C.c_double,
                                         _dp, C.POINTER(C.c_int), _dp]),
            "orc_smr_leaves": (C.c_int, [mp, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.c_int]),
            "orc_smr_ghosts": (C.c_int, [mp, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), _dp, _dp]),
            "orc_run_smr": (C.c_int, [mp, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), _dp, C.c_double,
                                      C.c_int, C.c_double, _dp, C.POINTER(C.c_int), _dp]),
            "orc_smr_totals": (None, [mp, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), _dp, _dp]),
            "orc_totals": (None, [mp, _dp, _dp]),
            "orc_rhs_cells": (C.c_int, [mp, _dp, C.c_double, C.c_int, _i64p, _dp]),
            "orc_step_cells": (C.c_int, [mp, _dp, C.c_double, C.c_int, _i64p, _dp]),
            "orc_exact_star": (C.c_int, [C.c_double] * 7 + [C.c_int, _dp, _dp]),
            "orc_exact_sample": (C.c_int, [C.c_double] * 8 + [_dp, _dp, _dp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_dp)


def _field(mesh, a):
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(mesh.shape)
    return a


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc < 0:
        raise OracleError(f"{what}: invalid arguments")
    if rc > 0:
        raise OracleError(f"{what}: {rc} non-physical cell(s)")


def minmod(a, b):
    return lib().orc_minmod(float(a), float(b))


def prim_to_cons(mesh, W):
    W = _field(mesh, W)
    U = np.empty_like(W)
    lib().orc_prim_to_cons(C.byref(mesh.to_c()), _p(W), _p(U))
    return U


def cons_to_prim(mesh, U):
    U = _field(mesh, U)
    W = np.empty_like(U)
    _check(lib().orc_cons_to_prim(C.byref(mesh.to_c()), _p(U), _p(W)), "cons_to_prim")
    return W


def hllc(gamma, WL, WR, detail=False):
    """HLLC flux in the face-normal frame; WL/WR = (rho, u, t..., p)."""
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    nc = WL.size
    F = np.empty(nc)
    det = np.empty(4 + 8 * nc) if detail else None
    lib().orc_hllc(float(gamma), nc - 3, _p(WL), _p(WR), _p(F),
                   _p(det) if detail else C.cast(None, _dp))
    if not detail:
        return F
    names = ["UL", "UR", "FL", "FR", "UsL", "UsR", "FsL", "FsR"]
    d = {"sL": det[0], "s_star": det[1], "sR": det[2], "p_star": det[3]}
    for i, nm in enumerate(names):
        d[nm] = det[4 + i * nc: 4 + (i + 1) * nc].copy()
    return F, d


def plm_face(w4):
    w4 = np.ascontiguousarray(w4, dtype=np.float64)
    wl, wr = C.c_double(), C.c_double()
    lib().orc_plm_face(_p(w4), C.byref(wl), C.byref(wr))
    return wl.value, wr.value


def cfl_dt(mesh, U, cfl):
    U = _field(mesh, U)
    dt = lib().orc_cfl_dt(C.byref(mesh.to_c()), _p(U), float(cfl))
    if not dt > 0:
        raise OracleError("cfl_dt: non-physical state")
    return dt


def padded_primitive(mesh, U):
    """Primitive state with n_gh = 2 ghost layers filled (corners left zero)."""
    W = cons_to_prim(mesh, U)
    nd = mesh.ndim
    pad = [(0, 0)] + [(2, 2) if (2 - a) < nd else (0, 0) for a in range(3)]
    Wp = np.pad(W, pad)
    lib().orc_fill_ghosts(C.byref(mesh.to_c()), _p(Wp))
    return Wp


def rhs(mesh, U, dt):
    U = _field(mesh, U)
    dU = np.empty_like(U)
    _check(lib().orc_rhs(C.byref(mesh.to_c()), _p(U), float(dt), _p(dU)), "rhs")
    return dU


def heun_step(mesh, U, dt):
    U = _field(mesh, U).copy()
    _check(lib().orc_heun_step(C.byref(mesh.to_c()), _p(U), float(dt)), "heun_step")
    return U


def rhs_prim(mesh, W, dt, order):
    """Stage right-hand side from a primitive state, order 1 (piecewise
    constant) or 2 (PLM)."""
    W = _field(mesh, W)
    dU = np.empty_like(W)
    _check(lib().orc_rhs_prim(C.byref(mesh.to_c()), _p(W), float(dt), int(order), _p(dU)), "rhs_prim")
    return dU


def vl2_step(mesh, U, dt):
    U = _field(mesh, U).copy()
    _check(lib().orc_vl2_step(C.byref(mesh.to_c()), _p(U), float(dt)), "vl2_step")
    return U


def run(mesh, U, cfl, max_steps=0, t_end=0.0, t0=0.0):
    """Run CFL-limited steps of the mesh's integrator; returns (U, t, steps, dts)."""
    U = _field(mesh, U).copy()
    t = C.c_double(t0)
    steps = C.c_int(0)
    cap = max_steps if max_steps > 0 else 1_000_000
    dts = np.zeros(cap)
    rc = lib().orc_run(C.byref(mesh.to_c()), _p(U), float(cfl), int(max_steps), float(t_end),
                       C.byref(t), C.byref(steps), _p(dts) if max_steps > 0 else C.cast(None, _dp))
    _check(rc, "run")
    return U, t.value, steps.value, dts[: steps.value] if max_steps > 0 else None


def run_blocks(mesh, blocks, U, cfl, max_steps=0, t_end=0.0, t0=0.0):
    """run() on the mesh split into blocks[0] x blocks[1] x blocks[2] equal
    blocks with c-boundary ghost exchange; U in the mesh layout."""
    U = _field(mesh, U).copy()
    B = (C.c_int32 * 3)(*(list(blocks) + [1] * (3 - len(blocks))))
    t = C.c_double(t0)
    steps = C.c_int(0)
    cap = max_steps if max_steps > 0 else 1_000_000
    dts = np.zeros(cap)
    rc = lib().orc_run_blocks(C.byref(mesh.to_c()), B, _p(U), float(cfl), int(max_steps), float(t_end),
                              C.byref(t), C.byref(steps), _p(dts) if max_steps > 0 else C.cast(None, _dp))
    _check(rc, "run_blocks")
    return U, t.value, steps.value, dts[: steps.value] if max_steps > 0 else None


def _blocks3(blocks):
    return (C.c_int32 * 3)(*(list(blocks) + [1] * (3 - len(blocks))))


def _refined(refined):
    r = np.ascontiguousarray(list(refined) if len(refined) else [0], dtype=np.int32)
    return len(refined), r.ctypes.data_as(C.POINTER(C.c_int32)), r


class SMR:
    """Static refinement of a block mesh: the blocks listed in refined (codes
    level * 2^26 + index on that level's block grid; a plain root index for
    level 0) are split into 2^ndim blocks of half the size, and refinement
    is added until face-neighbouring leaves differ by at most one level.
    Fields are block-layout arrays of shape (nleaf, ncomp, bz, by, bx)."""

    def __init__(self, mesh, blocks, refined):
        self.mesh = mesh
        self.blocks = tuple(blocks) + (1,) * (3 - len(blocks))
        self.refined = [int(r) for r in refined]
        B = _blocks3(self.blocks)
        nr, rp, keep = _refined(self.refined)
        cap = 1 << 16
        out = np.zeros((cap, 4), dtype=np.int32)
        n = lib().orc_smr_leaves(C.byref(mesh.to_c()), B, nr, rp, out.ctypes.data_as(C.POINTER(C.c_int32)), cap)
        if n < 0:
            raise OracleError("smr: invalid refinement")
        self.leaves = out[:n].copy()
        nn = list(mesh.n) + [1] * (3 - mesh.ndim)
        self.bn = tuple(nn[d] // self.blocks[d] for d in range(3))
        self.shape = (n, mesh.ncomp, self.bn[2], self.bn[1], self.bn[0])

    def _args(self):
        nr, rp, keep = _refined(self.refined)
        self._keep = keep
        return C.byref(self.mesh.to_c()), _blocks3(self.blocks), nr, rp

    def centres(self):
        """Cell-centre coordinates per leaf: a list of ndim arrays of shape
        (nleaf, bz, by, bx)."""
        m = self.mesh
        out = []
        for d in range(m.ndim):
            dx0 = (m.hi[d] - m.lo[d]) / m.n[d]
            lev = self.leaves[:, 0].astype(np.float64)
            dxl = dx0 / 2.0 ** lev
            org = m.lo[d] + self.leaves[:, 1 + d] * self.bn[d] * dxl
            idx = np.arange(self.bn[d], dtype=np.float64)
            shp = [1, 1, 1]
            shp[2 - d] = self.bn[d]
            x = org[:, None, None, None] + (idx.reshape(shp)[None] + 0.5) * dxl[:, None, None, None]
            out.append(np.broadcast_to(x, (len(self.leaves), self.bn[2], self.bn[1], self.bn[0])).copy())
        return out

    def ghosts(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(self.shape)
        pad = [s + (4 if (2 - a) < self.mesh.ndim else 0) for a, s in enumerate(self.shape[2:])]
        out = np.zeros((self.shape[0], self.shape[1], *pad))
        rc = lib().orc_smr_ghosts(*self._args(), _p(W), _p(out))
        _check(rc, "smr_ghosts")
        return out

    def run(self, U, cfl, max_steps=0, t_end=0.0, t0=0.0):
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape).copy()
        t = C.c_double(t0)
        steps = C.c_int(0)
        cap = max_steps if max_steps > 0 else 1_000_000
        dts = np.zeros(cap)
        rc = lib().orc_run_smr(*self._args(), _p(U), float(cfl), int(max_steps), float(t_end), C.byref(t),
                               C.byref(steps), _p(dts) if max_steps > 0 else C.cast(None, _dp))
        _check(rc, "run_smr")
        return U, t.value, steps.value, dts[: steps.value] if max_steps > 0 else None

    def totals(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape)
        T = np.empty(self.mesh.ncomp)
        lib().orc_smr_totals(*self._args(), _p(U), _p(T))
        return T

    def _pointwise(self, F, fn):
        # the conversions are cell by cell: apply them to all cells as one row
        F = np.ascontiguousarray(F, dtype=np.float64).reshape(self.shape)
        nc, n = self.mesh.ncomp, self.shape[0]
        cells = n * int(np.prod(self.bn))
        nd = self.mesh.ndim
        row = Mesh((cells,) + (1,) * (nd - 1), self.mesh.gamma, bc=((BC_FREE, BC_FREE),) * nd)
        G = fn(row, np.moveaxis(F, 1, 0).reshape(row.shape))
        return np.moveaxis(G.reshape(nc, n, *self.shape[2:]), 0, 1).copy()

    def prim_to_cons(self, W):
        return self._pointwise(W, prim_to_cons)

    def cons_to_prim(self, U):
        return self._pointwise(U, cons_to_prim)


def totals(mesh, U):
    U = _field(mesh, U)
    T = np.empty(mesh.ncomp)
    lib().orc_totals(C.byref(mesh.to_c()), _p(U), _p(T))
    return T


def _cells(cells):
    return np.ascontiguousarray(cells, dtype=np.int64)


def rhs_cells(mesh, U, dt, cells):
    U = _field(mesh, U)
    cells = _cells(cells)
    out = np.empty((mesh.ncomp, cells.size))
    _check(lib().orc_rhs_cells(C.byref(mesh.to_c()), _p(U), float(dt), cells.size,
                               cells.ctypes.data_as(_i64p), _p(out)), "rhs_cells")
    return out


def step_cells(mesh, U, dt, cells):
    U = _field(mesh, U)
    cells = _cells(cells)
    out = np.empty((mesh.ncomp, cells.size))
    _check(lib().orc_step_cells(C.byref(mesh.to_c()), _p(U), float(dt), cells.size,
                                cells.ctypes.data_as(_i64p), _p(out)), "step_cells")
    return out


def exact_star(gamma, left, right, method=0):
    """(p*, u*) of the exact Riemann problem; left/right = (rho, u, p)."""
    ps, us = C.c_double(), C.c_double()
    rc = lib().orc_exact_star(float(gamma), *map(float, left), *map(float, right), int(method),
                              C.byref(ps), C.byref(us))
    if rc:
        raise OracleError("exact_star: vacuum or non-positive data")
    return ps.value, us.value


def exact_sample(gamma, left, right, xi):
    """Exact (rho, u, p) at similarity coordinates xi (array)."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    out = np.empty((3, xi.size))
    r, u, p = C.c_double(), C.c_double(), C.c_double()
    L = lib()
    for i, x in enumerate(xi):
        rc = L.orc_exact_sample(float(gamma), *map(float, left), *map(float, right), float(x),
                                C.byref(r), C.byref(u), C.byref(p))
        if rc:
            raise OracleError("exact_sample: vacuum or non-positive data")
        out[:, i] = (r.value, u.value, p.value)
    return out


def l1_paper(q, q0):
    """Normalised L1 error of eq. l1_err (Sec. 4.1)."""
    q = np.asarray(q, dtype=np.float64).ravel()
    q0 = np.asarray(q0, dtype=np.float64).ravel()
    return float(np.abs(q - q0).sum() / (q0.size * (q0.max() - q0.min())))


def rel_l1(a, ref):
    """Relative L1 difference sum|a - ref| / sum|ref| of one component."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.abs(a - ref).sum() / np.abs(ref).sum())
