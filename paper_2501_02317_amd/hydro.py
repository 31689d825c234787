"""ctypes binding of libhydro.so (C ABI in include/hydro.h).

Argument marshalling only: every step of the solver runs in the HIP
kernels.  PyTorch provides the device workspace and the HIP stream.
Importing this module loads the library and raises ImportError when it has
not been built (``python -m paper_2501_02317_amd.build``); there is no
fallback implementation.
"""
import ctypes as C
import os

import numpy as np
# PyTorch first: its HIP runtime is then the one the library binds to, so
# device memory from torch and the library's own HIP calls share a runtime.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhydro.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2501_02317_amd.build`")
_lib = C.CDLL(LIB_PATH)

FP64, MIXED = 0, 1
BC_PERIODIC, BC_FREE, BC_OUTFLOW, BC_REFLECT = 0, 1, 2, 3
OK, E_INVAL, E_NOMEM, E_DEVICE, E_NONPHYSICAL, E_STATE = 0, -1, -2, -3, -4, -5


HEUN, VL2 = 0, 1


class Config(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3),
                ("hi", C.c_double * 3), ("gamma", C.c_double), ("cfl", C.c_double),
                ("precision", C.c_int32), ("bc", (C.c_int32 * 2) * 3), ("integrator", C.c_int32),
                ("blocks", C.c_int32 * 3)]


_dp = C.POINTER(C.c_double)
_vp = C.c_void_p
_h = C.c_void_p
_SIG = {
    "hydro_workspace_bytes": (C.c_size_t, [C.POINTER(Config)]),
    "hydro_create": (C.c_int, [C.POINTER(Config), _vp, C.c_size_t, _vp, C.POINTER(_h)]),
    "hydro_set_state": (C.c_int, [_h, _dp]),
    "hydro_set_primitive": (C.c_int, [_h, _dp]),
    "hydro_get_state": (C.c_int, [_h, _dp]),
    "hydro_set_primitive_device": (C.c_int, [_h, _vp]),
    "hydro_get_state_device": (C.c_int, [_h, _vp]),
    "hydro_state_device": (C.c_int, [_h, C.POINTER(_vp)]),
    "hydro_set_block_streams": (C.c_int, [_h, C.c_int]),
    "hydro_smr_workspace_bytes": (C.c_size_t, [C.POINTER(Config), C.c_int, C.POINTER(C.c_int32)]),
    "hydro_smr_create": (C.c_int, [C.POINTER(Config), C.c_int, C.POINTER(C.c_int32), _vp, C.c_size_t, _vp,
                                   C.POINTER(_h)]),
    "hydro_smr_leaves": (C.c_int, [C.POINTER(Config), C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                   C.c_int]),
    "hydro_cfl_dt": (C.c_int, [_h, _dp]),
    "hydro_step": (C.c_int, [_h, C.c_double]),
    "hydro_step_auto": (C.c_int, [_h, C.c_int, C.c_double]),
    "hydro_conserved_totals": (C.c_int, [_h, _dp]),
    "hydro_conserved_totals_noalloc": (C.c_int, [C.POINTER(Config), _vp, _vp, _vp]),
    "hydro_time": (C.c_int, [_h, _dp]),
    "hydro_steps_done": (C.c_int, [_h, C.POINTER(C.c_int64)]),
    "hydro_stage_rhs": (C.c_int, [_h, C.c_double, _dp]),
    "hydro_padded_primitive": (C.c_int, [_h, _dp]),
    "hydro_set_tile": (C.c_int, [_h, C.c_int, C.c_int, C.c_int]),
    "hydro_set_stage_tile": (C.c_int, [_h, C.c_int, C.c_int, C.c_int, C.c_int]),
    "hydro_get_stage_tile": (C.c_int, [_h, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                       C.POINTER(C.c_int)]),
    "hydro_tile_candidates": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_int), C.c_int]),
    "hydro_autotune": (C.c_int, [_h, C.c_int, C.c_double, C.POINTER(C.c_int), _dp]),
    "hydro_batch_autotune": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int), _dp]),
    "hydro_profile": (C.c_int, [_h, C.c_int]),
    "hydro_profile_read": (C.c_int, [_h, _dp, _dp, C.POINTER(C.c_int64)]),
    "hydro_set_run_limit": (C.c_int, [_h, C.c_int64, C.c_double]),
    "hydro_run_done": (C.c_int, [_h, C.POINTER(C.c_int)]),
    "hydro_destroy": (C.c_int, [_h]),
    "hydro_batch_workspace_bytes": (C.c_size_t, [C.c_int, C.POINTER(_h)]),
    "hydro_batch_create": (C.c_int, [C.c_int, C.POINTER(_h), _vp, C.c_size_t, C.c_int, C.POINTER(_h)]),
    "hydro_batch_step": (C.c_int, [_h, C.c_int]),
    "hydro_batch_info": (C.c_int, [_h, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
    "hydro_batch_status": (C.c_int, [_h, C.POINTER(C.c_int), C.POINTER(C.c_int64), C.POINTER(C.c_int)]),
    "hydro_batch_destroy": (C.c_int, [_h]),
    "hydro_strerror": (C.c_char_p, [C.c_int]),
    "hydro_riemann_fluxes": (C.c_int, [C.c_int, C.c_int, C.c_double, C.c_int64, _vp, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args


class HydroError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        msg = _lib.hydro_strerror(status).decode()
        super().__init__(f"{what}: {msg} ({status})" if what else f"{msg} ({status})")


def _check(status, what):
    if status != OK:
        raise HydroError(status, what)


def strerror(status):
    return _lib.hydro_strerror(int(status)).decode()


def make_config(n, gamma, cfl, precision=FP64, lo=None, hi=None, bc=None, integrator=HEUN, blocks=None):
    """Config for the active axes' cell counts n (x first); blocks: blocks
    per active axis of a split mesh (None: one block)."""
    nd = len(n)
    cfg = Config()
    cfg.ndim = nd
    lo = lo or (0.0,) * nd
    hi = hi or (1.0,) * nd
    bc = bc or ((BC_PERIODIC, BC_PERIODIC),) * nd
    for d in range(3):
        act = d < nd
        cfg.n[d] = int(n[d]) if act else 1
        cfg.lo[d] = float(lo[d]) if act else 0.0
        cfg.hi[d] = float(hi[d]) if act else 1.0
        for s in range(2):
            cfg.bc[d][s] = int(bc[d][s]) if act else BC_PERIODIC
    cfg.gamma = float(gamma)
    cfg.cfl = float(cfl)
    cfg.precision = int(precision)
    cfg.integrator = int(integrator)
    blocks = tuple(blocks) if blocks else (1,) * nd
    for d in range(3):
        cfg.blocks[d] = int(blocks[d]) if d < len(blocks) else 1
    return cfg


def workspace_bytes(cfg, refined=None):
    if refined is not None:
        r = _refined_arr(refined)
        return int(_lib.hydro_smr_workspace_bytes(C.byref(cfg), len(refined), r))
    return int(_lib.hydro_workspace_bytes(C.byref(cfg)))


def _refined_arr(refined):
    return (C.c_int32 * max(1, len(refined)))(*[int(r) for r in refined])


def smr_leaves(cfg, refined):
    """(level, c0, c1, c2) per leaf of a refinement of cfg's blocks (refined:
    codes level * 2^26 + index on that level's block grid; root indices for
    level 0)."""
    r = _refined_arr(refined)
    cap = 1 << 12
    out = (C.c_int32 * (4 * cap))()
    n = _lib.hydro_smr_leaves(C.byref(cfg), len(refined), r, out, cap)
    if n < 0:
        raise HydroError(n, "invalid refinement")
    return np.array(out[: 4 * n], dtype=np.int32).reshape(n, 4)


def _ptr(a):
    return a.ctypes.data_as(_dp)


class Hydro:
    """One mesh resident on the GPU.

    Fields are float64 numpy arrays of shape (ncomp, nz, ny, nx).
    """

    def __init__(self, n, gamma, cfl, precision=FP64, lo=None, hi=None, bc=None, device=None,
                 stream=None, workspace=None, integrator=HEUN, blocks=None, refined=None):
        import torch

        self.cfg = make_config(n, gamma, cfl, precision, lo, hi, bc, integrator, blocks)
        self.integrator = int(integrator)
        self.blocks = tuple(max(1, self.cfg.blocks[d]) for d in range(len(n)))
        self.refined = None if refined is None else [int(r) for r in refined]
        self.ndim = len(n)
        self.n = tuple(int(v) for v in n)
        self.precision = int(precision)
        self.ncomp = self.ndim + 2
        nn = list(n) + [1] * (3 - len(n))
        self.shape = (self.ncomp, nn[2], nn[1], nn[0])
        if self.refined is not None:
            # a refined mesh: fields in the block layout of its leaves
            self.leaves = smr_leaves(self.cfg, self.refined)
            b = list(self.blocks) + [1] * (3 - len(self.blocks))
            self.shape = (len(self.leaves), self.ncomp, nn[2] // b[2], nn[1] // b[1], nn[0] // b[0])
        nbytes = workspace_bytes(self.cfg, self.refined)
        if nbytes == 0:
            raise HydroError(E_INVAL, "invalid configuration")
        if workspace is not None:
            # caller-provided device memory (uint8 CUDA tensor, >= nbytes, 256-byte aligned)
            if workspace.numel() < nbytes or workspace.data_ptr() % 256:
                raise HydroError(E_INVAL, "workspace too small or misaligned")
            self.device = workspace.device
            self.workspace = workspace
        else:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8,
                                         device=torch.device(device if device is not None else "cuda"))
            self.device = self.workspace.device  # with its index
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = _h()
        if self.refined is not None:
            _check(_lib.hydro_smr_create(C.byref(self.cfg), len(self.refined), _refined_arr(self.refined),
                                         _vp(self.workspace.data_ptr()), nbytes, _vp(stream.cuda_stream),
                                         C.byref(h)), "hydro_smr_create")
        else:
            _check(_lib.hydro_create(C.byref(self.cfg), _vp(self.workspace.data_ptr()), nbytes,
                                     _vp(stream.cuda_stream), C.byref(h)), "hydro_create")
        self._h = h

    # ---- state
    def set_state(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64).reshape(self.shape)
        _check(_lib.hydro_set_state(self._h, _ptr(U)), "hydro_set_state")

    def set_primitive(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64).reshape(self.shape)
        _check(_lib.hydro_set_primitive(self._h, _ptr(W)), "hydro_set_primitive")

    def _device_field(self, t, what):
        """Refuse a tensor the C call would overrun: the library reads or
        writes ncomp * ncells doubles at the pointer on this mesh's device."""
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.device == self.device and tuple(t.shape) == tuple(self.shape)):
            raise HydroError(E_INVAL, f"{what}: needs a contiguous float64 tensor of shape {tuple(self.shape)} "
                                      f"on {self.device}")
        return _vp(t.data_ptr())

    def set_primitive_device(self, W):
        """W: float64 CUDA tensor of shape (ncomp, nz, ny, nx), contiguous, on
        this mesh's device.  The tensor must stay alive until the stream
        passes this call."""
        p = self._device_field(W, "set_primitive_device")
        _check(_lib.hydro_set_primitive_device(self._h, p), "hydro_set_primitive_device")

    def get_state_device(self, out):
        """Copy the state into a float64 CUDA tensor of the state's shape on
        this mesh's device (async on the mesh's stream)."""
        p = self._device_field(out, "get_state_device")
        _check(_lib.hydro_get_state_device(self._h, p), "hydro_get_state_device")

    def get_state(self, out=None):
        """Conserved state copied to host memory, into out if given (a
        C-contiguous float64 array of the state's shape, e.g. one kept across
        calls so its pages are not touched for the first time on every copy)."""
        if out is None:
            out = np.empty(self.shape)
        elif not (isinstance(out, np.ndarray) and out.dtype == np.float64 and out.flags.c_contiguous
                  and out.flags.writeable and tuple(out.shape) == tuple(self.shape)):
            raise ValueError(f"out must be a writeable C-contiguous float64 array of shape {tuple(self.shape)}")
        _check(_lib.hydro_get_state(self._h, _ptr(out)), "hydro_get_state")
        return out

    def state_view(self):
        """Zero-copy torch view of the device state (valid until the next
        step): shape (ncomp, nz, ny, nx), or for a split mesh the block
        layout (nblocks, ncomp, bz, by, bx)."""
        import torch
        p = _vp()
        _check(_lib.hydro_state_device(self._h, C.byref(p)), "hydro_state_device")
        off = p.value - self.workspace.data_ptr()
        n = int(np.prod(self.shape))
        v = self.workspace[off: off + 8 * n].view(torch.float64)
        nb = int(np.prod(self.blocks))
        if nb == 1 or self.refined is not None:
            return v.view(self.shape)
        b = list(self.blocks) + [1] * (3 - len(self.blocks))
        return v.view(nb, self.ncomp, self.shape[1] // b[2], self.shape[2] // b[1], self.shape[3] // b[0])

    def set_block_streams(self, on):
        """Launch each block's stages on their own streams (True) or one
        launch per stage over every block (False, the default)."""
        _check(_lib.hydro_set_block_streams(self._h, 1 if on else 0), "hydro_set_block_streams")

    # ---- stepping
    def cfl_dt(self):
        dt = C.c_double()
        _check(_lib.hydro_cfl_dt(self._h, C.byref(dt)), "hydro_cfl_dt")
        return dt.value

    def step(self, dt):
        _check(_lib.hydro_step(self._h, float(dt)), "hydro_step")

    def step_auto(self, nsteps, t_end=0.0):
        _check(_lib.hydro_step_auto(self._h, int(nsteps), float(t_end)), "hydro_step_auto")

    def set_run_limit(self, max_steps=0, t_end=0.0):
        """Device-dt steps stop advancing this mesh after max_steps more steps
        or at t_end (0: no limit)."""
        _check(_lib.hydro_set_run_limit(self._h, int(max_steps), float(t_end)), "hydro_set_run_limit")

    def run_done(self):
        d = C.c_int()
        _check(_lib.hydro_run_done(self._h, C.byref(d)), "hydro_run_done")
        return bool(d.value)

    def time(self):
        t = C.c_double()
        _check(_lib.hydro_time(self._h, C.byref(t)), "hydro_time")
        return t.value

    def steps_done(self):
        s = C.c_int64()
        _check(_lib.hydro_steps_done(self._h, C.byref(s)), "hydro_steps_done")
        return s.value

    def totals(self):
        T = np.empty(self.ncomp)
        _check(_lib.hydro_conserved_totals(self._h, _ptr(T)), "hydro_conserved_totals")
        return T

    # ---- single-row views for testing
    def stage_rhs(self, dt):
        dU = np.empty(self.shape)
        _check(_lib.hydro_stage_rhs(self._h, float(dt), _ptr(dU)), "hydro_stage_rhs")
        return dU

    def padded_primitive(self):
        shp = [self.ncomp] + [s + (4 if (2 - a) < self.ndim else 0)
                              for a, s in enumerate(self.shape[1:])]
        Wp = np.empty(shp)
        _check(_lib.hydro_padded_primitive(self._h, _ptr(Wp)), "hydro_padded_primitive")
        return Wp

    # ---- tiling
    def set_tile(self, tx, ty, kz, stage=0):
        """Tile of stage 1 or 2, or of both (stage 0)."""
        _check(_lib.hydro_set_stage_tile(self._h, int(stage), int(tx), int(ty), int(kz)),
               "hydro_set_stage_tile")

    def get_tile(self, stage=None):
        """(tx, ty, kz) of stage 1 or 2, or a pair of them (stage None)."""
        if stage is None:
            return self.get_tile(1), self.get_tile(2)
        tx, ty, kz = C.c_int(), C.c_int(), C.c_int()
        _check(_lib.hydro_get_stage_tile(self._h, int(stage), C.byref(tx), C.byref(ty), C.byref(kz)),
               "hydro_get_stage_tile")
        return tx.value, ty.value, kz.value

    def autotune(self, steps_per_tile=1, t_end=0.0, cache=None):
        """Pick each stage's fastest tile.  With a cache file (JSON) tiles
        stored for the same device, dimensionality, size and precision are
        set directly; otherwise hydro_autotune times every candidate over
        real steps of this run (after one untimed step) and the winners are
        stored.  Returns
        ((stage-1 tile, stage-2 tile), steps advanced)."""
        key = None
        if cache:
            key = _tile_key(self.ndim, self.n, self.precision)
            entry = _cache_read(cache).get(key)
            if entry:
                t1, t2 = (tuple(t) for t in entry["tiles"])
                self.set_tile(*t1, stage=1)
                self.set_tile(*t2, stage=2)
                return (t1, t2), 0
        s0 = self.steps_done()
        tiles, ms = (C.c_int * 6)(), (C.c_double * 2)()
        _check(_lib.hydro_autotune(self._h, int(steps_per_tile), float(t_end), tiles, ms), "hydro_autotune")
        t1, t2 = tuple(tiles[0:3]), tuple(tiles[3:6])
        if cache:
            _cache_store(cache, key, {"tiles": [list(t1), list(t2)], "ms_per_step": list(ms)})
        return (t1, t2), self.steps_done() - s0

    # ---- measurement
    def profile(self, cap):
        """Bracket the next cap launches of each stage kernel with HIP events."""
        _check(_lib.hydro_profile(self._h, int(cap)), "hydro_profile")

    def profile_read(self):
        """(ms of stage-1 launches, ms of stage-2 launches, (n1, n2))."""
        a, b = C.c_double(), C.c_double()
        n = (C.c_int64 * 2)()
        _check(_lib.hydro_profile_read(self._h, C.byref(a), C.byref(b), n), "hydro_profile_read")
        return a.value, b.value, (n[0], n[1])

    def close(self):
        if getattr(self, "_h", None):
            _lib.hydro_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent meshes stepped together (one launch per group and stage,
    optionally replayed from a HIP graph).  All members share one stream."""

    def __init__(self, members, use_graph=True):
        import torch
        self.members = list(members)
        n = len(self.members)
        arr = (_h * n)(*[m._h for m in self.members])
        self._arr = arr
        nbytes = int(_lib.hydro_batch_workspace_bytes(n, arr))
        if nbytes == 0:
            raise HydroError(E_INVAL, "batch members (NULL, repeated, broken or on different streams)")
        dev = self.members[0].device
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        b = _h()
        _check(_lib.hydro_batch_create(n, arr, _vp(self.workspace.data_ptr()), nbytes, 1 if use_graph else 0,
                                       C.byref(b)), "hydro_batch_create")
        self._b = b

    def step(self, nsteps):
        _check(_lib.hydro_batch_step(self._b, int(nsteps)), "hydro_batch_step")

    def status(self):
        """(done flags, completed steps, error flags) per member; blocks."""
        n = len(self.members)
        d = (C.c_int * n)()
        st = (C.c_int64 * n)()
        fl = (C.c_int * n)()
        _check(_lib.hydro_batch_status(self._b, d, st, fl), "hydro_batch_status")
        return list(d), list(st), list(fl)

    def autotune(self, steps_per_rule=2):
        """Pick the fastest tile rule for the batch's 1-D/2-D members over real
        batched steps; returns (rule index, ms per batched step)."""
        r, ms = C.c_int(), C.c_double()
        _check(_lib.hydro_batch_autotune(self._b, int(steps_per_rule), C.byref(r), C.byref(ms)),
               "hydro_batch_autotune")
        return r.value, ms.value

    def info(self):
        g, w, gr = C.c_int(), C.c_int64(), C.c_int()
        _check(_lib.hydro_batch_info(self._b, C.byref(g), C.byref(w), C.byref(gr)), "hydro_batch_info")
        return {"groups": g.value, "workgroups": w.value, "graph": bool(gr.value)}

    def close(self):
        if getattr(self, "_b", None):
            _lib.hydro_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def riemann_fluxes(precision, gamma, WL, WR, stream=None):
    """HLLC fluxes of face-normal state pairs on the GPU.

    WL, WR: float64 arrays (ntan+3, nfaces); returns F as numpy (ntan+3, nfaces).
    """
    import torch
    WL = np.ascontiguousarray(WL, dtype=np.float64)
    WR = np.ascontiguousarray(WR, dtype=np.float64)
    nc, nf = WL.shape
    dL = torch.from_numpy(WL).cuda()
    dR = torch.from_numpy(WR).cuda()
    dF = torch.empty_like(dL)
    s = stream or torch.cuda.current_stream()
    _check(_lib.hydro_riemann_fluxes(int(precision), nc - 3, float(gamma), nf, _vp(dL.data_ptr()),
                                     _vp(dR.data_ptr()), _vp(dF.data_ptr()), _vp(s.cuda_stream)),
           "hydro_riemann_fluxes")
    s.synchronize()
    return dF.cpu().numpy()


def conserved_totals_noalloc(cfg, U, out, stream=None):
    """hydro_conserved_totals_noalloc: the dV-weighted totals of the device
    state U (a contiguous float64 CUDA tensor in the layout of
    Hydro.state_view for the configuration cfg) written into out (a
    contiguous float64 CUDA tensor of ncomp values on U's device), enqueued on
    stream (default: the current stream) with no allocation and no host
    synchronisation."""
    import torch
    nc = cfg.ndim + 2
    cells = cfg.n[0] * cfg.n[1] * cfg.n[2]
    for t, k, what in ((U, nc * cells, "U"), (out, nc, "out")):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == k and t.device == U.device):
            raise HydroError(E_INVAL, f"conserved_totals_noalloc: {what} needs a contiguous float64 CUDA "
                                      f"tensor of {k} values on the state's device")
    s = stream or torch.cuda.current_stream(U.device)
    _check(_lib.hydro_conserved_totals_noalloc(C.byref(cfg), _vp(U.data_ptr()), _vp(out.data_ptr()),
                                                _vp(s.cuda_stream)), "hydro_conserved_totals_noalloc")


def tile_candidates(ndim, n, precision=FP64):
    """(tx, ty, kz) tiles the autotuner tries for a mesh of this shape."""
    cfg = make_config(n, 1.4, 0.4, precision)
    cnt = _lib.hydro_tile_candidates(C.byref(cfg), None, 0)
    _check(min(cnt, 0), "hydro_tile_candidates")
    buf = (C.c_int * (3 * cnt))()
    _lib.hydro_tile_candidates(C.byref(cfg), buf, cnt)
    return [tuple(buf[3 * i:3 * i + 3]) for i in range(cnt)]


def _tile_key(ndim, n, precision):
    import torch
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    return f"{arch}|{ndim}d|{'x'.join(str(v) for v in n)}|{'fp64' if precision == FP64 else 'mixed'}"


def _cache_read(path):
    import json
    try:
        with open(path) as f:
            return json.load(f)
    except (FileNotFoundError, ValueError):
        return {}


def _cache_store(path, key, entry):
    import json
    data = _cache_read(path)
    data[key] = entry
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def exported_symbols():
    """Names the library exports from the C ABI (for the ABI test)."""
    return sorted(_SIG)
