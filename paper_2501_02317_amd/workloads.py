"""Seeded synthetic initial conditions for the hydro workloads.

This module only draws and shapes input fields.  It holds none of the
method's arithmetic: every generator returns PRIMITIVE fields
W = (rho, v_1..v_ndim, p) as a float64 array of shape (ncomp, nz, ny, nx)
plus a plain description of the mesh and run; converting to conserved
variables is left to whichever solver consumes them.  Both the GPU path and
the CPU oracle read the same arrays from here.

Workloads (paper sections in brackets):
  * smooth_1d      -- 1-D periodic random-phase sine modes, gamma 1.4, CFL 0.4,
                      to t = 0.2 (256 cells by default).
  * two_state_1d   -- shock tube, free boundaries, discontinuity at x = 0.5
                      [Sec. 4.2]; sod_1d is (1,0,1)|(0.125,0,0.1).
  * random_two_state -- seeded non-vacuum shock-tube states.
  * linear_wave    -- sound / contact / shear eigenmodes on a periodic box
                      [Sec. 4.1].
  * turbulence_3d  -- log-normal density, Gaussian random velocity with
                      |v_k|^2 ~ k^-4 per mode (shell spectrum k^-2), uniform
                      p = 1/gamma so c_s = 1 at rho = 1.
  * shear_layer_2d -- double tanh shear layer with density ratio 1:2
                      [Sec. 4.5].
  * implosion_2d   -- diagonal two-state problem in a reflecting box
                      [Sec. 4.4, eq. lw-init].
  * batch_sizes    -- ragged 2-D mesh sizes for the batched workload.
  * smr_field      -- a smooth periodic random state (a few Fourier modes)
                      on the cell centres of a refined block mesh's leaves.
"""
from dataclasses import dataclass, field

import numpy as np

PERIODIC, FREE, OUTFLOW, REFLECT = 0, 1, 2, 3


@dataclass
class Case:
    """A workload: mesh, gas, run length and primitive initial state."""
    name: str
    n: tuple                  # active axes' cell counts, x first
    lo: tuple
    hi: tuple
    gamma: float
    cfl: float
    W: np.ndarray             # (ncomp, nz, ny, nx) primitive state
    bc: tuple = None          # per active axis (low, high)
    steps: int = 0            # fixed step count (0: run to t_end)
    t_end: float = 0.0
    meta: dict = field(default_factory=dict)

    def __post_init__(self):
        if self.bc is None:
            self.bc = ((PERIODIC, PERIODIC),) * len(self.n)

    @property
    def ndim(self):
        return len(self.n)

    @property
    def ncells(self):
        return int(np.prod(self.n))


def _shape(n):
    n = list(n) + [1] * (3 - len(n))
    return (n[2], n[1], n[0])


def _centres(n, lo, hi):
    """Cell-centre coordinates per active axis."""
    return [lo[d] + (np.arange(n[d]) + 0.5) * (hi[d] - lo[d]) / n[d] for d in range(len(n))]


def _pack(n, rho, vel, p):
    nd = len(n)
    W = np.empty((nd + 2,) + _shape(n))
    W[0] = rho
    for d in range(nd):
        W[1 + d] = vel[d]
    W[nd + 1] = p
    return W


def smooth_1d(N=256, seed=101, gamma=1.4, cfl=0.4, t_end=0.2):
    """rho = 1 + 0.2 sum_k (1/k) sin(2 pi k x + phi_k), v = 0.1 sum_k (1/k)
    sin(2 pi k x + psi_k), k = 1..8, p = 1 on the periodic unit interval."""
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2 * np.pi, 8)
    psi = rng.uniform(0.0, 2 * np.pi, 8)
    (x,) = _centres((N,), (0.0,), (1.0,))
    k = np.arange(1, 9)[:, None]
    rho = 1.0 + 0.2 * np.sum(np.sin(2 * np.pi * k * x + phi[:, None]) / k, axis=0)
    v = 0.1 * np.sum(np.sin(2 * np.pi * k * x + psi[:, None]) / k, axis=0)
    p = np.ones(N)
    return Case("smooth_1d", (N,), (0.0,), (1.0,), gamma, cfl,
                _pack((N,), rho, [v], p), t_end=t_end, meta={"seed": seed})


def two_state_1d(left, right, N=256, gamma=1.4, cfl=0.4, t_end=0.2, x0=0.5, name="two_state"):
    """Shock tube on [0, 1] with free boundaries; left/right = (rho, u, p)."""
    (x,) = _centres((N,), (0.0,), (1.0,))
    L = x < x0
    rho = np.where(L, left[0], right[0])
    v = np.where(L, left[1], right[1])
    p = np.where(L, left[2], right[2])
    return Case(name, (N,), (0.0,), (1.0,), gamma, cfl, _pack((N,), rho, [v], p),
                bc=((FREE, FREE),), t_end=t_end,
                meta={"left": tuple(left), "right": tuple(right), "x0": x0})


def sod_1d(N=256):
    return two_state_1d((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), N=N, name="sod_1d")


def implosion_2d(N=256, side=0.3, t_end=2.5, gamma=1.4, cfl=0.4):
    """Diagonal two-state problem with reflecting walls (the implosion of
    Sec. 4.4, eq. lw-init): (rho, p, v) = (0.125, 0.14, 0) where x + y <
    0.15, (1, 1, 0) elsewhere, on the square [0, side]^2 (side: a reading,
    twice the leg of the low-pressure triangle).  Symmetric under x <-> y."""
    n = (N, N)
    x, y = _centres(n, (0.0, 0.0), (side, side))
    low = (x[None, :] + y[:, None]) < 0.15
    rho = np.where(low, 0.125, 1.0)
    p = np.where(low, 0.14, 1.0)
    zero = np.zeros((N, N))
    W = _pack(n, rho.reshape(_shape(n)), [zero.reshape(_shape(n)), zero.reshape(_shape(n))],
              p.reshape(_shape(n)))
    bc = ((REFLECT, REFLECT), (REFLECT, REFLECT))
    return Case(f"implosion_{N}", n, (0.0, 0.0), (side, side), gamma, cfl, W, bc=bc, t_end=t_end)


def random_two_state(seed, gamma=1.4):
    """Non-vacuum two-state data: rho, p log-uniform in [0.1, 10], u in [-1, 1]."""
    rng = np.random.default_rng(seed)
    while True:
        rl, rr, pl, pr = np.exp(rng.uniform(np.log(0.1), np.log(10.0), 4))
        ul, ur = rng.uniform(-1.0, 1.0, 2)
        cl, cr = np.sqrt(gamma * pl / rl), np.sqrt(gamma * pr / rr)
        if 2.0 * (cl + cr) / (gamma - 1.0) > (ur - ul) + 1.0:
            return (float(rl), float(ul), float(pl)), (float(rr), float(ur), float(pr))


def linear_wave(kind, N, ndim=1, amp=1e-6, direction=1.0, gamma=5.0 / 3.0, cfl=0.4,
                profile="sine", ny=4):
    """Eigenmodes on a periodic unit box, run for one crossing (t = 1).

    Background rho0 = 1, p0 = 1/gamma so the sound speed is 1 [Sec. 4.1].
    kind: 'sound' (right-going acoustic mode), 'contact' (density only,
    advected at v_x = direction), 'shear' (v_y only, advected at v_x =
    direction; needs ndim = 2, run on an N x ny mesh).
    """
    n = (N,) if ndim == 1 else (N, ny)
    lo = (0.0,) * ndim
    hi = (1.0,) * ndim if ndim == 1 else (1.0, ny / N)
    xs = _centres(n, lo, hi)
    x = xs[0][None, None, :] * np.ones(_shape(n))
    if profile == "sine":
        f = np.sin(2 * np.pi * x)
    else:
        f = np.where(x < 0.5, 1.0, 0.0)
    rho0, p0 = 1.0, 1.0 / gamma
    c0 = np.sqrt(gamma * p0 / rho0)
    vel = [np.zeros(_shape(n)) for _ in range(ndim)]
    if kind == "sound":
        drho = amp * f
        rho = rho0 + drho
        vel[0] = vel[0] + (c0 / rho0) * drho
        p = p0 + c0 * c0 * drho
        t_end = 1.0 / c0
    elif kind == "contact":
        rho = rho0 + amp * f
        vel[0] = vel[0] + direction
        p = np.full(_shape(n), p0)
        t_end = 1.0
    elif kind == "shear":
        if ndim < 2:
            raise ValueError("shear waves need ndim >= 2")
        rho = np.full(_shape(n), rho0)
        vel[0] = vel[0] + direction
        vel[1] = vel[1] + amp * f
        p = np.full(_shape(n), p0)
        t_end = 1.0
    else:
        raise ValueError(kind)
    return Case(f"{kind}_wave", n, lo, hi, gamma, cfl, _pack(n, rho, vel, p), t_end=t_end,
                meta={"amp": amp, "direction": direction, "profile": profile})


def _grf(rng, n, kmin, kmax, slope):
    """Real Gaussian random field on an n^3 (or n^2) periodic grid: white
    noise filtered to kmin <= |k| <= kmax with per-mode amplitude |k|^slope."""
    shape = tuple(n)
    noise = rng.standard_normal(shape)
    F = np.fft.rfftn(noise)
    ks = [np.fft.fftfreq(m) * m for m in shape[:-1]] + [np.fft.rfftfreq(shape[-1]) * shape[-1]]
    grids = np.meshgrid(*ks, indexing="ij")
    kmag = np.sqrt(sum(g * g for g in grids))
    amp = np.zeros_like(kmag)
    sel = (kmag >= kmin) & (kmag <= kmax)
    amp[sel] = kmag[sel] ** slope
    F *= amp
    del grids, kmag, amp
    out = np.fft.irfftn(F, s=shape, axes=tuple(range(len(shape))))
    return out


def turbulence_3d(n=128, mach=1.0, seed=201, gamma=5.0 / 3.0, cfl=0.3, steps=200, kmax=16,
                  sigma=0.1, ndim=3):
    """n: cells per axis (int, with ndim axes) or a tuple of per-axis counts.

    Log-normal density (flat spectrum over 1 <= |k| <= kmax, std sigma in
    log space, unit mean) and a zero-mean Gaussian random velocity with
    per-mode |v_k|^2 ~ k^-4 (shell spectrum k^-2, ndim = 3) over the same
    band, scaled to rms |v| = mach (c_s = 1 with p = 1/gamma, rho = 1)."""
    rng = np.random.default_rng(seed)
    nn = tuple(int(v) for v in n) if isinstance(n, (tuple, list)) else (int(n),) * ndim
    ndim = len(nn)
    grid = _shape(nn)[3 - ndim:]
    s = _grf(rng, grid, 1.0, kmax, 0.0)
    s *= sigma / s.std()
    rho = np.exp(s)
    rho /= rho.mean()
    slope = -2.0 if ndim == 3 else -1.5  # |v_k| ~ k^-2 (3-D), k^-1.5 (2-D): shell E(k) ~ k^-2
    vel = []
    for _ in range(ndim):
        v = _grf(rng, grid, 1.0, kmax, slope)
        v -= v.mean()
        vel.append(v)
    vrms = np.sqrt(np.mean(sum(v * v for v in vel)))
    vel = [v * (mach / vrms) for v in vel]
    p = np.full(grid, 1.0 / gamma)
    # array axes are (z, y, x) and velocity components follow x, y, z: the
    # three random fields are independent, so assign them in axis order.
    full = _shape(nn)
    W = _pack(nn, rho.reshape(full), [v.reshape(full) for v in vel], p.reshape(full))
    lo = (0.0,) * ndim
    hi = (1.0,) * ndim
    name = f"turbulence_{ndim}d_" + "x".join(str(v) for v in nn)
    return Case(name, nn, lo, hi, gamma, cfl, W, steps=steps,
                meta={"seed": seed, "mach": mach, "kmax": kmax, "sigma": sigma})


def shear_layer_2d(nx, ny, seed, gamma=1.4, cfl=0.4, steps=300, width=0.02, amp=0.01):
    """Double shear layer on [-1/2, 1/2]^2 (periodic): rho = 1.5 + 0.5 tanh((|y|
    - 1/4)/w) (ratio 1:2), v_x = 0.5 tanh((|y| - 1/4)/w) (jump +-0.5), v_y =
    amp g(x) [exp(-(y - 1/4)^2 / (2 * 0.2^2)) + exp(-(y + 1/4)^2 / (2 * 0.2^2))]
    with g eight random-phase integer-k sines scaled to max |g| = 1; p = 2.5."""
    rng = np.random.default_rng(seed)
    x, y = _centres((nx, ny), (-0.5, -0.5), (0.5, 0.5))
    X = x[None, :]
    Y = y[:, None]
    th = np.tanh((np.abs(Y) - 0.25) / width)
    rho = 1.5 + 0.5 * th + 0.0 * X
    vx = 0.5 * th + 0.0 * X
    phases = rng.uniform(0.0, 2 * np.pi, 8)
    k = np.arange(1, 9)[:, None]
    g = np.sum(np.sin(2 * np.pi * k * (x[None, :] + 0.5) + phases[:, None]), axis=0)
    g /= np.abs(g).max()
    env = np.exp(-((Y - 0.25) ** 2) / (2 * 0.2 ** 2)) + np.exp(-((Y + 0.25) ** 2) / (2 * 0.2 ** 2))
    vy = amp * g[None, :] * env
    p = np.full((ny, nx), 2.5)
    n = (nx, ny)
    W = _pack(n, rho.reshape(_shape(n)), [vx.reshape(_shape(n)), vy.reshape(_shape(n))],
              p.reshape(_shape(n)))
    return Case(f"shear_layer_{nx}x{ny}", n, (-0.5, -0.5), (0.5, 0.5), gamma, cfl, W,
                steps=steps, meta={"seed": seed})


BATCH_SIZES = (64, 96, 128, 192, 256, 384, 512)


def batch_sizes(count=512, seed=401):
    """Per-mesh (nx, ny) drawn iid uniform from BATCH_SIZES."""
    rng = np.random.default_rng(seed)
    nx = rng.choice(BATCH_SIZES, count)
    ny = rng.choice(BATCH_SIZES, count)
    return [(int(a), int(b)) for a, b in zip(nx, ny)]


def batch_cases(count=512, seed=401, steps=300):
    return [shear_layer_2d(nx, ny, seed=4000 + m, steps=steps)
            for m, (nx, ny) in enumerate(batch_sizes(count, seed))]


def random_field_device(ndim, n, mach, gamma, seed, kmax=16, sigma=0.1, modes=48, device="cuda"):
    """Primitive state of a random-field request, generated on the GPU as a
    sum of seeded random Fourier modes (no FFT plans, so any mesh size costs
    the same to set up).  Each field is sum_i a_i cos(2 pi k_i . x + phi_i)
    over `modes` integer wavevectors with 1 <= |k_i| <= kmax, a_i ~ |k_i|^s
    with s = 0 for the log-density and a shell spectrum k^-2 for each
    velocity component; log-density std sigma, unit-mean density, zero-mean
    velocity with rms |v| = mach, p = 1/gamma.  Mode parameters come from a
    numpy generator seeded with `seed`.  Returns a contiguous float64 CUDA
    tensor of shape (ndim + 2, nz, ny, nx)."""
    import torch

    rng = np.random.default_rng(int(seed))
    kmax = max(1, int(kmax))
    cand = np.stack(np.meshgrid(*[np.arange(-kmax, kmax + 1)] * ndim, indexing="ij"), -1).reshape(-1, ndim)
    kn = np.sqrt((cand ** 2).sum(1))
    cand, kn = cand[(kn >= 1) & (kn <= kmax)], kn[(kn >= 1) & (kn <= kmax)]
    x = (torch.arange(n, device=device, dtype=torch.float64) + 0.5) / n
    slope = -2.0 if ndim == 3 else -1.5

    def field(s):
        pick = rng.integers(0, len(cand), modes)
        k = cand[pick]
        a = kn[pick] ** s * rng.standard_normal(modes)
        ph = rng.uniform(0.0, 2 * np.pi, modes)
        # the mode table (k, amplitude, phase) in one copy that does not wait
        # for the stream (from page-locked memory on a GPU)
        tab = torch.from_numpy(np.concatenate([k.astype(np.float64), a[:, None], ph[:, None]], axis=1))
        if torch.device(device).type == "cuda":
            tab = tab.pin_memory().to(device, non_blocking=True)
        # 2 pi k_d x_d of every mode along each axis, then the modes eight
        # at a time: phase plus the axis terms, cosine, amplitude, summed
        axis = [(2 * np.pi) * (tab[:, d].reshape(modes, 1) * x.view(1, n)) for d in range(ndim)]
        out = torch.zeros((n,) * ndim, device=device, dtype=torch.float64)
        for c0 in range(0, modes, 8):
            m = min(8, modes - c0)
            arg = tab[c0:c0 + m, ndim + 1].reshape(m, *[1] * ndim)
            for d in range(ndim):
                shp = [m] + [1] * ndim
                shp[1 + d] = n
                arg = arg + axis[d][c0:c0 + m].view(shp)
            amp = tab[c0:c0 + m, ndim].reshape(m, *[1] * ndim)
            out += (amp * torch.cos(arg)).sum(0)
        return out

    s = field(0.0)
    s = s * (sigma / s.std())
    rho = torch.exp(s)
    rho = rho / rho.mean()
    vel = []
    for _ in range(ndim):
        v = field(slope)
        vel.append(v - v.mean())
    vrms = torch.sqrt(torch.mean(sum(v * v for v in vel)))
    vel = [v * (mach / vrms) for v in vel]
    p = torch.full((n,) * ndim, 1.0 / gamma, device=device, dtype=torch.float64)
    # fields are indexed (x, y[, z]); the state layout is (z, y, x)
    stack = torch.stack([rho] + vel + [p])
    stack = stack.permute(0, *range(ndim, 0, -1))
    full = (1,) * (3 - ndim) + (n,) * ndim
    return stack.reshape((ndim + 2,) + full).contiguous()


def leaf_centres(leaves, n, blocks, lo=None, hi=None):
    """Cell-centre coordinates of each leaf of a refined block mesh: leaves
    rows are (level, c0, c1, c2) on the leaf's level; n the level-0 cell
    counts; returns ndim arrays of shape (nleaf, bz, by, bx)."""
    nd = len(n)
    lo = lo or (0.0,) * nd
    hi = hi or (1.0,) * nd
    leaves = np.asarray(leaves)
    bn = [n[d] // blocks[d] for d in range(nd)] + [1] * (3 - nd)
    out = []
    for d in range(nd):
        dxl = (hi[d] - lo[d]) / n[d] / 2.0 ** leaves[:, 0]
        org = lo[d] + leaves[:, 1 + d] * bn[d] * dxl
        shp = [1, 1, 1]
        shp[2 - d] = bn[d]
        x = org[:, None, None, None] + (np.arange(bn[d]).reshape(shp)[None] + 0.5) * dxl[:, None, None, None]
        out.append(np.broadcast_to(x, (len(leaves), bn[2], bn[1], bn[0])).copy())
    return out


def smr_field(leaves, n, blocks, gamma=5.0 / 3.0, mach=0.5, amp=0.2, seed=71, modes=6):
    """Block-layout primitive state (nleaf, ndim + 2, bz, by, bx) of a smooth
    periodic random field on a unit box: density and pressure 1 + amp f,
    velocities mach f, each f a mean of `modes` seeded sines with integer
    wavenumbers 1..2 per axis."""
    rng = np.random.default_rng(seed)
    nd = len(n)
    X = leaf_centres(leaves, n, blocks)

    def f(scale):
        acc = np.zeros(X[0].shape)
        for _ in range(modes):
            k = rng.integers(1, 3, size=nd)
            ph = rng.random() * 2 * np.pi
            acc = acc + np.sin(sum(2 * np.pi * k[d] * X[d] for d in range(nd)) + ph)
        return scale * acc / modes

    W = np.empty((len(X[0]), nd + 2) + X[0].shape[1:])
    W[:, 0] = 1.0 + f(amp)
    for d in range(nd):
        W[:, 1 + d] = f(mach)
    W[:, -1] = 1.0 / gamma + f(amp / gamma)
    return W
