"""Whole-run parity at the benchmark sizes: 128^3 Mach-1 for 200 steps (FP64)
and 256^3 Mach-2 for 100 steps (FP64 and mixed), and the van Leer integrator
(Sec. 3.3) on 128^3 Mach-1 for 100 steps (FP64 and mixed), the paper's
Table 1 grid (2-D 4096 x 1024) for 40 steps (FP64 and mixed), and the
benchmark's refined mesh for 40 steps (FP64 and mixed), GPU against the FP64
oracle run on the host cores (about six minutes of oracle time at 16
threads).  The oracle prints a progress line every ten steps straight to the
terminal (past pytest's output capture), so the run is never silent for long.
"""
import dataclasses
import os
import time

import numpy as np
import pytest

import oracle as O
from paper_2501_02317_amd import workloads as wl
from gpu_util import gpu_mesh, oracle_mesh, rel_l1, say

# the oracle runs inside the first test of each workload: minutes, not seconds
pytestmark = [pytest.mark.gpu, pytest.mark.slow, pytest.mark.timeout(900)]


@pytest.fixture(scope="module")
def H():
    import torch
    assert torch.cuda.is_available()
    from paper_2501_02317_amd import hydro
    return hydro


# name: (workload, integrator)
CASES = {
    "c2_128_mach1_200": (lambda: wl.turbulence_3d(n=128, mach=1.0, seed=201, steps=200, cfl=0.3), 0),
    "c3_256_mach2_100": (lambda: wl.turbulence_3d(n=256, mach=2.0, seed=301, steps=100, cfl=0.3), 0),
    "vl2_128_mach1_100": (lambda: wl.turbulence_3d(n=128, mach=1.0, seed=211, steps=100, cfl=0.3), 1),
    # the paper's Table 1 grid (Sec. 4.3): 4096 x 1024 square cells on [0,4] x [0,1]
    # (40 steps: the oracle's 2-D path runs on one thread, at about 3e6 cell-updates/s)
    "grid_4096x1024_40": (lambda: dataclasses.replace(
        wl.turbulence_3d(n=(4096, 1024), mach=1.0, seed=601, gamma=1.4, cfl=0.4, steps=40), hi=(4.0, 1.0)), 0),
}
_oracle_cache = {}


def oracle_result(name):
    if name not in _oracle_cache:
        make, integ = CASES[name]
        c = make()
        m = oracle_mesh(c, integ)
        U0 = O.prim_to_cons(m, c.W)
        t0 = time.perf_counter()
        # in chunks of 10 steps (each dt comes from the state it starts from,
        # so the chunks give the same result as one run), reporting progress
        U, t, s = U0, 0.0, 0
        while s < c.steps:
            k = min(10, c.steps - s)
            U, t, done, _ = O.run(m, U, c.cfl, max_steps=k, t0=t)
            s += done
            print(f"[oracle] {name}: step {s}/{c.steps} t={t:.6e} "
                  f"({time.perf_counter() - t0:.0f} s)", flush=True)
        el = time.perf_counter() - t0
        print(f"[oracle] {name}: {s} steps to t={t:.6e} in {el:.1f} s "
              f"({c.ncells * s / el:.3e} cell-updates/s, OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS')})",
              flush=True)
        _oracle_cache[name] = (c, m, U0, U, t, s)
    return _oracle_cache[name]


@pytest.mark.parametrize("name,precision,tol", [("c2_128_mach1_200", 0, 1e-12),
                                                ("c3_256_mach2_100", 0, 1e-12),
                                                ("c3_256_mach2_100", 1, 1e-5),
                                                ("vl2_128_mach1_100", 0, 1e-12),
                                                ("vl2_128_mach1_100", 1, 1e-5),
                                                ("grid_4096x1024_40", 0, 1e-12),
                                                ("grid_4096x1024_40", 1, 1e-5)])
def test_full_run_against_oracle(H, capsys, name, precision, tol):
    with capsys.disabled():
        c, m, U0, U_o, t_o, s_o = oracle_result(name)
    say("full run", name, precision)
    h = gpu_mesh(c, precision, CASES[name][1])
    h.step_auto(c.steps)
    U = h.get_state()
    t, s = h.time(), h.steps_done()
    T = h.totals()
    h.close()
    err = rel_l1(U, U_o)
    T0 = O.totals(m, U0)
    dV = np.prod(m.dx)
    drift = np.abs(T - T0) / (dV * np.abs(U0).reshape(m.ncomp, -1).sum(axis=1))
    with capsys.disabled():
        print(f"\n[parity] {name} precision={precision}: relL1 per component {err}, "
              f"t {t:.15e} vs oracle {t_o:.15e}, steps {s} vs {s_o}, totals drift / (dV sum|U|) {drift}",
              flush=True)
    assert s == s_o
    assert np.all(err <= tol)
    assert np.all(drift <= 1e-12)


# The refined mesh of the benchmark's refinement leg (Sec. 2.3.1, Sec. 3.1.2):
# 128^3 level-0 cells in 4x4x4 blocks of 32^3 with the central 2x2x2 blocks
# refined (120 leaves, 3.9 million cells), a smooth Mach-1 field, gamma 5/3,
# CFL 0.3, 40 Heun steps.
SMR_N, SMR_B, SMR_STEPS = (128, 128, 128), (4, 4, 4), 40
SMR_REFINED = [bx + 4 * (by + 4 * bz) for bz in (1, 2) for by in (1, 2) for bx in (1, 2)]
_smr_cache = {}


def oracle_smr_result():
    if not _smr_cache:
        m = O.Mesh(SMR_N, 5.0 / 3.0)
        S = O.SMR(m, SMR_B, SMR_REFINED)
        W = wl.smr_field(S.leaves, SMR_N, SMR_B, mach=1.0)
        U0 = S.prim_to_cons(W)
        print(f"[oracle] refined 128^3, {len(S.leaves)} leaves: {SMR_STEPS} steps ...", flush=True)
        t0 = time.perf_counter()
        U, t, s, _ = S.run(U0, 0.3, max_steps=SMR_STEPS)
        el = time.perf_counter() - t0
        cells = int(np.prod(S.shape)) // m.ncomp
        print(f"[oracle] refined 128^3: {s} steps to t={t:.6e} in {el:.1f} s "
              f"({cells * s / el:.3e} cell-updates/s)", flush=True)
        _smr_cache.update(S=S, W=W, U0=U0, U=U, t=t, s=s)
    return _smr_cache


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-5)])
def test_refined_run_against_oracle(H, capsys, precision, tol):
    with capsys.disabled():
        r = oracle_smr_result()
    S = r["S"]
    say("full run refined", precision)
    h = H.Hydro(SMR_N, 5.0 / 3.0, 0.3, precision=precision, blocks=SMR_B, refined=SMR_REFINED)
    assert np.array_equal(h.leaves, S.leaves)
    h.set_primitive(r["W"])
    T0 = h.totals()
    h.step_auto(SMR_STEPS)
    U, t, s, T = h.get_state(), h.time(), h.steps_done(), h.totals()
    h.close()
    nc = S.mesh.ncomp
    a = U.transpose(1, 0, 2, 3, 4).reshape(nc, -1)
    b = r["U"].transpose(1, 0, 2, 3, 4).reshape(nc, -1)
    err = np.abs(a - b).sum(axis=1) / np.abs(b).sum(axis=1)
    scale = S.totals(np.abs(r["U0"]))
    drift = np.abs(T - T0) / scale
    with capsys.disabled():
        print(f"\n[parity] refined 128^3 precision={precision}: relL1 per component {err}, "
              f"t {t:.15e} vs oracle {r['t']:.15e}, steps {s} vs {r['s']}, totals drift / sum|U| {drift}",
              flush=True)
    assert s == r["s"] == SMR_STEPS
    assert np.all(err <= tol)
    assert np.all(drift <= 1e-12)
