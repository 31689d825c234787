"""CPU hygiene of the oracle: results independent of the OpenMP thread count,
and a clean run under AddressSanitizer and UndefinedBehaviorSanitizer.

Both run the oracle in child processes (the thread count is fixed when the
OpenMP runtime starts, and a sanitizer runtime must be loaded first), over a
set of small runs that reach every entry point the tests use: the Heun and
van Leer runs in 1-D, 2-D and 3-D with every boundary rule, split and refined
meshes, totals, single-cell evaluation, HLLC and the exact Riemann solver.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import build as OB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
import numpy as np
sys.path.insert(0, sys.argv[2])
import oracle as O
from paper_2501_02317_amd import workloads as wl

out = {}
c = wl.turbulence_3d(n=(20, 12, 16), mach=1.5, seed=5, steps=4)
for integ in (O.HEUN, O.VL2):
    m = O.Mesh(c.n, c.gamma, c.lo, c.hi, c.bc, integrator=integ)
    U, t, s, dts = O.run(m, O.prim_to_cons(m, c.W), c.cfl, max_steps=4)
    out[f"turb3d_{integ}"] = U
    out[f"turb3d_{integ}_dts"] = dts
    out[f"turb3d_{integ}_tot"] = O.totals(m, U)
    U, t, s, dts = O.run_blocks(m, (2, 3, 2), O.prim_to_cons(m, c.W), c.cfl, max_steps=3)
    out[f"blocks3d_{integ}"] = U
m = O.Mesh(c.n, c.gamma, c.lo, c.hi, c.bc)
U0 = O.prim_to_cons(m, c.W)
out["cells"] = O.step_cells(m, U0, 1e-3, np.array([0, 7, 1000, m.shape[1] * m.shape[2] * m.shape[3] - 1]))
S = O.SMR(m, (2, 2, 2), [0, 5])
W = wl.smr_field(S.leaves, c.n, (2, 2, 2), gamma=c.gamma)
U, t, s, dts = S.run(S.prim_to_cons(W), c.cfl, max_steps=3)
out["smr"] = U
out["smr_tot"] = S.totals(U)
# every boundary rule, 2-D
imp = wl.implosion_2d(N=32, t_end=0.05)
m = O.Mesh(imp.n, imp.gamma, imp.lo, imp.hi, imp.bc)
U, t, s, dts = O.run(m, O.prim_to_cons(m, imp.W), imp.cfl, max_steps=6)
out["implosion"] = U
for bc in ((1, 2), (2, 3), (3, 1)):
    sod = wl.sod_1d(64)
    m = O.Mesh(sod.n, sod.gamma, sod.lo, sod.hi, (bc,))
    U, t, s, dts = O.run(m, O.prim_to_cons(m, sod.W), sod.cfl, t_end=0.05)
    out[f"sod_{bc[0]}{bc[1]}"] = U
rng = np.random.default_rng(3)
F = []
for _ in range(200):
    WL = np.array([np.exp(rng.uniform(-2, 2)), rng.uniform(-2, 2), rng.uniform(-2, 2), np.exp(rng.uniform(-2, 2))])
    WR = np.array([np.exp(rng.uniform(-2, 2)), rng.uniform(-2, 2), rng.uniform(-2, 2), np.exp(rng.uniform(-2, 2))])
    F.append(O.hllc(1.4, WL, WR))
out["hllc"] = np.array(F)
out["exact"] = np.array([O.exact_star(1.4, (1, 0, 1), (0.125, 0, 0.1), method=k) for k in (0, 1)])
np.savez(sys.argv[1], **out)
print("oracle script done", flush=True)
'''


def _run(tmp_path, tag, env_extra):
    out = tmp_path / f"{tag}.npz"
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", SCRIPT, str(out), ROOT], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    return np.load(out), r


def test_oracle_bitwise_independent_of_thread_count(tmp_path):
    """OpenMP only distributes independent faces and cells, so one thread and
    several give bitwise equal results."""
    OB.build(force=False)
    one, _ = _run(tmp_path, "t1", {"OMP_NUM_THREADS": "1"})
    many, _ = _run(tmp_path, "t5", {"OMP_NUM_THREADS": "5"})
    assert sorted(one.files) == sorted(many.files)
    for k in one.files:
        assert one[k].tobytes() == many[k].tobytes(), k


def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """A build with -fsanitize=address,undefined (errors fatal) runs the same
    entry points without a report, and gives the same results as the normal
    build."""
    so = tmp_path / "liborc_san.so"
    cmd = ["gcc", *[f for f in OB.FLAGS if f != "-O2"], "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", str(so),
           *[os.path.join(OB.HERE, s) for s in OB.SOURCES], "-lm"]
    subprocess.run(cmd, check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("no libasan runtime for gcc")
    san, r = _run(tmp_path, "san", {
        "ORACLE_LIB": str(so), "LD_PRELOAD": asan, "OMP_NUM_THREADS": "2",
        "ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    OB.build(force=False)
    ref, _ = _run(tmp_path, "ref", {"OMP_NUM_THREADS": "2"})
    for k in ref.files:
        # -O1 and -O2 evaluate the same IEEE operations (no contraction, no fast math)
        assert ref[k].tobytes() == san[k].tobytes(), k
