"""Throughput benchmark of the Godunov hydro step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Workload: 3-D periodic box, gamma = 5/3, 256^3 cells, seeded Mach-2
log-normal / Gaussian random-field initial state, CFL 0.3; the Heun step
(PLM + HLLC, device-resident CFL dt) run in mixed precision (the headline
value) and in FP64.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  value = mixed-precision cell-updates/s (one update =
one full two-stage Heun step of one cell).  roofline = the stage kernel
(both stage launches of a step, with their algorithmic bytes: stage 1 reads
U^n and writes U1, stage 2 reads U1 and U^n and writes U^{n+1}, 5 x ncomp x
8 B = 200 B per 3-D cell-update) against the 8 TB/s HBM peak, timed with HIP
events on the launch stream inside the timed region.  cpu_baseline = the
FP64 oracle on the host cores for one Heun step of the same 256^3 state.
by_precision.*.host_inclusive = the same run with the state handed over in
host memory (upload over PCIe, the steps, download), measured after the timed
region; it is never the value.  Further legs (each with a --no-* switch): the
van Leer integrator, the mesh split into blocks, a statically refined mesh,
the paper's Table 1 grid (2-D 4096 x 1024, with the paper's own figures for
context), the 512-mesh batch and the serving loop.
"""
import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-updates/s mixed vs FP64 at 256^3 (HBM roofline %); batched p50/p99 latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 2-D workload")
    ap.add_argument("--no-vl2", action="store_true", help="skip the van Leer integrator leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--no-blocks", action="store_true", help="skip the multi-block leg")
    ap.add_argument("--no-smr", action="store_true", help="skip the static-refinement leg")
    ap.add_argument("--no-paper-grid", action="store_true",
                    help="skip the 2-D 4096x1024 leg on the grid of the paper's Table 1")
    ap.add_argument("--smr-only", action="store_true",
                    help="run only the static-refinement leg and print its record (for kernel traces)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving leg and print its record (for kernel traces)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--serve-calib", type=int, default=300,
                    help="requests of the saturation run that measures capacity (and of its "
                         "one-at-a-time baseline)")
    ap.add_argument("--tile", default="",
                    help="fixed tile tx,ty,kz (kz 0: automatic) for both stages instead of autotuning")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the library's default stage tiles (no autotuning), e.g. for profiler "
                         "runs that should see one kernel per stage")
    ap.add_argument("--cpu-worker", default="",
                    help="internal: run one single-thread oracle worker seed,n,steps,start_at and exit")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes five times "
                         "(calibrates the HBM byte counters) and exit")
    return ap.parse_args()


def copy_calibration(nbytes):
    import torch
    n = nbytes // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 8, "launches": 5}), flush=True)


def stage_bytes(ndim, precision, integrator):
    """Algorithmic bytes per cell of the stage-1 and stage-2 launches.
    Heun: read U^n, write U1 (FP64); read U1 and U^n, write U^{n+1}.  van
    Leer: read U^n, write the predicted primitive state (compute type); read
    it and U^n, write U^{n+1}."""
    nc = ndim + 2
    if integrator == 0:
        return 2 * nc * 8, 3 * nc * 8
    r = 8 if precision == 0 else 4
    return nc * (8 + r), nc * (r + 16)


def bytes_per_update(ndim, precision=0, integrator=0):
    return sum(stage_bytes(ndim, precision, integrator))


SETTLE_S = 0.04   # seconds of back-to-back steps before a timed region


def settle(h, warmup, min_s=SETTLE_S, cap=2000):
    """The warm-up steps, followed by more untimed steps until the GPU has
    run steps back to back for min_s seconds: after host work or idle time
    the engine clock takes tens of milliseconds of load to climb back to its
    peak, and a timed region that starts earlier measures that climb.
    Returns the number of untimed steps taken."""
    import math
    import torch
    stream = torch.cuda.current_stream()
    done, elapsed, n = 0, 0.0, max(int(warmup), 1)
    while True:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        h.step_auto(n)
        b.record(stream)
        b.synchronize()
        done += n
        elapsed += a.elapsed_time(b) * 1e-3
        if elapsed >= min_s or done >= cap:
            return done
        per_step = elapsed / done
        n = min(cap - done, max(1, math.ceil((min_s - elapsed) / per_step) + 1))


def run_precision(H, case, precision, steps, warmup, tile=None, tune=True, integrator=0, blocks=None,
                  streams=False, host_io=False):
    import torch
    h = H.Hydro(case.n, case.gamma, case.cfl, precision=precision, lo=case.lo, hi=case.hi, bc=case.bc,
                integrator=integrator, blocks=blocks)
    h.set_primitive(case.W)
    if tile or not tune:
        if tile:
            h.set_tile(*tile)
        tiles = h.get_tile()
    else:
        tiles, _ = h.autotune(3)   # tuning steps are warm-up steps of the run
    if streams:
        h.set_block_streams(True)  # per-block launches (stage timing records none)
    # the seeded state kept on the device: resetting to it right before the
    # timed region takes a quarter of a millisecond, where an upload from
    # host memory would leave the GPU idle (and its clock falling) for tens
    W_dev = torch.from_numpy(np.ascontiguousarray(case.W)).to(h.device)
    untimed = settle(h, warmup)
    h.set_primitive_device(W_dev)  # timed run starts from the seeded state
    torch.cuda.synchronize()
    del W_dev
    h.profile(steps)
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    h.step_auto(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    ms1, ms2, (n1, n2) = h.profile_read()
    h.profile(0)
    # the timed launches advanced the run: stage kernels return early once a
    # run limit is reached, and timing such empty launches would mean nothing
    done = h.steps_done()
    if done != steps or (not streams and (n1 != steps or n2 != steps)):
        raise RuntimeError(f"timed run advanced {done} steps ({n1}, {n2} stage launches), expected {steps}")
    t_sim = h.time()
    T = h.totals()
    host = host_inclusive(h, case, steps) if host_io else None
    h.close()
    cells = case.ncells
    rate = cells * steps / (ms * 1e-3)
    nc = case.ndim + 2
    b1, b2 = stage_bytes(case.ndim, precision, integrator)
    alg_bytes = (b1 * n1 + b2 * n2) * cells                  # stage-1 and stage-2 launches
    kern_ms = ms1 + ms2
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    return {
        "rate": rate, "ms_per_step": ms / steps, "wall_s": wall, "t_sim": t_sim,
        "stage_ms": [ms1 / max(n1, 1), ms2 / max(n2, 1)], "launches": [n1, n2],
        "achieved_gbs": achieved, "frac": achieved / HBM_PEAK_GBS if achieved else None, "totals": T.tolist(),
        "step_frac": rate * bytes_per_update(case.ndim, precision, integrator) / 1e9 / HBM_PEAK_GBS,
        "tiles": [list(t) for t in tiles],
        "untimed_steps": untimed,
        "host_inclusive": host,
    }


def host_inclusive(h, case, steps):
    """The same run with the state handed over in host memory, after the
    timed region: primitive state uploaded over PCIe (and converted to
    conserved variables), the steps, the conserved state downloaded."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.set_primitive(case.W)
    t1 = time.perf_counter()
    h.step_auto(steps)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    U = h.get_state()
    t3 = time.perf_counter()
    h.get_state(out=U)                 # again, into host memory already touched
    t4 = time.perf_counter()
    return {"value": case.ncells * steps / (t3 - t0), "unit": "cell-updates/s",
            "upload_s": t1 - t0, "steps_s": t2 - t1, "download_s": t3 - t2,
            "download_reused_s": t4 - t3, "bytes_each_way": int(U.nbytes)}


def run_batch(H, wl, count, steps, precision):
    """Ragged 2-D shear-layer meshes: one batched, graph-replayed run against
    the same meshes stepped one at a time (hydro_step_auto per mesh)."""
    import torch
    cases = wl.batch_cases(count=count, seed=401, steps=steps)
    s = torch.cuda.Stream()
    ms = [H.Hydro(c.n, c.gamma, c.cfl, precision=precision, lo=c.lo, hi=c.hi, bc=c.bc, stream=s)
          for c in cases]

    def reset():
        for h, c in zip(ms, cases):
            h.set_primitive(c.W)
            h.set_run_limit(steps, 0.0)
        s.synchronize()

    # the seeded states kept on the device for the reset right before the
    # timed run (a host upload there would idle the GPU, see settle())
    W_dev = [torch.from_numpy(np.ascontiguousarray(c.W)).to(h.device) for h, c in zip(ms, cases)]

    def reset_device():
        for h, w in zip(ms, W_dev):
            h.set_primitive_device(w)
            h.set_run_limit(steps, 0.0)
        s.synchronize()

    cells = sum(c.ncells for c in cases)
    b = H.Batch(ms, use_graph=True)
    reset()
    rule, _ = b.autotune(2)                       # tile rule for the batch (real steps)
    reset()
    b.step(steps)                                 # warm-up: captures the graph
    s.synchronize()
    reset_device()
    del W_dev
    t0 = time.perf_counter()
    b.step(steps)
    s.synchronize()
    t_batch = time.perf_counter() - t0
    done, st, flags = b.status()
    assert all(done) and not any(flags)
    info = b.info()
    b.close()
    reset()
    t0 = time.perf_counter()
    for h in ms:
        h.step_auto(steps)
    s.synchronize()
    t_one = time.perf_counter() - t0
    for h in ms:
        h.close()
    return {"meshes": count, "cells": cells, "steps": steps,
            "precision": "mixed" if precision == H.MIXED else "fp64",
            "batched_cell_updates_per_s": cells * steps / t_batch,
            "one_at_a_time_cell_updates_per_s": cells * steps / t_one,
            "speedup": t_one / t_batch, "batched_s": t_batch, "one_at_a_time_s": t_one,
            "launch_groups": info["groups"], "graph": info["graph"], "tile_rule": rule}


def run_smr(H, wl, steps, warmup):
    """Two-level static refinement in 3-D: 128^3 level-0 cells in 4x4x4
    blocks of 32^3 with the central 2x2x2 blocks refined (120 leaves), mixed
    precision, against the same blocks unrefined (64 leaves of 32^3)."""
    import torch
    n, B = (128, 128, 128), (4, 4, 4)
    refined = [bx + 4 * (by + 4 * bz) for bz in (1, 2) for by in (1, 2) for bx in (1, 2)]

    def timed(ref):
        cfg = H.make_config(n, 5.0 / 3.0, 0.3, precision=H.MIXED, blocks=B)
        leaves = H.smr_leaves(cfg, ref)
        W = wl.smr_field(leaves, n, B, mach=1.0)
        h = H.Hydro(n, 5.0 / 3.0, 0.3, precision=H.MIXED, blocks=B, refined=ref)
        h.set_primitive(W)
        W_dev = torch.from_numpy(np.ascontiguousarray(W)).to(h.device)
        settle(h, warmup)
        h.set_primitive_device(W_dev)  # timed run from the seeded state (device-side reset)
        torch.cuda.synchronize()
        del W_dev
        stream = torch.cuda.current_stream()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        h.step_auto(steps)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        if h.steps_done() != steps:
            raise RuntimeError(f"refined timed run advanced {h.steps_done()} steps, expected {steps}")
        cells = int(W.shape[0] * np.prod(W.shape[2:]))
        h.close()
        return cells * steps / (ms * 1e-3), ms / steps, len(leaves), cells

    v, ms, nl, cells = timed(refined)
    v0, ms0, _, cells0 = timed([])
    return {"value": v, "ms_per_step": ms, "leaves": nl, "cells": cells, "precision": "mixed",
            "split_value": v0, "split_ms_per_step": ms0, "split_cells": cells0,
            "config": "128^3 level 0 in 4x4x4 blocks of 32^3, central 2x2x2 refined, smooth Mach-1 field"}


# The paper's own throughput on its Table 1 workload (2-D double Mach
# reflection on a 4096 x 1024 grid, Sec. 4.3), in 1e8 cells per second for
# one full step, by device: (single, mixed, double).  Context only: other
# hardware, and that run has reflecting and time-dependent boundaries where
# this leg's box is periodic.
PAPER_TABLE1 = {
    "RTX 4090 (CUDA)": (21.0, 16.0, 2.9),
    "Tesla A100 (CUDA)": (16.0, 14.0, 8.3),
    "RX 7900 XTX (HIP)": (8.9, 7.7, 2.8),
    "MI100 (HIP)": (8.2, 6.8, 3.0),
}


def run_paper_grid(H, wl, steps, warmup, tune=True):
    """The paper's Table 1 grid, 4096 x 1024 square cells on [0,4] x [0,1],
    gamma = 1.4, CFL 0.4: a seeded periodic random field (Mach 1) in place of
    the double Mach reflection, both precisions, autotuned tiles."""
    import dataclasses
    case = wl.turbulence_3d(n=(4096, 1024), mach=1.0, seed=601, gamma=1.4, cfl=0.4, steps=steps)
    case = dataclasses.replace(case, hi=(4.0, 1.0))
    out = {"grid": [4096, 1024], "cells": case.ncells, "data": "synthetic periodic random field, Mach 1",
           "alg_bytes_per_cell_update": bytes_per_update(2)}
    for name, prec in (("mixed", H.MIXED), ("fp64", H.FP64)):
        r = run_precision(H, case, prec, steps, warmup, None, tune)
        out[name] = {"value": r["rate"], "ms_per_step": r["ms_per_step"], "roofline_frac": r["frac"],
                     "tiles": r["tiles"]}
        print(f"[bench] paper grid {name}: {r['rate']:.3e} cell-updates/s, {r['ms_per_step']:.3f} ms/step",
              file=sys.stderr, flush=True)
    out["paper_table1_1e8_cells_per_s"] = {k: {"single": v[0], "mixed": v[1], "double": v[2]}
                                           for k, v in PAPER_TABLE1.items()}
    return out


def run_serving(count, calib):
    """Served capacity at saturation (calib requests, all at t = 0, after an
    untimed warm-up of four small requests) against the same requests served
    one at a time; then a Poisson stream of count requests offered at 0.8 x
    the measured capacity, with p50/p99 completion latency."""
    from paper_2501_02317_amd import serving as S

    def log(line):
        print(line, file=sys.stderr, flush=True)

    # a warm-up of the serving path (its first kernels load their code), not timed
    warm = S.request_stream(4, 1.0, seed=503, steps=(20, 40))
    for r in warm:
        r.arrival = 0.0
    S.Server(4 << 30, steps_per_iter=16).run(warm)
    sat = S.request_stream(calib, 1.0, seed=502)
    for r in sat:
        r.arrival = 0.0
    work = sum(r.cells * r.steps for r in sat)
    sat_srv = S.Server(96 << 30, steps_per_iter=16)
    t_served = sat_srv.run(sat, time_limit=300.0, log=log)
    capacity = work / t_served
    t0 = time.perf_counter()
    for r in S.request_stream(calib, 1.0, seed=502):
        S.serve_alone(r)
    t_one = time.perf_counter() - t0
    log(f"[serve] capacity {capacity:.3e} cell-updates/s, one at a time {work / t_one:.3e}")
    rate = 0.8 * capacity / S.mean_work()
    reqs = S.request_stream(count, rate, seed=501)
    srv = S.Server(96 << 30, steps_per_iter=16)
    wall = srv.run(reqs, time_limit=600.0, log=log)
    rep = S.latency_report(reqs)
    # host time per phase of the serving loop; "wait" is the status read,
    # which waits for the device
    rep["host_phase_s"] = {k: round(v, 3) for k, v in srv.phase_s.items()}
    rep["wall_s"] = wall
    rep["offered_rate_per_s"] = rate
    rep["offered_load_frac"] = 0.8
    rep["requests"] = count
    rep["calibration_requests"] = calib
    rep["iterations"] = srv.iterations
    rep["saturated_cell_updates_per_s"] = capacity
    rep["one_at_a_time_cell_updates_per_s"] = work / t_one
    rep["saturated_speedup"] = t_one / t_served
    rep["saturated_host_phase_s"] = {k: round(v, 3) for k, v in sat_srv.phase_s.items()}
    rep["saturated_wall_s"] = t_served
    return rep


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_worker(seed, n, steps, start_at):
    """One single-threaded oracle run (bench.py --cpu-worker): a seeded n^3
    Mach-1 random field, `steps` Heun steps from its CFL dt, started at the
    wall-clock time start_at so that concurrent workers overlap."""
    import oracle as O
    from paper_2501_02317_amd import workloads as wl
    c = wl.turbulence_3d(n=n, mach=1.0, seed=seed, steps=steps, cfl=0.3)
    m = O.Mesh(c.n, c.gamma, c.lo, c.hi, c.bc)
    U = O.prim_to_cons(m, c.W)
    time.sleep(max(0.0, start_at - time.time()))
    t0 = time.time()
    _, _, done, _ = O.run(m, U, c.cfl, max_steps=steps)
    t1 = time.time()
    print(json.dumps({"cells": c.ncells, "steps": done, "start": t0, "end": t1}), flush=True)


def cpu_workers(count, n, steps, seed0, delay=15.0):
    """count concurrent single-thread oracle processes; returns
    (cell-updates/s over the common window, per-worker records)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    start_at = time.time() + delay + 0.5 * count  # after every worker has built its state
    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker",
                               f"{seed0 + i},{n},{steps},{start_at}"], env=env, stdout=subprocess.PIPE,
                              text=True) for i in range(count)]
    recs = []
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle worker failed ({p.returncode})")
        recs.append(json.loads(out.strip().splitlines()[-1]))
    work = sum(r["cells"] * r["steps"] for r in recs)
    wall = max(r["end"] for r in recs) - min(r["start"] for r in recs)
    return work / wall, recs


def cpu_baseline(case):
    """The FP64 oracle on the host cores, as it stands (not tuned): one
    thread on a 128^3 mesh; one single-thread process per core of this
    process's CPU set (at most 16, the box's share), each on its own seeded
    128^3 mesh, run at once (the value); and the OpenMP build over those
    cores for one Heun step of the 256^3 benchmark state."""
    import oracle as O
    ncores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nproc = min(ncores, 16)
    single, _ = cpu_workers(1, 128, 2, 7000)
    allc, recs = cpu_workers(nproc, 128, 1, 7100)
    m = O.Mesh(case.n, case.gamma, case.lo, case.hi, case.bc)
    U = O.prim_to_cons(m, case.W)
    dt = O.cfl_dt(m, U, case.cfl)
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    t0 = time.perf_counter()
    O.heun_step(m, U, dt)
    el = time.perf_counter() - t0
    return {"value": allc, "unit": "cell-updates/s", "cores": nproc, "kind": "oracle",
            "sample": f"{nproc} concurrent single-thread oracle processes, each one FP64 Heun step of its own "
                      f"seeded 128^3 Mach-1 state ({sum(r['cells'] * r['steps'] for r in recs):.3g} "
                      f"cell-updates in the common window)",
            "single_core": single,
            "openmp": {"value": case.ncells / el, "threads": threads,
                       "sample": f"one Heun step of the {'x'.join(map(str, case.n))} Mach-2 state, {el:.1f} s"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity_cores": ncores}


def traffic_record(precision, tiles):
    """HBM bytes per step (stage-1 plus stage-2 launch) from the committed
    rocprofv3 counter summary, when it was taken from the current kernel
    source with the same stage tiles."""
    path = os.path.join(ROOT, "profiles", "stage_kernel_256cubed_traffic.md")
    src = os.path.join(ROOT, "paper_2501_02317_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    m = re.search(r"```json\n(.*?)\n```", open(path).read(), re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    entry = rec.get("by_precision", {}).get(precision)
    if rec.get("kernels_sha256") != digest or not entry or entry.get("tiles") != tiles:
        return None
    return entry.get("bytes_per_step_pair")


def main():
    args = parse()
    if args.cpu_worker:
        seed, n, steps, start_at = args.cpu_worker.split(",")
        cpu_worker(int(seed), int(n), int(steps), float(start_at))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU path is a design only)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    from paper_2501_02317_amd import hydro as H
    from paper_2501_02317_amd import workloads as wl
    if args.smr_only:
        # diagnostic mode for kernel traces of the refined-mesh leg alone
        print(json.dumps({"smr": run_smr(H, wl, args.steps, args.warmup)}), flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serving": run_serving(args.serve_count, args.serve_calib)}), flush=True)
        return

    case = wl.turbulence_3d(n=args.n, mach=2.0, seed=301, steps=100, cfl=0.3)
    print(f"[bench] workload {case.name} steps {args.steps} warmup {args.warmup}", file=sys.stderr,
          flush=True)
    res = {}
    for name, prec in (("mixed", H.MIXED), ("fp64", H.FP64)):
        if args.precision not in ("both", name):
            continue
        fixed = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
        res[name] = run_precision(H, case, prec, args.steps, args.warmup, fixed, not args.no_tune, host_io=True)
        print(f"[bench] {name}: {res[name]['rate']:.3e} cell-updates/s, "
              f"{res[name]['ms_per_step']:.3f} ms/step, stage kernel {res[name]['achieved_gbs']:.0f} GB/s",
              file=sys.stderr, flush=True)
    head = res.get("mixed") or res.get("fp64")
    head_name = "mixed" if "mixed" in res else "fp64"
    nc = case.ndim + 2
    cells = case.ncells
    alg_per_launch_pair = 5 * nc * 8 * cells
    traffic = traffic_record(head_name, head["tiles"])
    out = {
        "metric": METRIC,
        "value": head["rate"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32 reconstruction+riemann / fp64 update" if head_name == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"3-D periodic ideal gas gamma=5/3, {args.n}^3, seeded Mach-2 "
                               f"random field, CFL 0.3, PLM(minmod)+HLLC+Heun, device dt",
                   "n": list(case.n), "precision": head_name, "steps_per_run": args.steps},
        "roofline": {"bound": "hbm", "achieved": head["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": head["frac"],
                     "traffic": traffic,
                     "kernel": "stage_kernel (stage 1 + stage 2 launches)",
                     "alg_bytes_per_step": alg_per_launch_pair,
                     "stage_ms": head["stage_ms"]},
        "by_precision": {k: {"value": v["rate"], "ms_per_step": v["ms_per_step"],
                             "roofline_frac": v["frac"], "step_roofline_frac": v["step_frac"],
                             "stage_ms": v["stage_ms"], "achieved_gbs": v["achieved_gbs"],
                             "tiles": v["tiles"], "untimed_steps": v["untimed_steps"],
                             "host_inclusive": v["host_inclusive"]}
                         for k, v in res.items()},
    }
    if "mixed" in res and "fp64" in res:
        out["mixed_over_fp64"] = res["mixed"]["rate"] / res["fp64"]["rate"]
    if not args.no_vl2:
        # the memory-optimised van Leer integrator on the same workload
        vl = {}
        for name, prec in (("mixed", H.MIXED), ("fp64", H.FP64)):
            if args.precision not in ("both", name):
                continue
            r = run_precision(H, case, prec, args.steps, args.warmup, None, not args.no_tune, integrator=1)
            vl[name] = {"value": r["rate"], "ms_per_step": r["ms_per_step"], "stage_ms": r["stage_ms"],
                        "achieved_gbs": r["achieved_gbs"], "roofline_frac": r["frac"],
                        "alg_bytes_per_cell_update": bytes_per_update(case.ndim, prec, 1), "tiles": r["tiles"]}
            print(f"[bench] vl2 {name}: {r['rate']:.3e} cell-updates/s, {r['ms_per_step']:.3f} ms/step, "
                  f"stage kernels {r['achieved_gbs']:.0f} GB/s", file=sys.stderr, flush=True)
        out["vl2"] = vl
    if not args.no_blocks and "mixed" in res:
        # the same mesh split into blocks that read their ghosts from each
        # other: one launch per stage over every block, or each block's
        # stages on their own streams
        bl = {"unsplit": res["mixed"]["rate"]}
        for blocks in ((2, 2, 2), (4, 4, 4)):
            key = "x".join(map(str, blocks))
            bl[key] = {}
            for mode in ("fused", "streams"):
                r = run_precision(H, case, H.MIXED, args.steps, args.warmup, None, not args.no_tune,
                                  blocks=blocks, streams=mode == "streams")
                bl[key][mode] = {"value": r["rate"], "ms_per_step": r["ms_per_step"], "tiles": r["tiles"]}
                print(f"[bench] blocks {key} {mode}: {r['rate']:.3e} cell-updates/s, "
                      f"{r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        out["blocks"] = {"precision": "mixed", "integrator": "heun", **bl}
    if not args.no_smr and "mixed" in res:
        out["smr"] = run_smr(H, wl, args.steps, args.warmup)
        print(f"[bench] smr: {out['smr']['value']:.3e} cell-updates/s ({out['smr']['leaves']} leaves), "
              f"split mesh {out['smr']['split_value']:.3e}", file=sys.stderr, flush=True)
    if not args.no_paper_grid and "mixed" in res:
        out["paper_grid"] = run_paper_grid(H, wl, args.steps, args.warmup, not args.no_tune)
    if not args.no_batch:
        print("[bench] batched 2-D workload ...", file=sys.stderr, flush=True)
        out["batch"] = run_batch(H, wl, args.batch_count, 300, H.MIXED)
        print(f"[bench] batch: {out['batch']['batched_cell_updates_per_s']:.3e} vs one-at-a-time "
              f"{out['batch']['one_at_a_time_cell_updates_per_s']:.3e}", file=sys.stderr, flush=True)
    if not args.no_serve:
        print("[bench] serving ...", file=sys.stderr, flush=True)
        out["serving"] = run_serving(args.serve_count, args.serve_calib)
        print(f"[bench] serving: p50 {out['serving']['p50_s']:.3f} s p99 {out['serving']['p99_s']:.3f} s",
              file=sys.stderr, flush=True)
    if not args.no_cpu:
        print("[bench] oracle cpu baseline ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
