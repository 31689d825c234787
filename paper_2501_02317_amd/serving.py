"""Continuous-batching server for hydro simulations on one GPU.

Requests arrive over time (a seeded Poisson stream), wait in a FIFO queue,
and are admitted as soon as their device footprint fits the HBM budget and
a slot is free.  Every resident request keeps its state on the device; each
server iteration advances all of them together with one batched multi-step
call (hydro_batch_step), every request at its own CFL dt and up to its own
step count (a run limit held on the device).  Requests that reached their
step count are retired between iterations: their latency (completion minus
scheduled arrival) is recorded, their results optionally copied out, and
their memory returned to the pool; newly arrived requests join the next
iteration.  A request whose state turned non-physical is retired as failed.

Requests are compact specs; the initial state is generated on the device
from the spec's seed at admission (workloads.random_field_device), so
latency includes setting a request up.
"""
import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import hydro as H
from . import workloads as wl


@dataclass
class Request:
    rid: int
    ndim: int
    n: int
    steps: int
    mach: float
    gamma: float
    precision: int
    seed: int
    arrival: float                 # scheduled arrival, seconds after start
    admitted: float = None
    finished: float = None
    failed: bool = False
    steps_done: int = 0            # steps completed when the request was retired
    result: np.ndarray = None

    @property
    def cells(self):
        return self.n ** self.ndim

    @property
    def cfl(self):
        return 0.3 if self.ndim == 3 else 0.4

    @property
    def kmax(self):
        return min(16, self.n // 8)


def request_stream(count, rate, seed=501, n2=(64, 1024), n3=(32, 160), steps=(100, 2000)):
    """Seeded Poisson stream: 2-D or 3-D at 50/50, n log-uniform (2-D:
    multiple of 32; 3-D: multiple of 16), steps log-uniform, Mach U[0.5, 3],
    gamma from {1.4, 5/3}, FP64 or mixed at 50/50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        ndim = 2 if rng.random() < 0.5 else 3
        lo, hi, q = (n2[0], n2[1], 32) if ndim == 2 else (n3[0], n3[1], 16)
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))) / q) * q)
        n = max(lo, min(hi, n))
        k = int(round(math.exp(rng.uniform(math.log(steps[0]), math.log(steps[1])))))
        mach = float(rng.uniform(0.5, 3.0))
        gamma = 1.4 if rng.random() < 0.5 else 5.0 / 3.0
        prec = H.FP64 if rng.random() < 0.5 else H.MIXED
        out.append(Request(i, ndim, n, k, mach, gamma, prec, int(rng.integers(1 << 31)), t))
    return out


def mean_work(n2=(64, 1024), n3=(32, 160), steps=(100, 2000)):
    """Expected cells x steps of a request of request_stream (log-uniform moments)."""
    def moment(lo, hi, p):
        return (hi ** p - lo ** p) / (p * math.log(hi / lo))
    cells = 0.5 * moment(*n2, 2) + 0.5 * moment(*n3, 3)
    return cells * moment(*steps, 1)


class Arena:
    """First-fit allocator of 256-byte-aligned ranges of one device buffer."""

    ALIGN = 256

    def __init__(self, capacity):
        self.capacity = capacity
        self.free = [(0, capacity)]      # sorted (offset, size)
        self.used = {}

    def alloc(self, nbytes):
        need = (nbytes + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + need, size - need)
                self.used[off] = need
                return off
        return None

    def release(self, off):
        size = self.used.pop(off)
        self.free.append((off, size))
        self.free.sort()
        merged = []
        for o, s in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + s)
            else:
                merged.append((o, s))
        self.free = merged

    @property
    def in_use(self):
        return sum(self.used.values())


def footprint(req):
    nn = (req.n,) * req.ndim
    cfg = H.make_config(nn, req.gamma, req.cfl, req.precision)
    ic = (req.ndim + 2) * req.cells * 8          # device initial state, freed after upload
    return H.workspace_bytes(cfg) + ic


class Server:
    def __init__(self, hbm_bytes, steps_per_iter=16, max_members=256, keep_results=(), device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.pool = torch.empty(hbm_bytes, dtype=torch.uint8, device=self.device)
        self.arena = Arena(hbm_bytes)
        self.stream = torch.cuda.Stream(device=self.device)
        self.setup_stream = torch.cuda.Stream(device=self.device)
        self.K = steps_per_iter
        self.max_members = max_members
        # host time for request set-up per iteration: short while the device
        # is idle, longer while it steps the resident requests (set-up enqueues
        # its work without waiting for the stream)
        self.idle_admit_s = 0.02
        self.busy_admit_s = 0.05
        self.keep = set(keep_results)
        self.iterations = 0

    def _admit(self, r, now):
        torch = self.torch
        off = self.arena.alloc(footprint(r))
        if off is None:
            return None
        nn = (r.n,) * r.ndim
        cfg = H.make_config(nn, r.gamma, r.cfl, r.precision)
        wsb = H.workspace_bytes(cfg)
        ws = self.pool[off: off + wsb]
        h = H.Hydro(nn, r.gamma, r.cfl, precision=r.precision, stream=self.stream, workspace=ws)
        # the initial state on the set-up stream, beside the steps enqueued on
        # the batch's streams; its conversion on the batch's stream waits for it
        with torch.cuda.stream(self.setup_stream):
            W = wl.random_field_device(r.ndim, r.n, r.mach, r.gamma, r.seed, kmax=r.kmax,
                                       device=self.device)
        ready = torch.cuda.Event()
        ready.record(self.setup_stream)
        self.stream.wait_event(ready)
        h.set_primitive_device(W)
        h.set_run_limit(r.steps, 0.0)
        r.admitted = now
        return {"req": r, "h": h, "off": off, "W": W}

    def run(self, requests, time_limit=None, log=None, log_every=10.0):
        """Serve requests (their arrival fields are offsets from the start).
        log: optional callable given a progress line every log_every seconds.

        One iteration: (re)build the batch when its membership changed, enqueue
        K batched steps, admit the requests that arrived meanwhile (their
        set-up is host work that overlaps the steps on the device, for at
        most busy_admit_s; their initial states are generated on a stream of
        their own beside the steps, and converted behind the steps), then
        read every member's status (the one synchronisation) and retire the
        finished ones.  Host time per phase is accumulated in self.phase_s."""
        pending = collections.deque(sorted(requests, key=lambda q: q.arrival))
        total, finished, next_log = len(pending), 0, log_every
        queue = collections.deque()
        active = []          # members of the current batch
        joining = []         # admitted, joining at the next rebuild
        batch = None
        ph = self.phase_s = collections.defaultdict(float)
        start = time.perf_counter()

        def admit(now, limit_s=None):
            # limit_s: host time after which no further request is set up in
            # this call (the device is waiting for work)
            t = time.perf_counter()
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            while queue and len(active) + len(joining) < self.max_members:
                if limit_s is not None and joining and time.perf_counter() - t > limit_s:
                    break
                m = self._admit(queue[0], now)
                if m is None:
                    break
                queue.popleft()
                joining.append(m)
            ph["admit"] += time.perf_counter() - t

        while pending or queue or active or joining:
            now = time.perf_counter() - start
            if time_limit is not None and now > time_limit:
                break
            if not active and not joining:
                # the device is idle: start it on the first requests, and set
                # up the others while it steps them
                admit(now, self.idle_admit_s)
                if not joining:
                    if pending:
                        time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - start)))
                    continue
            if joining or batch is None:
                t = time.perf_counter()
                if batch is not None:
                    batch.close()
                active.extend(joining)
                joining = []
                batch = H.Batch([m["h"] for m in active], use_graph=False)
                ph["build"] += time.perf_counter() - t
            t = time.perf_counter()
            batch.step(self.K)
            ph["enqueue"] += time.perf_counter() - t
            admit(time.perf_counter() - start, self.busy_admit_s)   # overlaps the steps
            t = time.perf_counter()
            done, steps, flags = batch.status()        # synchronises the stream
            ph["wait"] += time.perf_counter() - t
            self.iterations += 1
            t = time.perf_counter()
            now = time.perf_counter() - start
            keep = []
            retired = False
            for m, d, f, k in zip(active, done, flags, steps):
                m["W"] = None                           # upload has completed
                if d or f:
                    r = m["req"]
                    r.finished = now
                    finished += 1
                    r.failed = bool(f)
                    r.steps_done = int(k)
                    if r.rid in self.keep:
                        r.result = m["h"].get_state()
                    m["h"].close()
                    self.arena.release(m["off"])
                    retired = True
                else:
                    keep.append(m)
            active = keep
            if retired:
                if batch is not None:
                    batch.close()
                batch = None                            # rebuilt at the next iteration
            for m in joining:
                m["W"] = None
            ph["retire"] += time.perf_counter() - t
            if log is not None and now >= next_log:
                log(f"[serve] {now:.0f} s: {finished}/{total} finished, {len(active)} resident, "
                    f"{len(queue)} queued, {self.iterations} iterations")
                next_log = now + log_every
        if batch is not None:
            batch.close()
        for m in active + joining:
            m["h"].close()
            self.arena.release(m["off"])
        return time.perf_counter() - start


def latency_report(requests, warmup_frac=0.05):
    done = [r for r in requests if r.finished is not None and not r.failed]
    done.sort(key=lambda r: r.arrival)
    skip = int(len(done) * warmup_frac)
    lat = np.array([r.finished - r.arrival for r in done[skip:]])
    wait = np.array([r.admitted - r.arrival for r in done[skip:]])
    serv = np.array([r.finished - r.admitted for r in done[skip:]])
    work = sum(r.cells * r.steps for r in done)
    t0 = min(r.arrival for r in requests)
    t1 = max(r.finished for r in done) if done else t0
    return {
        "completed": len(done),
        "failed": sum(1 for r in requests if r.failed),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_queue_s": float(wait.mean()) if len(wait) else None,
        "mean_service_s": float(serv.mean()) if len(serv) else None,
        "cell_updates_per_s": work / (t1 - t0) if t1 > t0 else None,
        # the spec of every failed request (its initial state follows from
        # the spec alone), so it can be re-run on its own or by the oracle
        "failed_requests": [
            {"rid": r.rid, "ndim": r.ndim, "n": r.n, "steps": r.steps, "steps_done": r.steps_done,
             "mach": r.mach, "gamma": r.gamma, "precision": "fp64" if r.precision == H.FP64 else "mixed",
             "seed": r.seed} for r in requests if r.failed],
    }


def serve_alone(req, device="cuda"):
    """One request on its own (the reference for the mix-invariance check and
    the one-at-a-time baseline): returns the final state."""
    import torch
    nn = (req.n,) * req.ndim
    s = torch.cuda.Stream(device=device)
    h = H.Hydro(nn, req.gamma, req.cfl, precision=req.precision, stream=s)
    with torch.cuda.stream(s):
        W = wl.random_field_device(req.ndim, req.n, req.mach, req.gamma, req.seed, kmax=req.kmax,
                                   device=device)
    h.set_primitive_device(W)
    h.step_auto(req.steps)
    s.synchronize()
    U = h.get_state()
    h.close()
    return U
