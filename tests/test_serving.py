"""Serving: host logic on the CPU; on the GPU, every request's result is the
same in the mix as alone, and admission respects the memory budget."""
import numpy as np
import pytest

from gpu_util import bitwise_equal, say


def test_arena_first_fit_and_merge():
    from paper_2501_02317_amd.serving import Arena
    a = Arena(10_240)
    o1 = a.alloc(1000)
    o2 = a.alloc(3000)
    assert (o1, o2) == (0, 1024)
    assert a.alloc(7200) is None
    a.release(o1)
    o3 = a.alloc(500)
    assert o3 == 0
    a.release(o2)
    a.release(o3)
    assert a.free == [(0, 10_240)] and a.in_use == 0
    assert a.alloc(10_240) == 0


def test_request_stream_is_seeded_and_in_range():
    from paper_2501_02317_amd.serving import request_stream
    r1 = request_stream(200, 20.0, seed=7)
    r2 = request_stream(200, 20.0, seed=7)
    assert [(r.n, r.steps, r.seed) for r in r1] == [(r.n, r.steps, r.seed) for r in r2]
    arr = np.array([r.arrival for r in r1])
    assert np.all(np.diff(arr) > 0)
    assert 5.0 < arr[-1] < 20.0                      # about count / rate
    for r in r1:
        if r.ndim == 2:
            assert 64 <= r.n <= 1024 and r.n % 32 == 0
        else:
            assert 32 <= r.n <= 160 and r.n % 16 == 0
        assert 100 <= r.steps <= 2000 and 0.5 <= r.mach <= 3.0
    assert 0.3 < np.mean([r.ndim == 2 for r in r1]) < 0.7


def test_latency_report():
    from paper_2501_02317_amd.serving import Request, latency_report
    rs = []
    for i in range(100):
        r = Request(i, 2, 64, 10, 1.0, 1.4, 1, i, arrival=float(i))
        r.admitted = r.arrival + 0.5
        r.finished = r.arrival + 1.0 + (i % 10) * 0.1
        rs.append(r)
    rep = latency_report(rs, warmup_frac=0.0)
    assert rep["completed"] == 100 and rep["failed"] == 0
    assert abs(rep["p50_s"] - 1.45) < 0.06 and rep["p99_s"] <= 1.9 + 1e-9
    assert abs(rep["mean_queue_s"] - 0.5) < 1e-12


@pytest.mark.gpu
def test_results_in_the_mix_equal_alone():
    import torch
    assert torch.cuda.is_available()
    from paper_2501_02317_amd import serving as S
    reqs = S.request_stream(32, 800.0, seed=11, n2=(64, 160), n3=(32, 48), steps=(10, 40))
    say("serving mix", len(reqs))
    srv = S.Server(2 << 30, steps_per_iter=8, keep_results=[r.rid for r in reqs])
    srv.run(reqs)
    assert srv.iterations > 1
    for r in reqs:
        assert r.finished is not None and not r.failed
        say("alone", r.rid, r.ndim, r.n, r.steps, r.precision)
        assert bitwise_equal(S.serve_alone(r), r.result), r.rid


@pytest.mark.gpu
def test_admission_respects_memory_budget():
    import torch
    assert torch.cuda.is_available()
    from paper_2501_02317_amd import serving as S
    reqs = S.request_stream(10, 1000.0, seed=12, n2=(128, 128), n3=(48, 48), steps=(10, 20))
    for r in reqs:
        r.arrival = 0.0                                      # all waiting at the start
    fp = [S.footprint(r) for r in reqs]
    # the largest request fits alone and the first two fit together, but not all ten
    budget = max(max(fp), fp[0] + fp[1]) + 4096
    assert budget < sum(fp)
    say("admission budget", budget)
    srv = S.Server(budget, steps_per_iter=8)
    srv.run(reqs)
    assert all(r.finished is not None and not r.failed for r in reqs)
    # at every admission, the requests resident then fit the budget together
    resident_at = []
    for r in reqs:
        resident = [q for q in reqs if q.admitted <= r.admitted < q.finished]
        assert sum(S.footprint(q) for q in resident) <= budget
        resident_at.append(len(resident))
    # requests ran concurrently (both first requests were admitted at once),
    # and the budget made some wait for memory to free up
    assert max(resident_at) >= 2
    assert any(q.admitted >= p.finished for p in reqs for q in reqs if q is not p)


# The one request of the 2000-request serving run that was retired as failed:
# 3-D 64^3, Mach 3.0, gamma 5/3, FP64, this seed (its spec as the bench's
# serving record lists it).  Its flow expands until the pressure reaches zero.
FAILED_SPEC = dict(ndim=3, n=64, mach=2.9989993467151863, gamma=5.0 / 3.0, seed=1069413739)


def failed_request_state():
    from paper_2501_02317_amd import workloads as wl
    s = FAILED_SPEC
    W = wl.random_field_device(s["ndim"], s["n"], s["mach"], s["gamma"], s["seed"], kmax=min(16, s["n"] // 8),
                               device="cpu")
    return W.numpy()


def test_failed_request_is_nonphysical_in_the_oracle_too():
    """The method has no density or pressure floors: the FP64 oracle takes
    the failed request's state through 52 steps and meets a non-physical cell
    in step 53, as the GPU did (it retired the request in the iteration that
    ends with step 64)."""
    import oracle as O
    W = failed_request_state()
    m = O.Mesh((64, 64, 64), FAILED_SPEC["gamma"], (0.0,) * 3, (1.0,) * 3, ((0, 0),) * 3)
    U, t, s, _ = O.run(m, O.prim_to_cons(m, W), 0.3, max_steps=52)
    assert s == 52
    assert O.cons_to_prim(m, U)[4].min() > 0.0
    with pytest.raises(O.OracleError, match="non-physical"):
        O.run(m, U, 0.3, max_steps=1, t0=t)


@pytest.mark.gpu
def test_failed_request_fails_in_the_same_step_on_the_gpu():
    """The FP64 GPU path on the failed request alone: after 52 steps it
    matches the oracle and is physical; step 53 raises the non-physical flag."""
    import torch
    assert torch.cuda.is_available()
    import oracle as O
    from paper_2501_02317_amd import hydro as H
    from gpu_util import rel_l1
    W = failed_request_state()
    m = O.Mesh((64, 64, 64), FAILED_SPEC["gamma"], (0.0,) * 3, (1.0,) * 3, ((0, 0),) * 3)
    U_o, t_o, s_o, _ = O.run(m, O.prim_to_cons(m, W), 0.3, max_steps=52)
    say("failed request alone", FAILED_SPEC)
    h = H.Hydro((64, 64, 64), FAILED_SPEC["gamma"], 0.3, precision=H.FP64)
    h.set_primitive(W)
    h.step_auto(52)
    U = h.get_state()
    assert h.steps_done() == 52
    assert np.all(rel_l1(U, U_o) <= 1e-12)
    assert h.time() == pytest.approx(t_o, rel=1e-13)  # a blocking call: no flag yet
    h.step_auto(1)
    with pytest.raises(H.HydroError) as e:
        h.time()
    assert e.value.status == H.E_NONPHYSICAL
    h.close()
