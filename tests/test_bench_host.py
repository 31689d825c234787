"""Host-side parts of bench.py: the one-GPU refusal, the algorithmic bytes
the roofline is priced on (the reads and writes each stage must make, Sec.
3.3), and the traffic record's key.  CPU only."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("ndim,nc", [(1, 3), (2, 4), (3, 5)])
def test_heun_bytes(ndim, nc):
    # stage 1: read U^n, write U1; stage 2: read U1 and U^n, write U^{n+1}; FP64
    assert bench.stage_bytes(ndim, 0, 0) == (2 * nc * 8, 3 * nc * 8)
    assert bench.stage_bytes(ndim, 1, 0) == bench.stage_bytes(ndim, 0, 0)
    assert bench.bytes_per_update(ndim) == 5 * nc * 8


def test_van_leer_bytes():
    # predictor: read U^n (FP64), write the predicted primitive state in the
    # compute type; corrector: read it and U^n, write U^{n+1}
    assert bench.bytes_per_update(3, 1, 1) == 5 * (8 + 4) + 5 * (4 + 16) == 160
    assert bench.bytes_per_update(3, 0, 1) == 5 * (8 + 8) + 5 * (8 + 16) == 200


def test_traffic_record_is_keyed_to_tiles_and_source():
    path = os.path.join(ROOT, "profiles", "stage_kernel_256cubed_traffic.md")
    rec = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
    for prec, entry in rec["by_precision"].items():
        assert bench.traffic_record(prec, [[1, 1, 1], [1, 1, 1]]) is None
        got = bench.traffic_record(prec, entry["tiles"])
        assert got is None or got == entry["bytes_per_step_pair"]


def test_concurrent_oracle_workers_report_a_common_window():
    # two single-thread oracle processes on small seeded meshes: the rate is
    # their summed cell-updates over the window from the first start to the
    # last end, and every worker did the steps it was asked for
    rate, recs = bench.cpu_workers(2, 16, 2, 9000, delay=3.0)
    assert len(recs) == 2
    assert all(r["cells"] == 16 ** 3 and r["steps"] == 2 and r["end"] > r["start"] for r in recs)
    wall = max(r["end"] for r in recs) - min(r["start"] for r in recs)
    assert rate == pytest.approx(2 * 2 * 16 ** 3 / wall)
