"""CPU checks of the benchmark driver: it refuses more than one GPU before
touching a device, and the committed counter summaries it reads are
self-consistent (bytes per launch from the scaled FETCH/WRITE counters,
algorithmic bytes 16 per cell of the workload)."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))),
                         ids=os.path.basename)
def test_traffic_summaries_are_consistent(path):
    import shellgen
    import bench
    rec = json.load(open(path))
    sh = shellgen.workload(rec["workload"])
    assert rec["algorithmic_bytes_per_launch"] == 16 * sh.n
    counted = (rec["fetch_kib_per_launch"] / rec["fetch_scale"] +
               rec["write_kib_per_launch"] / rec["write_scale"]) * 1024
    # (the stored scales and counters are rounded)
    assert abs(counted - rec["bytes_per_launch"]) <= 1e-4 * counted
    assert os.path.basename(path) == f"traffic_{rec['class']}_{rec['workload']}.json"
    got, note = bench.measured_traffic(rec["workload"], rec["class"])
    # either the sources still match (the summary's bytes) or bench says why not
    assert got == rec["bytes_per_launch"] or (got is None and "changed" in note)
