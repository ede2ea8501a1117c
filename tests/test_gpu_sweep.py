"""The |S| x B trade-off sweep (sweep.py) run end to end on a small grid of
the n=16384 workload: one JSON line per (|S|, B) point; at B = M-1 the
predictive mean is the full GP's whatever the support set; raising B from 0
(PIC) towards M-1 moves the mean towards the full GP's; every point reports a
time, an RMSE and an LML."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sweep_small_grid(lib, tmp_path):
    out = tmp_path / "sweep.jsonl"
    print("case sweep fgp |S| in {16, 256}, B in {0, 2, 15}", flush=True)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "sweep.py"), "--workloads", "fgp", "--sizes", "16,256",
                        "--orders", "0,2,15", "--out", str(out)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    rows = [json.loads(l) for l in out.read_text().splitlines()]
    assert len(rows) == 6
    for row in rows:
        print(f"  |S|={row['s']} B={row['B']}: {row['fit_predict_s']:.3f} s, RMSE {row['rmse']:.4f}, "
              f"vs full GP {row['mean_rel_to_fgp']:.2e}", flush=True)
        assert row["fit_predict_s"] > 0 and row["rmse"] > 0 and row["lml"] < 0
    by = {(row["s"], row["B"]): row for row in rows}
    for s in (16, 256):
        assert by[(s, 15)]["mean_rel_to_fgp"] < 1e-10
        assert by[(s, 2)]["mean_rel_to_fgp"] < by[(s, 0)]["mean_rel_to_fgp"]
