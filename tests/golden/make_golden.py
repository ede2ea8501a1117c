"""Write the stored expected values for the full-size parity tests.

Calls only the CPU oracle (oracle/) on inputs drawn by synth/; nothing here
touches the GPU library.  For each workload it stores a digest of the drawn
inputs (so a test can tell that it regenerated the same problem), the log
marginal likelihood, and the predictive mean and variance at a fixed sample
of test points.

    python tests/golden/make_golden.py cfg1 cfg2
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import lma as olma  # noqa: E402

SAMPLE = 1024


def sample_index(n_u, k=SAMPLE):
    rng = np.random.default_rng(20150125)
    return np.sort(rng.choice(n_u, size=min(k, n_u), replace=False))


def make(name):
    k = {"cfg0": 0, "cfg1": 1, "cfg2": 2}[name]
    t0 = time.time()
    p = synth.make_config(k)
    print(f"{name}: inputs drawn in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    r = olma.fit_predict(p)
    print(f"{name}: oracle fit+predict in {time.time() - t0:.1f} s", flush=True)
    idx = sample_index(p.n_u)
    out = {
        "workload": name,
        "source": "oracle.lma.fit_predict (float64, whitened windows)",
        "digest": p.digest(),
        "lml": r["lml"],
        "sample_index": idx.tolist(),
        "mean": r["mean"][idx].tolist(),
        "var": r["var"][idx].tolist(),
        "mean_norm": float(np.linalg.norm(r["mean"])),
        "var_norm": float(np.linalg.norm(r["var"])),
        "rmse": float(np.sqrt(np.mean((r["mean"] - p.y_u) ** 2))) if p.y_u is not None else None,
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["cfg1", "cfg2"]:
        make(nm)
