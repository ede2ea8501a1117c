"""Write the stored expected values for the full-size parity tests.

Calls only the CPU oracle (oracle/) on inputs drawn by synth/; nothing here
touches the GPU library.  For each workload it stores a digest of the drawn
inputs (so a test can tell that it regenerated the same problem), the log
marginal likelihood, and the predictive mean and variance at a fixed sample
of test points.  For the likelihood-gradient workload (cfg3: n=131072, d=8,
M=128, B=2, |S|=512, no test set) it stores the log marginal likelihood and
its gradient in (log l, log sigma_s^2, log sigma_n^2) from the oracle's adjoint.

    python tests/golden/make_golden.py cfg1 cfg2 cfg3
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


def make_grad(name, k):
    t0 = time.time()
    p = synth.make_config(k)
    print(f"{name}: inputs drawn in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    lml, grad = olma.lml_grad(p)
    print(f"{name}: oracle log marginal likelihood and gradient in {time.time() - t0:.1f} s", flush=True)
    out = {
        "workload": name,
        "source": "oracle.lma.lml_grad (float64, adjoint over whitened windows)",
        "digest": p.digest(),
        "lml": lml,
        "grad": [float(v) for v in grad],
        "log_hyp": [float(v) for v in p.log_hyp],
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}", flush=True)


def make(name):
    if name == "cfg3":
        return make_grad(name, 3)
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
