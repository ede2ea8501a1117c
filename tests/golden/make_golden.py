"""Write the stored expected values for the full-size parity tests.

Calls only the CPU oracle (oracle/) on inputs drawn by synth/; nothing here
touches the GPU library.  For each prediction workload it stores a digest of
the drawn inputs (so a test can tell that it regenerated the same problem) and
the log marginal likelihood in <name>_oracle.json, and the complete predictive
mean and variance vectors in <name>_oracle.npz.  For the likelihood-gradient
workload (cfg3: n=131072, d=8, M=128, B=2, |S|=512, no test set) it stores the
log marginal likelihood and its gradient in (log l, log sigma_s^2,
log sigma_n^2) from the oracle's adjoint.

Workloads: cfg0 (n=2048), cfg1 (n=65536), cfg2 (n=524288, the benchmark
shape), cfg3 (gradient), and two extremes of the |S| x B sweep at n=16384:
sweep_B15 (M=16, B=15 = M-1: one window of all 16384 points, |S|=1024) and
sweep_S2048 (|S|=2048, B=2).

    python tests/golden/make_golden.py cfg0 cfg1 cfg2 cfg3 sweep_B15 sweep_S2048
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

PREDICT = {"cfg0": lambda: synth.make_config(0), "cfg1": lambda: synth.make_config(1),
           "cfg2": lambda: synth.make_config(2),
           "sweep_B15": lambda: synth.make_sweep16k(1024, 15),
           "sweep_S2048": lambda: synth.make_sweep16k(2048, 2)}


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
    t0 = time.time()
    p = PREDICT[name]()
    print(f"{name}: inputs drawn in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    r = olma.fit_predict(p)
    dt = time.time() - t0
    print(f"{name}: oracle fit+predict in {dt:.1f} s", flush=True)
    out = {
        "workload": name,
        "source": "oracle.lma.fit_predict (float64, whitened windows)",
        "digest": p.digest(),
        "lml": r["lml"],
        "mean_norm": float(np.linalg.norm(r["mean"])),
        "var_norm": float(np.linalg.norm(r["var"])),
        "rmse": float(np.sqrt(np.mean((r["mean"] - p.y_u) ** 2))) if p.y_u is not None else None,
        "oracle_seconds": dt,
        "oracle_threads": os.cpu_count(),
    }
    path = os.path.join(HERE, f"{name}_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f)
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), mean=r["mean"], var=r["var"])
    print(f"wrote {path} and the .npz vectors", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["cfg0", "cfg1"]:
        make(nm)
