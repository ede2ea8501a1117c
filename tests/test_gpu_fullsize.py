"""Parity at the full workload sizes, against stored oracle values.

The expected values were written by tests/golden/make_golden.py, which calls
only the CPU oracle.  The inputs are regenerated here from the same seeds; the
stored digest checks that they are the same problem.  Outputs compared: the
log marginal likelihood, and the predictive mean and variance at a fixed sample
of 1024 test points (plus the norms of the full vectors), in the launch
configuration the benchmark times."""
import json
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"fp64": 1e-9, "mixed": 1e-4}


def load_golden(name):
    path = os.path.join(HERE, "golden", f"{name}_oracle.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


def check_digest(p, gold):
    dg = p.digest()
    for k, v in gold["digest"].items():
        if isinstance(v, float):
            assert abs(dg[k] - v) <= 1e-9 * max(1.0, abs(v)), k
        else:
            assert dg[k] == v, k


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("name,k", [("cfg0", 0), ("cfg1", 1), ("cfg2", 2)])
def test_fullsize_against_stored_oracle(lib, name, k):
    gold = load_golden(name)
    p = synth.make_config(k)
    check_digest(p, gold)
    idx = np.asarray(gold["sample_index"])
    for prec in ("fp64", "mixed"):
        print(f"case {name} n={p.n} {prec}", flush=True)
        st = lib.fit_problem(p, precision=prec)
        mean, var = st.predict(p.U, p.u_block_ptr)
        lml = st.lml()
        st.free()
        mean, var = mean.cpu().numpy(), var.cpu().numpy()
        em = rel(mean[idx], gold["mean"])
        ev = rel(var[idx], gold["var"])
        el = abs(lml - gold["lml"]) / abs(gold["lml"])
        en = abs(np.linalg.norm(mean) - gold["mean_norm"]) / gold["mean_norm"]
        evn = abs(np.linalg.norm(var) - gold["var_norm"]) / gold["var_norm"]
        print(f"  rel err mean {em:.2e} var {ev:.2e} lml {el:.2e} |mean| {en:.2e} |var| {evn:.2e}", flush=True)
        tol = TOL[prec]
        assert max(em, ev, el, en, evn) <= tol
