"""What the trained warm-start network gains over plain optimisation from the
default start, on held-out GP-prior sets (n=65536, d=8) not used in training
or in the recorded evaluation: Adam (lr 0.05) on the LMA likelihood from both
starts; LML* = the best value either run reaches; counted: steps until
|LML - LML*| <= 1e-3 |LML*| (150 if never)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_gains_over_default_start(lib):
    from paper_1411_4510_amd.train_warmstart import evaluate_set, summarise
    from paper_1411_4510_amd.warmstart import WarmStart
    ws = WarmStart()
    rows = []
    for i in (20, 21, 22, 23):
        r = evaluate_set(i, ws, steps=150)
        print(f"  set {i}: start LML default {r['lml_default_start']:.1f} net {r['lml_net_start']:.1f}; "
              f"steps default {r['steps_default']} net {r['steps_net']} (LML* {r['lml_star']:.1f})", flush=True)
        rows.append(r)
    s = summarise(rows, 150)
    print(f"  {s}", flush=True)
    better_start = sum(r["lml_net_start"] >= r["lml_default_start"] for r in rows)
    assert better_start >= 3
    assert s["mean_steps_net"] < s["mean_steps_default"]


def test_warm_start_prediction_is_finite_and_deterministic(lib):
    from synth import gpsets
    from paper_1411_4510_amd.warmstart import WarmStart
    ws = WarmStart()
    p = gpsets.gp_set("heldout", 30)
    a, b = ws.predict(p.X, p.y), ws.predict(p.X, p.y)
    assert a.shape == (p.d + 2,) and np.all(np.isfinite(a))
    assert np.array_equal(a, b)
