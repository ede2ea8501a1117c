"""Warm-start network pipeline: labels, training, evaluation.

  python -m paper_1411_4510_amd.train_warmstart labels --count 20000 --workers 8 --out DIR
  python -m paper_1411_4510_amd.train_warmstart train --labels DIR --out params.npy
  python -m paper_1411_4510_amd.train_warmstart evaluate --params params.npy --count 100

labels:   for every training set (synth.gpsets, n=4096, d in 1..8) the
          hyperparameters that maximise its LMA likelihood (B=2, |S|=256),
          by bounded L-BFGS from the hyperparameters it was drawn with, the
          library giving the likelihood and its gradient; worker processes
          share the GPU, results are written per chunk of 100 sets (resumable).
train:    the network (lma_ds_* kernels) on the labels: masked MSE, Adam,
          minibatches of whole sets, a validation split, best parameters kept.
evaluate: on held-out sets (n=65536, d=8, M=64), LML* is the converged
          maximum: the better of two bounded L-BFGS runs (gradient tolerance
          1e-6) from the default start and from the network's start (falling
          back to the default when the network's start is worse or not
          finite).  Then Adam (lr 0.05, at most 500 steps) from each start
          until |LML - LML*| <= 1e-3 |LML*|; reported over the same sets:
          steps and wall time (network inference included), a run that never
          gets there counted at the cap (its steps and its full time).
"""
from __future__ import annotations

import argparse
import glob
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

CHUNK = 100


def log(*a):
    print(*a, flush=True)


# ---------------------------------------------------------------------------
# labels
# ---------------------------------------------------------------------------
def _label_worker(args):
    wid, chunks, out, deadline, maxiter = args
    import synth  # noqa: F401
    from synth import gpsets
    from . import LmlProblem, load
    from .hyperopt import lbfgs
    load()
    done = 0
    t0 = time.time()
    for c in chunks:
        if time.time() > deadline:
            break
        path = os.path.join(out, f"labels_{c:06d}.npz")
        if os.path.exists(path):
            continue
        rec = {k: [] for k in ("index", "d", "theta", "lml", "nfev", "success", "theta_true")}
        for i in range(c, c + CHUNK):
            p = gpsets.gp_set("train", i)
            prob = LmlProblem.from_problem(p)
            r = lbfgs(prob, p.log_hyp, maxiter=maxiter)
            th = np.zeros(p.d + 2)
            th[:] = r["theta"]
            rec["index"].append(i)
            rec["d"].append(p.d)
            rec["theta"].append(np.pad(th, (0, 10 - th.size)))
            rec["theta_true"].append(np.pad(p.log_hyp, (0, 10 - p.d - 2)))
            rec["lml"].append(r["lml"])
            rec["nfev"].append(r["nfev"])
            rec["success"].append(r["success"])
            if (i - c) % 10 == 9:
                log(f"worker {wid}: set {i} ({time.time() - t0:.0f} s)")
        tmp = path + ".tmp.npz"
        np.savez(tmp, **{k: np.asarray(v) for k, v in rec.items()})
        os.replace(tmp, path)
        done += 1
        log(f"worker {wid}: chunk {c} done ({done} chunks, {done * CHUNK / (time.time() - t0):.1f} sets/s, "
            f"mean evaluations {np.mean(rec['nfev']):.1f})")
    return done


def cmd_labels(a):
    os.makedirs(a.out, exist_ok=True)
    chunks = list(range(a.first, a.first + a.count, CHUNK))
    todo = [c for c in chunks if not os.path.exists(os.path.join(a.out, f"labels_{c:06d}.npz"))]
    log(f"{len(todo)} of {len(chunks)} chunks to label with {a.workers} workers")
    deadline = time.time() + a.time_limit
    parts = [(w, todo[w::a.workers], a.out, deadline, a.maxiter) for w in range(a.workers)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(a.workers) as pool:
        n = sum(pool.map(_label_worker, parts))
    log(f"labelled {n} chunks")


def load_labels(dirs):
    recs = []
    for d in dirs:
        for f in sorted(glob.glob(os.path.join(d, "labels_*.npz"))):
            z = np.load(f)
            recs.append({k: z[k] for k in z.files})
    out = {k: np.concatenate([r[k] for r in recs]) for k in recs[0]}
    order = np.argsort(out["index"])
    return {k: v[order] for k, v in out.items()}


def label_rows(theta, d):
    """(label row, mask row) of the network for fitted log-hyperparameters."""
    lab = np.zeros(10, dtype=np.float32)
    msk = np.zeros(10, dtype=np.float32)
    lab[:d] = theta[:d]
    lab[8], lab[9] = theta[d], theta[d + 1]
    msk[:d] = 1.0
    msk[8:] = 1.0
    return lab, msk


def _gen_xy(i):
    from synth import gpsets
    p = gpsets.gp_set("train", int(i))
    X = np.zeros((p.n, 8), dtype=np.float64)
    X[:, :p.d] = p.X
    return X, p.y, p.d


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------
def mean_label_loss(labs, msks, tr, val, batch):
    """Validation loss of predicting every output as its masked mean over the
    training sets (the reference point for the network's loss; same per-set
    masked mean square and the same full validation batches)."""
    mean = (labs[tr] * msks[tr]).sum(0) / np.maximum(msks[tr].sum(0), 1.0)
    tot, cnt = 0.0, 0
    for s in range(0, len(val) - batch + 1, batch):
        v = val[s:s + batch]
        r = (mean[None, :] - labs[v]) * msks[v]
        tot += float(np.sum(np.sum(r * r, 1) / np.sum(msks[v], 1)))
        cnt += batch
    return tot / max(cnt, 1)


def cmd_train(a):
    import torch
    from .warmstart import Network, he_init
    L = load_labels(a.labels)
    ok = np.isfinite(L["lml"]) & np.all(np.isfinite(L["theta"]), axis=1)
    idx, dims, theta = L["index"][ok], L["d"][ok], L["theta"][ok]
    n_sets = len(idx)
    log(f"{n_sets} labelled sets ({int((~ok).sum())} fits dropped)")
    rng = np.random.default_rng(a.seed)
    perm = rng.permutation(n_sets)
    nval = min(a.val, n_sets // 10)
    val, tr = perm[:nval], perm[nval:]
    n = 4096
    feats = torch.empty((n_sets, n, 17), dtype=torch.float32, device="cuda")
    net = Network(max_rows=a.batch * n, max_sets=a.batch)
    t0 = time.time()
    ctx = mp.get_context("spawn")
    with ctx.Pool(a.workers) as pool:
        for k, (X, y, d) in enumerate(pool.imap(_gen_xy, idx, chunksize=32)):
            net.features(X[:, :d], y, out=feats[k])
            if k % 2000 == 0:
                log(f"features {k}/{n_sets} ({time.time() - t0:.0f} s)")
    labs = np.zeros((n_sets, 10), dtype=np.float32)
    msks = np.zeros((n_sets, 10), dtype=np.float32)
    for k in range(n_sets):
        labs[k], msks[k] = label_rows(theta[k], int(dims[k]))
    base_loss = mean_label_loss(labs, msks, tr, val, a.batch)
    log(f"mean-label validation loss {base_loss:.4f}")
    labs_d = torch.as_tensor(labs, device="cuda")
    msks_d = torch.as_tensor(msks, device="cuda")
    net.set_params(he_init(a.seed))
    ptr = np.arange(a.batch + 1, dtype=np.int64) * n
    sn = np.full(a.batch, n, dtype=np.int64)

    def val_loss():
        tot, cnt = 0.0, 0
        for s in range(0, nval - a.batch + 1, a.batch):
            b = torch.as_tensor(val[s:s + a.batch], device="cuda")
            out = net.forward(feats[b].reshape(-1, 17), ptr, sn).cpu().numpy()
            r = (out - labs[val[s:s + a.batch]]) * msks[val[s:s + a.batch]]
            tot += float(np.sum(np.sum(r * r, 1) / np.sum(msks[val[s:s + a.batch]], 1)))
            cnt += a.batch
        return tot / max(cnt, 1)

    steps_per_epoch = len(tr) // a.batch
    total = a.epochs * steps_per_epoch
    best, best_params, step = np.inf, None, 0
    hist = []
    for ep in range(a.epochs):
        if time.time() - t0 > a.time_limit:
            log(f"time limit reached after {ep} epochs")
            break
        order = rng.permutation(tr)
        tl = 0.0
        for s in range(steps_per_epoch):
            sel = order[s * a.batch:(s + 1) * a.batch]
            b = torch.as_tensor(sel, device="cuda")
            net.forward(feats[b].reshape(-1, 17), ptr, sn)
            lr = a.lr * 0.5 * (1 + np.cos(np.pi * step / total))
            l, _ = net.backward(labs_d[b], msks_d[b], want_loss=(s % 50 == 0))
            net.adam(lr)
            if l is not None:
                tl = l
            step += 1
        vl = val_loss()
        hist.append({"epoch": ep, "train_loss": tl, "val_loss": vl})
        log(f"epoch {ep}: train loss {tl:.4f} val loss {vl:.4f} ({time.time() - t0:.0f} s)")
        if vl < best:
            best, best_params = vl, net.get_params()
    np.save(a.out, best_params)
    with open(os.path.splitext(a.out)[0] + "_train.json", "w") as f:
        json.dump({"sets": int(n_sets), "val_sets": int(nval), "best_val_loss": best,
                   "mean_label_val_loss": base_loss, "history": hist,
                   "batch": a.batch, "lr": a.lr, "epochs": a.epochs}, f)
    log(f"best validation loss {best:.4f}; parameters written to {a.out}")


# ---------------------------------------------------------------------------
# warm start and evaluation
# ---------------------------------------------------------------------------
def steps_to(hist, target, rtol=1e-3):
    for k, v in enumerate(hist):
        if abs(v - target) <= rtol * abs(target):
            return k
    return None


def _start_lml(prob, th):
    """LML at a start, or -inf when a covariance there is not positive definite."""
    from . import LmaError
    try:
        v = prob(th, grad=False)
    except LmaError:
        return -np.inf
    return v if np.isfinite(v) else -np.inf


def evaluate_set(i, ws, steps=500, lr=0.05, lbfgs_iter=200, n=None):
    """LML* by converged L-BFGS, then Adam from the default start and from the
    warm start on held-out set i (n points; default 65536), each stopping at
    LML*."""
    import synth
    from synth import gpsets
    from . import LmlProblem
    from .hyperopt import adam, lbfgs
    p = gpsets.gp_set("heldout", i, n=n)
    prob = LmlProblem.from_problem(p)
    th0 = synth.default_theta0(p.y, p.d)
    t0 = time.perf_counter()
    thn = ws.predict(p.X, p.y)
    t_inf = time.perf_counter() - t0
    l0, ln = _start_lml(prob, th0), _start_lml(prob, thn)
    fallback = not np.isfinite(ln) or ln < l0
    start = th0 if fallback else thn
    row = {"index": i, "lml_default_start": float(l0), "lml_net_start": float(ln), "fallback": bool(fallback),
           "inference_s": t_inf, "theta_true": p.log_hyp.tolist(), "theta_net": np.asarray(thn).tolist(),
           "theta_default": th0.tolist(), "step_cap": steps}
    if not np.isfinite(l0) and not np.isfinite(ln):
        row.update(failed="no start with a positive definite covariance")
        return row
    fits = [lbfgs(prob, th, maxiter=lbfgs_iter, gtol=1e-6) for th in ((th0, start) if np.isfinite(l0) else (start,))]
    star = max(f["lml"] for f in fits)
    row.update(lml_star=float(star), lbfgs_evals=[int(f["nfev"]) for f in fits],
               lbfgs_converged=[bool(f["success"]) for f in fits])
    log(f"set {i}: LML* {star:.1f} from L-BFGS ({row['lbfgs_evals']} evaluations)")
    for name, th, extra in (("default", th0, 0.0), ("net", start, t_inf)):
        if name == "default" and not np.isfinite(l0):
            row.update(steps_default=steps, seconds_default=None, reached_default=False)
            continue
        r = adam(prob, th, steps=steps, lr=lr, target=star)
        row[f"steps_{name}"] = r["steps"] if r["reached"] else steps
        row[f"reached_{name}"] = bool(r["reached"])
        row[f"seconds_{name}"] = r["seconds"] + extra
        row[f"best_{name}"] = float(r["best"])
        log(f"set {i}: Adam from the {name} start, {row[f'steps_{name}']} steps")
    return row


def summarise(rows, cap):
    rows = [r for r in rows if "failed" not in r]
    kd = np.array([r["steps_default"] for r in rows], dtype=float)
    kn = np.array([r["steps_net"] for r in rows], dtype=float)
    td = np.array([np.nan if r["seconds_default"] is None else r["seconds_default"] for r in rows], dtype=float)
    tn = np.array([r["seconds_net"] for r in rows], dtype=float)
    both = np.isfinite(td)
    return {"sets": len(rows), "median_steps_default": float(np.median(kd)), "median_steps_net": float(np.median(kn)),
            "mean_steps_default": float(np.mean(kd)), "mean_steps_net": float(np.mean(kn)),
            "reached_default": int(sum(r["reached_default"] for r in rows)),
            "reached_net": int(sum(r["reached_net"] for r in rows)),
            "win_rate": float(np.mean(kn < kd)), "ties": float(np.mean(kn == kd)),
            "median_seconds_default": float(np.median(td[both])) if both.any() else None,
            "median_seconds_net": float(np.median(tn[both])) if both.any() else None,
            "fallbacks": int(sum(r["fallback"] for r in rows)), "step_cap": cap,
            "note": "steps and seconds of a run that never reaches LML* are counted at the cap; medians over the "
                    "same sets"}


def cmd_evaluate(a):
    from .warmstart import WarmStart
    ws = WarmStart(a.params)
    rows = []
    t0 = time.time()
    def write():
        if a.out:   # after every set, so that an interrupted run keeps what it finished
            tmp = a.out + ".tmp"
            with open(tmp, "w") as f:
                json.dump({"summary": summarise(rows, a.steps), "sets": rows}, f)
            os.replace(tmp, a.out)

    todo = [int(t) for t in a.indices.split(",")] if a.indices else range(a.first, a.first + a.count)
    for i in todo:
        r = evaluate_set(i, ws, steps=a.steps)
        rows.append(r)
        write()
        if "failed" in r:
            log(f"set {i}: {r['failed']}")
            continue
        log(f"set {i}: steps default {r['steps_default']} net {r['steps_net']} "
            f"(start LML {r['lml_default_start']:.1f} vs {r['lml_net_start']:.1f}, LML* {r['lml_star']:.1f}, "
            f"L-BFGS evaluations {r['lbfgs_evals']}; {time.time() - t0:.0f} s)")
    log(json.dumps(summarise(rows, a.steps)))


def cmd_merge_eval(a):
    """Merge evaluation outputs (disjoint set ranges) into the parameters' record."""
    rows, cap = [], None
    for path in a.inputs:
        with open(path) as f:
            e = json.load(f)
        rows += e["sets"]
        cap = e["summary"]["step_cap"]
    rows.sort(key=lambda r: r["index"])
    idx = [r["index"] for r in rows]
    if len(set(idx)) != len(idx):
        raise SystemExit("overlapping evaluation sets")
    with open(a.record) as f:
        rec = json.load(f)
    rec["evaluation"] = summarise(rows, cap)
    rec["evaluation_sets"] = rows
    with open(a.record, "w") as f:
        json.dump(rec, f, indent=1)
    log(json.dumps(rec["evaluation"]))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    p1 = sub.add_parser("labels")
    p1.add_argument("--first", type=int, default=0)
    p1.add_argument("--count", type=int, default=20000)
    p1.add_argument("--workers", type=int, default=8)
    p1.add_argument("--out", required=True)
    p1.add_argument("--time-limit", type=float, default=1e9)
    p1.add_argument("--maxiter", type=int, default=40)
    p2 = sub.add_parser("train")
    p2.add_argument("--labels", nargs="+", required=True)
    p2.add_argument("--out", required=True)
    p2.add_argument("--epochs", type=int, default=40)
    p2.add_argument("--batch", type=int, default=64)
    p2.add_argument("--lr", type=float, default=1e-3)
    p2.add_argument("--val", type=int, default=1000)
    p2.add_argument("--seed", type=int, default=0)
    p2.add_argument("--workers", type=int, default=12)
    p2.add_argument("--time-limit", type=float, default=1e9, help="stop starting epochs after this many seconds")
    p3 = sub.add_parser("evaluate")
    p3.add_argument("--params", required=True)
    p3.add_argument("--first", type=int, default=0)
    p3.add_argument("--count", type=int, default=100)
    p3.add_argument("--indices", default="", help="comma-separated set indices (instead of --first/--count)")
    p3.add_argument("--steps", type=int, default=500)
    p3.add_argument("--out", default=None)
    p4 = sub.add_parser("merge-eval")
    p4.add_argument("--inputs", nargs="+", required=True)
    p4.add_argument("--record", required=True)
    a = ap.parse_args(argv)
    {"labels": cmd_labels, "train": cmd_train, "evaluate": cmd_evaluate, "merge-eval": cmd_merge_eval}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
