#!/usr/bin/env python3
"""|S| x B trade-off sweep of LMA on one MI355X (paper: Remark 3 and the
experiments on the spectrum between PIC at B = 0 and the full GP at B = M-1).

Two synthetic workloads:

* ``fgp`` -- n = 16384 points in [0,1]^8 from a GP sample (l_i ~ logU[0.1, 1],
  sf2 = 1, sn2 = 0.05), M = 16 k-means blocks of 1024, 4096 test points.  B runs
  from 0 (PIC) to M - 1 = 15, where LMA is the full GP whatever the support set,
  so every point of the sweep is also compared with the full-GP predictive mean.
* ``large`` -- the n = 524288, d = 21 mixture workload (M = 256 blocks of
  1024..3072, 65536 test points), B in 0..3, model noise sn2 = 1.01 (the rough
  component of the outputs taken as noise).

Support sets are nested: |S| rows are the first |S| of one random permutation
of the training points.  For each (|S|, B): the fit + predict time (median of
the timed repetitions after a warm-up, inputs resident in HBM), the RMSE and
the mean negative log predictive probability against the noisy test outputs
(over the points with a positive predictive variance, with the count of the
others), and the LML.  Prints one JSON line per point and writes all of them to --out.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def nested_supports(X, sizes):
    import synth
    return {s: synth.nested_support(X, s) for s in sizes}


def run_point(lma, torch, Xd, yd, Ud, p, S, B, log_hyp, reps, precision):
    Sd = torch.as_tensor(S, dtype=torch.float64, device="cuda")

    def once():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = lma.fit(Xd, yd, p.block_ptr, Sd, B, log_hyp, p.prior_mean, precision=precision)
        mean, var = st.predict(Ud, p.u_block_ptr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        lml_val = st.lml()
        st.free()
        return dt, mean, var, lml_val

    once()
    times = []
    for _ in range(reps):
        dt, mean, var, lml_val = once()
        times.append(dt)
    return float(np.median(times)), mean.cpu().numpy(), var.cpu().numpy(), lml_val


def scores(mean, var, y_u):
    """RMSE over all test points; MNLP over the test points whose predictive
    variance is positive (between B = 0 and B = M - 1 the variance of a few
    points can be negative, see the count reported beside it)."""
    err = mean - y_u
    rmse = float(np.sqrt(np.mean(err ** 2)))
    ok = var > 0
    mnlp = float(0.5 * np.mean(np.log(2 * np.pi * var[ok]) + err[ok] ** 2 / var[ok]))
    return rmse, mnlp, int(np.sum(~ok))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="fgp,large")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--reps", type=int, default=1, help="timed repetitions per point")
    ap.add_argument("--out", default="")
    ap.add_argument("--sizes", default="", help="comma-separated |S| values (default: the workload's)")
    ap.add_argument("--orders", default="", help="comma-separated Markov orders B (default: the workload's)")
    args = ap.parse_args()

    import torch
    import synth
    import paper_1411_4510_amd as lma

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    lma.load()
    rows = []
    out = open(args.out, "w") if args.out else None
    for wl in [w for w in args.workloads.split(",") if w]:
        t0 = time.perf_counter()
        if wl == "fgp":
            p = synth.make_uniform_kmeans(1, 16384, 8, 16, 0, 16, 4096, 0.05, name="n16384")
            sizes, Bs, log_hyp = [16, 64, 256, 1024], [0, 1, 2, 4, 8, 15], p.log_hyp
        elif wl == "large":
            p = synth.make_config(2)
            sizes, Bs = [256, 512, 1024, 2048], [0, 1, 2, 3]
            log_hyp = p.log_hyp.copy()
            log_hyp[-1] = np.log(1.01)
        else:
            raise SystemExit(f"unknown workload {wl}")
        if args.sizes:
            sizes = [int(v) for v in args.sizes.split(",")]
        if args.orders:
            Bs = [int(v) for v in args.orders.split(",")]
        log(f"{wl}: inputs drawn in {time.perf_counter() - t0:.1f} s (n={p.n} d={p.d} M={p.M} n_u={p.n_u})")
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
        Xd, yd, Ud = dev(p.X), dev(p.y), dev(p.U)
        supports = nested_supports(p.X, sizes)
        fgp_mean = None
        if wl == "fgp":
            # B = M - 1: the full GP, independent of the support set
            _, fgp_mean, _, _ = run_point(lma, torch, Xd, yd, Ud, p, supports[sizes[-1]], p.M - 1, log_hyp, 1,
                                          args.precision)
        for s in sizes:
            for B in Bs:
                dt, mean, var, lml_val = run_point(lma, torch, Xd, yd, Ud, p, supports[s], B, log_hyp, args.reps,
                                                   args.precision)
                rmse, mnlp, nonpos = scores(mean, var, p.y_u)
                row = {"workload": wl, "n": p.n, "d": p.d, "M": p.M, "n_u": p.n_u, "s": s, "B": B,
                       "precision": args.precision, "fit_predict_s": dt, "rmse": rmse, "mnlp": mnlp,
                       "var_nonpositive": nonpos, "lml": lml_val}
                if fgp_mean is not None:
                    row["mean_rel_to_fgp"] = float(np.linalg.norm(mean - fgp_mean) / np.linalg.norm(fgp_mean))
                rows.append(row)
                print(json.dumps(row), flush=True)
                if out:
                    out.write(json.dumps(row) + "\n")
                    out.flush()
        del Xd, yd, Ud
        lma.release_cache()
        torch.cuda.empty_cache()
    if out:
        out.close()


if __name__ == "__main__":
    main()
