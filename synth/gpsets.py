"""Datasets drawn from Gaussian-process priors for the warm-start network.

Training sets: n = 4096 points uniform in [0,1]^d, d uniform in 1..8; held-out
sets: n = 65536, d = 8.  Hyperparameters are drawn log-uniformly (per-input
length-scales in [0.05, 2], signal variance in [0.1, 10], noise variance in
[1e-3, 0.5]); outputs are a random-Fourier-feature approximation of a draw
from the zero-mean SE-ARD prior plus Gaussian noise, standardised to zero mean
and unit variance (the network and the likelihood fits work in that scale).
Blocks: sorted on the first input, 256 points each for the training sets
(M = 16), 1024 for the held-out sets (M = 64); support set: 256 random inputs;
Markov order B = 2.

Every set is identified by (kind, index) and drawn from its own seed, so any
subset can be regenerated independently.  Inputs only: nothing here computes
anything of the method.
"""
import numpy as np

from . import ROOT_SEED, Problem, _loguniform, rff_draw, sorted_partition

ELL = (0.05, 2.0)
SF2 = (0.1, 10.0)
SN2 = (1e-3, 0.5)
KIND = {"train": 1, "heldout": 2}


def gp_set(kind: str, index: int, n: int = None, d: int = None, s: int = None, block: int = None, B: int = 2,
           F: int = 512):
    """One dataset as an LMA Problem (log_hyp = the hyperparameters it was drawn
    with, rescaled to the standardised outputs)."""
    if kind not in KIND:
        raise ValueError(kind)
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(7, KIND[kind], int(index)))
    r_d, r_h, r_x, r_f, r_e, r_s = [np.random.default_rng(c) for c in ss.spawn(6)]
    if kind == "train":
        n = n or 4096
        d = d or int(r_d.integers(1, 9))
        s = s or 256
        block = block or 256
    else:
        n = n or 65536
        d = d or 8
        s = s or 256
        block = block or 1024
    ell = _loguniform(r_h, *ELL, size=d)
    sf2 = float(_loguniform(r_h, *SF2))
    sn2 = float(_loguniform(r_h, *SN2))
    X0 = r_x.uniform(0.0, 1.0, size=(n, d))
    f = rff_draw(r_f, [X0], ell, sf2, F)[0]
    y0 = f + np.sqrt(sn2) * r_e.standard_normal(n)
    mu, sd = float(y0.mean()), float(y0.std())
    y0 = (y0 - mu) / sd
    M = n // block
    perm, bp, _, _ = sorted_partition(X0, [block] * M)
    X, y = X0[perm], y0[perm]
    S = X[np.sort(r_s.choice(n, size=s, replace=False))].copy()
    log_hyp = np.r_[np.log(ell), np.log(sf2 / sd ** 2), np.log(sn2 / sd ** 2)]
    return Problem(X=X, y=y, block_ptr=bp, S=S, B=B, log_hyp=log_hyp, prior_mean=0.0,
                   name=f"gp-{kind}-{index}")
