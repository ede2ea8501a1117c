"""Hyperparameter fitting by maximising the LMA log marginal likelihood.

Both optimisers call the library once per step (lma_lml with its gradient);
the loops themselves are host code over d+2 numbers.
"""
from __future__ import annotations

import time

import numpy as np

from . import LmaError, LmlProblem

# box for the log-hyperparameters of standardised outputs (keeps the residual
# covariances well conditioned during line searches)
LO_ELL, HI_ELL = np.log(0.02), np.log(50.0)
LO_SF2, HI_SF2 = np.log(1e-3), np.log(1e2)
LO_SN2, HI_SN2 = np.log(1e-4), np.log(10.0)


def bounds(d: int):
    return [(LO_ELL, HI_ELL)] * d + [(LO_SF2, HI_SF2), (LO_SN2, HI_SN2)]


def adam(problem: LmlProblem, theta0, steps: int = 50, lr: float = 0.05, betas=(0.9, 0.999), eps: float = 1e-8,
         target: float = None, rtol: float = 1e-3, callback=None):
    """Adam ascent on the LML through the LMALogML autograd Function.

    Stops after `steps` steps, or as soon as |LML - target| <= rtol |target|
    when a target is given.  Returns a dict with the LML before each step, the
    final theta, the step count and the wall time."""
    import torch
    from . import LMALogML
    th = torch.tensor(np.asarray(theta0, dtype=np.float64), requires_grad=True)
    opt = torch.optim.Adam([th], lr=lr, betas=betas, eps=eps)
    hist, best, best_th = [], -np.inf, th.detach().numpy().copy()
    t0 = time.perf_counter()
    reached = None
    for k in range(steps):
        opt.zero_grad()
        val = LMALogML.apply(th, problem)
        v = float(val.item())
        hist.append(v)
        if v > best:
            best, best_th = v, th.detach().numpy().copy()
        if target is not None and abs(v - target) <= rtol * abs(target):
            reached = k
            break
        (-val).backward()
        opt.step()
        with torch.no_grad():
            th.clamp_(min=-12.0, max=12.0)
        if callback:
            callback(k, v, th.detach().numpy())
    return {"lml": hist, "theta": th.detach().numpy().copy(), "best": best, "best_theta": best_th,
            "steps": len(hist) if reached is None else reached, "reached": reached is not None,
            "seconds": time.perf_counter() - t0}


def lbfgs(problem: LmlProblem, theta0, maxiter: int = 40, gtol: float = 1e-4):
    """Bounded L-BFGS on -LML (scipy), the library giving value and gradient.

    A start or trial point where a covariance is not positive definite counts
    as infinitely bad, so the line search backs off."""
    from scipy.optimize import minimize
    d = len(theta0) - 2
    nev = [0]

    def f(th):
        nev[0] += 1
        try:
            v, g = problem(th)
        except LmaError:
            return np.inf, np.zeros_like(th)
        if not np.isfinite(v) or not np.all(np.isfinite(g)):
            return np.inf, np.zeros_like(th)
        return -v, -np.asarray(g)

    x0 = np.clip(np.asarray(theta0, dtype=np.float64), [b[0] for b in bounds(d)], [b[1] for b in bounds(d)])
    r = minimize(f, x0, jac=True, method="L-BFGS-B", bounds=bounds(d),
                 options={"maxiter": maxiter, "gtol": gtol, "ftol": 1e-12})
    return {"theta": r.x, "lml": -float(r.fun), "nfev": nev[0], "success": bool(r.success) and np.isfinite(r.fun),
            "message": str(r.message)}
