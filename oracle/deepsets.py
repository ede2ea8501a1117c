"""Oracle of the warm-start network (test infrastructure only).

A deep-sets regressor from a dataset {(x_i, y_i)} to the log-hyperparameters
that maximise its LMA likelihood: a per-point encoder phi (two ReLU layers of
width 256), a mean over the points, and a head rho (a ReLU layer of width 256
and a linear layer to 10 outputs = 8 log length-scales, log sigma_s^2,
log sigma_n^2, in the scale of the standardised outputs).  Per-point features
(17): x * mask (8, zero beyond the input dimension d), the standardised
output (1), and the dimension mask (8).

The network is defined with its rounding: the weights used in products are the
bfloat16 roundings of float32 master weights; the inputs of the two per-point
layers (features, first-layer activations) and the per-point output gradients
of the backward pass are rounded to bfloat16 where they enter a product;
everything else (sums, bias, ReLU, mean, head) is exact arithmetic here
(float32 accumulation in the kernels).  A ReLU unit counts as active when its
rounded activation is positive.  exact=True drops every rounding (the plain
real-valued network, for finite-difference checks).  Loss per dataset: mean squared error
over its valid outputs (log l_1..log l_d, log sigma_s^2, log sigma_n^2);
batch loss: mean over datasets.  Adam (Kingma & Ba) on the master weights.

Plain float64 numpy; no blocking or fusion.
"""
import numpy as np

DMAX = 8
NF = 2 * DMAX + 1
WIDTH = 256
NOUT = DMAX + 2
SHAPES = {"W1": (WIDTH, NF), "b1": (WIDTH,), "W2": (WIDTH, WIDTH), "b2": (WIDTH,),
          "W3": (WIDTH, WIDTH), "b3": (WIDTH,), "W4": (NOUT, WIDTH), "b4": (NOUT,)}
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def bf16(a):
    """Round to the nearest bfloat16 (ties to even), via float32."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(X, y, d):
    """Per-point features of one dataset: [x * mask (8), (y - mean)/std, mask (8)]."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    F = np.zeros((n, NF))
    F[:, :d] = X[:, :d]
    y = np.asarray(y, dtype=np.float64)
    F[:, DMAX] = (y - y.mean()) / y.std()
    F[:, DMAX + 1:DMAX + 1 + d] = 1.0
    return F


def valid_mask(d):
    m = np.zeros(NOUT)
    m[:d] = 1.0
    m[DMAX:] = 1.0
    return m


def init_params(rng):
    """He-uniform weights, zero biases (float32 master values)."""
    p = {}
    for k in ORDER:
        if k.startswith("W"):
            fan_in = SHAPES[k][1]
            lim = np.sqrt(6.0 / fan_in)
            p[k] = rng.uniform(-lim, lim, size=SHAPES[k]).astype(np.float32).astype(np.float64)
        else:
            p[k] = np.zeros(SHAPES[k])
    return p


def forward(params, feats, exact=False):
    """feats: list of [n_b, 17] arrays.  Returns outputs [B, 10] and a cache."""
    r = (lambda a: np.asarray(a, dtype=np.float64)) if exact else bf16
    W = {k: r(params[k]) for k in ("W1", "W2", "W3", "W4")}
    cache = {"W": W, "sets": [], "exact": exact}
    outs = []
    for F in feats:
        Fb = r(F)
        Z1 = Fb @ W["W1"].T + params["b1"]
        H1b = r(np.maximum(Z1, 0.0))
        Z2 = H1b @ W["W2"].T + params["b2"]
        H2 = np.maximum(Z2, 0.0)
        H2b = r(H2)
        p = H2.mean(axis=0)
        z3 = W["W3"] @ p + params["b3"]
        h3 = np.maximum(z3, 0.0)
        o = W["W4"] @ h3 + params["b4"]
        cache["sets"].append(dict(Fb=Fb, H1b=H1b, H2b=H2b, p=p, z3=z3, h3=h3))
        outs.append(o)
    return np.array(outs), cache


def loss(outs, labels, masks):
    r = (outs - labels) * masks
    return float(np.mean(np.sum(r * r, axis=1) / np.sum(masks, axis=1)))


def backward(params, cache, outs, labels, masks):
    """Gradient of loss() with respect to every parameter."""
    W = cache["W"]
    r = (lambda a: np.asarray(a, dtype=np.float64)) if cache["exact"] else bf16
    B = outs.shape[0]
    g = {k: np.zeros(SHAPES[k]) for k in ORDER}
    for b, c in enumerate(cache["sets"]):
        do = 2.0 * (outs[b] - labels[b]) * masks[b] / masks[b].sum() / B
        g["W4"] += np.outer(do, c["h3"])
        g["b4"] += do
        dz3 = (W["W4"].T @ do) * (c["z3"] > 0)
        g["W3"] += np.outer(dz3, c["p"])
        g["b3"] += dz3
        dp = W["W3"].T @ dz3
        n = c["H2b"].shape[0]
        dZ2b = r(np.broadcast_to(dp / n, c["H2b"].shape) * (c["H2b"] > 0))
        g["W2"] += dZ2b.T @ c["H1b"]
        g["b2"] += dZ2b.sum(axis=0)
        dZ1b = r((dZ2b @ W["W2"]) * (c["H1b"] > 0))
        g["W1"] += dZ1b.T @ c["Fb"]
        g["b1"] += dZ1b.sum(axis=0)
    return g


def adam_step(params, grads, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t = 1, 2, ...) on the master weights, in place."""
    for k in ORDER:
        m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
