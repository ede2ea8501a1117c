"""Warm-start network kernels against the network oracle: features, forward
outputs, loss and gradients (float32 accumulation and bfloat16 products on
the GPU against float64 arithmetic with the same bfloat16 roundings), Adam
steps, determinism and a short training run.

Tolerances: the oracle rounds the same operands to bfloat16, so the two sides
differ by float32 accumulation (relative 1e-6) plus the occasional operand
that float32 and float64 round to neighbouring bfloat16 values (a relative
change of 2^-8 in one activation of one point, averaged into the mean over
hundreds of points): 1e-3 on outputs and loss, 5e-3 on each gradient tensor."""
import numpy as np
import pytest

from oracle import deepsets as ods

pytestmark = pytest.mark.gpu

SIZES = (300, 128, 1000, 4096, 77)
DIMS = (1, 4, 8, 8, 3)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def datasets(seed, sizes=SIZES, dims=DIMS):
    rng = np.random.default_rng(seed)
    out = []
    for n, d in zip(sizes, dims):
        X = rng.uniform(0, 1, size=(n, d))
        y = 2.0 * np.sin(3 * X).sum(1) + 0.3 * rng.standard_normal(n) + 1.5
        out.append((X, y, d))
    return out


def params(seed):
    rng = np.random.default_rng(seed)
    p = ods.init_params(rng)
    for k in ("b1", "b2", "b3", "b4"):
        p[k] = (0.05 * rng.standard_normal(ods.SHAPES[k])).astype(np.float32).astype(np.float64)
    return p


def batch(sets):
    """Oracle features (float32-rounded) and the aligned device layout."""
    import torch
    from paper_1411_4510_amd import warmstart as ws
    feats = [ods.features(X, y, d).astype(np.float32).astype(np.float64) for X, y, d in sets]
    ptr, sn = ws.aligned_layout([f.shape[0] for f in feats])
    dev = np.zeros((ptr[-1], 17), dtype=np.float32)
    for f, o in zip(feats, ptr[:-1]):
        dev[o:o + f.shape[0]] = f
    return feats, torch.as_tensor(dev, device="cuda"), ptr, sn


@pytest.fixture(scope="module")
def ws(lib):
    from paper_1411_4510_amd import warmstart
    return warmstart


def test_features_match_oracle(ws):
    net = ws.Network(8192, 4)
    for X, y, d in datasets(1):
        F = net.features(X, y).cpu().numpy().astype(np.float64)
        Fo = ods.features(X, y, d)
        assert np.max(np.abs(F - Fo)) <= 2e-6 * max(1.0, np.max(np.abs(Fo)))


def test_forward_backward_match_oracle(ws):
    p = params(2)
    sets = datasets(3)
    feats, dev, ptr, sn = batch(sets)
    rng = np.random.default_rng(4)
    labels = rng.normal(size=(len(sets), 10))
    masks = np.array([ods.valid_mask(d) for _, _, d in sets])
    net = ws.Network(int(ptr[-1]), len(sets))
    net.set_params(ws.pack(p))
    out = net.forward(dev, ptr, sn).cpu().numpy()
    loss, grad = net.backward(labels, masks, want_grad=True)
    oo, cache = ods.forward(p, feats)
    lo = ods.loss(oo, labels, masks)
    go = ods.backward(p, cache, oo, labels, masks)
    print(f"  outputs rel {rel(out, oo):.2e} loss rel {abs(loss - lo) / lo:.2e}", flush=True)
    assert rel(out, oo) <= 1e-3
    assert abs(loss - lo) <= 1e-3 * lo
    g = ws.unpack(grad.cpu().numpy())
    for k in ods.ORDER:
        e = rel(g[k], go[k])
        print(f"  grad {k}: rel {e:.2e}", flush=True)
        assert e <= 5e-3, k


def test_adam_steps_match_oracle(ws):
    p = params(5)
    sets = datasets(6, sizes=(500, 260), dims=(2, 8))
    feats, dev, ptr, sn = batch(sets)
    labels = np.random.default_rng(7).normal(size=(2, 10))
    masks = np.array([ods.valid_mask(d) for _, _, d in sets])
    net = ws.Network(int(ptr[-1]), 2)
    net.set_params(ws.pack(p))
    po = {k: v.copy() for k, v in p.items()}
    m = {k: np.zeros(ods.SHAPES[k]) for k in ods.ORDER}
    v = {k: np.zeros(ods.SHAPES[k]) for k in ods.ORDER}
    lr = 1e-3
    for t in (1, 2):
        net.forward(dev, ptr, sn)
        net.backward(labels, masks, want_loss=False)
        net.adam(lr)
        oo, cache = ods.forward(po, feats)
        go = ods.backward(po, cache, oo, labels, masks)
        ods.adam_step(po, go, m, v, t, lr)
        pg = ws.unpack(net.get_params())
        for k in ods.ORDER:
            # compare where the oracle's gradient is clearly non-zero (elsewhere
            # the step direction is decided by rounding)
            big = np.abs(go[k]) > 0.05 * np.sqrt(np.mean(go[k] ** 2)) + 1e-30
            assert np.all(np.abs(pg[k][big] - po[k][big]) <= 1e-5 * lr * t + 1e-6), (t, k)
            assert np.all(np.abs(pg[k] - p[k]) <= 2 * lr * t + 1e-6), (t, k)


def test_deterministic(ws):
    p = params(8)
    feats, dev, ptr, sn = batch(datasets(9))
    labels = np.zeros((len(sn), 10))
    masks = np.ones((len(sn), 10))
    net = ws.Network(int(ptr[-1]), len(sn))
    net.set_params(ws.pack(p))
    r = []
    for _ in range(2):
        o = net.forward(dev, ptr, sn).cpu().numpy()
        l, g = net.backward(labels, masks, want_grad=True)
        r.append((o, l, g.cpu().numpy()))
    assert np.array_equal(r[0][0], r[1][0]) and r[0][1] == r[1][1] and np.array_equal(r[0][2], r[1][2])


def test_training_reduces_loss(ws):
    sets = datasets(10, sizes=(700, 900, 400, 1200), dims=(2, 5, 8, 3))
    feats, dev, ptr, sn = batch(sets)
    labels = np.random.default_rng(11).normal(size=(4, 10))
    masks = np.array([ods.valid_mask(d) for _, _, d in sets])
    net = ws.Network(int(ptr[-1]), 4)
    net.set_params(ws.he_init(12))
    losses = []
    for _ in range(60):
        net.forward(dev, ptr, sn)
        l, _ = net.backward(labels, masks)
        net.adam(3e-3)
        losses.append(l)
    print(f"  loss {losses[0]:.3f} -> {losses[-1]:.3f}", flush=True)
    assert losses[-1] < 0.2 * losses[0]
