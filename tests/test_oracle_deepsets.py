"""Pins of the warm-start network oracle (CPU): bfloat16 rounding against
torch's conversion, the exact backward pass against central differences,
invariances of the set function, and Adam's first step in closed form."""
import numpy as np
import pytest

from oracle import deepsets as ods


def small_batch(seed, sizes=(40, 17, 63), dims=(1, 4, 8)):
    rng = np.random.default_rng(seed)
    feats, labels, masks = [], [], []
    for n, d in zip(sizes, dims):
        X = rng.uniform(0, 1, size=(n, d))
        y = np.sin(3 * X).sum(1) + 0.1 * rng.standard_normal(n)
        feats.append(ods.features(X, y, d))
        labels.append(rng.normal(size=ods.NOUT))
        masks.append(ods.valid_mask(d))
    return feats, np.array(labels), np.array(masks)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        # exact ties: 1 + 2^-8 (to even: down), 1 + 3*2^-8 (to even: up)
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, -0.0]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(ods.bf16(x32), ref)
    assert ods.bf16([1.0 + 2.0 ** -8])[0] == 1.0
    assert ods.bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6


def test_features_layout():
    X = np.array([[0.1, 0.2], [0.3, 0.4], [0.5, 0.9]])
    y = np.array([1.0, 2.0, 4.0])
    F = ods.features(X, y, 2)
    assert F.shape == (3, 17)
    assert np.allclose(F[:, :2], X) and np.all(F[:, 2:8] == 0)
    assert abs(F[:, 8].mean()) < 1e-15 and abs(F[:, 8].std() - 1.0) < 1e-14
    assert np.all(F[:, 9:11] == 1) and np.all(F[:, 11:] == 0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(2)
    params = ods.init_params(rng)
    for k in ("b1", "b2", "b3", "b4"):
        params[k] = 0.05 * rng.standard_normal(ods.SHAPES[k])
    feats, labels, masks = small_batch(3)
    outs, cache = ods.forward(params, feats, exact=True)
    g = ods.backward(params, cache, outs, labels, masks)
    h = 1e-6
    for k in ods.ORDER:
        flat = params[k].reshape(-1)
        for idx in rng.choice(flat.size, size=6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = ods.loss(ods.forward(params, feats, exact=True)[0], labels, masks)
            flat[idx] = old - h
            lm = ods.loss(ods.forward(params, feats, exact=True)[0], labels, masks)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, idx, fd, an)


def test_set_function_invariances():
    rng = np.random.default_rng(4)
    params = ods.init_params(rng)
    feats, _, _ = small_batch(5)
    F = feats[2]
    for exact in (True, False):
        base = ods.forward(params, [F], exact=exact)[0]
        perm = ods.forward(params, [F[rng.permutation(F.shape[0])]], exact=exact)[0]
        dup = ods.forward(params, [np.concatenate([F, F])], exact=exact)[0]
        assert np.allclose(base, perm, rtol=1e-12, atol=1e-12)
        assert np.allclose(base, dup, rtol=1e-12, atol=1e-12)


def test_masked_outputs_do_not_matter():
    rng = np.random.default_rng(6)
    params = ods.init_params(rng)
    feats, labels, masks = small_batch(7)
    outs, cache = ods.forward(params, feats)
    l0 = ods.loss(outs, labels, masks)
    g0 = ods.backward(params, cache, outs, labels, masks)
    labels2 = labels.copy()
    labels2[masks == 0] += 100.0
    assert ods.loss(outs, labels2, masks) == l0
    g1 = ods.backward(params, cache, outs, labels2, masks)
    for k in ods.ORDER:
        assert np.array_equal(g0[k], g1[k])
    # a 1-D dataset alone: its masked outputs 1..7 carry no gradient into W4 / b4
    o1, c1 = ods.forward(params, feats[:1])
    g2 = ods.backward(params, c1, o1, labels[:1], masks[:1])
    assert np.all(g2["W4"][1:8] == 0) and np.all(g2["b4"][1:8] == 0)
    assert np.any(g2["W4"][0] != 0) and np.any(g2["W4"][8:] != 0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    params = {k: rng.standard_normal(ods.SHAPES[k]) for k in ods.ORDER}
    grads = {k: rng.standard_normal(ods.SHAPES[k]) for k in ods.ORDER}
    m = {k: np.zeros(ods.SHAPES[k]) for k in ods.ORDER}
    v = {k: np.zeros(ods.SHAPES[k]) for k in ods.ORDER}
    before = {k: params[k].copy() for k in ods.ORDER}
    lr, eps = 1e-3, 1e-8
    ods.adam_step(params, grads, m, v, 1, lr, eps=eps)
    for k in ods.ORDER:
        assert np.allclose(before[k] - params[k], lr * grads[k] / (np.abs(grads[k]) + eps), rtol=1e-12, atol=0)
