"""Warm-start network: binding of the lma_ds_* entry points (include/lma_ds.h)
and the warm-start wrapper used before hyperparameter optimisation.

Every step of the network runs in the library's kernels; this module only
marshals arguments (torch tensors provide device memory and streams).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _check, _stream, load

PARAMS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "warmstart_params.npy")
NPARAM = 138762
NFEAT = 17
NOUT = 10
DMAX = 8
WIDTH = 256
LAYOUT = (("W1", (WIDTH, NFEAT)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (NOUT, WIDTH)), ("b4", (NOUT,)))


def pack(params: dict) -> np.ndarray:
    """Parameter dict -> the library's float32 vector (order of LAYOUT)."""
    v = np.concatenate([np.asarray(params[k], dtype=np.float32).reshape(-1) for k, _ in LAYOUT])
    assert v.size == NPARAM
    return np.ascontiguousarray(v)


def unpack(vec) -> dict:
    vec = np.asarray(vec, dtype=np.float32)
    out, o = {}, 0
    for k, shp in LAYOUT:
        n = int(np.prod(shp))
        out[k] = vec[o:o + n].reshape(shp).copy()
        o += n
    return out


def he_init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, shp in LAYOUT:
        if k.startswith("W"):
            lim = np.sqrt(6.0 / shp[1])
            p[k] = rng.uniform(-lim, lim, size=shp)
        else:
            p[k] = np.zeros(shp)
    return pack(p)


def aligned_layout(sizes):
    """set_ptr (multiples of 128) and set_n for datasets of the given sizes."""
    sizes = np.asarray(sizes, dtype=np.int64)
    rows = (sizes + 127) // 128 * 128
    ptr = np.zeros(len(sizes) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum(rows)
    return ptr, sizes.copy()


class Network:
    """The network's device state (parameters, Adam moments, workspace)."""

    def __init__(self, max_rows: int, max_sets: int):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.lma_ds_create(int(max_rows), int(max_sets), ctypes.byref(h)))
        self._h = h

    def set_params(self, vec):
        v = np.ascontiguousarray(np.asarray(vec, dtype=np.float32))
        if v.size != NPARAM:
            raise ValueError(f"need {NPARAM} parameters")
        _check(self._lib.lma_ds_set_params(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self) -> np.ndarray:
        v = np.zeros(NPARAM, dtype=np.float32)
        _check(self._lib.lma_ds_get_params(self._h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return v

    def features(self, X, y, out=None, stream=None):
        """Per-point features [n, 17] (float32, device) of one dataset (X [n, d], y [n])."""
        import torch
        Xd = torch.as_tensor(X, dtype=torch.float64, device="cuda").contiguous()
        yd = torch.as_tensor(y, dtype=torch.float64, device="cuda").reshape(-1).contiguous()
        n, d = Xd.shape
        if out is None:
            out = torch.empty((n, NFEAT), dtype=torch.float32, device="cuda")
        _check(self._lib.lma_ds_features(self._h, ctypes.c_void_p(Xd.data_ptr()), ctypes.c_void_p(yd.data_ptr()),
                                         n, d, ctypes.c_void_p(out.data_ptr()), _stream(torch, stream)))
        return out

    def forward(self, feats, set_ptr, set_n, stream=None):
        """Outputs [nsets, 10] (float32, device) for feature rows laid out by set_ptr / set_n."""
        import torch
        ptr = np.ascontiguousarray(np.asarray(set_ptr, dtype=np.int64))
        sn = np.ascontiguousarray(np.asarray(set_n, dtype=np.int64))
        nsets = len(sn)
        if feats.dtype != torch.float32 or not feats.is_cuda or not feats.is_contiguous():
            raise ValueError("feats must be a contiguous float32 device tensor")
        if feats.shape[0] < ptr[-2] + sn[-1] or feats.shape[1] != NFEAT:
            raise ValueError("feats must have [rows, 17] with rows covering every set")
        out = torch.empty((nsets, NOUT), dtype=torch.float32, device="cuda")
        _check(self._lib.lma_ds_forward(self._h, nsets, ptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        sn.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        ctypes.c_void_p(feats.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                        _stream(torch, stream)))
        self._keep = (ptr, sn)
        return out

    def backward(self, labels, masks, want_grad=False, want_loss=True, stream=None):
        """Gradient of the batch loss of the last forward; returns (loss, grad)."""
        import torch
        lab = torch.as_tensor(labels, dtype=torch.float32, device="cuda").contiguous()
        msk = torch.as_tensor(masks, dtype=torch.float32, device="cuda").contiguous()
        grad = torch.empty(NPARAM, dtype=torch.float32, device="cuda") if want_grad else None
        loss = ctypes.c_double()
        _check(self._lib.lma_ds_backward(self._h, ctypes.c_void_p(lab.data_ptr()), ctypes.c_void_p(msk.data_ptr()),
                                         ctypes.c_void_p(grad.data_ptr()) if grad is not None else None,
                                         ctypes.byref(loss) if want_loss else None, _stream(torch, stream)))
        return (loss.value if want_loss else None), grad

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        import torch
        _check(self._lib.lma_ds_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                     _stream(torch, stream)))

    def free(self):
        if getattr(self, "_h", None):
            self._lib.lma_ds_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def valid_mask(d: int) -> np.ndarray:
    m = np.zeros(NOUT, dtype=np.float32)
    m[:d] = 1.0
    m[DMAX:] = 1.0
    return m


def to_log_hyp(out_row, d: int, y) -> np.ndarray:
    """Network outputs (standardised-output scale) -> log_hyp of the raw data."""
    o = np.asarray(out_row, dtype=np.float64)
    lv = float(np.log(np.var(np.asarray(y, dtype=np.float64))))
    return np.concatenate([o[:d], [o[DMAX] + lv, o[DMAX + 1] + lv]])


def to_label(log_hyp, d: int, y) -> np.ndarray:
    """log_hyp of the raw data -> the network's target row (standardised-output scale)."""
    lh = np.asarray(log_hyp, dtype=np.float64)
    lv = float(np.log(np.var(np.asarray(y, dtype=np.float64))))
    lab = np.zeros(NOUT)
    lab[:d] = lh[:d]
    lab[DMAX] = lh[d] - lv
    lab[DMAX + 1] = lh[d + 1] - lv
    return lab


class WarmStart:
    """Starting log-hyperparameters for LMA fitting, predicted by the trained
    network (parameters from train_warmstart, shipped beside this module).

    predict(X, y) expects standardised outputs (zero mean, unit variance) and
    inputs in the unit cube; returns [log l_1..log l_d, log sigma_s^2,
    log sigma_n^2]."""

    def __init__(self, params=None, max_rows=65536):
        self.net = Network(max_rows=max_rows, max_sets=1)
        self.net.set_params(np.load(params or PARAMS_PATH) if params is None or isinstance(params, str) else params)
        self.max_rows = max_rows

    def predict(self, X, y):
        import torch
        n, d = X.shape
        if d > DMAX:
            raise ValueError("the warm-start network covers d <= 8")
        rows = (n + 127) // 128 * 128
        if rows > self.max_rows:
            raise ValueError("dataset larger than the network workspace")
        feats = torch.zeros((rows, NFEAT), dtype=torch.float32, device="cuda")
        self.net.features(X, y, out=feats[:n])
        out = self.net.forward(feats, [0, rows], [n]).cpu().numpy()[0]
        return np.r_[out[:d], out[DMAX], out[DMAX + 1]].astype(np.float64)
