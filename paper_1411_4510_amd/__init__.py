"""Python binding of the MI355X LMA library (liblma.so, C ABI in include/lma.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of liblma.so.  PyTorch supplies device memory and the current HIP stream.
There is no CPU fallback: if the library is missing, load() raises.

    import paper_1411_4510_amd as lma
    st = lma.fit(X, y, block_ptr, S, B, log_hyp, prior_mean=0.0, precision="fp64")
    mean, var = st.predict(U, u_block_ptr)
    val = lma.lml(X, y, block_ptr, S, B, log_hyp)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblma.so")

LMA_OK, LMA_E_ARG, LMA_E_NOT_PD, LMA_E_HIP, LMA_E_NOMEM, LMA_E_INTERNAL = 0, 1, 2, 3, 4, 5
PRECISION = {"fp64": 0, "mixed": 1}
EXPORTS = ("lma_fit", "lma_predict", "lma_predict_cov", "lma_lml", "lma_free", "lma_state_lml", "lma_state_bytes", "lma_state_chunks",
           "lma_last_error", "lma_failed_block", "lma_version", "lma_profile_enable",
           "lma_profile_read", "lma_release_cache")
PART_EXPORTS = ("lma_kmeans_assign", "lma_kmeans_update", "lma_kmeans_update_noalloc", "lma_kmeans",
                "lma_chain_order", "lma_kmeans_seed", "lma_bounded_assign", "lma_partition")
DS_EXPORTS = ("lma_ds_create", "lma_ds_free", "lma_ds_set_params", "lma_ds_get_params", "lma_ds_features",
              "lma_ds_forward", "lma_ds_backward", "lma_ds_adam")


class LmaError(RuntimeError):
    def __init__(self, status, message, block=None):
        super().__init__(f"[{status}] {message}" + (f" (block {block})" if block is not None else ""))
        self.status = status
        self.block = block


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("s", ctypes.c_int64),
        ("M", ctypes.c_int64), ("B", ctypes.c_int64),
        ("X", ctypes.c_void_p), ("y", ctypes.c_void_p),
        ("block_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("S", ctypes.c_void_p),
        ("log_hyp", ctypes.POINTER(ctypes.c_double)),
        ("prior_mean", ctypes.c_double),
        ("precision", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("mem_budget_bytes", ctypes.c_int64),
    ]


class Profile(ctypes.Structure):
    _fields_ = [
        ("update_ms", ctypes.c_double), ("diag_ms", ctypes.c_double),
        ("trsm_ms", ctypes.c_double), ("other_ms", ctypes.c_double),
        ("update_alg_flops", ctypes.c_double), ("update_alg_flops_f64", ctypes.c_double),
        ("update_launches", ctypes.c_int64), ("other_launches", ctypes.c_int64),
        ("gemm_ms", ctypes.c_double), ("gemm_alg_flops", ctypes.c_double),
        ("contract_ms", ctypes.c_double), ("contract_alg_flops", ctypes.c_double),
        ("gemm_launches", ctypes.c_int64), ("contract_launches", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Load liblma.so (built in-tree by build()); raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (paper_1411_4510_amd.build)")
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes the library bind to that runtime instead of loading a second one
    # (two HIP/HSA runtimes in one process cannot both open the device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i64, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.lma_fit.argtypes = [ctypes.POINTER(_Problem), vp, ctypes.POINTER(vp)]
    lib.lma_fit.restype = st
    lib.lma_predict.argtypes = [vp, i64, vp, ctypes.POINTER(i64), vp, vp, vp]
    lib.lma_predict.restype = st
    lib.lma_predict_cov.argtypes = [vp, i64, vp, ctypes.POINTER(i64), vp, vp, vp]
    lib.lma_predict_cov.restype = st
    lib.lma_lml.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(ctypes.c_double),
                            ctypes.POINTER(ctypes.c_double), vp]
    lib.lma_lml.restype = st
    lib.lma_free.argtypes = [vp]
    lib.lma_free.restype = None
    lib.lma_state_lml.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.lma_state_lml.restype = st
    for name in ("lma_state_bytes", "lma_state_chunks"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = ctypes.c_int64
    lib.lma_last_error.restype = ctypes.c_char_p
    lib.lma_failed_block.restype = i64
    lib.lma_version.restype = ctypes.c_char_p
    lib.lma_release_cache.argtypes = []
    lib.lma_release_cache.restype = None
    lib.lma_profile_enable.argtypes = [ctypes.c_int]
    lib.lma_profile_enable.restype = None
    lib.lma_profile_read.argtypes = [ctypes.POINTER(Profile), ctypes.c_int]
    lib.lma_profile_read.restype = st
    fp, f32 = ctypes.POINTER(ctypes.c_float), ctypes.c_float
    lib.lma_ds_create.argtypes = [i64, i64, ctypes.POINTER(vp)]
    lib.lma_ds_create.restype = st
    lib.lma_ds_free.argtypes = [vp]
    lib.lma_ds_free.restype = None
    lib.lma_ds_set_params.argtypes = [vp, fp]
    lib.lma_ds_set_params.restype = st
    lib.lma_ds_get_params.argtypes = [vp, fp]
    lib.lma_ds_get_params.restype = st
    lib.lma_ds_features.argtypes = [vp, vp, vp, i64, ctypes.c_int32, vp, vp]
    lib.lma_ds_features.restype = st
    lib.lma_ds_forward.argtypes = [vp, i64, ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp]
    lib.lma_ds_forward.restype = st
    lib.lma_ds_backward.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp]
    lib.lma_ds_backward.restype = st
    lib.lma_ds_adam.argtypes = [vp, f32, f32, f32, f32, vp]
    lib.lma_ds_adam.restype = st
    i32 = ctypes.c_int32
    lib.lma_kmeans_assign.argtypes = [vp, i64, i32, vp, i32, vp, vp, vp]
    lib.lma_kmeans_assign.restype = st
    lib.lma_kmeans_update.argtypes = [vp, i64, i32, vp, i32, vp, vp, vp]
    lib.lma_kmeans_update.restype = st
    lib.lma_kmeans_update_noalloc.argtypes = [vp, i64, i32, vp, i32, vp, vp, vp]
    lib.lma_kmeans_update_noalloc.restype = st
    lib.lma_kmeans.argtypes = [vp, i64, i32, vp, i32, i32, vp, vp, vp]
    lib.lma_kmeans.restype = st
    lib.lma_chain_order.argtypes = [vp, i32, i32, vp]
    lib.lma_chain_order.restype = st
    lib.lma_kmeans_seed.argtypes = [vp, i64, i32, i32, vp, vp, vp, vp]
    lib.lma_kmeans_seed.restype = st
    lib.lma_bounded_assign.argtypes = [vp, i64, i32, vp, i32, i64, i64, vp, vp, vp, vp]
    lib.lma_bounded_assign.restype = st
    lib.lma_partition.argtypes = [vp, i64, vp, i64, i32, i32, i64, i64, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.lma_partition.restype = st
    _lib = lib
    return lib


def _check(status):
    if status != LMA_OK:
        msg = _lib.lma_last_error().decode()
        block = int(_lib.lma_failed_block()) if status == LMA_E_NOT_PD else None
        if block == -3:     # a non-finite likelihood or gradient: no single block
            block = None
        raise LmaError(status, msg, block)


def _dev(a, torch, dtype=None):
    """Device float64 contiguous tensor from a numpy array or tensor."""
    dtype = dtype or torch.float64
    if isinstance(a, torch.Tensor):
        t = a.to(device="cuda", dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")
    return t.contiguous()


def _stream(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _Inputs:
    """Keeps device copies and host arrays alive for the duration of a call."""

    def __init__(self, X, y, block_ptr, S, B, log_hyp, prior_mean, precision, mem_budget):
        import torch
        self.X = _dev(X, torch)
        self.y = _dev(y, torch).reshape(-1)
        self.S = _dev(S, torch)
        self.bp = np.ascontiguousarray(np.asarray(block_ptr, dtype=np.int64))
        self.lh = np.ascontiguousarray(np.asarray(log_hyp, dtype=np.float64))
        n, d = self.X.shape
        pr = _Problem()
        pr.n, pr.d, pr.s = n, d, self.S.shape[0]
        pr.M, pr.B = len(self.bp) - 1, int(B)
        pr.X, pr.y, pr.S = self.X.data_ptr(), self.y.data_ptr(), self.S.data_ptr()
        pr.block_ptr = self.bp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
        pr.log_hyp = self.lh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        pr.prior_mean = float(prior_mean)
        pr.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        pr.reserved = 0
        pr.mem_budget_bytes = int(mem_budget)
        self.problem = pr


class State:
    """A fitted LMA model (owns an lma_state)."""

    def __init__(self, handle, M):
        self._h = handle
        self.M = M

    def predict(self, U, u_block_ptr, want_var=True, stream=None):
        """Predictive mean and variance (device float64 tensors)."""
        import torch
        Ud = _dev(U, torch)
        ubp = np.ascontiguousarray(np.asarray(u_block_ptr, dtype=np.int64))
        n_u = Ud.shape[0]
        mean = torch.empty(n_u, dtype=torch.float64, device="cuda")
        var = torch.empty(n_u, dtype=torch.float64, device="cuda") if want_var else None
        _check(_lib.lma_predict(self._h, n_u, ctypes.c_void_p(Ud.data_ptr()),
                                ubp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                ctypes.c_void_p(mean.data_ptr()),
                                ctypes.c_void_p(var.data_ptr()) if var is not None else None,
                                _stream(torch, stream)))
        return mean, var

    def predict_cov(self, U, u_block_ptr, want_mean=True, stream=None):
        """Predictive mean (or None) and full covariance [n_u, n_u] (device
        float64 tensors)."""
        import torch
        Ud = _dev(U, torch)
        ubp = np.ascontiguousarray(np.asarray(u_block_ptr, dtype=np.int64))
        n_u = Ud.shape[0]
        mean = torch.empty(n_u, dtype=torch.float64, device="cuda") if want_mean else None
        cov = torch.empty((n_u, n_u), dtype=torch.float64, device="cuda")
        _check(_lib.lma_predict_cov(self._h, n_u, ctypes.c_void_p(Ud.data_ptr()),
                                    ubp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.c_void_p(mean.data_ptr()) if mean is not None else None,
                                    ctypes.c_void_p(cov.data_ptr()), _stream(torch, stream)))
        return mean, cov

    def lml(self):
        out = ctypes.c_double()
        _check(_lib.lma_state_lml(self._h, ctypes.byref(out)))
        return out.value

    def nbytes(self):
        """Device bytes the state holds."""
        return int(_lib.lma_state_bytes(self._h))

    def chunks(self):
        """Window chunks (1: every window's factor is resident)."""
        return int(_lib.lma_state_chunks(self._h))

    def free(self):
        if self._h:
            _lib.lma_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def fit(X, y, block_ptr, S, B, log_hyp, prior_mean=0.0, precision="fp64", mem_budget=0, stream=None):
    """lma_fit: local and global summaries of the LMA model (Definitions 1-2)."""
    import torch
    load()
    inp = _Inputs(X, y, block_ptr, S, B, log_hyp, prior_mean, precision, mem_budget)
    h = ctypes.c_void_p()
    _check(_lib.lma_fit(ctypes.byref(inp.problem), _stream(torch, stream), ctypes.byref(h)))
    return State(h, inp.problem.M)


def lml(X, y, block_ptr, S, B, log_hyp, prior_mean=0.0, precision="fp64", grad=False, mem_budget=0,
        stream=None):
    """lma_lml: log marginal likelihood (and its gradient in log_hyp)."""
    load()
    inp = _Inputs(X, y, block_ptr, S, B, log_hyp, prior_mean, precision, mem_budget)
    return _lml_call(inp, grad, stream)


def _lml_call(inp, grad, stream=None):
    import torch
    out = ctypes.c_double()
    g = np.zeros(inp.problem.d + 2) if grad else None
    _check(_lib.lma_lml(ctypes.byref(inp.problem), ctypes.byref(out),
                        g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if grad else None,
                        _stream(torch, stream)))
    return (out.value, g) if grad else out.value


class LmlProblem:
    """Training data of an LMA likelihood, uploaded once; call with log_hyp.

    log_hyp = [log l_1..log l_d, log sigma_s^2, log sigma_n^2]."""

    def __init__(self, X, y, block_ptr, S, B, prior_mean=0.0, precision="fp64", mem_budget=0):
        load()
        d = np.asarray(X.shape)[1] if hasattr(X, "shape") else len(X[0])
        self._inp = _Inputs(X, y, block_ptr, S, B, np.zeros(int(d) + 2), prior_mean, precision, mem_budget)
        self.d = int(d)

    def __call__(self, log_hyp, grad=True, stream=None):
        lh = np.ascontiguousarray(np.asarray(log_hyp, dtype=np.float64).reshape(-1))
        if lh.shape[0] != self.d + 2:
            raise ValueError(f"log_hyp must have d+2 = {self.d + 2} entries")
        self._inp.lh = lh
        self._inp.problem.log_hyp = lh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        return _lml_call(self._inp, grad, stream)

    @classmethod
    def from_problem(cls, p, precision="fp64", **kw):
        return cls(p.X, p.y, p.block_ptr, p.S, p.B, p.prior_mean, precision=precision, **kw)


_LML_FN = None


def _lml_function():
    global _LML_FN
    if _LML_FN is None:
        import torch

        class LMALogML(torch.autograd.Function):
            """LML(log_hyp) with the hand-written adjoint as its backward.

            LMALogML.apply(log_hyp, problem) -> 0-d tensor; problem is an LmlProblem."""

            @staticmethod
            def forward(ctx, log_hyp, problem):
                val, g = problem(log_hyp.detach().to("cpu", torch.float64).numpy(), grad=True)
                ctx.save_for_backward(torch.as_tensor(g, dtype=log_hyp.dtype, device=log_hyp.device))
                return torch.tensor(val, dtype=log_hyp.dtype, device=log_hyp.device)

            @staticmethod
            def backward(ctx, grad_out):
                (g,) = ctx.saved_tensors
                return grad_out * g, None

        _LML_FN = LMALogML
    return _LML_FN


def __getattr__(name):
    if name == "LMALogML":
        return _lml_function()
    raise AttributeError(name)


def fit_problem(p, precision="fp64", **kw):
    """fit() for a synthetic Problem object (X, y, block_ptr, S, B, log_hyp, prior_mean)."""
    return fit(p.X, p.y, p.block_ptr, p.S, p.B, p.log_hyp, p.prior_mean, precision=precision, **kw)


def profile_enable(on=True):
    """Bracket every library kernel launch with HIP events (live timing)."""
    load()
    _lib.lma_profile_enable(1 if on else 0)


def profile_read(reset=True):
    load()
    out = Profile()
    _check(_lib.lma_profile_read(ctypes.byref(out), 1 if reset else 0))
    return out.as_dict()


def release_cache():
    """Free the device memory the library keeps for reuse between calls."""
    load()
    _lib.lma_release_cache()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def kmeans_assign(P, C, want_dist=True, stream=None):
    """Nearest centre of each point (include/lma_part.h): (label int32 [n],
    squared distance float64 [n] or None) as device tensors."""
    import torch
    load()
    Pd, Cd = _dev(P, torch), _dev(C, torch)
    n, d = Pd.shape
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    dist2 = torch.empty(n, dtype=torch.float64, device="cuda") if want_dist else None
    _check(_lib.lma_kmeans_assign(_ptr(Pd), n, d, _ptr(Cd), Cd.shape[0], _ptr(label), _ptr(dist2),
                                  _stream(torch, stream)))
    return label, dist2


def kmeans_update(P, label, C, stream=None):
    """Centre update of Lloyd's iteration: (new centres [k, d], counts int64 [k])."""
    import torch
    load()
    Pd = _dev(P, torch)
    Cd = _dev(C, torch).clone()
    lab = torch.as_tensor(label, device="cuda").to(torch.int32).contiguous()
    count = torch.empty(Cd.shape[0], dtype=torch.int64, device="cuda")
    _check(_lib.lma_kmeans_update(_ptr(Pd), Pd.shape[0], Pd.shape[1], _ptr(lab), Cd.shape[0], _ptr(Cd),
                                  _ptr(count), _stream(torch, stream)))
    return Cd, count


def kmeans(P, C0, iters, stream=None):
    """Lloyd's iteration from centres C0: (centres, label, squared distance)."""
    import torch
    load()
    Pd = _dev(P, torch)
    Cd = _dev(C0, torch).clone()
    n = Pd.shape[0]
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    dist2 = torch.empty(n, dtype=torch.float64, device="cuda")
    _check(_lib.lma_kmeans(_ptr(Pd), n, Pd.shape[1], _ptr(Cd), Cd.shape[0], int(iters), _ptr(label), _ptr(dist2),
                           _stream(torch, stream)))
    return Cd, label, dist2


def chain_order(C):
    """Order of the blocks along the Markov chain from their centres (host
    numpy [k, d] -> int32 permutation [k]; no device work)."""
    load()
    Ch = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
    order = np.empty(Ch.shape[0], dtype=np.int32)
    _check(_lib.lma_chain_order(Ch.ctypes.data_as(ctypes.c_void_p), Ch.shape[0], Ch.shape[1],
                                order.ctypes.data_as(ctypes.c_void_p)))
    return order


def version():
    load()
    return _lib.lma_version().decode()


def kmeans_seed(P, k, rand, stream=None):
    """k-means++ seeding: (centres [k, d], point indices int64 [k]) as device
    tensors; rand: k random 32-bit integers (host)."""
    import torch
    load()
    Pd = _dev(P, torch)
    r = np.ascontiguousarray(np.asarray(rand, dtype=np.uint32))
    if r.shape != (k,):
        raise ValueError("rand must hold k values")
    C = torch.empty((k, Pd.shape[1]), dtype=torch.float64, device="cuda")
    idx = torch.empty(k, dtype=torch.int64, device="cuda")
    _check(_lib.lma_kmeans_seed(_ptr(Pd), Pd.shape[0], Pd.shape[1], int(k), r.ctypes.data_as(ctypes.c_void_p),
                                _ptr(C), _ptr(idx), _stream(torch, stream)))
    return C, idx


def bounded_assign(P, C, lo, hi, stream=None):
    """Capacity-bounded assignment: (label int32 [n], count int64 [k]) device
    tensors and the number of proposal rounds."""
    import torch
    load()
    Pd, Cd = _dev(P, torch), _dev(C, torch)
    n, k = Pd.shape[0], Cd.shape[0]
    label = torch.empty(n, dtype=torch.int32, device="cuda")
    count = torch.empty(k, dtype=torch.int64, device="cuda")
    rounds = ctypes.c_int32()
    _check(_lib.lma_bounded_assign(_ptr(Pd), n, Pd.shape[1], _ptr(Cd), k, int(lo), int(hi), _ptr(label),
                                   _ptr(count), ctypes.byref(rounds), _stream(torch, stream)))
    return label, count, int(rounds.value)


def partition(X, M, lo, hi, iters, rand, U=None, stream=None):
    """Block partition (lma_partition): dict with perm, u_perm (device int64),
    block_ptr, u_block_ptr (numpy int64) and centres [M, d] in block order."""
    import torch
    load()
    Xd = _dev(X, torch)
    n, d = Xd.shape
    Ud = _dev(U, torch) if U is not None else None
    n_u = 0 if Ud is None else Ud.shape[0]
    r = np.ascontiguousarray(np.asarray(rand, dtype=np.uint32))
    if r.shape != (M,):
        raise ValueError("rand must hold M values")
    perm = torch.empty(n, dtype=torch.int64, device="cuda")
    u_perm = torch.empty(n_u, dtype=torch.int64, device="cuda")
    bp = np.zeros(M + 1, dtype=np.int64)
    ubp = np.zeros(M + 1, dtype=np.int64)
    cen = torch.empty((M, d), dtype=torch.float64, device="cuda")
    _check(_lib.lma_partition(_ptr(Xd), n, _ptr(Ud) if Ud is not None else None, n_u, d, int(M), int(lo), int(hi),
                              int(iters), r.ctypes.data_as(ctypes.c_void_p), _ptr(perm),
                              bp.ctypes.data_as(ctypes.c_void_p), _ptr(u_perm) if n_u else None,
                              ubp.ctypes.data_as(ctypes.c_void_p), _ptr(cen), _stream(torch, stream)))
    return dict(perm=perm, block_ptr=bp, u_perm=u_perm, u_block_ptr=ubp, centres=cen)
