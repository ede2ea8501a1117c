"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: float64 mode, relative 2-norm error <= 1e-9 per output vector (mean,
variance) and relative error <= 1e-9 on the log marginal likelihood; mixed
mode <= 1e-4 on the same measures."""
import numpy as np
import pytest

import synth
from oracle import lma as olma

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-4}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_fit_predict(lib, p, precision):
    st = lib.fit_problem(p, precision=precision)
    mean, var = st.predict(p.U, p.u_block_ptr)
    out = mean.cpu().numpy(), var.cpu().numpy(), st.lml()
    st.free()
    return out


def check(lib, p, precision, ref=None):
    print(f"case {p.name} n={p.n} d={p.d} M={p.M} s={p.s} B={p.B} n_u={p.n_u} {precision}", flush=True)
    ref = ref or olma.fit_predict(p)
    m, v, l = gpu_fit_predict(lib, p, precision)
    em, ev, el = rel(m, ref["mean"]), rel(v, ref["var"]), abs(l - ref["lml"]) / abs(ref["lml"])
    print(f"  rel err mean {em:.2e} var {ev:.2e} lml {el:.2e}", flush=True)
    tol = TOL[precision]
    assert em <= tol and ev <= tol and el <= tol
    assert np.all(np.isfinite(m)) and np.all(np.isfinite(v))
    return em, ev, el


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("B", [0, 1, 2, 5])
def test_tiny_uneven_blocks_every_order(lib, B, precision):
    """Blocks of 17-40 points (one partial tile each), an empty test block, and
    B from PIC (0) to the full GP (M-1 = 5)."""
    p = synth.make_random(seed=3, n=180, d=2, M=6, s=12, n_u=40, B=B, empty_test_block=2,
                          prior_mean=0.3, name="tiny")
    check(lib, p, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("B", [1, 3])
def test_several_tiles_ragged(lib, B, precision):
    """Blocks of 200-700 points, |S| = 200 (two tiles, ragged), d = 5: windows
    span several 128-row tiles with ragged tails in W_m and D_m."""
    p = synth.make_random(seed=11, n=3000, d=5, M=7, s=200, n_u=600, B=B, uneven=(200, 700),
                          ell_range=(0.3, 1.5), sn2=0.02, name="ragged")
    check(lib, p, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_config0(lib, precision):
    """n=2048, d=4, M=8 blocks of 256, B=1, |S|=64, 256 test points."""
    check(lib, synth.make_config(0), precision)


DEGENERATE = {
    # one block: one window with an empty W_0 (LMA = PIC = the full GP); B is clamped to M - 1
    "one_block": dict(seed=21, n=150, d=3, M=1, s=20, n_u=30, B=0, uneven=(150, 150)),
    "one_block_B3": dict(seed=21, n=150, d=3, M=1, s=20, n_u=30, B=3, uneven=(150, 150)),
    # blocks of a single point, and of one or two points, with empty test blocks
    "single_point_blocks": dict(seed=22, n=12, d=2, M=12, s=4, n_u=10, B=2, uneven=(1, 1)),
    "one_or_two_point_blocks": dict(seed=23, n=30, d=2, M=20, s=5, n_u=15, B=3, uneven=(1, 2)),
    # a support set of one point
    "support_of_one": dict(seed=24, n=300, d=2, M=4, s=1, n_u=40, B=1, uneven=(50, 100)),
    # smallest and largest input dimension
    "d1": dict(seed=25, n=300, d=1, M=5, s=10, n_u=50, B=2, uneven=(40, 80)),
    "d64": dict(seed=26, n=400, d=64, M=4, s=30, n_u=60, B=1, uneven=(80, 120), ell_range=(3.0, 8.0)),
    # B beyond M - 1 (clamped: the full GP)
    "B_beyond_M": dict(seed=27, n=300, d=2, M=4, s=12, n_u=40, B=9, uneven=(50, 100)),
}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_shapes(lib, name, precision):
    """Degenerate shapes of the method: a single block, blocks of one point,
    |S| = 1, d = 1 and d = 64 (the largest supported), B >= M."""
    p = synth.make_random(name=name, **DEGENERATE[name])
    check(lib, p, precision)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mean_only_prediction(lib, precision):
    """lma_predict with var = NULL: the mean alone, equal to the mean of the
    full call and within the bar of the oracle's."""
    p = synth.make_random(seed=29, n=1500, d=3, M=6, s=60, n_u=200, B=2, uneven=(150, 350),
                          empty_test_block=4, name="mean_only")
    ref = olma.fit_predict(p)
    st = lib.fit_problem(p, precision=precision)
    m_only, v_none = st.predict(p.U, p.u_block_ptr, want_var=False)
    m_full, _ = st.predict(p.U, p.u_block_ptr)
    st.free()
    assert v_none is None
    m_only, m_full = m_only.cpu().numpy(), m_full.cpu().numpy()
    assert rel(m_only, ref["mean"]) <= TOL[precision]
    assert np.max(np.abs(m_only - m_full)) <= 1e-12 * np.max(np.abs(m_full))


def test_wide_windows_and_negative_variances(lib):
    """n=16384 in [0,1]^8, M=16 k-means blocks of 1024, |S|=64, B=4: windows of
    5120 points (40 tiles), test points appended to five windows each.  At this
    order the predictive variance of Eq. (4) is negative for a few test points
    (the covariance over training and test points is indefinite between
    B = 0 and B = M - 1); the GPU reports the same values, with the same signs
    wherever the oracle's value is clear of zero."""
    p = synth.make_uniform_kmeans(1, 16384, 8, 16, 4, 64, 4096, 0.05, name="wide")
    order = np.random.default_rng(20150125).permutation(p.n)
    p = p.with_(S=p.X[np.sort(order[:64])].copy())
    ref = olma.fit_predict(p)
    assert np.sum(ref["var"] < 0) >= 1
    for precision in ("fp64", "mixed"):
        check(lib, p, precision, ref)
    _, v, _ = gpu_fit_predict(lib, p, "fp64")
    clear = np.abs(ref["var"]) > 1e-6
    assert np.array_equal(v[clear] < 0, ref["var"][clear] < 0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_band_and_on_the_fly_entries_agree(lib, monkeypatch, precision):
    """Windows that read their residual entries from the shared band (the
    default when B >= 1) and windows that form them in the update kernel
    (LMA_NO_BAND) give the same fit: both within the oracle bar, and within
    rounding of each other."""
    p = synth.make_random(seed=17, n=2600, d=4, M=6, s=150, n_u=300, B=2, uneven=(150, 650),
                          ell_range=(0.3, 1.5), sn2=0.02, name="band")
    ref = olma.fit_predict(p)
    a = gpu_fit_predict(lib, p, precision)
    monkeypatch.setenv("LMA_NO_BAND", "1")
    b = gpu_fit_predict(lib, p, precision)
    monkeypatch.delenv("LMA_NO_BAND")
    for out in (a, b):
        assert rel(out[0], ref["mean"]) <= TOL[precision] and rel(out[1], ref["var"]) <= TOL[precision]
        assert abs(out[2] - ref["lml"]) <= TOL[precision] * abs(ref["lml"])
    agree = {"fp64": 1e-12, "mixed": 1e-6}[precision]
    print(f"  band vs on-the-fly: mean {rel(a[0], b[0]):.2e} var {rel(a[1], b[1]):.2e} "
          f"lml {abs(a[2] - b[2]) / abs(b[2]):.2e}", flush=True)
    assert rel(a[0], b[0]) <= agree and rel(a[1], b[1]) <= agree
    assert abs(a[2] - b[2]) <= agree * abs(b[2])


@pytest.mark.parametrize("precision,B", [("fp64", 2), ("mixed", 2), ("fp64", 0), ("mixed", 6)])
def test_memory_budget_streams_window_factors(lib, precision, B):
    """A memory budget below the resident state's size: the fit keeps one chunk
    of window factors at a time, and prediction and the gradient factor the
    windows again chunk by chunk.  Results match the oracle, and the resident
    path within rounding; a budget that cannot hold one window is an error."""
    p = synth.make_random(seed=23, n=2600, d=3, M=7, s=150, n_u=300, B=B, uneven=(150, 650), name="budget")
    ref = olma.fit_predict(p)
    st = lib.fit_problem(p, precision=precision)
    full, nch = st.nbytes(), st.chunks()
    m0, v0 = (t.cpu().numpy() for t in st.predict(p.U, p.u_block_ptr))
    l0 = st.lml()
    st.free()
    assert nch == 1
    budget = int(0.6 * full)
    st = lib.fit_problem(p, precision=precision, mem_budget=budget)
    nbytes, nch = st.nbytes(), st.chunks()
    m1, v1 = (t.cpu().numpy() for t in st.predict(p.U, p.u_block_ptr))
    l1 = st.lml()
    st.free()
    print(f"  resident {full} bytes; budget {budget}: {nbytes} bytes in {nch} chunks", flush=True)
    assert nch >= 2 and nbytes <= budget
    tol = TOL[precision]
    assert rel(m1, ref["mean"]) <= tol and rel(v1, ref["var"]) <= tol
    assert abs(l1 - ref["lml"]) <= tol * abs(ref["lml"])
    agree = {"fp64": 1e-11, "mixed": 1e-6}[precision]
    print(f"  streamed vs resident: mean {rel(m1, m0):.2e} var {rel(v1, v0):.2e} "
          f"lml {abs(l1 - l0) / abs(l0):.2e}", flush=True)
    assert rel(m1, m0) <= agree and rel(v1, v0) <= agree and abs(l1 - l0) <= agree * abs(l0)
    la, ga = lib.lml(p.X, p.y, p.block_ptr, p.S, p.B, p.log_hyp, p.prior_mean, precision=precision, grad=True)
    lb, gb = lib.lml(p.X, p.y, p.block_ptr, p.S, p.B, p.log_hyp, p.prior_mean, precision=precision, grad=True,
                     mem_budget=budget)
    lo, go = olma.lml_grad(p)
    print(f"  gradient streamed vs resident {rel(gb, ga):.2e}, vs oracle {rel(gb, go):.2e}", flush=True)
    assert abs(lb - la) <= agree * abs(la) and rel(gb, ga) <= 1e3 * agree
    assert abs(lb - lo) <= tol * abs(lo) and rel(gb, go) <= tol
    with pytest.raises(lib.LmaError):
        lib.fit_problem(p, precision=precision, mem_budget=1 << 20)


def test_fp64_is_deterministic(lib):
    p = synth.make_random(seed=5, n=900, d=3, M=5, s=70, n_u=100, B=2, uneven=(100, 250))
    a = gpu_fit_predict(lib, p, "fp64")
    b = gpu_fit_predict(lib, p, "fp64")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_lml_entry_point(lib):
    p = synth.make_random(seed=7, n=500, d=3, M=4, s=40, n_u=0, B=1, uneven=(80, 160))
    ref = olma.lml(p)
    val = lib.lml(p.X, p.y, p.block_ptr, p.S, p.B, p.log_hyp, p.prior_mean)
    assert abs(val - ref) <= 1e-9 * abs(ref)


def test_bad_partition_is_rejected(lib):
    p = synth.make_random(seed=7, n=200, d=2, M=4, s=10, n_u=0, B=1)
    bad = p.block_ptr.copy()
    bad[2] = bad[1]
    with pytest.raises(lib.LmaError) as e:
        lib.fit(p.X, p.y, bad, p.S, p.B, p.log_hyp)
    assert e.value.status == lib.LMA_E_ARG


def test_non_pd_window_reports_its_block(lib):
    """A NaN input makes the residual covariance of the windows that hold it
    non positive definite; the error names a block whose window holds it and
    no NaN result is returned."""
    p = synth.make_random(seed=9, n=400, d=2, M=5, s=16, n_u=0, B=1, uneven=(60, 100))
    X = p.X.copy()
    k = 3
    X[p.block_ptr[k] + 2, 0] = np.nan
    S = p.S.copy()
    # keep the NaN out of the support set
    S[:] = np.nan_to_num(S)
    with pytest.raises(lib.LmaError) as e:
        lib.fit(X, p.y, p.block_ptr, S, p.B, p.log_hyp)
    assert e.value.status == lib.LMA_E_NOT_PD
    assert k - p.B <= e.value.block <= k


def test_non_pd_support_covariance(lib):
    p = synth.make_random(seed=9, n=400, d=2, M=5, s=16, n_u=0, B=1, uneven=(60, 100))
    S = p.S.copy()
    S[3, 1] = np.nan
    with pytest.raises(lib.LmaError) as e:
        lib.fit(p.X, p.y, p.block_ptr, S, p.B, p.log_hyp)
    assert e.value.status == lib.LMA_E_NOT_PD and e.value.block == -1
    # the next call that succeeds names no block
    st = lib.fit(p.X, p.y, p.block_ptr, p.S, p.B, p.log_hyp)
    st.free()
    assert lib.load().lma_failed_block() == -3
