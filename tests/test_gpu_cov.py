"""Full predictive covariance on the GPU (lma_predict_cov, Theorem 2's
Sigma^LMA_UU / Eq. (4) beyond the diagonal) against the oracle: the dense
definition for small problems, the oracle's window form (pinned to the dense
definition) for larger ones.  Bars as for the variance: float64 within 1e-9
and mixed within 1e-4, both for the relative Frobenius error and for the
largest entry error relative to the largest entry; the diagonal equals
lma_predict's variance and the mean lma_predict's mean."""
import numpy as np
import pytest

import synth
from oracle import dense
from oracle import lma as olma

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 1e-4}


def errs(a, b):
    fro = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    ent = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    return fro, ent


def run(lib, p, precision, ref_cov, ref_mean, mem_budget=0):
    print(f"case {p.name} n={p.n} M={p.M} s={p.s} B={p.B} n_u={p.n_u} {precision}", flush=True)
    st = lib.fit_problem(p, precision=precision, mem_budget=mem_budget)
    mean, cov = st.predict_cov(p.U, p.u_block_ptr)
    m2, v2 = st.predict(p.U, p.u_block_ptr)
    nch = st.chunks()
    st.free()
    mean, cov, m2, v2 = (t.cpu().numpy() for t in (mean, cov, m2, v2))
    fro, ent = errs(cov, ref_cov)
    em = float(np.linalg.norm(mean - ref_mean) / np.linalg.norm(ref_mean))
    diag = float(np.max(np.abs(np.diag(cov) - v2)) / np.max(np.abs(v2)))
    print(f"  cov rel Frobenius {fro:.2e}, max entry {ent:.2e}; mean {em:.2e}; diag vs variance {diag:.2e}; "
          f"chunks {nch}", flush=True)
    tol = TOL[precision]
    assert fro <= tol and ent <= tol and em <= tol
    assert diag <= 1e-12
    assert np.max(np.abs(mean - m2)) <= 1e-12 * np.max(np.abs(m2))
    return cov, nch


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("B", [0, 1, 2, 5])
def test_against_the_dense_definition(lib, B, precision):
    """Blocks of 17-40 points, an empty test block, support set off the data;
    B from PIC (0) to the full GP (M-1 = 5)."""
    p = synth.make_random(seed=31, n=180, d=2, M=6, s=12, n_u=60, B=B, empty_test_block=3,
                          prior_mean=0.2, s_from_X=False, name="cov_tiny")
    ref_mean, ref_cov = dense.predict(p, full_cov=True)
    run(lib, p, precision, ref_cov, ref_mean)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("B", [1, 3])
def test_several_tiles_ragged(lib, B, precision):
    """Blocks of 200-700 points, |S| = 200, 600 test points: pair tiles span
    several test tiles per block with ragged tails, windows of several tiles."""
    p = synth.make_random(seed=11, n=3000, d=5, M=7, s=200, n_u=600, B=B, uneven=(200, 700),
                          ell_range=(0.3, 1.5), sn2=0.02, empty_test_block=4, name="cov_ragged")
    ref_mean, ref_cov = olma.predict_cov(p)
    run(lib, p, precision, ref_cov, ref_mean)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_far_pairs_carry_only_the_low_rank_term(lib, precision):
    """M=12, B=2: most pairs of test blocks are more than B apart; their GPU
    entries are the oracle's within the bar (they are the low-rank term alone),
    and the in-band entries too."""
    p = synth.make_random(seed=41, n=1200, d=3, M=12, s=40, n_u=240, B=2, uneven=(60, 140),
                          name="cov_far")
    ref_mean, ref_cov = olma.predict_cov(p)
    cov, _ = run(lib, p, precision, ref_cov, ref_mean)
    ublk = np.repeat(np.arange(p.M), np.diff(p.u_block_ptr))
    far = np.abs(ublk[:, None] - ublk[None, :]) > p.B
    scale = np.max(np.abs(ref_cov))
    assert np.max(np.abs(cov[far] - ref_cov[far])) <= TOL[precision] * scale


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_memory_budget_streams_windows(lib, precision):
    """Window factors held one chunk at a time: the whitened products of each
    chunk are added after its solves; the result matches the oracle."""
    p = synth.make_random(seed=23, n=2600, d=3, M=7, s=150, n_u=300, B=2, uneven=(150, 650), name="cov_budget")
    ref_mean, ref_cov = olma.predict_cov(p)
    st = lib.fit_problem(p, precision=precision)
    full = st.nbytes()
    st.free()
    _, nch = run(lib, p, precision, ref_cov, ref_mean, mem_budget=int(0.6 * full))
    assert nch >= 2


def test_mean_optional_and_empty_test_set(lib):
    p = synth.make_random(seed=5, n=400, d=2, M=4, s=20, n_u=50, B=1, uneven=(80, 120), name="cov_opt")
    ref_mean, ref_cov = olma.predict_cov(p)
    st = lib.fit_problem(p, precision="fp64")
    mean, cov = st.predict_cov(p.U, p.u_block_ptr, want_mean=False)
    assert mean is None
    assert errs(cov.cpu().numpy(), ref_cov)[0] <= 1e-9
    _, cov0 = st.predict_cov(np.zeros((0, p.d)), np.zeros(p.M + 1, dtype=np.int64))
    assert cov0.shape == (0, 0)
    with pytest.raises(lib.LmaError) as e:
        bad = p.u_block_ptr.copy()
        bad[1] = bad[2] + 1
        st.predict_cov(p.U, bad)
    assert e.value.status == lib.LMA_E_ARG
    st.free()
