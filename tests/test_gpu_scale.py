"""Whitening refresh at vocabulary scale against the FP64 oracle.

The refresh (section "Online Decomposition of the Second Moment": W with
W^T M2~ W = I from the top-D eigenpairs of the centred second moment) is run
on one full 131 072-document batch of the tweet-shaped workload (V = 20 000),
where the Gram products Q^T Y split their rows into 256 chunks and the
products with the V x V accumulator take their full size.  The oracle applies
M2~ as an operator over the sparse frequency rows and takes its top
eigenpairs by Lanczos iteration (`whitening_operator`, pinned to the dense
eigendecomposition in tests/test_oracle_pins.py).

Bars: integer statistics bit-exact; M1 within 1e-16 of the definition
summed in extended precision (the library's sums are exact); eigenvalues within
1e-10 of the largest; columns of W within 1e-7 relative wherever an
eigenvalue's gap to its neighbours exceeds 1e-7 of the largest (all of them
here); W^T M2~ W = I within 1e-8, with M2~ W formed from the CSR rows.
The subspace iteration runs enough iterations to converge to those bars:
the ratio lambda_{p+1} / lambda_D is about 0.75 (D = 50, p = 100) and 0.57
(D = 100, p = 200) on this corpus.
"""
import numpy as np
import pytest

from oracle import tlda_oracle as O
from synth import SPECS, generate, iter_batches

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")


@pytest.fixture(scope="module")
def tweet_batch():
    spec = SPECS["c2"]
    c = generate(spec, n_docs=spec.batch)
    rp, ci, va, _ = next(iter_batches(c))
    W, lam, U, m, N = O.whitening_operator([(rp, ci, va)], spec.V, 100, spec.alpha0, extra=10)
    st = O.batch_stats(rp, ci, va, spec.V)
    # M1 = (1/N) sum_d f_d with each f_d = c / L in FP64 and the sums in
    # extended precision: the library accumulates M1 exactly, and the
    # oracle's FP64 column sums (about 65 000 terms for the hottest words)
    # carry rounding errors up to a few 1e-13 of their value
    L = np.add.reduceat(va.astype(np.float64), rp[:-1].astype(np.int64))
    L[np.diff(rp) == 0] = 0.0
    rows = np.repeat(np.arange(rp.size - 1), np.diff(rp))
    keep = L[rows] >= 3
    acc = np.zeros(spec.V, dtype=np.longdouble)
    np.add.at(acc, ci[keep], (va[keep].astype(np.float64) / L[rows][keep]).astype(np.longdouble))
    m_exact = (acc / N).astype(np.float64)
    np.testing.assert_allclose(m, m_exact, rtol=1e-12, atol=1e-16)
    return {"spec": spec, "batch": (rp, ci, va), "W": W, "lam": lam, "U": U, "m": m, "N": N,
            "stats": st, "m_exact": m_exact}


@pytest.mark.parametrize("route", ["default", "vector"])
@pytest.mark.parametrize("D,iters", [(50, 150), (100, 100)])
def test_refresh_at_vocabulary_scale_matches_oracle(tweet_batch, D, iters, route, monkeypatch):
    """route: the refresh's dense products on the default route, or on the
    library's vector-ALU tile kernel (TLDA_TUNE_GEMM=1)."""
    if route == "vector":
        monkeypatch.setenv("TLDA_TUNE_GEMM", "1")
    spec = tweet_batch["spec"]
    rp, ci, va = tweet_batch["batch"]
    ctx = tl.tlda_create(spec.V, D, D, spec.alpha0, eig_iters=iters)
    tl.tlda_update_moments(ctx, tl.CsrBatch.from_numpy(rp, ci, va), tl.TLDA_REFRESH_W)
    N, skipped, totals = tl.tlda_get_stats(ctx)
    st = tweet_batch["stats"]
    assert N == st["n_kept"] == tweet_batch["N"] and skipped == st["n_skipped"]
    assert np.array_equal(totals, st["token_totals"])
    W, eig, m = tl.tlda_get_whitening(ctx)
    np.testing.assert_allclose(m, tweet_batch["m_exact"], rtol=0, atol=1e-16)
    lam = tweet_batch["lam"][:D]
    assert np.abs(eig - lam).max() <= 1e-10 * lam[0]
    gaps = np.minimum(np.r_[np.inf, -np.diff(tweet_batch["lam"])],
                      np.r_[-np.diff(tweet_batch["lam"]), np.inf])[:D]
    wide = gaps > 1e-7 * lam[0]
    assert wide.all()
    W_ref = tweet_batch["W"][:, :D]
    col_err = np.linalg.norm(W - W_ref, axis=0) / np.linalg.norm(W_ref, axis=0)
    assert col_err.max() < 1e-7, (int(np.argmax(col_err)), float(col_err.max()))
    # W^T M2~ W = (alpha0 + 1)/N X^T X with X the oracle's whitening of the
    # batch by this W (dropped rows zero): the identity from the CSR rows
    X = O.whiten_csr(rp, ci, va, spec.V, m, W)
    np.testing.assert_allclose((spec.alpha0 + 1.0) / N * (X.T @ X), np.eye(D), atol=1e-8)
