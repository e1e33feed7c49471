"""The BF16 rounding bounds used by the GPU parity tests, checked on the CPU.

Each bound is checked against a numpy emulation of the rounded computation
(FP32 arithmetic, BF16 rounding by the format's definition, rows summed per
block in FP32): the emulation must stay inside the bound, and the same
emulation with a planted mistake (a dropped term, a wrong sign) must not.
"""
import numpy as np
import pytest

from bf16_ref import (_classic_rows, bf16_round, classic_bf16_bound, classic_magnitude,
                      classic_row_square_sum, classic_rows_per_block, z16_like_kernel)
from oracle import tlda_oracle as O
from synth import make_csr_rows

F32 = np.float32


def _rows(n, V, seed):
    rng = np.random.default_rng(seed)
    rows = [{}, {3: 1, 9: 1}, {5: 2}, {7: 3}]
    while len(rows) < n:
        words = rng.choice(V, size=int(rng.integers(1, 40)), replace=False)
        rows.append({int(w): int(rng.integers(1, 4)) for w in words})
    return make_csr_rows(rows[:n], V)


def _emulate(rp, ci, va, W16, Phi, m, alpha0, nblk, plant=None):
    """The BF16 classic kernel's arithmetic in numpy: Z16 = bf16(fp32 W16 Phi),
    per-document sums and coefficients in FP32, reduction rows rounded to
    BF16, each block's rows and mean terms summed in FP32, blocks in FP64."""
    c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0
    c2 = alpha0 * (alpha0 + 1.0) / 2.0
    c2r, a0r = F32(c2 / c3), F32(alpha0 ** 2 / c3)
    Z = z16_like_kernel(W16, Phi).astype(F32)
    mw = (W16.T @ m).astype(F32)
    r = (mw @ Phi.astype(F32)).astype(F32)
    n = rp.size - 1
    K = Phi.shape[1]
    al, be, ga, e = (np.zeros((n, K), F32) for _ in range(4))
    for d in range(n):
        a, b = int(rp[d]), int(rp[d + 1])
        v, z = va[a:b].astype(F32), Z[ci[a:b]]
        L = F32(v.sum())
        if L < 3:
            continue
        s = (v[:, None] * z).sum(axis=0, dtype=F32)
        q = (v[:, None] * z * z).sum(axis=0, dtype=F32)
        l2 = F32(1.0) / (L * (L - F32(1.0)))
        l3 = l2 / (L - F32(2.0))
        al[d] = l3 * (s * s - q) - F32(2.0) * c2r * l2 * r * s
        be[d] = F32(-2.0) * l3 * s + F32(2.0) * c2r * l2 * r
        ga[d] = F32(2.0) * l3
        e[d] = -c2r * l2 * (s * s - q) + a0r * r * r
        if plant == "sign":
            be[d] = -be[d]
    if plant == "mean":
        e[:] = 0
    doc = np.repeat(np.arange(n), np.diff(rp))
    z = Z[ci]
    o = va.astype(F32)[:, None] * ((ga[doc] * z + be[doc]) * z + al[doc])
    o = bf16_round(o).astype(F32)
    W32 = W16.astype(F32)
    out = np.zeros((W16.shape[1], K))
    ntiles = (n + 15) // 16
    for blk in range(nblk):
        docs = np.concatenate([np.arange(t * 16, min(n, t * 16 + 16))
                               for t in range(blk, ntiles, nblk)] or [np.zeros(0, int)])
        if docs.size == 0:
            continue
        sel = np.isin(doc, docs)
        part = W32[ci[sel]].T @ o[sel] + np.outer(mw, e[docs].sum(axis=0, dtype=F32))
        out += part.astype(F32).astype(np.float64)
    return c3 * out


@pytest.mark.parametrize("D,K,n,nblk", [(5, 5, 600, 7), (20, 30, 400, 3), (50, 50, 300, 5)])
def test_classic_bf16_bound_covers_the_rounded_computation(D, K, n, nblk):
    V = 300
    rp, ci, va = _rows(n, V, D + K)
    rng = np.random.default_rng(D * K)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    W16 = bf16_round(Q * rng.uniform(5, 30, size=D)[None, :])
    m = rng.dirichlet(np.ones(V))
    Phi = rng.standard_normal((D, K)).astype(F32) * F32(0.3)
    P64 = Phi.astype(np.float64)
    a0 = 1.5
    Z16 = z16_like_kernel(W16, Phi)
    ref, n_kept = O.classic_data_term(rp, ci, va, V, m, W16, P64, a0, Z=Z16)
    bound = classic_bf16_bound(rp, ci, va, W16, Z16, P64, m, a0, min_blocks=nblk)
    got = _emulate(rp, ci, va, W16, Phi, m, a0, nblk)
    err = np.abs(got - ref)
    assert (err <= bound).all()
    # not vacuous: well inside the data term, and the emulation's error is
    # a visible share of it
    scale = np.abs(ref).max()
    print(f"bound max {bound.max() / scale:.3g}, error max {err.max() / scale:.3g} of max |data|")
    assert bound.max() < 0.05 * scale and err.max() > 0.01 * bound.max()
    for plant in ("sign", "mean"):
        bad = _emulate(rp, ci, va, W16, Phi, m, a0, nblk, plant=plant)
        assert (np.abs(bad - ref) > bound).any(), plant


def test_classic_magnitude_sums_the_terms_document_by_document():
    """The grouped row form of the magnitude sum against the nine terms of
    the data term written per document with magnitudes (y = |W|^T c,
    s = c.|z|, g = |W|^T (c |z|), q = c.z^2, h = |W|^T (c z^2)), and the
    triangle inequality |data term| <= magnitude sum."""
    V, D, K, a0 = 60, 4, 3, 1.3
    rp, ci, va = _rows(120, V, 5)
    rng = np.random.default_rng(1)
    W = rng.standard_normal((V, D))
    Phi = rng.standard_normal((D, K))
    m = rng.dirichlet(np.ones(V))
    Wa, Za = np.abs(W), np.abs(W @ Phi)
    mw = W.T @ m
    ra = np.abs(mw @ Phi)
    c3, c2 = (a0 + 1) * (a0 + 2) / 2, a0 * (a0 + 1) / 2
    want = np.zeros((D, K))
    for d in range(rp.size - 1):
        a, b = int(rp[d]), int(rp[d + 1])
        cnt, cols = va[a:b].astype(float), ci[a:b]
        L = cnt.sum()
        if L < 3:
            continue
        l2 = 1 / (L * (L - 1))
        l3 = l2 / (L - 2)
        y = Wa[cols].T @ cnt
        s = cnt @ Za[cols]
        g = Wa[cols].T @ (cnt[:, None] * Za[cols])
        q = cnt @ Za[cols] ** 2
        h = Wa[cols].T @ (cnt[:, None] * Za[cols] ** 2)
        want += c3 * l3 * (np.outer(y, s * s) + 2 * s * g + np.outer(y, q) + 2 * h)
        want += c2 * l2 * (2 * ra * (np.outer(y, s) + g) + np.outer(np.abs(mw), s * s + q))
        want += a0 ** 2 * np.outer(np.abs(mw), ra * ra)
    got = classic_magnitude(rp, ci, va, Wa, Za, np.abs(mw), ra, a0)
    np.testing.assert_allclose(got, want, rtol=1e-12)
    data, _ = O.classic_data_term(rp, ci, va, V, m, W, Phi, a0)
    assert (np.abs(data) <= got).all()


def test_classic_rows_add_up_to_the_data_term():
    """The signed reduction rows W_w (x) o_w plus m_w (x) e_d summed over the
    batch give the oracle's data term, and their entry-wise square sum
    matches a loop over the nonzeros."""
    V, D, K, a0 = 60, 4, 3, 0.8
    rp, ci, va = _rows(150, V, 9)
    rng = np.random.default_rng(2)
    W = rng.standard_normal((V, D))
    Phi = rng.standard_normal((D, K))
    m = rng.dirichlet(np.ones(V))
    mw = W.T @ m
    r = mw @ Phi
    total = np.zeros((D, K))
    sq = np.zeros((D, K))
    for cols, row, e in _classic_rows(rp, ci, va, W @ Phi, r, a0, sign=True, chunk=37):
        total += W[cols].T @ row + np.outer(mw, e.sum(axis=0))
        for j, w in enumerate(cols):
            sq += np.outer(W[w], row[j]) ** 2
    data, _ = O.classic_data_term(rp, ci, va, V, m, W, Phi, a0)
    np.testing.assert_allclose(total, data, rtol=1e-10, atol=1e-12 * np.abs(data).max())
    np.testing.assert_allclose(classic_row_square_sum(rp, ci, va, W, W @ Phi, r, a0), sq,
                               rtol=1e-12)


def test_rows_per_block_bound():
    rp = np.concatenate([[0], np.cumsum(np.arange(1, 41))])     # 40 documents, 1..40 words
    rows, docs = classic_rows_per_block(rp, tile=16, min_blocks=2)
    # 3 tiles over 2 blocks: the largest two tiles (docs 16-31 and 32-39)
    assert docs == 32 and rows == int(np.arange(17, 33).sum() + np.arange(33, 41).sum())
