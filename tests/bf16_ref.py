"""Helpers for the BF16 parity tests: the format's rounding, the oracle's
gradient on BF16-rounded operands, and the magnitude sums of the derived
rounding bound (see tests/test_gpu_bf16.py for the derivation).

With u = 2^-8 the BF16 unit roundoff, B = |X|^T S^2 and
C = |X|^T (|S| (|X| |Phi|)) (X, Phi rounded, S = X Phi), both scaled by the
gradient's 3 c3 / n:
  * the step from FP32 X (tlda_cp_step) stays within 2u B + D 2^-23 C;
  * a fused step (whitening kept on chip, X rounded from the kernel's own
    FP32 row, which may differ from the oracle's in the last bit and so round
    to the neighbouring BF16 value) stays within 4u (B + C);
plus 2^-22 |ref| for the FP32 penalty term and the final rounding.
"""
import numpy as np

from oracle import tlda_oracle as O

U_BF16 = 2.0 ** -8


def bf16_round(a):
    """Nearest BF16 value of fp32(a), ties to even (the format's definition:
    keep the upper 16 bits of the FP32 pattern after adding half an ulp)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rounded_gradient(X, Phi, n, alpha0, theta):
    """Oracle gradient with the data term on BF16-rounded X and Phi and the
    penalty term on the FP32 Phi; plus the scaled magnitude sums B and C."""
    Xh, Ph = bf16_round(X), bf16_round(Phi)
    Phi64 = np.asarray(Phi, dtype=np.float64)
    zero = np.zeros((1, Phi.shape[0]))
    pen = O.cp_gradient(zero, Phi64, n, alpha0, theta)
    data = O.cp_gradient(Xh, Ph, n, alpha0, theta) - O.cp_gradient(zero, Ph, n, alpha0, theta)
    S = Xh @ Ph
    B = np.abs(Xh).T @ (S * S)
    C = np.abs(Xh).T @ (np.abs(S) * (np.abs(Xh) @ np.abs(Ph)))
    scale = 3.0 * (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0 / max(n, 1)
    return pen + data, scale * B, scale * C


def fused_bound(ref, B, C):
    """Element-wise bound of a fused BF16 step's gradient against `ref`."""
    return 4 * U_BF16 * (B + C) + 2.0 ** -22 * np.abs(ref)


def assert_within(got, ref, bound, what):
    excess = np.abs(np.asarray(got, dtype=np.float64) - ref) - bound
    worst = float(excess.max())
    assert worst <= 0.0, f"{what}: exceeds the rounding bound by {worst:g}"


# --------------------------------------------------------------------------
# Classic rung in BF16.  The kernel accumulates the data term
# (oracle.classic_data_term) from rows W16_w (x) bf16(o_w), o_w =
# c_w (a_d + b_d z_w + g_d z_w^2), plus m_w (x) e_d, with the scores z taken
# from Z16 = bf16(W16 Phi) (an FP32 dot product over d in order, then rounded).
# The reference is the oracle on W16 and that same Z16 (`z16_like_kernel`);
# what remains is
#   * the rounding of each row o_w to BF16: independent errors of at most
#     u |o_w|, so by Hoeffding's inequality their sum stays within
#     lam u sqrt(sum_w (W16_w o_w)^2) except with probability
#     2 exp(-lam^2 / 2) per entry (the probabilistic model of rounding errors
#     of Higham and Mary, 2019; lam = 8: 2.5e-14);
#   * FP32 accumulation of a block's R rows and T documents: at most R + T
#     roundings of 2^-24 of a partial sum bounded by the magnitude sum Mag,
#     within lam 2^-24 sqrt(R + T) Mag by the same argument;
#   * FP32 evaluation of s, q, r and the coefficients: at most Lmax + D + 64
#     roundings along a chain, each bounded by Mag.
# Mag is the data term with every factor replaced by its magnitude; the
# implicit form cancels heavily (Mag is tens of times |data term|), which is
# why a worst-case bound u Mag would be vacuous here.
# --------------------------------------------------------------------------
LAMBDA = 8.0


def z16_like_kernel(W16, Phi):
    """bf16 of the FP32 dot product sum_d W16[w, d] Phi[d, k] taken in order of
    d with fused multiply-adds (the product of a BF16 and an FP32 value is
    exact in FP64, and so, to within a double rounding that needs a tie at
    2^-29 odds, is the FP64 sum rounded to FP32)."""
    W = np.asarray(W16, dtype=np.float64)
    P = np.asarray(Phi, dtype=np.float32).astype(np.float64)
    s = np.zeros((W.shape[0], P.shape[1]), dtype=np.float32)
    for d in range(W.shape[1]):
        s = (W[:, d:d + 1] * P[d][None, :] + s.astype(np.float64)).astype(np.float32)
    return bf16_round(s)


def _classic_rows(rp, ci, va, Z, r, alpha0, sign, chunk=16384):
    """Per nonzero (in chunks of documents): the reduction row o (or its
    magnitude bound when sign is False) and, per document, e; Z holds the
    scores (or their magnitudes)."""
    rp = np.asarray(rp, dtype=np.int64)
    ci = np.asarray(ci, dtype=np.int64)
    va = np.asarray(va, dtype=np.float64)
    n = rp.size - 1
    c3 = (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0
    c2 = alpha0 * (alpha0 + 1.0) / 2.0
    csum = np.concatenate([[0.0], np.cumsum(va)])
    L = csum[rp[1:]] - csum[rp[:-1]]
    keep = L >= 3
    Ls = np.where(keep, L, 3.0)
    l2 = np.where(keep, 1.0 / (Ls * (Ls - 1.0)), 0.0)
    l3 = np.where(keep, l2 / (Ls - 2.0), 0.0)
    K = Z.shape[1]
    t = 1.0 if sign else -1.0          # magnitudes: every minus sign becomes a plus
    for d0 in range(0, n, chunk):
        d1 = min(n, d0 + chunk)
        a, b = int(rp[d0]), int(rp[d1])
        if a == b:
            continue
        cols, v = ci[a:b], va[a:b]
        doc = np.repeat(np.arange(d0, d1), np.diff(rp[d0:d1 + 1]))
        z = Z[cols]
        vz = v[:, None] * z
        cz = np.vstack([np.zeros((1, K)), np.cumsum(vz, axis=0)])
        cq = np.vstack([np.zeros((1, K)), np.cumsum(vz * z, axis=0)])
        lo, hi = rp[d0:d1] - a, rp[d0 + 1:d1 + 1] - a
        s, q = cz[hi] - cz[lo], cq[hi] - cq[lo]
        S, Q = s[doc - d0], q[doc - d0]
        L2, L3 = l2[doc][:, None], l3[doc][:, None]
        row = v[:, None] * (2.0 * c3 * L3 * z * z
                            + t * (-2.0 * c3 * L3 * S + t * 2.0 * c2 * L2 * r[None, :]) * z
                            + c3 * L3 * (S * S - t * Q) - t * 2.0 * c2 * L2 * r[None, :] * S)
        e = keep[d0:d1, None] * (-t * c2 * l2[d0:d1, None] * (s * s - t * q)
                                 + alpha0 ** 2 * r[None, :] ** 2)
        yield cols, row, e


def classic_magnitude(rp, ci, va, Wa, Za, mwa, ra, alpha0):
    """The classic data term with every factor replaced by a magnitude:
    c3 l3 (y s^2 + 2 s g + y q + 2 h) + c2 l2 (2 r (y s + g) + m_w (s^2 + q))
    + alpha0^2 m_w r^2, with s, g, q, h, y summed from |W| = Wa (V x D), score
    magnitudes Za (V x K), mwa >= |W^T M1| (D) and ra >= |r| (K), grouped as
    the kernel's reduction rows.  Returns D x K."""
    out = np.zeros((Wa.shape[1], Za.shape[1]))
    esum = np.zeros(Za.shape[1])
    for cols, row, e in _classic_rows(rp, ci, va, Za, ra, alpha0, sign=False):
        out += Wa[cols].T @ row
        esum += e.sum(axis=0)
    return out + np.outer(mwa, esum)


def classic_row_square_sum(rp, ci, va, W16, Z16, r, alpha0):
    """sum over nonzeros of (W16_w (x) o_w)^2, entry by entry (D x K)."""
    out = np.zeros((W16.shape[1], Z16.shape[1]))
    W2 = np.asarray(W16, dtype=np.float64) ** 2
    for cols, row, _ in _classic_rows(rp, ci, va, Z16, r, alpha0, sign=True):
        out += W2[cols].T @ (row * row)
    return out


def classic_rows_per_block(rp, tile=16, min_blocks=256):
    """Upper bounds on the reduction rows and documents that one block of the
    classic kernel accumulates: tiles of `tile` documents are dealt to
    min(tiles, >= min_blocks) blocks in turn."""
    rp = np.asarray(rp, dtype=np.int64)
    n = rp.size - 1
    nt = max(1, (n + tile - 1) // tile)
    ends = np.minimum(np.arange(1, nt + 1) * tile, n)
    per_tile = rp[ends] - rp[np.arange(nt) * tile]
    tpb = -(-nt // min(nt, min_blocks))
    return int(np.sort(per_tile)[::-1][:tpb].sum()), tile * tpb


def classic_bf16_bound(rp, ci, va, W16, Z16, Phi, m, alpha0, min_blocks=256):
    """Entry-wise bound on |data_gpu - data_ref| (D x K, in the data term's
    units) for the BF16 classic kernel against the oracle's data term on W16
    and Z16 = z16_like_kernel(W16, Phi) (see the derivation above)."""
    u = U_BF16
    D = W16.shape[1]
    P = np.asarray(Phi, dtype=np.float64)
    mw = W16.T @ m
    r = mw @ P
    mag = classic_magnitude(rp, ci, va, np.abs(W16), np.abs(Z16), np.abs(mw), np.abs(r), alpha0)
    sq = classic_row_square_sum(rp, ci, va, W16, Z16, r, alpha0)
    rows, docs = classic_rows_per_block(rp, min_blocks=min_blocks)
    lmax = int(np.diff(np.asarray(rp, dtype=np.int64)).max(initial=0))
    return (LAMBDA * u * (1 + u) * np.sqrt(sq)
            + LAMBDA * 2.0 ** -24 * np.sqrt(rows + docs) * mag
            + (lmax + D + 64) * 2.0 ** -24 * mag)
