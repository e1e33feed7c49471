"""Plain, slow, FP64 CPU oracle of the online tensor-LDA hot path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code,
constants or helpers with the HIP library.

Every function follows one passage of the paper (arXiv 2511.07809), written out
in the paper's order and notation in double precision, with dense matrices and
no blocking or fusion.  Readings of passages that are ambiguous or garbled are
named where they are used (R1..R9 below); the pins that tie each function to
something other than itself live in tests/test_oracle_pins.py.

Readings
  R1  f_i is the frequency vector c_i / L_i of a document (notation table), so
      that mu_i = nu_i + M1 is a word distribution.
  R2  Documents with fewer than three tokens are dropped (pre-processing list in
      the package section); N counts kept documents only, and dropped rows of a
      whitened batch are zero and excluded from the gradient's batch mean.
  R3  The centred second moment uses 1/N with the sum over i = 1..N.
  R4  W is defined by W^T M2~ W = I (online second-moment section): W = U diag(l)^-1/2
      from the top-D eigenpairs of M2~; the printed closed form with a
      sqrt(alpha0 + 1)/N factor contradicts that identity and is not used.
      Eigenpairs are ordered by decreasing eigenvalue and each eigenvector is
      signed so that its entry of largest magnitude is positive.
  R5  The whitened vector of a document is x = W^T (f - M1), a D-vector.
  R6  The gradient's 1/n is the number of kept documents of the batch.
  R7  Recovery (post-processing section): for centred moments the population
      identities E[M2~] = sum a_i nu_i nu_i^T and sum a_i nu_i = 0 (a_i =
      alpha_i / alpha0) make the whitened factors v_i = W^T nu_i a tight frame
      with a_i |v_i|^2 = 1 - a_i.  A converged CP factor equals
      (a_i / (1 + theta))^(1/3) v_i, so with w_i = (1 + theta)^(1/3) phi_i the
      weight a_i is the root in (0, 1) of a^(1/3) |w_i|^2 + a = 1,
      nu_i = (W^T)^+ a_i^(-1/3) w_i, mu_i = nu_i + M1 and alpha_i = a_i / sum a.
  R8  Inference (the package's document-topic output): theta_d is the
      minimiser over the probability simplex of |x_d - A theta|^2 with
      A = W^T (mu - M1 1^T), found by projected gradient with step 1/|A^T A|_2.
  R9  Appendix cumulants: per-document pair and triple sums are normalised by
      L(L-1) and L(L-1)(L-2) (ordered distinct tokens), and the alpha0 term of
      M3 multiplies the pair moment by M1 (the form the theorem's proof uses).
  R14 Classic rung: the SGD of the batched section run on the appendix's
      alpha0-corrected moments (R9) instead of the centred ones.  W whitens
      M2 = (alpha0+1) mean P2 - alpha0 M1 M1^T; the data term of the gradient
      is the per-document piece of M3 contracted implicitly with (W, phi, phi);
      recovery is the orthogonal one of the post-processing section:
      lambda_i = (1+theta)|phi_i|^3, mu_i = lambda_i (W^T)^+ phi_i/|phi_i|,
      alpha_i proportional to lambda_i^-2.
  R15 Fully online mode: the paper keeps Phi across batches while W changes
      and does not say how Phi is carried over.  Phi is re-based as
      Phi_new = W_new^T (W_old^T)^+ Phi_old (the factors' centred word-space
      vectors seen through the new whitening; the shift of M1 between batches
      is not carried, it is O(batch / N)).  The incremental PCA is read as the
      top-D eigenpairs of the running M2~ over every batch seen so far, which
      is what an incremental PCA of the centred data tracks.
"""
from __future__ import annotations

import itertools
from typing import Iterable, Sequence

import numpy as np

__all__ = [
    "doc_lengths", "batch_stats", "frequency_rows", "first_moment",
    "centered_second_moment", "centered_second_moment_merged", "whitening",
    "whiten", "cp_gradient", "cp_gradient_explicit", "cp_loss", "cp_step",
    "unwhiten", "simplex_project", "infer_doc_topics", "match_topics",
    "uncentered_cumulants", "whitened_tensor", "tensor_power_method",
    "classic_recover", "fit_batched", "classic_second_moment", "classic_data_term",
    "classic_cp_gradient", "classic_unwhiten", "fit_batched_classic", "rebase_phi",
    "fit_online",
]


# --------------------------------------------------------------------------
# Integer statistics (R2): exact, independent of batching.
# --------------------------------------------------------------------------
def doc_lengths(row_ptr: np.ndarray, val: np.ndarray) -> np.ndarray:
    """L_d = sum of the document's counts, as exact integers."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    counts = np.asarray(val).astype(np.int64)
    L = np.zeros(row_ptr.shape[0] - 1, dtype=np.int64)
    for d in range(L.shape[0]):
        L[d] = int(counts[row_ptr[d]:row_ptr[d + 1]].sum())
    return L


def batch_stats(row_ptr, col_idx, val, V: int) -> dict:
    """Kept/skipped document counts and per-word token totals of kept documents."""
    L = doc_lengths(row_ptr, val)
    keep = L >= 3
    totals = np.zeros(V, dtype=np.int64)
    counts = np.asarray(val).astype(np.int64)
    for d in np.nonzero(keep)[0]:
        for j in range(int(row_ptr[d]), int(row_ptr[d + 1])):
            totals[int(col_idx[j])] += int(counts[j])
    return {"n_rows": int(L.shape[0]), "n_kept": int(keep.sum()),
            "n_skipped": int((~keep).sum()), "L": L, "keep": keep,
            "token_totals": totals}


def frequency_rows(row_ptr, col_idx, val, V: int) -> np.ndarray:
    """Dense n x V matrix of frequency vectors f_d = c_d / L_d (R1); rows of
    dropped documents (R2) are zero."""
    L = doc_lengths(row_ptr, val)
    n = L.shape[0]
    F = np.zeros((n, V), dtype=np.float64)
    for d in range(n):
        if L[d] < 3:
            continue
        for j in range(int(row_ptr[d]), int(row_ptr[d + 1])):
            F[d, int(col_idx[j])] += float(val[j]) / float(L[d])
    return F


# --------------------------------------------------------------------------
# Centred cumulants (section "Computing the Centered Cumulants").
# --------------------------------------------------------------------------
def first_moment(batches: Iterable[Sequence], V: int) -> tuple[np.ndarray, int]:
    """M1 = (1/N) sum_i f_i over the kept documents of all batches."""
    total = np.zeros(V)
    N = 0
    for rp, ci, va in batches:
        st = batch_stats(rp, ci, va, V)
        F = frequency_rows(rp, ci, va, V)
        total += F[st["keep"]].sum(axis=0)
        N += st["n_kept"]
    return total / N, N


def centered_second_moment(batches, m: np.ndarray, N: int, alpha0: float) -> np.ndarray:
    """M2~ = (alpha0 + 1)/N sum_i x~_i x~_i^T with x~_i = f_i - M1 (R3)."""
    V = m.shape[0]
    S = np.zeros((V, V))
    for rp, ci, va in batches:
        st = batch_stats(rp, ci, va, V)
        Xt = frequency_rows(rp, ci, va, V)[st["keep"]] - m[None, :]
        S += Xt.T @ Xt
    return (alpha0 + 1.0) / N * S


def centered_second_moment_merged(batches, V: int, alpha0: float):
    """The same M2~ from per-batch means and scatter matrices, merged pairwise
    (Chan, Golub & LeVeque's update): the form an online pass can keep."""
    n_a, mean_a, scat_a = 0, np.zeros(V), np.zeros((V, V))
    for rp, ci, va in batches:
        st = batch_stats(rp, ci, va, V)
        F = frequency_rows(rp, ci, va, V)[st["keep"]]
        n_b = F.shape[0]
        if n_b == 0:
            continue
        mean_b = F.mean(axis=0)
        scat_b = (F - mean_b).T @ (F - mean_b)
        n = n_a + n_b
        delta = mean_b - mean_a
        scat_a = scat_a + scat_b + np.outer(delta, delta) * (n_a * n_b / n)
        mean_a = mean_a + delta * (n_b / n)
        n_a = n
    return mean_a, (alpha0 + 1.0) / n_a * scat_a, n_a


# --------------------------------------------------------------------------
# Whitening (section "Online Decomposition of the Second Moment").
# --------------------------------------------------------------------------
def whitening(M2: np.ndarray, D: int):
    """W with W^T M2~ W = I_D from the top-D eigenpairs (R4).
    Returns (W, top-D eigenvalues, top-D eigenvectors U)."""
    evals, evecs = np.linalg.eigh(M2)
    order = np.argsort(evals)[::-1][:D]
    lam = evals[order]
    U = evecs[:, order].copy()
    for k in range(D):
        j = int(np.argmax(np.abs(U[:, k])))
        if U[j, k] < 0:
            U[:, k] = -U[:, k]
    if np.any(lam <= 0):
        raise ValueError("second moment has fewer than D positive eigenvalues")
    W = U / np.sqrt(lam)[None, :]
    return W, lam, U


def whiten(row_ptr, col_idx, val, V: int, m: np.ndarray, W: np.ndarray) -> np.ndarray:
    """X = (F - 1 M1^T) W for the kept rows; dropped rows are zero (R2, R5)."""
    st = batch_stats(row_ptr, col_idx, val, V)
    F = frequency_rows(row_ptr, col_idx, val, V)
    X = (F - m[None, :]) @ W
    X[~st["keep"]] = 0.0
    return X


def _frequency_csr(row_ptr, col_idx, val, V: int):
    """Sparse n x V matrix of the frequency rows f_d = c_d / L_d (R1), rows of
    dropped documents (R2) emptied, and the keep mask."""
    import scipy.sparse as sp
    L = doc_lengths(row_ptr, val)
    keep = L >= 3
    C = sp.csr_matrix((np.asarray(val, dtype=np.float64), np.asarray(col_idx),
                       np.asarray(row_ptr)), shape=(L.shape[0], V))
    scale = np.where(keep, 1.0 / np.maximum(L, 1), 0.0)
    return sp.diags(scale) @ C, keep


def whiten_csr(row_ptr, col_idx, val, V: int, m: np.ndarray, W: np.ndarray) -> np.ndarray:
    """The same X as `whiten` without the dense n x V frequency matrix: the
    centred product (F - 1 M1^T) W split as F W - 1 (W^T M1)^T, with F a
    sparse (CSR) matrix, dropped rows zero (R2, R5).  A regrouping of the
    definition, for full-size batches."""
    F, keep = _frequency_csr(row_ptr, col_idx, val, V)
    X = np.asarray(F @ W) - (W.T @ m)[None, :]
    X[~keep] = 0.0
    return X


def whitening_operator(batches, V: int, D: int, alpha0: float, extra: int = 10):
    """W with W^T M2~ W = I_D (R3, R4) for a vocabulary too large for a dense
    V x V matrix: M2~ v = (alpha0 + 1)/N (F^T (F v) - N M1 (M1^T v)) is applied
    as an operator over the sparse frequency rows of every batch, and its top
    D + extra eigenpairs come from Lanczos iteration (ARPACK, to machine
    precision); the top D are kept, ordered and signed as in `whitening`.
    Returns (W, top-D eigenvalues, U, M1, N)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    parts = [_frequency_csr(rp, ci, va, V) for rp, ci, va in batches]
    F = sp.vstack([p[0] for p in parts]).tocsr()
    N = int(sum(int(p[1].sum()) for p in parts))
    m = np.asarray(F.sum(axis=0)).ravel() / N
    a1 = alpha0 + 1.0

    def apply(v):
        v = np.asarray(v).reshape(V, -1)
        return a1 / N * np.asarray(F.T @ (F @ v)) - a1 * np.outer(m, m @ v)

    op = sla.LinearOperator((V, V), matvec=apply, matmat=apply, dtype=np.float64)
    k = min(D + extra, V - 1)
    evals, evecs = sla.eigsh(op, k=k, which="LA", tol=0.0)
    order = np.argsort(evals)[::-1][:D]
    lam = evals[order]
    U = evecs[:, order].copy()
    for j in range(D):
        i = int(np.argmax(np.abs(U[:, j])))
        if U[i, j] < 0:
            U[:, j] = -U[:, j]
    if np.any(lam <= 0):
        raise ValueError("second moment has fewer than D positive eigenvalues")
    return U / np.sqrt(lam)[None, :], lam, U, m, N


# --------------------------------------------------------------------------
# Third-moment CP decomposition (section "Online Learning of the Third Moment").
# --------------------------------------------------------------------------
def _c3(alpha0: float) -> float:
    return (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0


def cp_gradient(X: np.ndarray, Phi: np.ndarray, n: int, alpha0: float,
                theta: float) -> np.ndarray:
    """The batch gradient of eq. vec_deriv:
    3(1+theta) Phi (Phi^T Phi * Phi^T Phi) - 3 c3 / n X^T (X Phi * X Phi)."""
    G = Phi.T @ Phi
    S = X @ Phi
    return 3.0 * (1.0 + theta) * Phi @ (G * G) - 3.0 * _c3(alpha0) / n * X.T @ (S * S)


def whitened_tensor(X: np.ndarray, n: int, alpha0: float) -> np.ndarray:
    """The explicit D x D x D whitened centred third moment
    c3 / n sum_d x_d (x) x_d (x) x_d of a batch."""
    D = X.shape[1]
    T = np.zeros((D, D, D))
    for x in X:
        T += np.einsum("i,j,k->ijk", x, x, x)
    return _c3(alpha0) / n * T


def cp_gradient_explicit(X, Phi, n, alpha0, theta):
    """The same gradient from the explicit tensor T: the data term of column k
    is 3 T(I, phi_k, phi_k)."""
    T = whitened_tensor(X, n, alpha0)
    G = Phi.T @ Phi
    grad = 3.0 * (1.0 + theta) * Phi @ (G * G)
    for k in range(Phi.shape[1]):
        grad[:, k] -= 3.0 * np.einsum("ijk,j,k->i", T, Phi[:, k], Phi[:, k])
    return grad


def _khatri_rao(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Column-wise Khatri-Rao product: column k is a_k (x) b_k."""
    return np.einsum("ik,jk->ijk", A, B).reshape(A.shape[0] * B.shape[0], A.shape[1])


def cp_loss(X, Phi, n, alpha0, theta) -> float:
    """Objective of eq. vec_pb_equiv in Khatri-Rao form:
    (1+theta)/2 |Phi (Phi kr Phi)^T|_F^2 - c3/n <Phi (Phi kr Phi)^T, X^T (X kr X)>,
    where X kr X pairs every row with itself (row-wise Khatri-Rao)."""
    Tphi = Phi @ _khatri_rao(Phi, Phi).T                     # D x D^2
    XX = np.einsum("ni,nj->nij", X, X).reshape(X.shape[0], -1)  # n x D^2
    Tdata = X.T @ XX                                          # D x D^2
    return 0.5 * (1.0 + theta) * float(np.sum(Tphi * Tphi)) - _c3(alpha0) / n * float(np.sum(Tphi * Tdata))


def cp_step(X, Phi, n, alpha0, theta, beta):
    """One stochastic gradient update Phi <- Phi - beta dL/dPhi."""
    return Phi - beta * cp_gradient(X, Phi, n, alpha0, theta)


# --------------------------------------------------------------------------
# Recovering the topic model parameters (post-processing section), reading R7.
# --------------------------------------------------------------------------
def _frame_weight(r: float) -> float:
    """Root a in (0, 1] of a^(1/3) r + a = 1 (bisection; r >= 0)."""
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid ** (1.0 / 3.0) * r + mid < 1.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def unwhiten(Phi: np.ndarray, U: np.ndarray, lam: np.ndarray, m: np.ndarray,
             theta: float) -> dict:
    """Topic-word matrix and topic weights from the learned factors.
    (W^T)^+ = U diag(lam)^(1/2) for W = U diag(lam)^(-1/2)."""
    K = Phi.shape[1]
    w = (1.0 + theta) ** (1.0 / 3.0) * Phi
    a = np.array([_frame_weight(float(w[:, k] @ w[:, k])) for k in range(K)])
    v = w / a[None, :] ** (1.0 / 3.0)
    nu = (U * np.sqrt(lam)[None, :]) @ v
    mu = nu + m[:, None]
    clipped = np.clip(mu, 0.0, None)
    sums = clipped.sum(axis=0, keepdims=True)
    sums[sums == 0] = 1.0
    return {"mu": mu, "mu_simplex": clipped / sums, "alpha": a / a.sum(),
            "a": a, "lambda": (1.0 + theta) * np.linalg.norm(Phi, axis=0) ** 3,
            "nu": nu}


# --------------------------------------------------------------------------
# Document-topic inference (R8).
# --------------------------------------------------------------------------
def simplex_project(v: np.ndarray) -> np.ndarray:
    """Euclidean projection onto {t >= 0, sum t = 1}: sort, find the largest
    index whose threshold keeps it positive, shift and clip."""
    u = np.sort(v)[::-1]
    css = np.cumsum(u)
    rho = 0
    for j in range(v.shape[0]):
        if u[j] - (css[j] - 1.0) / (j + 1) > 0:
            rho = j
    tau = (css[rho] - 1.0) / (rho + 1)
    return np.maximum(v - tau, 0.0)


def inference_matrix(mu: np.ndarray, m: np.ndarray, W: np.ndarray) -> np.ndarray:
    """A = W^T (mu - M1 1^T): topics mapped into the whitened space."""
    return W.T @ (mu - m[:, None])


def infer_doc_topics(X: np.ndarray, A: np.ndarray, max_iter: int, tol: float = 0.0) -> np.ndarray:
    """Projected gradient on |x - A t|^2 over the simplex for every row of X,
    from t = 1/K, with step 1 / lambda_max(A^T A); stops when the L1 change of
    an iterate falls below tol (tol = 0: always max_iter steps)."""
    K = A.shape[1]
    G = A.T @ A
    step = 1.0 / float(np.max(np.linalg.eigvalsh(G)))
    out = np.zeros((X.shape[0], K))
    for d in range(X.shape[0]):
        b = A.T @ X[d]
        t = np.full(K, 1.0 / K)
        for _ in range(max_iter):
            t_new = simplex_project(t - step * (G @ t - b))
            change = float(np.abs(t_new - t).sum())
            t = t_new
            if change < tol:
                break
        out[d] = t
    return out


# --------------------------------------------------------------------------
# Topic matching (simulation section: best permutation to the planted topics).
# --------------------------------------------------------------------------
def match_topics(est: np.ndarray, truth: np.ndarray) -> dict:
    """Permutation of estimated columns minimising the mean L1 distance to the
    planted columns; exhaustive for K <= 7, Hungarian assignment otherwise."""
    K = truth.shape[1]
    cost = np.abs(est[:, :, None] - truth[:, None, :]).sum(axis=0)  # est x truth
    if K <= 7:
        best = None
        for p in itertools.permutations(range(K)):
            c = sum(cost[p[j], j] for j in range(K))
            if best is None or c < best[0]:
                best = (c, p)
        perm = np.array(best[1])
    else:
        from scipy.optimize import linear_sum_assignment
        r, c = linear_sum_assignment(cost)
        perm = np.empty(K, dtype=int)
        perm[c] = r
    l1 = np.array([cost[perm[j], j] for j in range(K)])
    corr = np.array([np.corrcoef(est[:, perm[j]], truth[:, j])[0, 1] for j in range(K)])
    return {"perm": perm, "l1": l1, "mean_l1": float(l1.mean()), "corr": corr}


# --------------------------------------------------------------------------
# Appendix: uncentred cumulants with the alpha0 corrections (tiny V only), and
# the classic whitened tensor power method (reading R9).
# --------------------------------------------------------------------------
def uncentered_cumulants(row_ptr, col_idx, val, V: int, alpha0: float):
    """Explicit M1 (V), M2 (V x V), M3 (V x V x V) of the appendix."""
    st = batch_stats(row_ptr, col_idx, val, V)
    N = st["n_kept"]
    c3 = _c3(alpha0)
    c2 = alpha0 * (alpha0 + 1.0) / 2.0
    M1 = np.zeros(V)
    P2 = np.zeros((V, V))
    P3 = np.zeros((V, V, V))
    for d in np.nonzero(st["keep"])[0]:
        c = np.zeros(V)
        for j in range(int(row_ptr[d]), int(row_ptr[d + 1])):
            c[int(col_idx[j])] += float(val[j])
        L = float(st["L"][d])
        M1 += c / L
        P2 += (np.outer(c, c) - np.diag(c)) / (L * (L - 1.0))
        t = np.einsum("a,b,c->abc", c, c, c)
        for a in range(V):
            if c[a] == 0:
                continue
            t[a, a, :] -= c[a] * c          # both first indices on one word
            t[a, :, a] -= c[a] * c          # first and third
            t[:, a, a] -= c[a] * c          # second and third
            t[a, a, a] += 2.0 * c[a]        # all three
        P3 += t / (L * (L - 1.0) * (L - 2.0))
    M1 /= N
    P2 /= N
    P3 /= N
    M2 = (alpha0 + 1.0) * P2 - alpha0 * np.outer(M1, M1)
    pair_m = (np.einsum("ab,c->abc", P2, M1) + np.einsum("ac,b->abc", P2, M1)
              + np.einsum("bc,a->abc", P2, M1))
    M3 = c3 * P3 - c2 * pair_m + alpha0 ** 2 * np.einsum("a,b,c->abc", M1, M1, M1)
    return M1, M2, M3


def tensor_power_method(T: np.ndarray, K: int, restarts: int = 20, iters: int = 100,
                        seed: int = 0):
    """Robust tensor power method with deflation: for each component, the best
    of several random starts of v <- T(I, v, v) / |T(I, v, v)|, refined, then
    deflated out of T."""
    rng = np.random.default_rng(seed)
    T = T.copy()
    D = T.shape[0]
    lams, vecs = [], []
    for _ in range(K):
        best = None
        for _r in range(restarts):
            v = rng.standard_normal(D)
            v /= np.linalg.norm(v)
            for _i in range(iters):
                v = np.einsum("ijk,j,k->i", T, v, v)
                v /= np.linalg.norm(v)
            lam = float(np.einsum("ijk,i,j,k->", T, v, v, v))
            if best is None or lam > best[0]:
                best = (lam, v)
        v = best[1]
        for _i in range(iters):
            v = np.einsum("ijk,j,k->i", T, v, v)
            v /= np.linalg.norm(v)
        lam = float(np.einsum("ijk,i,j,k->", T, v, v, v))
        lams.append(lam)
        vecs.append(v)
        T = T - lam * np.einsum("i,j,k->ijk", v, v, v)
    return np.array(lams), np.stack(vecs, axis=1)


def classic_recover(M2: np.ndarray, M3: np.ndarray, K: int, seed: int = 0):
    """Spectral LDA on the uncentred moments: whiten M2 with its top-K pairs,
    decompose T = M3(W, W, W) by the power method, and unwhiten:
    mu_i = lambda_i (W^T)^+ v_i, alpha_i proportional to lambda_i^-2."""
    W, lam2, U = whitening(M2, K)
    T = np.einsum("abc,ai,bj,ck->ijk", M3, W, W, W)
    lam, v = tensor_power_method(T, K, seed=seed)
    mu = (U * np.sqrt(lam2)[None, :]) @ v * lam[None, :]
    a = lam ** -2.0
    return {"mu": mu, "alpha": a / a.sum(), "lambda": lam}


# --------------------------------------------------------------------------
# Estimator rung with the classic alpha0-corrected moments (appendix, R9), run
# through the same batched SGD: the whitened third moment is contracted
# implicitly, per document, from the unbiased pair and triple pieces.
# --------------------------------------------------------------------------
def classic_second_moment(batches, m: np.ndarray, N: int, alpha0: float) -> np.ndarray:
    """M2 = (alpha0 + 1) mean_d P2_d - alpha0 M1 M1^T with the unbiased pair
    piece P2_d = (c c^T - diag c) / (L (L - 1)), summed over kept documents."""
    V = m.shape[0]
    P2 = np.zeros((V, V))
    for rp, ci, va in batches:
        st = batch_stats(rp, ci, va, V)
        for d in np.nonzero(st["keep"])[0]:
            a, b = int(rp[d]), int(rp[d + 1])
            c = np.zeros(V)
            np.add.at(c, ci[a:b], va[a:b].astype(np.float64))
            L = float(st["L"][d])
            P2 += (np.outer(c, c) - np.diag(c)) / (L * (L - 1.0))
    return (alpha0 + 1.0) * P2 / N - alpha0 * np.outer(m, m)


def classic_data_term(row_ptr, col_idx, val, V: int, m: np.ndarray, W: np.ndarray,
                      Phi: np.ndarray, alpha0: float, Z: np.ndarray = None) -> tuple:
    """Sum over the batch's kept documents of M3_d(W, W, W)(I, phi_k, phi_k),
    column k, with M3_d = c3 P3_d - c2 (P2_d x M1 + its two permutations) +
    alpha0^2 M1^3 the per-document piece of the appendix's M3 (c2 =
    alpha0 (alpha0 + 1) / 2).  Written out per document with y = W^T c,
    z = W Phi, s = y.phi, g = W^T (c z), q = c.z^2, h = W^T (c z^2),
    r = (W^T M1).phi, l2 = 1/(L(L-1)), l3 = 1/(L(L-1)(L-2)):
      c3 l3 (y s^2 - 2 s g - y q + 2 h) - c2 l2 (2 r (y s - g) + m_w (s^2 - q))
      + alpha0^2 m_w r^2.
    Z, if given, replaces the per-word scores W Phi (V x K) wherever a word's
    score enters: in g, q, h and in s = sum_w c_w z_w (equal to y.phi when
    Z = W Phi); a test evaluates the term on rounded scores this way.
    Returns (D x K sum, number of kept documents)."""
    st = batch_stats(row_ptr, col_idx, val, V)
    c3 = _c3(alpha0)
    c2 = alpha0 * (alpha0 + 1.0) / 2.0
    given = Z is not None
    if not given:
        Z = W @ Phi
    mw = W.T @ m
    r = mw @ Phi
    out = np.zeros(Phi.shape)
    for d in np.nonzero(st["keep"])[0]:
        a, b = int(row_ptr[d]), int(row_ptr[d + 1])
        cols = col_idx[a:b].astype(np.int64)
        cnt = val[a:b].astype(np.float64)
        L = float(st["L"][d])
        l2 = 1.0 / (L * (L - 1.0))
        l3 = l2 / (L - 2.0)
        Wd, Zd = W[cols], Z[cols]                 # rows of the document's words
        y = Wd.T @ cnt
        s = cnt @ Zd if given else y @ Phi
        g = Wd.T @ (cnt[:, None] * Zd)
        q = cnt @ (Zd * Zd)
        h = Wd.T @ (cnt[:, None] * Zd * Zd)
        out += c3 * l3 * (np.outer(y, s * s) - 2.0 * s[None, :] * g - np.outer(y, q) + 2.0 * h)
        out -= c2 * l2 * (2.0 * r[None, :] * (np.outer(y, s) - g) + np.outer(mw, s * s - q))
        out += alpha0 ** 2 * np.outer(mw, r * r)
    return out, int(st["n_kept"])


def classic_cp_gradient(row_ptr, col_idx, val, V, m, W, Phi, alpha0, theta):
    """3(1+theta) Phi (Phi^T Phi * Phi^T Phi) - (3/n) sum_d M3_d(W,W,W)(I, phi, phi)."""
    data, n = classic_data_term(row_ptr, col_idx, val, V, m, W, Phi, alpha0)
    G = Phi.T @ Phi
    return 3.0 * (1.0 + theta) * Phi @ (G * G) - 3.0 / max(n, 1) * data


def classic_unwhiten(Phi: np.ndarray, U: np.ndarray, lam: np.ndarray, theta: float) -> dict:
    """Classic recovery (R14, the relation of the post-processing section in
    the orthonormal case): lambda_i = (1+theta)
    |phi_i|^3, mu_i = lambda_i (W^T)^+ phi_i / |phi_i| = lambda_i U diag(l)^1/2
    phi_i / |phi_i|, alpha_i proportional to lambda_i^-2; mu clipped and
    renormalised onto the simplex."""
    nrm = np.linalg.norm(Phi, axis=0)
    lamb = (1.0 + theta) * nrm ** 3
    mu = (U * np.sqrt(lam)[None, :]) @ (Phi / nrm[None, :]) * lamb[None, :]
    a = lamb ** -2.0
    mu_s = np.maximum(mu, 0.0)
    mu_s = mu_s / mu_s.sum(axis=0, keepdims=True)
    return {"mu": mu, "mu_simplex": mu_s, "alpha": a / a.sum(), "lambda": lamb}


def fit_batched_classic(batches: list, V: int, K: int, D: int, alpha0: float, theta: float,
                        beta: float, passes: int, Phi0: np.ndarray) -> dict:
    m, N = first_moment(batches, V)
    M2 = classic_second_moment(batches, m, N, alpha0)
    W, lam, U = whitening(M2, D)
    Phi = Phi0.copy()
    for _ in range(passes):
        for rp, ci, va in batches:
            G = classic_cp_gradient(rp, ci, va, V, m, W, Phi, alpha0, theta)
            if batch_stats(rp, ci, va, V)["n_kept"] > 0:
                Phi = Phi - beta * G
    out = classic_unwhiten(Phi, U, lam, theta)
    out.update({"Phi": Phi, "W": W, "eig": lam, "U": U, "m": m, "N": N, "M2": M2})
    return out


# --------------------------------------------------------------------------
# The batched method end to end (batched-implementation section): one pass for
# the moments, whitening, then passes of one gradient step per batch.
# --------------------------------------------------------------------------
def fit_batched(batches: list, V: int, K: int, D: int, alpha0: float, theta: float,
                beta: float, passes: int, Phi0: np.ndarray) -> dict:
    m, N = first_moment(batches, V)
    M2 = centered_second_moment(batches, m, N, alpha0)
    W, lam, U = whitening(M2, D)
    Phi = Phi0.copy()
    Xs = []
    for rp, ci, va in batches:
        st = batch_stats(rp, ci, va, V)
        Xs.append((whiten(rp, ci, va, V, m, W), st["n_kept"]))
    for _ in range(passes):
        for X, n in Xs:
            if n > 0:
                Phi = cp_step(X, Phi, n, alpha0, theta, beta)
    out = unwhiten(Phi, U, lam, m, theta)
    out.update({"Phi": Phi, "W": W, "eig": lam, "U": U, "m": m, "N": N, "M2": M2})
    return out


# --------------------------------------------------------------------------
# The fully online method (fully-online section, R15): factors from a batched
# run on an initial portion, then per new batch: the moments, a new whitening
# of the running M2~, Phi carried into the new whitened space, the whitened
# batch and one gradient step.  No earlier batch is revisited.
# --------------------------------------------------------------------------
def rebase_phi(Phi: np.ndarray, W_old: np.ndarray, W_new: np.ndarray) -> np.ndarray:
    """Phi_new = W_new^T (W_old^T)^+ Phi_old (R15): the factors' centred
    word-space vectors (W_old^T)^+ phi, seen through the new whitening."""
    return W_new.T @ np.linalg.pinv(W_old.T) @ Phi


def fit_online(init_batches: list, stream_batches: list, V: int, K: int, D: int, alpha0: float,
               theta: float, beta: float, init_passes: int, Phi0: np.ndarray) -> dict:
    """R15: Phi from fit_batched on init_batches; then for each batch of
    stream_batches the running M1 and M2~ over every batch seen so far, W from
    them (R4), Phi rebased from the previous W, X with the new M1 and W, and
    one gradient step (skipped when the batch keeps no document)."""
    fit = fit_batched(init_batches, V, K, D, alpha0, theta, beta, init_passes, Phi0)
    Phi, W = fit["Phi"], fit["W"]
    seen = list(init_batches)
    trace = []
    for rp, ci, va in stream_batches:
        seen.append((rp, ci, va))
        m, N = first_moment(seen, V)
        W_new, lam, U = whitening(centered_second_moment(seen, m, N, alpha0), D)
        Phi = rebase_phi(Phi, W, W_new)
        W = W_new
        n = batch_stats(rp, ci, va, V)["n_kept"]
        if n > 0:
            Phi = cp_step(whiten(rp, ci, va, V, m, W), Phi, n, alpha0, theta, beta)
        trace.append(Phi.copy())
    out = unwhiten(Phi, U, lam, m, theta)
    out.update({"Phi": Phi, "W": W, "eig": lam, "U": U, "m": m, "N": N, "trace": trace,
                "Phi_init": fit["Phi"], "W_init": fit["W"]})
    return out
