"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself: a
hand-worked fixture, a library routine the definition reduces to, a closed
form, an invariant, brute force on tiny inputs, or a planted model.
"""
import itertools

import numpy as np
import pytest

from oracle import tlda_oracle as O
from synth import SPECS, CorpusSpec, generate, init_phi, iter_batches, make_csr_rows


def _golden_corpus(golden):
    entries = golden("tiny_corpus.txt")
    V = int(dict(entries)["V"][0])
    rows = []
    for key, vals in entries:
        if key == "doc":
            rows.append({int(w): int(c) for w, c in (v.split(":") for v in vals)})
    expect = {k: v for k, v in entries if k.startswith("expect")}
    return V, make_csr_rows(rows, V), expect


def test_integer_stats_hand_worked(golden):
    V, (rp, ci, va), ex = _golden_corpus(golden)
    st = O.batch_stats(rp, ci, va, V)
    assert st["L"].tolist() == [int(x) for x in ex["expect_L"]]
    assert st["keep"].astype(int).tolist() == [int(x) for x in ex["expect_kept"]]
    assert st["n_kept"] == int(ex["expect_N"][0])
    assert st["n_skipped"] == int(ex["expect_skipped"][0])
    assert st["token_totals"].tolist() == [int(x) for x in ex["expect_token_totals"]]


def test_first_moment_hand_worked(golden):
    V, (rp, ci, va), ex = _golden_corpus(golden)
    m, N = O.first_moment([(rp, ci, va)], V)
    num = np.array([int(x) for x in ex["expect_M1_num"]], dtype=float)
    assert N == 3
    np.testing.assert_allclose(m, num / int(ex["expect_M1_den"][0]), rtol=0, atol=1e-15)


def test_integer_stats_independent_of_batching():
    spec = SPECS["c1"]
    c = generate(spec, n_docs=1500)
    ref = O.batch_stats(c.indptr, c.indices, c.data, spec.V)
    for bs in (1, 7, 256, 1500):
        N = 0
        tot = np.zeros(spec.V, dtype=np.int64)
        for rp, ci, va, _ in iter_batches(c, bs):
            st = O.batch_stats(rp, ci, va, spec.V)
            N += st["n_kept"]
            tot += st["token_totals"]
        assert N == ref["n_kept"]
        assert np.array_equal(tot, ref["token_totals"])
    # every token of every kept document is counted exactly once
    assert ref["token_totals"].sum() == ref["L"][ref["keep"]].sum()


def _c1_batches(n_docs=3000, batch=1000):
    c = generate(SPECS["c1"], n_docs=n_docs)
    return c, [(rp, ci, va) for rp, ci, va, _ in iter_batches(c, batch)]


def test_first_moment_is_a_distribution():
    c, batches = _c1_batches()
    m, N = O.first_moment(batches, c.spec.V)
    assert N == 3000
    assert abs(m.sum() - 1.0) < 1e-13 and m.min() >= 0


def test_centered_second_moment_is_scaled_covariance():
    """M2~ reduces to (alpha0 + 1) times the biased sample covariance."""
    c, batches = _c1_batches()
    V, a0 = c.spec.V, c.spec.alpha0
    m, N = O.first_moment(batches, V)
    M2 = O.centered_second_moment(batches, m, N, a0)
    F = np.vstack([O.frequency_rows(*b, V) for b in batches])
    np.testing.assert_allclose(M2, (a0 + 1) * np.cov(F.T, bias=True), rtol=1e-10, atol=1e-15)
    # the centred rows sum to zero, so the all-ones vector is in the kernel
    assert np.abs(M2 @ np.ones(V)).max() < 1e-14


def test_batched_demeaned_moments_match_full_batch():
    """Per-batch means and scatters merged pairwise equal the full-batch M2~."""
    c, batches = _c1_batches()
    V, a0 = c.spec.V, c.spec.alpha0
    m, N = O.first_moment(batches, V)
    full = O.centered_second_moment(batches, m, N, a0)
    mean_m, merged, n_m = O.centered_second_moment_merged(batches, V, a0)
    assert n_m == N
    np.testing.assert_allclose(mean_m, m, rtol=0, atol=1e-15)
    assert np.linalg.norm(merged - full) <= 1e-12 * np.linalg.norm(full)


def test_whitening_identity_and_whitened_corpus():
    c, batches = _c1_batches()
    V, K, a0 = c.spec.V, c.spec.K, c.spec.alpha0
    m, N = O.first_moment(batches, V)
    M2 = O.centered_second_moment(batches, m, N, a0)
    W, lam, U = O.whitening(M2, K)
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(K), atol=1e-10)
    assert np.all(np.diff(lam) <= 0)
    for k in range(K):
        j = np.argmax(np.abs(U[:, k]))
        assert U[j, k] > 0
    X = np.vstack([O.whiten(*b, V, m, W) for b in batches])
    # full-corpus invariants: whitened rows have zero mean and (a0+1)/N X^T X = I
    assert np.abs(X.sum(axis=0)).max() < 1e-9
    np.testing.assert_allclose((a0 + 1) / N * X.T @ X, np.eye(K), atol=1e-10)


def test_sparse_whitening_equals_the_dense_definition():
    """whiten_csr regroups (F - 1 M1^T) W as F W - 1 (W^T M1)^T over a sparse
    F: it must equal the dense definition row for row, dropped rows zero."""
    c, batches = _c1_batches()
    V = c.spec.V
    rng = np.random.default_rng(3)
    W = rng.standard_normal((V, 7)) * 20.0
    m = rng.dirichlet(np.ones(V))
    extra = make_csr_rows([{}, {4: 1, 9: 1}, {0: 5}, {2: 1, 499: 2}], V)
    for rp, ci, va in list(batches[:2]) + [extra]:
        X = O.whiten_csr(rp, ci, va, V, m, W)
        ref = O.whiten(rp, ci, va, V, m, W)
        assert np.abs(X - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.all(O.whiten_csr(*extra, V, m, W)[[0, 1]] == 0.0)


@pytest.mark.parametrize("D", [5, 30])
def test_operator_whitening_equals_the_dense_eigendecomposition(D):
    """The Lanczos whitening of M2~ applied as an operator against the dense
    M2~ and LAPACK's symmetric eigensolver: same M1, N, eigenvalues, columns
    (same order and sign rule) and the identity W^T M2~ W = I."""
    c, batches = _c1_batches()
    V, a0 = c.spec.V, c.spec.alpha0
    m, N = O.first_moment(batches, V)
    M2 = O.centered_second_moment(batches, m, N, a0)
    W_ref, lam_ref, U_ref = O.whitening(M2, D)
    W, lam, U, m2, N2 = O.whitening_operator(batches, V, D, a0)
    assert N2 == N
    np.testing.assert_allclose(m2, m, rtol=0, atol=1e-15)
    assert np.abs(lam - lam_ref).max() <= 1e-12 * lam_ref[0]
    gaps = np.minimum(np.r_[np.inf, -np.diff(lam_ref)], np.r_[-np.diff(lam_ref), np.inf])
    wide = gaps > 1e-4 * lam_ref[0]
    assert wide.sum() >= min(D, 5)
    assert np.abs(U[:, wide] - U_ref[:, wide]).max() < 1e-8
    np.testing.assert_allclose(W.T @ M2 @ W, np.eye(D), atol=1e-9)


def test_dropped_rows_are_zero_and_excluded():
    V = 6
    rp, ci, va = make_csr_rows([{0: 2, 1: 1}, {2: 1}, {}, {3: 1, 4: 1, 5: 3}, {1: 1, 5: 1}], V)
    st = O.batch_stats(rp, ci, va, V)
    assert st["n_kept"] == 2 and st["n_skipped"] == 3
    W = np.random.default_rng(0).standard_normal((V, 3))
    X = O.whiten(rp, ci, va, V, np.full(V, 1.0 / V), W)
    assert np.all(X[[1, 2, 4]] == 0) and np.all(X[[0, 3]] != 0)


def _rand_X_phi(n=40, D=6, K=4, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, D)), rng.standard_normal((D, K))


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_gradient_implicit_equals_explicit_tensor(theta):
    X, Phi = _rand_X_phi()
    g1 = O.cp_gradient(X, Phi, X.shape[0], 1.0, theta)
    g2 = O.cp_gradient_explicit(X, Phi, X.shape[0], 1.0, theta)
    assert np.abs(g1 - g2).max() <= 1e-12 * np.abs(g2).max()


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_gradient_is_derivative_of_objective(theta):
    X, Phi = _rand_X_phi(seed=1)
    n, a0 = X.shape[0], 2.0
    g = O.cp_gradient(X, Phi, n, a0, theta)
    h = 1e-5
    fd = np.zeros_like(Phi)
    for i in range(Phi.shape[0]):
        for k in range(Phi.shape[1]):
            P1, P2 = Phi.copy(), Phi.copy()
            P1[i, k] += h
            P2[i, k] -= h
            fd[i, k] = (O.cp_loss(X, P1, n, a0, theta) - O.cp_loss(X, P2, n, a0, theta)) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * np.abs(g).max()


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_gradient_vanishes_at_orthogonal_fixed_point(theta):
    """For T = sum_i lam_i v_i^(x)3 with orthonormal v_i, the factors
    (lam_i / (1 + theta))^(1/3) v_i are a stationary point."""
    D, K, a0 = 7, 4, 1.0
    rng = np.random.default_rng(2)
    Vq, _ = np.linalg.qr(rng.standard_normal((D, K)))
    lam = np.array([1.5, 2.0, 3.0, 4.5])
    c3 = (a0 + 1) * (a0 + 2) / 2
    X = ((K * lam / c3) ** (1 / 3))[:, None] * Vq.T      # one row per component
    T = O.whitened_tensor(X, K, a0)
    np.testing.assert_allclose(T, np.einsum("i,ai,bi,ci->abc", lam, Vq, Vq, Vq), atol=1e-13)
    Phi = (lam / (1 + theta)) ** (1 / 3) * Vq
    assert np.abs(O.cp_gradient(X, Phi, K, a0, theta)).max() < 1e-12
    # and a generic point is not stationary
    assert np.abs(O.cp_gradient(X, Phi + 0.1, K, a0, theta)).max() > 1e-3


def _planted_population(seed=3, V=40, K=5):
    rng = np.random.default_rng(seed)
    mu = rng.dirichlet(np.full(V, 0.3), size=K).T
    alpha = np.array([0.1, 0.2, 0.3, 0.15, 0.25])[:K]
    a0 = alpha.sum()
    a = alpha / a0
    m = mu @ a
    nu = mu - m[:, None]
    return mu, alpha, a0, a, m, nu


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_recovery_of_planted_topics_from_population_moments(theta):
    """With the exact centred population moments (sum a_i nu_i nu_i^T and
    sum a_i nu_i^(x)3), SGD from a perturbed start returns to the planted
    decomposition and unwhitening gives back the planted mu and alpha."""
    mu, alpha, a0, a, m, nu = _planted_population()
    K = mu.shape[1]
    M2 = (nu * a) @ nu.T
    # the population centred M2 has rank K - 1 because sum a_i nu_i = 0
    ev = np.linalg.eigvalsh(M2)[::-1]
    assert ev[K - 1] < 1e-15 * ev[0]
    D = K - 1
    W, lam, U = O.whitening(M2, D)
    v = W.T @ nu
    np.testing.assert_allclose(a * (v * v).sum(axis=0), 1 - a, atol=1e-12)  # tight frame
    c3 = (a0 + 1) * (a0 + 2) / 2
    X = ((K * a / c3) ** (1 / 3))[:, None] * v.T
    Phi_star = (a / (1 + theta)) ** (1 / 3) * v
    assert np.abs(O.cp_gradient(X, Phi_star, K, a0, theta)).max() < 1e-12
    Phi = Phi_star + 0.05 * np.random.default_rng(1).standard_normal(Phi_star.shape)
    for _ in range(4000):
        Phi = O.cp_step(X, Phi, K, a0, theta, 0.005)
    r = O.unwhiten(Phi, U, lam, m, theta)
    assert np.abs(r["mu"] - mu).max() < 1e-7
    assert np.abs(r["alpha"] - a).max() < 1e-7
    np.testing.assert_allclose(r["mu"].sum(axis=0), 1.0, atol=1e-12)


def test_theorem_1_recentering_population():
    """Theorem 1: sum a_i (nu_i + M1)^(x)3 is the uncentred population third
    moment sum a_i mu_i^(x)3 (the vectors nu_i + M1 are the topics)."""
    mu, alpha, a0, a, m, nu = _planted_population(V=12)
    lhs = np.einsum("i,ai,bi,ci->abc", a, nu + m[:, None], nu + m[:, None], nu + m[:, None])
    rhs = np.einsum("i,ai,bi,ci->abc", a, mu, mu, mu)
    np.testing.assert_allclose(lhs, rhs, atol=1e-15)


def test_pair_and_triple_terms_brute_force():
    """The appendix moments of a single document equal averages over its
    ordered pairs and triples of distinct token positions."""
    V, a0 = 5, 0.7
    tokens = [0, 2, 2, 4, 0, 0, 1]
    counts = {w: tokens.count(w) for w in set(tokens)}
    rp, ci, va = make_csr_rows([counts], V)
    M1, M2, M3 = O.uncentered_cumulants(rp, ci, va, V, a0)
    L = len(tokens)
    P2 = np.zeros((V, V))
    for s, t in itertools.permutations(range(L), 2):
        P2[tokens[s], tokens[t]] += 1
    P2 /= L * (L - 1)
    P3 = np.zeros((V, V, V))
    for s, t, u in itertools.permutations(range(L), 3):
        P3[tokens[s], tokens[t], tokens[u]] += 1
    P3 /= L * (L - 1) * (L - 2)
    f = np.bincount(tokens, minlength=V) / L
    np.testing.assert_allclose(M1, f, atol=1e-15)
    np.testing.assert_allclose(M2, (a0 + 1) * P2 - a0 * np.outer(f, f), atol=1e-14)
    c3, c2 = (a0 + 1) * (a0 + 2) / 2, a0 * (a0 + 1) / 2
    sym = (np.einsum("ab,c->abc", P2, f) + np.einsum("ac,b->abc", P2, f)
           + np.einsum("bc,a->abc", P2, f))
    np.testing.assert_allclose(M3, c3 * P3 - c2 * sym + a0 ** 2 * np.einsum("a,b,c->abc", f, f, f),
                               atol=1e-14)


def _small_lda(N, seed, V=12, K=3, L=12):
    spec = CorpusSpec("t", V=V, K=K, N=N, doc_len_lambda=L - 1, alpha0=0.6, topic_conc=0.4,
                      zipf_s=None, zipf_mix=0.0, batch=N, seed=seed)
    return generate(spec), spec


def test_uncentered_cumulants_match_population_identities():
    """Monte Carlo: M2 -> sum a_i mu_i mu_i^T and M3 -> sum a_i mu_i^(x)3."""
    c, spec = _small_lda(N=40000, seed=11)
    M1, M2, M3 = O.uncentered_cumulants(c.indptr, c.indices, c.data, spec.V, spec.alpha0)
    a = c.alpha / c.alpha.sum()
    P2 = (c.mu * a) @ c.mu.T
    P3 = np.einsum("i,ai,bi,ci->abc", a, c.mu, c.mu, c.mu)
    np.testing.assert_allclose(M1, c.mu @ a, atol=3e-3)
    assert np.linalg.norm(M2 - P2) < 0.05 * np.linalg.norm(P2)
    assert np.linalg.norm(M3 - P3) < 0.08 * np.linalg.norm(P3)


def test_power_method_recovers_orthogonal_tensor():
    rng = np.random.default_rng(5)
    D, K = 6, 4
    Vq, _ = np.linalg.qr(rng.standard_normal((D, K)))
    lam = np.array([3.0, 2.2, 1.7, 1.1])
    T = np.einsum("i,ai,bi,ci->abc", lam, Vq, Vq, Vq)
    lh, vh = O.tensor_power_method(T, K, restarts=10, iters=60, seed=1)
    np.testing.assert_allclose(lh, lam, atol=1e-10)
    np.testing.assert_allclose(np.abs(vh.T @ Vq), np.eye(K), atol=1e-8)


def test_classic_spectral_recovery_of_planted_topics_improves_with_N():
    errs = []
    for N in (2000, 32000):
        c, spec = _small_lda(N=N, seed=21)
        M1, M2, M3 = O.uncentered_cumulants(c.indptr, c.indices, c.data, spec.V, spec.alpha0)
        r = O.classic_recover(M2, M3, spec.K, seed=0)
        errs.append(O.match_topics(r["mu"], c.mu)["mean_l1"])
    assert errs[1] < 0.6 * errs[0]
    assert errs[1] < 0.15


def test_simplex_projection_kkt_and_enumeration():
    rng = np.random.default_rng(7)
    for K in (1, 2, 3):
        for _ in range(50):
            v = rng.standard_normal(K) * 2
            p = O.simplex_project(v)
            assert abs(p.sum() - 1) < 1e-12 and p.min() >= 0
            # brute force: best point over every face of the simplex
            best = None
            for r in range(1, K + 1):
                for S in itertools.combinations(range(K), r):
                    S = list(S)
                    q = np.zeros(K)
                    q[S] = v[S] - (v[S].sum() - 1) / len(S)
                    if q.min() < -1e-15:
                        continue
                    d = np.sum((q - v) ** 2)
                    if best is None or d < best[0]:
                        best = (d, q)
            np.testing.assert_allclose(p, best[1], atol=1e-12)
    # KKT at larger K: v - p = tau on the support, <= tau off it
    v = rng.standard_normal(40)
    p = O.simplex_project(v)
    s = p > 0
    tau = (v - p)[s]
    assert np.ptp(tau) < 1e-12 and np.all((v - p)[~s] <= tau[0] + 1e-12)


def test_inference_recovers_exact_mixtures():
    rng = np.random.default_rng(8)
    mu, alpha, a0, a, m, nu = _planted_population(V=30)
    M2 = (nu * a) @ nu.T
    W, lam, U = O.whitening(M2, 4)
    A = O.inference_matrix(mu, m, W)
    th = rng.dirichlet(np.full(5, 0.5), size=6)
    X = (W.T @ ((mu @ th.T) - m[:, None])).T
    est = O.infer_doc_topics(X, A, max_iter=20000, tol=1e-13)
    np.testing.assert_allclose(est, th, atol=1e-6)


def test_match_topics_hungarian_equals_exhaustive():
    rng = np.random.default_rng(9)
    truth = rng.dirichlet(np.ones(20), size=6).T
    est = truth[:, [3, 0, 5, 1, 4, 2]] + 0.01 * rng.random((20, 6))
    ex = O.match_topics(est, truth)
    assert ex["perm"].tolist() == [1, 3, 5, 0, 4, 2]
    from scipy.optimize import linear_sum_assignment
    cost = np.abs(est[:, :, None] - truth[:, None, :]).sum(axis=0)
    r, cidx = linear_sum_assignment(cost)
    assert abs(cost[r, cidx].mean() - ex["mean_l1"]) < 1e-12


def test_batched_fit_config1_runs_and_reports_recovery():
    """End-to-end batched fit on the 500-word workload.  The fitted factors are
    finite, the recovered topics are distributions, and they are closer to the
    planted topics than the corpus mean is.  How close depends on the start:
    the paper-literal centred moments keep a multinomial-noise bias and the
    loss has several local minima, so truth recovery is reported, not gated."""
    spec = SPECS["c1"]
    c = generate(spec)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
    out = O.fit_batched(batches, spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.03, 30,
                        init_phi(spec.K, spec.K, 3))
    assert np.all(np.isfinite(out["Phi"]))
    err = O.match_topics(out["mu_simplex"], c.mu)["mean_l1"]
    base = np.mean(np.abs(c.mu - out["m"][:, None]).sum(axis=0))
    np.testing.assert_allclose(out["mu_simplex"].sum(axis=0), 1.0, atol=1e-12)
    assert err < base


# ----------------------------------------------------------------------------
# the classic alpha0-corrected rung
# ----------------------------------------------------------------------------
def test_classic_second_moment_matches_the_explicit_cumulants_over_batches():
    c, spec = _small_lda(N=900, seed=31)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c, 250)]
    m, N = O.first_moment(batches, spec.V)
    M1, M2, _ = O.uncentered_cumulants(c.indptr, c.indices, c.data, spec.V, spec.alpha0)
    np.testing.assert_allclose(m, M1, atol=1e-15)
    np.testing.assert_allclose(O.classic_second_moment(batches, m, N, spec.alpha0), M2,
                               atol=1e-15)


def test_classic_data_term_equals_the_explicit_whitened_contraction():
    """The implicit per-document form (y s^2, g, q, h terms) against the
    explicit M3 tensor contracted with (W, phi_k, phi_k)."""
    c, spec = _small_lda(N=300, seed=32)
    rng = np.random.default_rng(3)
    D, K = 4, 3
    W = rng.standard_normal((spec.V, D))
    Phi = rng.standard_normal((D, K))
    M1, _, M3 = O.uncentered_cumulants(c.indptr, c.indices, c.data, spec.V, spec.alpha0)
    data, n = O.classic_data_term(c.indptr, c.indices, c.data, spec.V, M1, W, Phi, spec.alpha0)
    T = np.einsum("abc,ai,bj,ck->ijk", M3, W, W, W)
    expl = n * np.stack([np.einsum("ijk,j,k->i", T, Phi[:, k], Phi[:, k]) for k in range(K)],
                        axis=1)
    np.testing.assert_allclose(data, expl, rtol=1e-11, atol=1e-11 * np.abs(expl).max())
    # the same with the word scores passed in (s summed from the scores)
    data_z, n_z = O.classic_data_term(c.indptr, c.indices, c.data, spec.V, M1, W, Phi,
                                      spec.alpha0, Z=W @ Phi)
    assert n_z == n
    np.testing.assert_allclose(data_z, expl, rtol=1e-11, atol=1e-11 * np.abs(expl).max())


def test_classic_gradient_is_the_derivative_of_its_objective():
    c, spec = _small_lda(N=200, seed=33)
    rng = np.random.default_rng(4)
    D, K, theta = 3, 3, 0.5
    W = rng.standard_normal((spec.V, D)) * 2
    Phi = rng.standard_normal((D, K))
    M1, _, M3 = O.uncentered_cumulants(c.indptr, c.indices, c.data, spec.V, spec.alpha0)
    T = np.einsum("abc,ai,bj,ck->ijk", M3, W, W, W)

    def loss(P):
        G = P.T @ P
        return (1 + theta) / 2 * (G ** 3).sum() - np.einsum("ijk,il,jl,kl->", T, P, P, P)

    g = O.classic_cp_gradient(c.indptr, c.indices, c.data, spec.V, M1, W, Phi, spec.alpha0, theta)
    h = 1e-6
    fd = np.zeros_like(Phi)
    for idx in np.ndindex(Phi.shape):
        e = np.zeros_like(Phi)
        e[idx] = h
        fd[idx] = (loss(Phi + e) - loss(Phi - e)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_classic_unwhiten_recovers_population_topics(theta):
    """Population moments M2 = sum a mu mu^T, M3 = sum a mu^3: the whitened
    factors sqrt(a_i) W^T mu_i are orthonormal, T = sum a_i^(-1/2) v_i^3, the
    CP fixed point is ((a_i^(-1/2)) / (1 + theta))^(1/3) v_i, and the classic
    recovery returns mu and a exactly."""
    rng = np.random.default_rng(5)
    V, K = 30, 4
    mu = rng.dirichlet(np.full(V, 0.3), size=K).T
    a = rng.dirichlet(np.ones(K) * 2)
    M2 = (mu * a) @ mu.T
    W, lam, U = O.whitening(M2, K)
    v = np.sqrt(a)[None, :] * (W.T @ mu)
    np.testing.assert_allclose(v.T @ v, np.eye(K), atol=1e-10)
    Phi = v * np.cbrt(a ** -0.5 / (1 + theta))[None, :]
    out = O.classic_unwhiten(Phi, U, lam, theta)
    np.testing.assert_allclose(out["mu"], mu, atol=1e-10)
    np.testing.assert_allclose(out["alpha"], a, atol=1e-10)


def test_classic_fit_from_the_planted_start_stays_near_the_truth():
    """On the 500-word workload the classic rung keeps a start at the planted
    factors within 0.1 mean L1 of the planted topics (it is the estimator, not
    the start, that is checked here)."""
    spec = SPECS["c1"]
    c = generate(spec)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
    m, N = O.first_moment(batches, spec.V)
    W, lam, U = O.whitening(O.classic_second_moment(batches, m, N, spec.alpha0), spec.K)
    a = c.alpha / c.alpha.sum()
    Phi0 = (np.sqrt(a)[None, :] * (W.T @ c.mu)) * np.cbrt(a ** -0.5)[None, :]
    fit = O.fit_batched_classic(batches, spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.03, 5, Phi0)
    assert O.match_topics(fit["mu_simplex"], c.mu)["mean_l1"] < 0.1


# ----------------------------------------------------------------------------
# the fully online mode (R15)
# ----------------------------------------------------------------------------
def test_rebase_transports_whitened_topic_vectors_between_whitenings():
    """Any two whitenings of the same population M2~ see the centred topics
    nu_i as W^T nu_i; rebasing the old view gives the new one exactly (here
    the new whitening is the old one rotated and rescaled), and the planted CP
    fixed point goes to the fixed point of the rotated problem."""
    mu, alpha, a0, a, m, nu = _planted_population()
    K = mu.shape[1]
    M2 = (nu * a) @ nu.T
    W_old, lam, U = O.whitening(M2, K - 1)
    R, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((K - 1, K - 1)))
    for s in (1.0, 2.5):
        W_new = W_old @ R / np.sqrt(s)
        np.testing.assert_allclose(O.rebase_phi(W_old.T @ nu, W_old, W_new), W_new.T @ nu,
                                   atol=1e-12)
    Phi_star = (a / 2.0) ** (1 / 3) * (W_old.T @ nu)
    np.testing.assert_allclose(O.rebase_phi(Phi_star, W_old, W_old @ R), R.T @ Phi_star,
                               atol=1e-12)
    np.testing.assert_allclose(O.rebase_phi(Phi_star, W_old, W_old), Phi_star, atol=1e-12)


def test_online_over_copies_of_one_batch_reduces_to_plain_steps():
    """Streaming copies of the initial batch leaves M1 and M2~ (so W) unchanged,
    so the online fit equals the batched fit with one more pass per copy."""
    c, spec = _small_lda(N=400, seed=41)
    B = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c, 400)][0]
    Phi0 = init_phi(spec.K, spec.K, 3)
    on = O.fit_online([B], [B, B, B], spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.05, 4, Phi0)
    ref = O.fit_batched([B], spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.05, 7, Phi0)
    np.testing.assert_allclose(on["Phi"], ref["Phi"], atol=1e-10)
    assert len(on["trace"]) == 3


def test_online_whitening_covers_every_batch_seen():
    c, spec = _small_lda(N=900, seed=42)
    bs = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c, 300)]
    Phi0 = init_phi(spec.K, spec.K, 4)
    on = O.fit_online(bs[:1], bs[1:], spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.02, 2, Phi0)
    full = O.fit_batched(bs, spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.02, 0, Phi0)
    np.testing.assert_allclose(on["W"], full["W"], atol=1e-12)
    np.testing.assert_allclose(on["m"], full["m"], atol=1e-15)
    init = O.fit_batched(bs[:1], spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.02, 2, Phi0)
    np.testing.assert_allclose(on["Phi_init"], init["Phi"], atol=1e-15)
