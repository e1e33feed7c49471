"""The classic alpha0-corrected estimator rung on the GPU (TLDA_CLASSIC)
against the FP64 oracle, through the C ABI.

Bars: statistics and whitening as for the centred moments (FP64: eigenvalues
1e-10, W 1e-7 relative); the FP32 gradient within 1e-5 relative Frobenius
error of the oracle's; the data term recovered from it (3/n sum of the
per-document third-moment pieces) within 1e-4 (the recovery subtracts the
penalty term, which magnifies the gradient's FP32 rounding; the data term
itself carries about 1e-6, measured by running the same implicit formula in
FP32 on the CPU); recovered topics within 1e-6 of the oracle's recovery.
BF16 contexts: the oracle evaluated on the operands the kernel rounds (W16,
Z16), the rest within the entry-wise bound derived in tests/bf16_ref.py.
"""
import numpy as np
import pytest
import torch

from bf16_ref import assert_within, bf16_round, classic_bf16_bound, z16_like_kernel
from oracle import tlda_oracle as O
from synth import SPECS, generate, init_phi, iter_batches, make_csr_rows

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")

V = 400


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rows(n, seed, max_words=45, long_rows=0):
    rng = np.random.default_rng(seed)
    rows = [{}, {3: 1, 9: 1}, {5: 2}, {7: 3}]      # empty, short (dropped) and L = 3 rows
    for _ in range(long_rows):                      # rows longer than a staged chunk
        words = rng.choice(V, size=int(rng.integers(70, 200)), replace=False)
        rows.append({int(w): int(rng.integers(1, 6)) for w in words})
    while len(rows) < n:
        words = rng.choice(V, size=int(rng.integers(1, max_words)), replace=False)
        rows.append({int(w): int(rng.integers(1, 4)) for w in words})
    return make_csr_rows(rows[:n], V)


def _whitening(D, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    return Q * rng.uniform(5, 30, size=D)[None, :], rng.dirichlet(np.ones(V))


@pytest.mark.parametrize("D,K,n", [(5, 5, 1000), (10, 7, 1601), (20, 30, 777), (33, 40, 515),
                                   (50, 50, 1203), (64, 64, 300), (100, 100, 229),
                                   (128, 128, 130), (3, 12, 64), (1, 1, 37), (120, 16, 90)])
@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_classic_gradient_and_step_match_oracle(D, K, n, theta):
    rp, ci, va = _rows(n, D * 31 + K, long_rows=3)
    W, m = _whitening(D, D * 7 + K)
    a0 = 1.5 if K % 2 else 0.7
    Phi = (init_phi(D, K, D + K) * 0.3).astype(np.float32)
    ctx = tl.tlda_create(V, K, D, a0, theta, classic=True)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    beta = 1e-3
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(rp, ci, va), beta, Pd, g, None, nk)
    torch.cuda.synchronize()
    P64 = Phi.astype(np.float64)
    ref_g = O.classic_cp_gradient(rp, ci, va, V, m, W, P64, a0, theta)
    data, n_kept = O.classic_data_term(rp, ci, va, V, m, W, P64, a0)
    assert int(nk.item()) == n_kept
    gg = g.cpu().numpy().astype(np.float64)
    assert rel(gg, ref_g) < 1e-5
    G = P64.T @ P64
    pen = 3.0 * (1.0 + theta) * P64 @ (G * G)
    assert rel((pen - gg) * n_kept / 3.0, data) < 1e-4
    assert rel(Pd.cpu().numpy(), P64 - beta * ref_g) < 1e-5


def _bf16_reference(rp, ci, va, V, m, W, Phi, a0, theta):
    """The oracle's gradient on the operands the BF16 classic kernel rounds
    (W16 = bf16(fp32 W), Z16 as the kernel forms it) and the derived bound
    on the rest (tests/bf16_ref.py), in gradient units."""
    W16 = bf16_round(W)
    P64 = Phi.astype(np.float64)
    Z16 = z16_like_kernel(W16, Phi)
    data, n_kept = O.classic_data_term(rp, ci, va, V, m, W16, P64, a0, Z=Z16)
    G = P64.T @ P64
    ref = 3.0 * (1.0 + theta) * P64 @ (G * G) - 3.0 / max(n_kept, 1) * data
    bound = 3.0 / max(n_kept, 1) * classic_bf16_bound(rp, ci, va, W16, Z16, P64, m, a0)
    return ref, bound + 2.0 ** -22 * np.abs(ref), n_kept


@pytest.mark.parametrize("D,K,n", [(5, 5, 1000), (20, 30, 777), (50, 50, 1203), (64, 64, 300),
                                   (100, 100, 229), (128, 128, 130), (3, 12, 64), (1, 1, 37)])
def test_classic_bf16_gradient_matches_oracle(D, K, n):
    """BF16 classic rung: W16 = bf16(W) for the gathers, Z16 = bf16(W16 Phi),
    reduction rows rounded to BF16 for the matrix cores.  The oracle is
    evaluated on the same W16 and Z16; the rest (row rounding, FP32
    accumulation) is held to the derived entry-wise bound.  The error against
    the unrounded FP64 gradient is printed."""
    rp, ci, va = _rows(n, D * 37 + K, long_rows=3)
    W, m = _whitening(D, D * 11 + K)
    a0, theta = 1.5, 0.5
    Phi = (init_phi(D, K, D + K) * 0.3).astype(np.float32)
    ctx = tl.tlda_create(V, K, D, a0, theta, classic=True, bf16=True)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(rp, ci, va), 1e-3, Pd, g, None, nk)
    torch.cuda.synchronize()
    ref, bound, n_kept = _bf16_reference(rp, ci, va, V, m, W, Phi, a0, theta)
    assert int(nk.item()) == n_kept
    gg = g.cpu().numpy().astype(np.float64)
    assert_within(gg, ref, bound, f"classic BF16 gradient D={D} K={K}")
    exact = O.classic_cp_gradient(rp, ci, va, V, m, W, Phi.astype(np.float64), a0, theta)
    print(f"D={D} K={K}: {rel(gg, exact):.3g} relative to the unrounded FP64 gradient")


def test_classic_step_writes_whitened_rows_and_skips_empty_batches():
    D = K = 8
    rp, ci, va = _rows(300, 5)
    W, m = _whitening(D, 6)
    ctx = tl.tlda_create(V, K, D, 1.0, classic=True)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.from_numpy((init_phi(D, K, 2) * 0.5).astype(np.float32)).cuda()
    X = torch.empty((300, D), dtype=torch.float32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(rp, ci, va), 0.0, Pd, None, X)
    torch.cuda.synchronize()
    Xr = O.whiten(rp, ci, va, V, m, W)
    assert rel(X.cpu().numpy(), Xr) < 1e-5
    P0 = Pd.clone()
    e_rp = np.zeros(1, dtype=np.int32)
    nk = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(e_rp, np.zeros(0, np.int32),
                                                       np.zeros(0, np.float32)),
                           0.1, Pd, None, None, nk)
    torch.cuda.synchronize()
    assert torch.equal(P0, Pd) and int(nk.item()) == 0
    # a batch of dropped documents only: n = 0, no step
    rp2, ci2, va2 = make_csr_rows([{1: 1}, {}, {2: 1, 3: 1}], V)
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(rp2, ci2, va2), 0.1, Pd, None, None, nk)
    torch.cuda.synchronize()
    assert torch.equal(P0, Pd) and int(nk.item()) == 0


def test_classic_step_is_bit_reproducible():
    D = K = 50
    rp, ci, va = _rows(20000, 9)
    W, m = _whitening(D, 10)
    ctx = tl.tlda_create(V, K, D, 1.0, classic=True)
    tl.tlda_set_whitening(ctx, W, m)
    b = tl.CsrBatch.from_numpy(rp, ci, va)
    outs = []
    for _ in range(2):
        Pd = torch.from_numpy((init_phi(D, K, 3) * 0.3).astype(np.float32)).cuda()
        for _ in range(3):
            tl.tlda_whiten_cp_step(ctx, b, 1e-3, Pd)
        outs.append(Pd.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.fixture(scope="module")
def c1_classic():
    spec = SPECS["c1"]
    c = generate(spec)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
    m, N = O.first_moment(batches, spec.V)
    M2 = O.classic_second_moment(batches, m, N, spec.alpha0)
    W, lam, U = O.whitening(M2, spec.K)
    return {"spec": spec, "corpus": c, "batches": batches, "m": m, "M2": M2, "W": W,
            "lam": lam, "U": U}


def test_classic_refresh_matches_oracle_whitening(c1_classic):
    d = c1_classic
    spec = d["spec"]
    ctx = tl.tlda_create(spec.V, spec.K, spec.K, spec.alpha0, classic=True, eig_iters=100)
    for rp, ci, va, _ in iter_batches(d["corpus"], 777):      # ragged batches
        tl.tlda_update_moments(ctx, tl.CsrBatch.from_numpy(rp, ci, va))
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    W, eig, m = tl.tlda_get_whitening(ctx)
    np.testing.assert_allclose(m, d["m"], rtol=0, atol=1e-15)
    assert rel(eig, d["lam"]) < 1e-10
    assert rel(W, d["W"]) < 1e-7
    np.testing.assert_allclose(W.T @ d["M2"] @ W, np.eye(spec.K), atol=1e-8)


@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_classic_unwhiten_matches_oracle(c1_classic, theta):
    d = c1_classic
    spec = d["spec"]
    ctx = tl.tlda_create(spec.V, spec.K, spec.K, spec.alpha0, theta, classic=True,
                         eig_iters=100)
    for b in d["batches"]:
        tl.tlda_update_moments(ctx, tl.CsrBatch.from_numpy(*b))
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    W, eig, _ = tl.tlda_get_whitening(ctx)
    U = W * np.sqrt(eig)[None, :]
    Phi = (init_phi(spec.K, spec.K, 4) * 0.8).astype(np.float32)
    for flags in (0, tl.TLDA_PROJECT_SIMPLEX):
        mu, alpha, lam = tl.tlda_unwhiten(ctx, torch.from_numpy(Phi).cuda(), flags)
        ref = O.classic_unwhiten(Phi.astype(np.float64), U, eig, theta)
        key = "mu_simplex" if flags else "mu"
        assert rel(mu.cpu().numpy(), ref[key]) < 1e-9
        assert rel(alpha.cpu().numpy(), ref["alpha"]) < 1e-9
        assert rel(lam.cpu().numpy(), ref["lambda"]) < 1e-9


def test_classic_fit_matches_oracle_fit(c1_classic):
    """Five passes of the classic rung from the planted start on the 500-word
    workload: Phi within 1e-4 of the oracle's fit (FP32 steps against FP64)
    and the recovered topics within 0.1 mean L1 of the planted ones."""
    d = c1_classic
    spec = d["spec"]
    c = d["corpus"]
    a = c.alpha / c.alpha.sum()
    Phi0 = (np.sqrt(a)[None, :] * (d["W"].T @ c.mu)) * np.cbrt(a ** -0.5)[None, :]
    ref = O.fit_batched_classic(d["batches"], spec.V, spec.K, spec.K, spec.alpha0, 0.0, 0.03, 5,
                                Phi0)
    ctx = tl.tlda_create(spec.V, spec.K, spec.K, spec.alpha0, classic=True)
    tl.tlda_set_whitening(ctx, d["W"], d["m"])
    Pd = torch.from_numpy(Phi0.astype(np.float32)).cuda()
    dev = [tl.CsrBatch.from_numpy(*b) for b in d["batches"]]
    for _ in range(5):
        for b in dev:
            tl.tlda_whiten_cp_step(ctx, b, 0.03, Pd)
    torch.cuda.synchronize()
    assert rel(Pd.cpu().numpy(), ref["Phi"]) < 1e-4
    mu, _, _ = tl.tlda_unwhiten(ctx, Pd, tl.TLDA_PROJECT_SIMPLEX)
    assert O.match_topics(mu.cpu().numpy(), c.mu)["mean_l1"] < 0.1


def test_classic_config_errors():
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_create(V, 10, 130, 1.0, classic=True)
    assert e.value.status == 2
    ctx = tl.tlda_create(V, 4, 4, 1.0, classic=True)
    W, m = _whitening(4, 1)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.zeros((4, 4), dtype=torch.float32, device="cuda")
    X = torch.zeros((8, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_cp_step(ctx, X, 8, None, 0.1, Pd)
    assert e.value.status == 4


@pytest.mark.parametrize("bf16", [False, True])
def test_classic_step_full_size_tweet_batch(bf16):
    """One full 131 072-document batch of the tweet-shaped workload (V = 20 000,
    K = D = 50), the launch configuration the benchmark times, against the
    oracle's per-document gradient over the same batch (FP32 1e-5; BF16 on
    the rounded operands within the derived bound)."""
    spec = SPECS["c2"]
    c = generate(spec, n_docs=spec.batch)
    rp, ci, va, _ = next(iter_batches(c))
    D = K = spec.K
    rng = np.random.default_rng(23)
    Q, _ = np.linalg.qr(rng.standard_normal((spec.V, D)))
    W = Q * rng.uniform(20, 200, size=D)[None, :]
    m = np.bincount(ci, weights=va, minlength=spec.V) / va.sum()
    Phi = (init_phi(D, K, 9) * 0.3).astype(np.float32)
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.0, classic=True, bf16=bf16)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    tl.tlda_whiten_cp_step(ctx, tl.CsrBatch.from_numpy(rp, ci, va), 1e-4, Pd, g)
    torch.cuda.synchronize()
    if bf16:
        ref, bound, _ = _bf16_reference(rp, ci, va, spec.V, m, W, Phi, spec.alpha0, 0.0)
        assert_within(g.cpu().numpy(), ref, bound, "classic BF16 gradient, full batch")
    else:
        ref = O.classic_cp_gradient(rp, ci, va, spec.V, m, W, Phi.astype(np.float64),
                                    spec.alpha0, 0.0)
        assert rel(g.cpu().numpy(), ref) < 1e-5
