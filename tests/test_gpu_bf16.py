"""GPU parity of the BF16 precision path (TLDA_BF16) against the FP64 oracle.

The BF16 path rounds exactly three things, each round to nearest even: the
FP32 whitening copy (W16 = bf16(fp32(W)), with its own mean projection), the
MFMA operands X and Phi, and the squared scores S^2.  The tests therefore
compare with the oracle evaluated on the same rounded values, which the test
forms itself from the BF16 format's definition, and bound what remains:

* whitening: X = (F - 1 M1^T) W16 is FP32 arithmetic on exact inputs, so it
  meets the FP32 bar (1e-5 relative) against the oracle's whitening by W16;
* gradient data term R1 = X^T (X Phi)^2: with u = 2^-8 the BF16 unit
  roundoff, rounding S^2 moves each term x s^2 by at most u |x| s^2, so
  |R1 - R1_ref| <= u B with B = |X|^T S^2; FP32 accumulation adds far less.
  The tests allow 2u B (the second u covers the FP32 accumulation of R1),
  plus D 2^-23 C with C = |X|^T (|S| (|X| |Phi|)) for the FP32 sums that
  form S (each off by at most D 2^-24 |X| |Phi|).  In the fused step X
  itself is rounded from the kernel's own FP32 row, which can differ from
  the oracle's in the last FP32 bit and so round to the neighbouring BF16
  value: that adds u B + 2u C, and the fused tests allow 4u (B + C).
End to end, the topics of a batched fit must stay within the 0.02 mean-L1
topic tolerance of the FP64 oracle's fit.
"""
import numpy as np
import pytest
import torch

from oracle import tlda_oracle as O
from synth import SPECS, generate, init_phi, iter_batches, make_csr_rows

from bf16_ref import U_BF16, assert_within, bf16_round, fused_bound, rounded_gradient

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")

REL32 = 1e-5


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev_batch(rp, ci, va):
    return tl.CsrBatch.from_numpy(rp, ci, va)


def make_ctx(V, K, D, alpha0=1.0, theta=0.0, **kw):
    return tl.tlda_create(V, K, D, alpha0, theta, bf16=True, **kw)


def _rows(V, n, seed, max_len=45):
    rng = np.random.default_rng(seed)
    rows = [{}, {3: 1, 9: 1}]
    for _ in range(n):
        words = rng.choice(V, size=rng.integers(1, max_len), replace=False)
        rows.append({int(w): int(rng.integers(1, 4)) for w in words})
    return make_csr_rows(rows, V)


def _whitening(V, D, seed, lo=5.0, hi=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    return Q * rng.uniform(lo, hi, size=D)[None, :], rng.dirichlet(np.ones(V))


# ----------------------------------------------------------------------------
# whitening through the BF16 copy
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("D", [1, 3, 5, 8, 10, 20, 32, 33, 50, 64, 65, 100, 128])
def test_bf16_whiten_is_the_whitening_by_the_rounded_matrix(D):
    V = 300
    rp, ci, va = _rows(V, 157, seed=D, max_len=40)
    W, m = _whitening(V, D, seed=D + 1, lo=5, hi=50)
    ctx = make_ctx(V, 1, D)
    tl.tlda_set_whitening(ctx, W, m)
    X, nk = tl.tlda_whiten_batch(ctx, dev_batch(rp, ci, va))
    got = X.cpu().numpy()
    ref = O.whiten(rp, ci, va, V, m, bf16_round(W))
    assert rel(got, ref) < REL32
    st = O.batch_stats(rp, ci, va, V)
    assert np.all(got[~st["keep"]] == 0.0)
    assert int(nk.item()) == st["n_kept"]
    # distance to the whitening by the unrounded W (reported, bounded loosely)
    assert rel(got, O.whiten(rp, ci, va, V, m, W)) < 2e-2


# ----------------------------------------------------------------------------
# CP gradient step from FP32 X (tlda_cp_step)
# ----------------------------------------------------------------------------
def _cp_case(n, D, K, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, D)) * scale
    Phi = init_phi(D, K, seed) * 1.3
    return X.astype(np.float32), Phi.astype(np.float32)


@pytest.mark.parametrize("D,K,n", [(5, 5, 1000), (10, 10, 3001), (20, 20, 777), (50, 50, 4099),
                                   (64, 64, 2048), (100, 100, 1500), (128, 100, 515),
                                   (128, 128, 700), (7, 3, 999), (3, 12, 64), (1, 1, 5),
                                   (30, 60, 333), (65, 17, 129)])
@pytest.mark.parametrize("theta", [0.0, 1.0])
def test_bf16_cp_gradient_within_rounding_bound(D, K, n, theta):
    a0 = 1.0 if D != 100 else 2.0
    X, Phi = _cp_case(n, D, K, seed=D * 131 + K)
    ctx = make_ctx(max(D, 3), K, D, a0, theta)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    beta = 1e-3
    tl.tlda_cp_step(ctx, torch.from_numpy(X).cuda(), n, None, beta, Pd, g)
    ref, B, C = rounded_gradient(X, Phi, n, a0, theta)
    got = g.cpu().numpy().astype(np.float64)
    bound = 2 * U_BF16 * B + D * 2.0 ** -23 * C + 2.0 ** -22 * np.abs(ref)
    assert_within(got, ref, bound, "gradient")
    upd = Phi.astype(np.float64) - beta * got
    assert rel(Pd.cpu().numpy(), upd) < 1e-6
    # error against the unrounded FP64 gradient, reported with a loose bound
    assert rel(got, O.cp_gradient(X.astype(np.float64), Phi.astype(np.float64), n, a0,
                                  theta)) < 5e-2


def test_bf16_cp_step_kept_count_empty_batch_and_reproducibility():
    D = K = 6
    X, Phi = _cp_case(300, D, K, seed=3)
    X[100:200] = 0.0
    ctx = make_ctx(10, K, D)
    Xd = torch.from_numpy(X).cuda()
    Pd = torch.from_numpy(Phi).cuda()
    nk = torch.tensor([200], dtype=torch.int32, device="cuda")
    g = torch.empty_like(Pd)
    tl.tlda_cp_step(ctx, Xd, 300, nk, 0.01, Pd, g)
    ref, B, C = rounded_gradient(X, Phi, 200, 1.0, 0.0)
    assert_within(g.cpu().numpy(), ref, 2 * U_BF16 * B + D * 2.0 ** -23 * C + 1e-7 * np.abs(ref),
                   "gradient with kept count")
    P0 = Pd.clone()
    tl.tlda_cp_step(ctx, Xd, 300, torch.zeros(1, dtype=torch.int32, device="cuda"), 0.01, Pd, g)
    assert torch.equal(P0, Pd)
    tl.tlda_cp_step(ctx, Xd, 0, None, 0.01, Pd, g)
    assert torch.equal(P0, Pd)
    outs = []
    for _ in range(2):
        P = torch.from_numpy(Phi).cuda()
        for _ in range(4):
            tl.tlda_cp_step(ctx, Xd, 300, None, 1e-3, P)
        outs.append(P.cpu())
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("n,D,K,V,a0", [(131072, 50, 50, 20000, 1.0),
                                        (262144, 100, 100, 50000, 2.0)])
def test_bf16_cp_step_full_batch_shapes(n, D, K, V, a0):
    """The benchmark's batch shapes: 131 072 x 50 and 262 144 x 100."""
    X, Phi = _cp_case(n, D, K, seed=17 + D, scale=0.5)
    ctx = make_ctx(V, K, D, a0)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    tl.tlda_cp_step(ctx, torch.from_numpy(X).cuda(), n, None, 1e-4, Pd, g)
    ref, B, C = rounded_gradient(X, Phi, n, a0, 0.0)
    got = g.cpu().numpy().astype(np.float64)
    assert_within(got, ref, 2 * U_BF16 * B + D * 2.0 ** -23 * C + 2.0 ** -22 * np.abs(ref),
                   "full-size gradient")


# ----------------------------------------------------------------------------
# fused whitening + CP step
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("D,K", [(5, 5), (10, 7), (20, 20), (33, 40), (50, 50), (64, 64),
                                 (100, 100), (128, 96), (128, 128), (8, 100), (100, 8),
                                 (1, 1), (7, 1), (16, 3), (33, 2)])
def test_bf16_fused_step_matches_rounded_oracle(D, K):
    """The fused BF16 step (which also forms the finish's squared Gram
    entries) against the oracle on the rounded operands.  At K < 16 a finish
    block's 16 entries span several rows of Phi (up to 16 at K = 1)."""
    V = 400
    rp, ci, va = _rows(V, 1500, seed=D * 7 + K)
    W, m = _whitening(V, D, seed=D * 7 + K + 1)
    a0, theta, beta = 1.5, 0.5, 2e-3
    ctx = make_ctx(V, K, D, a0, theta)
    tl.tlda_set_whitening(ctx, W, m)
    Phi0 = (init_phi(D, K, 2) * 0.8).astype(np.float32)
    Pd = torch.from_numpy(Phi0).cuda()
    g = torch.empty_like(Pd)
    n_rows = len(rp) - 1
    Xo = torch.empty((n_rows, D), dtype=torch.float32, device="cuda")
    nk = torch.empty(1, dtype=torch.int32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, dev_batch(rp, ci, va), beta, Pd, g, Xo, nk)
    X_ref = O.whiten(rp, ci, va, V, m, bf16_round(W))
    n_ref = O.batch_stats(rp, ci, va, V)["n_kept"]
    assert int(nk.item()) == n_ref
    assert rel(Xo.cpu().numpy(), X_ref) < REL32
    ref, B, C = rounded_gradient(X_ref, Phi0, n_ref, a0, theta)
    got = g.cpu().numpy().astype(np.float64)
    assert_within(got, ref, 4 * U_BF16 * (B + C) + 2.0 ** -22 * np.abs(ref), "fused gradient")
    assert rel(Pd.cpu().numpy(), Phi0.astype(np.float64) - beta * got) < 1e-6


def test_bf16_fused_step_at_the_largest_vocabulary():
    """V = 131 072, the largest vocabulary a context takes, with column
    indices over the whole range (0 and V - 1 included): the fused BF16 step
    against the oracle on the rounded whitening, to the bound above."""
    V, D, K = 131072, 50, 50
    rng = np.random.default_rng(131)
    rp, ci, va = make_csr_rows([{0: 2, V - 1: 1, V // 2: 1}, {V - 1: 3}] + [
        {int(w): int(rng.integers(1, 4)) for w in rng.choice(V, size=rng.integers(1, 45),
                                                              replace=False)}
        for _ in range(600)], V)
    W, m = _whitening(V, D, seed=132, lo=200.0, hi=2000.0)
    a0, theta, beta = 1.0, 0.0, 1e-3
    ctx = make_ctx(V, K, D, a0, theta)
    tl.tlda_set_whitening(ctx, W, m)
    Phi0 = (init_phi(D, K, 4) * 0.8).astype(np.float32)
    Pd = torch.from_numpy(Phi0).cuda()
    g = torch.empty_like(Pd)
    n_rows = len(rp) - 1
    Xo = torch.empty((n_rows, D), dtype=torch.float32, device="cuda")
    nk = torch.empty(1, dtype=torch.int32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, dev_batch(rp, ci, va), beta, Pd, g, Xo, nk)
    X_ref = O.whiten(rp, ci, va, V, m, bf16_round(W))
    n_ref = O.batch_stats(rp, ci, va, V)["n_kept"]
    assert int(nk.item()) == n_ref
    assert rel(Xo.cpu().numpy(), X_ref) < REL32
    ref, B, C = rounded_gradient(X_ref, Phi0, n_ref, a0, theta)
    got = g.cpu().numpy().astype(np.float64)
    assert_within(got, ref, 4 * U_BF16 * (B + C) + 2.0 ** -22 * np.abs(ref), "fused gradient")


@pytest.mark.parametrize("workload", ["c2", "c3"])
def test_bf16_fused_step_full_size_within_rounding_bound(workload):
    """The fused BF16 step on one full batch of the tweet-shaped workload
    (131 072 x 50) and of the streaming workload (262 144 x 100, V = 50 000),
    in the launch configuration the benchmark times, against the oracle's
    gradient of the same batch whitened by W16 = bf16(W), element by element
    within the derived bound 4u (B + C) + 2^-22 |ref|.  X is the oracle's
    sparse whitening (tied to the dense definition on sampled rows); the
    kept-row count is exact.  The streaming batch is also staged through the
    compact 16-bit host format and must give the same gradient bit for bit."""
    spec = SPECS[workload]
    c = generate(spec, n_docs=spec.batch)
    rp, ci, va, _ = next(iter_batches(c))
    D = K = spec.K
    rng = np.random.default_rng(37)
    Q, _ = np.linalg.qr(rng.standard_normal((spec.V, D)))
    W = Q * rng.uniform(20, 200, size=D)[None, :]
    m = np.bincount(ci, weights=va, minlength=spec.V) / va.sum()
    Wh = bf16_round(W)
    X = O.whiten_csr(rp, ci, va, spec.V, m, Wh)
    for r in np.concatenate([rng.choice(rp.size - 1, 40, replace=False), [0, rp.size - 2]]):
        a_, b_ = int(rp[r]), int(rp[r + 1])
        one = O.whiten(np.array([0, b_ - a_]), ci[a_:b_], va[a_:b_], spec.V, m, Wh)[0]
        np.testing.assert_allclose(X[r], one, rtol=0, atol=1e-12 * max(1.0, np.abs(one).max()))
    n_ref = int(O.batch_stats(rp, ci, va, spec.V)["n_kept"])
    Phi = (init_phi(D, K, 3) * 0.5).astype(np.float32)
    ref, B, C = rounded_gradient(X, Phi, n_ref, spec.alpha0, 0.0)
    ctx = make_ctx(spec.V, K, D, spec.alpha0)
    tl.tlda_set_whitening(ctx, W, m)
    Pd = torch.from_numpy(Phi).cuda()
    g = torch.empty_like(Pd)
    nk = torch.zeros(1, dtype=torch.int32, device="cuda")
    tl.tlda_whiten_cp_step(ctx, dev_batch(rp, ci, va), 1e-4, Pd, g, None, nk)
    torch.cuda.synchronize()
    assert int(nk.item()) == n_ref
    got = g.cpu().numpy().astype(np.float64)
    assert_within(got, ref, fused_bound(ref, B, C), f"{workload} full-size fused gradient")
    assert rel(Pd.cpu().numpy(), Phi.astype(np.float64) - 1e-4 * got) < 1e-6
    if workload == "c3":
        host = tl.CsrBatchU16(rp, ci, va)
        staged = tl.tlda_stage_batch_u16(ctx, host, 1)
        P2 = torch.from_numpy(Phi).cuda()
        g2 = torch.empty_like(P2)
        tl.tlda_whiten_cp_step(ctx, staged, 1e-4, P2, g2)
        torch.cuda.synchronize()
        assert torch.equal(g2, g) and torch.equal(P2, Pd)


def test_bf16_fused_equals_split_at_full_size_and_is_reproducible():
    """At the benchmark's batch shape the fused BF16 step and BF16 whiten +
    cp_step round the same FP32 rows, so they agree to FP32 summation order."""
    spec = SPECS["c2"]
    c = generate(spec, n_docs=spec.batch)
    rp, ci, va, _ = next(iter_batches(c))
    D = K = spec.K
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((spec.V, D)))
    W = Q * rng.uniform(20, 200, size=D)[None, :]
    m = np.bincount(ci, weights=va, minlength=spec.V)
    m /= m.sum()
    ctx = make_ctx(spec.V, K, D, spec.alpha0)
    tl.tlda_set_whitening(ctx, W, m)
    b = dev_batch(rp, ci, va)
    Phi0 = torch.from_numpy(init_phi(D, K, 5).astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        P = Phi0.clone()
        for _ in range(3):
            tl.tlda_whiten_cp_step(ctx, b, 1e-4, P)
        outs.append(P.cpu())
    assert torch.equal(outs[0], outs[1])
    P2 = Phi0.clone()
    for _ in range(3):
        X, nk = tl.tlda_whiten_batch(ctx, b)
        tl.tlda_cp_step(ctx, X, b.n_rows, nk, 1e-4, P2)
    assert rel(outs[0].numpy(), P2.cpu().numpy()) < REL32
    # sampled rows of the BF16 whitening against the oracle, one by one
    X, nk = tl.tlda_whiten_batch(ctx, b)
    got = X.cpu().numpy()
    Wh = bf16_round(W)
    for r in np.concatenate([rng.choice(spec.batch, 200, replace=False), [0, spec.batch - 1]]):
        a_, b_ = int(rp[r]), int(rp[r + 1])
        one = O.whiten(np.array([0, b_ - a_]), ci[a_:b_], va[a_:b_], spec.V, m, Wh)[0]
        assert np.linalg.norm(got[r] - one) <= REL32 * max(np.linalg.norm(one), 1.0)
    assert int(nk.item()) == O.batch_stats(rp, ci, va, spec.V)["n_kept"]


# ----------------------------------------------------------------------------
# end to end: topics of a batched fit
# ----------------------------------------------------------------------------
def test_bf16_batched_fit_topics_match_oracle():
    spec = SPECS["c1"]
    c = generate(spec)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
    passes, beta, theta = 20, 0.03, 0.0
    Phi0 = init_phi(spec.K, spec.K, 4)
    ref = O.fit_batched(batches, spec.V, spec.K, spec.K, spec.alpha0, theta, beta, passes, Phi0)
    ctx = make_ctx(spec.V, spec.K, spec.K, spec.alpha0, theta, eig_iters=100)
    dbs = [dev_batch(*b) for b in batches]
    for b in dbs:
        tl.tlda_update_moments(ctx, b)
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    Pd = torch.from_numpy(Phi0.astype(np.float32)).cuda()
    for _ in range(passes):
        for b in dbs:
            tl.tlda_whiten_cp_step(ctx, b, beta, Pd)
    mu, alpha, lam = tl.tlda_unwhiten(ctx, Pd, tl.TLDA_PROJECT_SIMPLEX)
    got = mu.cpu().numpy()
    l1 = np.abs(got - ref["mu_simplex"]).sum(axis=0)
    assert l1.mean() <= 0.02
    truth = O.match_topics(got, c.mu)["mean_l1"]
    truth_ref = O.match_topics(ref["mu_simplex"], c.mu)["mean_l1"]
    assert abs(truth - truth_ref) <= 0.02


def test_bf16_context_shape_limit_and_checkpoint_roundtrip():
    with pytest.raises(tl.TldaError) as e:
        make_ctx(300, 10, 129)
    assert e.value.status == 2
    with pytest.raises(tl.TldaError) as e:
        make_ctx(300, 129, 10)
    assert e.value.status == 2
    # the BF16 copy is rebuilt from a loaded checkpoint
    V, D, K = 200, 12, 12
    rp, ci, va = _rows(V, 300, seed=4, max_len=30)
    W, m = _whitening(V, D, seed=5)
    a = make_ctx(V, K, D)
    tl.tlda_set_whitening(a, W, m)
    blob = tl.tlda_save_state(a)
    bctx = make_ctx(V, K, D)
    tl.tlda_load_state(bctx, blob)
    xa, _ = tl.tlda_whiten_batch(a, dev_batch(rp, ci, va))
    xb, _ = tl.tlda_whiten_batch(bctx, dev_batch(rp, ci, va))
    assert torch.equal(xa, xb)


def test_timing_events_bracket_the_main_kernel():
    V, D, K = 300, 20, 20
    rp, ci, va = _rows(V, 3000, seed=8)
    W, m = _whitening(V, D, seed=9)
    for bf16 in (False, True):
        ctx = tl.tlda_create(V, K, D, 1.0, 0.0, bf16=bf16)
        tl.tlda_set_whitening(ctx, W, m)
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        stops = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        for e in starts + stops:
            e.record()
        tl.tlda_set_timing_events(ctx, starts, stops)
        P = torch.from_numpy(init_phi(D, K, 1).astype(np.float32)).cuda()
        b = dev_batch(rp, ci, va)
        tl.tlda_whiten_cp_step(ctx, b, 1e-3, P)
        X, nk = tl.tlda_whiten_batch(ctx, b)
        tl.tlda_cp_step(ctx, X, b.n_rows, nk, 1e-3, P)
        torch.cuda.synchronize()
        ms = [s.elapsed_time(t) for s, t in zip(starts, stops)]
        assert all(0.0 < x < 1000.0 for x in ms)
        tl.tlda_set_timing_events(ctx, [], [])
        tl.tlda_whiten_cp_step(ctx, b, 1e-3, P)
        torch.cuda.synchronize()
