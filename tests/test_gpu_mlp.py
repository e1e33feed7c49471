"""GPU checks of the document-topic encoder against its FP64 oracle
(oracle/mlp_oracle.py), through the C ABI.

The encoder's matrix products take BF16 operands (weights, the input rows and
the hidden activations, each rounded to nearest even) with FP32 accumulation.
The oracle is evaluated on the same rounded weights and inputs (rounded by the
test with the format's definition); the hidden activations and the
back-propagated errors are rounded on the GPU only, at most three times on
the forward path and six on the backward path, each by at most u = 2^-8
relatively.  The bars are 5u for the output proportions and 10u for the
gradients (relative Frobenius error per tensor), and 2u for the loss.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M
from oracle import tlda_oracle as O
from synth import SPECS, generate, iter_batches

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")

U = 2.0 ** -8


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def bf16_round(a):
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def init_params(d_in, hidden, k_out, seed, scale=1.0):
    """Seeded uniform initialisation, +-sqrt(6 / (fan_in + fan_out)) per matrix."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, shp in M.shapes(d_in, hidden, k_out).items():
        if len(shp) == 2:
            lim = scale * np.sqrt(6.0 / (shp[0] + shp[1]))
            p[k] = rng.uniform(-lim, lim, size=shp)
        else:
            p[k] = rng.uniform(-0.1, 0.1, size=shp)
    return p


def rounded(params):
    return {k: (bf16_round(v) if v.ndim == 2 else np.asarray(v, dtype=np.float32).astype(np.float64))
            for k, v in params.items()}


def make_mlp(d_in, hidden, k_out, max_batch, params):
    m = tl.tlda_mlp_create(d_in, hidden, k_out, max_batch)
    tl.tlda_mlp_set_params(m, M.pack(params).astype(np.float32))
    return m


SHAPES = [(50, 256, 50, 1000), (7, 33, 5, 130), (100, 256, 100, 300), (3, 64, 2, 64),
          (50, 256, 50, 4096)]


@pytest.mark.parametrize("d_in,hidden,k_out,n", SHAPES)
def test_forward_matches_oracle(d_in, hidden, k_out, n):
    params = init_params(d_in, hidden, k_out, seed=d_in + hidden)
    X = np.random.default_rng(1).standard_normal((n, d_in)).astype(np.float32)
    m = make_mlp(d_in, hidden, k_out, 256, params)
    P = tl.tlda_mlp_forward(m, torch.from_numpy(X).cuda()).cpu().numpy()
    ref = M.forward(rounded(params), bf16_round(X))["P"]
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-5)
    assert rel(P, ref) < 5 * U
    # parameters round-trip
    assert np.array_equal(tl.tlda_mlp_get_params(m), M.pack(params).astype(np.float32))


@pytest.mark.parametrize("d_in,hidden,k_out,n", SHAPES)
def test_gradients_match_oracle(d_in, hidden, k_out, n):
    params = init_params(d_in, hidden, k_out, seed=3 * d_in + hidden, scale=1.5)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((n, d_in)).astype(np.float32)
    T = rng.dirichlet(np.full(k_out, 0.3), size=n).astype(np.float32)
    m = make_mlp(d_in, hidden, k_out, max(n, 1), params)
    g, loss = tl.tlda_mlp_gradients(m, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda())
    gref, lref = M.gradients(rounded(params), bf16_round(X), T.astype(np.float64))
    got = M.unpack(g.cpu().numpy().astype(np.float64), d_in, hidden, k_out)
    for k in M.PARAM_ORDER:
        assert rel(got[k], gref[k]) < 10 * U, k
    assert abs(float(loss.item()) - lref) <= 2 * U * abs(lref)


def test_adam_step_follows_the_oracle():
    d_in, hidden, k_out, n = 50, 256, 50, 512
    params = init_params(d_in, hidden, k_out, seed=7)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((n, d_in)).astype(np.float32)
    T = rng.dirichlet(np.full(k_out, 0.3), size=n).astype(np.float32)
    m = make_mlp(d_in, hidden, k_out, n, params)
    lr = 1e-3
    tl.tlda_mlp_train_step(m, torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), lr)
    got = M.unpack(tl.tlda_mlp_get_params(m).astype(np.float64), d_in, hidden, k_out)
    gref, _ = M.gradients(rounded(params), bf16_round(X), T.astype(np.float64))
    ref = M.adam_step({k: np.asarray(v, dtype=np.float32).astype(np.float64)
                       for k, v in params.items()}, gref, {}, lr)
    for k in M.PARAM_ORDER:
        # the first step moves every entry by lr * g / (|g| + eps): where the
        # oracle's gradient is not tiny, the move must agree in sign and size
        big = np.abs(gref[k]) > 0.05 * np.abs(gref[k]).max()
        d = np.abs(got[k] - ref[k])[big]
        assert np.all(d <= 0.05 * lr + 1e-7), k


def test_training_reduces_the_loss_of_a_teacher_task():
    d_in, hidden, k_out = 20, 128, 10
    teacher = init_params(d_in, hidden, k_out, seed=11, scale=2.0)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((8192, d_in)).astype(np.float32)
    T = M.forward(teacher, X.astype(np.float64))["P"].astype(np.float32)
    student = init_params(d_in, hidden, k_out, seed=12)
    m = make_mlp(d_in, hidden, k_out, 1024, student)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    loss = torch.empty(1, device="cuda")
    entropy = float(-(T * np.log(T)).sum() / T.shape[0])
    l0 = M.loss(M.forward(student, X.astype(np.float64))["P"], T.astype(np.float64))
    for epoch in range(30):
        for b in range(0, 8192, 1024):
            tl.tlda_mlp_train_step(m, Xd[b:b + 1024], Td[b:b + 1024], 2e-3, loss)
    trained = M.unpack(tl.tlda_mlp_get_params(m).astype(np.float64), d_in, hidden, k_out)
    l1 = M.loss(M.forward(trained, X.astype(np.float64))["P"], T.astype(np.float64))
    # cross-entropy is at least the targets' entropy; training closes most of the gap
    assert l1 - entropy < 0.2 * (l0 - entropy)


# ----------------------------------------------------------------------------
# the solve as judge and fallback
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def c1_setup():
    spec = SPECS["c1"]
    c = generate(spec)
    batches = [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]
    m1, N = O.first_moment(batches, spec.V)
    M2 = O.centered_second_moment(batches, m1, N, spec.alpha0)
    W, lam, Uv = O.whitening(M2, spec.K)
    return spec, c, batches, m1, W


def test_judge_keeps_good_rows_and_solves_the_others(c1_setup):
    spec, c, batches, m1, W = c1_setup
    K = spec.K
    ctx = tl.tlda_create(spec.V, K, K, spec.alpha0)
    tl.tlda_set_whitening(ctx, W, m1)
    rp, ci, va = batches[0]
    X, _ = tl.tlda_whiten_batch(ctx, tl.CsrBatch.from_numpy(rp, ci, va))
    n = X.shape[0]
    mu = torch.from_numpy(np.ascontiguousarray(c.mu)).cuda()
    m = make_mlp(K, 64, K, 512, init_params(K, 64, K, seed=21))
    raw = tl.tlda_mlp_forward(m, X).cpu().numpy()
    A = O.inference_matrix(np.ascontiguousarray(c.mu), m1, W)
    Xo = O.whiten(rp, ci, va, spec.V, m1, W)
    ref = O.infer_doc_topics(Xo[:100], A, 3000)
    # an infinite tolerance accepts every encoder output unchanged
    th, ns = tl.tlda_infer_doc_topics_mlp(ctx, m, X, n, mu, 1e30, 500)
    assert int(ns.item()) == 0
    assert np.array_equal(th.cpu().numpy(), raw)
    # a zero tolerance steps every row to the oracle's minimiser, from the
    # encoder's output and, without an encoder, from 1/K
    for enc in (m, None):
        th, ns = tl.tlda_infer_doc_topics_mlp(ctx, enc, X, n, mu, 0.0, 3000)
        assert int(ns.item()) == n
        assert np.abs(th.cpu().numpy()[:100] - ref).sum(axis=1).max() < 2e-3
    # min_steps refinement steps happen whatever the tolerance; only rows that
    # need more are counted
    th, ns = tl.tlda_infer_doc_topics_mlp(ctx, m, X, n, mu, 1e30, 500, min_steps=3)
    assert int(ns.item()) == 0
    assert np.all(np.any(th.cpu().numpy() != raw, axis=1))
    # a middle tolerance: rows whose encoder output passes keep it, the others
    # are stepped until they pass (oracle gaps, with FP32 slack)
    gaps = M.simplex_ls_gap(Xo, A, raw.astype(np.float64))
    tol = float(np.median(gaps))
    th, ns = tl.tlda_infer_doc_topics_mlp(ctx, m, X, n, mu, tol, 5000)
    out = th.cpu().numpy()
    changed = np.any(out != raw, axis=1)
    assert int(ns.item()) == int(changed.sum())
    assert 0.3 * n < changed.sum() < 0.7 * n
    assert np.all(gaps[~changed] <= tol * (1 + 1e-3) + 1e-6)
    after = M.simplex_ls_gap(Xo, A, out.astype(np.float64))
    assert np.all(after[changed] <= tol * (1 + 1e-2) + 1e-5)


def test_encoder_rejects_mismatched_widths_and_bad_arguments(c1_setup):
    spec, c, batches, m1, W = c1_setup
    ctx = tl.tlda_create(spec.V, spec.K, spec.K, spec.alpha0)
    tl.tlda_set_whitening(ctx, W, m1)
    m = make_mlp(spec.K + 1, 32, spec.K, 64, init_params(spec.K + 1, 32, spec.K, seed=1))
    X = torch.zeros((4, spec.K + 1), device="cuda")
    mu = torch.from_numpy(np.ascontiguousarray(c.mu)).cuda()
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_infer_doc_topics_mlp(ctx, m, X, 4, mu, 0.1, 10)
    assert e.value.status == 2
    X65 = torch.zeros((65, spec.K + 1), device="cuda")
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_mlp_gradients(m, X65, torch.full((65, spec.K), 1.0 / spec.K, device="cuda"))
    assert e.value.status == 2
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_mlp_create(10, 2000, 5, 16)
    assert e.value.status == 2
    bad = M.pack(init_params(spec.K + 1, 32, spec.K, seed=1)).astype(np.float32)
    bad[3] = np.nan
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_mlp_set_params(m, bad)
    assert e.value.status == 1


def test_trained_encoder_gains_over_the_plain_solve():
    """Trained on solve outputs of tweet-shaped documents, the encoder's start
    point reaches a converged solve in far fewer projected-gradient steps than
    the uniform start: with the same small step budget its result is much
    closer, and its raw output alone is closer than the budgeted plain solve."""
    spec = SPECS["c2"]
    n_train, n_test = 196608, 32768
    c = generate(spec, n_docs=n_train + n_test)
    K = spec.K
    ctx = tl.tlda_create(spec.V, K, K, spec.alpha0)
    X = torch.empty((c.n_docs, K), dtype=torch.float32, device="cuda")
    for rp, ci, va, first in iter_batches(c):
        b = tl.CsrBatch.from_numpy(rp, ci, va)
        if first < n_train:
            tl.tlda_update_moments(ctx, b)
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    for rp, ci, va, first in iter_batches(c):
        n = rp.shape[0] - 1
        tl.tlda_whiten_batch(ctx, tl.CsrBatch.from_numpy(rp, ci, va), X[first:first + n])
    mu = torch.from_numpy(np.ascontiguousarray(c.mu)).cuda()
    Xtr, Xte = X[:n_train].contiguous(), X[n_train:].contiguous()
    Ttr, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xtr, n_train, mu, 1e-7, 2000)
    m = make_mlp(K, 256, K, 4096, init_params(K, 256, K, seed=5))
    gen = torch.Generator().manual_seed(3)
    for ep in range(6):
        perm = torch.randperm(n_train, generator=gen).cuda()
        Xs, Ts = Xtr[perm].contiguous(), Ttr[perm].contiguous()
        for s in range(0, n_train, 4096):
            tl.tlda_mlp_train_step(m, Xs[s:s + 4096], Ts[s:s + 4096], 2e-3)
    conv, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xte, n_test, mu, 0.0, 5000)
    budget = 16

    def l1(th):
        return float((th - conv).abs().sum(dim=1).mean())

    cold, _ = tl.tlda_infer_doc_topics_mlp(ctx, None, Xte, n_test, mu, 0.0, budget)
    warm, _ = tl.tlda_infer_doc_topics_mlp(ctx, m, Xte, n_test, mu, 0.0, budget)
    raw = tl.tlda_mlp_forward(m, Xte)
    assert l1(warm) < 0.5 * l1(cold)
    assert l1(raw) < l1(cold)
