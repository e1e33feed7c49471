"""Batched time slices through the C ABI: one multi-slice step (a persistent
reduction launch over every slice plus one finish launch) against the
single-slice fused step of each slice, the autotuner, and replays of a
captured HIP graph against eager execution.

The single-slice BF16 step is itself checked against the FP64 oracle
(tests/test_gpu_bf16.py); here the multi-slice step must reproduce it up to
the order of its FP32 partial sums (the two launches split a slice's rows
over different numbers of blocks): 1e-5 relative.  Replays of a graph run
the same kernels with the same launch shapes as eager steps and must match
them bit for bit.
"""
import numpy as np
import pytest
import torch

from synth import init_phi, make_csr_rows

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")

V = 300


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    rows = [{}, {3: 1, 9: 1}] if n >= 2 else []
    for _ in range(max(n - len(rows), 0)):
        words = rng.choice(V, size=rng.integers(1, 40), replace=False)
        rows.append({int(w): int(rng.integers(1, 4)) for w in words})
    return make_csr_rows(rows[:n], V)


def _slice(D, K, n_rows, seed, stream):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    W = Q * rng.uniform(5, 30, size=D)[None, :]
    m = rng.dirichlet(np.ones(V))
    ctx = tl.tlda_create(V, K, D, 1.0 + 0.5 * (seed % 3), 0.25 * (seed % 2), bf16=True,
                         stream=stream)
    tl.tlda_set_whitening(ctx, W, m)
    rp, ci, va = _rows(n_rows, seed + 100)
    return ctx, tl.CsrBatch.from_numpy(rp, ci, va), (init_phi(D, K, seed) * 0.9).astype(np.float32)


SLICES = [(10, 10, 3000), (20, 20, 1500), (50, 50, 4100), (7, 7, 1), (64, 64, 700),
          (20, 10, 2300), (33, 40, 0), (50, 50, 130)]


@pytest.fixture()
def side_stream():
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    return s


def _build(stream, slices=SLICES, seed0=1):
    ctxs, batches, phis0 = [], [], []
    for i, (D, K, n) in enumerate(slices):
        c, b, p = _slice(D, K, n, seed0 + i, stream)
        ctxs.append(c)
        batches.append(b)
        phis0.append(p)
    torch.cuda.synchronize()
    return ctxs, batches, phis0


def test_multi_step_matches_single_slice_steps(side_stream):
    ctxs, batches, phis0 = _build(side_stream)
    betas = [1e-3 * (1 + i) for i in range(len(ctxs))]
    Ps = [torch.from_numpy(p).cuda() for p in phis0]
    nk = torch.zeros(len(ctxs), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    plan = tl.tlda_multi_create(ctxs, batches, Ps, betas, nk)
    for _ in range(3):
        tl.tlda_multi_step(plan)
    side_stream.synchronize()
    for i, (c, b, p0) in enumerate(zip(ctxs, batches, phis0)):
        P = torch.from_numpy(p0).cuda()
        n1 = torch.zeros(1, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        for _ in range(3):
            tl.tlda_whiten_cp_step(c, b, betas[i], P, None, None, n1)
        side_stream.synchronize()
        if b.n_rows == 0:
            assert torch.equal(Ps[i].cpu(), torch.from_numpy(p0))
            assert int(nk[i].item()) == 0
        else:
            assert rel(Ps[i].cpu().numpy(), P.cpu().numpy()) < 1e-5, SLICES[i]
            assert int(nk[i].item()) == int(n1.item())


# One slice per shape class of the multi-slice kernel: D in {5, 12, 30, 50}
# (8-column groups G = 1, 2, 4, 8 of the BF16 whitening copy; padded D 32 or
# 64) times K in {10, 20, 50} (padded K 16, 32, 64), with uneven row counts.
SHAPE_CLASSES = [(D, K) for D in (5, 12, 30, 50) for K in (10, 20, 50)]


@pytest.mark.parametrize("tile", [(64, 4), (32, 4), (64, 8)])
def test_multi_step_matches_oracle_in_every_shape_class(side_stream, tile):
    """One multi-slice step over twelve slices (every shape class the
    persistent kernel dispatches on) plus an empty slice, each against the
    oracle's gradient of its own batch whitened by its own W16 = bf16(W),
    within the derived element-wise bound of a fused BF16 step.  The gradient
    is recovered from the update, (Phi0 - Phi1) / beta, which adds at most
    2^-24 |Phi1| / beta; the kept-row counts must be exact."""
    from bf16_ref import assert_within, bf16_round, fused_bound, rounded_gradient
    from oracle import tlda_oracle as O
    ctxs, batches, phis0, host, whit, params = [], [], [], [], [], []
    slices = [(D, K, 97 + 331 * i) for i, (D, K) in enumerate(SHAPE_CLASSES)] + [(20, 20, 0)]
    for i, (D, K, n) in enumerate(slices):
        seed = 50 + i
        rng = np.random.default_rng(seed)
        Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
        W = Q * rng.uniform(5, 30, size=D)[None, :]
        m = rng.dirichlet(np.ones(V))
        a0, theta = 1.0 + 0.5 * (i % 3), 0.25 * (i % 2)
        ctx = tl.tlda_create(V, K, D, a0, theta, bf16=True, stream=side_stream)
        tl.tlda_set_whitening(ctx, W, m)
        rp, ci, va = _rows(n, seed + 100)
        ctxs.append(ctx)
        batches.append(tl.CsrBatch.from_numpy(rp, ci, va))
        phis0.append((init_phi(D, K, seed) * 0.9).astype(np.float32))
        host.append((rp, ci, va))
        whit.append((W, m))
        params.append((a0, theta))
    betas = [2e-3 * (1 + i % 4) for i in range(len(ctxs))]
    Ps = [torch.from_numpy(p).cuda() for p in phis0]
    nk = torch.full((len(ctxs),), -1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    plan = tl.tlda_multi_create(ctxs, batches, Ps, betas, nk)
    tl.tlda_multi_set_tile(plan, *tile)
    assert tl.tlda_multi_get_tile(plan) == tile
    tl.tlda_multi_step(plan)
    side_stream.synchronize()
    for i, ((D, K, n), (rp, ci, va), (W, m), (a0, theta)) in enumerate(
            zip(slices, host, whit, params)):
        st = O.batch_stats(rp, ci, va, V)
        assert int(nk[i].item()) == st["n_kept"], slices[i]
        P1 = Ps[i].cpu().numpy().astype(np.float64)
        if st["n_kept"] == 0:
            assert np.array_equal(P1, phis0[i]), slices[i]
            continue
        X_ref = O.whiten(rp, ci, va, V, m, bf16_round(W))
        ref, B, C = rounded_gradient(X_ref, phis0[i], st["n_kept"], a0, theta)
        got = (phis0[i].astype(np.float64) - P1) / betas[i]
        bound = fused_bound(ref, B, C) + 2.0 ** -24 * np.abs(P1) / betas[i]
        assert_within(got, ref, bound, f"slice {i} (D={D}, K={K}, n={n})")


def test_autotune_restores_phi_and_chooses_a_valid_shape(side_stream):
    ctxs, batches, phis0 = _build(side_stream, seed0=11)
    Ps = [torch.from_numpy(p).cuda() for p in phis0]
    torch.cuda.synchronize()
    plan = tl.tlda_multi_create(ctxs, batches, Ps, [2e-3] * len(ctxs))
    default = tl.tlda_multi_get_blocks(plan)
    assert tl.tlda_multi_get_tile(plan) == (64, 4)
    best = tl.tlda_multi_autotune(plan, 2)
    assert best > 0 and tl.tlda_multi_get_blocks(plan) == best
    best_tile = tl.tlda_multi_get_tile(plan)
    assert best_tile in ((64, 4), (32, 4), (64, 8))
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_multi_set_tile(plan, 48, 4)
    assert e.value.status == 1
    assert tl.tlda_multi_get_tile(plan) == best_tile
    for P, p0 in zip(Ps, phis0):
        assert torch.equal(P.cpu(), torch.from_numpy(p0))
    # every tile and launch shape gives the same step up to the partial-sum order
    outs = []
    for tile, blocks in (((64, 4), default), (best_tile, best), ((32, 4), 37), ((64, 8), 37)):
        for P, p0 in zip(Ps, phis0):
            P.copy_(torch.from_numpy(p0).cuda())
        torch.cuda.synchronize()
        tl.tlda_multi_set_tile(plan, *tile)
        tl.tlda_multi_set_blocks(plan, blocks)
        tl.tlda_multi_step(plan)
        side_stream.synchronize()
        outs.append([P.cpu().numpy().copy() for P in Ps])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert rel(a, b) < 1e-5


def test_graph_replays_match_eager_steps(side_stream):
    slices_a = SLICES[:5]
    ctxs, batches, phis0 = _build(side_stream, slices_a, seed0=21)
    # two batch indices: a second set of batches for the same slices
    batches2 = [_rows(n // 2 + 1, 500 + i) for i, (_, _, n) in enumerate(slices_a)]
    batches2 = [tl.CsrBatch.from_numpy(*r) for r in batches2]
    betas = [1e-3] * len(ctxs)

    def fresh():
        return [torch.from_numpy(p).cuda() for p in phis0]

    # eager
    Pe = fresh()
    torch.cuda.synchronize()
    p1 = tl.tlda_multi_create(ctxs, batches, Pe, betas)
    p2 = tl.tlda_multi_create(ctxs, batches2, Pe, betas)
    eager = []
    for _ in range(3):
        tl.tlda_multi_step(p1)
        tl.tlda_multi_step(p2)
        side_stream.synchronize()
        eager.append([P.cpu().numpy().copy() for P in Pe])
    # graph of one pass (both batch indices), replayed three times with
    # unrelated eager work and synchronisations in between
    Pg = fresh()
    torch.cuda.synchronize()
    g1 = tl.tlda_multi_create(ctxs, batches, Pg, betas)
    g2 = tl.tlda_multi_create(ctxs, batches2, Pg, betas)
    graph = tl.tlda_graph_capture([g1, g2])
    for r in range(3):
        tl.tlda_graph_launch(graph)
        side_stream.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        for a, b in zip([P.cpu().numpy() for P in Pg], eager[r]):
            assert np.array_equal(a, b)


def test_multi_rejects_bad_plans(side_stream):
    ctxs, batches, phis0 = _build(side_stream, SLICES[:2], seed0=31)
    Ps = [torch.from_numpy(p).cuda() for p in phis0]
    torch.cuda.synchronize()
    fp32 = tl.tlda_create(V, 10, 10, 1.0, stream=side_stream)
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_multi_create([ctxs[0], fp32], batches, Ps, [1e-3, 1e-3])
    assert e.value.status == 2
    big = tl.tlda_create(V, 100, 100, 1.0, bf16=True, stream=side_stream)
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_multi_create([ctxs[0], big], batches, Ps, [1e-3, 1e-3])
    assert e.value.status == 2
    classic = tl.tlda_create(V, 20, 20, 1.0, bf16=True, classic=True, stream=side_stream)
    rng0 = np.random.default_rng(3)
    tl.tlda_set_whitening(classic, np.linalg.qr(rng0.standard_normal((V, 20)))[0] * 10,
                          rng0.dirichlet(np.ones(V)))
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_multi_create([ctxs[0], classic], batches, Ps, [1e-3, 1e-3])
    assert e.value.status == 1
    nowhite = tl.tlda_create(V, 20, 20, 1.0, bf16=True, stream=side_stream)
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_multi_create([ctxs[0], nowhite], batches, Ps, [1e-3, 1e-3])
    assert e.value.status == 4
    # contexts on the null stream cannot be captured
    c0 = tl.tlda_create(V, 10, 10, 1.0, bf16=True, stream=torch.cuda.default_stream())
    rng = np.random.default_rng(0)
    tl.tlda_set_whitening(c0, np.linalg.qr(rng.standard_normal((V, 10)))[0] * 10,
                          rng.dirichlet(np.ones(V)))
    P0 = torch.from_numpy(init_phi(10, 10, 1).astype(np.float32)).cuda()
    plan = tl.tlda_multi_create([c0], [batches[0]], [P0], [1e-3])
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_graph_capture([plan])
    assert e.value.status == 1


def test_release_frees_the_accumulator_and_keeps_the_whitening(side_stream):
    rp, ci, va = _rows(2000, 77)
    b = tl.CsrBatch.from_numpy(rp, ci, va)
    ctx = tl.tlda_create(V, 12, 12, 1.0, bf16=True, stream=side_stream)
    torch.cuda.synchronize()
    tl.tlda_update_moments(ctx, b)
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W | tl.TLDA_RELEASE)
    W, eig, m = tl.tlda_get_whitening(ctx)
    N, skipped, totals = tl.tlda_get_stats(ctx)
    assert N == 0 and skipped == 0 and not totals.any()
    X1, _ = tl.tlda_whiten_batch(ctx, b)
    side_stream.synchronize()
    # a fresh accumulation after the release gives the same whitening
    tl.tlda_update_moments(ctx, b)
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    W2, _, _ = tl.tlda_get_whitening(ctx)
    assert rel(W2, W) < 1e-9
    X2, _ = tl.tlda_whiten_batch(ctx, b)
    side_stream.synchronize()
    assert rel(X1.cpu().numpy(), X2.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("bf16,D,K", [(True, 50, 50), (True, 20, 10), (False, 50, 50),
                                      (False, 7, 5), (True, 100, 100), (False, 64, 64),
                                      (False, 100, 100), (False, 120, 40)])
def test_captured_steps_of_one_context_match_eager(side_stream, bf16, D, K):
    """Replays of the captured steps equal the eager steps bit for bit (the
    two largest shapes also capture the once-per-step Gram kernel)."""
    rng = np.random.default_rng(D + K)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    W = Q * rng.uniform(5, 30, size=D)[None, :]
    m = rng.dirichlet(np.ones(V))
    ctx = tl.tlda_create(V, K, D, 1.0, 0.5, bf16=bf16, validate_csr=True, stream=side_stream)
    tl.tlda_set_whitening(ctx, W, m)
    batches = [tl.CsrBatch.from_numpy(*_rows(n, 900 + n)) for n in (2500, 1, 777)]
    Phi0 = (init_phi(D, K, 3) * 0.9).astype(np.float32)
    beta = 2e-3
    Pe = torch.from_numpy(Phi0).cuda()
    torch.cuda.synchronize()
    eager = []
    for _ in range(3):
        for b in batches:
            tl.tlda_whiten_cp_step(ctx, b, beta, Pe)
        side_stream.synchronize()
        eager.append(Pe.cpu().numpy().copy())
    Pg = torch.from_numpy(Phi0).cuda()
    torch.cuda.synchronize()
    g = tl.tlda_graph_capture_steps(ctx, batches, beta, Pg)
    for r in range(3):
        tl.tlda_graph_launch(g)
        side_stream.synchronize()
        junk = torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert np.array_equal(Pg.cpu().numpy(), eager[r]), r


def test_captured_steps_reject_unsupported_contexts(side_stream):
    rp, ci, va = _rows(100, 5)
    b = tl.CsrBatch.from_numpy(rp, ci, va)
    rng = np.random.default_rng(1)
    P = torch.zeros((150, 40), dtype=torch.float32, device="cuda")
    big = tl.tlda_create(V, 40, 150, 1.0, stream=side_stream)      # FP32, beyond fused shapes
    Q, _ = np.linalg.qr(rng.standard_normal((V, 150)))
    tl.tlda_set_whitening(big, Q * 10, rng.dirichlet(np.ones(V)))
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_graph_capture_steps(big, [b], 1e-3, P)
    assert e.value.status == 2
    cl = tl.tlda_create(V, 8, 8, 1.0, classic=True, stream=side_stream)
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_graph_capture_steps(cl, [b], 1e-3, P[:8, :8].contiguous())
    assert e.value.status == 1
    nul = tl.tlda_create(V, 8, 8, 1.0, bf16=True, stream=torch.cuda.default_stream())
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_graph_capture_steps(nul, [b], 1e-3, P[:8, :8].contiguous())
    assert e.value.status == 1
    nw = tl.tlda_create(V, 8, 8, 1.0, bf16=True, stream=side_stream)   # no whitening yet
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_graph_capture_steps(nw, [b], 1e-3, P[:8, :8].contiguous())
    assert e.value.status == 4
