"""The allocation-free step (tlda_whiten_cp_step_noalloc) against
tlda_whiten_cp_step through the C ABI: two calls in a row on one context,
the second with a smaller batch, each compared with the allocating step run
from the same Phi on the same batch.  Bar: the FP32 bar of the whitened
moments, 1e-5 relative (the two differ only in the order of the FP32
partial sums when the allocation-free grid is capped, and not at all when it
is not).  Also: the shapes and contexts it refuses, and the kept-row counts
(exact)."""
import numpy as np
import pytest
import torch

from synth import SPECS, generate, init_phi, iter_batches

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")

REL32 = 1e-5


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def tweet():
    spec = SPECS["c2"]
    c = generate(spec, n_docs=spec.batch)
    rp, ci, va, _ = next(iter_batches(c))
    small = 5000
    return spec, (rp, ci, va), (rp[:small + 1].copy(), ci[:rp[small]].copy(),
                                va[:rp[small]].copy())


def _whitening(V, D, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((V, D)))
    return Q * rng.uniform(20, 200, size=D)[None, :], rng.dirichlet(np.ones(V))


@pytest.mark.parametrize("D,K,bf16,tuned_blocks", [(50, 50, True, 0), (100, 100, True, 2048),
                                                   (50, 50, False, 0), (20, 30, False, 0),
                                                   (100, 100, False, 0)])
def test_noalloc_step_matches_the_allocating_step(tweet, D, K, bf16, tuned_blocks, monkeypatch):
    """tuned_blocks = 2048 makes the allocating step use 2048 blocks, where
    the allocation-free grid is capped at floor(4 Mi / (D K)) = 419."""
    if tuned_blocks:
        monkeypatch.setenv("TLDA_TUNE_BF16_BLOCKS", str(tuned_blocks))
    spec, big, small = tweet
    W, m = _whitening(spec.V, D, D * 3 + K)
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, 0.5, bf16=bf16)
    tl.tlda_set_whitening(ctx, W, m)
    Phi0 = (init_phi(D, K, 7) * 0.6).astype(np.float32)
    P_ref = torch.from_numpy(Phi0).cuda()
    P_na = torch.from_numpy(Phi0).cuda()
    for rp, ci, va in (big, small):
        b = tl.CsrBatch.from_numpy(rp, ci, va)
        g_ref, g_na = torch.empty_like(P_ref), torch.full_like(P_na, float("nan"))
        n_ref = torch.empty(1, dtype=torch.int32, device="cuda")
        n_na = torch.full((1,), -1, dtype=torch.int32, device="cuda")
        X_ref = torch.empty((b.n_rows, D), device="cuda")
        X_na = torch.full((b.n_rows, D), float("nan"), device="cuda")
        tl.tlda_whiten_cp_step(ctx, b, 1e-4, P_ref, g_ref, X_ref, n_ref)
        tl.tlda_whiten_cp_step_noalloc(ctx, b, 1e-4, P_na, g_na, X_na, n_na)
        torch.cuda.synchronize()
        assert int(n_na.item()) == int(n_ref.item())
        assert torch.equal(X_na, X_ref)
        assert rel(g_na.cpu().numpy(), g_ref.cpu().numpy()) < REL32, b.n_rows
        assert rel(P_na.cpu().numpy(), P_ref.cpu().numpy()) < REL32, b.n_rows


def test_noalloc_step_refuses_what_it_does_not_cover(tweet):
    spec, big, _ = tweet
    b = tl.CsrBatch.from_numpy(*big)
    W, m = _whitening(spec.V, 150, 1)
    ctx = tl.tlda_create(spec.V, 40, 150, spec.alpha0)             # FP32 above the fused shapes
    tl.tlda_set_whitening(ctx, W, m)
    P = torch.from_numpy(init_phi(150, 40, 1).astype(np.float32)).cuda()
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_whiten_cp_step_noalloc(ctx, b, 1e-4, P)
    assert e.value.status == 2
    W, m = _whitening(spec.V, 20, 2)
    classic = tl.tlda_create(spec.V, 20, 20, spec.alpha0, classic=True)
    tl.tlda_set_whitening(classic, W, m)
    P = torch.from_numpy(init_phi(20, 20, 1).astype(np.float32)).cuda()
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_whiten_cp_step_noalloc(classic, b, 1e-4, P)
    assert e.value.status == 1
    fresh = tl.tlda_create(spec.V, 20, 20, spec.alpha0)           # no whitening yet
    with pytest.raises(tl.TldaError) as e:
        tl.tlda_whiten_cp_step_noalloc(fresh, b, 1e-4, P)
    assert e.value.status == 4
