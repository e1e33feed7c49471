"""The fully online mode on the GPU against the FP64 oracle, through the C ABI:
warm-started whitening refreshes, the Phi rebase, and the online fit (a
batched start, then per new batch: moments, warm refresh, rebase, one step).

Bars: whitening 1e-7 relative (as for cold refreshes, FP64); the rebased Phi
(FP32 output of an FP64 transform) 1e-6; the online Phi after every batch
1e-4 (FP32 steps against FP64, as for the batched fit); for BF16 contexts the
recovered topics within 0.02 mean L1 of the oracle's.
"""
import numpy as np
import pytest
import torch

from oracle import tlda_oracle as O
from synth import SPECS, generate, init_phi, iter_batches

pytestmark = pytest.mark.gpu

tl = pytest.importorskip("paper_2511_07809_amd.tlda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def c1():
    spec = SPECS["c1"]
    c = generate(spec)
    return spec, c, [(rp, ci, va) for rp, ci, va, _ in iter_batches(c)]


def _eigen_whitening(batches, spec, D):
    m, N = O.first_moment(batches, spec.V)
    W, lam, U = O.whitening(O.centered_second_moment(batches, m, N, spec.alpha0), D)
    return W, m


def test_rebase_matches_oracle(c1):
    spec, _, bs = c1
    D = K = spec.K
    W_old, m_old = _eigen_whitening(bs[:2], spec, D)
    W_new, m_new = _eigen_whitening(bs, spec, D)
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0)
    tl.tlda_set_whitening(ctx, W_old, m_old)
    with pytest.raises(tl.TldaError) as e:     # nothing replaced yet
        tl.tlda_rebase_phi(ctx, torch.zeros((D, K), dtype=torch.float32, device="cuda"))
    assert e.value.status == 4
    tl.tlda_set_whitening(ctx, W_new, m_new)
    Phi = init_phi(D, K, 7).astype(np.float32)
    Pd = torch.from_numpy(Phi).cuda()
    tl.tlda_rebase_phi(ctx, Pd)
    torch.cuda.synchronize()
    ref = O.rebase_phi(Phi.astype(np.float64), W_old, W_new)
    assert rel(Pd.cpu().numpy(), ref) < 1e-6
    # rebasing again maps from W_new to W_new: the identity
    tl.tlda_set_whitening(ctx, W_new, m_new)
    P2 = Pd.clone()
    tl.tlda_rebase_phi(ctx, P2)
    torch.cuda.synchronize()
    assert rel(P2.cpu().numpy(), Pd.cpu().numpy()) < 1e-6


def test_warm_refresh_converges_to_the_cold_refresh(c1):
    spec, _, bs = c1
    D = K = spec.K
    warm = tl.tlda_create(spec.V, K, D, spec.alpha0, eig_iters=100, eig_warm_iters=30)
    cold = tl.tlda_create(spec.V, K, D, spec.alpha0, eig_iters=100)
    for b in bs[:3]:
        tl.tlda_update_moments(warm, tl.CsrBatch.from_numpy(*b))
    tl.tlda_update_moments(warm, None, tl.TLDA_REFRESH_WARM)   # no previous block: cold
    for b in bs[3:]:
        tl.tlda_update_moments(warm, tl.CsrBatch.from_numpy(*b), tl.TLDA_REFRESH_WARM)
    for b in bs:
        tl.tlda_update_moments(cold, tl.CsrBatch.from_numpy(*b))
    tl.tlda_update_moments(cold, None, tl.TLDA_REFRESH_W)
    Ww, ew, mw = tl.tlda_get_whitening(warm)
    Wc, ec, mc = tl.tlda_get_whitening(cold)
    W_ref, m_ref = _eigen_whitening(bs, spec, D)
    assert rel(ew, ec) < 1e-10
    assert rel(Ww, Wc) < 1e-7 and rel(Ww, W_ref) < 1e-7
    np.testing.assert_allclose(mw, m_ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("bf16", [False, True])
def test_online_fit_matches_oracle(c1, bf16):
    """Two initial batches fitted batched for 3 passes, then the three other
    batches online.  FP32 context: Phi after every batch within 1e-4.  The
    BF16 context's steps round X, Phi and S^2 to BF16, so it takes the BF16
    path's topic bar: recovered topics within 0.02 mean L1 of the oracle's."""
    spec, _, bs = c1
    D = K = spec.K
    beta, passes = 0.03, 3
    Phi0 = init_phi(D, K, 1)
    ref = O.fit_online(bs[:2], bs[2:], spec.V, K, D, spec.alpha0, 0.0, beta, passes, Phi0)
    ctx = tl.tlda_create(spec.V, K, D, spec.alpha0, bf16=bf16, eig_iters=100, eig_warm_iters=40)
    dev = [tl.CsrBatch.from_numpy(*b) for b in bs]
    for b in dev[:2]:
        tl.tlda_update_moments(ctx, b)
    tl.tlda_update_moments(ctx, None, tl.TLDA_REFRESH_W)
    Pd = torch.from_numpy(Phi0.astype(np.float32)).cuda()
    for _ in range(passes):
        for b in dev[:2]:
            tl.tlda_whiten_cp_step(ctx, b, beta, Pd)
    torch.cuda.synchronize()
    if not bf16:
        assert rel(Pd.cpu().numpy(), ref["Phi_init"]) < 1e-4
    for i, b in enumerate(dev[2:]):
        tl.tlda_update_moments(ctx, b, tl.TLDA_REFRESH_WARM)
        tl.tlda_rebase_phi(ctx, Pd)
        tl.tlda_whiten_cp_step(ctx, b, beta, Pd)
        torch.cuda.synchronize()
        if not bf16:
            assert rel(Pd.cpu().numpy(), ref["trace"][i]) < 1e-4, i
    W, _, _ = tl.tlda_get_whitening(ctx)
    assert rel(W, ref["W"]) < 1e-7
    mu, _, _ = tl.tlda_unwhiten(ctx, Pd, tl.TLDA_PROJECT_SIMPLEX)
    l1 = np.abs(mu.cpu().numpy() - ref["mu_simplex"]).sum(axis=0)
    assert l1.mean() <= (0.02 if bf16 else 1e-3)
