"""Pins of the encoder oracle (oracle/mlp_oracle.py) to facts other than
itself: textbook values of the normal distribution function, the symmetry of
gelu, finite differences of the loss, the first Adam step in closed form, and
a hand-worked duality gap."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M
from oracle import tlda_oracle as O


def test_gelu_textbook_values_and_symmetry():
    # Phi(1) and Phi(2) from a standard normal table
    assert M.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, abs=1e-15)
    assert M.gelu(np.array([-1.0]))[0] == pytest.approx(-0.15865525393145707, abs=1e-15)
    assert M.gelu(np.array([2.0]))[0] == pytest.approx(2.0 * 0.9772498680518208, abs=1e-15)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    z = np.linspace(-6, 6, 101)
    # Phi(z) + Phi(-z) = 1  =>  gelu(z) - gelu(-z) = z
    np.testing.assert_allclose(M.gelu(z) - M.gelu(-z), z, atol=1e-14)
    assert abs(M.gelu(np.array([8.0]))[0] - 8.0) < 1e-12
    assert abs(M.gelu(np.array([-8.0]))[0]) < 1e-12


def test_gelu_grad_is_the_derivative():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(M.gelu_grad(z), fd, atol=1e-8)
    assert M.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)


def test_softmax_rows_and_shift_invariance():
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((7, 5)) * 3
    P = M.softmax(Z)
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-15)
    np.testing.assert_allclose(M.softmax(Z + 100.0), P, atol=1e-15)
    e = np.exp(Z)
    np.testing.assert_allclose(P, e / e.sum(axis=1, keepdims=True), rtol=1e-13)


def _tiny(seed, d_in=3, hidden=4, k_out=3, B=5):
    rng = np.random.default_rng(seed)
    params = {k: rng.standard_normal(s) * 0.7 for k, s in M.shapes(d_in, hidden, k_out).items()}
    X = rng.standard_normal((B, d_in))
    T = rng.dirichlet(np.ones(k_out), size=B)
    return params, X, T


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradients_match_central_differences(seed):
    params, X, T = _tiny(seed)
    g, L = M.gradients(params, X, T)
    assert L == pytest.approx(M.loss(M.forward(params, X)["P"], T), rel=1e-15)
    h = 1e-6
    for k in M.PARAM_ORDER:
        fd = np.zeros_like(params[k])
        for idx in np.ndindex(params[k].shape):
            p_plus = {kk: v.copy() for kk, v in params.items()}
            p_minus = {kk: v.copy() for kk, v in params.items()}
            p_plus[k][idx] += h
            p_minus[k][idx] -= h
            fd[idx] = (M.loss(M.forward(p_plus, X)["P"], T) -
                       M.loss(M.forward(p_minus, X)["P"], T)) / (2 * h)
        np.testing.assert_allclose(g[k], fd, rtol=1e-6, atol=1e-9, err_msg=k)


def test_pack_unpack_roundtrip_and_order():
    params, _, _ = _tiny(4)
    flat = M.pack(params)
    assert flat.shape == (3 * 4 + 4 + 4 * 4 + 4 + 4 * 3 + 3,)
    assert np.array_equal(flat[:12], params["W1"].ravel())
    back = M.unpack(flat, 3, 4, 3)
    for k in M.PARAM_ORDER:
        assert np.array_equal(back[k], params[k])


def test_first_adam_step_in_closed_form():
    params, X, T = _tiny(5)
    g, _ = M.gradients(params, X, T)
    lr = 1e-2
    new = M.adam_step(params, g, {}, lr)
    for k in M.PARAM_ORDER:
        # bias correction makes m_hat = g and v_hat = g^2 at t = 1
        np.testing.assert_allclose(new[k], params[k] - lr * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12)


def test_duality_gap_hand_worked_and_bounds_the_suboptimality():
    A = np.eye(3)
    x = np.array([[0.2, 0.3, 0.5]])
    t = np.array([[1.0, 0.0, 0.0]])
    # g = t - x = (0.8, -0.3, -0.5): gap = 0.8 - (-0.5) = 1.3; h = 0.49
    assert M.simplex_ls_gap(x, A, t)[0] == pytest.approx(1.3, abs=1e-15)
    assert M.simplex_ls_value(x, A, t)[0] == pytest.approx(0.49, abs=1e-15)
    assert M.simplex_ls_gap(x, A, x)[0] == pytest.approx(0.0, abs=1e-15)
    rng = np.random.default_rng(6)
    A = rng.standard_normal((6, 4))
    X = rng.standard_normal((20, 6))
    star = O.infer_doc_topics(X, A, 5000, 1e-15)
    assert np.all(np.abs(M.simplex_ls_gap(X, A, star)) < 1e-8)
    h_star = M.simplex_ls_value(X, A, star)
    for _ in range(5):
        Th = rng.dirichlet(np.ones(4), size=20)
        gap = M.simplex_ls_gap(X, A, Th)
        assert np.all(gap >= M.simplex_ls_value(X, A, Th) - h_star - 1e-12)
