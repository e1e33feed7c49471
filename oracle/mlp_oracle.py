"""Plain FP64 CPU oracle of the learned document-topic encoder.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  It shares no code,
constants or helpers with the HIP library.

The encoder is this library's stand-in for the per-document simplex-constrained
solve of the inference step (the package section's document-topic output,
solved as in reading R8 of tlda_oracle): a multilayer perceptron maps a
whitened document x (D values) to topic proportions on the simplex,

    Z1 = X W1 + b1,  H1 = gelu(Z1),
    Z2 = H1 W2 + b2, H2 = gelu(Z2),
    Z3 = H2 W3 + b3, P = softmax(Z3)   (row-wise),

with gelu(z) = z Phi(z), Phi the standard normal distribution function
(written with erf), trained on pairs (x, t) where t is the simplex solve's
output, by the mean cross-entropy of the rows, -(1/B) sum_d sum_k t_dk log P_dk.
Parameters are stored input-major (W1 is D x H), so a layer is X W + b.

The judge of an encoder output is the duality gap of the solve it replaces:
for h(t) = |x - A t|^2 / 2 over the simplex, g = A^T (A t - x), and
gap(t) = g.t - min_k g_k >= h(t) - min h  (convexity: for the minimiser t*,
h(t) - h(t*) <= g.(t - t*) <= g.t - min_k g_k).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def shapes(d_in: int, hidden: int, k_out: int) -> dict:
    return {"W1": (d_in, hidden), "b1": (hidden,), "W2": (hidden, hidden), "b2": (hidden,),
            "W3": (hidden, k_out), "b3": (k_out,)}


def pack(params: dict) -> np.ndarray:
    """Flat vector in the order W1, b1, W2, b2, W3, b3 (row-major matrices)."""
    return np.concatenate([np.asarray(params[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unpack(flat: np.ndarray, d_in: int, hidden: int, k_out: int) -> dict:
    out, o = {}, 0
    for k, shp in shapes(d_in, hidden, k_out).items():
        n = int(np.prod(shp))
        out[k] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def gelu(z: np.ndarray) -> np.ndarray:
    """z Phi(z) with Phi(z) = (1 + erf(z / sqrt 2)) / 2."""
    return z * 0.5 * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z: np.ndarray) -> np.ndarray:
    """d/dz [z Phi(z)] = Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def softmax(z: np.ndarray) -> np.ndarray:
    """Row-wise exp(z - max) / sum exp(z - max)."""
    e = np.exp(z - z.max(axis=1, keepdims=True))
    return e / e.sum(axis=1, keepdims=True)


def forward(params: dict, X: np.ndarray) -> dict:
    """All intermediate values of the forward pass (FP64)."""
    Z1 = X @ params["W1"] + params["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ params["W2"] + params["b2"]
    H2 = gelu(Z2)
    Z3 = H2 @ params["W3"] + params["b3"]
    return {"X": X, "Z1": Z1, "H1": H1, "Z2": Z2, "H2": H2, "Z3": Z3, "P": softmax(Z3)}


def loss(P: np.ndarray, T: np.ndarray) -> float:
    """Mean over rows of the cross-entropy -sum_k t_k log p_k."""
    return float(-(T * np.log(P)).sum() / P.shape[0])


def gradients(params: dict, X: np.ndarray, T: np.ndarray) -> tuple[dict, float]:
    """Back-propagation of the mean cross-entropy, layer by layer (chain rule):
    dZ3 = (P - T) / B; dW3 = H2^T dZ3, db3 = column sums; dZ2 = (dZ3 W3^T) *
    gelu'(Z2); and so on down to W1."""
    f = forward(params, X)
    B = X.shape[0]
    dZ3 = (f["P"] - T) / B
    g = {"W3": f["H2"].T @ dZ3, "b3": dZ3.sum(axis=0)}
    dZ2 = (dZ3 @ params["W3"].T) * gelu_grad(f["Z2"])
    g["W2"] = f["H1"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ params["W2"].T) * gelu_grad(f["Z1"])
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g, loss(f["P"], T)


def adam_step(params: dict, grads: dict, state: dict, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8) -> dict:
    """One Adam step (Kingma & Ba, 2015, Algorithm 1): m and v moving
    averages of the gradient and its square, bias-corrected by 1 - beta^t."""
    t = state.get("t", 0) + 1
    out = {}
    for k in PARAM_ORDER:
        m = beta1 * state.get("m_" + k, 0.0) + (1.0 - beta1) * grads[k]
        v = beta2 * state.get("v_" + k, 0.0) + (1.0 - beta2) * grads[k] ** 2
        state["m_" + k], state["v_" + k] = m, v
        mhat = m / (1.0 - beta1 ** t)
        vhat = v / (1.0 - beta2 ** t)
        out[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    state["t"] = t
    return out


def simplex_ls_gap(X: np.ndarray, A: np.ndarray, Theta: np.ndarray) -> np.ndarray:
    """Duality gap of h(t) = |x - A t|^2 / 2 over the simplex at each row t of
    Theta (rows of X are the documents): g = A^T (A t - x), gap = g.t - min g."""
    G = (Theta @ A.T - X) @ A
    return (G * Theta).sum(axis=1) - G.min(axis=1)


def simplex_ls_value(X: np.ndarray, A: np.ndarray, Theta: np.ndarray) -> np.ndarray:
    """h(t) = |x - A t|^2 / 2 for each row."""
    R = Theta @ A.T - X
    return 0.5 * (R * R).sum(axis=1)
