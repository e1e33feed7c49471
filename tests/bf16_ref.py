"""Helpers for the BF16 parity tests: the format's rounding, the oracle's
gradient on BF16-rounded operands, and the magnitude sums of the derived
rounding bound (see tests/test_gpu_bf16.py for the derivation).

With u = 2^-8 the BF16 unit roundoff, B = |X|^T S^2 and
C = |X|^T (|S| (|X| |Phi|)) (X, Phi rounded, S = X Phi), both scaled by the
gradient's 3 c3 / n:
  * the step from FP32 X (tlda_cp_step) stays within 2u B + D 2^-23 C;
  * a fused step (whitening kept on chip, X rounded from the kernel's own
    FP32 row, which may differ from the oracle's in the last bit and so round
    to the neighbouring BF16 value) stays within 4u (B + C);
plus 2^-22 |ref| for the FP32 penalty term and the final rounding.
"""
import numpy as np

from oracle import tlda_oracle as O

U_BF16 = 2.0 ** -8


def bf16_round(a):
    """Nearest BF16 value of fp32(a), ties to even (the format's definition:
    keep the upper 16 bits of the FP32 pattern after adding half an ulp)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rounded_gradient(X, Phi, n, alpha0, theta):
    """Oracle gradient with the data term on BF16-rounded X and Phi and the
    penalty term on the FP32 Phi; plus the scaled magnitude sums B and C."""
    Xh, Ph = bf16_round(X), bf16_round(Phi)
    Phi64 = np.asarray(Phi, dtype=np.float64)
    zero = np.zeros((1, Phi.shape[0]))
    pen = O.cp_gradient(zero, Phi64, n, alpha0, theta)
    data = O.cp_gradient(Xh, Ph, n, alpha0, theta) - O.cp_gradient(zero, Ph, n, alpha0, theta)
    S = Xh @ Ph
    B = np.abs(Xh).T @ (S * S)
    C = np.abs(Xh).T @ (np.abs(S) * (np.abs(Xh) @ np.abs(Ph)))
    scale = 3.0 * (alpha0 + 1.0) * (alpha0 + 2.0) / 2.0 / max(n, 1)
    return pen + data, scale * B, scale * C


def fused_bound(ref, B, C):
    """Element-wise bound of a fused BF16 step's gradient against `ref`."""
    return 4 * U_BF16 * (B + C) + 2.0 ** -22 * np.abs(ref)


def assert_within(got, ref, bound, what):
    excess = np.abs(np.asarray(got, dtype=np.float64) - ref) - bound
    worst = float(excess.max())
    assert worst <= 0.0, f"{what}: exceeds the rounding bound by {worst:g}"
