"""Coefficients of the single-precision atan polynomial in hg_device.h.

atan(t) ~ t P(t^2) on t in [0, 1], P of degree 7: a near-minimax fit of the
absolute error by Lawson's algorithm (iteratively reweighted least squares,
weights multiplied by the current absolute error) on 4000 Chebyshev nodes
of [0, 1], in double precision, then rounded to single precision.  Prints the
coefficients from the highest power down (the order hg_device.h evaluates
them by Horner's rule) and the largest error of that evaluation in exactly
emulated single-precision arithmetic (each fma rounded once).

Usage: python paper_2409_10327_amd/csrc/fit_atan_poly.py
"""
from __future__ import annotations

import numpy as np

DEGREE = 7
NODES = 4000
ITERS = 400


def fit() -> np.ndarray:
    k = np.arange(NODES)
    t = 0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / NODES)
    s = t * t
    A = t[:, None] * s[:, None] ** np.arange(DEGREE + 1)[None, :]
    y = np.arctan(t)
    w = np.full(NODES, 1.0 / NODES)
    c = None
    for _ in range(ITERS):
        sw = np.sqrt(w)
        c = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)[0]
        e = np.abs(A @ c - y)
        w = w * e
        w /= w.sum()
    return c[::-1].astype(np.float32)  # highest power first


def eval_f32(coef_hi_first: np.ndarray, t: np.ndarray) -> np.ndarray:
    """t P(t^2) by Horner's rule in single precision, one rounding per fma."""
    t = t.astype(np.float32)
    s = (t * t).astype(np.float32)
    p = np.full_like(t, coef_hi_first[0])
    for c in coef_hi_first[1:]:
        p = (p.astype(np.float64) * s.astype(np.float64) + np.float64(c)).astype(np.float32)
    return (p * t).astype(np.float32)


def max_error(coef_hi_first: np.ndarray, n: int = 1 << 22) -> float:
    t = np.linspace(0.0, 1.0, n, dtype=np.float32)
    return float(np.max(np.abs(eval_f32(coef_hi_first, t).astype(np.float64) - np.arctan(t.astype(np.float64)))))


if __name__ == "__main__":
    c = fit()
    print("coefficients (t^15 .. t^1):", ", ".join(f"{float(v):.9g}f" for v in c))
    print(f"max |error| in FP32 evaluation over [0, 1]: {max_error(c):.3g} rad")
