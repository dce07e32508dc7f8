"""Coefficients of the FP32 arctangent used by the near-field kernel.

atan(t) ~= t * P(t^2) on [0, 1] with deg P = 6.  The fit minimises the
maximum relative error by Lawson's iteration (iteratively re-weighted least
squares, which converges to the minimax approximation) on 20,001 points;
the resulting coefficients are rounded to float32.  Max relative error of
the fit: 7.4e-7; absolute error of the float32 Horner evaluation: 6.5e-7.

    python paper_2311_14312_amd/csrc/fit_atan_poly.py
"""
import numpy as np


def fit(deg=6, iters=200):
    t = np.linspace(1e-6, 1.0, 20001)
    u = t * t
    f = np.arctan(t) / t
    V = np.vander(u, deg + 1, increasing=True)
    w = np.ones_like(u)
    for _ in range(iters):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(V * sw[:, None], f * sw, rcond=None)
        err = V @ c - f
        w = w * np.abs(err)
        w /= w.sum()
    return c.astype(np.float32)


if __name__ == "__main__":
    print(", ".join(f"{v:.8e}f" for v in fit()))
