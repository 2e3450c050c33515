"""Coefficients of the float32 arctangent used by the mixed sweeps.

atan(z) on [0, 1] is written z * p(z^2) with p a polynomial of degree 7; the
coefficients minimise the maximum relative error (iterated reweighted least
squares on a Chebyshev grid, a Lawson-style approximation of the minimax fit).
Prints the coefficients and the float64 error bound of the fit; the kernels
carry the printed values.  Run: python paper_2602_05492_amd/csrc/fit_atan.py
"""
import numpy as np


def fit(deg=7, iters=60):
    k = np.arange(4000)
    z = 0.5 + 0.5 * np.cos(np.pi * (k + 0.5) / len(k))          # Chebyshev points on [0, 1]
    z = np.concatenate([z, [1.0, 1e-6]])
    s = z * z
    V = np.stack([z * s ** j for j in range(deg + 1)], axis=1)
    t = np.arctan(z)
    w = np.ones_like(z)
    for _ in range(iters):
        A = V / t[:, None]
        c, *_ = np.linalg.lstsq(A * np.sqrt(w)[:, None], np.sqrt(w), rcond=None)
        err = np.abs(V @ c / t - 1.0)
        w = w * (err + 1e-20)
        w /= w.sum()
    return c


if __name__ == "__main__":
    c = fit()
    zz = np.linspace(0.0, 1.0, 2_000_001)[1:]
    approx = zz * np.polyval(c[::-1], zz * zz)
    rel = np.abs(approx / np.arctan(zz) - 1.0).max()
    print("coefficients (z * sum c_j z^(2j)):")
    for j, v in enumerate(c):
        print(f"  c{j} = {v:.9e}f")
    print(f"max relative error on (0, 1]: {rel:.3e}")
