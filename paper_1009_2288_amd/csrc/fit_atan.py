"""Coefficients of the float32 arctangent guess in ``proj.hip`` (``guess_atan``).

An odd polynomial of degree 15, c0 u + c1 u^3 + ... + c7 u^15, approximating
atan(u) on [0, 1] in the minimax sense, found by Lawson's algorithm
(iteratively reweighted least squares: each pass multiplies a point's weight
by its current absolute error, which drives the weighted least-squares fit
toward the equioscillating minimax polynomial).  Run it to print the
coefficients in the order the kernel's Horner scheme uses (highest first) and
the maximum error in exact arithmetic (about 3.8e-8 rad).
"""
import numpy as np


def fit(degree_terms: int = 8, passes: int = 400):
    x = np.unique(np.concatenate([np.cos(np.linspace(0.0, np.pi / 2, 20001)), np.linspace(0.0, 1.0, 20001)]))
    a = np.stack([x ** (2 * k + 1) for k in range(degree_terms)], 1)
    y = np.arctan(x)
    w = np.full(x.shape, 1.0 / x.size)
    for _ in range(passes):
        sw = np.sqrt(w)
        c = np.linalg.lstsq(a * sw[:, None], y * sw, rcond=None)[0]
        err = np.abs(a @ c - y)
        w = w * err
        w /= w.sum()
    return c, float(err.max())


if __name__ == "__main__":
    c, e = fit()
    for v in c[::-1]:
        print(f"{v:.9e}f")
    print(f"max |error| on [0, 1]: {e:.3e} rad")
