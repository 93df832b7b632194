"""Bias term of the modified killing rate, by grid quadrature on the 2-D torus.

TEST INFRASTRUCTURE / ANALYSIS ONLY: plain FP64 numpy, never called by the
library or the benchmark's timed path.

With the modified killing rate the bias of Diffusion Restore is controlled by
L*p / p (Sec. 5.1, Eq. bias; Sec. 5.2, Eq. adjoint-bias; the bias figure of
the appendix), where L = h (P - I) is the local dynamics embedded in
continuous time with holding rate h = 1/dt (Eq. diffusion-restore-holding-rate)
and P is the Euler-Maruyama kernel (Eq. local-dynamics)

    P(x, .) = N(x + dt b(x), dt sigma2 I).

The drift is the one the chain step uses (Alg. 5.1 with the rotational term of
the local dynamics): b = (sigma2 / 2) grad log p + (gamma / 2) J grad log p,
J (s1, s2) = (s2, -s1).  Then

    L*p / p (y) = (P*p (y) / p (y) - 1) / dt,
    P*p (y)     = sum over grid points x of p(x) N(y; x + dt b(x), dt sigma2 I) h^2,

summed over the images of x on the torus.  Sampling a Gaussian of standard
deviation sd on a grid of spacing h <= sd / 3 makes the sum exact to far below
FP64 rounding (Poisson summation), so the only approximation is the finite
window of +-W cells, W covering 7 sd plus the drift shift.

Pins (tests/test_oracle_pins.py): for a Gaussian target N(c, s^2 I) the kernel
maps p to N(c, (s^2 (a^2 + beta^2) + dt sigma2) I) with a = 1 - dt sigma2 /
(2 s^2), beta = dt gamma / (2 s^2) (the rotation keeps the covariance
isotropic), which gives L*p/p in closed form; for a smooth multi-mode
target the term halves with dt (the O(dt) claim); and the drift, rotation
included, is the oracle chain's own move (mean displacement of one step).

`python -m oracle.bias` prints the term for the 2-D four-mode wrapped Gaussian
mixture (seed 11) at several dt with the paper's stddev at dt = 1e-5.
"""
from __future__ import annotations

import math

import numpy as np


def wrapped_mixture(weights, means, stds, c0: float = 0.0, images: int = 1):
    """Density p = c0 + sum_k w_k WN(mu_k, s_k^2 I) on T^2 (images within
    +-`images` periods) and its gradient, as a function of grid arrays."""
    weights, means, stds = np.asarray(weights, float), np.asarray(means, float), np.asarray(stds, float)

    def fn(X, Y):
        p = np.full(X.shape, c0, dtype=np.float64)
        gx = np.zeros(X.shape)
        gy = np.zeros(X.shape)
        for w, m, s in zip(weights, means, stds):
            norm = w / (2.0 * math.pi * s * s)
            for i in range(-images, images + 1):
                for j in range(-images, images + 1):
                    dx = X - m[0] - i
                    dy = Y - m[1] - j
                    g = norm * np.exp(-(dx * dx + dy * dy) / (2.0 * s * s))
                    p += g
                    gx += -dx / (s * s) * g
                    gy += -dy / (s * s) * g
        return p, gx, gy

    return fn


def em_bias_term(density, n: int, dt: float, sigma2: float, gamma: float = 0.0):
    """L*p / p on the n x n cell-centred grid of the unit torus.  Returns
    (X, Y, p, term)."""
    h = 1.0 / n
    sd = math.sqrt(dt * sigma2)
    if h > sd / 3.0:
        raise ValueError(f"grid too coarse: h = {h:.3g} > sd/3 = {sd / 3:.3g}")
    c = (np.arange(n) + 0.5) * h
    X, Y = np.meshgrid(c, c, indexing="ij")
    p, gx, gy = density(X, Y)
    sx, sy = gx / p, gy / p  # grad log p
    bx = 0.5 * sigma2 * sx + 0.5 * gamma * sy
    by = 0.5 * sigma2 * sy - 0.5 * gamma * sx
    shift = dt * max(np.abs(bx).max(), np.abs(by).max())
    W = int(math.ceil((7.0 * sd + shift) / h))
    var = dt * sigma2
    norm = h * h / (2.0 * math.pi * var)
    pstar = np.zeros_like(p)
    # y = x + o h: gather from x = y - o h (rolled arrays), y - mean(x) = o h - dt b(x)
    for oi in range(-W, W + 1):
        px_i = np.roll(p, oi, axis=0)
        bx_i = np.roll(bx, oi, axis=0)
        by_i = np.roll(by, oi, axis=0)
        ex = oi * h - dt * bx_i
        for oj in range(-W, W + 1):
            ey = oj * h - dt * np.roll(by_i, oj, axis=1)
            exj = np.roll(ex, oj, axis=1)
            pstar += np.roll(px_i, oj, axis=1) * np.exp(-(exj * exj + ey * ey) / (2.0 * var))
    pstar *= norm
    return X, Y, p, (pstar / p - 1.0) / dt


def gaussian_term_closed_form(X, Y, c, s: float, dt: float, sigma2: float, gamma: float = 0.0):
    """L*p / p for p = N(c, s^2 I) (on the plane) under the kernel above."""
    a = 1.0 - dt * sigma2 / (2.0 * s * s)
    beta = dt * gamma / (2.0 * s * s)
    v = s * s * (a * a + beta * beta) + dt * sigma2
    r2 = (X - c[0]) ** 2 + (Y - c[1]) ** 2
    ratio = (s * s / v) * np.exp(-r2 / (2.0 * v) + r2 / (2.0 * s * s))
    return (ratio - 1.0) / dt


def main():
    import sys
    import os

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_2605_08916_amd import inputs

    mix = inputs.mixture_target(d=2, seed=11)
    dens = wrapped_mixture(mix["weights"], mix["means"], mix["stds"], c0=0.1)
    sigma2 = (5e-3) ** 2 / 1e-5  # the chain step's stddev 5e-3 at dt = 1e-5
    print("four-mode wrapped Gaussian mixture on T^2 (seed 11, c0 = 0.1), sigma^2 = 2.5, gamma = 0.5")
    print("dt        grid   max|L*p/p|    p-weighted mean |L*p/p|   max|L*p/p| * dt")
    for dt in (1e-3, 1e-4, 1e-5):
        sd = math.sqrt(dt * sigma2)
        # the integrand's finest scale is the kernel or the narrowest mode (0.03)
        n = int(math.ceil(3.0 / min(sd, 0.03)))
        _, _, p, t = em_bias_term(dens, n, dt, sigma2, gamma=0.5)
        wmean = float((np.abs(t) * p).sum() / p.sum())
        print(f"{dt:8.0e}  {n:5d}  {np.abs(t).max():12.4e}  {wmean:24.4e}  {np.abs(t).max() * dt:14.4e}", flush=True)


if __name__ == "__main__":
    main()
