"""Seeded synthetic inputs shared by the tests, the benchmark and the
reference checks.

This module holds none of the solver's arithmetic: only closed-form cell and
face averages of smooth manufactured fields (products of one-dimensional
averages), seeded noise, and box layouts.  Arrays are returned as dense
per-level arrays with axis d = spatial direction d (x first).  Noise is drawn
with numpy's PCG64 ``default_rng(seed)``; the mean and standard deviation are
those of the workload descriptions (N(0, 1e-3^2) per cell).
"""
import math

import numpy as np


# ----------------------------------------------------------------------------
# one-dimensional averages
def avg_sin(a, b, x0, h, n):
    """Averages of sin(a x + b) over the cells [x0 + i h, x0 + (i+1) h]."""
    xl = x0 + h * np.arange(n)
    return (np.cos(a * xl + b) - np.cos(a * (xl + h) + b)) / (a * h)


def avg_cos(a, b, x0, h, n):
    """Averages of cos(a x + b) over the cells [x0 + i h, x0 + (i+1) h]."""
    xl = x0 + h * np.arange(n)
    return (np.sin(a * (xl + h) + b) - np.sin(a * xl + b)) / (a * h)


def avg_poly(coef, x0, h, n):
    """Averages of the polynomial sum_k coef[k] x^k over the cells."""
    xl = x0 + h * np.arange(n)
    xr = xl + h
    out = np.zeros(n)
    for k, a in enumerate(coef):
        out += a * (xr ** (k + 1) - xl ** (k + 1)) / ((k + 1) * h)
    return out


def outer(*vecs):
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


def noise(shape, seed, std=1e-3):
    return np.random.default_rng(seed).normal(0.0, std, size=shape)


# ----------------------------------------------------------------------------
# workloads
def sinprod_avg(n, h, k=2.0):
    """Cell averages of prod_d sin(k pi x_d) on [0, n h]^D."""
    return outer(*[avg_sin(k * math.pi, 0.0, 0.0, h, m) for m in n])


def cosprod_avg(n, h, k=2.0):
    return outer(*[avg_cos(k * math.pi, 0.0, 0.0, h, m) for m in n])


def single_level_rhs(n, h, op, c, seed=0, noise_std=1e-3):
    """Right-hand side of the single-level workloads: the manufactured field
    u = prod sin(2 pi x_d) through the continuous operator, plus seeded
    noise.  Helmholtz: (1 + D 4 pi^2 c) <u> + eps.  Poisson: -D 4 pi^2 <u>
    + eps, minus its mean."""
    D = len(n)
    u = sinprod_avg(n, h)
    eps = noise(tuple(n), seed, noise_std) if noise_std else 0.0
    if op == "helmholtz":
        return (1.0 + D * 4 * math.pi ** 2 * c) * u + eps
    f = -D * 4 * math.pi ** 2 * u + eps
    return f - f.mean()


def batched_boxes(nboxes=1024, seed=0, mmin=2, mmax=32):
    """Side lengths 8 m, m ~ U{mmin..mmax}, one per independent box."""
    rng = np.random.default_rng(seed)
    m = rng.integers(mmin, mmax + 1, size=nboxes)
    return [int(8 * v) for v in m]


def batched_rhs(side, h, seed, nmodes=8):
    """Sum of nmodes Fourier modes sum_j a_j <sin(p_j pi x / L) sin(q_j pi y / L)>
    on the box [0, L]^2, L = side h; p, q ~ U{1..8}, a ~ N(0, 1)."""
    rng = np.random.default_rng(seed)
    L = side * h
    f = np.zeros((side, side))
    for _ in range(nmodes):
        p, q = rng.integers(1, 9, size=2)
        a = rng.normal()
        f += a * outer(avg_sin(p * math.pi / L, 0.0, 0.0, h, side), avg_sin(q * math.pi / L, 0.0, 0.0, h, side))
    return f


def disk_boxes(centres_radii, nfine, bs):
    """Fine boxes of bs^2 cells tiling the fine grid nfine^2 on [0,1]^2 whose
    centre lies strictly inside one of the disks (centre, radius)."""
    hf = 1.0 / nfine
    boxes = []
    for bj in range(nfine // bs):
        for bi in range(nfine // bs):
            cx = (bi * bs + bs / 2) * hf
            cy = (bj * bs + bs / 2) * hf
            if any((cx - x) ** 2 + (cy - y) ** 2 < r * r for (x, y), r in centres_radii):
                boxes.append(((bi * bs, bj * bs), (bi * bs + bs - 1, bj * bs + bs - 1)))
    return boxes


def amr_two_level_boxes():
    """Two-level layout: level 0 one 256^2 box on [0,1]^2; level 1 the 32^2
    boxes of the 512^2 grid whose centres lie inside the disk of radius 0.25
    at (0.5, 0.5) or the disk of radius 0.08 at (0.8, 0.2) (56 boxes, two
    face-connected components)."""
    return [[((0, 0), (255, 255))], disk_boxes([((0.5, 0.5), 0.25), ((0.8, 0.2), 0.08)], 512, 32)]
