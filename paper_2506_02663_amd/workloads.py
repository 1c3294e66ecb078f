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


def amr_two_level_boxes(ratio=2):
    """Two-level layout: level 0 one 256^2 box on [0,1]^2; level 1 the 32^2
    boxes of the 512^2 grid whose centres lie inside the disk of radius 0.25
    at (0.5, 0.5) or the disk of radius 0.08 at (0.8, 0.2) (56 boxes, two
    face-connected components).  ratio 4: the same patches as 64^2 boxes of
    the 1024^2 grid."""
    n = 256 * ratio
    return [[((0, 0), (255, 255))], disk_boxes([((0.5, 0.5), 0.25), ((0.8, 0.2), 0.08)], n, 16 * ratio)]


# ----------------------------------------------------------------------------
# three-level vortex workload
def _tag_boxes(centres, radius, n, bs):
    """bs^2 boxes of the n^2 grid on [0,1]^2 whose centre lies within radius
    of one of the centres; as a set of (bi, bj) box indices."""
    hb = bs / n
    out = set()
    for bj in range(n // bs):
        for bi in range(n // bs):
            cx, cy = (bi + 0.5) * hb, (bj + 0.5) * hb
            if any((cx - x) ** 2 + (cy - y) ** 2 <= radius * radius for x, y in centres):
                out.add((bi, bj))
    return out


def vortex_centres(seed=0):
    rng = np.random.default_rng(seed)
    return [tuple(rng.uniform(0.3, 0.7, size=2)) for _ in range(2)]


def three_level_vortex_boxes(seed=0, base=512, bs=64, r1=0.15, r2=0.075, buffer=4):
    """Level 0: one base^2 box on [0,1]^2.  Level 1 (2 base)^2 and level 2
    (4 base)^2: the bs^2 boxes whose centre lies within r1 / r2 of one of two
    seeded vortex centres (uniform in [0.3, 0.7]^2), level 1 grown so that it
    covers the parent cells of every level-2 box plus `buffer` level-1 cells
    around them (room for the coarse-fine interpolation windows)."""
    centres = vortex_centres(seed)
    n1, n2 = 2 * base, 4 * base
    l2 = _tag_boxes(centres, r2, n2, bs)
    l1 = _tag_boxes(centres, r1, n1, bs)
    for bi, bj in l2:
        lo = (bi * bs // 2 - buffer, bj * bs // 2 - buffer)
        hi = ((bi + 1) * bs // 2 - 1 + buffer, (bj + 1) * bs // 2 - 1 + buffer)
        for ci in range(max(lo[0], 0) // bs, min(hi[0], n1 - 1) // bs + 1):
            for cj in range(max(lo[1], 0) // bs, min(hi[1], n1 - 1) // bs + 1):
                l1.add((ci, cj))

    def boxes(tags):
        return [((bi * bs, bj * bs), (bi * bs + bs - 1, bj * bs + bs - 1)) for bi, bj in sorted(tags)]
    return [[((0, 0), (base - 1, base - 1))], boxes(l1), boxes(l2)], centres


def lamb_oseen_avg(centres, lo, n, h, circ=(1.0, -1.0), sigma=0.05, order=3):
    """Cell averages (Gauss-Legendre, order^2 points per cell) of the velocity
    of Lamb-Oseen vortices of circulations circ at the centres, on the n[0] x
    n[1] cells starting at index lo with cell size h.  Returns (u, v) indexed
    [x, y]."""
    g, w = np.polynomial.legendre.leggauss(order)
    g, w = 0.5 * (g + 1.0), 0.5 * w
    xs = (lo[0] + np.arange(n[0]))[:, None] * h
    ys = (lo[1] + np.arange(n[1]))[None, :] * h
    u = np.zeros(n)
    v = np.zeros(n)
    for a, wa in zip(g, w):
        for b, wb in zip(g, w):
            x = xs + a * h
            y = ys + b * h
            for (cx, cy), G in zip(centres, circ):
                dx, dy = x - cx, y - cy
                r2 = dx * dx + dy * dy
                fac = G / (2 * math.pi) * (1.0 - np.exp(-r2 / sigma ** 2)) / np.maximum(r2, 1e-300)
                u += wa * wb * (-dy * fac)
                v += wa * wb * (dx * fac)
    return u, v


def smooth_field_avg(lo, n, h, seed, nmodes=4):
    """Cell averages of a seeded smooth field sum_j a_j sin(p_j pi x + s_j)
    sin(q_j pi y + t_j) on the cells starting at index lo."""
    rng = np.random.default_rng(seed)
    out = np.zeros(n)
    for _ in range(nmodes):
        p, q = rng.integers(1, 5, size=2)
        s, t = rng.uniform(0, 2 * math.pi, size=2)
        a = rng.normal()
        out += a * outer(avg_sin(p * math.pi, s, lo[0] * h, h, n[0]), avg_sin(q * math.pi, t, lo[1] * h, h, n[1]))
    return out


def four_vortex_velocity(n):
    """Initial velocity of the four-way vortex merging of Section 7.3 on the
    periodic unit square, as values at the n^2 cell centres: the vorticity is
    the sum of four tanh-profiled vortices (strengths -150, 50, 50, 50), the
    stream function solves the periodic Poisson equation Delta psi = -omega
    (by FFT of the point values: synthetic input data, not the method), and
    u = (psi_y, -psi_x).  Returns (u, v) as n x n arrays indexed [x, y]."""
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    gam = [-150.0, 50.0, 50.0, 50.0]
    ctr = [(0.5, 0.5), (0.59, 0.5), (0.455, 0.5 + 0.045 * math.sqrt(3)), (0.455, 0.5 - 0.045 * math.sqrt(3))]
    om = sum(0.5 * g * (1 + np.tanh(3 - 100 * np.hypot(X - cx, Y - cy))) for g, (cx, cy) in zip(gam, ctr))
    k = 2 * math.pi * np.fft.fftfreq(n, 1.0 / n)
    KX, KY = np.meshgrid(k, k, indexing="ij")
    k2 = KX ** 2 + KY ** 2
    k2[0, 0] = 1.0
    ph = np.fft.fft2(om) / k2
    ph[0, 0] = 0.0
    u = np.real(np.fft.ifft2(1j * KY * ph))
    v = np.real(np.fft.ifft2(-1j * KX * ph))
    return u, v
