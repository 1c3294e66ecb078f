"""Test fixtures: manufactured problems with closed-form cell and face
averages (no solver arithmetic).  A field is a sum of products of 1-D
functions; each 1-D factor supplies its averages, point values and
derivatives."""
import math

import numpy as np

from oracle.level import PAD


class Poly1:
    """1-D polynomial sum_k c[k] x^k."""

    def __init__(self, coef):
        self.c = [float(v) for v in coef]

    def avg(self, x0, h, n):
        xl = x0 + h * np.arange(n)
        xr = xl + h
        return sum(a * (xr ** (k + 1) - xl ** (k + 1)) / ((k + 1) * h) for k, a in enumerate(self.c))

    def val(self, x):
        return sum(a * x ** k for k, a in enumerate(self.c))

    def der(self, x):
        return sum(k * a * x ** (k - 1) for k, a in enumerate(self.c) if k)

    def d1(self):
        return Poly1([k * a for k, a in enumerate(self.c)][1:] or [0.0])

    def d2(self):
        return Poly1([k * (k - 1) * a for k, a in enumerate(self.c)][2:] or [0.0])

    def __neg__(self):
        return Poly1([-a for a in self.c])


class Trig1:
    """1-D function A sin(w x + b)."""

    def __init__(self, w, b=0.0, A=1.0):
        self.w, self.b, self.A = w, b, A

    def avg(self, x0, h, n):
        xl = x0 + h * np.arange(n)
        return self.A * (np.cos(self.w * xl + self.b) - np.cos(self.w * (xl + h) + self.b)) / (self.w * h)

    def val(self, x):
        return self.A * math.sin(self.w * x + self.b)

    def der(self, x):
        return self.A * self.w * math.cos(self.w * x + self.b)

    def d2(self):
        return Trig1(self.w, self.b, -self.A * self.w ** 2)


def _outer(vecs):
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return out


def problem(lev, terms, op, c, x0=0.0):
    """Cell averages of u, of (I - c Lap) u or Lap u, and the face data of
    the level's fill kinds ('D': face averages of u, 'N': face averages of
    the outward normal derivative) on every row end.  Returns padded dense
    arrays (u, f, fd)."""
    D, n, h = lev.dim, lev.shape, lev.h
    u = lev.zeros()
    lap = lev.zeros()
    for term in terms:
        avgs = [t.avg(x0, h, m) for t, m in zip(term, n)]
        u[lev.inner] += _outer(avgs)
        for d in range(D):
            a2 = list(avgs)
            a2[d] = term[d].d2().avg(x0, h, n[d])
            lap[lev.inner] += _outer(a2)
    f = u - c * lap if op == "helmholtz" else lap
    f[~lev.mask] = 0.0
    u[~lev.mask] = 0.0
    fd = {}
    for d in range(D):
        for s in (0, 1):
            kinds = lev.end_kind(d, s)
            arr = lev.zeros()
            idx = np.argwhere(kinds != None)  # noqa: E711
            for pos in idx:
                i = pos - PAD
                xf = x0 + (i[d] + s) * h
                tot = 0.0
                for term in terms:
                    prod = 1.0
                    for dd in range(D):
                        if dd == d:
                            if kinds[tuple(pos)] == "N":
                                prod *= term[dd].der(xf) * (1 if s == 1 else -1)
                            else:
                                prod *= term[dd].val(xf)
                        else:
                            prod *= term[dd].avg(x0 + i[dd] * h, h, 1)[0]
                    tot += prod
                arr[tuple(pos)] = tot
            fd[(d, s)] = arr
    return u, f, fd
