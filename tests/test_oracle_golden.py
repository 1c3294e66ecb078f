"""The oracle's Section 3 formulas against the coefficients the paper prints
(tests/golden/section3_coefficients.txt, one line per equation row): each
formula is applied to unit vectors in exact rational arithmetic and must
return the printed coefficient divided by the printed denominator, for every
operand and for the boundary datum."""
import os
from fractions import Fraction as Fr

import pytest

from oracle import fv

HERE = os.path.dirname(os.path.abspath(__file__))


def rows():
    out = {}
    for line in open(os.path.join(HERE, "golden", "section3_coefficients.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, _, ops, den, coef, datum = [p.strip() for p in line.split("|")]
        out[name] = (ops.split(), den, [Fr(c) for c in coef.split()], datum)
    return out


ROWS = rows()
H = Fr(1, 7)  # any nonzero mesh width


def denominator(den):
    k, *hp = den.split()
    return Fr(k) * ({"h": H, "h^2": H * H}[hp[0]] if hp else 1)


def datum_value(datum):
    if datum == "-":
        return None
    k, *hp = datum.split()
    return Fr(k) * (H if hp else 1)


def evaluate(name, args, g):
    if name == "laplacian_1d":
        return fv.laplacian_1d(*args, H)
    if name == "gradient_1d":
        return fv.gradient_1d(*args, H)
    if name == "face_value":
        return fv.face_value(*args)
    if name == "face_derivative":
        return fv.face_derivative(*args, H)
    if name.startswith("dirichlet"):
        return fv.dirichlet_ghosts(*args, g)[int(name[-1]) - 1]
    return fv.neumann_ghosts(*args, g, H)[int(name[-1]) - 1]


@pytest.mark.parametrize("name", sorted(ROWS))
def test_printed_coefficients(name):
    ops, den, coef, datum = ROWS[name]
    n = len(ops)
    assert len(coef) == n
    for j in range(n):
        args = [Fr(1) if m == j else Fr(0) for m in range(n)]
        assert evaluate(name, args, Fr(0)) == coef[j] / denominator(den), (name, ops[j])
    want = datum_value(datum)
    if want is not None:
        assert evaluate(name, [Fr(0)] * n, Fr(1)) == want


def test_every_row_is_covered():
    assert set(ROWS) == {"laplacian_1d", "gradient_1d", "face_value", "face_derivative", "dirichlet_ghost1",
                         "dirichlet_ghost2", "neumann_ghost1", "neumann_ghost2"}
