"""Pins of the oracle's coarse-fine interface conditions (oracle/cic.py,
Section 6.3 CIC-1..3 and eq. correctingFaceAvg):

* the time matrix equals the printed entries of eq. timeInterp
  (tests/golden/time_interp_matrix.txt) in exact rational arithmetic, and
  under the readings taken (columns from t_(-3) to t_(-0), second row
  d phi/dt) it reproduces every cubic in time and its derivative exactly,
  quartics not;
* the face data are exact when the coarse data are the cell averages of a
  polynomial of degree <= 3 in each variable times a cubic in time (AMRCFI
  is exact to degree 4, eq. cell2face to degree 3, the time matrix to
  degree 3): face averages and outward normal derivatives at t*, and their
  time derivatives, against closed forms; a degree-5 field is not
  reproduced;
* the correction makes every component's compatibility sum vanish, moves
  only the normal face averages of coarse-fine faces, by one constant per
  component, and leaves the exact data of a divergence-free polynomial
  velocity unchanged (its sum is already zero by the divergence theorem)."""
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import amr, cic
from oracle.level import PAD
from tests.polyfix import Poly1

GOLDEN = __file__.replace("test_oracle_cic.py", "golden/time_interp_matrix.txt")


def _printed_rows():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("row"):
            rows.append([p.strip() for p in line.split("|")[1:]])
    return rows


def _eval(expr, k, eta):
    """Value of a printed polynomial entry ('3 k eta^2 - 6 k^2 eta', ...) in
    exact arithmetic: monomials are products of a coefficient, k^a, eta^b."""
    expr = expr.replace(" - ", " + -").replace("-", "-1 ") if expr.startswith("-") else expr.replace(" - ", " + -")
    total = Fr(0)
    for term in expr.split("+"):
        term = term.strip()
        if not term:
            continue
        val = Fr(1)
        for factor in term.split():
            if factor in ("-", "-1"):
                val = -val
                continue
            m = re.fullmatch(r"(-?)(k|eta)(?:\^(\d+))?", factor)
            if m:
                base = k if m.group(2) == "k" else eta
                val *= base ** int(m.group(3) or 1) * (-1 if m.group(1) else 1)
            else:
                val *= Fr(factor)
        total += val
    return total


@pytest.mark.parametrize("k,eta", [(Fr(1, 3), Fr(1, 7)), (Fr(2), Fr(-3, 2)), (Fr(5, 4), Fr(5, 4))])
def test_time_matrix_is_the_printed_one(k, eta):
    rows = _printed_rows()
    T = cic.time_interp_matrix(k, eta)
    for r in range(2):
        for j in range(4):
            assert T[r][j] == _eval(rows[r][j], k, eta) / (6 * k ** 3), (r, j)


@pytest.mark.parametrize("k,eta", [(Fr(1, 3), Fr(1, 7)), (Fr(1, 10), Fr(3, 40)), (Fr(2), Fr(0)), (Fr(1), Fr(1))])
def test_time_matrix_reproduces_cubics(k, eta):
    t1 = Fr(3, 11)  # t_(-1)
    times = [t1 - 2 * k, t1 - k, t1, t1 + k]  # the columns: t_(-3) .. t_(-0)
    T = cic.time_interp_matrix(k, eta)
    ts = t1 + eta
    for coef in ([Fr(2), Fr(-1), Fr(3), Fr(5, 2)], [Fr(0), Fr(1)], [Fr(1)]):
        q = lambda t: sum(c * t ** i for i, c in enumerate(coef))  # noqa: E731
        dq = lambda t: sum(i * c * t ** (i - 1) for i, c in enumerate(coef) if i)  # noqa: E731
        data = [q(t) for t in times]
        assert sum(T[0][j] * data[j] for j in range(4)) == q(ts)
        assert sum(T[1][j] * data[j] for j in range(4)) == dq(ts)
    # a quartic is not reproduced (the matrix is fourth order, not higher)
    data = [t ** 4 for t in times]
    if eta not in (0, k, -k, -2 * k):
        assert sum(T[0][j] * data[j] for j in range(4)) != ts ** 4


# ---------------------------------------------------------------------------
def hierarchy(ratio=2):
    # level 1: two boxes (an L-shaped component) and a separate box;
    # coarse-fine faces on every side, physical faces too
    if ratio == 4:
        boxes = [[((0, 0), (15, 15))],
                 [((0, 16), (31, 31)), ((32, 16), (47, 47)), ((16, 48), (31, 63))]]
        return amr.Hierarchy((16, 16), 1.0 / 16, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=4)
    boxes = [[((0, 0), (15, 15))],
             [((0, 8), (15, 15)), ((16, 8), (23, 23)), ((8, 24), (15, 31))]]
    return amr.Hierarchy((16, 16), 1.0 / 16, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)})


def cell_avgs(lev, px, py, scale=1.0):
    a = lev.zeros()
    a[lev.inner] = scale * np.multiply.outer(px.avg(0.0, lev.h, lev.shape[0]), py.avg(0.0, lev.h, lev.shape[1]))
    return a


PX = Poly1([0.3, -1.2, 2.0, 0.7])   # degree 3
PY = Poly1([-0.5, 0.4, 1.1, -0.9])  # degree 3
QT = [1.5, -0.8, 0.6, 0.35]         # cubic in time


def qt(t):
    return sum(c * t ** i for i, c in enumerate(QT))


def dqt(t):
    return sum(i * c * t ** (i - 1) for i, c in enumerate(QT) if i)


@pytest.mark.parametrize("kind", ["value", "normal_derivative"])
@pytest.mark.parametrize("ratio", [2, 4])
def test_face_data_exact_on_polynomials(kind, ratio):
    H = hierarchy(ratio)
    coarse, fine = H.levels
    k, eta, t0 = 0.05, 0.02, 0.4  # t_(-0) = t0, t_(-i) = t0 - i k, t* = t_(-1) + eta
    hist = [cell_avgs(coarse, PX, PY, qt(t0 - i * k)) for i in range(4)]
    fd, dfd = cic.cic_face_data(H, 1, hist, k, eta, kind)
    ts = t0 - k + eta
    h = fine.h
    n = 0
    for d in range(2):
        for s in (0, 1):
            sg = 1 if s else -1
            for pos in cic.cf_row_ends(fine, d, s):
                e = pos - PAD
                xf = (e[d] + s) * h  # the face's coordinate along d
                o = 1 - d
                if d == 0:
                    along, across = PX, PY
                else:
                    along, across = PY, PX
                tr = float(across.avg(e[o] * h, h, 1)[0])
                if kind == "value":
                    want = along.val(xf) * tr
                else:
                    want = sg * along.der(xf) * tr
                got, gotd = fd[(d, s)][tuple(pos)], dfd[(d, s)][tuple(pos)]
                assert abs(got - want * qt(ts)) <= 1e-12 * (1 + abs(want)), (d, s, e)
                assert abs(gotd - want * dqt(ts)) <= 1e-10 * (1 + abs(want)), (d, s, e)
                n += 1
    assert n > 40
    # a degree-5 profile is not reproduced
    hist5 = [cell_avgs(coarse, Poly1([0, 0, 0, 0, 0, 1.0]), PY, 1.0) for _ in range(4)]
    fd5, _ = cic.cic_face_data(H, 1, hist5, k, eta, "value")
    pos = cic.cf_row_ends(fine, 0, 1)[0]
    e = pos - PAD
    want = ((e[0] + 1) * h) ** 5 * float(PY.avg(e[1] * h, h, 1)[0])
    assert abs(fd5[(0, 1)][tuple(pos)] - want) > 1e-9


def test_correction_restores_compatibility():
    H = hierarchy()
    fine = H.levels[1]
    rng = np.random.default_rng(5)
    fdv = []
    for d in range(2):
        per = fine.zero_face_data()
        for key in per:
            e = fine.row_end(*key)
            per[key][e] = rng.normal(size=int(e.sum()))
        fdv.append(per)
    before = cic.compatibility_defects(fine, fdv)
    out, delta = cic.cic_correct(fine, fdv)
    after = cic.compatibility_defects(fine, out)
    assert np.abs(before).max() > 1e-2
    assert np.abs(after).max() < 1e-12 * np.abs(before).max() * 100
    # only normal components of coarse-fine faces moved, by +-delta of their component
    for d in range(2):
        for e_ in range(2):
            for s in (0, 1):
                diff = out[d][(e_, s)] - fdv[d][(e_, s)]
                cf = fine.row_end(e_, s) & ~fine.end_is_physical(e_, s)
                if d != e_:
                    assert np.all(diff == 0.0)
                    continue
                assert np.all(diff[~cf] == 0.0)
                sg = 1.0 if s else -1.0
                assert np.allclose(diff[cf], sg * delta[fine.labels[cf]], rtol=0, atol=1e-14)


def test_divergence_free_velocity_needs_no_correction():
    # w = (P(x) Q'(y), -P'(x) Q(y)): exact face data of a divergence-free field
    H = hierarchy()
    coarse, fine = H.levels
    P, Q = Poly1([0.2, 0.5, -0.3, 0.4]), Poly1([0.1, -0.2, 0.6, 0.25])
    comps = [(P, Q.d1()), (-P.d1(), Q)]
    k, eta = 0.1, 0.04
    fdv = []
    for d, (fx, fy) in enumerate(comps):
        hist = [cell_avgs(coarse, fx, fy) for _ in range(4)]  # steady in time
        fd, _ = cic.cic_face_data(H, 1, hist, k, eta, "value")
        # physical faces: exact face averages of the same field
        for s in (0, 1):
            for dd in range(2):
                phys = np.argwhere(fine.end_is_physical(dd, s))
                for pos in phys:
                    e = pos - PAD
                    xf = (e[dd] + s) * fine.h
                    along, across = (fx, fy) if dd == 0 else (fy, fx)
                    fd[(dd, s)][tuple(pos)] = along.val(xf) * float(across.avg(e[1 - dd] * fine.h, fine.h, 1)[0])
        fdv.append(fd)
    defects = cic.compatibility_defects(fine, fdv)
    assert np.abs(defects).max() < 1e-12
    out, delta = cic.cic_correct(fine, fdv)
    assert np.abs(delta).max() < 1e-12
