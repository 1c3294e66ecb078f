"""Oracle: the coarse-fine interface conditions of a refined level (Section
6.3, CIC-1..3) and the correction of their normal face averages that
restores the discrete compatibility condition (Section 6.4, eqs.
velocity_disc_solvabilityCond and correctingFaceAvg).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The face data a level solved on its own needs on its coarse-fine faces are
computed from the coarse level's data at four earlier coarse times:

* CIC-1: the face between a row-end cell e of the fine level and the
  position beyond it (outward along d) has two fine cells on each side
  along the normal, e - s, e inside and e + s, e + 2s outside (s the
  outward unit step);
* CIC-2: for each coarse time t_(-i), i = 0..3, the fine cell averages of
  those four cells are interpolated from the coarse data by AMRCFI (the
  tensor-product conservative quartic of oracle/amr.py, evaluated at fine
  cells inside the level as well as outside), and eq. cell2face turns them
  into the face average (first row) or the face average of the derivative
  (second row; the outward normal derivative here);
* CIC-3: eq. timeInterp takes those four face averages to the time t*.

Readings of eq. timeInterp (garbled in print):

* the columns of the printed matrix belong to the times t_(-1) - 2k,
  t_(-1) - k, t_(-1), t_(-1) + k, i.e. (t_(-3), t_(-2), t_(-1), t_(-0)) with
  t_(-i) = t_(-0) - i k: the first row puts weight 1 on the third column at
  eta = 0 and on the fourth at eta = k, the opposite of the order of the
  printed data vector;
* with the printed prefactor 1/(6k^3) the second row yields d phi/dt itself
  (its entries are O(k^2)), not k d phi/dt as the left-hand side reads.

The functions here follow those readings; ``hist`` lists the coarse data
from the newest, hist[i] = phi(t_(-i)).
"""
import numpy as np

from . import fv
from .amr import weights, window_shift
from .level import PAD


def time_interp_matrix(k, eta):
    """The 2 x 4 matrix of eq. timeInterp, columns (t_(-3), t_(-2), t_(-1),
    t_(-0)), entries as printed divided by 6k^3: row 0 gives phi(t*), row 1
    d phi / dt (t*), t* = t_(-1) + eta.  Plain arithmetic: works on
    Fractions."""
    e, e2, e3 = eta, eta * eta, eta * eta * eta
    k2, k3 = k * k, k * k * k
    r0 = [-e3 + k2 * e, 3 * e3 + 3 * k * e2 - 6 * k2 * e, -3 * e3 - 6 * k * e2 + 3 * k2 * e + 6 * k3,
          e3 + 3 * k * e2 + 2 * k2 * e]
    r1 = [-3 * e2 + k2, 9 * e2 + 6 * k * e - 6 * k2, -9 * e2 - 12 * k * e + 3 * k2, 3 * e2 + 6 * k * e + 2 * k2]
    return [[v / (6 * k3) for v in r0], [v / (6 * k3) for v in r1]]


def fine_average(H, l, Uc, g):
    """AMRCFI value of the fine cell at level-l index g (tuple) from the
    coarse array Uc: the average over that cell of the tensor-product quartic
    whose averages over the 5^D window around its parent equal Uc."""
    coarse = H.levels[l - 1]
    D = coarse.dim
    P = [gi // H.ratio for gi in g]
    a = [gi % H.ratio for gi in g]
    shifts = [window_shift(P[d], coarse.shape[d]) for d in range(D)]
    lo = [P[d] + shifts[d] - 2 for d in range(D)]
    sl = tuple(slice(PAD + lo[d], PAD + lo[d] + 5) for d in range(D))
    if not coarse.mask[sl].all():
        raise ValueError("interpolation window leaves level %d" % (l - 1))
    val = Uc[sl]
    for d in range(D):
        val = np.tensordot(weights(H.ratio)[(shifts[d], a[d])], val, axes=([0], [0]))
    return float(val)


def cf_row_ends(lev, d, s):
    """Row-end cells of the level on side s along d whose outer neighbour is
    inside the domain and not a cell of the level: the coarse-fine faces
    (padded index arrays)."""
    return np.argwhere(lev.row_end(d, s) & ~lev.end_is_physical(d, s))


def cic_face_data(H, l, hist, k, eta, kind="value"):
    """Face data of level l on its coarse-fine faces at t* = t_(-1) + eta
    (CIC-1..3, in the paper's order: space for every coarse time, then
    time).  kind 'value': face averages (eq. cell2face, first row);
    'normal_derivative': face averages of the outward normal derivative
    (second row).  Returns (fd, dfd): {(d, s): padded array} holding, at the
    row-end cell, the datum at t* and its time derivative; zero elsewhere."""
    fine = H.levels[l]
    h = fine.h
    T = time_interp_matrix(k, eta)
    fd, dfd = fine.zero_face_data(), fine.zero_face_data()
    for d in range(fine.dim):
        for s in (0, 1):
            sg = 1 if s else -1
            for pos in cf_row_ends(fine, d, s):
                e = pos - PAD
                per_time = []
                for i in range(4):  # hist[i] = phi(t_(-i))
                    vals = []
                    for m in (-1, 0, 1, 2):  # e - s, e, e + s, e + 2s along the outward normal
                        g = e.copy()
                        g[d] += m * sg
                        vals.append(fine_average(H, l, hist[i], tuple(int(v) for v in g)))
                    if kind == "value":
                        per_time.append(fv.face_value(vals[0], vals[1], vals[2], vals[3]))
                    else:  # derivative along the outward normal
                        per_time.append(fv.face_derivative(vals[0], vals[1], vals[2], vals[3], h))
                # columns of the matrix run from t_(-3) to t_(-0)
                data = [per_time[3], per_time[2], per_time[1], per_time[0]]
                fd[(d, s)][tuple(pos)] = sum(T[0][j] * data[j] for j in range(4))
                dfd[(d, s)][tuple(pos)] = sum(T[1][j] * data[j] for j in range(4))
    return fd, dfd


def compatibility_defects(lev, fdv):
    """Per face-connected component c of the level: sum over its
    coarse-fine and physical faces of the outward normal velocity face
    average (eq. velocity_disc_solvabilityCond; every face of a level has
    the same area).  fdv[d]: face data of velocity component d; the normal
    component on a face normal to d is component d times the outward sign."""
    tot = np.zeros(lev.ncomp)
    for d in range(lev.dim):
        for s in (0, 1):
            sg = 1.0 if s else -1.0
            end = lev.row_end(d, s)
            np.add.at(tot, lev.labels[end], sg * fdv[d][(d, s)][end])
    return tot


def cic_correct(lev, fdv):
    """Eq. correctingFaceAvg: on every component with coarse-fine faces, one
    constant delta added to the outward normal face average of every one of
    its coarse-fine faces, -delta |faces| = the component's compatibility
    defect.  Returns (corrected copy of fdv, deltas per component)."""
    out = [{key: v.copy() for key, v in per.items()} for per in fdv]
    defect = compatibility_defects(lev, fdv)
    ncf = np.zeros(lev.ncomp, dtype=int)
    for d in range(lev.dim):
        for s in (0, 1):
            cf = lev.row_end(d, s) & ~lev.end_is_physical(d, s)
            np.add.at(ncf, lev.labels[cf], 1)
    delta = np.where(ncf > 0, -defect / np.maximum(ncf, 1), 0.0)
    for d in range(lev.dim):
        for s in (0, 1):
            sg = 1.0 if s else -1.0
            cf = lev.row_end(d, s) & ~lev.end_is_physical(d, s)
            out[d][(d, s)][cf] += sg * delta[lev.labels[cf]]
    return out, delta
