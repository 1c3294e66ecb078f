"""Oracle: the finite-volume formulas of Section 3 (spatial discretization).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every function here is plain arithmetic on its arguments, so it works
unchanged on Python ``fractions.Fraction`` scalars (used by the exactness
pins) and on numpy float64 arrays (used by the solver).
"""


def laplacian_1d(um2, um1, u0, up1, up2, h):
    """One direction of the discrete Laplacian, eq. (discreteOps c):
    (1/12h^2)(-u[i-2] + 16u[i-1] - 30u[i] + 16u[i+1] - u[i+2])."""
    return (-um2 + 16 * um1 - 30 * u0 + 16 * up1 - up2) / (12 * h * h)


def gradient_1d(um2, um1, up1, up2, h):
    """One component of the discrete gradient, eq. (discreteOps a):
    (1/12h)(-u[i+2] + 8u[i+1] - 8u[i-1] + u[i-2])."""
    return (-up2 + 8 * up1 - 8 * um1 + um2) / (12 * h)


def face_value(um1, u0, up1, up2):
    """Face average on the high face i+1/2 from cell averages,
    first row of eq. (cell2face)."""
    return (-up2 + 7 * up1 + 7 * u0 - um1) / 12


def face_derivative(um1, u0, up1, up2, h):
    """Face average of the normal derivative on the high face i+1/2,
    second row of eq. (cell2face):
    (1/12h)(-u[i+2] + 15u[i+1] - 15u[i] + u[i-1])."""
    return (-up2 + 15 * up1 - 15 * u0 + um1) / (12 * h)


def dirichlet_ghosts(u0, u1, u2, u3, g):
    """Fifth-order Dirichlet ghost fill, eq. (velBCHomoDiri5th).

    u0 is the cell that abuts the boundary face, u1..u3 the next interior
    cells going away from the face, g the face average of the Dirichlet
    datum on that face.  Returns (first ghost, second ghost) going outward.
    The printed coefficient 75/3 of the second ghost equals 25.
    """
    g1 = (-77 * u0 + 43 * u1 - 17 * u2 + 3 * u3) / 12 + 5 * g
    g2 = (-505 * u0 + 335 * u1 - 145 * u2 + 27 * u3) / 12 + 25 * g
    return g1, g2


def neumann_ghosts(u0, u1, u2, u3, gn, h):
    """Fifth-order Neumann ghost fill, eq. (Neumann5).

    gn is the face average of the derivative along the OUTWARD normal.
    """
    g1 = (5 * u0 + 9 * u1 - 5 * u2 + u3) / 10 + 6 * h * gn / 5
    g2 = (-75 * u0 + 145 * u1 - 75 * u2 + 15 * u3) / 10 + 6 * h * gn
    return g1, g2


def dirichlet_face_normal_derivative(u0, u1, u2, u3, g, h):
    """Face average of the outward normal derivative from a Dirichlet datum
    and four interior cell averages, eq. (smoothExtend5p-face-deri)."""
    return (-415 * u0 + 161 * u1 - 55 * u2 + 9 * u3) / (72 * h) + 25 * g / (6 * h)
