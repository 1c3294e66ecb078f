"""The exact bottom solve's factorisation on the host (amg_dense_inverse:
blocked Gauss-Jordan elimination with partial pivoting, the inverse the
coarsest depth's solve applies): integer matrices with exact inverses,
matrices that need row exchanges, sizes around the 64-column blocks, the
bordered 4th-order Laplacians the bottom assembles, thread counts, and the
error returns.  No GPU: the call touches no device."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02663_amd", "libamg.so")


@pytest.fixture(scope="module")
def A():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2506_02663_amd import amg
    return amg


def test_exact_small_inverses(A):
    # integer matrices of determinant 1: their inverses are integer and exact
    m = np.array([[2.0, 1.0], [1.0, 1.0]])
    assert np.array_equal(A.dense_inverse(m), np.array([[1.0, -1.0], [-1.0, 2.0]]))
    m = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 3.0], [0.0, 0.0, 1.0]])
    assert np.array_equal(A.dense_inverse(m), np.array([[1.0, -2.0, 6.0], [0.0, 1.0, -3.0], [0.0, 0.0, 1.0]]))
    assert np.array_equal(A.dense_inverse(np.array([[4.0]])), np.array([[0.25]]))


@pytest.mark.parametrize("n", [3, 64, 100])
def test_row_exchanges(A, n):
    # a permuted diagonal: every pivot comes from another row (zero diagonal)
    rng = np.random.default_rng(n)
    perm = np.roll(np.arange(n), 1)
    d = 2.0 ** rng.integers(-3, 4, n)
    m = np.zeros((n, n))
    m[np.arange(n), perm] = d
    want = np.zeros((n, n))
    want[perm, np.arange(n)] = 1.0 / d  # exact: powers of two
    assert np.array_equal(A.dense_inverse(m, threads=2), want)


@pytest.mark.parametrize("n", [1, 5, 63, 64, 65, 127, 130, 257])
@pytest.mark.parametrize("threads", [1, 4])
def test_random_matrices(A, n, threads):
    rng = np.random.default_rng(1000 + n)
    m = rng.normal(size=(n, n)) + n ** 0.5 * np.eye(n)
    inv = A.dense_inverse(m, threads=threads)
    assert np.abs(m @ inv - np.eye(n)).max() < 1e-12 * n
    ref = np.linalg.inv(m)
    assert np.abs(inv - ref).max() <= 1e-11 * np.abs(ref).max()


def bordered_laplacian(nx, ny):
    """The periodic 2D 4th-order stencil (its null vector the constant),
    bordered with the zero-mean constraint, as the bottom assembles a
    singular component."""
    n = nx * ny
    m = np.zeros((n + 1, n + 1))
    for y in range(ny):
        for x in range(nx):
            i = x + nx * y
            m[i, i] += -60.0
            for o, w in ((1, 16.0), (-1, 16.0), (2, -1.0), (-2, -1.0)):
                m[i, (x + o) % nx + nx * y] += w
                m[i, x + nx * ((y + o) % ny)] += w
            m[i, n] = m[n, i] = 1.0
    return m


@pytest.mark.parametrize("shape", [(8, 8), (12, 10), (16, 16)])
def test_bordered_laplacian(A, shape):
    m = bordered_laplacian(*shape)
    inv = A.dense_inverse(m, threads=3)
    n = m.shape[0]
    assert np.abs(m @ inv - np.eye(n)).max() < 1e-12
    # the top-left block maps a zero-mean right-hand side to the zero-mean
    # solution of the singular system
    rng = np.random.default_rng(7)
    f = rng.normal(size=n - 1)
    f -= f.mean()
    u = inv[:-1, :-1] @ f
    assert abs(u.mean()) < 1e-13
    assert np.abs(m[:-1, :-1] @ u - f).max() < 1e-11 * np.abs(f).max()


def test_errors(A):
    with pytest.raises(A.AmgError) as e:
        A.dense_inverse(np.array([[1.0, 2.0], [2.0, 4.0]]))  # singular
    assert e.value.code == A.EUNSUPPORTED
    m = np.eye(70)
    m[:, 66] = 0.0  # a zero column in the second block of columns
    with pytest.raises(A.AmgError) as e:
        A.dense_inverse(m, threads=2)
    assert e.value.code == A.EUNSUPPORTED
    with pytest.raises(A.AmgError) as e:
        A.dense_inverse(np.eye(3), threads=0)
    assert e.value.code == A.EINVAL
    with pytest.raises(ValueError):
        A.dense_inverse(np.ones((2, 3)))
