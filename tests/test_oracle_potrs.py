"""Pins of the oracle's solve with the Cholesky factor (potrs): A^{-1} B for
A = X^T X, the consumer of the factorization of Fig. 2a.  Each check rests on
something other than the oracle's own recurrence: a closed form, exact dyadic
arithmetic, dense Gaussian elimination, or the residual of A Y = B."""
import numpy as np
import pytest

from paper_1906_08613_amd import inputs as I

U64 = 2.0 ** -53


def test_diagonal_factor_closed_form(orc):
    d = np.array([2.0, 0.5, 3.0, 1.25])
    X = np.diag(d)
    B = np.arange(12, dtype=np.float64).reshape(4, 3) - 5.0
    Y, info = orc.potrs(X, B)
    assert info == 0
    assert np.allclose(Y, B / (d ** 2)[:, None], rtol=1e-15, atol=0)


def test_exact_dyadic_case(orc):
    # power-of-2 diagonal, integer strict upper part, integer Y: every
    # intermediate of both substitutions is an exact dyadic number
    X = np.array([[2.0, 1.0, -3.0, 2.0],
                  [0.0, 4.0, 1.0, -1.0],
                  [0.0, 0.0, 1.0, 5.0],
                  [0.0, 0.0, 0.0, 2.0]])
    Yt = np.array([[1.0, -2.0], [3.0, 0.0], [-1.0, 4.0], [2.0, 1.0]])
    B = (X.T.astype(np.int64) @ X.astype(np.int64) @ Yt.astype(np.int64)).astype(np.float64)
    Y, info = orc.potrs(X + np.tril(np.full((4, 4), 7.0), -1), B)   # the strict lower part is not read
    assert info == 0
    assert np.array_equal(Y, Yt)


@pytest.mark.parametrize("n,m", [(1, 1), (3, 2), (9, 5), (17, 1)])
def test_matches_dense_elimination(orc, n, m):
    rng = np.random.default_rng(10 + n)
    X = np.triu(rng.uniform(-1, 1, (n, n))) + np.diag(rng.uniform(1, 2, n))
    A = X.T @ X
    B = rng.normal(size=(n, m))
    Y, info = orc.potrs(X, B)
    assert info == 0
    for j in range(m):
        y, st = orc.gepp(A, B[:, j])
        assert st == 0
        assert np.allclose(Y[:, j], y, rtol=0, atol=1e-12 * np.abs(y).max())


def test_residual_after_factorization(orc):
    n, m = 40, 7
    A = I.potrf_problem("potrs-pin", n, 1)[0]
    X, info = orc.potrf(A)
    assert info == 0
    B = np.random.default_rng(3).normal(size=(n, m))
    Y, info = orc.potrs(X, B)
    assert info == 0
    r = np.abs(A @ Y - B).max()
    assert r <= 20 * n * U64 * np.abs(A).max() * np.abs(Y).max() * n


def test_zero_pivot_reports_and_leaves_b(orc):
    X = np.triu(np.ones((4, 4))) + np.eye(4)
    X[2, 2] = 0.0
    B = np.ones((4, 2))
    Y, info = orc.potrs(X, B)
    assert info == 3
    assert np.array_equal(Y, B)


def test_batch_equals_single(orc):
    n, m, b = 12, 3, 5
    rng = np.random.default_rng(7)
    X = np.triu(rng.uniform(-1, 1, (b, n, n))) + np.eye(n) * 2.0
    B = rng.normal(size=(b, n, m))
    Yb, info = orc.potrs_batch(X, B)
    assert np.all(info == 0)
    for k in range(b):
        Y, _ = orc.potrs(X[k], B[k])
        assert np.array_equal(Yb[k], Y)


# ------------------------------------------------------------ inverse (potri)
def test_inverse_diagonal_closed_form(orc):
    d = np.array([2.0, 0.25, 3.0])
    Y, info = orc.potri(np.diag(d))
    assert info == 0
    assert np.allclose(Y, np.diag(1.0 / d ** 2), rtol=1e-15, atol=0)


def test_inverse_exact_unit_factor(orc):
    # unit diagonal, integer entries: X^{-1} is an integer matrix and so is
    # A^{-1} = X^{-1} X^{-T}; every intermediate is an exact integer
    X = np.array([[1.0, 2.0, -1.0, 3.0],
                  [0.0, 1.0, 4.0, -2.0],
                  [0.0, 0.0, 1.0, 1.0],
                  [0.0, 0.0, 0.0, 1.0]])
    Xi = np.rint(np.linalg.inv(X))
    assert np.array_equal(Xi @ X, np.eye(4))
    Y, info = orc.potri(X)
    assert info == 0
    assert np.array_equal(Y, Xi @ Xi.T)


@pytest.mark.parametrize("n", [1, 6, 13])
def test_inverse_matches_elimination_and_residual(orc, n):
    A = I.potrf_problem("potri-pin", n, 1)[0]
    X, info = orc.potrf(A)
    assert info == 0
    Y, info = orc.potri(X)
    assert info == 0
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        y, st = orc.gepp(A, e)
        assert st == 0 and np.allclose(Y[:, j], y, rtol=0, atol=1e-13 * np.abs(y).max())
    assert np.abs(A @ Y - np.eye(n)).max() <= 1e-13


def test_inverse_zero_pivot(orc):
    X = np.triu(np.ones((3, 3)))
    X[1, 1] = 0.0
    Y, info = orc.potri(X)
    assert info == 2 and np.array_equal(Y, np.eye(3))
