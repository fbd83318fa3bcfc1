"""Pins of the CPU oracle against what the paper and the mathematics fix.

The paper prints no worked numerical example, so the oracle is pinned by:
exact hand-worked cases (tests/golden), closed forms for diagonal, 1x1 and
2x2 inputs, brute-force Kronecker solves on tiny n, library routines for the
same equations (numpy/scipy, used here only), the defining identities, and the
reduction of the Lyapunov equation to the Sylvester equation with U = L^T.
Each pin is chosen so that a dropped term, a wrong sign, a wrong index or a
transposed operand in the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from paper_1906_08613_amd import inputs as I
from tests.golden.load import load


# ------------------------------------------------------------ exact goldens
def test_golden_potrf_exact(orc):
    g = load("potrf_int3.txt")
    X, info = orc.potrf(g["A"])
    assert info == 0
    assert np.array_equal(X, g["X"])


def test_golden_trsyl_exact(orc):
    g = load("trsyl_dyadic3.txt")
    X, info = orc.trsyl(g["L"], g["U"], g["C"])
    assert info == 0
    assert np.array_equal(X, g["X"])


def test_golden_trlyap_exact(orc):
    g = load("trlyap_dyadic3.txt")
    X, info = orc.trlyap(g["L"], np.tril(g["S"]))
    assert info == 0
    assert np.array_equal(X, g["X"])


def test_golden_fixtures_are_consistent():
    # the fixtures themselves satisfy the printed equations (guards typing slips)
    g = load("potrf_int3.txt")
    assert np.array_equal(g["X"].T @ g["X"], g["A"])
    g = load("trsyl_dyadic3.txt")
    assert np.array_equal(g["L"] @ g["X"] + g["X"] @ g["U"], g["C"])
    g = load("trlyap_dyadic3.txt")
    assert np.array_equal(g["L"] @ g["X"] + g["X"] @ g["L"].T, g["S"])


# ------------------------------------------------------------- closed forms
def test_closed_form_1x1(orc):
    X, info = orc.potrf(np.array([[9.0]]))
    assert info == 0 and X[0, 0] == 3.0
    X, info = orc.trsyl(np.array([[3.0]]), np.array([[5.0]]), np.array([[4.0]]))
    assert info == 0 and X[0, 0] == 0.5
    X, info = orc.trlyap(np.array([[2.0]]), np.array([[6.0]]))
    assert info == 0 and X[0, 0] == 1.5


def test_closed_form_diagonal(orc):
    rng = np.random.default_rng(1)
    n = 7
    a = rng.uniform(1, 4, n)
    X, info = orc.potrf(np.diag(a))
    assert info == 0
    assert np.allclose(X, np.diag(np.sqrt(a)), rtol=0, atol=1e-15)
    l, u = rng.uniform(1, 2, n), rng.uniform(1, 2, n)
    C = rng.standard_normal((n, n))
    X, info = orc.trsyl(np.diag(l), np.diag(u), C)
    assert np.allclose(X, C / (l[:, None] + u[None, :]), rtol=1e-15, atol=0)
    S = C + C.T
    X, info = orc.trlyap(np.diag(l), S)
    assert np.allclose(X, S / (l[:, None] + l[None, :]), rtol=1e-15, atol=0)


def test_closed_form_2x2(orc):
    a11, a12, a22 = 4.0, 2.0, 5.0
    X, _ = orc.potrf(np.array([[a11, a12], [a12, a22]]))
    x11 = np.sqrt(a11)
    x12 = a12 / x11
    x22 = np.sqrt(a22 - x12 ** 2)
    assert np.allclose(X, [[x11, x12], [0, x22]], rtol=1e-15)
    L = np.array([[1.5, 0.0], [0.7, 2.5]])
    U = np.array([[1.25, -0.3], [0.0, 0.75]])
    C = np.array([[1.0, 2.0], [3.0, 4.0]])
    X, _ = orc.trsyl(L, U, C)
    x11 = C[0, 0] / (L[0, 0] + U[0, 0])
    x12 = (C[0, 1] - x11 * U[0, 1]) / (L[0, 0] + U[1, 1])
    x21 = (C[1, 0] - L[1, 0] * x11) / (L[1, 1] + U[0, 0])
    x22 = (C[1, 1] - L[1, 0] * x12 - x21 * U[0, 1]) / (L[1, 1] + U[1, 1])
    assert np.allclose(X, [[x11, x12], [x21, x22]], rtol=1e-15)
    # Lyapunov 2x2 is the Sylvester case with U = L^T
    S = np.array([[1.0, 0.5], [0.5, 2.0]])
    X, _ = orc.trlyap(L, S)
    Y, _ = orc.trsyl(L, L.T, S)
    assert np.allclose(X, Y, rtol=1e-15)


# ------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11])
def test_kron_bruteforce_sylvester(orc, n):
    L, U, C = I.trsyl_problem("kron", n, 3)
    for b in range(3):
        X, info = orc.trsyl(L[b], U[b], C[b])
        Y, st = orc.kron_sylv(L[b], U[b], C[b])
        assert info == 0 and st == 0
        assert np.max(np.abs(X - Y)) <= 1e-13 * np.max(np.abs(Y))


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10])
def test_kron_bruteforce_lyapunov(orc, n):
    L, S = I.trlyap_problem("kron", n, 3)
    for b in range(3):
        X, info = orc.trlyap(L[b], np.tril(S[b]))
        Y, st = orc.kron_lyap(L[b], np.tril(S[b]))
        assert info == 0 and st == 0
        assert np.max(np.abs(X - Y)) <= 1e-13 * np.max(np.abs(Y))


def test_gepp_against_known_solution(orc):
    # a system whose first pivot is zero, so pivoting must happen
    M = np.array([[0.0, 2.0, 1.0], [1.0, 1.0, 0.0], [2.0, 0.0, 3.0]])
    y = np.array([1.0, -2.0, 0.5])
    r, st = orc.gepp(M, M @ y)
    assert st == 0 and np.allclose(r, y, rtol=1e-15, atol=1e-15)


# --------------------------------------------------------- library routines
@pytest.mark.parametrize("n", [4, 16, 33])
def test_numpy_cholesky(orc, n):
    A = I.potrf_problem("lib", n, 2)
    for b in range(2):
        X, info = orc.potrf(np.triu(A[b]))
        assert info == 0
        assert np.allclose(X, np.linalg.cholesky(A[b]).T, rtol=0, atol=1e-13 * n)
        assert np.all(np.tril(X, -1) == 0)


@pytest.mark.parametrize("n", [4, 16, 33])
def test_scipy_sylvester(orc, n):
    L, U, C = I.trsyl_problem("lib", n, 2)
    for b in range(2):
        X, info = orc.trsyl(L[b], U[b], C[b])
        Y = sla.solve_sylvester(L[b], U[b], C[b])
        assert info == 0
        assert np.max(np.abs(X - Y)) <= 1e-12 * np.max(np.abs(Y))


@pytest.mark.parametrize("n", [4, 16, 33])
def test_scipy_lyapunov(orc, n):
    L, S = I.trlyap_problem("lib", n, 2)
    for b in range(2):
        X, info = orc.trlyap(L[b], np.tril(S[b]))
        Y = sla.solve_continuous_lyapunov(L[b], S[b])   # solves A X + X A^H = Q
        assert info == 0
        assert np.max(np.abs(X - Y)) <= 1e-12 * np.max(np.abs(Y))


# ------------------------------------------------------------------- invariants
def test_only_referenced_triangles_are_read(orc):
    n = 9
    A = I.potrf_problem("tri", n, 1)[0]
    L, U, C = [m[0] for m in I.trsyl_problem("tri", n, 1)]
    junk = np.full((n, n), np.nan)
    X1, _ = orc.potrf(np.triu(A) + np.tril(junk, -1))
    X2, _ = orc.potrf(A)
    assert np.array_equal(X1, X2)
    Y1, _ = orc.trsyl(np.tril(L) + np.triu(junk, 1), np.triu(U) + np.tril(junk, -1), C)
    Y2, _ = orc.trsyl(L, U, C)
    assert np.array_equal(Y1, Y2)
    S = C + C.T
    Z1, _ = orc.trlyap(np.tril(L) + np.triu(junk, 1), np.tril(S) + np.triu(junk, 1))
    Z2, _ = orc.trlyap(L, S)
    assert np.array_equal(Z1, Z2)


@pytest.mark.parametrize("n", [16, 64, 128])
def test_defining_identities(orc, n):
    A = I.potrf_problem("inv", n, 2)
    X, info = orc.potrf_batch(A)
    assert np.all(info == 0)
    assert np.all(orc.eta_potrf_batch(A, X) <= 1e-13)
    assert np.all(np.diagonal(X, axis1=1, axis2=2) > 0)
    assert np.all(np.tril(X, -1) == 0)
    L, U, C = I.trsyl_problem("inv", n, 2)
    Y, info = orc.trsyl_batch(L, U, C)
    assert np.all(info == 0)
    R = C - L @ Y - Y @ U
    assert np.max(np.abs(R)) <= 1e-13 * np.max(np.abs(C)) * n
    assert np.all(orc.eta_trsyl_batch(L, U, C, Y) <= 1e-13)
    L, S = I.trlyap_problem("inv", n, 2)
    Z, info = orc.trlyap_batch(L, S)
    assert np.all(info == 0)
    assert np.array_equal(Z, np.swapaxes(Z, 1, 2))            # exactly symmetric
    assert np.all(orc.eta_trlyap_batch(L, S, Z) <= 1e-13)
    # Lyapunov = Sylvester with U = L^T (reduction within the method)
    W, _ = orc.trsyl_batch(L, np.swapaxes(L, 1, 2), S)
    assert np.max(np.abs(W - Z)) <= 1e-13 * np.max(np.abs(Z))
    assert np.max(np.abs(W - np.swapaxes(W, 1, 2))) <= 1e-14 * np.max(np.abs(W)) * n


def test_eta_measures_are_exact_on_exact_solutions(orc):
    g = load("potrf_int3.txt")
    assert orc.eta_potrf(g["A"], g["X"]) == 0.0
    g = load("trsyl_dyadic3.txt")
    assert orc.eta_trsyl(g["L"], g["U"], g["C"], g["X"]) == 0.0
    g = load("trlyap_dyadic3.txt")
    assert orc.eta_trlyap(g["L"], g["S"], g["X"]) == 0.0
    # and sensitive to a one-ulp-scale change of a single entry
    g = load("trsyl_dyadic3.txt")
    X = g["X"].copy()
    X[2, 1] += 1e-6
    assert orc.eta_trsyl(g["L"], g["U"], g["C"], X) > 1e-8


# --------------------------------------------------------------- error codes
def test_info_not_positive_definite(orc):
    A = np.eye(4)
    A[2, 2] = -1.0
    _, info = orc.potrf(A)
    assert info == 3
    _, info = orc.potrf(-np.eye(3))
    assert info == 1
    A = np.eye(3)
    A[1, 1] = np.nan
    _, info = orc.potrf(A)
    assert info == 2


def test_info_zero_denominator(orc):
    n = 4
    L = np.eye(n)
    U = np.eye(n)
    L[2, 2] = -1.0                       # l_22 + u_jj = 0 for every j: first at (2, 0)
    _, info = orc.trsyl(L, U, np.ones((n, n)))
    assert info == 1 + 2 + 0 * n
    U2 = np.eye(n) * 2.0
    U2[3, 3] = -1.0                      # l_ii + u_33 = 0 only for i with l_ii = 1: first (0, 3)
    _, info = orc.trsyl(np.eye(n), U2, np.ones((n, n)))
    assert info == 1 + 0 + 3 * n
    Ll = np.eye(n)
    Ll[1, 1] = -1.0                      # l_11 + l_00 = 0: first at (1, 0)
    _, info = orc.trlyap(Ll, np.eye(n))
    assert info == 1 + 1 + 0 * n


def test_generators_deterministic():
    a = I.trsyl_problem("det", 12, 5)
    b = I.trsyl_problem("det", 12, 5)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # any sub-range regenerates the same instances
    c = I.trsyl_problem("det", 12, 2, start=3)
    assert np.array_equal(c[2], a[2][3:5])
    # SplitMix64 first outputs for seed 0 (published test vector of the mixer)
    v = I.splitmix64([0], 3)[0]
    assert [int(t) for t in v] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
def test_kappa_generators_realise_kappa(orc, kappa):
    n = 10
    A = I.potrf_kappa("kap", n, 3, kappa)
    c = np.linalg.cond(A)
    assert np.all((c > kappa / 1.01) & (c < kappa * 1.01))
    L, U, C = I.trsyl_kappa("kap", n, 3, kappa)
    for b in range(3):
        K = np.kron(np.eye(n), L[b]) + np.kron(U[b].T, np.eye(n))
        ck = np.linalg.cond(K)
        assert kappa / 10 <= ck <= kappa * 10
