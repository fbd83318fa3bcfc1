"""Pins of the oracle's backward-error measures on hand-worked 2 x 2 cases.

Every gate of the mixed-precision path (eta <= 1e-12) and the benchmark's
check rest on these three functions, so each denominator term is pinned by a
case with a nonzero residual whose norms were worked out by hand as integers:

  potrf : eta = ||A - X^T X||_F / ||A||_F
  trsyl : eta = ||C - L X - X U||_F / ((||L||_F + ||U||_F) ||X||_F + ||C||_F)
  trlyap: eta = ||S - L X - X L^T||_F / (2 ||L||_F ||X||_F + ||S||_F)

(the equations are those of the paper's Fig. 2 caption; the normalisations
are the standard normwise backward errors of the three problems).  Each case
is chosen so that dropping a norm, counting an off-diagonal entry of a
symmetric matrix once instead of twice, or changing the Lyapunov factor 2
moves eta away from the printed fraction.  Entries outside the referenced
triangles are set to large junk values, which must not enter any norm.
"""
import numpy as np
import pytest

JUNK = 1.0e3


def test_eta_potrf_hand_case(orc):
    # A (symmetric, upper triangle given)      X (upper)
    #   [4 2]                                   [2 0]
    #   [2 5]                                   [0 2]
    # X^T X = 4 I, R = A - X^T X = [[0, 2], [2, 1]]
    # ||R||_F^2 = 0 + 4 + 4 + 1 = 9          -> 3
    # ||A||_F^2 = 16 + 4 + 4 + 25 = 49       -> 7  (off-diagonal counted twice)
    A = np.array([[4.0, 2.0], [JUNK, 5.0]])
    X = np.array([[2.0, 0.0], [JUNK, 2.0]])
    assert orc.eta_potrf(A, X) == 3.0 / 7.0
    # the wrong readings give other values: a one-sided ||A|| (sqrt 45) or a
    # residual over the upper triangle only (sqrt 5)
    assert abs(3.0 / 7.0 - 3.0 / np.sqrt(45.0)) > 1e-3
    assert abs(3.0 / 7.0 - np.sqrt(5.0) / 7.0) > 1e-3


def test_eta_trsyl_hand_case(orc):
    # L = [[1, 0], [-2, 2]]   ||L||_F^2 = 1 + 4 + 4 = 9         -> 3
    # U = [[2, 4], [0, 4]]    ||U||_F^2 = 4 + 16 + 16 = 36      -> 6
    # X = [[-2, -2], [-2, -2]] ||X||_F^2 = 16                   -> 4
    # L X = [[-2, -2], [0, 0]], X U = [[-4, -16], [-4, -16]]
    # L X + X U = [[-6, -18], [-4, -16]]
    # C = [[-8, -20], [-3, -16]]  ||C||_F^2 = 64 + 400 + 9 + 256 = 729 -> 27
    # R = C - L X - X U = [[-2, -2], [1, 0]]  ||R||_F^2 = 9    -> 3
    # eta = 3 / ((3 + 6) * 4 + 27) = 3 / 63 = 1 / 21
    L = np.array([[1.0, JUNK], [-2.0, 2.0]])
    U = np.array([[2.0, 4.0], [JUNK, 4.0]])
    X = np.array([[-2.0, -2.0], [-2.0, -2.0]])
    C = np.array([[-8.0, -20.0], [-3.0, -16.0]])
    eta = orc.eta_trsyl(L, U, C, X)
    assert eta == pytest.approx(1.0 / 21.0, rel=1e-15)
    # each term matters: without ||C|| 3/36, without ||U|| 3/39, without ||L|| 3/51
    for wrong in (3.0 / 36.0, 3.0 / 39.0, 3.0 / 51.0):
        assert abs(eta - wrong) > 1e-3


def test_eta_trlyap_hand_case(orc):
    # L = [[1, 0], [-2, 2]]      ||L||_F = 3
    # X = [[2, -2], [-2, 2]]     ||X||_F^2 = 16                  -> 4
    # L X = [[2, -2], [-8, 8]],  X L^T = (L X)^T = [[2, -8], [-2, 8]]
    # L X + X L^T = [[4, -10], [-10, 16]]
    # S = [[4, -12], [-12, 15]]  ||S||_F^2 = 16 + 144 + 144 + 225 = 529 -> 23
    # R = [[0, -2], [-2, -1]]    ||R||_F^2 = 9                   -> 3
    # eta = 3 / (2 * 3 * 4 + 23) = 3 / 47
    L = np.array([[1.0, JUNK], [-2.0, 2.0]])
    S = np.array([[4.0, JUNK], [-12.0, 15.0]])   # lower triangle given
    X = np.array([[2.0, -2.0], [-2.0, 2.0]])
    eta = orc.eta_trlyap(L, S, X)
    assert eta == pytest.approx(3.0 / 47.0, rel=1e-15)
    # factor 1 instead of 2: 3/35; ||S|| with the off-diagonal once: 3/(24 + sqrt 385)
    for wrong in (3.0 / 35.0, 3.0 / (24.0 + np.sqrt(385.0))):
        assert abs(eta - wrong) > 1e-4


def test_eta_scale_invariance(orc):
    # the normwise backward errors are invariant under scaling the equation:
    # (L, U, C) -> (a L, a U, a C) leaves X and eta unchanged; (A, X) ->
    # (a^2 A, a X) likewise for the factorisation
    rng = np.random.default_rng(3)
    n, a = 5, 8.0
    L = np.tril(rng.standard_normal((n, n))) + 3 * np.eye(n)
    U = np.triu(rng.standard_normal((n, n))) + 3 * np.eye(n)
    C = rng.standard_normal((n, n))
    X = rng.standard_normal((n, n))          # not a solution: eta is O(1)
    e1 = orc.eta_trsyl(L, U, C, X)
    e2 = orc.eta_trsyl(a * L, a * U, a * C, X)
    assert e1 > 0.1 and e2 == pytest.approx(e1, rel=1e-14)
    S = C + C.T
    e1 = orc.eta_trlyap(L, S, X + X.T)
    e2 = orc.eta_trlyap(a * L, a * S, X + X.T)
    assert e1 > 0.1 and e2 == pytest.approx(e1, rel=1e-14)
    B = rng.standard_normal((n, n))
    A = B.T @ B + n * np.eye(n)
    Xu = np.triu(rng.standard_normal((n, n)))
    e1 = orc.eta_potrf(A, Xu)
    e2 = orc.eta_potrf(a * a * A, a * Xu)
    assert e1 > 0.1 and e2 == pytest.approx(e1, rel=1e-14)
