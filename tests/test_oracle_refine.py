"""Pins of the oracle's mixed-precision refinement model.

The paper computes in FP64 only; the refinement model is textbook iterative
refinement (Sylvester/Lyapunov) and the Newton correction of a Cholesky
factor.  Pins: the 1x1 Cholesky correction is Heron's square-root step, a
diagonal Sylvester system is refined exactly in one step, well-conditioned
inputs converge in few steps to the tolerance, and each fallback condition
raises its flag and returns the FP64 answer.
"""
import numpy as np
import pytest

import oracle
from paper_1906_08613_amd import inputs as I


def test_potrf_1x1_newton_is_heron(orc):
    # for n = 1 the correction x + (a - x^2)/(2x) is Heron's step (x^2 + a)/(2x)
    a = 2.0
    x0 = float(np.float32(np.sqrt(np.float32(a))))
    heron = (x0 * x0 + a) / (2.0 * x0)
    X, info, it, fl, eta = orc.refine(0, np.array([[a]]), max_iter=1, tau=1e-14)
    assert info == 0 and it == 1 and fl & oracle.CONVERGED
    # the correction is formed in FP32 from an FP64 residual: agreement to u32 * |step|
    assert abs(X[0, 0] - heron) <= 1e-14
    assert abs(X[0, 0] - x0) > 1e-9


def test_diagonal_sylvester_refines_exactly_in_one_step(orc):
    n = 6
    rng = np.random.default_rng(0)
    l, u = rng.uniform(1, 2, n), rng.uniform(1, 2, n)
    C = rng.standard_normal((n, n))
    X, info, it, fl, eta = orc.refine(1, np.diag(l), np.diag(u), C, tau=1e-15)
    assert info == 0 and it <= 1 and fl & oracle.CONVERGED
    assert np.allclose(X, C / (l[:, None] + u[None, :]), rtol=1e-15)


@pytest.mark.parametrize("op", [0, 1, 2])
@pytest.mark.parametrize("kappa", [1e2, 1e4])
def test_converges_to_tolerance(orc, op, kappa):
    n = 24
    if op == 0:
        A = I.potrf_kappa("ref", n, 1, kappa)[0]
        X, info, it, fl, eta = orc.refine(0, A, tau=1e-13)
        Xr, _ = orc.potrf(A)
    elif op == 1:
        L, U, C = [m[0] for m in I.trsyl_kappa("ref", n, 1, kappa)]
        X, info, it, fl, eta = orc.refine(1, L, U, C, tau=1e-13)
        Xr, _ = orc.trsyl(L, U, C)
    else:
        L, S = [m[0] for m in I.trlyap_kappa("ref", n, 1, kappa)]
        X, info, it, fl, eta = orc.refine(2, L, None, S, tau=1e-13)
        Xr, _ = orc.trlyap(L, S)
    assert info == 0 and fl & oracle.CONVERGED and not fl & oracle.FALLBACK
    assert 1 <= it <= 3
    assert eta <= 1e-13
    assert oracle.forward_error(X, Xr) <= 1e-16 * kappa * n * 10


def test_max_iter_zero_falls_back(orc):
    L, U, C = [m[0] for m in I.trsyl_problem("ref0", 16, 1)]
    X, info, it, fl, eta = orc.refine(1, L, U, C, max_iter=0, tau=1e-13)
    Xr, _ = orc.trsyl(L, U, C)
    assert fl & oracle.FALLBACK and it == 0
    assert np.array_equal(X, Xr)


def test_ill_conditioned_breaks_down_or_falls_back(orc):
    A = I.potrf_kappa("ref12", 24, 1, 1e12)[0]
    X, info, it, fl, eta = orc.refine(0, A, tau=1e-13)
    assert fl & (oracle.FALLBACK | oracle.BREAKDOWN)
    Xr, ir = orc.potrf(A)
    assert info == ir
    if info == 0:
        assert np.array_equal(X, Xr)


def test_nonfinite_flag(orc):
    L, U, C = [m[0] for m in I.trsyl_problem("nan", 5, 1)]
    C = C.copy()
    C[1, 2] = np.inf
    X, info, it, fl, eta = orc.refine(1, L, U, C)
    assert fl & oracle.NONFINITE
