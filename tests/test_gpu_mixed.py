"""GPU parity of the mixed-precision path with FP64 refinement.

Gate (per instance): backward error eta <= 1e-12 (the refinement target tau
is 1e-13), and forward error against the FP64 oracle within
max(1e-12, 4 n kappa u64, 2 kappa tau), u64 = 2^-53: a backward error eta
allows a forward error up to about kappa * eta, the oracle's own backward
error is a few n u64, and refinement stops as soon as eta <= tau.
Refinement decisions are checked against the oracle's refinement model and
by forcing each fallback condition from the host.
"""
import numpy as np
import pytest

import paper_1906_08613_amd as tla
from paper_1906_08613_amd import inputs as I
from tests.gpu_util import elem_err, frob_err, rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U64 = 2.0 ** -53
MIXED = ["mixed_f32", "mixed_f16", "mixed_bf16"]


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = tla.Handle(0)
    yield hd
    hd.close()


TAU = 1e-13


def fwd_ok(X, Xr, n, kappa):
    # the forward-error bound from eta <= tau is normwise; entry by entry (each
    # against its column's largest entry) it holds up to the factor sqrt(n)
    return frob_err(X, Xr).max() <= fwd_tol(n, kappa) and elem_err(X, Xr).max() <= np.sqrt(n) * fwd_tol(n, kappa)


def fwd_tol(n, kappa):
    return max(1e-12, 4 * n * kappa * U64, 2 * kappa * TAU)


def solve(h, op, mats, prec, plan=None):
    h.set_plan(op, prec, plan)
    if op == "potrf":
        d = tla.to_device_cm(np.triu(mats[0]))
        ops = tla.potrf(h, d, prec)
        torch.cuda.synchronize()
        return np.triu(tla.from_device_cm(d)), ops
    if op == "trsyl":
        dL, dU, dC = (tla.to_device_cm(m) for m in mats)
        ops = tla.trsyl(h, dL, dU, dC, prec)
        torch.cuda.synchronize()
        return tla.from_device_cm(dC), ops
    dL, dS = tla.to_device_cm(mats[0]), tla.to_device_cm(np.tril(mats[1]))
    ops = tla.trlyap(h, dL, dS, prec)
    torch.cuda.synchronize()
    return tla.from_device_cm(dS), ops


def problem(op, n, batch, kappa, tag="mixed"):
    if op == "potrf":
        return (I.potrf_kappa(tag, n, batch, kappa),)
    if op == "trsyl":
        return I.trsyl_kappa(tag, n, batch, kappa)
    return I.trlyap_kappa(tag, n, batch, kappa)


def oracle_solve(orc, op, mats):
    if op == "potrf":
        X, info = orc.potrf_batch(mats[0])
        return X, info, orc.eta_potrf_batch
    if op == "trsyl":
        X, info = orc.trsyl_batch(*mats)
        return X, info, orc.eta_trsyl_batch
    X, info = orc.trlyap_batch(*mats)
    return X, info, orc.eta_trlyap_batch


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
@pytest.mark.parametrize("prec", MIXED)
@pytest.mark.parametrize("kappa", [1e2, 1e4, 1e6])
@pytest.mark.parametrize("n", [17, 32, 64])
def test_mixed_matches_oracle(h, orc, op, prec, kappa, n):
    print(f"mixed {op} {prec} kappa={kappa:g} n={n}", flush=True)
    mats = problem(op, n, 16, kappa)
    X, ops = solve(h, op, mats, prec)
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    info = ops.info.cpu().numpy()
    st = tla.stat_view(ops.stat)
    assert np.all(info == ir)
    eta = eta_fn(*mats, X)
    assert eta.max() <= 1e-12, (eta.max(), st)
    assert fwd_ok(X, Xr, n, kappa)
    # every instance either converged or was solved again in FP64
    ok = (st["flags"] & tla.STAT_CONVERGED) | (st["flags"] & (tla.STAT_FALLBACK | tla.STAT_BREAKDOWN))
    assert np.all(ok != 0)
    conv = (st["flags"] & tla.STAT_CONVERGED) != 0
    assert np.all(st["eta"][conv] <= 1e-13)
    if prec == "mixed_f32" and kappa <= 1e4:
        assert conv.all(), st
        assert st["iters"].max() <= 3


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_iterations_match_refinement_model(h, orc, op):
    n, kappa = 24, 1e2
    mats = problem(op, n, 6, kappa, tag="model")
    X, ops = solve(h, op, mats, "mixed_f32")
    st = tla.stat_view(ops.stat)
    opi = {"potrf": 0, "trsyl": 1, "trlyap": 2}[op]
    for b in range(6):
        args = [m[b] for m in mats]
        if op == "potrf":
            _, info, it, fl, eta = orc.refine(0, args[0], tau=1e-13)
        elif op == "trsyl":
            _, info, it, fl, eta = orc.refine(1, args[0], args[1], args[2], tau=1e-13)
        else:
            _, info, it, fl, eta = orc.refine(2, args[0], None, args[1], tau=1e-13)
        assert fl & 1 and st["flags"][b] & 1
        assert abs(int(st["iters"][b]) - it) <= 1


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_max_iter_zero_forces_fp64_fallback(h, orc, op):
    n = 40
    mats = problem(op, n, 8, 1e2, tag="fb")
    plan = (0, 16, 1, 4)
    h.set_refine(1e-13, 0)
    try:
        X, ops = solve(h, op, mats, "mixed_f32", plan)
    finally:
        h.set_refine(1e-13, 8)
    st = tla.stat_view(ops.stat)
    assert np.all(st["flags"] & tla.STAT_FALLBACK)
    assert np.all(st["iters"] == 0)
    # the fallback runs the FP64 kernel code of the same plan: identical bits
    Y, ops64 = solve(h, op, mats, "f64", plan)
    assert np.array_equal(X, Y)


def test_ill_conditioned_cholesky_falls_back(h, orc):
    n, kappa = 32, 1e12
    A = I.potrf_kappa("ill", n, 8, kappa)
    X, ops = solve(h, "potrf", (A,), "mixed_f32")
    st = tla.stat_view(ops.stat)
    Xr, ir = orc.potrf_batch(A)
    assert np.all(st["flags"] & (tla.STAT_FALLBACK | tla.STAT_BREAKDOWN))
    assert np.all(ops.info.cpu().numpy() == ir)
    if np.all(ir == 0):
        assert orc.eta_potrf_batch(A, X).max() <= 1e-12


@pytest.mark.parametrize("op", ["trsyl", "trlyap"])
def test_fp32_denominator_underflow_breaks_down(h, orc, op):
    # l_00 = 1e-46 and u_00 = 0: nonzero in FP64, zero once rounded to FP32
    n = 24
    mats = [m.copy() for m in problem(op, n, 4, 1e2, tag="uflow")]
    mats[0][1, 0, 0] = 1e-46
    if op == "trsyl":
        mats[1][1, 0, 0] = 0.0
    X, ops = solve(h, op, mats, "mixed_f32")
    st = tla.stat_view(ops.stat)
    assert st["flags"][1] & tla.STAT_BREAKDOWN
    assert not st["flags"][0] & tla.STAT_BREAKDOWN
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    assert np.all(ops.info.cpu().numpy() == ir)
    assert rel_err(X, Xr).max() <= 1e-12


def test_bf16_cholesky_breakdown_is_flagged(h, orc):
    # BF16 trailing updates cannot factor kappa = 1e6 matrices: flagged and redone in FP64
    n = 64
    A = I.potrf_kappa("bf16", n, 8, 1e6)
    X, ops = solve(h, "potrf", (A,), "mixed_bf16")
    st = tla.stat_view(ops.stat)
    assert np.any(st["flags"] & (tla.STAT_BREAKDOWN | tla.STAT_FALLBACK))
    assert orc.eta_potrf_batch(A, X).max() <= 1e-12


def test_nonfinite_input_flagged(h):
    n = 20
    L, U, C = I.trsyl_problem("nan", n, 2)
    C = C.copy()
    C[1, 3, 4] = np.nan
    X, ops = solve(h, "trsyl", (L, U, C), "mixed_f32")
    st = tla.stat_view(ops.stat)
    assert st["flags"][1] & tla.STAT_NONFINITE
    assert not st["flags"][0] & tla.STAT_NONFINITE


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_every_mixed_plan(h, orc, op):
    n = 40
    mats = problem(op, n, 4, 1e3, tag="plans")
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    for prec in MIXED:
        for i in range(tla.num_candidates(op)):
            plan = tla.candidate(op, i).astuple()
            print(f"{op} {prec} plan={plan}", flush=True)
            if prec == "mixed_f16" and tla.variant_name(op, plan[0]) == "jacobi-sweeps":
                # the splitting-iteration solve has BF16 and FP32 products only
                with pytest.raises(tla.TlaError):
                    solve(h, op, mats, prec, plan)
                h.set_plan(op, prec, None)
                continue
            X, ops = solve(h, op, mats, prec, plan)
            assert eta_fn(*mats, X).max() <= 1e-12, (prec, plan)
            assert fwd_ok(X, Xr, n, 1e3), (prec, plan)


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
@pytest.mark.parametrize("n", [100, 128])
def test_mixed_large_n_placements(h, orc, op, n):
    # the FP64 solution no longer fits next to the FP32 work matrix: it lives
    # in the handle's workspace and the FP64 fallback is a second launch
    kappa = 1e4
    mats = problem(op, n, 6, kappa, tag="large")
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    for prec in ["mixed_f32", "mixed_bf16"]:
        print(f"{op} n={n} {prec}", flush=True)
        X, ops = solve(h, op, mats, prec)
        assert np.all(ops.info.cpu().numpy() == ir)
        assert eta_fn(*mats, X).max() <= 1e-12, prec
        assert fwd_ok(X, Xr, n, kappa), prec


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
@pytest.mark.parametrize("prec", MIXED)
@pytest.mark.parametrize("kappa", [1e2, 1e6])
def test_mixed_n128_condition_grid(h, orc, op, prec, kappa):
    # the mixed configuration's largest size at both ends of its condition
    # range, every mixed precision: converged or solved again in FP64, and
    # within the gate either way
    n = 128
    print(f"mixed n=128 {op} {prec} kappa={kappa:g}", flush=True)
    mats = problem(op, n, 4, kappa, tag="grid128")
    X, ops = solve(h, op, mats, prec)
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    st = tla.stat_view(ops.stat)
    assert np.all(ops.info.cpu().numpy() == ir)
    assert eta_fn(*mats, X).max() <= 1e-12, st
    assert fwd_ok(X, Xr, n, kappa)
    ok = (st["flags"] & tla.STAT_CONVERGED) | (st["flags"] & (tla.STAT_FALLBACK | tla.STAT_BREAKDOWN))
    assert np.all(ok != 0)


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_second_pass_fallback_matches_fp64(h, orc, op):
    n = 128
    mats = problem(op, n, 4, 1e2, tag="fb128")
    plan = (0, 16, 1, 4)
    h.set_refine(1e-13, 0)
    try:
        X, ops = solve(h, op, mats, "mixed_f32", plan)
    finally:
        h.set_refine(1e-13, 8)
    st = tla.stat_view(ops.stat)
    assert np.all(st["flags"] & tla.STAT_FALLBACK)
    Y, _ = solve(h, op, mats, "f64", plan)
    assert np.array_equal(X, Y)


SKIP_ABOVE_LDS = ("mixed precision above n = 128 is switched off: its 16-wave kernels with the work "
                  "matrices in the workspace faulted the GPU on their first Lyapunov run (n = 200), cause not found")


@pytest.mark.skip(reason=SKIP_ABOVE_LDS)
@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
@pytest.mark.parametrize("n", [200, 256])
def test_mixed_above_lds_sizes(h, orc, op, n):
    # above the LDS-resident sizes the FP32 work matrices and the FP64
    # solution live in the workspace (16 waves per instance)
    kappa = 1e2
    mats = problem(op, n, 3, kappa, tag="big")
    Xr, ir, eta_fn = oracle_solve(orc, op, mats)
    for prec in ["mixed_f32", "mixed_bf16"]:
        print(f"{op} n={n} {prec}", flush=True)
        X, ops = solve(h, op, mats, prec)
        assert np.all(ops.info.cpu().numpy() == ir)
        st = tla.stat_view(ops.stat)
        assert np.all(st["flags"] & tla.STAT_CONVERGED), st["flags"]
        assert eta_fn(*mats, X).max() <= 1e-12, prec
        assert fwd_ok(X, Xr, n, kappa), prec


@pytest.mark.skip(reason=SKIP_ABOVE_LDS)
@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_mixed_above_lds_sizes_fallback_is_fp64(h, orc, op):
    # no corrections allowed: every instance goes to the FP64 second pass,
    # which is the FP64 kernel of the same size and variant
    n = 200
    mats = problem(op, n, 2, 1e2, tag="bigfb")
    h.set_refine(1e-13, 0)
    try:
        X, ops = solve(h, op, mats, "mixed_f32")
    finally:
        h.set_refine(1e-13, 8)
    st = tla.stat_view(ops.stat)
    assert np.all(st["flags"] & tla.STAT_FALLBACK)
    Y, _ = solve(h, op, mats, "f64")
    assert np.array_equal(X, Y)


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_mixed_workspace_placement_fallback_is_fp64(h, orc, op):
    # placement 3 (work matrices in the workspace) hands unconverged
    # instances to the LDS-resident FP64 kernel of the same variant and waves
    n = 72
    plan = (0, 16, 1, 2, 3)
    mats = problem(op, n, 3, 1e2, tag="wsfb")
    h.set_refine(1e-13, 0)
    try:
        X, ops = solve(h, op, mats, "mixed_f32", plan)
    finally:
        h.set_refine(1e-13, 8)
    assert np.all(tla.stat_view(ops.stat)["flags"] & tla.STAT_FALLBACK)
    Y, _ = solve(h, op, mats, "f64", (0, 16, 1, 2, 0 if op == "potrf" else 1))
    assert np.array_equal(X, Y)
