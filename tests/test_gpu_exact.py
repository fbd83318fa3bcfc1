"""Exact-size kernels (the in-place FP64 kernels compiled at run time for the
call's n): parity with the oracle and with the ahead-of-time kernels, batches
whose instances have other orders than n_max, caching, and the fall-back to
the ahead-of-time kernel when the kernel headers are not found."""
import os

import numpy as np
import pytest

import paper_1906_08613_amd as tla
from paper_1906_08613_amd import inputs as I
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = tla.Handle(0)
    yield hd
    hd.close()


def solve(h, op, mats, n_vec=None):
    n = mats[0].shape[-1]
    if op == "potrf":
        d = tla.to_device_cm(np.triu(mats[0]))
        ops = tla.Operands(n, d)
        if n_vec is not None:
            ops.n.copy_(torch.tensor(n_vec, dtype=torch.int32))
        tla.potrf(h, d, ops=ops)
        out = d
    elif op == "trsyl":
        dL, dU, dC = (tla.to_device_cm(m) for m in mats)
        ops = tla.Operands(n, dL, dU, dC)
        if n_vec is not None:
            ops.n.copy_(torch.tensor(n_vec, dtype=torch.int32))
        tla.trsyl(h, dL, dU, dC, ops=ops)
        out = dC
    else:
        dL, dS = tla.to_device_cm(mats[0]), tla.to_device_cm(np.tril(mats[1]))
        ops = tla.Operands(n, dL, dS)
        if n_vec is not None:
            ops.n.copy_(torch.tensor(n_vec, dtype=torch.int32))
        tla.trlyap(h, dL, dS, ops=ops)
        out = dS
    torch.cuda.synchronize()
    X = tla.from_device_cm(out)
    return (np.triu(X) if op == "potrf" else X), ops.info.cpu().numpy()


def problem(op, n, batch, tag):
    if op == "potrf":
        return (I.potrf_problem(tag, n, batch),)
    if op == "trsyl":
        return I.trsyl_problem(tag, n, batch)
    return I.trlyap_problem(tag, n, batch)


def oracle(orc, op, mats):
    if op == "potrf":
        return orc.potrf_batch(mats[0])
    if op == "trsyl":
        return orc.trsyl_batch(*mats)
    return orc.trlyap_batch(*mats)


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
@pytest.mark.parametrize("n", [1, 5, 16, 17, 33, 64, 100, 128])
def test_exact_size_matches_oracle_and_generic(h, orc, op, n):
    print(f"exact {op} n={n}", flush=True)
    mats = problem(op, n, 6, "exact")
    h.set_exact_size(False)
    Xg, ig = solve(h, op, mats)
    c0, f0 = h.exact_size_stats()
    h.set_exact_size(True)
    try:
        Xe, ie = solve(h, op, mats)
    finally:
        h.set_exact_size(False)
    c1, f1 = h.exact_size_stats()
    assert f1 == f0 and c1 == c0 + 1      # compiled once, for this (op, n)
    Xr, ir = oracle(orc, op, mats)
    assert np.all(ie == ir) and np.all(ig == ir)
    assert rel_err(Xe, Xr).max() <= 1e-12
    assert rel_err(Xe, Xg).max() <= 1e-13
    if op == "trlyap":
        assert np.array_equal(Xe, np.swapaxes(Xe, 1, 2))


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_exact_size_other_orders_in_the_batch(h, orc, op):
    # n_max = 48 but the instances have 48, 9, 31, 47 and 0: the kernel's
    # generic branch solves the others
    n = 48
    mats = problem(op, n, 5, "exact-mix")
    n_vec = [48, 9, 31, 47, 0]
    h.set_exact_size(True)
    try:
        X, info = solve(h, op, mats, n_vec)
        X2, _ = solve(h, op, mats, n_vec)   # cached kernel
    finally:
        h.set_exact_size(False)
    assert np.array_equal(X, X2)
    assert np.all(info == 0)
    for b, m in enumerate(n_vec):
        if m == 0:
            continue
        sub = tuple(M[b:b + 1, :m, :m] for M in mats)
        Xr, _ = oracle(orc, op, sub)
        assert rel_err(X[b:b + 1, :m, :m], Xr).max() <= 1e-12, (b, m)


def test_exact_size_falls_back_without_headers(orc):
    # a handle whose kernel directory does not exist: nothing compiles, the
    # ahead-of-time kernel runs, results unchanged
    old = os.environ.get("TLA_KERNEL_DIR")
    os.environ["TLA_KERNEL_DIR"] = "/nonexistent/tla-kernels"
    try:
        hf = tla.Handle(0)
        hf.set_exact_size(True)
        mats = problem("trsyl", 20, 3, "exact-fb")
        X, info = solve(hf, "trsyl", mats)
        assert hf.exact_size_stats() == (0, 1)
        Xr, ir = oracle(orc, "trsyl", mats)
        assert np.all(info == ir) and rel_err(X, Xr).max() <= 1e-12
        hf.close()
    finally:
        if old is None:
            del os.environ["TLA_KERNEL_DIR"]
        else:
            os.environ["TLA_KERNEL_DIR"] = old


@pytest.mark.parametrize("op", ["potrf", "trsyl"])
def test_exact_size_measured_mode(orc, op):
    # mode 2: the first call of a key times the plan both ways, then keeps
    # the faster; results are the oracle's either way
    hm = tla.Handle(0)
    hm.set_exact_size(2)
    mats = problem(op, 32, 4, "exact-m")
    X1, i1 = solve(hm, op, mats)
    compiled, failed = hm.exact_size_stats()
    assert compiled == 1 and failed == 0     # the timing compiled the exact kernel
    X2, i2 = solve(hm, op, mats)
    assert hm.exact_size_stats() == (1, 0)    # verdict and kernel kept
    assert np.array_equal(X1, X2)
    Xr, ir = oracle(orc, op, mats)
    assert np.all(i1 == ir) and rel_err(X1, Xr).max() <= 1e-12
    hm.close()
