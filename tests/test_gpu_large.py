"""Large sizes (n > 128): in-place FP64 kernels over global memory, every
variant, against the oracle (relative Frobenius error 1e-12, inputs with
condition numbers of about 2); the strict lower triangle of the Cholesky
input must stay untouched."""
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


@pytest.mark.parametrize("n", [129, 200, 256])
def test_large_potrf_variants(h, orc, n):
    A = I.potrf_problem("large", n, 2)
    Xr, _ = orc.potrf_batch(A)
    for v in range(3):
        print(f"potrf n={n} v={v}", flush=True)
        h.set_plan("potrf", "f64", (v, 16, 1, 4, 0))
        host = np.triu(A) + np.tril(np.full((n, n), 3.5), -1)
        dA = tla.to_device_cm(host)
        ops = tla.potrf(h, dA)
        torch.cuda.synchronize()
        X = tla.from_device_cm(dA)
        il = np.tril_indices(n, -1)
        assert np.all(X[:, il[0], il[1]] == 3.5)
        assert np.all(ops.info.cpu().numpy() == 0)
        assert rel_err(np.triu(X), Xr).max() <= 1e-12, v
    h.set_plan("potrf", "f64", None)


@pytest.mark.parametrize("n", [129, 256])
def test_large_trsyl_variants(h, orc, n):
    L, U, C = I.trsyl_problem("large", n, 2)
    Xr, _ = orc.trsyl_batch(L, U, C)
    for v in tla.blocked_variants("trsyl"):
        print(f"trsyl n={n} v={v}", flush=True)
        h.set_plan("trsyl", "f64", (v, 16, 1, 4, 0))
        dL, dU, dC = tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)
        ops = tla.trsyl(h, dL, dU, dC)
        torch.cuda.synchronize()
        assert np.all(ops.info.cpu().numpy() == 0)
        assert rel_err(tla.from_device_cm(dC), Xr).max() <= 1e-12, v
    h.set_plan("trsyl", "f64", None)


@pytest.mark.parametrize("n", [129, 256])
def test_large_trlyap_variants(h, orc, n):
    L, S = I.trlyap_problem("large", n, 2)
    Xr, _ = orc.trlyap_batch(L, S)
    for v in tla.blocked_variants("trlyap"):
        print(f"trlyap n={n} v={v}", flush=True)
        h.set_plan("trlyap", "f64", (v, 16, 1, 4, 0))
        dL, dS = tla.to_device_cm(L), tla.to_device_cm(np.tril(S))
        ops = tla.trlyap(h, dL, dS)
        torch.cuda.synchronize()
        X = tla.from_device_cm(dS)
        assert np.all(ops.info.cpu().numpy() == 0)
        assert np.array_equal(X, np.swapaxes(X, 1, 2))
        assert rel_err(X, Xr).max() <= 1e-12, v
    h.set_plan("trlyap", "f64", None)


def test_large_sampled_parity_512(h, orc):
    # the largest sizes: a sample of instances through the oracle
    n = 512
    L, U, C = I.trsyl_problem("large512", n, 4)
    dL, dU, dC = tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)
    tla.trsyl(h, dL, dU, dC)
    torch.cuda.synchronize()
    X = tla.from_device_cm(dC)
    Xr, _ = orc.trsyl_batch(L[:1], U[:1], C[:1])
    assert rel_err(X[:1], Xr).max() <= 1e-12
    assert orc.eta_trsyl_batch(L, U, C, X).max() <= 1e-13
    A = I.potrf_problem("large512", n, 4)
    dA = tla.to_device_cm(np.triu(A))
    tla.potrf(h, dA)
    torch.cuda.synchronize()
    assert orc.eta_potrf_batch(A, np.triu(tla.from_device_cm(dA))).max() <= 1e-13


@pytest.mark.parametrize("op", ["potrf", "trsyl", "trlyap"])
def test_largest_size_1024_against_oracle(h, orc, op):
    # n = 1024 (the largest size of the benchmark's large-size workload), one
    # instance per operation through the default plan, element-wise against
    # the oracle
    n = 1024
    print(f"{op} n={n}", flush=True)
    if op == "potrf":
        A = I.potrf_problem("large1024", n, 1)
        dA = tla.to_device_cm(np.triu(A))
        ops = tla.potrf(h, dA)
        torch.cuda.synchronize()
        X = np.triu(tla.from_device_cm(dA))
        Xr, ir = orc.potrf_batch(A)
        eta = orc.eta_potrf_batch(A, X)
    elif op == "trsyl":
        L, U, C = I.trsyl_problem("large1024", n, 1)
        dL, dU, dC = tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)
        ops = tla.trsyl(h, dL, dU, dC)
        torch.cuda.synchronize()
        X = tla.from_device_cm(dC)
        Xr, ir = orc.trsyl_batch(L, U, C)
        eta = orc.eta_trsyl_batch(L, U, C, X)
    else:
        L, S = I.trlyap_problem("large1024", n, 1)
        dL, dS = tla.to_device_cm(L), tla.to_device_cm(np.tril(S))
        ops = tla.trlyap(h, dL, dS)
        torch.cuda.synchronize()
        X = tla.from_device_cm(dS)
        Xr, ir = orc.trlyap_batch(L, S)
        eta = orc.eta_trlyap_batch(L, S, X)
        assert np.array_equal(X, np.swapaxes(X, 1, 2))
    assert np.all(ops.info.cpu().numpy() == ir) and np.all(ir == 0)
    assert rel_err(X, Xr).max() <= 1e-12
    # element-wise: every entry within 1e-12 of the largest entry of its column
    colmax = np.abs(Xr).max(axis=1, keepdims=True)
    assert np.max(np.abs(X - Xr) / np.where(colmax == 0, 1.0, colmax)) <= 1e-12
    assert eta.max() <= 1e-13


def test_large_potrf_panels_uneven_n_and_failures(h, orc):
    # the left-looking large Cholesky runs by block panels of 128 rows: uneven
    # orders in one batch (below, at and across panel edges), a leading
    # dimension above n, and instances that fail in the first and in a later
    # panel, against the oracle; the strict lower triangle stays untouched
    n_max, ld = 300, 305
    ns = [300, 0, 129, 257, 140, 128, 300, 1]
    batch = len(ns)
    host = np.full((batch, n_max, n_max), 3.5)
    ref = []
    for b, nb in enumerate(ns):
        if nb == 0:
            ref.append(None)
            continue
        A = I.potrf_problem(f"panel-{b}", nb, 1)[0]
        if b == 4:
            A[70, 70] = -1.0          # not positive definite: fails in the first panel
        if b == 6:
            A[200, 200] = -50.0 * nb  # fails in the second panel
        host[b, :nb, :nb] = np.triu(A) + np.tril(np.full((nb, nb), 3.5), -1)
        ref.append(A)
    dA = tla.to_device_cm(host, ld=ld)
    ops = tla.Operands(n_max, dA)
    ops.n.copy_(torch.tensor(ns, dtype=torch.int32))
    h.set_plan("potrf", "f64", (1, 16, 1, 4, 0))
    print("potrf panels uneven", flush=True)
    tla.potrf(h, dA, ops=ops)
    torch.cuda.synchronize()
    h.set_plan("potrf", "f64", None)
    X = tla.from_device_cm(dA, n_max)
    info = ops.info.cpu().numpy()
    for b, nb in enumerate(ns):
        if nb == 0:
            assert info[b] == 0 and np.array_equal(X[b], host[b])
            continue
        Xr, ir = orc.potrf_batch(ref[b][None])
        assert info[b] == ir[0], (b, info[b], ir[0])
        il = np.tril_indices(nb, -1)
        assert np.all(X[b, :nb, :nb][il] == 3.5)
        # nothing outside the instance's n x n block is touched
        assert np.all(X[b, nb:, :] == 3.5) and np.all(X[b, :, nb:] == 3.5)
        if ir[0] == 0:
            assert rel_err(np.triu(X[b, :nb, :nb])[None], Xr).max() <= 1e-12, b


def test_large_trsyl_blocks_uneven_n_and_zero_denominator(h, orc):
    # the tile-wavefront large Sylvester runs as a wavefront over 128 x 128
    # blocks: orders below, at and across block edges in one batch, padded
    # leading dimensions, and an instance with a zero denominator
    n_max, ld = 400, 403
    ns = [400, 0, 129, 385, 200, 1, 256]
    batch = len(ns)
    Lh, Uh, Ch = (np.full((batch, n_max, n_max), 7.0) for _ in range(3))
    for b, nb in enumerate(ns):
        if nb == 0:
            continue
        L, U, C = I.trsyl_problem(f"blocks-{b}", nb, 1)
        if b == 4:
            L[0, 150, 150] = 1.5
            U[0, 170, 170] = -1.5   # l_150,150 + u_170,170 = 0
        Lh[b, :nb, :nb], Uh[b, :nb, :nb], Ch[b, :nb, :nb] = L[0], U[0], C[0]
    dL, dU, dC = (tla.to_device_cm(M, ld=ld) for M in (Lh, Uh, Ch))
    ops = tla.Operands(n_max, dL, dU, dC)
    ops.n.copy_(torch.tensor(ns, dtype=torch.int32))
    print("trsyl blocks uneven", flush=True)
    tla.trsyl(h, dL, dU, dC, ops=ops)
    torch.cuda.synchronize()
    X = tla.from_device_cm(dC, n_max)
    info = ops.info.cpu().numpy()
    for b, nb in enumerate(ns):
        if nb == 0:
            assert info[b] == 0 and np.array_equal(X[b], Ch[b])
            continue
        Xr, ir = orc.trsyl_batch(Lh[b:b + 1, :nb, :nb], Uh[b:b + 1, :nb, :nb], Ch[b:b + 1, :nb, :nb])
        assert info[b] == ir[0], (b, info[b], ir[0])
        assert np.all(X[b, nb:, :] == 7.0) and np.all(X[b, :, nb:] == 7.0)
        if ir[0] == 0:
            assert rel_err(X[b, :nb, :nb][None], Xr).max() <= 1e-12, b
