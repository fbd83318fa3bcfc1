"""GPU parity of the solve with the Cholesky factor (potrs) against the FP64
oracle: uniform and ragged batches, sizes that span several tiles with ragged
tails, many and few right-hand sides, the GPU factor feeding the solve, and
the argument and zero-pivot edge cases."""
import numpy as np
import pytest

import paper_1906_08613_amd as tla
from paper_1906_08613_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 1e-12


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = tla.Handle(0)
    yield hd
    hd.close()


def factors(orc, n, batch, tag):
    A = I.potrf_problem(tag, n, batch)
    X, info = orc.potrf_batch(A)
    assert np.all(info == 0)
    return A, X


def rel(Y, Yr):
    return np.abs(Y - Yr).max() / max(np.abs(Yr).max(), 1e-300)


@pytest.mark.parametrize("n,m", [(1, 1), (5, 3), (16, 16), (40, 7), (64, 16), (64, 70), (100, 33), (128, 1),
                                 (200, 20), (300, 5)])
def test_parity_uniform(h, orc, n, m):
    batch = 4
    A, X = factors(orc, n, batch, f"potrs-{n}")
    B = np.random.default_rng(n * 100 + m).normal(size=(batch, n, m))
    Yr, ir = orc.potrs_batch(X, B)
    dX = tla.to_device_cm(X)
    dB = tla.to_device_rect(B)
    print(f"potrs n={n} m={m}", flush=True)
    ops = tla.potrs(h, dX, dB, n)
    torch.cuda.synchronize()
    assert np.all(ops.info.cpu().numpy() == 0)
    Y = tla.from_device_rect(dB, n)
    for k in range(batch):
        assert rel(Y[k], Yr[k]) <= TOL, (n, m, k, rel(Y[k], Yr[k]))


def test_gpu_factor_then_solve(h, orc):
    n, m, batch = 72, 9, 6
    A = I.potrf_problem("potrs-chain", n, batch)
    dA = tla.to_device_cm(np.triu(A))
    tla.potrf(h, dA, "f64")
    B = np.random.default_rng(5).normal(size=(batch, n, m))
    dB = tla.to_device_rect(B)
    ops = tla.potrs(h, dA, dB, n)
    torch.cuda.synchronize()
    assert np.all(ops.info.cpu().numpy() == 0)
    Y = tla.from_device_rect(dB, n)
    for k in range(batch):
        r = np.abs(A[k] @ Y[k] - B[k]).max() / (np.abs(A[k]).max() * np.abs(Y[k]).max())
        assert r <= 1e-13, r


def test_ragged_sizes_and_edge_cases(h, orc):
    # per-instance n, right-hand sides and leading dimensions in one call
    cases = [(10, 3, 10, 12), (33, 17, 40, 33), (0, 4, 1, 1), (6, 0, 6, 6), (20, 2, 19, 20),
             (20, 2, 20, 19), (9, 5, 9, 9), (70, 40, 70, 80)]
    n_max, m_max = 70, 40
    rng = np.random.default_rng(11)
    X_list, B_list, dev = [], [], []
    for idx, (n, m, ldx, ldb) in enumerate(cases):
        if n > 0:
            A = I.potrf_problem(f"potrs-r{idx}", n, 1)[0]
            X, _ = orc.potrf(A)
        else:
            X = np.zeros((0, 0))
        if idx == 6:
            X = X.copy()
            X[4, 4] = 0.0          # zero pivot: info 5, B untouched
        B = rng.normal(size=(n, m))
        # column-major storage: row j of Xd is column j of X (a leading dimension
        # below n is passed as given, the buffer itself always holds the matrix)
        Xd = np.zeros((max(n, 1), max(ldx, n, 1)))
        Xd[:n, :n] = X.T
        Bd = np.zeros((max(m, 1), max(ldb, n, 1)))
        Bd[:m, :n] = B.T
        X_list.append(X)
        B_list.append(B)
        dev.append((torch.from_numpy(Xd).cuda(), torch.from_numpy(Bd).cuda()))
    cuda = dict(dtype=torch.int32, device="cuda")
    nn = torch.tensor([c[0] for c in cases], **cuda)
    mm = torch.tensor([c[1] for c in cases], **cuda)
    ldx = torch.tensor([c[2] for c in cases], **cuda)
    ldb = torch.tensor([c[3] for c in cases], **cuda)
    px = torch.tensor([d[0].data_ptr() for d in dev], dtype=torch.int64, device="cuda")
    pb = torch.tensor([d[1].data_ptr() for d in dev], dtype=torch.int64, device="cuda")
    info = torch.full((len(cases),), 99, **cuda)
    h.potrs_batched(len(cases), n_max, nn, m_max, mm, px, ldx, pb, ldb, info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 0, 0, 0, -2, -2, 5, 0]
    for idx, (n, m, _, _) in enumerate(cases):
        Y = dev[idx][1].cpu().numpy()[:m, :n].T
        if idx in (0, 1, 7):
            Yr, ir = orc.potrs(X_list[idx], B_list[idx])
            assert ir == 0 and rel(Y, Yr) <= TOL, idx
        elif n > 0 and m > 0:
            assert np.array_equal(Y, B_list[idx]), idx      # rejected or singular: untouched


@pytest.mark.parametrize("n", [1, 17, 64, 100])
def test_inverse_parity(h, orc, n):
    batch = 3
    A, X = factors(orc, n, batch, f"potri-{n}")
    Yr, ir = orc.potri_batch(X)
    dX = tla.to_device_cm(X)
    dY = torch.full((batch, n, n), 7.0, dtype=torch.float64, device="cuda")
    print(f"potri n={n}", flush=True)
    ops = tla.potri(h, dX, dY, n)
    torch.cuda.synchronize()
    assert np.all(ops.info.cpu().numpy() == 0)
    Y = tla.from_device_cm(dY)
    for k in range(batch):
        assert rel(Y[k], Yr[k]) <= TOL, (n, k)
        assert np.abs(A[k] @ Y[k] - np.eye(n)).max() <= 1e-12


def test_inverse_zero_pivot_gives_identity(h, orc):
    n = 20
    A, X = factors(orc, n, 2, "potri-zero")
    X = X.copy()
    X[1, 7, 7] = 0.0
    dX = tla.to_device_cm(X)
    dY = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    ops = tla.potri(h, dX, dY, n)
    torch.cuda.synchronize()
    assert ops.info.cpu().tolist() == [0, 8]
    assert np.array_equal(tla.from_device_cm(dY)[1], np.eye(n))
