"""GPU parity of the FP32-I/O entry points (tla_spotrf_batched,
tla_strsyl_batched, tla_strlyap_batched) against the CPU oracle, through the
C ABI.

The inputs are rounded to FP32 first; the oracle solves those same FP32
values in FP64, so the only difference left is the GPU's FP32 arithmetic.

Tolerance, from the arithmetic (u = 2^-24, gamma_k = k u / (1 - k u)):
  * trsyl / trlyap: every x_ij is an inner product of length at most 2n + 1
    followed by a division, so the computed X satisfies
    L X + X U = C + dC with |dC| <= gamma_{2n+1} (|L||X| + |X||U| + |C|),
    hence a normwise backward error eta <= gamma_{2n+1};
  * potrf: the standard bound |A - X^T X| <= gamma_{n+1} |X^T||X| with
    ||X||_F^2 = trace(A) <= sqrt(n) ||A||_F gives eta <= gamma_{n+1} sqrt(n).
The blocked variants and the matrix cores change only the summation order,
which these bounds cover.  The inputs have condition numbers of about 2, so
the forward error against the oracle is held to 4 times the same bound.
"""
import numpy as np
import pytest

import paper_1906_08613_amd as tla
from paper_1906_08613_amd import inputs as I
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def gamma(k):
    return k * U32 / (1 - k * U32)


def eta_bound(op, n):
    return gamma(n + 1) * np.sqrt(n) if op == "potrf" else gamma(2 * n + 1)


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = tla.Handle(0)
    yield hd
    hd.close()


def f32(*ms):
    return [np.asarray(m, dtype=np.float32).astype(np.float64) for m in ms]


def dev32(M, ld=None):
    return tla.to_device_cm(M, ld=ld, dtype=np.float32)


SIZES = [1, 2, 5, 16, 17, 31, 64, 65, 100, 128, 129, 200, 256]


def batch_for(n):
    return 24 if n <= 128 else 4


@pytest.mark.parametrize("n", SIZES)
def test_spotrf_matches_oracle(h, orc, n):
    print(f"spotrf n={n}", flush=True)
    (A,) = f32(I.potrf_problem("gpu-s-potrf", n, batch_for(n)))
    dA = dev32(np.triu(A))
    ops = tla.spotrf(h, dA)
    torch.cuda.synchronize()
    X = np.triu(tla.from_device_cm(dA)).astype(np.float64)
    Xr, ir = orc.potrf_batch(A)
    assert np.all(ops.info.cpu().numpy() == 0) and np.all(ir == 0)
    eta = orc.eta_potrf_batch(A, X)
    assert eta.max() <= eta_bound("potrf", n), eta.max()
    assert rel_err(X, Xr).max() <= 4 * eta_bound("potrf", n)


@pytest.mark.parametrize("n", SIZES)
def test_strsyl_matches_oracle(h, orc, n):
    print(f"strsyl n={n}", flush=True)
    L, U, C = f32(*I.trsyl_problem("gpu-s-trsyl", n, batch_for(n)))
    dL, dU, dC = dev32(L), dev32(U), dev32(C)
    ops = tla.strsyl(h, dL, dU, dC)
    torch.cuda.synchronize()
    X = tla.from_device_cm(dC).astype(np.float64)
    Xr, ir = orc.trsyl_batch(L, U, C)
    assert np.all(ops.info.cpu().numpy() == 0) and np.all(ir == 0)
    eta = orc.eta_trsyl_batch(L, U, C, X)
    assert eta.max() <= eta_bound("trsyl", n), eta.max()
    assert rel_err(X, Xr).max() <= 4 * eta_bound("trsyl", n)


@pytest.mark.parametrize("n", SIZES)
def test_strlyap_matches_oracle(h, orc, n):
    print(f"strlyap n={n}", flush=True)
    L, S = f32(*I.trlyap_problem("gpu-s-trlyap", n, batch_for(n)))
    dL, dS = dev32(L), dev32(np.tril(S))
    ops = tla.strlyap(h, dL, dS)
    torch.cuda.synchronize()
    X = tla.from_device_cm(dS).astype(np.float64)
    Xr, ir = orc.trlyap_batch(L, S)
    assert np.all(ops.info.cpu().numpy() == 0) and np.all(ir == 0)
    assert np.array_equal(X, np.swapaxes(X, 1, 2))            # exactly symmetric
    eta = orc.eta_trlyap_batch(L, S, X)
    assert eta.max() <= eta_bound("trlyap", n), eta.max()
    assert rel_err(X, Xr).max() <= 4 * eta_bound("trlyap", n)


def test_single_uneven_n_padded_ld_and_untouched_triangles(h, orc):
    # per-instance n below n_max, ld > n, and the strict lower part of A and
    # everything beyond n left as the caller wrote it
    n_max, batch, ld = 40, 6, 47
    ns = [40, 33, 17, 1, 0, 24]
    (A,) = f32(I.potrf_problem("gpu-s-uneven", n_max, batch))
    host = np.zeros((batch, n_max, ld), dtype=np.float32)
    for b in range(batch):
        host[b, :, :n_max] = A[b].T
        host[b, :, n_max:] = 7.0                                  # beyond the rows of n_max
        for j in range(n_max):
            for i in range(n_max):
                if i > j or i >= ns[b] or j >= ns[b]:
                    host[b, j, i] = -3.0                          # junk outside the referenced part
    dA = torch.from_numpy(host).to("cuda")
    before = host.copy()
    o = tla.Operands(n_max, dA)
    o.n.copy_(torch.tensor(ns, dtype=torch.int32))
    h.spotrf_batched(batch, n_max, o.n, o.ptrs[0], o.lds[0], o.info)
    torch.cuda.synchronize()
    out = dA.cpu().numpy()
    assert o.info.cpu().tolist() == [0] * batch
    for b in range(batch):
        m = ns[b]
        keep = np.ones((n_max, ld), dtype=bool)
        for j in range(m):
            keep[j, :j + 1] = False                               # the upper triangle of the n x n block
        assert np.array_equal(out[b][keep], before[b][keep]), b
        if m:
            X = np.triu(out[b][:m, :m].T.astype(np.float64))
            Xr, _ = orc.potrf(A[b][:m, :m])
            assert rel_err(X[None], Xr[None])[0] <= 4 * eta_bound("potrf", m), b


def test_single_info_codes(h):
    n = 20
    # potrf: a negative pivot at 1-based position 7
    A = np.eye(n, dtype=np.float32) * 4
    A[6, 6] = -1.0
    dA = dev32(A[None])
    o = tla.spotrf(h, dA)
    # trsyl: l_33 + u_jj = 0 for u_jj = 1: first zero denominator at (3, 0)
    L = np.eye(n, dtype=np.float32)
    L[3, 3] = -1.0
    U = np.eye(n, dtype=np.float32)
    C = np.ones((n, n), dtype=np.float32)
    o2 = tla.strsyl(h, dev32(L[None]), dev32(U[None]), dev32(C[None]))
    # trlyap: l_22 + l_00 = 0 at (2, 0)
    Ll = np.eye(n, dtype=np.float32)
    Ll[2, 2] = -1.0
    o3 = tla.strlyap(h, dev32(Ll[None]), dev32(np.eye(n, dtype=np.float32)[None]))
    torch.cuda.synchronize()
    assert o.info.cpu().tolist() == [7]
    assert o2.info.cpu().tolist() == [1 + 3 + 0 * n]
    assert o3.info.cpu().tolist() == [1 + 2 + 0 * n]


def test_single_argument_errors(h):
    lib = tla.lib()
    assert lib.tla_spotrf_batched(None, 1, 4, None, None, None, None) == tla.E_ARG
    assert lib.tla_strsyl_batched(h.h, -1, 4, None, None, None, None, None, None, None, None) == tla.E_ARG
    assert lib.tla_strlyap_batched(h.h, 1, 5000, None, None, None, None, None, None) == tla.E_UNSUPPORTED
    assert lib.tla_spotrf_batched(h.h, 0, 4, None, None, None, None) == tla.OK
