"""The allocation-free ragged entry point (tla_ragged_batched_noalloc)
against the allocating one (tla_ragged_batched), through the C ABI: the same
class workers and per-instance bodies, so the outputs must agree bit for bit,
on two calls in a row, the second with a smaller batch (the shared scratch
array keeps the first call's contents).  Also its limits and a sample against
the oracle."""
import numpy as np
import pytest

import paper_1906_08613_amd as tla
from paper_1906_08613_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hd = tla.Handle(0)
    yield hd
    hd.close()


def make_mats(tag, batch):
    ops, ns = I.ragged_mix(tag, batch, 3, 128)
    mats = []
    for b, (op, n) in enumerate(zip(ops, ns)):
        if op == 0:
            mats.append((np.triu(I.potrf_problem(tag, int(n), 1, start=b)[0]),))
        elif op == 1:
            mats.append(tuple(m[0] for m in I.trsyl_problem(tag, int(n), 1, start=b)))
        else:
            L, S = I.trlyap_problem(tag, int(n), 1, start=b)
            mats.append((L[0], np.tril(S[0])))
    return ops, ns, mats


def run_both(h, tag, batch):
    ops, ns, mats = make_mats(tag, batch)
    print(f"no-alloc ragged {tag} batch={batch}", flush=True)
    ref = tla.RaggedBatch(ops, mats)
    tla.ragged(h, ref, "f64")
    got = tla.RaggedBatch(ops, mats)
    tla.ragged_noalloc(h, got, "f64")
    torch.cuda.synchronize()
    return ops, ns, mats, ref, got


def test_noalloc_equals_allocating_path_twice(h, orc):
    # first call, then a smaller one: the second must not see the first's queue
    for tag, batch in (("na-big", 700), ("na-small", 90)):
        ops, ns, mats, ref, got = run_both(h, tag, batch)
        assert torch.equal(ref.info, got.info)
        assert np.all(got.info.cpu().numpy() == 0)
        assert torch.equal(ref.buf, got.buf), tag
        # and a sample against the oracle, to the FP64 tolerance
        for b in range(0, batch, max(1, batch // 12)):
            X = got.result(b)
            if ops[b] == 0:
                Xr, _ = orc.potrf(mats[b][0])
                X = np.triu(X)
            elif ops[b] == 1:
                Xr, _ = orc.trsyl(*mats[b])
            else:
                Xr, _ = orc.trlyap(*mats[b])
            err = np.linalg.norm(X - Xr) / np.linalg.norm(Xr)
            assert err <= 1e-12, (tag, b, ops[b], ns[b], err)


def test_noalloc_limits(h):
    ops, ns, mats = make_mats("na-lim", 4)
    rb = tla.RaggedBatch(ops, mats)
    # above the scratch array's maximum batch: rejected before any work
    with pytest.raises(tla.TlaError):
        h.ragged_batched_noalloc("f64", (1 << 20) + 1, rb.n_max, rb.desc, rb.info, rb.stat)
    # the mixed precisions need the handle's workspace
    with pytest.raises(tla.TlaError):
        tla.ragged_noalloc(h, rb, "mixed_f32")
    # above the LDS-resident maximum n
    with pytest.raises(tla.TlaError):
        tla.ragged_noalloc(h, rb, "f64", n_max=129)
    # the input is still untouched and the valid call works afterwards
    tla.ragged_noalloc(h, rb, "f64")
    torch.cuda.synchronize()
    assert np.all(rb.info.cpu().numpy() == 0)
