"""Ragged batches (mixed operations and sizes in one persistent launch,
captured as a HIP graph): parity with the oracle per instance, equality with
the uniform kernels of the same plan, graph replay, invalid descriptors."""
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


def make_batch(tag, batch, n_lo=3, n_hi=128):
    ops, ns = I.ragged_mix(tag, batch, n_lo, n_hi)
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


def oracle_one(orc, op, m):
    if op == 0:
        return orc.potrf(m[0])
    if op == 1:
        return orc.trsyl(*m)
    return orc.trlyap(*m)


def eta_one(orc, op, m, X):
    if op == 0:
        return orc.eta_potrf(m[0], np.triu(X))
    if op == 1:
        return orc.eta_trsyl(*m, X)
    return orc.eta_trlyap(*m, X)


@pytest.mark.parametrize("prec", ["f64", "mixed_f32"])
def test_ragged_matches_oracle(h, orc, prec):
    ops, ns, mats = make_batch("rag", 240)
    rb = tla.RaggedBatch(ops, mats)
    tla.ragged(h, rb, prec)
    torch.cuda.synchronize()
    info = rb.info.cpu().numpy()
    assert np.all(info == 0)
    for b in range(rb.batch):
        X = rb.result(b)
        if ops[b] == 0:
            X = np.triu(X)
        Xr, ir = oracle_one(orc, ops[b], mats[b])
        assert eta_one(orc, ops[b], mats[b], X) <= 1e-12, (b, ops[b], ns[b])
        if prec == "f64":
            assert rel_err(X[None], Xr[None])[0] <= 1e-12, (b, ops[b], ns[b])


def test_ragged_equals_uniform_same_plan(h):
    # instances of one op and n through the ragged path and the uniform path
    # with the same variant, tile, engine and waves: identical bits
    for op, n, waves in [(1, 20, 2), (1, 50, 4), (2, 90, 4), (0, 60, 4), (0, 128, 4)]:
        tag = f"eq{op}-{n}"
        if op == 0:
            M = (I.potrf_problem(tag, n, 5),)
        elif op == 1:
            M = I.trsyl_problem(tag, n, 5)
        else:
            M = I.trlyap_problem(tag, n, 5)
        mats = [tuple(np.triu(m[b]) if op == 0 else (np.tril(m[b]) if (op == 2 and k == 1) else m[b])
                      for k, m in enumerate(M)) for b in range(5)]
        rb = tla.RaggedBatch([op] * 5, mats)
        h.set_picker(tla.PICK_DEFAULT)
        tla.ragged(h, rb, "f64")
        name = ["potrf", "trsyl", "trlyap"][op]
        h.set_plan(name, "f64", (0, 16, 1, waves))
        dev = [tla.to_device_cm(np.stack([mm[k] for mm in mats])) for k in range(len(mats[0]))]
        if op == 0:
            tla.potrf(h, dev[0])
        elif op == 1:
            tla.trsyl(h, *dev)
        else:
            tla.trlyap(h, *dev)
        torch.cuda.synchronize()
        h.set_plan(name, "f64", None)
        h.set_picker(tla.PICK_TABLE)
        U = tla.from_device_cm(dev[-1] if op else dev[0])
        for b in range(5):
            R = rb.result(b)
            if op == 0:
                assert np.array_equal(np.triu(R), np.triu(U[b])), (op, n, b)
            else:
                assert np.array_equal(R, U[b]), (op, n, b)


def test_graph_replay_reproduces(h):
    ops, ns, mats = make_batch("replay", 120)
    rb = tla.RaggedBatch(ops, mats)
    pristine = rb.buf.clone()
    tla.ragged(h, rb, "f64")          # captures the graph
    torch.cuda.synchronize()
    first = rb.buf.clone()
    for rep in range(3):              # replays, with eager work in between
        rb.buf.copy_(pristine)
        torch.cuda.synchronize()
        tla.ragged(h, rb, "f64")
        torch.cuda.synchronize()
        assert torch.equal(rb.buf, first), rep
    assert np.all(rb.info.cpu().numpy() == 0)


def test_ragged_invalid_descriptors(h):
    ops = [0, 1, 2, 1, 0]
    mats = [(np.eye(4) * 2,), tuple(m[0] for m in I.trsyl_problem("bad", 6, 1)),
            tuple(m[0] for m in I.trlyap_problem("bad", 5, 1)), tuple(m[0] for m in I.trsyl_problem("bad", 3, 1)),
            (np.eye(7),)]
    rb = tla.RaggedBatch(ops, mats)
    d = rb.desc_host.copy()
    d["op"][1] = 7            # unknown operation
    d["n"][2] = 0             # quick return
    d["ldc"][3] = 2           # ld < n
    d["n"][4] = 9             # n > n_max
    rb.desc = torch.from_numpy(d.view(np.uint8).copy()).to("cuda")
    h.ragged_batched("f64", rb.batch, 8, rb.desc, rb.info, rb.stat)
    torch.cuda.synchronize()
    assert rb.info.cpu().tolist() == [0, -3, 0, -2, -1]
    assert np.allclose(np.triu(rb.result(0)), np.eye(4) * np.sqrt(2))


def test_ragged_maps_uncompiled_variants_to_wavefront(h, tmp_path):
    # a tuning table whose best Sylvester / Lyapunov variants are not compiled
    # into the ragged workers: they run the tile wavefront, bit for bit the
    # same as with the built-in default plans
    ops, ns, mats = make_batch("rag-map", 60)
    path = str(tmp_path / "t.txt")
    lines = ["# op n prec batch variant tile engine waves place seconds"]
    for n in range(4, 129, 4):
        lines.append(f"0 {n} 0 60 0 16 1 2 0 1.0e-5")
        lines.append(f"1 {n} 0 60 7 16 1 2 1 1.0e-5")
        lines.append(f"2 {n} 0 60 3 16 1 2 1 1.0e-5")
    open(path, "w").write("\n".join(lines) + "\n")
    h2 = tla.Handle(0)
    h2.load_table(path)
    h2.set_picker(tla.PICK_TABLE)
    rb_t = tla.RaggedBatch(ops, mats)
    tla.ragged(h2, rb_t, "f64")
    h2.set_picker(tla.PICK_DEFAULT)
    rb_d = tla.RaggedBatch(ops, mats)
    tla.ragged(h2, rb_d, "f64")
    torch.cuda.synchronize()
    assert np.all(rb_t.info.cpu().numpy() == 0)
    for b in range(rb_t.batch):
        assert np.array_equal(rb_t.result(b), rb_d.result(b)), (b, ops[b], ns[b])
    h2.close()


def test_ragged_graph_after_workspace_regrowth(orc):
    # A captured ragged graph bakes in the handle's workspace address.  A
    # larger uniform mixed call reallocates that workspace; the next ragged
    # call with the same arguments must not replay the old graph (it would
    # write freed memory) but capture a new one: its results still match the
    # oracle.  A refinement-setting change likewise forces a new capture.
    hd = tla.Handle(0)
    hd.set_picker(tla.PICK_DEFAULT)
    ops, ns, mats = make_batch("regrow", 96)
    rb = tla.RaggedBatch(ops, mats)
    pristine = rb.buf.clone()

    def check_ragged(tag):
        torch.cuda.synchronize()
        assert np.all(rb.info.cpu().numpy() == 0), tag
        for b in range(rb.batch):
            X = rb.result(b)
            if ops[b] == 0:
                X = np.triu(X)
            assert eta_one(orc, ops[b], mats[b], X) <= 1e-12, (tag, b, ops[b], ns[b])

    tla.ragged(hd, rb, "mixed_f32")              # captures, small workspace
    check_ragged("first")
    # uniform mixed Cholesky at n = 128 over 8192 instances: its workspace
    # (FP64 solution and an FP32 matrix per instance) is larger than the
    # ragged call's, so the handle reallocates it
    n, batch = 128, 8192
    g = torch.Generator(device="cuda").manual_seed(7)
    B = torch.rand((batch, n, n), generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    A = B.transpose(1, 2).contiguous() @ B + n * torch.eye(n, device="cuda", dtype=torch.float64)
    A0 = A[:4].cpu().numpy()                     # symmetric: [b, j, i] == [b, i, j]
    Ad = A.contiguous()
    o = tla.potrf(hd, Ad, "mixed_f32")
    torch.cuda.synchronize()
    assert np.all(o.info.cpu().numpy() == 0)
    Xg = np.triu(tla.from_device_cm(Ad[:4]))
    for b in range(4):
        assert orc.eta_potrf(A0[b], Xg[b]) <= 1e-12, b
    del A, B, Ad
    rb.buf.copy_(pristine)
    rb.info.zero_()
    tla.ragged(hd, rb, "mixed_f32")              # same arguments: must recapture
    check_ragged("after regrowth")
    rb.buf.copy_(pristine)
    rb.info.zero_()
    hd.set_refine(1e-13, 6)                      # new refinement settings: recapture
    tla.ragged(hd, rb, "mixed_f32")
    check_ragged("after set_refine")
    hd.close()
