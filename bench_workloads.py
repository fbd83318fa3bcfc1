"""The benchmark's secondary workloads (one JSON line each), run with
python bench.py --workload {potrf16,sweep,ragged,large,planner,potrs,variants,plan,exact,general,peaks}.

potrf16 : FP64 Cholesky, 1024 instances at n = 16, replayed many times inside
          one HIP graph (the batch is too small to fill the GPU by itself).
sweep   : FP64 Sylvester and Lyapunov, n = 4, 8, ..., 128, 4096 instances each,
          tuned plans.
ragged  : 65536 mixed instances (40% Cholesky, 30% Sylvester, 30% Lyapunov),
          n uniform on {3..128}, FP64 and mixed, one graph-captured call.
large   : 256 instances at n = 256, 512, 1024, FP64, tuned variants.
planner : autotuner timings for n = 3..128 and the MLP trained on them;
          regret of the learned picker on held-out n against the measured best.
potrs   : solve with the Cholesky factor, FP64, n = 64, 16 right-hand sides,
          8192 instances (the factor's consumer), with the CPU oracle on a sample.
variants: best time of each blocked-algorithm variant (over tiles, engines,
          waves and placements), FP64, n = 16 .. 1024: 4096 instances up to
          n = 128, 256 above (one in-place plan per variant there).
exact   : exact-size kernels (compiled at run time for each n) against the
          ahead-of-time kernels of the same plan, FP64, n = 4..128.
peaks   : re-measured HBM and FP64 product ceilings, and the cold / hot regimes of
          FP64 trsyl at n = 64.
general : general Sylvester and Lyapunov equations through the Schur front
          end (Schur forms, transforms, triangular solve), FP64 and mixed,
          n = 16, 32, 64, 8192 instances.
plan    : one operation (first of --ops) at --n, --batch, --prec with the plan
          given by --plan, timed by the library's own timer (for profiling
          one kernel).
All inputs are synthetic and seeded (paper_1906_08613_amd.inputs); results
are checked against the CPU oracle on a sample.
"""
from __future__ import annotations

import json
import time

import numpy as np


def _flops(op, n):
    return n ** 3 / 3.0 if op == 0 else 2.0 * n ** 3


def _bytes(op, n):
    if op == 0:
        return n * (n + 1) * 8
    if op == 1:
        return (n * (n + 1) + 2 * n * n) * 8
    return (n * (n + 1) + n * n) * 8


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def potrf16(a):
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    n, batch, reps = 16, 1024, 200
    h = tla.Handle(0)
    A = I.potrf_problem("cfg0", n, batch)
    # one input copy per launch of the graph, so that every launch factors the
    # pristine matrices (an in-place launch would otherwise re-factor the
    # previous launch's output); all copies are restored outside the timed region
    pristine = tla.to_device_cm(np.triu(A))
    copies = pristine.unsqueeze(0).repeat(reps, 1, 1, 1).contiguous()
    ops = [tla.Operands(n, copies[r]) for r in range(reps)]
    s = torch.cuda.Stream()
    h.set_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        o = ops[0]
        h.potrf_batched("f64", batch, n, o.n, o.ptrs[0], o.lds[0], o.info, o.stat)  # warm-up
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            for o in ops:
                h.potrf_batched("f64", batch, n, o.n, o.ptrs[0], o.lds[0], o.info, o.stat)
    times = []
    for _ in range(5):
        copies.copy_(pristine.unsqueeze(0).expand_as(copies))
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        # the graph replays on the current stream: the events bracket it there
        with torch.cuda.stream(s):
            e0.record()
            g.replay()
            e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3 / reps)
    # the last replay's outputs: every copy holds one launch's factor
    X0 = np.triu(tla.from_device_cm(copies[0]))
    Xl = np.triu(tla.from_device_cm(copies[reps - 1]))
    Xr, _ = oracle.potrf_batch(A[:64])
    t = float(np.median(times))
    t0 = time.perf_counter()
    oracle.potrf_batch(A)
    tc = time.perf_counter() - t0
    print(json.dumps({"workload": "potrf f64 n=16 x1024 (graph of 200 launches, each on its own pristine copy)",
                      "solves_per_s": batch / t,
                      "gflops": batch * _flops(0, n) / t / 1e9, "gbs": batch * _bytes(0, n) / t / 1e9,
                      "us_per_launch": t * 1e6,
                      "fwd_err_max": float(max(oracle.forward_error(X0[:64], Xr).max(),
                                               oracle.forward_error(Xl[:64], Xr).max())),
                      "info_nonzero": int(sum(int((o.info != 0).sum()) for o in (ops[0], ops[-1]))),
                      "cpu_oracle_solves_per_s": batch / tc, "cpu_threads": oracle.max_threads()}))


def sweep(a):
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    h = tla.Handle(0)
    batch = 4096
    sizes = list(range(4, 129, 4))
    # the autotuner's plan for every size (outside the timed launches)
    h.tune(["trsyl", "trlyap"], sizes, ["f64"], batch=batch, reps=2)
    for opname, op in (("trsyl", 1), ("trlyap", 2)):
        for n in sizes:
            if op == 1:
                L, U, C = I.trsyl_problem("cfg1", n, batch)
                dL, dU, dC = tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)
                ops = tla.Operands(n, dL, dU, dC)
                run = lambda: h.trsyl_batched("f64", batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1],
                                              ops.lds[1], ops.ptrs[2], ops.lds[2], ops.info)
                pristine, work = dC.clone(), dC
            else:
                L, S = I.trlyap_problem("cfg1", n, batch)
                dL, dS = tla.to_device_cm(L), tla.to_device_cm(np.tril(S))
                ops = tla.Operands(n, dL, dS)
                run = lambda: h.trlyap_batched("f64", batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1],
                                               ops.lds[1], ops.info)
                pristine, work = dS.clone(), dS
            ts = []
            for _ in range(4):
                work.copy_(pristine)
                torch.cuda.synchronize()
                e0, e1 = _events(torch)
                e0.record()
                run()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            t = float(np.median(ts[1:]))
            X = tla.from_device_cm(work)[:8]
            if op == 1:
                Xr, _ = oracle.trsyl_batch(L[:8], U[:8], C[:8])
            else:
                Xr, _ = oracle.trlyap_batch(L[:8], S[:8])
            print(json.dumps({"workload": f"{opname} f64 n={n} x{batch}", "n": n,
                              "solves_per_s": batch / t, "gflops": batch * _flops(op, n) / t / 1e9,
                              "gbs": batch * _bytes(op, n) / t / 1e9, "ms": t * 1e3,
                              "plan": list(h.get_plan(opname, n, "f64", batch).astuple()),
                              "fwd_err_max": float(oracle.forward_error(X, Xr).max())}), flush=True)


def _ragged_batch(tag, batch):
    from paper_1906_08613_amd import inputs as I
    ops, ns = I.ragged_mix(tag, batch)
    mats = [None] * batch
    for op in range(3):
        for n in np.unique(ns[ops == op]):
            idx = np.nonzero((ops == op) & (ns == n))[0]
            n = int(n)
            if op == 0:
                A = I.potrf_problem(tag + "p", n, len(idx))
                for k, b in enumerate(idx):
                    mats[b] = (np.triu(A[k]),)
            elif op == 1:
                L, U, C = I.trsyl_problem(tag + "s", n, len(idx))
                for k, b in enumerate(idx):
                    mats[b] = (L[k], U[k], C[k])
            else:
                L, S = I.trlyap_problem(tag + "l", n, len(idx))
                for k, b in enumerate(idx):
                    mats[b] = (L[k], np.tril(S[k]))
    return ops, ns, mats


def ragged(a):
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    batch = 65536
    ops, ns, mats = _ragged_batch("cfg3", batch)
    rb = tla.RaggedBatch(ops, mats)
    pristine = rb.buf.clone()
    h = tla.Handle(0)
    flops = sum(_flops(int(o), int(n)) for o, n in zip(ops, ns))
    nbytes = sum(_bytes(int(o), int(n)) for o, n in zip(ops, ns))
    for prec in ("f64", "mixed_f32"):
        ts = []
        for rep in range(4):
            rb.buf.copy_(pristine)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record()
            tla.ragged(h, rb, prec)          # first call captures the graph, later ones replay it
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        t = float(np.median(ts[1:]))
        idx = np.linspace(0, batch - 1, 48).astype(int)
        worst = 0.0
        for b in idx:
            X = rb.result(b)
            m = mats[b]
            if ops[b] == 0:
                e = oracle.eta_potrf(m[0], np.triu(X))
            elif ops[b] == 1:
                e = oracle.eta_trsyl(*m, X)
            else:
                e = oracle.eta_trlyap(*m, X)
            worst = max(worst, e)
        print(json.dumps({"workload": f"ragged {batch} (40/30/30 potrf/trsyl/trlyap, n~U{{3..128}}) prec={prec}",
                          "solves_per_s": batch / t, "gflops_nominal": flops / t / 1e9, "gbs": nbytes / t / 1e9,
                          "ms": t * 1e3, "first_call_ms_incl_capture": ts[0] * 1e3,
                          "eta_max_sample": worst,
                          "info_nonzero": int((rb.info.cpu().numpy() != 0).sum())}), flush=True)
    sub = [mats[b] for b in range(512)]
    t0 = time.perf_counter()
    for b, m in enumerate(sub):
        if ops[b] == 0:
            oracle.potrf(m[0])
        elif ops[b] == 1:
            oracle.trsyl(*m)
        else:
            oracle.trlyap(*m)
    tc = time.perf_counter() - t0
    print(json.dumps({"workload": "ragged cpu oracle sample", "instances": 512, "solves_per_s": 512 / tc,
                      "threads": 1}))


def large(a):
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    h = tla.Handle(0)
    batch = 256
    # the autotuner's variant for every (op, n): at these sizes only the variant differs
    h.tune(["potrf", "trsyl", "trlyap"], [256, 512, 1024], ["f64"], batch=batch, reps=2)
    for n in (256, 512, 1024):
        for opname, op in (("potrf", 0), ("trsyl", 1), ("trlyap", 2)):
            if op == 0:
                A = I.potrf_problem("cfg4", n, batch)
                d = [tla.to_device_cm(np.triu(A))]
                o = tla.Operands(n, *d)
                run = lambda: h.potrf_batched("f64", batch, n, o.n, o.ptrs[0], o.lds[0], o.info)
            elif op == 1:
                L, U, C = I.trsyl_problem("cfg4", n, batch)
                d = [tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)]
                o = tla.Operands(n, *d)
                run = lambda: h.trsyl_batched("f64", batch, n, o.n, o.ptrs[0], o.lds[0], o.ptrs[1], o.lds[1],
                                              o.ptrs[2], o.lds[2], o.info)
            else:
                L, S = I.trlyap_problem("cfg4", n, batch)
                d = [tla.to_device_cm(L), tla.to_device_cm(np.tril(S))]
                o = tla.Operands(n, *d)
                run = lambda: h.trlyap_batched("f64", batch, n, o.n, o.ptrs[0], o.lds[0], o.ptrs[1], o.lds[1],
                                               o.info)
            work = d[-1]
            pristine = work.clone()
            ts = []
            for _ in range(2):
                work.copy_(pristine)
                torch.cuda.synchronize()
                e0, e1 = _events(torch)
                e0.record()
                run()
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1) * 1e-3)
            t = min(ts)
            X = tla.from_device_cm(work[:1])
            if op == 0:
                eta = oracle.eta_potrf_batch(A[:1], np.triu(X))
            elif op == 1:
                eta = oracle.eta_trsyl_batch(L[:1], U[:1], C[:1], X)
            else:
                eta = oracle.eta_trlyap_batch(L[:1], S[:1], X)
            print(json.dumps({"workload": f"{opname} f64 n={n} x{batch}", "solves_per_s": batch / t,
                              "gflops": batch * _flops(op, n) / t / 1e9,
                              "frac_fp64_peak": batch * _flops(op, n) / t / 78.6e12,
                              "ms": t * 1e3, "eta_sample": float(eta.max())}), flush=True)
            del d, o, work, pristine
            torch.cuda.empty_cache()


def planner(a):
    import os
    import tempfile
    import paper_1906_08613_amd as tla
    h = tla.Handle(0)
    ops = ["potrf", "trsyl", "trlyap"]
    ns = list(range(3, 129, 5))
    # above n = 128 only FP64 exists and only the variant selects a kernel
    ns_large = [160, 192, 224, 288, 320, 384, 448]
    t0 = time.perf_counter()
    h.tune(ops, ns, ["f64", "mixed_f32"], batch=1024, reps=2)
    h.tune(ops, ns_large, ["f64"], batch=256, reps=2)
    t_tune = time.perf_counter() - t0
    path = os.path.join(tempfile.mkdtemp(), "table.txt")
    h.save_table(path)

    def load(p):
        rec = np.loadtxt(p, comments="#")
        return {(int(r[0]), int(r[1]), int(r[2]), tuple(int(x) for x in r[4:9])): r[9] for r in rec}

    times = load(path)
    held = [n for n in ns if n % 7 == 0]
    t0 = time.perf_counter()
    hm = tla.Handle(0)
    hm.load_table(path)
    loss = hm.mlp_train(epochs=3000, lr=3e-3, seed=5, exclude_mod=7)
    t_train = time.perf_counter() - t0
    hu = tla.Handle(0)
    hu.load_table(path)
    hu.mlp_train(epochs=0, lr=3e-3, seed=5, exclude_mod=7)
    # the large evaluation sizes, never seen in training: measured separately
    eval_large = [256, 512, 1024]
    he = tla.Handle(0)
    he.tune(ops, eval_large, ["f64"], batch=256, reps=2)
    path_e = os.path.join(tempfile.mkdtemp(), "table_large.txt")
    he.save_table(path_e)
    times_e = load(path_e)

    def regret(handle, mode, table, sizes, precs, batch, by_variant=False):
        handle.set_picker(mode)
        out = []
        for op in range(3):
            for prec in precs:
                for n in sizes:
                    cand = {k[3]: v for k, v in table.items() if k[0] == op and k[1] == n and k[2] == prec}
                    best = min(cand.values())
                    pick = handle.get_plan(op, n, prec, batch).astuple()
                    if by_variant:  # one measured plan per variant above n = 128
                        t = min(v for k, v in cand.items() if k[0] == pick[0])
                    else:
                        t = cand.get(tuple(pick), np.inf)
                    out.append(t / best - 1.0)
        return np.array(out)

    hm.set_picker_judge(0.0, 0)
    r_mlp = regret(hm, tla.PICK_MLP, times, held, (0, 1), 1024)
    r_mlp_large = regret(hm, tla.PICK_MLP, times_e, eval_large, (0,), 256, True)
    hm.set_picker_judge(0.10, 4)
    r_judged = regret(hm, tla.PICK_MLP, times, held, (0, 1), 1024)
    r_judged_large = regret(hm, tla.PICK_MLP, times_e, eval_large, (0,), 256, True)
    judged, mispredicted = hm.picker_judge_stats()
    r_untrained = regret(hu, tla.PICK_MLP, times, held, (0, 1), 1024)
    r_default = regret(hu, tla.PICK_DEFAULT, times, held, (0, 1), 1024)
    r_default_large = regret(hu, tla.PICK_DEFAULT, times_e, eval_large, (0,), 256, True)
    print(json.dumps({"workload": "planner: autotuner n=3..128 step 5 (f64 + mixed_f32, batch 1024) and "
                                  "n=160..448 (f64, batch 256); MLP trained without n % 7 == 0; evaluated on the "
                                  "held-out n and on n = 256, 512, 1024 (f64, batch 256, not trained on)",
                      "held_out_n": held, "records": len(times), "tune_seconds": t_tune, "train_seconds": t_train,
                      "train_loss": loss,
                      "regret_mlp_mean": float(r_mlp.mean()), "regret_mlp_max": float(r_mlp.max()),
                      "regret_mlp_judged_mean": float(r_judged.mean()),
                      "regret_mlp_judged_max": float(r_judged.max()),
                      "judge_timed_picks": judged, "judge_mispredictions": mispredicted,
                      "regret_untrained_mean": float(r_untrained.mean()),
                      "regret_default_plan_mean": float(r_default.mean()),
                      "large_n": eval_large,
                      "regret_mlp_large": [round(float(x), 4) for x in r_mlp_large],
                      "regret_mlp_judged_large": [round(float(x), 4) for x in r_judged_large],
                      "regret_default_plan_large": [round(float(x), 4) for x in r_default_large]}))


def exact(a):
    """Exact-size kernels (compiled at run time for each n) against the
    ahead-of-time in-place kernels of the same plan, FP64."""
    import torch
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    h = tla.Handle(0)
    batch = 4096
    rows = []
    for op in ("potrf", "trsyl", "trlyap"):
        for n in (4, 8, 12, 16, 24, 32, 48, 64, 96, 128):
            if op == "potrf":
                mats = (np.triu(I.potrf_problem("exact", n, batch)),)
            elif op == "trsyl":
                mats = I.trsyl_problem("exact", n, batch)
            else:
                L, S = I.trlyap_problem("exact", n, batch)
                mats = (L, np.tril(S))
            dev = [tla.to_device_cm(m) for m in mats]
            pristine = dev[-1].clone()
            ops = tla.Operands(n, *dev)

            def run():
                dev[-1].copy_(pristine)
                if op == "potrf":
                    h.potrf_batched("f64", batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.info, ops.stat)
                elif op == "trsyl":
                    h.trsyl_batched("f64", batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                                    ops.ptrs[2], ops.lds[2], ops.info, ops.stat)
                else:
                    h.trlyap_batched("f64", batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                                     ops.info, ops.stat)

            def timed(reps=7):
                run()
                torch.cuda.synchronize()
                ts, tc = [], []
                for _ in range(reps):
                    e0, e1 = _events(torch)
                    e2, e3 = _events(torch)
                    e2.record()
                    dev[-1].copy_(pristine)
                    e3.record()
                    e0.record()
                    run()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e2.elapsed_time(e1) * 1e-3)
                    tc.append(e2.elapsed_time(e3) * 1e-3)
                return float(np.median(ts) - np.median(tc))

            h.set_exact_size(False)
            tg = timed()
            h.set_exact_size(True)
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            t_compile = time.perf_counter() - t0
            te = timed()
            h.set_exact_size(False)
            rows.append({"op": op, "n": n, "generic_us": round(tg * 1e6, 1), "exact_us": round(te * 1e6, 1),
                         "speedup": round(tg / te, 3), "first_call_s": round(t_compile, 2)})
            print(json.dumps(rows[-1]), flush=True)
    print(json.dumps({"workload": f"exact-size kernels vs ahead-of-time, FP64, {batch} instances, default plans",
                      "rows": rows, "compiled": h.exact_size_stats()[0]}))


def general(a):
    """General Sylvester / Lyapunov through the Schur front end, FP64 and
    mixed triangular solves, n = 16, 32, 64, 8192 instances each."""
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    h = tla.Handle(0)
    batch = a.batch if a.batch else 8192
    for op in ("gesyl", "gelyap"):
        for n in (16, 32, 64):
            if op == "gesyl":
                A, B, C = I.gesyl_problem("general", n, batch)
                dev = [tla.to_device_cm(A), tla.to_device_cm(B), tla.to_device_cm(C)]
            else:
                A, S = I.gelyap_problem("general", n, batch)
                dev = [tla.to_device_cm(A), tla.to_device_cm(np.tril(S))]
            pristine = dev[-1].clone()
            ops = tla.Operands(n, *dev)
            for prec in ("f64", "mixed_f32"):
                def run():
                    if op == "gesyl":
                        tla.gesyl(h, dev[0], dev[1], dev[2], prec, ops)
                    else:
                        tla.gelyap(h, dev[0], dev[1], prec, ops)
                ts = []
                for _ in range(4):
                    dev[-1].copy_(pristine)
                    torch.cuda.synchronize()
                    e0, e1 = _events(torch)
                    e0.record()
                    run()
                    e1.record()
                    torch.cuda.synchronize()
                    ts.append(e0.elapsed_time(e1) * 1e-3)
                t = float(np.median(ts[1:]))
                info = ops.info.cpu().numpy()
                X = tla.from_device_cm(dev[-1][:64])
                if op == "gesyl":
                    eta = float(oracle.eta_gesyl_batch(A[:64], B[:64], C[:64], X).max())
                else:
                    eta = float(oracle.eta_gelyap_batch(A[:64], S[:64], X).max())
                row = {"workload": f"{op} {prec} n={n} x{batch}", "solves_per_s": batch / t, "ms": t * 1e3,
                       "flagged": int((info != 0).sum()), "eta_max_sample64": eta}
                if prec == "f64":
                    # host references on a sample: the oracle (Kronecker system,
                    # O(n^6)) where it finishes, and SciPy's Schur-based solver
                    import scipy.linalg as sl
                    k = 4 if n <= 32 else 1
                    t0 = time.perf_counter()
                    if op == "gesyl":
                        oracle.gesyl_batch(A[:k], B[:k], C[:k])
                    else:
                        oracle.gelyap_batch(A[:k], S[:k])
                    row["cpu_oracle_solves_per_s"] = k / (time.perf_counter() - t0)
                    k = 64
                    t0 = time.perf_counter()
                    for b in range(k):
                        if op == "gesyl":
                            sl.solve_sylvester(A[b], B[b], C[b])
                        else:
                            sl.solve_continuous_lyapunov(A[b], S[b])
                    row["cpu_scipy_1thread_solves_per_s"] = k / (time.perf_counter() - t0)
                print(json.dumps(row), flush=True)
    h.close()


def peaks(a):
    """Re-measured ceilings of this GPU and the cold / hot regimes of the
    headline Sylvester solve: HBM streaming rates (device copy, read-only
    reduction), the library's batched FP64 product rate, and FP64 trsyl at
    n = 64 with inputs rotating through sets larger than the caches (cold)
    versus a small batch re-solved in the same buffers (hot)."""
    import torch
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = _events(torch)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts))

    nbytes = 4 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    t = timed(lambda: dst.copy_(src))
    copy_gbs = 2 * nbytes / t / 1e9
    t = timed(lambda: src.sum())
    read_gbs = nbytes / t / 1e9
    del src, dst
    A = torch.randn(64, 1024, 1024, dtype=torch.float64, device="cuda")
    B = torch.randn(64, 1024, 1024, dtype=torch.float64, device="cuda")
    t = timed(lambda: torch.bmm(A, B))
    gemm_tfs = 2 * 64 * 1024 ** 3 / t / 1e12
    del A, B
    print(json.dumps({"workload": "peaks", "hbm_copy_gbs": copy_gbs, "hbm_read_gbs": read_gbs,
                      "hbm_datasheet_gbs": 8000.0, "fp64_library_gemm_tfs": gemm_tfs,
                      "fp64_datasheet_tfs": 78.6}), flush=True)

    # cold / hot: FP64 trsyl, n = 64, in place on C (restored outside the timed region)
    h = tla.Handle(0)
    n = 64

    def setup(batch, tag):
        L, U, C = I.trsyl_problem(tag, n, batch)
        dev = [tla.to_device_cm(L), tla.to_device_cm(U), tla.to_device_cm(C)]
        return dev, dev[2].clone(), tla.Operands(n, *dev)

    def launch(dev, ops):
        h.trsyl_batched("f64", ops.batch, n, ops.n, ops.ptrs[0], ops.lds[0], ops.ptrs[1], ops.lds[1],
                        ops.ptrs[2], ops.lds[2], ops.info, ops.stat)

    def per_instance(sets, reps):
        ts = []
        for r in range(reps):
            dev, pristine, ops = sets[r % len(sets)]
            dev[2].copy_(pristine)
            torch.cuda.synchronize()
            e0, e1 = _events(torch)
            e0.record()
            launch(dev, ops)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3 / ops.batch)
        return float(np.median(ts[1:]))

    cold_sets = [setup(8192, f"cold{k}") for k in range(4)]   # 4 x 0.8 GB of operands
    cold = per_instance(cold_sets, 9)
    del cold_sets
    # hot: a batch whose operands fit the 256 MB MALL (2048 x 99 KB), re-solved
    # in the same buffers; it fills only part of the GPU (five resident
    # instances per SIMD need 5120), so its per-instance time also carries the
    # lower occupancy
    hot_set = [setup(2048, "hot")]
    hot = per_instance(hot_set, 9)
    cold_small = [setup(2048, f"coldsmall{k}") for k in range(8)]  # 8 x 200 MB rotating
    cold2 = per_instance(cold_small, 9)
    by = (n * (n + 1) + 2 * n * n) * 8
    print(json.dumps({"workload": "trsyl f64 n=64: cold (rotating sets larger than the caches) vs hot (same buffers)",
                      "cold_8192_us_per_instance": cold * 1e6, "cold_8192_gbs": by / cold / 1e9,
                      "cold_2048_us_per_instance": cold2 * 1e6, "hot_2048_us_per_instance": hot * 1e6,
                      "cold_2048_gbs": by / cold2 / 1e9, "hot_2048_gbs": by / hot / 1e9}), flush=True)
    h.close()


def potrs(a):
    import torch
    import oracle
    import paper_1906_08613_amd as tla
    from paper_1906_08613_amd import inputs as I
    n, m, batch = 64, 16, 8192
    h = tla.Handle(0)
    A = I.potrf_problem("potrs", n, batch)
    dX = tla.to_device_cm(np.triu(A))
    tla.potrf(h, dX, "f64")
    X = tla.from_device_cm(dX)
    B = np.random.default_rng(64).normal(size=(batch, n, m))
    dB = tla.to_device_rect(B)
    pristine = dB.clone()
    ox, ob = tla.Operands(n, dX), tla.Operands(n, dB)
    nrhs = torch.full((batch,), m, dtype=torch.int32, device="cuda")
    ts = []
    for _ in range(6):
        dB.copy_(pristine)
        torch.cuda.synchronize()
        e0, e1 = _events(torch)
        e0.record()
        h.potrs_batched(batch, n, ox.n, m, nrhs, ox.ptrs[0], ox.lds[0], ob.ptrs[0], ob.lds[0], ob.info)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    t = float(np.median(ts[1:]))
    Y = tla.from_device_rect(dB[:8], n)
    Yr, _ = oracle.potrs_batch(np.triu(X[:8]), B[:8])
    fl = 2.0 * n * n * m                      # two triangular solves with m right-hand sides
    by = (n * (n + 1) // 2 + 2 * n * m) * 8   # upper factor read, B read and written
    sample = 1024
    t0 = time.perf_counter()
    oracle.potrs_batch(np.triu(X[:sample]), B[:sample], oracle.max_threads())
    tc = time.perf_counter() - t0
    print(json.dumps({"workload": f"potrs f64 n={n} nrhs={m} x{batch}", "solves_per_s": batch / t,
                      "gflops": batch * fl / t / 1e9, "gbs": batch * by / t / 1e9,
                      "hbm_frac": batch * by / t / 8e12, "ms": t * 1e3,
                      "fwd_err_max": float(np.abs(Y - Yr).max() / np.abs(Yr).max()),
                      "cpu_oracle_solves_per_s": sample / tc, "cpu_threads": oracle.max_threads()}))
    h.close()


def plan(a):
    import torch  # noqa: F401  (device context for the library)
    import paper_1906_08613_amd as tla
    op = a.ops.split(",")[0]
    p = tuple(int(x) for x in (a.plan or "0,16,1,4,0").split(","))
    h = tla.Handle(0)
    t = h.time_plan(op, a.n, a.prec, a.batch, p, reps=3)
    fl = {"potrf": a.n ** 3 / 3.0}.get(op, 2.0 * a.n ** 3)
    print(json.dumps({"workload": f"{op} {a.prec} n={a.n} x{a.batch} plan={list(p)}", "seconds": t,
                      "solves_per_s": a.batch / t, "gflops": a.batch * fl / t / 1e9}))
    h.close()


def variants(a):
    import torch  # noqa: F401  (device context for the library)
    import paper_1906_08613_amd as tla
    h = tla.Handle(0)
    for op in ["potrf", "trsyl", "trlyap"]:
        for n in [16, 32, 48, 64, 96, 128, 256, 512, 1024]:
            batch = 4096 if n <= 128 else 256
            cands = [tla.candidate(op, i) for i in range(tla.num_candidates(op))]
            if n > 128:  # one kernel per variant above the LDS-resident sizes
                cands = [c for c in cands if c.place == 3 and c.waves == 4]
            best = {}
            for p in cands:
                try:
                    t = h.time_plan(op, n, "f64", batch, p, reps=3)
                except tla.TlaError:
                    continue
                if p.variant not in best or t < best[p.variant][0]:
                    best[p.variant] = (t, list(p.astuple()))
            win = min(best, key=lambda v: best[v][0])
            print(json.dumps({"workload": f"{op} f64 n={n} x{batch}", "winner": tla.variant_name(op, win),
                              "winner_plan": best[win][1],
                              "us_per_variant": {tla.variant_name(op, v): round(best[v][0] * 1e6, 1)
                                                 for v in sorted(best)}}), flush=True)
    h.close()


def run(a):
    {"potrf16": potrf16, "sweep": sweep, "ragged": ragged, "large": large, "planner": planner,
     "potrs": potrs, "variants": variants, "plan": plan, "exact": exact, "general": general,
     "peaks": peaks}[a.workload](a)
