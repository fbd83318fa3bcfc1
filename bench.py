#!/usr/bin/env python3
"""Benchmark of the batched small-solver hot path on one MI355X.

Workload (one "step"): 8192 instances each of the upper Cholesky X^T X = A,
the triangular Sylvester L X + X U = C and the triangular Lyapunov
L X + X L^T = S at n = 64, condition number about 1e2, solved by the batched
kernels of libtla in the requested precision (mixed FP32 + FP64 refinement by
default), FP64 inputs and outputs resident in HBM.  Every solve is in place,
so each timed step works on its own fresh copy of the in/out operands,
prepared before the timed region.

Printed: one JSON line with solves/s over the three operations, GF/s with the
nominal flop counts (n^3/3 and 2n^3), the FP64 path measured in the same run
for comparison, the roofline fraction of the dominant kernel, and the CPU
oracle timed on the host cores over the same instances (about ten seconds of
whole passes on all threads, plus a one-thread pass over a quarter).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, GB/s
FP64_PEAK_TFS = 78.6        # MI355X FP64 matrix / vector, TFLOP/s


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=64)
    p.add_argument("--batch", type=int, default=8192)
    p.add_argument("--kappa", type=float, default=1e2)
    p.add_argument("--prec", default="mixed_f32", choices=["f64", "mixed_f32", "mixed_f16", "mixed_bf16"])
    p.add_argument("--no-fp64-compare", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="wall time of the all-threads oracle run (whole passes over the step's instances)")
    p.add_argument("--ops", default="potrf,trsyl,trlyap")
    p.add_argument("--workload", default="headline",
                   choices=["headline", "potrf16", "sweep", "ragged", "large", "planner", "potrs", "variants", "plan", "exact", "general", "peaks"],
                   help="headline: the metric's configuration (default); the others print their own lines")
    p.add_argument("--plan", default=None, metavar="V,T,E,W,P",
                   help="--workload plan: time this plan (variant,tile,engine,waves,place) for the first of --ops")
    p.add_argument("--no-tune", action="store_true", help="skip autotuning the headline configuration first")
    p.add_argument("--table", default=None, help="load a tuning table instead of tuning")
    p.add_argument("--save-table", default=None, help="write the tuning table here")
    p.add_argument("--traffic-summary", nargs=4, default=None,
                   metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                   help="write profiles/hbm_traffic.json from rocprofv3 counter CSVs of this benchmark and of "
                        "--copy-calibration 1024 (no GPU needed)")
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a plain device-to-device copy of this many MiB (HBM counter calibration)")
    return p.parse_args()


def copy_calibration(mib):
    """A plain copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))


def traffic_summary(fetch_csv, write_csv, cfetch_csv, cwrite_csv, prec, n, batch):
    """Writes profiles/hbm_traffic.json from rocprofv3 --pmc FETCH_SIZE and
    WRITE_SIZE runs of this benchmark (one dispatch per kernel: the one with the
    most traffic) and of --copy-calibration (a plain copy of known size, whose
    readings give the counters' byte scale); prints the table rows."""
    import csv
    import re

    def per_kernel(path, counter):
        best = {}
        for r in csv.DictReader(open(path)):
            if r["Counter_Name"] != counter:
                continue
            k, v = r["Kernel_Name"], float(r["Counter_Value"])
            best[k] = max(best.get(k, 0.0), v)
        return best

    cf, cw = per_kernel(cfetch_csv, "FETCH_SIZE"), per_kernel(cwrite_csv, "WRITE_SIZE")
    copy_f = max(v for k, v in cf.items() if "copyBuffer" in k or "elementwise" in k or "copy" in k.lower())
    copy_w = max(v for k, v in cw.items() if "copyBuffer" in k or "elementwise" in k or "copy" in k.lower())
    mib = 1024  # the calibration copy: --copy-calibration 1024
    fetch_scale = mib * 1024.0 / copy_f   # counters in KiB
    write_scale = mib * 1024.0 / copy_w
    fe, wr = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    entries = {}
    rows = []
    for k in sorted(fe):
        m = re.search(r"k_(potrf|trsyl|trlyap)_(f64|large|mixed|single)|k_jacobi_mixed<\d+, \d+, (true|false)>", k)
        if not m:
            continue
        if m.group(1):
            op = m.group(1)
            kp = prec if m.group(2) == "mixed" else "f64"
        else:
            op = "trlyap" if m.group(3) == "true" else "trsyl"
            kp = prec
        fb = fe[k] * 1024.0 * fetch_scale
        wb = wr.get(k, 0.0) * 1024.0 * write_scale
        key = f"{op}/{kp}/n{n}/b{batch}"
        alg = batch * min_bytes(op, n)
        rows.append(f"| `{k}` | {fe[k]:.0f} | {wr.get(k, 0.0):.0f} | {fb / 1e6:.1f} MB | {wb / 1e6:.1f} MB | "
                    f"{alg / 1e6:.1f} MB | {(fb + wb) / alg:.2f} |")
        if key not in entries or fb + wb > entries[key]["fetch_bytes"] + entries[key]["write_bytes"]:
            entries[key] = {"kernel": k, "fetch_bytes": fb, "write_bytes": wb}
    out = {"lib_hash": lib_hash(), "source": "profiles/hbm_traffic_n64.md", "fetch_scale": fetch_scale,
           "write_scale": write_scale, "entries": entries}
    json.dump(out, open(os.path.join(ROOT, "profiles", "hbm_traffic.json"), "w"), indent=1)
    print(f"calibration: copy of {mib} MiB reads FETCH_SIZE {copy_f:.0f} KiB, WRITE_SIZE {copy_w:.0f} KiB; "
          f"scales {fetch_scale:.3f} (reads), {write_scale:.3f} (writes)")
    print("\n".join(rows))


def flops(op, n):
    return n ** 3 / 3.0 if op == "potrf" else 2.0 * n ** 3


def min_bytes(op, n):
    """Algorithmic HBM bytes per instance: referenced input triangles read once, result written once."""
    w = 8
    if op == "potrf":
        return n * (n + 1) * w                      # upper A in, upper X out
    if op == "trsyl":
        return (n * (n + 1) + 2 * n * n) * w        # lower L + upper U + C in, X out
    return (n * (n + 1) + n * n) * w                # lower L + lower S in, full symmetric X out


def make_inputs(op, n, batch, kappa):
    from paper_1906_08613_amd import inputs as I
    tag = "bench"
    if op == "potrf":
        return (I.potrf_kappa(tag, n, batch, kappa),)
    if op == "trsyl":
        return I.trsyl_kappa(tag, n, batch, kappa)
    return I.trlyap_kappa(tag, n, batch, kappa)


class OpBench:
    """Device operands of one operation: read-only coefficients plus one fresh
    copy of the in/out operand per step."""

    def __init__(self, tla, torch, h, op, host, copies, prec):
        self.op, self.h, self.prec, self.torch, self.tla = op, h, prec, torch, tla
        self.host = host
        n = host[0].shape[-1]
        self.n, self.batch = n, host[0].shape[0]
        if op == "potrf":
            self.pristine = tla.to_device_cm(np.triu(host[0]))
            self.coef = []
        elif op == "trsyl":
            self.coef = [tla.to_device_cm(host[0]), tla.to_device_cm(host[1])]
            self.pristine = tla.to_device_cm(host[2])
        else:
            self.coef = [tla.to_device_cm(host[0])]
            self.pristine = tla.to_device_cm(np.tril(host[1]))
        self.copies = [self.pristine.clone() for _ in range(copies)]
        self.ops = [tla.Operands(n, *self.coef, c) for c in self.copies]

    def run(self, k, prec=None):
        tla, o = self.tla, self.ops[k]
        prec = prec or self.prec
        if self.op == "potrf":
            self.h.potrf_batched(prec, o.batch, o.n_max, o.n, o.ptrs[0], o.lds[0], o.info, o.stat)
        elif self.op == "trsyl":
            self.h.trsyl_batched(prec, o.batch, o.n_max, o.n, o.ptrs[0], o.lds[0], o.ptrs[1], o.lds[1],
                                 o.ptrs[2], o.lds[2], o.info, o.stat)
        else:
            self.h.trlyap_batched(prec, o.batch, o.n_max, o.n, o.ptrs[0], o.lds[0], o.ptrs[1], o.lds[1],
                                  o.info, o.stat)

    def restore(self):
        for c in self.copies:
            c.copy_(self.pristine)


def time_path(torch, benches, prec, steps, warmup):
    """Whole-step wall time (sync on both sides) and per-op kernel time from
    events on the solver's stream."""
    stream = torch.cuda.current_stream()
    for b in benches:
        b.restore()
    torch.cuda.synchronize()
    for w in range(warmup):
        for b in benches:
            b.run(w, prec)
    torch.cuda.synchronize()
    for b in benches:
        b.restore()
    torch.cuda.synchronize()
    ev = {b.op: [] for b in benches}
    t0 = time.perf_counter()
    for k in range(steps):
        for b in benches:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.run(k, prec)
            e1.record(stream)
            ev[b.op].append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern = {op: float(np.mean([a.elapsed_time(c) for a, c in v])) * 1e-3 for op, v in ev.items()}
    return wall, kern


def verify(orc, tla, benches, sample=48):
    """Backward errors and forward errors vs the oracle on a sample of the last step's results."""
    out = {}
    for b in benches:
        idx = np.linspace(0, b.batch - 1, sample).astype(int)
        res = tla.from_device_cm(b.copies[0])[idx]
        info = b.ops[0].info.cpu().numpy()[idx]
        if b.op == "potrf":
            A = b.host[0][idx]
            X = np.triu(res)
            eta = orc.eta_potrf_batch(A, X)
            Xr, _ = orc.potrf_batch(A)
        elif b.op == "trsyl":
            L, U, C = (m[idx] for m in b.host)
            eta = orc.eta_trsyl_batch(L, U, C, res)
            Xr, _ = orc.trsyl_batch(L, U, C)
            X = res
        else:
            L, S = (m[idx] for m in b.host)
            eta = orc.eta_trlyap_batch(L, S, res)
            Xr, _ = orc.trlyap_batch(L, S)
            X = res
        fe = orc.forward_error(X, Xr)
        st = tla.stat_view(b.ops[0].stat)[idx]
        out[b.op] = {"eta_max": float(eta.max()), "fwd_err_max": float(fe.max()),
                     "info_nonzero": int((info != 0).sum()),
                     "iters_mean": float(st["iters"].mean()),
                     "fallbacks": int(((st["flags"] & 6) != 0).sum())}
    return out


def cpu_baseline(orc, benches_host, seconds):
    """The oracle as it stands on the host cores: the whole step's instances,
    passed through repeatedly until about `seconds` of wall time, on all
    threads; then one pass over a quarter of them on one thread."""
    def one_pass(threads, count):
        t, solves, fl = 0.0, 0, 0.0
        for op, host in benches_host:
            n = host[0].shape[-1]
            sub = [m[:count] for m in host]
            t0 = time.perf_counter()
            if op == "potrf":
                orc.potrf_batch(sub[0], threads)
            elif op == "trsyl":
                orc.trsyl_batch(*sub, threads)
            else:
                orc.trlyap_batch(*sub, threads)
            t += time.perf_counter() - t0
            solves += count
            fl += count * flops(op, n)
        return t, solves, fl
    threads = orc.max_threads()
    batch = min(host[0].shape[0] for _, host in benches_host)
    t = s_ = f = 0.0
    reps = 0
    while t < seconds and reps < 100:
        dt, ds, df = one_pass(threads, batch)
        t, s_, f, reps = t + dt, s_ + ds, f + df, reps + 1
    small = max(batch // 4, 1)
    t1, s1, f1 = one_pass(1, small)
    return {"value": s_ / t, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole step ({batch} instances of each of {len(benches_host)} ops at the bench n) "
                      f"passed {reps} times ({t:.1f} s) on {threads} threads, FP64 triple loops, OpenMP over "
                      f"instances; one-thread pass over {small} of each ({t1:.1f} s)",
            "gflops": f / t / 1e9, "value_1thread": s1 / t1, "gflops_1thread": f1 / t1 / 1e9,
            "cpu_model": cpu_model()}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def lib_hash():
    """Digest of the built library: counter summaries are only reused for the same kernels."""
    import hashlib
    import paper_1906_08613_amd as tla
    return hashlib.sha256(open(tla.LIB_PATH, "rb").read()).hexdigest()[:16]


def traffic_for(kernel_op, prec, n, batch, splitting=None):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or
    None when the summary is missing, the library has changed since, or the
    summary's kernel is not the one this run's plan launches (splitting: the
    plan is the splitting-iteration solve, k_jacobi_mixed)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    key = f"{kernel_op}/{prec}/n{n}/b{batch}"
    e = d.get("entries", {}).get(key)
    if not e or d.get("lib_hash") != lib_hash():
        return None
    if splitting is not None and ("jacobi" in e.get("kernel", "")) != splitting:
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def main():
    a = parse()
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    if a.traffic_summary:
        traffic_summary(*a.traffic_summary, a.prec, a.n, a.batch)
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design "
                                   "note, not a measured path", "n_gpus": a.gpus}))
        sys.exit(2)
    if a.workload != "headline":
        import bench_workloads
        bench_workloads.run(a)
        return
    import torch
    import paper_1906_08613_amd as tla
    import oracle as orc

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    orc.build()
    h = tla.Handle(0)
    n, batch = a.n, a.batch
    ops = a.ops.split(",")
    # plans: the autotuner's choice for this configuration (outside the timed region)
    if a.table:
        h.load_table(a.table)
    elif not a.no_tune:
        h.tune(ops, [n], ["f64", a.prec], batch=batch, reps=3)
    if a.save_table:
        h.save_table(a.save_table)
    copies = max(a.steps, a.warmup)
    hosts = [(op, make_inputs(op, n, batch, a.kappa)) for op in ops]
    benches = [OpBench(tla, torch, h, op, host, copies, a.prec) for op, host in hosts]

    wall, kern = time_path(torch, benches, a.prec, a.steps, a.warmup)
    check = verify(orc, tla, benches)
    solves = batch * len(ops) * a.steps
    fl = sum(batch * flops(op, n) for op in ops) * a.steps
    res = {
        "metric": "solves/s and GF/s at n=64, mixed+refined vs FP64, both at 1e-12 rel residual",
        "value": solves / wall,
        "unit": "solves/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"f64": "f64", "mixed_f32": "f32+f64", "mixed_f16": "f16+f32+f64",
                  "mixed_bf16": "bf16+f32+f64"}[a.prec],
        "data": "synthetic",
        "config": {"workload": f"potrf+trsyl+trlyap, n={n}, {batch} instances each, kappa={a.kappa:g}, "
                               f"prec={a.prec}", "n": n, "batch_per_op": batch, "kappa": a.kappa,
                   "ops": ops, "prec": a.prec},
        "gflops": fl / wall / 1e9,
        "kernel_seconds": kern,
        "check": check,
    }
    if a.prec != "f64" and not a.no_fp64_compare:
        w64, k64 = time_path(torch, benches, "f64", a.steps, a.warmup)
        res["fp64"] = {"value": solves / w64, "unit": "solves/s", "gflops": fl / w64 / 1e9,
                       "ms_per_step": w64 / a.steps * 1e3, "kernel_seconds": k64,
                       "check": verify(orc, tla, benches)}
        res["speedup_vs_fp64"] = res["value"] / res["fp64"]["value"]
    # roofline of the dominant kernel: algorithmic bytes per launch / its mean launch time
    dom = max(kern, key=kern.get)
    ach = batch * min_bytes(dom, n) / kern[dom] / 1e9
    dom_plan = h.get_plan(dom, n, a.prec, batch)
    splitting = a.prec != "f64" and tla.variant_name(dom, dom_plan.variant) == "jacobi-sweeps"
    res["roofline"] = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": traffic_for(dom, a.prec, n, batch, splitting),
                       "algorithmic_bytes": batch * min_bytes(dom, n),
                       "fp64_tflops": batch * flops(dom, n) / kern[dom] / 1e12}
    res["plans"] = {op: list(h.get_plan(op, n, a.prec, batch).astuple()) for op in ops}
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(orc, hosts, a.cpu_seconds)
    print(json.dumps(res))
    h.close()


if __name__ == "__main__":
    main()
