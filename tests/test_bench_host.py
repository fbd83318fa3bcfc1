"""Host-side logic of the benchmark: the one-GPU guard, the nominal flop and
algorithmic byte counts, the traffic lookup's library check, and the CPU
oracle baseline's fields (on a tiny workload)."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_nominal_flops_and_algorithmic_bytes():
    # paper's flop convention: n^3/3 for Cholesky, 2 n^3 for Sylvester and Lyapunov
    assert bench.flops("potrf", 64) == 64 ** 3 / 3
    assert bench.flops("trsyl", 64) == 2 * 64 ** 3 == bench.flops("trlyap", 64)
    # referenced triangles once in, result once out (8-byte words)
    n = 5
    tri = n * (n + 1) // 2
    assert bench.min_bytes("potrf", n) == 8 * (tri + tri)
    assert bench.min_bytes("trsyl", n) == 8 * (tri + tri + n * n + n * n)
    assert bench.min_bytes("trlyap", n) == 8 * (tri + tri + n * n)


def test_traffic_lookup_requires_the_same_library(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    entry = {"trsyl/mixed_f32/n64/b8192": {"kernel": "k", "fetch_bytes": 3.0, "write_bytes": 4.0}}
    (prof / "hbm_traffic.json").write_text(json.dumps({"lib_hash": "abc", "entries": entry}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "lib_hash", lambda: "abc")
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192) == 7.0
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 4096) is None
    # the summary's kernel must be the one the run's plan launches
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192, splitting=False) == 7.0
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192, splitting=True) is None
    entry["trsyl/mixed_f32/n64/b8192"]["kernel"] = "tla::k_jacobi_mixed<4, 1, false>"
    (prof / "hbm_traffic.json").write_text(json.dumps({"lib_hash": "abc", "entries": entry}))
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192, splitting=True) == 7.0
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192, splitting=False) is None
    monkeypatch.setattr(bench, "lib_hash", lambda: "other")
    assert bench.traffic_for("trsyl", "mixed_f32", 64, 8192) is None


def test_cpu_baseline_fields():
    import oracle as orc
    orc.build()
    hosts = [(op, bench.make_inputs(op, 6, 8, 1e2)) for op in ["potrf", "trsyl", "trlyap"]]
    r = bench.cpu_baseline(orc, hosts, 0.05)
    assert r["kind"] == "oracle" and r["unit"] == "solves/s"
    assert r["value"] > 0 and r["value_1thread"] > 0 and r["cores"] >= 1
    assert "8 instances" in r["sample"]
    # the oracle results on these inputs are finite
    X, info = orc.potrf_batch(hosts[0][1][0])
    assert np.all(info == 0) and np.all(np.isfinite(X))
