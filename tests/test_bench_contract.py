"""Host-side parts of bench.py: the one-GPU refusal and the keying of the
committed counter records (no GPU needed)."""
import argparse
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def ns(**kw):
    d = dict(workload="hminus_scan", exchange=0, precond="block_jacobi", prec="fp64", restart=300)
    d.update(kw)
    return argparse.Namespace(**d)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_variant_names_every_option_that_changes_the_kernels():
    assert bench.traffic_variant(ns()) == "hminus_scan"
    assert bench.traffic_variant(ns(workload="ps_q127", restart=60)) == "ps_q127"
    seen = {bench.traffic_variant(v) for v in (ns(exchange=1), ns(exchange=-1), ns(precond="coupled"),
                                                ns(prec="fp32"), ns(restart=200))}
    assert len(seen) == 5 and "hminus_scan" not in seen


def test_counter_records_apply_only_to_their_own_configuration(tmp_path, monkeypatch):
    src = tmp_path / "kernels.hip"
    src.write_text("// kernels\n")
    import hashlib
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    rec = {"entries": {"hminus_scan:mdot": {"kernels_hip_sha256": sha, "hbm_bytes_per_launch": 123.0}}}
    tf = tmp_path / "hbm_traffic.json"
    tf.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tf))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    assert bench.measured_traffic(bench.traffic_variant(ns()), "mdot") == 123.0
    assert bench.measured_traffic(bench.traffic_variant(ns(exchange=1)), "mdot") is None
    assert bench.measured_traffic(bench.traffic_variant(ns()), "mupdate") is None
    src.write_text("// changed kernels\n")
    assert bench.measured_traffic(bench.traffic_variant(ns()), "mdot") is None
