"""bench.py's command line on the host: runs on more than one GPU are refused
with a message before any GPU work (the estimator is measured on one GPU)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=60, env=env)


def test_more_than_one_gpu_exits_with_a_message():
    r = _bench("--gpus", "2", "--steps", "1", "--warmup", "0")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_world_size_above_one_exits_with_a_message():
    env = dict(os.environ, WORLD_SIZE="2", RANK="0", LOCAL_RANK="0")
    r = _bench("--gpus", "1", env=env)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_stored_traffic_is_tied_to_the_kernel_sources(monkeypatch):
    """The roofline's measured HBM bytes are reported only for the kernel
    sources and workload they were counted on, and equal the record's
    FETCH_SIZE and WRITE_SIZE scaled by the plain-copy factors."""
    import json
    b = _bench_module()
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    k = "apply_f32_kernel<13, 12>"
    e, cp = rec[k], rec["copy_probe"]
    coeffs = e["coeffs"]
    assert coeffs == 64 * 128 * 12 * 1200
    v = b.stored_traffic(k, "fp32", coeffs)
    # the counters were taken on the committed kernel sources: a change to
    # them must come with new counters
    assert e["src_digest"] == b.src_digest("fp32")
    assert v == e["hbm_bytes_per_launch"]
    ks = "apply_split_kernel<13, 12, bf16x3>"
    assert rec[ks]["src_digest"] == b.src_digest("split")
    assert b.stored_traffic(ks, "split", coeffs) == rec[ks]["hbm_bytes_per_launch"]
    scaled = e["FETCH_SIZE_kib"] * 1024 * cp["fetch_scale"] + e["WRITE_SIZE_kib"] * 1024 * cp["write_scale"]
    assert abs(scaled - e["hbm_bytes_per_launch"]) <= 1e-6 * scaled
    assert b.stored_traffic(k, "fp32", coeffs + 1) is None
    monkeypatch.setattr(b, "src_digest", lambda family: "0" * 16)
    assert b.stored_traffic(k, "fp32", coeffs) is None
