"""bench.py on the CPU host: a request for more than one GPU is refused with
a JSON message and a non-zero status, before anything touches a device; the
reported HBM traffic is read from a committed counter summary only while the
counted kernel's sources are unchanged."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 2, r.stderr
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2
    assert "one GPU only" in line["error"]


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_read_only_for_unchanged_sources(tmp_path, monkeypatch):
    """roofline.traffic comes from a committed counter summary only while the
    kernel's listed sources hash to the value recorded with the counters;
    otherwise, or without a summary, it is null with the reason."""
    import hashlib
    bench = _bench_module()
    (tmp_path / "profiles").mkdir()
    (tmp_path / "src").mkdir()
    a, b = tmp_path / "src" / "k.hip", tmp_path / "src" / "t.json"
    a.write_bytes(b"kernel text\n")
    b.write_bytes(b'{"table": 1}\n')
    h = hashlib.sha256(a.read_bytes() + b.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "counters.md").write_text(
        "# counters\n\nbench-traffic: kernel=pcg_round workload=batched bytes_per_launch=1234.5 "
        f"sources=src/k.hip,src/t.json sha256={h}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("pcg_round", "batched") == (1234.5, "counters.md")
    t, why = bench.measured_traffic("pcg_round", "box")
    assert t is None and "no counter summary" in why
    t, why = bench.measured_traffic("accd", "batched")
    assert t is None and "no counter summary" in why
    a.write_bytes(b"kernel text, edited\n")
    t, why = bench.measured_traffic("pcg_round", "batched")
    assert t is None and "sources changed" in why


def test_committed_traffic_line_names_existing_sources():
    """Every committed bench-traffic line lists sources that exist, so the
    bench can check them."""
    import glob
    n = 0
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if line.startswith("bench-traffic:"):
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                for src in kv["sources"].split(","):
                    assert os.path.isfile(os.path.join(ROOT, src)), (path, src)
                assert len(kv["sha256"]) == 64 and float(kv["bytes_per_launch"]) > 0
                n += 1
    assert n >= 1
