"""bench.py's host-side contract (no GPU): one GPU only, and roofline inputs
taken from recorded counters only while the kernel sources they were
measured on are unchanged."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_counters_follow_their_sources(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "kernel.hip"
    src.write_text("// version 1\n")
    entry = {"sources": [str(src)], "hbm_bytes": 123, "valu_insts": 1000,
             "variants": {"28": {"hbm_bytes": 7}}}
    entry["source_hash"] = b.source_hash(entry["sources"])
    path = tmp_path / "counters.json"
    path.write_text(json.dumps({"k": entry}))
    monkeypatch.setattr(b, "COUNTERS", str(path))
    assert b.counted("k")["hbm_bytes"] == 123
    assert b.counted("k", 28) == {"hbm_bytes": 7}
    assert b.counted("k", 32) is None          # a variant never counted
    assert b.counted("other") is None
    src.write_text("// version 2\n")           # the kernel changed since
    assert b.counted("k") is None
    assert b.counted("k", 28) is None
    monkeypatch.setattr(b, "COUNTERS", str(tmp_path / "missing.json"))
    assert b.counted("k") is None


def test_alu_roofline_arithmetic():
    b = _bench()
    # 1e9 wave instructions x 64 lanes in 1 ms = 64 T lane-ops/s
    r = b.alu_roofline({"valu_insts": 1e9, "valu2_share": 0.1}, 1.0, "k")
    assert abs(r["achieved"] - 64.0) < 1e-9
    assert abs(r["frac"] - round(64.0 / (b.VALU_PEAK_LANE_OPS / 1e12), 4)) < 1e-12
    assert r["peak"] == 78.6 and r["bound"] == "alu"
    assert b.alu_roofline(None, 1.0, "k") is None
    assert b.alu_roofline({"hbm_bytes": 1}, 1.0, "k") is None


def test_recorded_counters_are_stamped():
    """Every recorded entry names its sources and carries a hash of them and
    the command lines that measured it (whether the hash is current depends
    on later edits, which bench.py then reports as null traffic)."""
    with open(os.path.join(ROOT, "profiles", "counters.json")) as fh:
        c = json.load(fh)
    assert "_scale" in c
    for k, e in c.items():
        if k.startswith("_"):
            continue
        assert e["sources"] and all(os.path.exists(os.path.join(ROOT, f)) for f in e["sources"])
        assert len(e["source_hash"]) == 16
        assert e["commands"] and all("rocprofv3 --pmc" in cmd for cmd in e["commands"])
