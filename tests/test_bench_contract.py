"""bench.py checks that need no GPU: more than one GPU is refused with a
message (the library has no multi-GPU path); the measured HBM traffic is
reported only for the kernel sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def _bench_module():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_is_reported_only_for_the_profiled_sources():
    """The committed HBM traffic of a k_update variant is reported only while the
    engine sources (comment lines aside) hash to the ones its counters were taken
    on, else null."""
    import json
    b = _bench_module()
    h = b.engine_source_hash()
    assert len(h) == 16
    for mode in ("fp64", "mixed"):
        with open(os.path.join(ROOT, "profiles", f"k_update_{mode}_n524288_traffic.json")) as f:
            rec = json.load(f)
        assert rec["hbm_bytes_per_launch"] > 0
        expected = rec["hbm_bytes_per_launch"] if rec["source_sha256_16"] == h else None
        assert b.measured_traffic(mode) == expected, mode
    assert b.measured_traffic("nonexistent-mode") is None


def test_source_hash_ignores_comments_only(tmp_path, monkeypatch):
    b = _bench_module()
    src = os.path.join(ROOT, "paper_1411_4510_amd", "csrc")
    work = tmp_path / "paper_1411_4510_amd" / "csrc"
    work.mkdir(parents=True)
    for fn in ("engine.hip", "engine.h", "mfma_core.h"):
        with open(os.path.join(src, fn)) as f:
            (work / fn).write_text(f.read())
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    h0 = b.engine_source_hash()
    eng = work / "engine.hip"
    eng.write_text(eng.read_text() + "\n// a comment line\n\n")
    assert b.engine_source_hash() == h0
    eng.write_text(eng.read_text() + "static int lma_changed_code_line = 0;\n")
    assert b.engine_source_hash() != h0
