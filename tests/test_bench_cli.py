"""bench.py runs on one GPU: asked for more it exits with status 2 and says
why, before touching any device."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _bench_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_traffic_only_for_the_profiled_workload():
    """The committed HBM traffic of the row kernel is reported for the
    workload the counters were taken on (six graphs of n = 32768) and for no
    other."""
    b = _bench_module()
    t = b.committed_traffic(6, 32768)
    assert t is not None and t > 0
    assert b.committed_traffic(2, 32768) is None
    assert b.committed_traffic(6, 16384) is None


def test_kernel_hash_ignores_comments_and_whitespace_only(tmp_path, monkeypatch):
    b = _bench_module()
    src = tmp_path / "k.hip"
    src.write_text("int f(int x) {\n    return x + 1;  // one more\n}\n/* block\n comment */\n")
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "KERNEL_SOURCES", ("k.hip",))
    h0 = b.kernel_sources_sha256()
    src.write_text("int f(int x)   {\n  return x + 1;  // a different comment\n}\n")
    assert b.kernel_sources_sha256() == h0
    src.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert b.kernel_sources_sha256() != h0
