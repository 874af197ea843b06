"""Host-side checks of bench.py that need no GPU: it refuses more than one
GPU with a message, and the hash that ties the committed HBM counter data to
the kernel sources ignores comments and layout but not code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_sources_hash_ignores_comments_but_not_code():
    import bench
    a = "int f(int x) {  // twice\n  return 2 * x; /* doubled */\n}\n"
    b = "int f(int x)\n{\n    return 2*x;\n}"
    c = "int f(int x) { return 3 * x; }"
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(a) != bench.code_only(c)
    h = bench.sources_hash()
    assert len(h) == 16 and h == bench.sources_hash()
