"""Host-side checks (CPU): the benchmark's contract, the product path's
independence from the oracle, and loud failure without the HIP library."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_kernel_digest_ignores_comments(tmp_path):
    sys.path.insert(0, ROOT)
    import bench

    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    a.write_text("int f() {  // one\n  return 1;\n}\n")
    b.write_text("// header\n\nint f() {\n  return 1;  // other\n}\n")
    assert bench.kernel_code(str(a)) == bench.kernel_code(str(b))
    b.write_text("int f() {\n  return 2;\n}\n")
    assert bench.kernel_code(str(a)) != bench.kernel_code(str(b))


def test_product_path_does_not_use_the_oracle():
    """Only tests, smoke() and the benchmark's CPU baseline may touch the oracle."""
    pkg = os.path.join(ROOT, "paper_2008_13447_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "oracle_" not in text and "valmod_oracle" not in text, f


def test_binding_fails_loudly_without_the_library(monkeypatch):
    from paper_2008_13447_amd import native

    monkeypatch.setattr(native, "_lib", None)
    monkeypatch.setattr(native, "LIB_PATH", os.path.join(ROOT, "no_such_library.so"))
    with pytest.raises(RuntimeError, match="HIP library missing"):
        native.lib()
