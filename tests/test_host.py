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


def test_profiled_traffic_only_for_its_workload_and_kernel(tmp_path, monkeypatch):
    """The bench reports the profiled HBM bytes only for the workload the profile
    was taken on and while the pass source matches the profiled digest."""
    sys.path.insert(0, ROOT)
    import bench

    src = tmp_path / "paper_2008_13447_amd" / "csrc"
    src.mkdir(parents=True)
    (src / "valmod_pass.hip").write_text("int f() {\n  return 1;\n}\n")
    prof = tmp_path / "profiles"
    prof.mkdir()
    import hashlib
    sha = hashlib.sha256(bench.kernel_code(str(src / "valmod_pass.hip")).encode()).hexdigest()[:16]
    (prof / "k_pass_fp32_w.md").write_text(
        "# summary\n\n- FETCH_SIZE: 1 KiB\n\nworkload: wk\ntraffic_bytes_per_launch: 1234\n"
        f"kernel_source_sha256_16: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.profiled_traffic("fp32", "wk") == 1234.0
    assert bench.profiled_traffic("fp32", "other") is None
    assert bench.profiled_traffic("fp64", "wk") is None
    (src / "valmod_pass.hip").write_text("int f() {\n  return 2;\n}\n")
    assert bench.profiled_traffic("fp32", "wk") is None


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
