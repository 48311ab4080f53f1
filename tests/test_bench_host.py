"""Host logic of the benchmark (CPU): the algorithmic bytes of the pass and the
rule that reports counter traffic only for the kernel sources it was taken on."""
import os

import bench
from paper_2010_07422_amd.sweeps import pass_bytes


def test_pass_bytes_at_the_benchmark_shape():
    # 2 x 277 sampled rows of 10^4 BF16 entries, and the R x n factors read and
    # written on both sides in FP32: 11.08 MB + 1.60 MB
    assert pass_bytes(10000, 10000, 277, 277, 10, 2, 4) == 11_080_000 + 1_600_000
    assert pass_bytes(10000, 10000, 277, 277, 10, 8, 8) == 44_320_000 + 3_200_000
    # ragged shapes: the row side reads n2 entries per sampled row, the column side n1
    assert pass_bytes(300, 200, 7, 5, 3, 4, 4) == 4 * (7 * 200 + 5 * 300) + 2 * 4 * 3 * 500


def test_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    committed = bench.measured_traffic("bf16")
    assert committed is None or committed > 0
    text = open(bench.TRAFFIC_PROFILE).read()
    h = bench.pass_source_hash()
    # a profile taken on these sources is read ...
    good = tmp_path / "good.md"
    good.write_text(f"- source_sha256: `{h}`\n- traffic_bytes_bf16: 123\n- traffic_bytes_f64: 456\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(good))
    assert bench.measured_traffic("bf16") == 123 and bench.measured_traffic("f64") == 456
    # ... one taken on other sources is not
    bad = tmp_path / "bad.md"
    bad.write_text("- source_sha256: `" + "0" * 64 + "`\n- traffic_bytes_bf16: 123\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(bad))
    assert bench.measured_traffic("bf16") is None
    # a missing profile gives no traffic either
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "none.md"))
    assert bench.measured_traffic("bf16") is None
    assert "source_sha256" in text


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2 and "one GPU" in res.stderr
