"""Host logic of the benchmark's measurement: reading HBM traffic per launch from a counter
summary (per-dispatch average over the kernels of a class, refused when the summary was
taken from other kernel sources)."""
import os

import bench


def _write_summary(tmp_path, fingerprint):
    prof = tmp_path / "profiles"
    prof.mkdir()
    lines = [
        "# a workload",
        f"# sources sha256: {fingerprint}",
        "dispatches   read_MiB  write_MiB  kernel",
        "        10      100.0       50.0  pmr::(anonymous namespace)::kick_drift_kernel(Args)",
        "         2       10.0       20.0  pmr::(anonymous namespace)::row_count_kernel(x)",
        "         6       30.0       10.0  pmr::(anonymous namespace)::bucket_kernel(x)",
        "         4        1.0        1.0  pmr::(anonymous namespace)::adjoint_update_kernel(x)",
    ]
    (prof / bench.TRAFFIC_PROFILES["p128_m128_b4"]).write_text("\n".join(lines) + "\n")


def test_counter_traffic_averages_the_dispatches_of_a_class(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_fingerprint", lambda: "abc")
    _write_summary(tmp_path, "abc")
    MiB = 2 ** 20
    assert bench.counter_traffic("p128_m128_b4", "kick_drift") == 150.0 * MiB
    # the kernels of a class, weighted by their dispatch counts; other kernels are not part
    # of the class
    want = (2 * 30.0 + 6 * 40.0) / 8 * MiB
    assert abs(bench.counter_traffic("p128_m128_b4", "sort") - want) < 1e-6
    assert bench.counter_traffic("p128_m128_b4", "adj_update") == 2.0 * MiB
    # a class with no dispatch in the summary, an unknown class, a workload with no summary
    assert bench.counter_traffic("p128_m128_b4", "paint") is None
    assert bench.counter_traffic("p128_m128_b4", "no_such_class") is None
    assert bench.counter_traffic("p64_m64_b32", "kick_drift") is None


def test_counter_traffic_is_null_for_other_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_fingerprint", lambda: "new")
    _write_summary(tmp_path, "old")
    assert bench.counter_traffic("p128_m128_b4", "kick_drift") is None


def test_source_fingerprint_covers_every_kernel_source():
    fp = bench.source_fingerprint()
    assert len(fp) == 64 and int(fp, 16) >= 0
    src = os.path.join(bench.ROOT, "paper_1805_02247_amd", "csrc")
    assert any(f.endswith(".hip") for f in os.listdir(src))
    assert fp == bench.source_fingerprint()
