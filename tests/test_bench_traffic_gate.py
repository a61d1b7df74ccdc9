"""The gate that ties the committed rocprofv3 traffic summaries to the kernel
code they were taken on: the bench reports measured HBM traffic only while
the kernel sources hash as the summary records, comments aside (CPU only)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_committed_summaries_read_while_code_unchanged():
    """Each summary's kernels read back (bytes > 0) while the recorded hash is
    the code's; after a code change every one reads None (the bench then
    reports traffic null until the counters are taken again)."""
    for which, (summary, _) in bench.TRAFFIC_SETS.items():
        with open(os.path.join(ROOT, summary)) as f:
            lines = f.read().splitlines()
        kernels = [line.split()[1] for line in lines if line.startswith("traffic ")]
        recorded = [line.split()[1] for line in lines if line.startswith("kernel_source_sha256 ")]
        assert kernels and len(recorded) == 1, summary
        current = recorded[0] == bench.kernel_source_hash(which)
        for k in kernels:
            got = bench.read_traffic_summary(k, which)
            assert (got is not None and got > 0) if current else got is None, (which, k)


def test_hash_ignores_comments_but_not_code(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.TRAFFIC_SETS, "probe", ("none.txt", ("k.hip",)))
    src.write_text("int f(int x) {\n    return x + 1;  // next\n}\n")
    h0 = bench.kernel_source_hash("probe")
    src.write_text("// the successor\n/* of x */\nint f(int x) {\n\n    return x + 1;    // x + 1\n}\n")
    assert bench.kernel_source_hash("probe") == h0
    src.write_text("int f(int x) {\n    return x + 2;  // next\n}\n")
    assert bench.kernel_source_hash("probe") != h0
    src.write_text("int f(int x) {\n    return x + 1;  // next\n}\nint g() { return 0; }\n")
    assert bench.kernel_source_hash("probe") != h0
