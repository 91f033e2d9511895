"""Host logic of bench.py (no GPU): the roofline kernel's algorithmic bytes
and the traffic figure read from the committed counter summary, which must be
withheld once the kernel source differs from the one the counters were taken
with."""
import hashlib

import bench


def test_coarse_stencil_bytes_and_flops():
    # 40^3x80 level 1: 20000 coarse sites, d = 48, one 8-column tile
    b, f = bench.coarse1_bytes_flops(20000, 48, 1)
    assert b == 20000 * (9 * 4 * 48 * 48 + 12 * 48 * 8)
    assert f == 20000 * 9 * 48 * 48 * 8 * 8


def test_counter_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "coarse.hip"
    src.write_text("// kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "summary.md"
    prof.write_text("| traffic per launch (calibrated fetch + write) | 1.855 GB = 1.06 x algorithmic |\n"
                    f"| SHA-256 of paper_2201_03872_amd/csrc/coarse.hip when the counters were taken | {sha} |\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    assert bench.counter_traffic() == 1.855e9
    src.write_text("// kernel source, changed\n")
    assert bench.counter_traffic() is None
    monkeypatch.setattr(bench, "PROFILE", str(tmp_path / "missing.md"))
    assert bench.counter_traffic() is None

