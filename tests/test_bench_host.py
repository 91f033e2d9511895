"""Host logic of bench.py (no GPU): the algorithmic bytes of the coarse
stencil, the algorithmic flops of the SAP half sweep (the roofline kernel)
rebuilt from hop counts on a blocked lattice, and the traffic figure read
from a committed counter summary, which must be withheld once the kernel
source differs from the one the counters were taken with."""
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



def test_sap_flops_follow_the_block_hop_counts():
    """The SAP half sweep's algorithmic flops assume 6 in-block and 2
    block-leaving hops per site of a 4^4 block on average (a site on a block
    face loses the hop across it).  Count them on a lattice of 4^4 blocks and
    rebuild the per-launch figure from the counts: per pair of an even and an
    odd site and column, k Schur steps of (in-block hops of both sites) x 165
    flop plus the site terms, inner products and axpys; the right-hand side and
    the back substitution (the even site's in-block hops each); and the
    block-leaving hops of the block residual, which only the second of the two
    half sweeps computes (counted at half per launch)."""
    import numpy as np
    from oracle.multigrid import Blocking
    blk = Blocking((8, 8, 8, 8), (4, 4, 4, 4))
    inside = sum(blk.internal_mask(mu, fw) for mu in range(4) for fw in (True, False))
    assert np.allclose(inside.mean(), 6.0)
    leaving = 8 - inside.mean()
    V, k = 40 * 40 * 40 * 80, 5
    hop = 165
    per_pair = (k * (2 * inside.mean() * hop + 72 + 72 + 48 + 144 + 192)
                + 2 * (inside.mean() * hop + 48 + 72) + 2 * leaving * hop / 2)
    assert bench.sap_oe_flops_per_tile(V, k) == int(round((V // 4) * 8 * per_pair))
    assert abs(bench.sap_oe_flops_per_tile(V, k) - 154.5e9) < 0.05e9
