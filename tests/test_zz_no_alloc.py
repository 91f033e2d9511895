"""The no-allocation operator entry point (ddamg_apply_op_noalloc) against
the allocating one (ddamg_apply_op) and the FP64 oracle, through the C ABI.

Both entry points run the same kernels on the same data, so their results
are bitwise equal; the FP64 form also meets the oracle bar (1e-13 relative
per column).  Two calls in a row, the second with a smaller batch (the
scratch array keeps the first call's contents), on the fine and a coarse
level, FP64 and FP32; a batch beyond the scratch size is rejected on the
host before any device work.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, build_prolongator, galerkin

pytestmark = pytest.mark.gpu


def _relerr_cols(a, b):
    n = a.shape[0]
    return np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)


def test_apply_op_noalloc_matches_apply_op():
    import torch
    import paper_2201_03872_amd as dd
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    dd.load()
    dims, agg, N = (8, 8, 8, 8), (4, 4, 4, 4), 8
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, 91)
    p = dd.default_params(dims=dims, kappa=0.15, n_levels=2, sap_block=agg, agg=[agg, (1, 1, 1, 1)], n_tv=[N, 8],
                          setup_rounds=1)
    tv = S.gaussian_spinors(N, V, 92)
    print("no-alloc apply_op", dims, flush=True)
    ctx = dd.Context(p, U, tv_init=[tv])
    ctx.set_test_vectors(0, tv.reshape(N, V, 12))       # the oracle's P below uses these vectors
    op = O.WilsonTM(U, dims, kappa=0.15)
    blk = Blocking(dims, agg)
    coarse = galerkin(FineLevel(op), build_prolongator(tv.reshape(N, V, 12), blk), blk)
    Vc = blk.nblocks
    for level, ncol in ((0, 13), (0, 5), (1, 11), (1, 3)):
        mus = np.linspace(0.003, 0.2, ncol)
        if level == 0:
            x = S.gaussian_spinors(ncol, V, 93 + ncol)
            ref = op.apply(x, mus)
        else:
            x = S.gaussian_coarse(ncol, Vc, 2 * N, 94 + ncol)
            ref = coarse.apply(x, mus)
        xg = torch.from_numpy(x).cuda()
        for prec in (dd.FP64, dd.FP32):
            y_alloc = ctx.apply_op(level, prec, mus, xg).cpu().numpy()
            y = torch.full_like(xg, float("nan"))
            ctx.apply_op_noalloc(level, prec, mus, xg, y)
            y = y.cpu().numpy()
            diff = np.max(np.abs(y - y_alloc))
            err = np.max(_relerr_cols(y, ref))
            print(f"  level {level} ncol {ncol} prec {prec}: |noalloc - alloc| {diff:.1e}, vs oracle {err:.2e}",
                  flush=True)
            assert diff == 0.0
            if prec == dd.FP64:
                assert err < 1e-13
    # beyond the scratch size: rejected on the host, nothing launched
    big = 100          # 13 tiles of 6.3 MB per internal vector: 164 MB > 64 MiB
    xb = torch.zeros((big, V, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dd.DDAMGError) as e:
        ctx.apply_op_noalloc(0, dd.FP64, np.zeros(big), xb, torch.empty_like(xb))
    assert e.value.code == dd.EINVAL and "scratch" in str(e.value)
    ctx.close()
