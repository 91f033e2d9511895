"""GPU parity of the twisted-mass clover operator (c_sw != 0) through the C ABI,
against the FP64 oracle (whose clover term is pinned in test_oracle_clover.py):

* the clover field built on the device and the fine operator, FP64 (1e-13)
  and FP32 with both link formats (2e-6), on lattices of several tiles with a
  ragged column count; sampled sites of the 16^3x32 bench lattice against the
  oracle's site-by-site formula;
* SAP with the clover in the block operator: FP64 (1e-12), FP32 and the
  FP16-input form of the inner solve (1e-6 / 5e-5);
* the Galerkin coarse operator of oracle test vectors (FP64, 1e-13);
* a tuned mixed-precision solve: every column at the oracle's FP64 residual
  1e-10.
"""
import sys

import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, build_prolongator, galerkin

pytestmark = pytest.mark.gpu

CSW = 1.25


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def dd():
    import paper_2201_03872_amd as m
    m.load()
    return m


def relerr_cols(a, b):
    n = a.shape[0]
    return np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)


@pytest.mark.parametrize("dims,blk,ncol", [((4, 4, 4, 4), (2, 2, 2, 2), 13), ((8, 4, 4, 8), (4, 4, 4, 4), 11)])
def test_clover_operator(torch_cuda, dd, dims, blk, ncol):
    torch = torch_cuda
    say("clover operator", dims, blk, ncol)
    U = S.gauge_field(dims, 0.3, 141)
    ctx = dd.Context(dd.default_params(dims=dims, kappa=0.15, n_levels=1, sap_block=blk, csw=CSW), U)
    V = S.volume(dims)
    x = S.gaussian_spinors(ncol, V, 142)
    mus = np.linspace(-0.3, 0.5, ncol)
    op = O.WilsonTM(U, dims, kappa=0.15, csw=CSW)
    ref = op.apply(x, mus)
    # the clover term is not negligible here
    assert np.max(relerr_cols(O.WilsonTM(U, dims, kappa=0.15).apply(x, mus), ref)) > 0.05
    xg = torch.from_numpy(x).cuda()
    y64 = ctx.apply_op(0, dd.FP64, mus, xg).cpu().numpy()
    e64 = np.max(relerr_cols(y64, ref))
    say("  fp64", e64)
    assert e64 < 1e-13
    for links in (0, 1):
        ctx.set_tuning("fp32_links", links)
        y32 = ctx.apply_op(0, dd.FP32, mus, xg).cpu().numpy()
        e32 = np.max(relerr_cols(y32, ref))
        say("  fp32 links", links, e32)
        assert e32 < 2e-6
    ctx.close()


def test_clover_operator_bench_lattice_sampled(torch_cuda, dd):
    torch = torch_cuda
    dims = (16, 16, 16, 32)
    V = S.volume(dims)
    say("clover operator 16^3x32, sampled sites")
    U = S.gauge_field(dims, 0.3, 143)
    ctx = dd.Context(dd.default_params(dims=dims, kappa=0.15, n_levels=1, sap_block=(4, 4, 4, 4), csw=CSW), U)
    ncol = 12
    mus = np.tile(np.array([0.002, 0.01, 0.03, 0.1]), 3)
    x = S.gaussian_spinors(ncol, V, 144)
    y = ctx.apply_op(0, dd.FP64, mus, torch.from_numpy(x).cuda()).cpu().numpy()
    op = O.WilsonTM(U, dims, kappa=0.15, csw=CSW)
    rng = np.random.default_rng(145)
    sites = np.concatenate([[0, V - 1, 4095, 4096 * 31], rng.integers(0, V, 12)])
    ref = op.apply_site(x, mus, sites)
    err = np.max(np.abs(y[:, sites] - ref)) / np.max(np.abs(ref))
    say("  sampled-site error", err)
    assert err < 1e-13
    ctx.close()


def test_clover_sap(torch_cuda, dd):
    torch = torch_cuda
    dims, blk = (8, 8, 4, 8), (4, 4, 4, 4)
    say("clover SAP", dims, blk)
    U = S.gauge_field(dims, 0.3, 146)
    ctx = dd.Context(dd.default_params(dims=dims, kappa=0.15, n_levels=1, sap_block=blk, sap_cycles=2,
                                       sap_mr_iters=3, csw=CSW), U)
    V = S.volume(dims)
    ncol = 9
    f = S.gaussian_spinors(ncol, V, 147)
    mus = np.linspace(0.001, 0.2, ncol)
    lev = FineLevel(O.WilsonTM(U, dims, kappa=0.15, csw=CSW))
    ref = O.sap(lev, Blocking(dims, blk), f.reshape(ncol, V, 12), mus, 2, 3).reshape(ncol, V, 4, 3)
    fg = torch.from_numpy(f).cuda()
    e64 = np.max(relerr_cols(ctx.apply_sap(dd.FP64, mus, fg).cpu().numpy(), ref))
    say("  fp64", e64)
    assert e64 < 1e-12
    hs = np.sqrt(12 * V) / 16

    def r16(a):
        return (a * hs).astype(np.float16).astype(np.float64) / hs
    f16 = r16(f.real) + 1j * r16(f.imag)
    ref16 = O.sap(lev, Blocking(dims, blk), f16.reshape(ncol, V, 12), mus, 2, 3).reshape(ncol, V, 4, 3)
    for variant in (2, 3):
        ctx.set_tuning("sap_variant", variant)
        e32 = np.max(relerr_cols(ctx.apply_sap(dd.FP32, mus, fg).cpu().numpy(), ref))
        e16 = np.max(relerr_cols(ctx.apply_sap(dd.FP16, mus, fg).cpu().numpy(), ref16))
        say("  variant", variant, "fp32", e32, "fp16 input", e16)
        assert e32 < 1e-6 and e16 < 5e-5      # measured 1.3e-7 and 7.4e-6
    ctx.close()


def test_clover_galerkin(torch_cuda, dd):
    torch = torch_cuda
    dims, agg, N = (8, 4, 4, 8), (2, 2, 2, 2), 8
    say("clover Galerkin", dims, agg, N)
    U = S.gauge_field(dims, 0.3, 148)
    V = S.volume(dims)
    tv = S.gaussian_spinors(N, V, 149).reshape(N, V, 12)
    p = dd.default_params(dims=dims, kappa=0.15, n_levels=2, sap_block=agg, agg=[agg, (2, 2, 2, 2)], n_tv=[N, 8],
                          setup_rounds=1, csw=CSW)
    ctx = dd.Context(p, U, tv_init=[tv])
    ctx.set_test_vectors(0, tv)
    blk = Blocking(dims, agg)
    coarse = galerkin(FineLevel(O.WilsonTM(U, dims, kappa=0.15, csw=CSW)), build_prolongator(tv, blk), blk)
    Bg = ctx.coarse_op(1)
    err = np.max(np.abs(Bg - coarse.blocks)) / np.max(np.abs(coarse.blocks))
    say("  coarse blocks", err)
    assert err < 1e-13
    ncol = 7
    xc = S.gaussian_coarse(ncol, blk.nblocks, 2 * N, 150)
    mus = np.linspace(0.001, 0.3, ncol)
    yc = ctx.apply_op(1, dd.FP64, mus, torch.from_numpy(xc).cuda()).cpu().numpy()
    assert np.max(relerr_cols(yc, coarse.apply(xc, mus))) < 1e-13
    ctx.close()


def test_clover_tuned_solve(torch_cuda, dd):
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    mus = np.array(w.mus)
    b = S.rhs_for(w)
    say("clover tuned solve", w.dims, len(mus), b.shape[0])
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block, sap_cycles=1,
                          sap_mr_iters=8, outer_restart=10, max_outer=200, inner_iters=30, inner_tol=1e-2,
                          inner_fp16=1, precision=dd.MIXED, csw=CSW)
    ctx = dd.Context(p, U)
    x, info, st = ctx.solve(mus, torch.from_numpy(b).cuda())
    s = ctx.stats()
    op = O.WilsonTM(U, w.dims, kappa=w.kappa, csw=CSW)
    nr, ns = b.shape[0], len(mus)
    bb = np.repeat(b, ns, axis=0)
    rel = O.col_norm(bb - op.apply(x.cpu().numpy(), np.tile(mus, nr))) / O.col_norm(bb)
    say(f"  status {st}, outer {s['outer_iters']}, inner {s['n_inner_iters']}, worst {rel.max():.2e}")
    assert st == dd.OK and all(i["converged"] for i in info)
    assert np.all(rel <= 1e-10 * (1 + 1e-6))
    ctx.close()
