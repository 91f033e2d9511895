"""GPU parity at the full sizes of the 32^3x64 batching workload, the
40^3x80 large-volume workload and (for the tuned path's smoother) the 16^3x32
bench workload, through the C ABI.

The oracle cannot apply the operator to whole fields of this size column by
column in test time, so it is evaluated site by site on sampled sites (its
own formula, independent of the library), and properties that hold at any
size are checked on whole fields (gamma5-hermiticity).  At 32^3x64 a small
uneven batch is solved with the tuned solver and every column's residual is
checked by the library's FP64 residual and by the oracle on sampled sites.
"""
import sys

import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def dd():
    import paper_2201_03872_amd as m
    m.load()
    return m


def sampled_sites(V, n, seed):
    rng = np.random.default_rng(seed)
    return sorted(set([0, V - 1] + [int(v) for v in rng.integers(0, V, n)]))


def operator_checks(torch, dd, ctx, op, dims, mus):
    V = S.volume(dims)
    ncol = len(mus)
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.complex(torch.randn((ncol, V, 4, 3), dtype=torch.float64, device="cuda", generator=gen),
                      torch.randn((ncol, V, 4, 3), dtype=torch.float64, device="cuda", generator=gen))
    sites = sampled_sites(V, 40, 9)
    xs = x.cpu().numpy()
    ref = op.apply_site(xs, mus, sites)
    y = ctx.apply_op(0, dd.FP64, mus, x)
    err = np.max(np.abs(y.cpu().numpy()[:, sites] - ref)) / np.max(np.abs(ref))
    say(f"  FP64 operator, sampled sites: {err:.2e}")
    assert err < 1e-13
    y32 = ctx.apply_op(0, dd.FP32, mus, x)
    err32 = np.max(np.abs(y32.cpu().numpy()[:, sites] - ref)) / np.max(np.abs(ref))
    say(f"  FP32 operator, sampled sites: {err32:.2e}")
    assert err32 < 2e-6
    # gamma5-hermiticity on whole fields
    g5 = torch.tensor([1, 1, -1, -1], dtype=torch.float64, device="cuda").view(1, 1, 4, 1)
    phi = x.roll(1, dims=0).contiguous()
    lhs = torch.sum(phi.conj() * g5 * ctx.apply_op(0, dd.FP64, mus, (g5 * x).contiguous()), dim=(1, 2, 3))
    rhs = torch.sum(ctx.apply_op(0, dd.FP64, -mus, phi).conj() * x, dim=(1, 2, 3))
    assert torch.max(torch.abs(lhs - rhs) / torch.abs(lhs)).item() < 1e-12


def test_batched_workload_full_size(torch_cuda, dd):
    torch = torch_cuda
    w = S.workload("tm_32x32x32x64_batched")
    say("32^3x64: generating the gauge field")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    # the bench's tuned solver: FP64 FGMRES(4) over FP32 FGMRES(40, FP16 basis)
    # over SAP with 4 MR steps on the odd-even reduced blocks
    p = dd.params_for_workload(w, n_levels=1, sap_cycles=1, sap_mr_iters=4, sap_oddeven=1, outer_restart=4,
                               max_outer=3000, inner_iters=40, inner_tol=1e-2, inner_fp16=1, precision=dd.MIXED)
    ctx = dd.Context(p, U)
    operator_checks(torch, dd, ctx, op, w.dims, np.array([1e-3, 0.02, 0.3, 1.0]))
    # a small uneven batch of the workload's systems (1 rhs x 2 shifts, 1 rhs x 1 shift)
    V = S.volume(w.dims)
    counts = S.c3_solve_counts(24, 403)
    systems = [(np.asarray(counts[1][1]), S.gaussian_spinors(counts[1][0], V, 501)),
               (np.asarray(counts[4][1]), S.gaussian_spinors(counts[4][0], V, 502))]
    say(f"  solving {[(b.shape[0], len(m)) for m, b in systems]}")
    xs, infos, st = ctx.solve_batch([(m, torch.from_numpy(b).cuda()) for m, b in systems])
    say(f"  status {st}, stats {ctx.stats()}")
    assert st == dd.OK
    sites = sampled_sites(V, 40, 11)
    for (mus, b), x, info in zip(systems, xs, infos):
        assert all(i["converged"] and i["true_rel_res"] <= 1e-10 for i in info)
        xh = x.cpu().numpy()
        mm = np.tile(mus, b.shape[0])
        bb = np.repeat(b, len(mus), axis=0)
        r = bb[:, sites] - op.apply_site(xh, mm, sites)
        bn = O.col_norm(bb)
        worst = np.max(np.linalg.norm(r.reshape(len(mm), -1), axis=1) / bn)
        say(f"  sampled-site residual / ||b||: {worst:.2e}")
        assert worst <= 1e-10
    ctx.close()


def test_large_volume_operator_full_size(torch_cuda, dd):
    torch = torch_cuda
    w = S.workload("tm_40x40x40x80_4rhs_8shift")
    say("40^3x80: generating the gauge field")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    ctx = dd.Context(dd.params_for_workload(w, n_levels=1, precision=dd.MIXED), U)
    operator_checks(torch, dd, ctx, op, w.dims, np.array([w.mus[0], w.mus[-1]]))
    ctx.close()


def test_oddeven_sap_bench_lattice(torch_cuda, dd):
    """The tuned path's smoother at the bench's full size (16^3x32, 4^4
    blocks): FP64 odd-even SAP against the oracle on two columns, the FP32
    form (the cycle's smoother) and the FP32 form with FP16-stored
    right-hand sides (as the inner solve runs it) on the same columns."""
    torch = torch_cuda
    w = S.workload("tm_16x16x16x32_12rhs_4shift")
    say("16^3x32 odd-even SAP")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    V = S.volume(w.dims)
    ctx = dd.Context(dd.params_for_workload(w, n_levels=1, sap_cycles=1, sap_mr_iters=2, sap_oddeven=1), U)
    f = S.gaussian_spinors(2, V, 611)
    mus = np.array([0.002, 0.1])
    lev = FineLevel(O.WilsonTM(U, w.dims, kappa=w.kappa))
    ref = O.sap(lev, Blocking(w.dims, (4, 4, 4, 4)), f.reshape(2, V, 12), mus, 1, 2, oddeven=True).reshape(2, V, 4, 3)
    fg = torch.from_numpy(f).cuda()
    x64 = ctx.apply_sap(dd.FP64, mus, fg).cpu().numpy()
    rel = lambda a: np.max(np.linalg.norm((a - ref).reshape(2, -1), axis=1) / np.linalg.norm(ref.reshape(2, -1), axis=1))
    say(f"  fp64 {rel(x64):.2e}")
    assert rel(x64) < 1e-12
    x32 = ctx.apply_sap(dd.FP32, mus, fg).cpu().numpy()
    say(f"  fp32 {rel(x32):.2e}")
    assert rel(x32) < 1e-6          # measured 1.1e-7
    x16 = ctx.apply_sap(dd.FP16, mus, fg).cpu().numpy()
    say(f"  fp32 with FP16 right-hand sides {rel(x16):.2e}")
    assert rel(x16) < 2e-3          # FP16 storage of f: 2^-11 relative per entry
    ctx.close()
