"""GPU tests of the outer solve's column scheduler, through the C ABI.

* Uneven batches: independent systems with different rhs x shift counts
  (drawn like the 32^3x64 batching workload, on an 8^4 field) solved in one
  simultaneous batch; every column's solution is checked by the FP64 oracle
  residual (<= 1e-10).
* Converged columns leave at restarts and the active set is compacted; with a
  cap on the columns in flight, waiting columns join as others leave.
* The degenerate single-column batch and the argument checks.
"""
import sys

import numpy as np
import pytest

import synthetic as S
import oracle as O

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


def systems_for(dims, n_sys, seed):
    V = S.volume(dims)
    out = []
    for k, (n_rhs, mus) in enumerate(S.c3_solve_counts(n_sys, seed)):
        out.append((np.asarray(mus, dtype=np.float64), S.gaussian_spinors(n_rhs, V, 900 + k)))
    return out


def check_batch(op, systems, xs, infos, tol=1e-10):
    worst = 0.0
    for (mus, b), x, info in zip(systems, xs, infos):
        n_rhs, n_shift = b.shape[0], len(mus)
        bb = np.repeat(b, n_shift, axis=0)
        rel = O.col_norm(bb - op.apply(x.cpu().numpy(), np.tile(mus, n_rhs))) / O.col_norm(bb)
        assert np.all(rel <= tol * (1 + 1e-6)), rel
        assert all(i["converged"] for i in info)
        # the library's own FP64 residual agrees with the oracle's
        lib = np.array([i["true_rel_res"] for i in info])
        assert np.allclose(lib, rel, rtol=1e-3, atol=1e-14)
        worst = max(worst, rel.max())
    return worst


@pytest.mark.parametrize("max_active", [0, 8, 13])
def test_uneven_batch(torch_cuda, dd, max_active):
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    systems = systems_for(w.dims, 5, 403)
    ncol = sum(b.shape[0] * len(m) for m, b in systems)
    say(f"uneven batch: {[(b.shape[0], len(m)) for m, b in systems]} = {ncol} columns, max_active {max_active}")
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block, sap_cycles=1,
                          sap_mr_iters=8, outer_restart=20, max_outer=2000, precision=dd.MIXED,
                          max_active_cols=max_active)
    ctx = dd.Context(p, U)
    xs, infos, st = ctx.solve_batch([(m, torch.from_numpy(b).cuda()) for m, b in systems])
    stats = ctx.stats()
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    worst = check_batch(op, systems, xs, infos)
    its = [i["outer_iters"] for inf in infos for i in inf]
    say(f"  status {st}, worst {worst:.2e}, column iterations {min(its)}..{max(its)}, "
        f"compactions {stats['col_removals']}, batch iterations {stats['outer_iters']}")
    assert st == dd.OK
    assert stats["col_removals"] >= 1
    if max_active:
        # the batch runs longer than the slowest column because of waiting columns
        assert stats["outer_iters"] > max(its)
    ctx.close()


def test_batch_equals_separate_solves(torch_cuda, dd):
    """A system solved inside a batch and on its own converge to the same x
    (both to 1e-10; their difference is bounded by the conditioning)."""
    torch = torch_cuda
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block, precision=dd.MIXED,
                          tol=1e-12)
    ctx = dd.Context(p, U)
    V = S.volume(w.dims)
    sysA = (np.array([0.01, 0.3]), S.gaussian_spinors(2, V, 31))
    sysB = (np.array([0.05]), S.gaussian_spinors(3, V, 32))
    xs, infos, st = ctx.solve_batch([(m, torch.from_numpy(b).cuda()) for m, b in (sysA, sysB)])
    assert st == dd.OK
    for (m, b), xb in zip((sysA, sysB), xs):
        x1, _, st1 = ctx.solve(m, torch.from_numpy(b).cuda())
        assert st1 == dd.OK
        d = (xb - x1).abs().max().item() / x1.abs().max().item()
        assert d < 1e-8, d
    ctx.close()


def test_single_column_and_argument_checks(torch_cuda, dd):
    torch = torch_cuda
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block)
    ctx = dd.Context(p, U)
    b = torch.from_numpy(S.gaussian_spinors(1, S.volume(w.dims), 41)).cuda()
    xs, infos, st = ctx.solve_batch([(np.array([0.02]), b)])
    assert st == dd.OK and len(xs[0]) == 1 and infos[0][0]["converged"]
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    check_batch(op, [(np.array([0.02]), b.cpu().numpy())], xs, infos)
    # a system without shifts, and a cap below zero, are rejected on the host
    with pytest.raises(dd.DDAMGError) as e:
        ctx.solve_batch([(np.array([0.02]), b), (np.zeros(0), b)])
    assert e.value.code == dd.EINVAL
    with pytest.raises(dd.DDAMGError) as e:
        dd.Context(dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block,
                                     max_active_cols=-1), U)
    assert e.value.code == dd.EINVAL
    ctx.close()


@pytest.mark.parametrize("precision,fp16,oddeven", [("MIXED", 0, 0), ("MIXED", 1, 0), ("PLAIN_FP64", 0, 0),
                                                     ("MIXED", 1, 1), ("PLAIN_FP64", 0, 1)])
def test_inner_fgmres_refinement(torch_cuda, dd, precision, fp16, oddeven):
    """Outer FP64 FGMRES preconditioned by an inner FGMRES (FP32 in the mixed
    form, optionally with its Arnoldi basis stored in FP16) around SAP: every
    column reaches the FP64 oracle residual 1e-10 within a few outer steps."""
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    mus = np.array(w.mus)
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    blk = (4, 4, 4, 4) if oddeven else w.sap_block      # odd-even block solves need 4^4 blocks
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=blk, sap_cycles=1, outer_restart=10, max_outer=200, inner_iters=30, inner_tol=1e-2,
                          inner_fp16=fp16, precision=getattr(dd, precision), sap_oddeven=oddeven)
    ctx = dd.Context(p, U)
    x, info, st = ctx.solve(mus, b)
    s = ctx.stats()
    say(f"inner FGMRES ({precision}, FP16 basis {fp16}, odd-even SAP {oddeven}): outer {s['outer_iters']}, "
        f"inner {s['n_inner_iters']}")
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    check_batch(op, [(mus, S.rhs_for(w))], [x], [info])
    assert st == dd.OK and s["n_inner_iters"] > s["outer_iters"] and s["outer_iters"] <= 20
    ctx.close()


@pytest.mark.parametrize("bound", [1, 4, 1024])
def test_fp16_basis_entry_scale_bound(torch_cuda, dd, bound):
    """The FP16 inner basis is stored unnormalised at a predicted norm; a
    vector whose entry scale leaves [1/B, B] is stored again at its exact
    norm.  B = 1 takes that path at every step (every vector normalised),
    B = 1024 almost never; every form reaches the FP64 oracle residual
    1e-10, and B = 1 restores at least one vector per inner step."""
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    mus = np.array(w.mus)
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=(4, 4, 4, 4), sap_cycles=1,
                          sap_mr_iters=4, outer_restart=4, max_outer=200, inner_iters=30, inner_tol=1e-2,
                          inner_fp16=1, precision=dd.MIXED, sap_oddeven=1)
    ctx = dd.Context(p, U)
    ctx.set_tuning("fp16_rescale", bound)
    assert ctx.get_tuning("fp16_rescale") == bound
    x, info, st = ctx.solve(mus, b)
    s = ctx.stats()
    say(f"FP16 basis, entry-scale bound {bound}: outer {s['outer_iters']}, inner {s['n_inner_iters']}, "
        f"restored {s['n_fp16_restores']}")
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    check_batch(op, [(mus, S.rhs_for(w))], [x], [info])
    assert st == dd.OK and s["outer_iters"] <= 20
    if bound == 1:
        assert s["n_fp16_restores"] >= s["n_inner_iters"] - s["outer_iters"]
    for bad in (0, 1025):
        with pytest.raises(dd.DDAMGError) as e:
            ctx.set_tuning("fp16_rescale", bad)
        assert e.value.code == dd.EINVAL
    ctx.close()


def test_sap_kernel_timing_stats(torch_cuda, dd):
    """DDAMG_KNOB_TIME_SAP: HIP events around every SAP kernel launch of a
    solve, summed into the stats (two half sweeps per one-cycle SAP call);
    off, the fields stay zero and the solve is unchanged."""
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    mus = np.array(w.mus)
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=(4, 4, 4, 4), sap_cycles=1,
                          sap_mr_iters=4, outer_restart=4, max_outer=200, inner_iters=30, inner_tol=1e-2,
                          inner_fp16=1, precision=dd.MIXED, sap_oddeven=1)
    ctx = dd.Context(p, U)
    x0, _, st0 = ctx.solve(mus, b)
    s0 = ctx.stats()
    assert s0["n_sap_kernels"] == 0 and s0["sap_kernel_ms"] == 0.0
    ctx.set_tuning("time_sap", 1)
    x1, info, st1 = ctx.solve(mus, b)
    s1 = ctx.stats()
    say(f"SAP kernel timing: {s1['n_sap_kernels']} launches, {s1['sap_kernel_ms']:.3f} ms, "
        f"{s1['n_sap_kernel_tiles']} tiles, {s1['n_sap_calls']} SAP calls")
    assert st0 == st1 == dd.OK
    assert s1["n_sap_kernels"] == 2 * s1["n_sap_calls"] > 0
    assert s1["n_sap_kernel_tiles"] >= s1["n_sap_kernels"] and s1["sap_kernel_ms"] > 0
    assert s1["outer_iters"] == s0["outer_iters"] and s1["n_inner_iters"] == s0["n_inner_iters"]
    assert torch.equal(x0, x1)
    ctx.close()


def test_two_level_solve_with_oddeven_smoother(torch_cuda, dd):
    """The odd-even SAP as the fine smoother of the two-level K-cycle (4^4 SAP
    blocks = aggregates): every column reaches the oracle's FP64 residual."""
    torch = torch_cuda
    dims = (8, 8, 8, 8)
    U = S.gauge_field(dims, 0.3, 221)
    V = S.volume(dims)
    mus = np.array([0.005, 0.05])
    b = S.gaussian_spinors(2, V, 222)
    p = dd.default_params(dims=dims, kappa=0.14, n_levels=2, sap_block=(4, 4, 4, 4), agg=[(4, 4, 4, 4), (2, 2, 2, 2)],
                          n_tv=[16, 8], setup_rounds=2, sap_cycles=2, sap_mr_iters=3, sap_oddeven=1,
                          precision=dd.MIXED, max_outer=300)
    ctx = dd.Context(p, U)
    x, info, st = ctx.solve(mus, torch.from_numpy(b).cuda())
    s = ctx.stats()
    say(f"two-level, odd-even SAP: status {st}, outer {s['outer_iters']}, bottom solves {s['n_bottom_solves']}")
    check_batch(O.WilsonTM(U, dims, kappa=0.14), [(mus, b)], [x], [info])
    assert st == dd.OK and s["n_bottom_solves"] > 0
    ctx.close()
