"""The non-degenerate twisted-mass doublet operator and its solve on the GPU
against the FP64 oracle (oracle.nondegenerate), through the C ABI.

Bars: the FP64 doublet operator within 1e-13 of the oracle per doublet (the
degenerate stencil's bar; the flavour coupling adds one exact FP64 term), FP32
within 2e-6 (the FP32 stencil's); solves reach the doublet's true FP64
residual 1e-10 by the oracle's operator, and the library's own after-solve
FP64 check agrees with the oracle's residual to 1e-13.
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
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def dd():
    import paper_2201_03872_amd as m
    m.load()
    return m


def pair_relerr(a, b):
    n = a.shape[0]
    return np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_doublet_operator(torch_cuda, dd, csw):
    torch = torch_cuda
    dims = (8, 4, 4, 8)
    V = S.volume(dims)
    say("doublet operator", dims, "csw", csw)
    U = S.gauge_field(dims, 0.3, 131)
    p = dd.default_params(dims=dims, kappa=0.15, n_levels=1, sap_block=(4, 4, 4, 4), csw=csw)
    ctx = dd.Context(p, U)
    op = O.WilsonTM(U, dims, kappa=0.15, csw=csw)
    n_pair = 5                                    # 10 columns: two tiles, the second ragged
    mubar = np.linspace(0.01, 0.3, n_pair)
    epsbar = np.linspace(0.2, 0.02, n_pair)
    x = S.gaussian_spinors(2 * n_pair, V, 132).reshape(n_pair, 2, V, 4, 3)
    ref = O.nd_apply(op, x, mubar, epsbar)
    xg = torch.from_numpy(x).cuda()
    y64 = ctx.apply_op_nd(dd.FP64, mubar, epsbar, xg).cpu().numpy()
    y32 = ctx.apply_op_nd(dd.FP32, mubar, epsbar, xg).cpu().numpy()
    e64, e32 = np.max(pair_relerr(y64, ref)), np.max(pair_relerr(y32, ref))
    say(f"  FP64 {e64:.2e}, FP32 {e32:.2e}")
    assert e64 < 1e-13 and e32 < 2e-6
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_doublet_solve(torch_cuda, dd, precision):
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    say("doublet solve", w.name, "precision", precision)
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    V = w.volume
    ctx = dd.Context(dd.params_for_workload(w, precision=precision, coarse_gamma5=1, max_outer=400),
                     U, tv_init=S.setup_start_vectors(w))
    mubar = np.array([0.1, 0.15, 0.02])
    epsbar = np.array([0.05, 0.12, 0.01])
    b = S.gaussian_spinors(6, V, 133).reshape(3, 2, V, 4, 3)
    x, info, st = ctx.solve_nd(mubar, epsbar, torch.from_numpy(b).cuda())
    assert st == dd.OK
    xs = x.cpu().numpy()
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    r = b - O.nd_apply(op, xs, mubar, epsbar)
    rel = np.linalg.norm(r.reshape(3, -1), axis=1) / np.linalg.norm(b.reshape(3, -1), axis=1)
    err = np.array([info[2 * i]["err_vs_fp64"] for i in range(3)])
    say("  doublet residuals (oracle)", rel, "iters", [i["outer_iters"] for i in info])
    assert np.all(rel <= 1e-10 * (1 + 1e-6))
    assert np.max(np.abs(err - rel)) < 1e-13
    # the two columns of a doublet share their iteration count and residual
    for i in range(3):
        assert info[2 * i]["outer_iters"] == info[2 * i + 1]["outer_iters"]
        assert info[2 * i]["true_rel_res"] == info[2 * i + 1]["true_rel_res"]
    ctx.close()


def test_zero_coupling_solves_the_two_flavours(torch_cuda, dd):
    """epsbar = 0: the doublet decouples, so its solve gives D(+mubar)^-1 b_u
    and D(-mubar)^-1 b_d (checked by the degenerate oracle operator)."""
    torch = torch_cuda
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    V = w.volume
    ctx = dd.Context(dd.params_for_workload(w), U, tv_init=S.setup_start_vectors(w))
    b = S.gaussian_spinors(2, V, 134).reshape(1, 2, V, 4, 3)
    x, info, st = ctx.solve_nd([0.07], [0.0], torch.from_numpy(b).cuda())
    assert st == dd.OK
    xs = x.cpu().numpy()
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    nb = np.linalg.norm(b)
    for f, mu in ((0, 0.07), (1, -0.07)):
        r = b[0, f] - op.apply(xs[0, f][None], [mu])[0]
        assert np.linalg.norm(r) <= 1e-10 * nb * (1 + 1e-6)
    ctx.close()
