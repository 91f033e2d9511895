"""GPU parity and behaviour of the learned PTC smoother, through the C ABI.

The device stores weights in BF16 and accumulates in FP32; the oracle is fed
the same BF16-rounded weights in FP64, so the bar is FP32 rounding (1e-5
relative for the layers and the smoother, 1e-4 for the weight gradients,
whose site sums are FP32 per lane).  Training, the use inside FGMRES and
the SAP fallback are checked on the 4^4 and 8^4 lattices (training on two
gauge fields, evaluation on a third).
"""
import sys

import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle import ptc as OP

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.asarray(a, dtype=np.float64)
    f = a.astype(np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    f = ((f + 0x7FFF + lsb) >> 16) << 16
    return f.astype(np.uint32).view(np.float32).astype(np.float64)


def cbf16(w):
    return bf16(w.real) + 1j * bf16(w.imag)


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


def ctx_for(dd, dims, **kw):
    U = S.gauge_field(dims, 0.3, 81)
    p = dd.default_params(dims=dims, kappa=0.15, n_levels=1, sap_block=(2, 2, 2, 2), **kw)
    return dd.Context(p, U), U


def relmax(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_layers_and_gradients(torch_cuda, dd):
    torch = torch_cuda
    dims = (4, 4, 4, 8)
    V = S.volume(dims)
    say("ptc layers", dims)
    ctx, U = ctx_for(dd, dims)
    op = O.WilsonTM(U, dims, kappa=0.15)
    W1, W2 = cbf16(OP.random_weights(2, 1, 3, 0.3)), cbf16(OP.random_weights(1, 2, 4, 0.3))
    ctx.set_smoother_weights(W1, W2)
    ncol = 11
    x = S.gaussian_spinors(ncol, V, 5)
    xg = torch.from_numpy(x[None].copy()).cuda()
    h = ctx.ptc_layer(1, False, xg).cpu().numpy()
    h_ref = OP.ptc_layer(op, W1, x[None])
    assert relmax(h, h_ref) < 1e-5
    y = ctx.ptc_layer(2, False, torch.from_numpy(h_ref).cuda()).cpu().numpy()
    assert relmax(y, OP.ptc_layer(op, W2, h_ref)) < 1e-5
    # adjoint layers
    g = S.gaussian_spinors(ncol, V, 6)[None]
    a2 = ctx.ptc_layer(2, True, torch.from_numpy(g.copy()).cuda()).cpu().numpy()
    assert relmax(a2, OP.ptc_layer_input_grad(op, W2, g)) < 1e-5
    g2 = np.stack([S.gaussian_spinors(ncol, V, 7), S.gaussian_spinors(ncol, V, 8)])
    a1 = ctx.ptc_layer(1, True, torch.from_numpy(g2).cuda()).cpu().numpy()
    assert relmax(a1, OP.ptc_layer_input_grad(op, W1, g2)) < 1e-5
    # weight gradients
    G1 = ctx.ptc_weight_grad(1, xg, torch.from_numpy(g2).cuda())
    assert relmax(G1, OP.ptc_layer_weight_grad(op, x[None], g2)) < 1e-4
    G2 = ctx.ptc_weight_grad(2, torch.from_numpy(h_ref).cuda(), torch.from_numpy(g.copy()).cuda())
    assert relmax(G2, OP.ptc_layer_weight_grad(op, h_ref, g)) < 1e-4
    # the whole smoother
    f = ctx.smoother_apply(torch.from_numpy(x).cuda()).cpu().numpy()
    assert relmax(f, OP.smoother_forward(op, W1, W2, x)[0]) < 1e-5
    ctx.close()


def jacobi_init(m0):
    """f(r) = r / (4 + m0) plus a small perturbation of the second channel."""
    W1 = np.zeros((9, 2, 1, 4, 4), dtype=np.complex128)
    W2 = np.zeros((9, 1, 2, 4, 4), dtype=np.complex128)
    W1[0, 0, 0] = np.eye(4)
    W1[0, 1, 0] = 0.01 * np.eye(4)
    W2[0, 0, 0] = np.eye(4) / (4 + m0)
    W2[0, 0, 1] = 0.01 * np.eye(4)
    return W1, W2


def test_training_reduces_loss_and_helps_on_a_held_out_field(torch_cuda, dd):
    """Train on two 8^4 gauge fields, solve on a third one (gauge covariance
    makes the weights field-independent): the trained net must cut the outer
    iterations of the untrained one; SAP is reported beside it."""
    torch = torch_cuda
    w = S.workload("tm_8x8x8x8_3level")
    say("train + solve", w.name)
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    mus = np.array(w.mus)
    base = dict(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block, outer_restart=30, max_outer=2000,
                precision=dd.MIXED, sap_cycles=1, sap_mr_iters=8)
    m0 = 1 / (2 * w.kappa) - 4
    weights = jacobi_init(m0)
    for k, seed in enumerate((3101, 3102)):
        ctx = dd.Context(dd.default_params(**base), S.gauge_field(w.dims, w.eps, seed))
        ctx.set_smoother_weights(*weights)
        hist = ctx.train_smoother(mus, steps=200, batch=16, lr=2e-3, sap_sweeps=2, seed=5 + k)
        say(f"  seed {seed}: loss first/last {hist[:5].mean():.4f} {hist[-5:].mean():.4f}")
        if k == 0:   # the second field continues from trained weights
            assert hist[-6:].mean() < 0.9 * hist[:6].mean()
        weights = ctx.smoother_weights()
        ctx.close()
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    ctx = dd.Context(dd.default_params(smoother=dd.SMOOTHER_LEARNED, smoother_cycles=4, **base), U)
    ctx.set_smoother_weights(*jacobi_init(m0))
    _, info0, _ = ctx.solve(mus, b)
    it0 = max(i["outer_iters"] for i in info0)
    ctx.set_smoother_weights(*weights)
    x, info1, st1 = ctx.solve(mus, b)
    it1 = max(i["outer_iters"] for i in info1)
    fb = ctx.stats()["learned_fallbacks"]
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    bb = np.repeat(S.rhs_for(w), len(mus), axis=0)
    rel = O.col_norm(bb - op.apply(x.cpu().numpy(), np.tile(mus, w.n_rhs))) / O.col_norm(bb)
    sap = dd.Context(dd.default_params(smoother=dd.SMOOTHER_SAP, **base), U)
    _, info_s, _ = sap.solve(mus, b)
    it_s = max(i["outer_iters"] for i in info_s)
    say(f"  held-out field: outer iterations untrained {it0}, trained {it1} ({fb} fallbacks), SAP(1,8) {it_s}")
    assert st1 == dd.OK and np.all(rel <= 1e-10 * (1 + 1e-6))
    assert it1 < 0.8 * it0
    ctx.close()
    sap.close()


def test_fallback_to_sap_when_the_network_fails(torch_cuda, dd):
    torch = torch_cuda
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    say("fallback", w.name)
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block,
                          smoother=dd.SMOOTHER_LEARNED, precision=dd.MIXED)
    ctx = dd.Context(p, U)
    W1, W2 = jacobi_init(1 / (2 * w.kappa) - 4)
    ctx.set_smoother_weights(W1, -20.0 * W2)          # a net that amplifies the residual
    b = torch.from_numpy(S.rhs_for(w)).cuda()
    x, info, st = ctx.solve(np.array(w.mus), b)
    assert st == dd.OK
    assert ctx.stats()["learned_fallbacks"] > 0
    # every column was in flight while the net failed: each records fallbacks
    assert all(i["fallbacks"] > 0 for i in info)
    op = O.WilsonTM(U, w.dims, kappa=w.kappa)
    bb = np.repeat(S.rhs_for(w), 3, axis=0)
    rel = O.col_norm(bb - op.apply(x.cpu().numpy(), np.tile(np.array(w.mus), 2))) / O.col_norm(bb)
    assert np.all(rel <= 1e-10 * (1 + 1e-6))
    ctx.close()


def test_learned_smoother_requires_weights(dd, torch_cuda):
    torch = torch_cuda
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block, smoother=dd.SMOOTHER_LEARNED)
    ctx = dd.Context(p, U)
    with pytest.raises(dd.DDAMGError) as e:
        ctx.solve(np.array(w.mus), torch.from_numpy(S.rhs_for(w)).cuda())
    assert e.value.code == dd.ESTATE
    ctx.close()


def test_smoother_file_round_trip_and_rejection(torch_cuda, dd, tmp_path):
    """ddamg_save_smoother / ddamg_load_smoother: a saved net loads back into
    another context bit for bit (the file holds the FP64 master weights); a
    foreign, short or missing file is rejected and leaves the weights alone."""
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = dd.default_params(dims=w.dims, kappa=w.kappa, n_levels=1, sap_block=w.sap_block)
    a, b = dd.Context(p, U), dd.Context(p, U)
    rng = np.random.default_rng(5)
    W1 = rng.standard_normal((9, 2, 1, 4, 4)) + 1j * rng.standard_normal((9, 2, 1, 4, 4))
    W2 = rng.standard_normal((9, 1, 2, 4, 4)) + 1j * rng.standard_normal((9, 1, 2, 4, 4))
    a.set_smoother_weights(W1, W2)
    f = tmp_path / "net.ddamg"
    a.save_smoother(str(f))
    assert f.stat().st_size == 8 + 4 + 2 * 288 * 16
    b.load_smoother(str(f))
    V1, V2 = b.smoother_weights()
    assert np.array_equal(V1, a.smoother_weights()[0]) and np.array_equal(V2, a.smoother_weights()[1])
    raw = f.read_bytes()
    for bad, why in ((b"XXXXXXXX" + raw[8:], "not a smoother file"), (raw[:100], "short"),
                     (raw + b"\0", "trailing")):
        g = tmp_path / "bad.ddamg"
        g.write_bytes(bad)
        with pytest.raises(dd.DDAMGError) as e:
            b.load_smoother(str(g))
        assert e.value.code == dd.EINVAL and why in str(e.value)
    with pytest.raises(dd.DDAMGError):
        b.load_smoother(str(tmp_path / "missing.ddamg"))
    assert np.array_equal(b.smoother_weights()[0], V1)
    a.close()
    b.close()
