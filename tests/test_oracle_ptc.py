"""Pins of the oracle's parallel-transport convolution smoother:

* one layer with Wilson weights reproduces the twisted-mass operator exactly
  (a different code path: transport + spin matrices, not projectors);
* gauge covariance f(Omega r; U^Omega) = Omega f(r; U);
* linearity in the input;
* the input-gradient layer is the adjoint of the layer (dot-product test);
* weight gradients agree with central finite differences in FP64.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle import ptc


def setup(dims=(2, 2, 4, 4), seed=51):
    U = S.gauge_field(dims, 0.4, seed)
    return O.WilsonTM(U, dims, kappa=0.15), U, S.volume(dims)


def test_single_layer_is_the_dirac_operator():
    op, U, V = setup((4, 2, 4, 6))
    x = S.gaussian_spinors(2, V, 3)
    for mu in (0.0, 0.2):
        W = ptc.dslash_weights(op.m0, mu)
        y = ptc.ptc_layer(op, W, x[None])[0]
        ref = op.apply(x, [mu, mu])
        assert np.max(np.abs(y - ref)) < 1e-13 * np.max(np.abs(ref))


def test_gauge_covariance():
    dims = (2, 4, 2, 4)
    op, U, V = setup(dims)
    Om = S.random_su3(V, 9)
    x_, y_, z_, t_ = S.site_coords(np.arange(V), dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c = [x_, y_, z_, t_]
        c[mu] = (c[mu] + 1) % dims[mu]
        j = S.site_index(*c, dims)
        Up[:, mu] = Om @ U[:, mu] @ np.conj(np.transpose(Om[j], (0, 2, 1)))
    opp = O.WilsonTM(Up, dims, kappa=0.15)
    W1, W2 = ptc.random_weights(2, 1, 1), ptc.random_weights(1, 2, 2)
    r = S.gaussian_spinors(2, V, 4)
    a, _ = ptc.smoother_forward(opp, W1, W2, np.einsum("vab,nvsb->nvsa", Om, r))
    b, _ = ptc.smoother_forward(op, W1, W2, r)
    b = np.einsum("vab,nvsb->nvsa", Om, b)
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_linearity():
    op, U, V = setup()
    W1, W2 = ptc.random_weights(2, 1, 5), ptc.random_weights(1, 2, 6)
    r1, r2 = S.gaussian_spinors(1, V, 7), S.gaussian_spinors(1, V, 8)
    a, b = 0.3 - 1.2j, 2.0 + 0.5j
    f = lambda r: ptc.smoother_forward(op, W1, W2, r)[0]
    assert np.max(np.abs(f(a * r1 + b * r2) - (a * f(r1) + b * f(r2)))) < 1e-12


def test_input_gradient_is_adjoint():
    op, U, V = setup()
    W = ptc.random_weights(2, 1, 10)
    x = S.gaussian_spinors(1, V, 11)[None]
    y = np.stack([S.gaussian_spinors(1, V, 12), S.gaussian_spinors(1, V, 13)])
    lhs = np.vdot(ptc.ptc_layer(op, W, x), y)
    rhs = np.vdot(x, ptc.ptc_layer_input_grad(op, W, y))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_weight_gradients_match_finite_differences():
    op, U, V = setup((2, 2, 2, 4))
    W1, W2 = ptc.random_weights(2, 1, 14, 0.3), ptc.random_weights(1, 2, 15, 0.3)
    r = S.gaussian_spinors(2, V, 16)
    e = S.gaussian_spinors(2, V, 17)
    loss, g1, g2 = ptc.smoother_loss_and_grads(op, W1, W2, r, e)
    rng = np.random.default_rng(0)
    h = 1e-6
    for which, W, g in ((1, W1, g1), (2, W2, g2)):
        for _ in range(6):
            idx = tuple(int(rng.integers(0, n)) for n in W.shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                Wp, Wm = W.copy(), W.copy()
                Wp[idx] += h * unit
                Wm[idx] -= h * unit
                args_p = (Wp, W2) if which == 1 else (W1, Wp)
                args_m = (Wm, W2) if which == 1 else (W1, Wm)
                lp = ptc.smoother_loss_and_grads(op, *args_p, r, e)[0]
                lm = ptc.smoother_loss_and_grads(op, *args_m, r, e)[0]
                fd = (lp - lm) / (2 * h)
                an = g[idx].real if part == 0 else g[idx].imag
                assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (which, idx, part, fd, an)
