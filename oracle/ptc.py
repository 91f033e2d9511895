"""Oracle: gauge-covariant parallel-transport convolution (PTC) network, FP64.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

A PTC layer maps C_in spinor channels to C_out channels:

    out_o(x) = sum_i sum_p W[p, o, i] (T_p in_i)(x)

over the nine paths p = 0 (identity), +x, +y, +z, +t, -x, -y, -z, -t with
    T_{+nu} phi(x) = U_nu(x) phi(x + nu),  T_{-nu} phi(x) = U_nu(x - nu)^dag phi(x - nu)
(the antiperiodic time sign included) and W[p, o, i] a complex 4x4 matrix
acting on spin only, so the layer commutes with gauge transformations.
The smoother is two layers, 1 -> 2 -> 1 channels, without activation: a
linear operator in its input.  One layer with W[0] = (4+m0) + i mu gamma5,
W[+nu] = -(1 - gamma_nu)/2, W[-nu] = -(1 + gamma_nu)/2 is the twisted-mass
Wilson operator itself.

Weights: complex128 array [9][C_out][C_in][4][4].  Vectors [n][V][4][3].
Gradients follow g = dL/dRe W + i dL/dIm W for a real loss L.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonTM, gammas, gamma5

__all__ = ["transport", "transport_adjoint_path", "ptc_layer", "ptc_layer_input_grad", "ptc_layer_weight_grad",
           "smoother_forward", "smoother_loss_and_grads", "dslash_weights", "random_weights"]


def transport(op: WilsonTM, phi, p):
    """T_p phi for path p (0 = identity, 1..4 = +mu, 5..8 = -mu), phi [n][V][4][3]."""
    if p == 0:
        return phi.copy()
    lat = op.to_lat(phi)
    mu = (p - 1) % 4
    fwd = p <= 4
    # the hop terms of the operator apply the projector; here only the transport
    ax = 1 + (3 - mu)
    nb = np.roll(lat, -1 if fwd else 1, axis=ax)
    if mu == 3:
        nb = nb * (op.bc_fwd if fwd else op.bc_bwd)[None, ..., None, None]
    if fwd:
        U = op.U[mu][None]
        out = np.einsum("...ab,...sb->...sa", U, nb)
    else:
        Ub = np.roll(op.U[mu], 1, axis=3 - mu)[None]
        out = np.einsum("...ba,...sb->...sa", np.conj(Ub), nb)
    return op.from_lat(out)


def transport_adjoint_path(p):
    """T_p^dagger = T_{p'}: the opposite path."""
    if p == 0:
        return 0
    return p + 4 if p <= 4 else p - 4


def ptc_layer(op, W, inp):
    """inp: [C_in][n][V][4][3] -> out [C_out][n][V][4][3]."""
    n_p, cout, cin = W.shape[:3]
    out = np.zeros((cout,) + inp.shape[1:], dtype=np.complex128)
    for p in range(9):
        for i in range(cin):
            t = transport(op, inp[i], p)
            for o in range(cout):
                out[o] += np.einsum("st,nvtc->nvsc", W[p, o, i], t)
    return out


def ptc_layer_input_grad(op, W, gout):
    """Adjoint of the layer applied to the output gradient:
    gin_i = sum_p T_p^dag (sum_o W[p,o,i]^dag gout_o)."""
    n_p, cout, cin = W.shape[:3]
    gin = np.zeros((cin,) + gout.shape[1:], dtype=np.complex128)
    for p in range(9):
        pa = transport_adjoint_path(p)
        for o in range(cout):
            t = transport(op, gout[o], pa)
            for i in range(cin):
                gin[i] += np.einsum("ts,nvtc->nvsc", np.conj(W[p, o, i]), t)
    return gin


def ptc_layer_weight_grad(op, inp, gout):
    """g[p,o,i][s,t] = 2 sum_{n,x,c} gout_o[s,c] conj((T_p inp_i)[t,c]) where
    gout = dL/d conj(out)."""
    cout, cin = gout.shape[0], inp.shape[0]
    g = np.zeros((9, cout, cin, 4, 4), dtype=np.complex128)
    for p in range(9):
        for i in range(cin):
            t = transport(op, inp[i], p)
            for o in range(cout):
                g[p, o, i] = 2.0 * np.einsum("nvsc,nvtc->st", gout[o], np.conj(t))
    return g


def smoother_forward(op, W1, W2, r):
    """f(r) = L2(L1(r)), r [n][V][4][3]."""
    h = ptc_layer(op, W1, r[None])
    return ptc_layer(op, W2, h)[0], h


def smoother_loss_and_grads(op, W1, W2, r, e):
    """Loss sum_c ||f(r_c) - e_c||^2 / ||e_c||^2 and its weight gradients."""
    y, h = smoother_forward(op, W1, W2, r)
    en = np.sum(np.abs(e.reshape(e.shape[0], -1)) ** 2, axis=1)
    d = y - e
    loss = float(np.sum(np.sum(np.abs(d.reshape(d.shape[0], -1)) ** 2, axis=1) / en))
    gy = d / en[:, None, None, None]            # dL/d conj(y)
    g2 = ptc_layer_weight_grad(op, h, gy[None])
    gh = ptc_layer_input_grad(op, W2, gy[None])
    g1 = ptc_layer_weight_grad(op, r[None], gh)
    return loss, g1, g2


def dslash_weights(m0, mu):
    """Single-layer weights that reproduce D(mu): [9][1][1][4][4]."""
    g = gammas()
    one = np.eye(4)
    W = np.zeros((9, 1, 1, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = (4.0 + m0) * one + 1j * mu * gamma5()
    for nu in range(4):
        W[1 + nu, 0, 0] = -0.5 * (one - g[nu])
        W[5 + nu, 0, 0] = -0.5 * (one + g[nu])
    return W


def random_weights(cout, cin, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    return scale * (rng.standard_normal((9, cout, cin, 4, 4)) + 1j * rng.standard_normal((9, cout, cin, 4, 4)))
