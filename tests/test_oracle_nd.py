"""Pins of the oracle's non-degenerate twisted-mass doublet operator
D_ND = D_W (x) 1 + i mubar gamma5 (x) tau3 - epsbar (x) tau1 against facts
fixed by the mathematics:

* free field: a plane wave times a constant spin-colour-flavour vector u is
  mapped to the same wave times A(p) u, A(p) = M(p) + i sum_nu gamma_nu
  sin p_nu + i mubar gamma5 tau3 - epsbar tau1, pointwise (pins the flavour
  structure, the signs of the twist and of epsbar, the boundary);
* free-field spectrum (derived: (A - M)^2 = (epsbar^2 - s^2 - mubar^2) -
  2 i epsbar (gamma.s) tau1, whose factor (gamma.s) tau1 has eigenvalues
  +-|s|): eigenvalues M(p) +- sqrt((epsbar -+ i |s|)^2 - mubar^2), each six
  times (spin-flavour 2, colour 3), dense on 2^3 x 4;
* gamma5 tau1-hermiticity: (gamma5 tau1) D_ND (gamma5 tau1) = D_ND^dagger,
  dense on 2^4 with a random gauge field;
* gauge covariance D_ND[U^Omega] Omega psi = Omega D_ND[U] psi;
* epsbar = 0: the two flavours decouple (u sees +mubar, d sees -mubar).
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O


def dense_nd(op, mubar, epsbar):
    n = 2 * op.V * 12
    E = np.eye(n, dtype=np.complex128).reshape(n, 2, op.V, 4, 3)
    cols = []
    for k in range(n):
        cols.append(O.nd_apply(op, E[k][None], [mubar], [epsbar]).reshape(-1))
    return np.array(cols).T


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
def test_free_field_plane_wave(dims):
    V = S.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    kappa = 0.13
    op = O.WilsonTM(U, dims, kappa=kappa)
    m0 = 1 / (2 * kappa) - 4
    rng = np.random.default_rng(7)
    x, y, z, t = S.site_coords(np.arange(V), dims)
    g = O.gammas()
    t1 = np.array([[0, 1], [1, 0]])
    t3 = np.diag([1.0, -1.0])
    for trial in range(3):
        mubar, epsbar = rng.uniform(0.01, 0.5), rng.uniform(0.01, 0.5)
        n = [int(rng.integers(0, d)) for d in dims]
        p = [2 * np.pi * n[k] / dims[k] for k in range(3)] + [(2 * n[3] + 1) * np.pi / dims[3]]
        u = rng.standard_normal((2, 4, 3)) + 1j * rng.standard_normal((2, 4, 3))    # [flavour][spin][colour]
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        psi = phase[None, :, None, None] * u[:, None]                             # [2][V][4][3]
        out = O.nd_apply(op, psi[None], [mubar], [epsbar])[0]
        M = m0 + sum(1 - np.cos(pk) for pk in p)
        # A(p) on (flavour, spin): kron(tau, spin) ordering [f][s]
        A = (M * np.eye(8) + 1j * np.kron(np.eye(2), sum(g[k] * np.sin(p[k]) for k in range(4)))
             + 1j * mubar * np.kron(t3, O.gamma5()) - epsbar * np.kron(t1, np.eye(4)))
        Au = np.einsum("ab,bc->ac", A, u.reshape(8, 3)).reshape(2, 4, 3)
        expect = phase[None, :, None, None] * Au[:, None]
        assert np.max(np.abs(out - expect)) < 1e-12


def test_free_field_spectrum_closed_form():
    dims = (2, 2, 2, 4)
    V = S.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    m0, mubar, epsbar = -0.3, 0.17, 0.23
    op = O.WilsonTM(U, dims, m0=m0)
    ev = np.linalg.eigvals(dense_nd(op, mubar, epsbar))
    expect = []
    for nx in range(2):
        for ny in range(2):
            for nz in range(2):
                for nt in range(4):
                    p = [np.pi * nx, np.pi * ny, np.pi * nz, (2 * nt + 1) * np.pi / 4]
                    M = m0 + sum(1 - np.cos(q) for q in p)
                    a = np.sqrt(sum(np.sin(q) ** 2 for q in p))
                    for sg in (1, -1):
                        z = np.sqrt((epsbar - 1j * sg * a) ** 2 - mubar ** 2 + 0j)
                        expect += [M + z] * 6 + [M - z] * 6
    expect = np.array(expect)
    assert len(expect) == len(ev)
    # multiset comparison: every eigenvalue matches one of the predicted ones
    # and the counts agree after rounding
    key = lambda a: np.lexsort((np.round(a.imag, 7), np.round(a.real, 7)))
    assert np.max(np.abs(ev[key(ev)] - expect[key(expect)])) < 1e-9


def test_gamma5_tau1_hermiticity_dense():
    dims = (2, 2, 2, 2)
    U = S.gauge_field(dims, 0.5, 21)
    op = O.WilsonTM(U, dims, kappa=0.14)
    V = op.V
    G = np.kron(np.array([[0, 1], [1, 0]]), np.kron(np.eye(V), np.kron(O.gamma5(), np.eye(3))))
    for mubar, epsbar in ((0.0, 0.1), (0.3, 0.2)):
        D = dense_nd(op, mubar, epsbar)
        assert np.max(np.abs(G @ D @ G - D.conj().T)) < 1e-14


def test_gauge_covariance():
    dims = (4, 2, 4, 6)
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.4, 23)
    Om = S.random_su3(V, 24)
    x, y, z, t = S.site_coords(np.arange(V), dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c = [x, y, z, t]
        c[mu] = (c[mu] + 1) % dims[mu]
        j = S.site_index(*c, dims)
        Up[:, mu] = Om @ U[:, mu] @ np.conj(np.transpose(Om[j], (0, 2, 1)))
    psi = S.gaussian_spinors(4, V, 25).reshape(2, 2, V, 4, 3)
    mubar, epsbar = np.array([0.05, 0.4]), np.array([0.2, 0.07])
    psi_p = np.einsum("vab,nfvsb->nfvsa", Om, psi)
    a = O.nd_apply(O.WilsonTM(Up, dims, kappa=0.15), psi_p, mubar, epsbar)
    b = np.einsum("vab,nfvsb->nfvsa", Om, O.nd_apply(O.WilsonTM(U, dims, kappa=0.15), psi, mubar, epsbar))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_zero_epsbar_decouples_flavours():
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 26), dims, kappa=0.15)
    psi = S.gaussian_spinors(2, V, 27).reshape(1, 2, V, 4, 3)
    y = O.nd_apply(op, psi, [0.11], [0.0])
    assert np.max(np.abs(y[0, 0] - op.apply(psi[:, 0], [0.11])[0])) < 1e-14
    assert np.max(np.abs(y[0, 1] - op.apply(psi[:, 1], [-0.11])[0])) < 1e-14
