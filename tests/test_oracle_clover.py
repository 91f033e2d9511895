"""Pins of the oracle's clover term (Sheikholeslami-Wohlert form, the reading
taken for the twisted-mass clover ensembles the paper runs on) against facts
fixed by the mathematics, not by re-typing the oracle's formula:

* a constant abelian field in the x-y plane (flux quantised on the torus)
  gives the closed form (c_sw / 2) sin(theta) diag(1, -1, 1, -1) x diag(1, -1, 0)
  at every site (pins the leaf paths and orientation, the 1/8 and i/4 factors
  and the sign of sigma_{mu nu});
* the free field has no clover term;
* gauge covariance C[U^Omega](x) = Omega(x) C[U](x) Omega(x)^dagger (a leaf
  that is not a closed loop breaks it);
* Hermitian, traceless and block diagonal in chirality;
* with the clover term the full operator keeps gamma5-hermiticity and the
  singular-value shift sigma_i(D(mu))^2 = sigma_i(D(0))^2 + mu^2 (dense);
* the site-by-site loop evaluation agrees with the field form.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel


def dense(op, mu):
    V = op.V
    E = np.eye(V * 12, dtype=np.complex128).reshape(V * 12, V, 4, 3)
    return op.apply(E, np.full(V * 12, mu)).reshape(V * 12, V * 12).T


def abelian_field(dims, n_flux):
    """U_x(x, y) = D(-theta y), U_y(x, Ly - 1) = D(theta Ly x), all other links
    1, with D(a) = diag(e^{ia}, e^{-ia}, 1) and theta = 2 pi n / (Lx Ly): every
    x-y plaquette is D(theta), every other plaquette is 1."""
    Lx, Ly, Lz, Lt = dims
    V = S.volume(dims)
    theta = 2 * np.pi * n_flux / (Lx * Ly)
    x, y, z, t = S.site_coords(np.arange(V), dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()

    def D(a):
        out = np.zeros((len(a), 3, 3), dtype=np.complex128)
        out[:, 0, 0] = np.exp(1j * a)
        out[:, 1, 1] = np.exp(-1j * a)
        out[:, 2, 2] = 1.0
        return out

    U[:, 0] = D(-theta * y)
    edge = y == Ly - 1
    U[edge, 1] = D(theta * Ly * x[edge])
    return U, theta


@pytest.mark.parametrize("dims,n_flux", [((4, 6, 2, 4), 1), ((6, 4, 4, 2), 2)])
def test_abelian_closed_form(dims, n_flux):
    U, theta = abelian_field(dims, n_flux)
    csw = 1.7
    op = O.WilsonTM(U, dims, kappa=0.13, csw=csw)
    expect = 0.5 * csw * np.sin(theta) * np.kron(np.diag([1, -1, 1, -1]), np.diag([1, -1, 0]))
    C = op.clover.reshape(-1, 12, 12)
    assert np.max(np.abs(C - expect[None])) < 1e-14
    # the plaquette itself (an independent check of the constructed field)
    i = 5
    Lx = dims[0]
    p = U[i, 0] @ U[i + 1 if (i % Lx) < Lx - 1 else i + 1 - Lx, 1] @ np.conj(U[i + Lx, 0]).T @ np.conj(U[i, 1]).T
    assert np.allclose(p, np.diag([np.exp(1j * theta), np.exp(-1j * theta), 1]))


def test_free_field_has_no_clover():
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    op = O.WilsonTM(U, dims, kappa=0.13, csw=2.0)
    assert np.max(np.abs(op.clover)) == 0.0


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
    C = O.WilsonTM(U, dims, kappa=0.15, csw=1.1).clover.reshape(V, 4, 3, 4, 3)
    Cp = O.WilsonTM(Up, dims, kappa=0.15, csw=1.1).clover.reshape(V, 4, 3, 4, 3)
    rot = np.einsum("vab,vsbtc,vdc->vsatd", Om, C, np.conj(Om))
    assert np.max(np.abs(Cp - rot)) < 1e-14 * max(1.0, np.max(np.abs(C))) * 10


def test_hermitian_traceless_chiral():
    dims = (4, 4, 4, 4)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 25), dims, kappa=0.15, csw=1.3)
    C = op.clover.reshape(V, 12, 12)
    assert np.max(np.abs(C)) > 0.05
    assert np.max(np.abs(C - np.conj(np.transpose(C, (0, 2, 1))))) < 1e-15
    assert np.max(np.abs(np.trace(C, axis1=1, axis2=2))) < 1e-14
    assert np.max(np.abs(C[:, :6, 6:])) == 0.0 and np.max(np.abs(C[:, 6:, :6])) == 0.0


def test_operator_gamma5_hermiticity_and_singular_value_shift():
    dims = (2, 2, 2, 2)
    U = S.gauge_field(dims, 0.5, 26)
    op = O.WilsonTM(U, dims, kappa=0.14, csw=1.5)
    g5 = np.kron(np.eye(16), np.kron(O.gamma5(), np.eye(3)))
    mu = 0.3
    Dp, Dm, D0 = dense(op, mu), dense(op, -mu), dense(op, 0.0)
    assert np.max(np.abs(g5 @ Dp @ g5 - Dm.conj().T)) < 1e-14
    s0 = np.sort(np.linalg.svd(D0, compute_uv=False))
    s1 = np.sort(np.linalg.svd(Dp, compute_uv=False))
    assert np.max(np.abs(s1 ** 2 - (s0 ** 2 + mu ** 2))) < 1e-12
    # the clover term changes the operator (the checks above are not vacuous)
    assert np.max(np.abs(D0 - dense(O.WilsonTM(U, dims, kappa=0.14), 0.0))) > 0.05


def test_site_formula_matches_field():
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 27), dims, kappa=0.15, csw=1.2)
    psi = S.gaussian_spinors(2, V, 28)
    mus = np.array([0.01, 0.3])
    full = op.apply(psi, mus)
    sites = [0, 7, V - 1, V // 2 + 3]
    assert np.max(np.abs(op.apply_site(psi, mus, sites) - full[:, sites])) < 1e-13


def test_block_operator_includes_clover():
    """SAP's block operator D_BB with one block covering the lattice is D."""
    dims = (4, 4, 4, 4)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 29), dims, kappa=0.15, csw=1.0)
    lev = FineLevel(op)
    x = S.gaussian_spinors(2, V, 30).reshape(2, V, 12)
    mus = np.array([0.02, 0.4])
    # a 4^4 block on a 4^4 lattice wraps onto itself: every hop is internal
    y_blk = lev.apply_block_diag(x, mus, Blocking(dims, dims))
    y = lev.apply(x, mus)
    assert np.max(np.abs(y_blk - y)) < 1e-13 * np.max(np.abs(y))
