"""Pins of the oracle's twisted-mass Wilson operator against facts fixed by the
mathematics (not by re-typing the oracle's formula):

* Clifford algebra and gamma5 = diag(1, 1, -1, -1) of the chiral basis;
* free field: a plane wave with antiperiodic time momentum is mapped to
  [M(p) + i sum_nu gamma_nu sin p_nu + i mu gamma5] times itself, pointwise
  (pins the projector sign, the 4 + m0 diagonal, the twist and the boundary);
* gamma5-hermiticity gamma5 D(mu) gamma5 = D(-mu)^dagger, dense on 2^4;
* gauge covariance D[U^Omega] Omega psi = Omega D[U] psi (pins link placement
  and daggers);
* singular-value shift sigma_i(D(mu))^2 = sigma_i(D(0))^2 + mu^2 (dense).
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O


def dense(op, mu):
    V = op.V
    E = np.eye(V * 12, dtype=np.complex128).reshape(V * 12, V, 4, 3)
    return op.apply(E, np.full(V * 12, mu)).reshape(V * 12, V * 12).T


def test_gamma_algebra():
    g = O.gammas()
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            ac = g[a] @ g[b] + g[b] @ g[a]
            assert np.allclose(ac, 2 * np.eye(4) * (a == b))
    assert np.allclose(O.gamma5(), np.diag([1, 1, -1, -1]))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 4, 6, 8)])
@pytest.mark.parametrize("mu", [0.0, 0.37])
def test_free_field_plane_wave(dims, mu):
    V = S.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    kappa = 0.13
    op = O.WilsonTM(U, dims, kappa=kappa)
    m0 = 1 / (2 * kappa) - 4
    rng = np.random.default_rng(5)
    i = np.arange(V)
    x, y, z, t = S.site_coords(i, dims)
    g = O.gammas()
    for trial in range(3):
        n = [int(rng.integers(0, d)) for d in dims]
        p = [2 * np.pi * n[k] / dims[k] for k in range(3)] + [(2 * n[3] + 1) * np.pi / dims[3]]
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        psi = phase[:, None, None] * u[None]
        out = op.apply(psi[None], [mu])[0]
        M = m0 + sum(1 - np.cos(pk) for pk in p)
        K = M * np.eye(4) + 1j * sum(g[k] * np.sin(p[k]) for k in range(4)) + 1j * mu * O.gamma5()
        expect = phase[:, None, None] * (K @ u)[None]
        assert np.max(np.abs(out - expect)) < 1e-12


def test_free_field_eigenvalues():
    """Eigenvalues M(p) +- i sqrt(sum sin^2 p + mu^2), each with multiplicity 6."""
    dims = (2, 2, 2, 4)
    V = S.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    mu = 0.2
    op = O.WilsonTM(U, dims, m0=-0.3)
    ev = np.linalg.eigvals(dense(op, mu))
    expect = []
    for nx in range(2):
        for ny in range(2):
            for nz in range(2):
                for nt in range(4):
                    p = [np.pi * nx, np.pi * ny, np.pi * nz, (2 * nt + 1) * np.pi / 4]
                    M = -0.3 + sum(1 - np.cos(q) for q in p)
                    w = np.sqrt(sum(np.sin(q) ** 2 for q in p) + mu ** 2)
                    expect += [M + 1j * w] * 6 + [M - 1j * w] * 6
    expect = np.array(expect)
    key = lambda a: np.lexsort((np.round(a.imag, 8), np.round(a.real, 8)))
    assert np.max(np.abs(ev[key(ev)] - expect[key(expect)])) < 1e-10


def test_gamma5_hermiticity_dense():
    dims = (2, 2, 2, 2)
    U = S.gauge_field(dims, 0.5, 11)
    op = O.WilsonTM(U, dims, kappa=0.14)
    g5 = np.kron(np.eye(16), np.kron(O.gamma5(), np.eye(3)))
    for mu in (0.0, 0.3):
        Dp = dense(op, mu)
        Dm = dense(op, -mu)
        assert np.max(np.abs(g5 @ Dp @ g5 - Dm.conj().T)) < 1e-14


def test_gamma5_hermiticity_random_vectors():
    dims = (4, 4, 4, 8)
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, 12)
    op = O.WilsonTM(U, dims, kappa=0.15)
    phi = S.gaussian_spinors(2, V, 1)
    psi = S.gaussian_spinors(2, V, 2)
    mus = np.array([0.01, 0.2])
    lhs = np.vdot(phi[0], op.gamma5_apply(op.apply(op.gamma5_apply(psi), mus))[0])
    rhs = np.vdot(op.apply(phi, -mus)[0], psi[0])
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gauge_covariance():
    dims = (4, 2, 4, 6)
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.4, 13)
    Om = S.random_su3(V, 14)
    Lx, Ly, Lz, Lt = dims
    i = np.arange(V)
    x, y, z, t = S.site_coords(i, dims)
    Up = np.empty_like(U)
    for mu in range(4):
        c = [x, y, z, t]
        c[mu] = (c[mu] + 1) % dims[mu]
        j = S.site_index(*c, dims)
        Up[:, mu] = Om @ U[:, mu] @ np.conj(np.transpose(Om[j], (0, 2, 1)))
    psi = S.gaussian_spinors(2, V, 15)
    psi_p = np.einsum("vab,nvsb->nvsa", Om, psi)
    mus = np.array([0.05, 0.5])
    a = O.WilsonTM(Up, dims, kappa=0.15).apply(psi_p, mus)
    b = np.einsum("vab,nvsb->nvsa", Om, O.WilsonTM(U, dims, kappa=0.15).apply(psi, mus))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))


def test_singular_value_shift():
    dims = (2, 2, 2, 2)
    U = S.gauge_field(dims, 0.5, 16)
    op = O.WilsonTM(U, dims, kappa=0.15)
    s0 = np.sort(np.linalg.svd(dense(op, 0.0), compute_uv=False))
    mu = 0.21
    s1 = np.sort(np.linalg.svd(dense(op, mu), compute_uv=False))
    assert np.max(np.abs(s1 ** 2 - (s0 ** 2 + mu ** 2))) < 1e-12
    assert s1.min() >= mu - 1e-14


def test_site_sampler_matches_field():
    dims = (4, 4, 2, 4)
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, 17)
    op = O.WilsonTM(U, dims, kappa=0.15)
    psi = S.gaussian_spinors(2, V, 18)
    mus = np.array([0.01, 0.3])
    full = op.apply(psi, mus)
    sites = [0, 5, V - 1, V // 2 + 3]
    assert np.max(np.abs(op.apply_site(psi, mus, sites) - full[:, sites])) < 1e-13
