"""Pins of the oracle's interpolation and coarse-grid correction (section 2:
the interpolation is built from test vectors per aggregate, the coarse
operator is its Galerkin projection):

* the interpolation is the QR factor of the test vectors with a positive real
  diagonal: per aggregate and chirality, P^dagger T is upper triangular with a
  real positive diagonal and P (P^dagger T) = T (the test vectors T restricted
  there), so the order of the columns and their phases are fixed;
* the coarse-grid correction P D_c^-1 P^dagger does not depend on the basis:
  rotating the columns of P by an arbitrary unitary per aggregate and
  chirality leaves it unchanged, while the coarse blocks themselves change.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, build_prolongator, prolong, galerkin


def _setup(dims=(4, 4, 2, 4), agg=(2, 2, 2, 2), N=4, seed=51):
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, seed)
    op = O.WilsonTM(U, dims, kappa=0.13)
    tv = S.gaussian_spinors(N, V, seed + 1).reshape(N, V, 12)
    blk = Blocking(dims, agg)
    return V, op, FineLevel(op), blk, tv


def _dense_P(P, blk):
    V, d, N = P.shape
    nc = blk.nblocks * 2 * N
    E = np.eye(nc, dtype=np.complex128).reshape(nc, blk.nblocks, 2 * N)
    return prolong(P, blk, E).reshape(nc, V * d).T


def _dense(apply, n, shape):
    E = np.eye(n, dtype=np.complex128).reshape((n,) + shape)
    return apply(E).reshape(n, n).T


@pytest.mark.parametrize("agg", [(2, 2, 2, 2), (4, 2, 1, 2)])
def test_interpolation_is_the_positive_diagonal_qr_factor(agg):
    V, op, lev, blk, tv = _setup(agg=agg, N=5)
    P = build_prolongator(tv, blk)
    N = tv.shape[0]
    for a in range(blk.nblocks):
        sites = np.nonzero(blk.id == a)[0]
        for s in range(2):
            comp = np.arange(6 * s, 6 * s + 6)
            T = tv[:, sites][:, :, comp].reshape(N, -1).T         # (sites x 6) x N
            Pa = P[sites][:, comp, :].reshape(-1, N)             # (sites x 6) x N
            R = Pa.conj().T @ T
            assert np.max(np.abs(np.tril(R, -1))) < 1e-12 * np.max(np.abs(R))
            d = np.diagonal(R)
            assert np.all(d.real > 0) and np.max(np.abs(d.imag)) < 1e-12 * np.max(d.real)
            assert np.max(np.abs(Pa @ R - T)) < 1e-12 * np.max(np.abs(T))


def test_coarse_grid_correction_is_basis_independent():
    V, op, lev, blk, tv = _setup()
    N = tv.shape[0]
    P = build_prolongator(tv, blk)
    rng = np.random.default_rng(53)
    # P -> P W with a random unitary W per aggregate and chirality
    P2 = P.copy()
    for a in range(blk.nblocks):
        sites = np.nonzero(blk.id == a)[0]
        for s in range(2):
            W, _ = np.linalg.qr(rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)))
            comp = slice(6 * s, 6 * s + 6)
            P2[sites, comp, :] = P[sites, comp, :] @ W
    mu = 0.05
    nc = blk.nblocks * 2 * N
    out = []
    for Pb in (P, P2):
        coarse = galerkin(lev, Pb, blk)
        Dc = _dense(lambda E: coarse.apply(E, np.full(E.shape[0], mu)), nc, (blk.nblocks, 2 * N))
        Pd = _dense_P(Pb, blk)
        out.append((Dc, Pd @ np.linalg.solve(Dc, Pd.conj().T)))
    (Dc1, C1), (Dc2, C2) = out
    assert np.max(np.abs(Dc1 - Dc2)) > 1e-3 * np.max(np.abs(Dc1))      # the blocks did change
    assert np.max(np.abs(C1 - C2)) < 1e-11 * np.max(np.abs(C1))
