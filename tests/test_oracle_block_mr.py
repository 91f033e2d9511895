"""Pins of the oracle's SAP block solvers at a finite number of MR steps
(section 2: the block systems of the Schwarz method are solved approximately
by a few minimal-residual steps), against the dense operator:

* plain block MR: every block B of every colour takes, per step, the step
  length alpha_B minimising ||rho_B - alpha D_BB rho_B|| (a one-column least
  squares on the dense block matrix D_BB, the full operator's submatrix over
  the block's sites), and rho_B, delta_B follow;
* odd-even block MR: the Schur complement S = D_oo - D_oe D_ee^-1 D_eo and
  the right-hand side r_o - D_oe D_ee^-1 r_e formed from the dense block
  matrix split by site parity, MR steps with least-squares step lengths on
  S, then x_e = D_ee^-1 (r_e - D_eo x_o);
* with both colours, one SAP cycle of k steps equals the two-colour
  Schwarz sweep with these k-step block solves.

The step counts are small (1-3), where a wrong step length (a missing
conjugate, a numerator and denominator swapped) changes the result, unlike
the converged comparisons with exact block inverses.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, site_parity

DIMS, BLOCK = (4, 4, 2, 2), (2, 2, 2, 2)


def _dense(op, V, mu):
    E = np.eye(V * 12, dtype=np.complex128).reshape(V * 12, V, 4, 3)
    return op.apply(E, np.full(V * 12, mu)).reshape(V * 12, V * 12).T


def _setup(kappa=0.12, seed=41):
    V = S.volume(DIMS)
    U = S.gauge_field(DIMS, 0.3, seed)
    op = O.WilsonTM(U, DIMS, kappa=kappa)
    return V, op, FineLevel(op), Blocking(DIMS, BLOCK)


def _block_idx(blk, b):
    return (np.nonzero(blk.id == b)[0][:, None] * 12 + np.arange(12)).reshape(-1)


def _mr_dense(A, r, k):
    """k MR steps on A x = r from zero, each step length by least squares."""
    x = np.zeros_like(r)
    rho = r.copy()
    for _ in range(k):
        q = A @ rho
        alpha = np.linalg.lstsq(q[:, None], rho, rcond=None)[0][0]
        x = x + alpha * rho
        rho = rho - alpha * q
    return x


def _oddeven_dense(Dbb, r, even_mask, k):
    e, o = np.nonzero(even_mask)[0], np.nonzero(~even_mask)[0]
    Dee, Deo, Doe, Doo = Dbb[np.ix_(e, e)], Dbb[np.ix_(e, o)], Dbb[np.ix_(o, e)], Dbb[np.ix_(o, o)]
    Dee_inv = np.linalg.inv(Dee)
    Sc = Doo - Doe @ Dee_inv @ Deo
    rhs = r[o] - Doe @ (Dee_inv @ r[e])
    xo = _mr_dense(Sc, rhs, k)
    x = np.zeros_like(r)
    x[o] = xo
    x[e] = Dee_inv @ (r[e] - Deo @ xo)
    return x


@pytest.mark.parametrize("k", [1, 2, 3])
def test_block_mr_steps_are_least_squares(k):
    V, op, lev, blk = _setup()
    mus = np.array([0.05, 0.2])
    r = S.gaussian_spinors(2, V, 42).reshape(2, V, 12)
    delta = O.block_mr(lev, blk, r, mus, k)
    for c, mu in enumerate(mus):
        D = _dense(op, V, mu)
        rv, dv = r[c].reshape(-1), delta[c].reshape(-1)
        for b in range(blk.nblocks):
            idx = _block_idx(blk, b)
            ref = _mr_dense(D[np.ix_(idx, idx)], rv[idx], k)
            assert np.max(np.abs(dv[idx] - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_block_mr_oddeven_steps_on_dense_schur_complement(k):
    V, op, lev, blk = _setup(seed=43)
    mus = np.array([0.01, 0.3])
    r = S.gaussian_spinors(2, V, 44).reshape(2, V, 12)
    x = O.block_mr_oddeven(lev, blk, r, mus, k)
    even_site = site_parity(DIMS) == 0
    for c, mu in enumerate(mus):
        D = _dense(op, V, mu)
        rv, xv = r[c].reshape(-1), x[c].reshape(-1)
        for b in range(blk.nblocks):
            idx = _block_idx(blk, b)
            even_dof = np.repeat(even_site[np.nonzero(blk.id == b)[0]], 12)
            ref = _oddeven_dense(D[np.ix_(idx, idx)], rv[idx], even_dof, k)
            assert np.max(np.abs(xv[idx] - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("oddeven", [False, True])
def test_sap_cycle_is_two_colour_sweep_of_k_step_block_solves(oddeven):
    V, op, lev, blk = _setup(seed=45)
    mu, k = 0.1, 2
    f = S.gaussian_spinors(1, V, 46).reshape(1, V, 12)
    x = O.sap(lev, blk, f, [mu], cycles=1, mr_iters=k, oddeven=oddeven)
    D = _dense(op, V, mu)
    even_site = site_parity(DIMS) == 0
    xd = np.zeros(V * 12, dtype=np.complex128)
    fv = f.reshape(-1)
    for colour in (0, 1):
        res = fv - D @ xd
        for b in np.nonzero(blk.colour_of_block == colour)[0]:
            idx = _block_idx(blk, b)
            Dbb = D[np.ix_(idx, idx)]
            if oddeven:
                xd[idx] += _oddeven_dense(Dbb, res[idx], np.repeat(even_site[np.nonzero(blk.id == b)[0]], 12), k)
            else:
                xd[idx] += _mr_dense(Dbb, res[idx], k)
    assert np.max(np.abs(x.reshape(-1) - xd)) < 1e-12 * np.max(np.abs(xd))
