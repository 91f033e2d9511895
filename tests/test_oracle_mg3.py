"""Pins of the oracle's coarse-level smoother and of its three-level cycle.

* ``mr_smoother``: every step is the one-dimensional least-squares problem
  min_alpha ||r - alpha D r|| (minimal residual), so its alpha equals a dense
  ``lstsq`` solution and the residual never grows (fine and coarse levels);
* the three-level cycle (paper section 2: the construction applied
  recursively; section 4: the middle level solved by FGMRES preconditioned by
  the next level, the bottom by GMRES or block GMRES): with coarse tolerances
  driven to rounding level its output equals the dense two-grid formula
  e = P D_c^-1 R r + S(r - D P D_c^-1 R r) with S the level's smoother, on
  the middle level (S = MR steps) and on the fine level (S = SAP);
* the three-level solve reaches the 1e-10 true residual and agrees with dense
  LU within cond * 1e-10, with per-column and with block GMRES at the bottom;
* the gamma5-Hermitian form of the coarse solves: gamma5_c D_c(mu) - i mu is
  Hermitian (so the Krylov operator is normal); with exact coarse solves the
  cycle is unchanged; on the middle level the form is an exact equivalence
  (right preconditioner MG(gamma5 v)), so the middle iterations and the cycle
  output equal those of the plain middle level step for step.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, build_prolongator, restrict, prolong, galerkin


def dense_of(apply, n_dof, shape):
    E = np.eye(n_dof, dtype=np.complex128).reshape((n_dof,) + shape)
    return apply(E).reshape(n_dof, n_dof).T


def dense_P(P, blk):
    V, d, N = P.shape
    nc = blk.nblocks * 2 * N
    E = np.eye(nc, dtype=np.complex128).reshape(nc, blk.nblocks, 2 * N)
    return prolong(P, blk, E).reshape(nc, V * d).T


def _mr_dense(D, f, steps):
    """x_{k+1} = x_k + a_k r_k with a_k the least-squares minimiser of
    ||r_k - a D r_k||; returns x and the residual norms."""
    x = np.zeros_like(f)
    r = f.copy()
    norms = [np.linalg.norm(r)]
    for _ in range(steps):
        q = D @ r
        a = np.linalg.lstsq(q[:, None], r, rcond=None)[0][0]
        x = x + a * r
        r = f - D @ x
        norms.append(np.linalg.norm(r))
    return x, norms


def test_mr_smoother_fine_level_is_least_squares():
    dims = (2, 2, 2, 2)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 41), dims, kappa=0.14)
    lev = FineLevel(op)
    mus = np.array([0.02, 0.4])
    f = S.gaussian_spinors(2, V, 42).reshape(2, V, 12)
    for c in range(2):
        D = dense_of(lambda E: op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mus[c])),
                     V * 12, (V, 12))
        # one step: alpha must be the dense least-squares minimiser
        x1 = O.mr_smoother(lev, f[c:c + 1], mus[c:c + 1], 1).reshape(-1)
        q = D @ f[c].reshape(-1)
        a = np.linalg.lstsq(q[:, None], f[c].reshape(-1), rcond=None)[0][0]
        assert np.max(np.abs(x1 - a * f[c].reshape(-1))) < 1e-14 * np.max(np.abs(x1))
        # several steps: the dense recurrence, and a residual that never grows
        xs, norms = _mr_dense(D, f[c].reshape(-1), 5)
        x5 = O.mr_smoother(lev, f[c:c + 1], mus[c:c + 1], 5).reshape(-1)
        assert np.max(np.abs(x5 - xs)) < 1e-12 * np.max(np.abs(xs))
        assert all(n1 <= n0 * (1 + 1e-14) for n0, n1 in zip(norms, norms[1:]))
        assert norms[-1] < norms[0]


def test_mr_smoother_coarse_level_is_least_squares():
    dims, agg, N = (4, 4, 4, 4), (2, 2, 2, 2), 4
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 43), dims, kappa=0.14)
    lev = FineLevel(op)
    blk = Blocking(dims, agg)
    P = build_prolongator(S.gaussian_spinors(N, V, 44).reshape(N, V, 12), blk)
    coarse = galerkin(lev, P, blk)
    nc = blk.nblocks * 2 * N
    mus = np.array([0.05, 0.0])
    f = S.gaussian_coarse(2, blk.nblocks, 2 * N, 45)
    x = O.mr_smoother(coarse, f, mus, 3)
    for c in range(2):
        D = dense_of(lambda E: coarse.apply(E, np.full(E.shape[0], mus[c])), nc, (blk.nblocks, 2 * N))
        xs, norms = _mr_dense(D, f[c].reshape(-1), 3)
        assert np.max(np.abs(x[c].reshape(-1) - xs)) < 1e-12 * np.max(np.abs(xs))
        assert all(n1 <= n0 * (1 + 1e-14) for n0, n1 in zip(norms, norms[1:]))


def _three_level(block=False, r_m=7e-2, r_b=1e-1, kappa=0.14, seed=51, g5=0):
    dims = (4, 4, 4, 4)
    U = S.gauge_field(dims, 0.3, seed)
    p = O.MGParams(agg=((2, 2, 2, 2), (2, 2, 2, 2)), n_tv=(8, 8), sap_block=(2, 2, 2, 2),
                   sap_cycles=2, sap_mr=4, mu_setup=0.01, r_m=r_m, r_b=r_b,
                   middle_maxit=200, middle_restart=200, bottom_maxit=200,
                   coarse_smooth_iters=2, coarsest_block=block, coarse_gamma5=g5)
    start = [S.gaussian_spinors(8, 256, seed + 1).reshape(8, 256, 12),
             S.gaussian_coarse(8, 16, 16, seed + 2)]
    return O.OracleMG(U, dims, kappa, p).setup(start)


@pytest.mark.parametrize("g5", [0, 2])
def test_three_level_cycle_equals_dense_formula(g5):
    """With the middle and bottom solves driven to rounding level the cycle's
    output is fixed by dense linear algebra on every level, whichever form
    (plain or gamma5-Hermitian) the coarse Krylov solves take."""
    mg = _three_level(r_m=1e-13, r_b=1e-13, g5=g5)
    assert [lv.V for lv in mg.levels] == [256, 16, 1]
    mus = np.array([0.01, 0.3])
    lev0, lev1, lev2 = mg.levels
    n1 = lev1.V * lev1.d
    n2 = lev2.V * lev2.d
    P0d = dense_P(mg.P[0], mg.blockings[0])
    P1d = dense_P(mg.P[1], mg.blockings[1])
    # middle level: e = P1 D2^-1 R1 r + MR_2steps(r - D1 P1 D2^-1 R1 r)
    rc = S.gaussian_coarse(2, lev1.V, lev1.d, 52)
    e1 = mg.cycle(1, rc, mus)
    for c in range(2):
        D1 = dense_of(lambda E: lev1.apply(E, np.full(E.shape[0], mus[c])), n1, (lev1.V, lev1.d))
        D2 = dense_of(lambda E: lev2.apply(E, np.full(E.shape[0], mus[c])), n2, (lev2.V, lev2.d))
        # the coarsest operator is the Galerkin product of the middle one
        assert np.max(np.abs(D2 - P1d.conj().T @ D1 @ P1d)) < 1e-13 * np.max(np.abs(D2))
        r = rc[c].reshape(-1)
        e = P1d @ np.linalg.solve(D2, P1d.conj().T @ r)
        s, _ = _mr_dense(D1, r - D1 @ e, 2)
        ref = e + s
        assert np.max(np.abs(e1[c].reshape(-1) - ref)) < 1e-10 * np.max(np.abs(ref))
    # fine level: e = P0 D1^-1 R0 r + SAP(r - D P0 D1^-1 R0 r)
    r0 = S.gaussian_spinors(2, 256, 53).reshape(2, 256, 12)
    e0 = mg.cycle(0, r0, mus)
    for c in range(2):
        D1 = dense_of(lambda E: lev1.apply(E, np.full(E.shape[0], mus[c])), n1, (lev1.V, lev1.d))
        e = (P0d @ np.linalg.solve(D1, P0d.conj().T @ r0[c].reshape(-1))).reshape(1, 256, 12)
        res = r0[c:c + 1] - lev0.apply(e, mus[c:c + 1])
        ref = e + O.sap(lev0, mg.sap_blocking, res, mus[c:c + 1], 2, 4)
        assert np.max(np.abs(e0[c:c + 1] - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.slow
@pytest.mark.parametrize("block", [False, True])
def test_three_level_solve_matches_dense_lu(block):
    mg = _three_level(block=block)
    V = 256
    mus = np.array([0.01, 0.01])            # one shift group of two columns (a block of 2)
    b = S.gaussian_spinors(2, V, 54)
    x, info = mg.solve(b, mus)
    rel = mg.true_relres(b, x, mus)
    assert np.all(rel <= 1e-10)
    # the middle and bottom solvers both ran
    assert len(mg.stats["middle_iters"]) > 0 and len(mg.stats["bottom_iters"]) > 0
    D = dense_of(lambda E: mg.fine_op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mus[0])),
                 V * 12, (V, 12))
    xs = np.linalg.solve(D, b.reshape(2, -1).T).T
    cond = np.linalg.cond(D)
    for c in range(2):
        assert np.linalg.norm(x[c].reshape(-1) - xs[c]) <= cond * 1e-10 * np.linalg.norm(xs[c])


def test_gamma5_coarse_operator_is_shifted_hermitian():
    mg = _three_level()
    for lev in mg.levels[1:]:
        n = lev.V * lev.d
        for mu in (0.0, 0.05):
            Q = dense_of(lambda E: lev.twist(lev.apply(E, np.full(E.shape[0], mu))), n, (lev.V, lev.d))
            H = Q - 1j * mu * np.eye(n)
            assert np.max(np.abs(H - H.conj().T)) < 1e-14 * np.max(np.abs(H))


def test_gamma5_middle_level_is_an_exact_equivalence():
    """FGMRES on gamma5 D_1 with the right preconditioner MG_2(gamma5 v) runs
    the plain middle iteration multiplied by gamma5 (a unitary map), so with
    the same bottom solver (gamma5 form in both) the iterations and the cycle
    output are the same."""
    a, b = _three_level(g5=1), _three_level(g5=2)
    mus = np.array([0.01, 0.2])
    r = S.gaussian_spinors(2, 256, 55).reshape(2, 256, 12)
    ea, eb = a.cycle(0, r, mus), b.cycle(0, r, mus)
    assert a.stats["middle_iters"] == b.stats["middle_iters"]
    assert a.stats["bottom_iters"] == b.stats["bottom_iters"]
    assert np.max(np.abs(ea - eb)) < 1e-9 * np.max(np.abs(ea))
