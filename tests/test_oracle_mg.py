"""Pins of the oracle's multigrid pieces and Krylov solvers against facts fixed
by the mathematics:

* P^H P = 1 per aggregate, gamma5 P = P gamma5_c, R P = 1;
* blockwise Galerkin coarse operator == dense P^H D P (fine->coarse and
  coarse->coarser, including coarse extents 2 and 1);
* coarse twist D_c(mu) - D_c(0) = i mu gamma5_c and coarse gamma5-hermiticity;
* Galerkin projector: with an exact coarse solve R(r - D P D_c^-1 R r) = 0;
* SAP with converged block solves == the dense two-colour Schwarz formula
  x = K_r f, x += K_b (f - D x) with K = inverse of the block principal submatrix,
  for plain block MR and for MR on the odd-even reduced block systems, whose
  back substitution leaves no residual on even sites;
* GMRES / block GMRES at full dimension == dense LU;
* the MG-preconditioned solve reaches the 1e-10 true residual and agrees with
  dense LU within cond * 1e-10.
"""
import numpy as np
import pytest

import synthetic as S
import oracle as O
from oracle.multigrid import Blocking, FineLevel, build_prolongator, restrict, prolong, galerkin


def dense_of(apply, n_dof, shape):
    E = np.eye(n_dof, dtype=np.complex128).reshape((n_dof,) + shape)
    return apply(E).reshape(n_dof, n_dof).T


def fine_setup(dims, agg, N, seed=21, kappa=0.14, eps=0.3):
    V = S.volume(dims)
    U = S.gauge_field(dims, eps, seed)
    op = O.WilsonTM(U, dims, kappa=kappa)
    lev = FineLevel(op)
    tv = S.gaussian_spinors(N, V, seed + 1).reshape(N, V, 12)
    blk = Blocking(dims, agg)
    P = build_prolongator(tv, blk)
    return op, lev, blk, P


def dense_P(P, blk):
    """P as a dense (V*d) x (nagg*2N) matrix built by prolonging unit coarse vectors."""
    V, d, N = P.shape
    nc = blk.nblocks * 2 * N
    E = np.eye(nc, dtype=np.complex128).reshape(nc, blk.nblocks, 2 * N)
    return prolong(P, blk, E).reshape(nc, V * d).T


@pytest.mark.parametrize("dims,agg", [((4, 4, 4, 4), (2, 2, 2, 2)), ((2, 2, 2, 4), (2, 1, 1, 2))])
def test_prolongator_orthonormal_chiral(dims, agg):
    op, lev, blk, P = fine_setup(dims, agg, 6)
    Pd = dense_P(P, blk)
    assert np.max(np.abs(Pd.conj().T @ Pd - np.eye(Pd.shape[1]))) < 1e-13
    V = S.volume(dims)
    g5 = np.kron(np.eye(V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    g5c = np.kron(np.eye(blk.nblocks), np.diag([1] * 6 + [-1] * 6))
    assert np.max(np.abs(g5 @ Pd - Pd @ g5c)) < 1e-14
    xc = S.gaussian_coarse(3, blk.nblocks, 12, 4)
    assert np.max(np.abs(restrict(P, blk, prolong(P, blk, xc)) - xc)) < 1e-13


@pytest.mark.parametrize("dims,agg", [((4, 4, 4, 4), (2, 2, 2, 2)), ((2, 2, 2, 4), (2, 1, 1, 2)),
                                      ((2, 4, 2, 2), (2, 2, 2, 2))])
def test_galerkin_equals_dense(dims, agg):
    N = 4
    op, lev, blk, P = fine_setup(dims, agg, N)
    V = S.volume(dims)
    coarse = galerkin(lev, P, blk)
    Pd = dense_P(P, blk)
    nc = blk.nblocks * 2 * N
    for mu in (0.0, 0.07):
        D = dense_of(lambda E: op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mu)),
                     V * 12, (V, 12))
        Dc = dense_of(lambda E: coarse.apply(E, np.full(E.shape[0], mu)), nc, (blk.nblocks, 2 * N))
        ref = Pd.conj().T @ D @ Pd
        assert np.max(np.abs(Dc - ref)) < 1e-13 * np.max(np.abs(ref))


def test_coarse_twist_and_gamma5_hermiticity():
    N = 4
    op, lev, blk, P = fine_setup((4, 4, 4, 4), (2, 2, 2, 2), N)
    coarse = galerkin(lev, P, blk)
    nc = blk.nblocks * 2 * N
    sh = (blk.nblocks, 2 * N)
    mu = 0.13
    D0 = dense_of(lambda E: coarse.apply(E, np.zeros(E.shape[0])), nc, sh)
    Dp = dense_of(lambda E: coarse.apply(E, np.full(E.shape[0], mu)), nc, sh)
    Dm = dense_of(lambda E: coarse.apply(E, np.full(E.shape[0], -mu)), nc, sh)
    g5c = np.kron(np.eye(blk.nblocks), np.diag([1] * N + [-1] * N))
    assert np.max(np.abs(Dp - D0 - 1j * mu * g5c)) < 1e-14
    assert np.max(np.abs(g5c @ Dp @ g5c - Dm.conj().T)) < 1e-13
    # blockwise form: B_nu(a + nu) = g5c F_nu(a)^H g5c
    Bl = coarse.blocks
    g = np.diag([1] * N + [-1] * N)
    cd = blk.cdims
    for mu_ in range(4):
        for a in range(blk.nblocks):
            c = list(S.site_coords(a, cd)); c[mu_] = (c[mu_] + 1) % cd[mu_]
            ap = S.site_index(*c, cd)
            if cd[mu_] > 2:
                assert np.max(np.abs(Bl[ap, 5 + mu_] - g @ Bl[a, 1 + mu_].conj().T @ g)) < 1e-13


def test_mu_factor_on_coarsest():
    N = 3
    op, lev, blk, P = fine_setup((2, 2, 2, 4), (2, 2, 2, 2), N)
    c1 = galerkin(lev, P, blk, mu_factor=1.0)
    c3 = galerkin(lev, P, blk, mu_factor=3.0)
    xc = S.gaussian_coarse(2, blk.nblocks, 2 * N, 7)
    mus = np.array([0.1, 0.02])
    d = c3.apply(xc, mus) - c1.apply(xc, mus)
    assert np.max(np.abs(d - 1j * 2.0 * mus[:, None, None] * c1.twist(xc))) < 1e-14


def test_coarse_to_coarser_galerkin():
    N, N2 = 4, 3
    op, lev, blk, P = fine_setup((4, 4, 4, 4), (2, 2, 2, 2), N)
    c2 = galerkin(lev, P, blk)
    blk2 = Blocking(blk.cdims, (2, 1, 2, 1))
    tv2 = S.gaussian_coarse(N2, blk.nblocks, 2 * N, 9)
    P2 = build_prolongator(tv2, blk2)
    c3 = galerkin(c2, P2, blk2)
    nc2 = blk.nblocks * 2 * N
    nc3 = blk2.nblocks * 2 * N2
    E = np.eye(nc3, dtype=np.complex128).reshape(nc3, blk2.nblocks, 2 * N2)
    P2d = prolong(P2, blk2, E).reshape(nc3, nc2).T
    mu = 0.05
    D2 = dense_of(lambda E: c2.apply(E, np.full(E.shape[0], mu)), nc2, (blk.nblocks, 2 * N))
    D3 = dense_of(lambda E: c3.apply(E, np.full(E.shape[0], mu)), nc3, (blk2.nblocks, 2 * N2))
    ref = P2d.conj().T @ D2 @ P2d
    assert np.max(np.abs(D3 - ref)) < 1e-13 * np.max(np.abs(ref))


def test_galerkin_projector():
    N = 4
    op, lev, blk, P = fine_setup((4, 4, 4, 4), (2, 2, 2, 2), N)
    coarse = galerkin(lev, P, blk)
    nc = blk.nblocks * 2 * N
    mu = 0.03
    Dc = dense_of(lambda E: coarse.apply(E, np.full(E.shape[0], mu)), nc, (blk.nblocks, 2 * N))
    r = S.gaussian_spinors(1, 256, 3).reshape(1, 256, 12)
    rc = restrict(P, blk, r)
    ec = np.linalg.solve(Dc, rc.reshape(-1)).reshape(rc.shape)
    r2 = r - lev.apply(prolong(P, blk, ec), [mu])
    assert np.max(np.abs(restrict(P, blk, r2))) < 1e-13 * np.max(np.abs(rc))


def test_sap_equals_dense_schwarz():
    dims = (4, 4, 2, 2)
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, 31)
    op = O.WilsonTM(U, dims, kappa=0.08)
    lev = FineLevel(op)
    blk = Blocking(dims, (2, 2, 2, 2))
    mu = 0.1
    D = dense_of(lambda E: op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mu)), V * 12, (V, 12))
    f = S.gaussian_spinors(1, V, 32).reshape(1, V, 12)
    x = O.sap(lev, blk, f, [mu], cycles=1, mr_iters=200)
    # dense two-colour Schwarz with exact block inverses
    site_col = blk.colour_of_block[blk.id]
    xd = np.zeros(V * 12, dtype=np.complex128)
    fv = f.reshape(-1)
    for colour in (0, 1):
        r = fv - D @ xd
        for b in np.nonzero(blk.colour_of_block == colour)[0]:
            idx = (np.nonzero(blk.id == b)[0][:, None] * 12 + np.arange(12)).reshape(-1)
            xd[idx] += np.linalg.solve(D[np.ix_(idx, idx)], r[idx])
    assert np.max(np.abs(x.reshape(-1) - xd)) < 1e-10 * np.max(np.abs(xd))


def test_gmres_full_dimension_is_exact():
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 8 * np.eye(n)
    B = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    ap = lambda X, act=None: (A @ X.T).T
    x, info = O.gmres(ap, B, 1e-14, n)
    xs = np.linalg.solve(A, B.T).T
    assert np.max(np.abs(x - xs)) < 1e-11
    xb, infob = O.block_gmres(lambda X: (A @ X.T).T, B, 1e-14, n)
    assert np.max(np.abs(xb - xs)) < 1e-11
    # block size 1 == GMRES
    x1, _ = O.block_gmres(lambda X: (A @ X.T).T, B[:1], 1e-8, 10)
    g1, _ = O.gmres(ap, B[:1], 1e-8, 10)
    assert np.max(np.abs(x1 - g1)) < 1e-10


def test_block_gmres_needs_fewer_iterations_than_gmres():
    rng = np.random.default_rng(4)
    n = 120
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 12 * np.eye(n)
    B = rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))
    xb, ib = O.block_gmres(lambda X: (A @ X.T).T, B, 1e-8, 60)
    xg, ig = O.gmres(lambda X, act=None: (A @ X.T).T, B, 1e-8, 200)
    assert np.all(ib["relres"] <= 1e-8)
    assert ib["iters"] < np.max(ig["iters"])


@pytest.mark.slow
def test_mg_solve_small_lattice_matches_dense_lu():
    w = S.workload("tm_4x4x4x4_2rhs_3shift")
    U = S.gauge_field(w.dims, w.eps, w.seed_gauge)
    p = O.MGParams(agg=w.agg, n_tv=w.n_tv, sap_block=w.sap_block, mu_setup=min(w.mus))
    mg = O.OracleMG(U, w.dims, w.kappa, p).setup(S.setup_start_vectors(w))
    b = np.repeat(S.rhs_for(w), len(w.mus), axis=0)[:3]
    mus = np.array(w.mus)
    x, info = mg.solve(b, mus)
    rel = mg.true_relres(b, x, mus)
    assert np.all(rel <= 1e-10)
    V = w.volume
    for c in range(3):
        D = dense_of(lambda E: mg.fine_op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mus[c])),
                     V * 12, (V, 12))
        xs = np.linalg.solve(D, b[c].reshape(-1))
        cond = np.linalg.cond(D)
        assert np.linalg.norm(x[c].reshape(-1) - xs) <= cond * 1e-10 * np.linalg.norm(xs)


@pytest.mark.parametrize("dims,block", [((4, 4, 2, 2), (2, 2, 2, 2)), ((8, 4, 4, 4), (4, 4, 4, 4))])
def test_oddeven_sap_equals_dense_schwarz(dims, block):
    """SAP whose block solves run MR on the odd-even reduced (Schur complement)
    systems converges to the same dense two-colour Schwarz formula."""
    V = S.volume(dims)
    U = S.gauge_field(dims, 0.3, 33)
    op = O.WilsonTM(U, dims, kappa=0.1)
    lev = FineLevel(op)
    blk = Blocking(dims, block)
    mu = 0.07
    D = dense_of(lambda E: op.apply(E.reshape(-1, V, 4, 3), np.full(E.shape[0], mu)), V * 12, (V, 12))
    f = S.gaussian_spinors(1, V, 34).reshape(1, V, 12)
    x = O.sap(lev, blk, f, [mu], cycles=1, mr_iters=150, oddeven=True)
    xd = np.zeros(V * 12, dtype=np.complex128)
    fv = f.reshape(-1)
    for colour in (0, 1):
        r = fv - D @ xd
        for b in np.nonzero(blk.colour_of_block == colour)[0]:
            idx = (np.nonzero(blk.id == b)[0][:, None] * 12 + np.arange(12)).reshape(-1)
            xd[idx] += np.linalg.solve(D[np.ix_(idx, idx)], r[idx])
    assert np.max(np.abs(x.reshape(-1) - xd)) < 1e-10 * np.max(np.abs(xd))


def test_oddeven_block_solve_back_substitution():
    """After any number of odd-even MR steps the even sites of every block
    satisfy their equations exactly: (r - D_BB x)_e = 0, and the odd-site
    residual equals r_o - D_oe D_ee^-1 r_e - S x_o (checked against the
    block operator itself)."""
    dims, block = (8, 4, 4, 4), (4, 4, 4, 4)
    V = S.volume(dims)
    op = O.WilsonTM(S.gauge_field(dims, 0.3, 35), dims, kappa=0.15)
    lev = FineLevel(op)
    blk = Blocking(dims, block)
    mus = np.array([0.01, 0.3])
    r = S.gaussian_spinors(2, V, 36).reshape(2, V, 12)
    even = (1 - O.multigrid.site_parity(dims))[None, :, None]
    for iters in (1, 3):
        x = O.block_mr_oddeven(lev, blk, r, mus, iters)
        res = r - lev.apply_block_diag(x, mus, blk)
        assert np.max(np.abs(res * even)) < 1e-13 * np.max(np.abs(r))
        assert np.max(np.abs(res * (1 - even))) > 1e-3      # the odd half is only approximate
    # more steps: the odd residual falls (MR minimises it step by step)
    n1 = np.linalg.norm(r - lev.apply_block_diag(O.block_mr_oddeven(lev, blk, r, mus, 2), mus, blk))
    n2 = np.linalg.norm(r - lev.apply_block_diag(O.block_mr_oddeven(lev, blk, r, mus, 6), mus, blk))
    assert n2 < n1
