"""Pins of the oracle's GMRES and flexible GMRES (section 4: FGMRES at the top
level, GMRES at the bottom), by what the methods are defined to compute
rather than by re-running their recurrences:

* k steps of GMRES from x0 = 0 give the minimal-residual vector of the Krylov
  space K_k(A, b): checked against a least-squares solve over an explicitly
  built (and QR-orthonormalised) Krylov basis, on a non-normal matrix;
* k steps of FGMRES with a fixed right preconditioner M are GMRES on AM:
  x = M y with y minimal over K_k(AM, b);
* with a preconditioner that changes at every step (the flexible case) the
  iterate is Z y with y minimising ||b - A Z y|| over the recorded
  preconditioned vectors z_j (it lies in span Z, not in the Krylov space of
  the v_j): a mistake that assembles the update from V instead of Z fails;
* an exact preconditioner (A^-1) solves in one step;
* restarts: the reported residual is the true one and never grows;
* the column inner product conjugates its first argument;
* k block-GMRES steps: each column's residual is minimal over the block
  Krylov space of all columns.
"""
import numpy as np

import oracle as O
from oracle.krylov import _givens


def _nonnormal(n=48, seed=11):
    rng = np.random.default_rng(seed)
    A = 2 * np.eye(n) + np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), 1) / np.sqrt(n)
    A += 0.3 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    B = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    return A, B


def _min_residual(AK, K, b):
    """argmin over y of ||b - AK y|| and the vector K y."""
    y, *_ = np.linalg.lstsq(AK, b, rcond=None)
    return K @ y, np.linalg.norm(b - AK @ y)


def _krylov(A, b, k):
    K = np.empty((len(b), k), dtype=complex)
    v = b.copy()
    for j in range(k):
        K[:, j] = v
        v = A @ v
    Q, _ = np.linalg.qr(K)
    return Q


def test_column_inner_product_conjugates_first_argument():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((2, 5)) + 1j * rng.standard_normal((2, 5))
    b = rng.standard_normal((2, 5)) + 1j * rng.standard_normal((2, 5))
    assert np.allclose(O.col_dot(1j * a, b), -1j * O.col_dot(a, b))
    assert np.allclose(O.col_dot(a, 1j * b), 1j * O.col_dot(a, b))
    assert np.allclose(O.col_dot(a, b), [np.vdot(a[c], b[c]) for c in range(2)])
    assert np.allclose(O.col_norm(a) ** 2, O.col_dot(a, a).real)


def test_givens_rotation_is_unitary_and_annihilates():
    rng = np.random.default_rng(3)
    for a, b in [(1 + 2j, -0.5 + 1j), (0j, 2 - 1j), (3 - 1j, 0j)] + \
            [tuple(rng.standard_normal(2) + 1j * rng.standard_normal(2)) for _ in range(5)]:
        c, s, r = _givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        assert np.allclose(G @ G.conj().T, np.eye(2), atol=1e-14)
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-14 * max(1, abs(r))
        assert abs(out[0] - r) < 1e-14 * max(1, abs(r))
        assert abs(abs(r) - np.hypot(abs(a), abs(b))) < 1e-14 * max(1, abs(r))


def test_gmres_iterate_is_krylov_minimal_residual():
    A, B = _nonnormal()
    ap = lambda X, act: (A @ X.T).T
    for k in (1, 4, 11):
        x, info = O.gmres(ap, B, 0.0, k)
        assert list(info["iters"]) == [k] * len(B)
        for c in range(len(B)):
            K = _krylov(A, B[c], k)
            xb, rb = _min_residual(A @ K, K, B[c])
            r = np.linalg.norm(B[c] - A @ x[c])
            assert abs(r - rb) <= 1e-11 * np.linalg.norm(B[c])
            assert np.linalg.norm(x[c] - xb) <= 1e-9 * np.linalg.norm(xb)
            assert abs(info["relres"][c] - r / np.linalg.norm(B[c])) < 1e-13


def test_fgmres_fixed_preconditioner_is_gmres_on_AM():
    A, B = _nonnormal(seed=12)
    rng = np.random.default_rng(13)
    n = A.shape[0]
    M = np.eye(n) + 0.2 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    ap = lambda X, act: (A @ X.T).T
    pc = lambda X, act: (M @ X.T).T
    k = 7
    x, info = O.fgmres(ap, pc, B, 0.0, k, k)
    for c in range(len(B)):
        K = _krylov(A @ M, B[c], k)
        xb, rb = _min_residual(A @ M @ K, M @ K, B[c])
        assert abs(np.linalg.norm(B[c] - A @ x[c]) - rb) <= 1e-11 * np.linalg.norm(B[c])
        assert np.linalg.norm(x[c] - xb) <= 1e-9 * np.linalg.norm(xb)


def test_fgmres_varying_preconditioner_minimises_over_z():
    A, B = _nonnormal(seed=14)
    n = A.shape[0]
    rng = np.random.default_rng(15)
    Z = [[] for _ in range(len(B))]

    def pc(X, act):     # a different preconditioner at every call; the outputs are recorded per column
        Mj = np.eye(n) + 0.5 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
        out = (Mj @ X.T).T
        for i, c in enumerate(act):
            Z[c].append(out[i].copy())
        return out

    k = 6
    x, _ = O.fgmres(lambda X, act: (A @ X.T).T, pc, B, 0.0, k, k)
    for c in range(len(B)):
        Zc = np.array(Z[c]).T
        assert Zc.shape == (n, k)
        xb, rb = _min_residual(A @ Zc, Zc, B[c])
        assert abs(np.linalg.norm(B[c] - A @ x[c]) - rb) <= 1e-11 * np.linalg.norm(B[c])
        assert np.linalg.norm(x[c] - xb) <= 1e-9 * np.linalg.norm(xb)
        # the iterate is not the minimiser over the Arnoldi vectors' own span
        K = _krylov(A, B[c], k)
        _, rk = _min_residual(A @ K, K, B[c])
        assert abs(rk - rb) > 1e-6 * np.linalg.norm(B[c])


def test_fgmres_exact_preconditioner_solves_in_one_step():
    A, B = _nonnormal(seed=16)
    Ainv = np.linalg.inv(A)
    x, info = O.fgmres(lambda X, act: (A @ X.T).T, lambda X, act: (Ainv @ X.T).T, B, 1e-12, 5, 20)
    assert list(info["iters"]) == [1] * len(B)
    xs = np.linalg.solve(A, B.T).T
    assert np.max(np.abs(x - xs)) < 1e-12 * np.max(np.abs(xs))


def test_restarted_residuals_are_true_and_monotone():
    A, B = _nonnormal(seed=17)
    ap = lambda X, act: (A @ X.T).T
    prev = np.ones(len(B))
    for cycles in range(1, 6):
        x, info = O.gmres(ap, B, 0.0, 4 * cycles, restart=4)
        true = O.col_norm(B - ap(x, None)) / O.col_norm(B)
        assert np.allclose(info["relres"], true, rtol=1e-12, atol=0)
        assert np.all(true <= prev * (1 + 1e-12))
        prev = true
    # to tolerance: every column stops at or below it
    x, info = O.gmres(ap, B, 1e-10, 400, restart=8)
    assert np.all(info["relres"] <= 1e-10)
    assert np.all(O.col_norm(B - ap(x, None)) / O.col_norm(B) <= 1e-10 * (1 + 1e-6))


def test_block_gmres_minimises_over_the_block_krylov_space():
    """k block-GMRES steps give every column the minimal residual over the
    block Krylov space span{B, AB, ..., A^(k-1) B} that all columns share
    (section 4: the block method enlarges each column's search space)."""
    A, B = _nonnormal(seed=18)
    n, s = A.shape[0], len(B)
    for k in (1, 3, 5):
        x, info = O.block_gmres(lambda X: (A @ X.T).T, B, 0.0, k)
        assert info["iters"] == k
        K = np.concatenate([np.linalg.matrix_power(A, j) @ B.T for j in range(k)], axis=1)
        Q, _ = np.linalg.qr(K)
        assert Q.shape == (n, k * s)
        for c in range(s):
            xb, rb = _min_residual(A @ Q, Q, B[c])
            assert abs(np.linalg.norm(B[c] - A @ x[c]) - rb) <= 1e-11 * np.linalg.norm(B[c])
            assert np.linalg.norm(x[c] - xb) <= 1e-9 * np.linalg.norm(xb)
            # no worse than the column's own Krylov space of the same dimension k
            Kc = _krylov(A, B[c], k)
            _, rc = _min_residual(A @ Kc, Kc, B[c])
            assert rb <= rc * (1 + 1e-12)
