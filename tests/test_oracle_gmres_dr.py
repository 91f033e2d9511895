"""Pins of the oracle's GMRES with deflated restarting (GMRES-DR(m, k)):

* k = 0 is restarted GMRES(m): same iterates as the oracle's GMRES(m) (which
  recomputes the residual explicitly at every restart) up to rounding;
* m >= n: one cycle solves exactly (dense LU);
* harmonic Ritz pairs: the standard form used at a restart against the
  generalised eigenproblem Hbar^H Hbar g = theta H_m^H g that defines them
  (scipy), on an Arnoldi relation of a random matrix;
* on a matrix whose spectrum has a few eigenvalues near the origin GMRES(m)
  stagnates while GMRES-DR(m, k) with k at least their number converges, and
  more deflation vectors do not cost iterations.
"""
import numpy as np
import scipy.linalg as sl

import oracle as O


def _matrix(n=240, nsmall=6, seed=3):
    rng = np.random.default_rng(seed)
    ev = np.concatenate([rng.uniform(0.001, 0.01, nsmall) * np.exp(1j * rng.uniform(0, 6.28, nsmall)),
                         1 + rng.uniform(0, 2, n - nsmall) + 1j * rng.uniform(-1, 1, n - nsmall)])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    A = Q @ np.diag(ev) @ Q.conj().T + 0.01 * rng.standard_normal((n, n))
    B = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    return A, B


def test_k0_is_restarted_gmres():
    A, B = _matrix(n=120)
    ap = lambda X, act: (A @ X.T).T
    x0, i0 = O.gmres_dr(ap, B, 1e-14, 12, 0, 60)
    x1, i1 = O.gmres(ap, B, 1e-14, 60, restart=12)
    assert list(i0["iters"]) == list(i1["iters"]) == [60, 60]
    assert np.max(np.abs(x0 - x1)) < 1e-9 * np.max(np.abs(x1))


def test_full_dimension_is_exact():
    rng = np.random.default_rng(4)
    n = 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 5 * np.eye(n)
    B = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
    x, info = O.gmres_dr(lambda X, act: (A @ X.T).T, B, 1e-13, n, 5, 10 * n)
    xs = np.linalg.solve(A, B.T).T
    assert np.max(np.abs(x - xs)) < 1e-10 * np.max(np.abs(xs))
    assert np.all(info["cycles"] == 1)


def test_harmonic_ritz_pairs_solve_the_generalised_problem():
    rng = np.random.default_rng(5)
    n, m, k = 80, 20, 6
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    V = np.zeros((n, m + 1), dtype=complex)
    H = np.zeros((m + 1, m), dtype=complex)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        w = A @ V[:, j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[:, i], w)
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    theta, G = O.harmonic_ritz(H, k)
    ref = sl.eigvals(H.conj().T @ H, H[:m, :m].conj().T)
    ref = ref[np.argsort(np.abs(ref))][:k]
    assert np.max(np.abs(np.sort_complex(theta) - np.sort_complex(ref))) < 1e-8 * np.max(np.abs(ref))
    for i in range(k):
        res = H.conj().T @ H @ G[:, i] - theta[i] * (H[:m, :m].conj().T @ G[:, i])
        assert np.linalg.norm(res) < 1e-9 * np.linalg.norm(H) ** 2 * np.linalg.norm(G[:, i])


def test_deflation_removes_stagnation():
    A, B = _matrix()
    ap = lambda X, act: (A @ X.T).T
    _, ig = O.gmres(ap, B, 1e-10, 2000, restart=30)
    assert np.all(ig["relres"] > 1e-6)                        # GMRES(30) stagnates
    its = []
    for k in (6, 10):
        x, info = O.gmres_dr(ap, B, 1e-10, 30, k, 2000)
        assert np.all(info["relres"] <= 1e-10 * (1 + 1e-6))
        its.append(int(info["iters"].max()))
    assert its[1] <= its[0] < 2000
