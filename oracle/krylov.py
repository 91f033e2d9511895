"""Oracle: Krylov solvers in plain FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

* GMRES and flexible GMRES (section 4: FGMRES at the top level with a 1e-10 goal
  residual; non-block FGMRES at the middle level; GMRES at the bottom).
* Block GMRES (section 4: block Krylov solvers enlarge the search space by
  combining the Krylov spaces of all rhs; block GMRES with incremental QR of
  the block Hessenberg).  A block only makes sense for columns that share one
  operator, i.e. one twisted-mass value.

Vectors are batches [n][...]; every column runs its own Arnoldi process.  The
columns advance together but each column's solution only uses the iterations
up to the one where that column met its tolerance, so a column's result is
the one a solo run would give.  Orthogonalisation here is modified
Gram-Schmidt (the paper's GPU-friendly classical Gram-Schmidt gives the same
result in exact arithmetic).
"""
from __future__ import annotations

import numpy as np

__all__ = ["gmres", "fgmres", "block_gmres", "gmres_dr", "harmonic_ritz", "col_dot", "col_norm"]


def col_dot(a, b):
    """per-column <a, b> = sum conj(a) b."""
    n = a.shape[0]
    return np.sum(np.conj(a).reshape(n, -1) * b.reshape(n, -1), axis=1)


def col_norm(a):
    n = a.shape[0]
    return np.sqrt(np.sum(np.abs(a.reshape(n, -1)) ** 2, axis=1))


def _givens(a, b):
    """complex Givens rotation [c s; -conj(s) c] with c real that maps (a, b) to (r, 0)."""
    if b == 0:
        return 1.0, 0.0 + 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b) + 0j
    na = abs(a)
    nr = np.hypot(na, abs(b))
    c = na / nr
    s = (a / na) * np.conj(b) / nr
    r = (a / na) * nr
    return c, s, r


def _arnoldi_cycle(apply, precond, r0, beta, m, tol_abs, flexible):
    """One restart cycle of (F)GMRES from residual r0 (norms beta).
    Returns the correction dx and per-column (iterations used, estimate)."""
    n = r0.shape[0]
    Vb = [r0 / np.where(beta > 0, beta, 1.0).reshape((n,) + (1,) * (r0.ndim - 1))]
    Zb = []
    H = np.zeros((n, m + 1, m), dtype=np.complex128)
    g = np.zeros((n, m + 1), dtype=np.complex128)
    g[:, 0] = beta
    cs = np.zeros((n, m)); sn = np.zeros((n, m), dtype=np.complex128)
    Hr = np.zeros((n, m + 1, m), dtype=np.complex128)      # rotated H (upper triangular part)
    k_used = np.full(n, -1)
    est = beta.astype(np.float64).copy()
    done = beta <= tol_abs
    k_used[done] = 0
    for j in range(m):
        z = precond(Vb[j]) if flexible else Vb[j]
        if flexible:
            Zb.append(z)
        w = apply(z)
        for i in range(j + 1):
            h = col_dot(Vb[i], w)
            H[:, i, j] = h
            w = w - h.reshape((n,) + (1,) * (w.ndim - 1)) * Vb[i]
        hn = col_norm(w)
        H[:, j + 1, j] = hn
        Vb.append(w / np.where(hn > 0, hn, 1.0).reshape((n,) + (1,) * (w.ndim - 1)))
        for c in range(n):
            col = H[c, :j + 2, j].copy()
            for i in range(j):
                a, b = col[i], col[i + 1]
                col[i] = cs[c, i] * a + sn[c, i] * b
                col[i + 1] = -np.conj(sn[c, i]) * a + cs[c, i] * b
            cc, ss, rr = _givens(col[j], col[j + 1])
            cs[c, j], sn[c, j] = cc, ss
            col[j], col[j + 1] = rr, 0.0
            Hr[c, :j + 2, j] = col
            gj = g[c, j]
            g[c, j] = cc * gj
            g[c, j + 1] = -np.conj(ss) * gj
            if not done[c]:
                est[c] = abs(g[c, j + 1])
                if est[c] <= tol_abs[c] or hn[c] == 0:
                    done[c] = True
                    k_used[c] = j + 1
        if np.all(done):
            break
    k_used[k_used < 0] = j + 1
    dx = np.zeros_like(r0)
    for c in range(n):
        k = k_used[c]
        if k == 0:
            continue
        y = np.linalg.solve(np.triu(Hr[c, :k, :k]), g[c, :k])
        basis = Zb if flexible else Vb
        for i in range(k):
            dx[c] += y[i] * basis[i][c]
    return dx, k_used, est


def gmres(apply, b, tol, maxit, x0=None, restart=None, flexible_precond=None):
    """Restarted (F)GMRES on a batch.  apply(x) acts on a [n_act][...] batch of
    the active columns; precond likewise (flexible when given).

    Stops a column when its true residual is <= tol * ||b_c||.
    Returns (x, info) with info = dict(iters, relres)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    m = maxit if restart is None else restart
    bnorm = col_norm(b)
    tol_abs = tol * np.where(bnorm > 0, bnorm, 1.0)
    iters = np.zeros(n, dtype=np.int64)
    active = np.arange(n)
    r = b - (apply(x, active) if x0 is not None else 0)
    rn = col_norm(r)
    while True:
        active = np.array([c for c in range(n) if rn[c] > tol_abs[c] and iters[c] < maxit], dtype=np.int64)
        if active.size == 0:
            break
        mm = int(min(m, maxit - iters[active].min()))
        ap = lambda v, act=active: apply(v, act)
        pc = None if flexible_precond is None else (lambda v, act=active: flexible_precond(v, act))
        dx, k, _ = _arnoldi_cycle(ap, pc, r[active], rn[active], mm, tol_abs[active],
                                  flexible_precond is not None)
        x[active] += dx
        iters[active] += k
        r_act = b[active] - apply(x[active], active)
        r[active] = r_act
        rn[active] = col_norm(r_act)
        if restart is None:
            break
    return x, dict(iters=iters, relres=rn / np.where(bnorm > 0, bnorm, 1.0))


def fgmres(apply, precond, b, tol, restart, maxit, x0=None):
    """Flexible GMRES(restart), the top-level solver of the paper's method."""
    return gmres(apply, b, tol, maxit, x0=x0, restart=restart, flexible_precond=precond)


def block_gmres(apply, B, tol, maxit, X0=None):
    """Block GMRES for s right-hand sides that share one operator.

    Block Arnoldi: V_0 R_0 = B - A X0 (QR), W = A V_j, H_ij = V_i^H W and
    W -= V_i H_ij for i <= j, V_{j+1} H_{j+1,j} = W (QR).  The correction is
    V_j Y with Y minimising ||E_1 R_0 - Hbar_j Y||_F column by column.  Stops
    when every column's residual is <= tol * ||b_c||."""
    B = np.asarray(B, dtype=np.complex128)
    s = B.shape[0]
    shape = B.shape
    X = np.zeros_like(B) if X0 is None else np.array(X0, dtype=np.complex128)
    R0 = B - apply(X) if X0 is not None else B.copy()
    bnorm = col_norm(B)
    tol_abs = tol * np.where(bnorm > 0, bnorm, 1.0)
    Rm = R0.reshape(s, -1).T                                   # [ndof][s]
    if np.all(col_norm(R0) <= tol_abs):
        return X, dict(iters=0, relres=col_norm(R0) / np.where(bnorm > 0, bnorm, 1.0))
    Q, Rhat = np.linalg.qr(Rm)
    Vs = [Q]
    Hbar = np.zeros(((maxit + 1) * s, maxit * s), dtype=np.complex128)
    j_done = maxit
    for j in range(maxit):
        W = apply(Vs[j].T.reshape(shape)).reshape(s, -1).T
        for i in range(j + 1):
            Hij = Vs[i].conj().T @ W
            Hbar[i * s:(i + 1) * s, j * s:(j + 1) * s] = Hij
            W = W - Vs[i] @ Hij
        Qn, Rn = np.linalg.qr(W)
        Hbar[(j + 1) * s:(j + 2) * s, j * s:(j + 1) * s] = Rn
        Vs.append(Qn)
        E = np.zeros(((j + 2) * s, s), dtype=np.complex128)
        E[:s] = Rhat
        Hj = Hbar[:(j + 2) * s, :(j + 1) * s]
        Y, *_ = np.linalg.lstsq(Hj, E, rcond=None)
        res = np.linalg.norm(E - Hj @ Y, axis=0)
        if np.all(res <= tol_abs):
            j_done = j + 1
            break
    k = j_done
    Hj = Hbar[:(k + 1) * s, :k * s]
    E = np.zeros(((k + 1) * s, s), dtype=np.complex128)
    E[:s] = Rhat
    Y, *_ = np.linalg.lstsq(Hj, E, rcond=None)
    Vmat = np.concatenate(Vs[:k], axis=1)                       # [ndof][k s]
    X = X + (Vmat @ Y).T.reshape(shape)
    relres = col_norm(B - apply(X)) / np.where(bnorm > 0, bnorm, 1.0)
    return X, dict(iters=k, relres=relres)


def harmonic_ritz(Hbar, k):
    """The k harmonic Ritz pairs of smallest modulus of an Arnoldi relation
    A V_m = V_{m+1} Hbar ((m+1) x m): theta and g solve
    (H_m + |h_{m+1,m}|^2 f e_m^T) g = theta g with f = H_m^{-H} e_m, which is
    the standard form of Hbar^H Hbar g = theta H_m^H g."""
    m = Hbar.shape[1]
    Hm = Hbar[:m, :m]
    em = np.zeros(m)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.conj().T, em)
    T = Hm + abs(Hbar[m, m - 1]) ** 2 * np.outer(f, em)
    theta, G = np.linalg.eig(T)
    idx = np.argsort(np.abs(theta), kind="stable")[:k]
    return theta[idx], G[:, idx]


def gmres_dr(apply, b, tol, m, k, maxit, x0=None):
    """GMRES with deflated restarting, GMRES-DR(m, k) (section 4 of the paper:
    deflated restarting at the coarsest level; Morgan's construction).

    Each cycle runs Arnoldi to m basis vectors and takes the least-squares
    correction.  At a restart the k harmonic Ritz vectors of smallest
    harmonic Ritz value, together with the residual's coordinate vector, span
    the first k+1 vectors of the next basis: with Q the orthonormal factor of
    [g_1 .. g_k (one zero row appended), c - Hbar y], V <- V Q and
    Hbar <- Q^H Hbar Q[:m, :k], and the residual coordinates become Q^H
    (c - Hbar y); Arnoldi then continues from vector k+1.  k = 0 is GMRES(m).
    Columns are independent (apply acts on the active batch).  Stops a column
    when its least-squares residual estimate is <= tol ||b_c||, or after maxit
    operator applications.  Returns (x, info: iters, relres (true), cycles)."""
    b = np.asarray(b, dtype=np.complex128)
    n = b.shape[0]
    shp = b.shape[1:]
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.complex128)
    r = b - (apply(x, np.arange(n)) if x0 is not None else 0)
    bnorm = col_norm(b)
    tol_abs = tol * np.where(bnorm > 0, bnorm, 1.0)
    iters = np.zeros(n, dtype=np.int64)
    cycles = np.zeros(n, dtype=np.int64)
    beta = col_norm(r)
    # per-column state: basis (list of vectors), Hbar, residual coordinates c, start index
    Vs = [[r[c] / beta[c]] if beta[c] > 0 else [] for c in range(n)]
    Hs = [np.zeros((m + 1, m), dtype=np.complex128) for _ in range(n)]
    cs = [np.concatenate([[beta[c]], np.zeros(m)]).astype(np.complex128) for c in range(n)]
    j0 = [0] * n
    done = [beta[c] <= tol_abs[c] for c in range(n)]
    while True:
        act = np.array([c for c in range(n) if not done[c]], dtype=np.int64)
        if act.size == 0:
            break
        # one Arnoldi step on every active column
        W = apply(np.stack([Vs[c][-1] for c in act]), act)
        for a, c in enumerate(act):
            j = len(Vs[c]) - 1
            w = W[a]
            for i in range(j + 1):
                h = np.vdot(Vs[c][i], w)
                Hs[c][i, j] = h
                w = w - h * Vs[c][i]
            hn = np.linalg.norm(w)
            Hs[c][j + 1, j] = hn
            Vs[c].append(w / hn if hn > 0 else w)
            iters[c] += 1
            Hj = Hs[c][:j + 2, :j + 1]
            y, *_ = np.linalg.lstsq(Hj, cs[c][:j + 2], rcond=None)
            rho = cs[c][:j + 2] - Hj @ y
            conv = np.linalg.norm(rho) <= tol_abs[c] or hn == 0 or iters[c] >= maxit
            if conv or j + 1 == m:
                V = np.stack(Vs[c][:j + 1])
                x[c] += np.tensordot(y, V, axes=1)
                cycles[c] += 1
                if conv:
                    done[c] = True
                    continue
                # deflated restart
                kk = min(k, m - 1)
                Vm1 = np.stack(Vs[c])                              # (m+1) basis vectors
                if kk > 0:
                    _, G = harmonic_ritz(Hs[c], kk)
                    P = np.concatenate([np.vstack([G, np.zeros((1, kk))]), rho[:, None]], axis=1)
                else:
                    P = rho[:, None]
                Q, _ = np.linalg.qr(P)
                Hn = Q.conj().T @ Hs[c] @ Q[:m, :kk]
                Vs[c] = list(np.tensordot(Q.T, Vm1, axes=1))       # V_new_i = sum_l V_l Q_li
                Hs[c] = np.zeros((m + 1, m), dtype=np.complex128)
                Hs[c][:kk + 1, :kk] = Hn
                cs[c] = np.zeros(m + 1, dtype=np.complex128)
                cs[c][:kk + 1] = Q.conj().T @ rho
                j0[c] = kk
    relres = col_norm(b - apply(x, np.arange(n))) / np.where(bnorm > 0, bnorm, 1.0)
    return x, dict(iters=iters, relres=relres, cycles=cycles)
