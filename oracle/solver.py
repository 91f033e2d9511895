"""Oracle: the multigrid-preconditioned multi-rhs x multi-shift solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Method (paper sections 2 and 4): FGMRES at the top level to a 1e-10 relative
residual, preconditioned by a multigrid cycle combining the red-black SAP
smoother with aggregation-based coarse-grid correction, applied recursively.
The middle level is solved by (non-block) FGMRES to r_m ~ 7e-2 preconditioned
by the next level, the bottom by GMRES (or block GMRES) to r_b ~ 1e-1.
Every right-hand side and every twisted-mass shift is one column; all columns
are inverted simultaneously.  The coarse operator is built once at mu = 0 and
the twist i*mu*gamma5_c is added per column, so one hierarchy serves every
shift (the coarse twist identity P^H (i mu gamma5) P = i mu gamma5_c).

Readings where the paper is silent (all documented with the build):
cycle = post-smoothing only; coarse-level smoother = a few MR steps;
setup = a few SAP (fine) / fixed-length GMRES (coarse) smoothing rounds of
random vectors, each followed by normalisation.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .dirac import WilsonTM
from .multigrid import (Blocking, FineLevel, CoarseOp, build_prolongator, restrict, prolong,
                        galerkin, sap, mr_smoother)
from .krylov import gmres, fgmres, block_gmres, gmres_dr, col_norm

__all__ = ["MGParams", "OracleMG"]


@dataclass
class MGParams:
    agg: tuple = ((2, 2, 2, 2),)
    n_tv: tuple = (8,)
    sap_block: tuple = (2, 2, 2, 2)
    sap_cycles: int = 4
    sap_mr: int = 4
    setup_rounds: int = 3               # smoothing rounds of the random start vectors
    setup_coarse_iters: int = 10        # fixed GMRES length per coarse setup round
    mu_setup: float = 0.0
    coarse_mu_factor: float = 1.0       # delta-mu on the coarsest level
    tol: float = 1e-10
    outer_restart: int = 10
    max_outer: int = 500
    r_m: float = 7e-2                   # middle-level relative tolerance
    r_b: float = 1e-1                   # bottom relative tolerance
    middle_restart: int = 20
    middle_maxit: int = 50
    bottom_maxit: int = 100
    coarse_smooth_iters: int = 2        # MR steps of the middle-level smoother
    coarsest_block: bool = False
    coarse_gamma5: int = 0              # Krylov on gamma5_c D_c: 0 off, 1 coarsest, 2 every coarse level
    bottom_dr_k: int = 0                # > 0: GMRES-DR(bottom_restart, k) at the coarsest level
    bottom_restart: int = 63


class OracleMG:
    def __init__(self, U, dims, kappa, params: MGParams):
        self.p = params
        self.fine_op = WilsonTM(U, dims, kappa=kappa)
        self.levels = [FineLevel(self.fine_op)]
        self.blockings: List[Blocking] = []
        self.P: List[np.ndarray] = []
        self.sap_blocking = Blocking(dims, params.sap_block)
        self.dims = [tuple(dims)]
        self.stats = dict(middle_iters=[], bottom_iters=[])

    # -- setup -----------------------------------------------------------------
    def setup(self, start_vectors):
        """start_vectors[l]: the random vectors of level transition l."""
        p = self.p
        for l, (agg, n) in enumerate(zip(p.agg, p.n_tv)):
            lev = self.levels[l]
            v = np.asarray(start_vectors[l], dtype=np.complex128).reshape(n, lev.V, lev.d)
            mus = np.full(n, p.mu_setup)
            for _ in range(p.setup_rounds):
                if l == 0:
                    v = sap(lev, self.sap_blocking, v, mus, p.sap_cycles, p.sap_mr)
                else:
                    v, _ = gmres(lambda x, act: lev.apply(x, mus[act]), v, 0.0, p.setup_coarse_iters)
                v = v / col_norm(v)[:, None, None]
            self.add_level(v, agg)
        return self

    def add_level(self, tv, agg):
        l = len(self.P)
        lev = self.levels[l]
        blk = Blocking(lev.dims, agg)
        P = build_prolongator(tv, blk)
        last = (l + 1 == len(self.p.agg))
        coarse = galerkin(lev, P, blk, mu_factor=self.p.coarse_mu_factor if last else 1.0)
        self.blockings.append(blk)
        self.P.append(P)
        self.levels.append(coarse)
        self.dims.append(blk.cdims)
        return coarse

    # -- cycle -----------------------------------------------------------------
    def cycle(self, l, r, mus):
        """MG_l(r): restrict, solve the next level (FGMRES to r_m preconditioned
        recursively, or GMRES / block GMRES to r_b at the bottom), prolong, then
        post-smooth the remaining residual."""
        p = self.p
        lev, nxt = self.levels[l], self.levels[l + 1]
        rc = restrict(self.P[l], self.blockings[l], r)
        bottom = (l + 2 == len(self.levels))
        # gamma5-Hermitian form: gamma5_c D_c(mu) e_c = gamma5_c r_c has the same
        # solution and residual norm; its operator Q_c + i dmu mu is normal
        g5 = p.coarse_gamma5 >= (1 if bottom else 2)
        op = (lambda x, m: nxt.twist(nxt.apply(x, m))) if g5 else nxt.apply
        rhs = nxt.twist(rc) if g5 else rc
        if bottom:
            if p.coarsest_block:
                ec = np.zeros_like(rc)
                for mu in np.unique(mus):
                    idx = np.nonzero(mus == mu)[0]
                    sol, info = block_gmres(lambda x, m=mu: op(x, np.full(x.shape[0], m)),
                                            rhs[idx], p.r_b, p.bottom_maxit)
                    ec[idx] = sol
                    self.stats["bottom_iters"].append(info["iters"])
            elif p.bottom_dr_k > 0:
                ec, info = gmres_dr(lambda x, act: op(x, mus[act]), rhs, p.r_b, p.bottom_restart, p.bottom_dr_k,
                                    p.bottom_maxit)
                self.stats["bottom_iters"].extend(list(info["iters"]))
            else:
                ec, info = gmres(lambda x, act: op(x, mus[act]), rhs, p.r_b, p.bottom_maxit)
                self.stats["bottom_iters"].extend(list(info["iters"]))
        else:
            # a preconditioner of gamma5_c D_c approximates D_c^-1 gamma5_c
            pre = (lambda x, act: self.cycle(l + 1, nxt.twist(x), mus[act])) if g5 else \
                  (lambda x, act: self.cycle(l + 1, x, mus[act]))
            ec, info = fgmres(lambda x, act: op(x, mus[act]), pre, rhs, p.r_m, p.middle_restart, p.middle_maxit)
            self.stats["middle_iters"].extend(list(info["iters"]))
        e = prolong(self.P[l], self.blockings[l], ec)
        res = r - lev.apply(e, mus)
        if l == 0:
            e = e + sap(lev, self.sap_blocking, res, mus, p.sap_cycles, p.sap_mr)
        else:
            e = e + mr_smoother(lev, res, mus, p.coarse_smooth_iters)
        return e

    # -- solve -------------------------------------------------------------------
    def solve(self, b, mus, x0=None):
        """x_c = D(mu_c)^{-1} b_c for every column, b: [n][V][4][3], mus: [n]."""
        p = self.p
        lev = self.levels[0]
        n = b.shape[0]
        bf = np.asarray(b, dtype=np.complex128).reshape(n, lev.V, 12)
        mus = np.asarray(mus, dtype=np.float64)
        x0f = None if x0 is None else np.asarray(x0).reshape(n, lev.V, 12)
        if len(self.levels) == 1:
            prec = lambda x, act: sap(lev, self.sap_blocking, x, mus[act], p.sap_cycles, p.sap_mr)
        else:
            prec = lambda x, act: self.cycle(0, x, mus[act])
        x, info = fgmres(lambda x, act: lev.apply(x, mus[act]), prec, bf, p.tol,
                         p.outer_restart, p.max_outer, x0=x0f)
        return x.reshape(n, lev.V, 4, 3), info

    def true_relres(self, b, x, mus):
        r = b - self.fine_op.apply(x, mus)
        return col_norm(r) / col_norm(b)
