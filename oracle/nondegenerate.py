"""Oracle: the non-degenerate twisted-mass operator on flavour doublets.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Section 1 of the paper: the multigrid method was generalised from the
degenerate to the non-degenerate twisted-mass operator.  The paper prints no
formula; the reading taken is the standard doublet operator

    D_ND(mubar, epsbar) = D_W (x) 1_f + i mubar gamma5 (x) tau3 - epsbar 1 (x) tau1

acting on psi = (psi_u, psi_d):

    (D_ND psi)_u = D(+mubar) psi_u - epsbar psi_d
    (D_ND psi)_d = D(-mubar) psi_d - epsbar psi_u

with D(mu) the degenerate operator of ``dirac.WilsonTM`` (m0 form, clover
term when present).  A doublet is stored as two consecutive columns
[pair][flavour u, d][V][4][3]; every pair has its own (mubar, epsbar).
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonTM

__all__ = ["nd_apply", "nd_mus"]


def nd_mus(mubar):
    """Per-column twisted masses of doublets: (+mubar_i, -mubar_i)."""
    mubar = np.asarray(mubar, dtype=np.float64).reshape(-1)
    return np.stack([mubar, -mubar], axis=1).reshape(-1)


def nd_apply(op: WilsonTM, psi, mubar, epsbar):
    """y = D_ND(mubar_i, epsbar_i) psi_i for every doublet i.
    psi: [n_pair][2][V][4][3] (or [2 n_pair][V][4][3]); returns the same shape."""
    psi = np.asarray(psi, dtype=np.complex128)
    shape = psi.shape
    n_pair = np.asarray(mubar).reshape(-1).size
    cols = psi.reshape(2 * n_pair, op.V, 4, 3)
    y = op.apply(cols, nd_mus(mubar)).reshape(n_pair, 2, op.V, 4, 3)
    eps = np.asarray(epsbar, dtype=np.float64).reshape(n_pair, 1, 1, 1)
    c = cols.reshape(n_pair, 2, op.V, 4, 3)
    y[:, 0] -= eps * c[:, 1]
    y[:, 1] -= eps * c[:, 0]
    return y.reshape(shape)
