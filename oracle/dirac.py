"""Oracle: the degenerate twisted-mass Wilson-Dirac operator, plain FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Operator (the paper's twisted-mass operator D_TM = D_W + i*dmu*mu*gamma5, Fig. 6
caption, with the Wilson part written in the m0 normalisation):

    D(mu) psi(x) = (4 + m0) psi(x) + i mu gamma5 psi(x)
                   - 1/2 sum_nu [ (1 - gamma_nu) U_nu(x) psi(x + nu)
                                + (1 + gamma_nu) U_nu(x - nu)^dagger psi(x - nu) ]

with m0 = 1/(2 kappa) - 4, periodic boundaries in x, y, z and antiperiodic in t
(a factor -1 on every hop that crosses the t = Lt-1 <-> 0 boundary; the factor
is applied to the hop, never folded into the links).

Gamma basis (chiral, Hermitian, Euclidean):
    gamma_k = [[0, -i sigma_k], [i sigma_k, 0]]   k = 1, 2, 3  (x, y, z)
    gamma_4 = [[0, 1], [1, 0]]                     (t)
    gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4 = diag(1, 1, -1, -1)
so chirality +1 is spins {0, 1} and chirality -1 is spins {2, 3}.

Arrays: gauge complex128 [V][4][3][3]; spinor multivector complex128
[n][V][4][3] with site index i = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np

__all__ = ["gammas", "gamma5", "WilsonTM", "lattice_shape"]


def gammas() -> np.ndarray:
    """gamma_1..gamma_4 in the chiral basis, shape (4, 4, 4), index mu = 0..3."""
    s1 = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    s2 = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    s3 = np.array([[1, 0], [0, -1]], dtype=np.complex128)
    z = np.zeros((2, 2), dtype=np.complex128)
    g = []
    for s in (s1, s2, s3):
        g.append(np.block([[z, -1j * s], [1j * s, z]]))
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return np.array(g)


def gamma5() -> np.ndarray:
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


def lattice_shape(dims):
    """numpy axis order (Lt, Lz, Ly, Lx) of a lexicographic site index."""
    Lx, Ly, Lz, Lt = dims
    return (Lt, Lz, Ly, Lx)


def _axis(mu: int) -> int:
    """lattice axis (in the (Lt, Lz, Ly, Lx) order) of direction mu."""
    return 3 - mu


def _colour(U, psi, dagger=False):
    """out[..., s, a] = sum_b U[..., a, b] psi[..., s, b]  (or U^dagger)."""
    out = np.zeros_like(psi)
    for a in range(3):
        for b in range(3):
            u = np.conj(U[..., b, a]) if dagger else U[..., a, b]
            out[..., :, a] += u[..., None] * psi[..., :, b]
    return out


def _spin(G, psi):
    """out[..., s, c] = sum_t G[s, t] psi[..., t, c]."""
    out = np.zeros_like(psi)
    for s in range(4):
        for t in range(4):
            if G[s, t] != 0:
                out[..., s, :] += G[s, t] * psi[..., t, :]
    return out


class WilsonTM:
    """FP64 twisted-mass Wilson operator on a 4-d lattice."""

    def __init__(self, U: np.ndarray, dims, kappa: float = None, m0: float = None):
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        if m0 is None:
            m0 = 1.0 / (2.0 * kappa) - 4.0
        self.m0 = float(m0)
        self.lat = lattice_shape(self.dims)
        U = np.asarray(U, dtype=np.complex128)
        assert U.shape == (self.V, 4, 3, 3)
        # U_lat[mu] has shape (Lt, Lz, Ly, Lx, 3, 3)
        self.U = [U[:, mu].reshape(self.lat + (3, 3)) for mu in range(4)]
        self.g = gammas()
        self.g5 = gamma5()
        self.one = np.eye(4, dtype=np.complex128)
        # boundary sign fields: forward hop from t = Lt-1 and backward hop from t = 0
        Lt = self.dims[3]
        self.bc_fwd = np.ones(self.lat[:1] + (1, 1, 1), dtype=np.float64)
        self.bc_fwd[Lt - 1] = -1.0
        self.bc_bwd = np.ones(self.lat[:1] + (1, 1, 1), dtype=np.float64)
        self.bc_bwd[0] = -1.0

    # -- shapes --------------------------------------------------------------
    def to_lat(self, psi):
        n = psi.shape[0]
        return psi.reshape((n,) + self.lat + (4, 3))

    def from_lat(self, psi_lat):
        n = psi_lat.shape[0]
        return psi_lat.reshape((n, self.V, 4, 3))

    # -- the hop terms -------------------------------------------------------
    def hop_forward(self, psi_lat, mu):
        """-1/2 (1 - gamma_mu) U_mu(x) psi(x + mu), with the t boundary sign."""
        ax = 1 + _axis(mu)
        nb = np.roll(psi_lat, -1, axis=ax)
        if mu == 3:
            nb = nb * self.bc_fwd[None, ..., None, None]
        t = _colour(self.U[mu][None], nb)
        return -0.5 * _spin(self.one - self.g[mu], t)

    def hop_backward(self, psi_lat, mu):
        """-1/2 (1 + gamma_mu) U_mu(x - mu)^dagger psi(x - mu), with the t sign."""
        ax = 1 + _axis(mu)
        nb = np.roll(psi_lat, 1, axis=ax)
        if mu == 3:
            nb = nb * self.bc_bwd[None, ..., None, None]
        Ub = np.roll(self.U[mu], 1, axis=_axis(mu))
        t = _colour(Ub[None], nb, dagger=True)
        return -0.5 * _spin(self.one + self.g[mu], t)

    def diag(self, psi_lat, mus):
        """(4 + m0) psi + i mu gamma5 psi, mu per column."""
        mus = np.asarray(mus, dtype=np.float64).reshape(-1)
        out = (4.0 + self.m0) * psi_lat
        tw = _spin(self.g5, psi_lat)
        out = out + 1j * mus.reshape((-1,) + (1,) * (psi_lat.ndim - 1)) * tw
        return out

    # -- the operator --------------------------------------------------------
    def apply(self, psi, mus, hop_weight=None):
        """y = D(mu_c) psi_c for every column c.  psi: [n][V][4][3].

        hop_weight(mu, forward) -> None or a lattice-shaped 0/1 mask that
        multiplies the hop term (used to restrict hops to blocks)."""
        psi = np.asarray(psi, dtype=np.complex128)
        p = self.to_lat(psi)
        out = self.diag(p, mus)
        for mu in range(4):
            f = self.hop_forward(p, mu)
            b = self.hop_backward(p, mu)
            if hop_weight is not None:
                wf = hop_weight(mu, True)
                wb = hop_weight(mu, False)
                if wf is not None:
                    f = f * wf[None, ..., None, None]
                if wb is not None:
                    b = b * wb[None, ..., None, None]
            out = out + f + b
        return self.from_lat(out)

    def apply_site(self, psi, mus, sites):
        """(D psi)(x) at the listed sites only, by direct evaluation of the
        stencil formula site by site (for sampled checks of large lattices)."""
        Lx, Ly, Lz, Lt = self.dims
        psi = np.asarray(psi)
        mus = np.asarray(mus, dtype=np.float64).reshape(-1)
        Uflat = [u.reshape(self.V, 3, 3) for u in self.U]
        out = np.zeros((psi.shape[0], len(sites), 4, 3), dtype=np.complex128)
        for k, i in enumerate(sites):
            x = i % Lx; y = (i // Lx) % Ly; z = (i // (Lx * Ly)) % Lz; t = i // (Lx * Ly * Lz)
            c = [x, y, z, t]
            acc = (4.0 + self.m0) * psi[:, i] + 1j * mus[:, None, None] * np.einsum(
                "st,ntc->nsc", self.g5, psi[:, i])
            for mu in range(4):
                cf = list(c); cf[mu] = (c[mu] + 1) % self.dims[mu]
                cb = list(c); cb[mu] = (c[mu] - 1) % self.dims[mu]
                jf = cf[0] + Lx * (cf[1] + Ly * (cf[2] + Lz * cf[3]))
                jb = cb[0] + Lx * (cb[1] + Ly * (cb[2] + Lz * cb[3]))
                sf = -1.0 if (mu == 3 and t == Lt - 1) else 1.0
                sb = -1.0 if (mu == 3 and t == 0) else 1.0
                hf = np.einsum("ab,nsb->nsa", Uflat[mu][i], psi[:, jf]) * sf
                hb = np.einsum("ba,nsb->nsa", np.conj(Uflat[mu][jb]), psi[:, jb]) * sb
                acc = acc - 0.5 * (np.einsum("st,ntc->nsc", self.one - self.g[mu], hf)
                                   + np.einsum("st,ntc->nsc", self.one + self.g[mu], hb))
            out[:, k] = acc
        return out

    def gamma5_apply(self, psi):
        return np.einsum("st,nvtc->nvsc", self.g5, psi)
