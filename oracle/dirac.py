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

Clover term (optional, c_sw != 0).  The paper's ensembles are twisted-mass
clover (section 2, Fig. 1 caption) but it gives no formula, so the standard
Sheikholeslami-Wohlert term is taken, in the m0 normalisation above:

    D(mu) += c_sw (i/4) sum_{mu != nu} sigma_{mu nu} F_{mu nu}(x)
    sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu]
    F_{mu nu}(x)  = (Q_{mu nu}(x) - Q_{mu nu}(x)^dagger) / 8

where Q_{mu nu}(x) is the sum of the four plaquettes of the (mu, nu) plane
that start and end at x, all run in the same sense (mu before nu).  Closed
loops cross the time boundary an even number of times, so the antiperiodic
sign drops out.  The term is Hermitian and commutes with gamma5, so it keeps
gamma5-hermiticity and splits into one 6x6 block per chirality.

Arrays: gauge complex128 [V][4][3][3]; spinor multivector complex128
[n][V][4][3] with site index i = x + Lx*(y + Ly*(z + Lz*t)).
"""
from __future__ import annotations

import numpy as np

__all__ = ["gammas", "gamma5", "sigma_munu", "clover_field", "WilsonTM", "lattice_shape"]


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


def sigma_munu() -> np.ndarray:
    """sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu], shape (4, 4, 4, 4)."""
    g = gammas()
    out = np.zeros((4, 4, 4, 4), dtype=np.complex128)
    for m in range(4):
        for n in range(4):
            out[m, n] = 0.5j * (g[m] @ g[n] - g[n] @ g[m])
    return out


def _dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def clover_field(U_lat, csw):
    """The clover term as a per-site 12x12 matrix, shape lat + (4, 3, 4, 3)
    (spin, colour, spin, colour).  U_lat[mu]: lat + (3, 3)."""
    def at(a, steps):
        """a(x + sum_d s_d d) for steps = {direction: s_d}."""
        for d, k in steps.items():
            a = np.roll(a, -k, axis=_axis(d))
        return a

    sig = sigma_munu()
    lat = U_lat[0].shape[:4]
    C = np.zeros(lat + (4, 3, 4, 3), dtype=np.complex128)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            Um, Un = U_lat[mu], U_lat[nu]
            # the four leaves: (+mu, +nu, -mu, -nu) and its three rotations
            l1 = Um @ at(Un, {mu: 1}) @ _dag(at(Um, {nu: 1})) @ _dag(Un)
            l2 = Un @ _dag(at(Um, {nu: 1, mu: -1})) @ _dag(at(Un, {mu: -1})) @ at(Um, {mu: -1})
            l3 = _dag(at(Um, {mu: -1})) @ _dag(at(Un, {mu: -1, nu: -1})) @ at(Um, {mu: -1, nu: -1}) @ at(Un, {nu: -1})
            l4 = _dag(at(Un, {nu: -1})) @ at(Um, {nu: -1}) @ at(Un, {nu: -1, mu: 1}) @ _dag(Um)
            Q = l1 + l2 + l3 + l4
            F = (Q - _dag(Q)) / 8.0
            C += csw * 0.25j * np.einsum("ac,...bd->...abcd", sig[mu, nu], F)
    return C


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

    def __init__(self, U: np.ndarray, dims, kappa: float = None, m0: float = None, csw: float = 0.0):
        self.dims = tuple(int(d) for d in dims)
        self.csw = float(csw)
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
        self._clover = None

    @property
    def clover(self):
        """The clover field (computed on first use; None without a clover term)."""
        if self.csw != 0.0 and self._clover is None:
            self._clover = clover_field(self.U, self.csw)
        return self._clover

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

    def clover_apply(self, psi_lat):
        """The clover term on lattice-shaped spinors [n] + lat + (4, 3) (zero
        without a clover term)."""
        if self.clover is None:
            return np.zeros_like(psi_lat)
        return np.einsum("...abcd,n...cd->n...ab", self.clover, psi_lat)

    def site_term(self, psi_lat):
        """The mu-independent site term (4 + m0) psi + clover psi."""
        out = (4.0 + self.m0) * psi_lat
        if self.clover is not None:
            out = out + self.clover_apply(psi_lat)
        return out

    def diag(self, psi_lat, mus):
        """(4 + m0 + clover) psi + i mu gamma5 psi, mu per column."""
        mus = np.asarray(mus, dtype=np.float64).reshape(-1)
        out = self.site_term(psi_lat)
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
            if self.csw != 0.0:
                acc = acc + np.einsum("abcd,ncd->nab", self.clover_at_site(i), psi[:, i])
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

    def clover_at_site(self, i):
        """The 12x12 clover matrix (4, 3, 4, 3) of site i, evaluated loop by
        loop from the links around the site (independent of the field form)."""
        Lx, Ly, Lz, Lt = self.dims
        Uflat = [u.reshape(self.V, 3, 3) for u in self.U]
        c0 = [i % Lx, (i // Lx) % Ly, (i // (Lx * Ly)) % Lz, i // (Lx * Ly * Lz)]

        def idx(c):
            return (c[0] % Lx) + Lx * ((c[1] % Ly) + Ly * ((c[2] % Lz) + Lz * (c[3] % Lt)))

        def link(c, d, forward):
            """the parallel transporter of one step from site c along +d
            (forward) or -d (backward)."""
            if forward:
                return Uflat[d][idx(c)]
            cb = list(c); cb[d] -= 1
            return np.conj(Uflat[d][idx(cb)]).T

        sig = sigma_munu()
        C = np.zeros((4, 3, 4, 3), dtype=np.complex128)
        for mu in range(4):
            for nu in range(4):
                if mu == nu:
                    continue
                Q = np.zeros((3, 3), dtype=np.complex128)
                for first, second in ((mu, nu), (nu, -mu - 1), (-mu - 1, -nu - 1), (-nu - 1, mu)):
                    # walk first, second, -first, -second (negative codes: backward)
                    path = [first, second, (-first - 1), (-second - 1)]
                    c = list(c0)
                    M = np.eye(3, dtype=np.complex128)
                    for step in path:
                        d, fw = (step, True) if step >= 0 else (-step - 1, False)
                        M = M @ link(c, d, fw)
                        c[d] += 1 if fw else -1
                    assert [a % n for a, n in zip(c, self.dims)] == [a % n for a, n in zip(c0, self.dims)]
                    Q += M
                F = (Q - Q.conj().T) / 8.0
                C += self.csw * 0.25j * np.einsum("ac,bd->abcd", sig[mu, nu], F)
        return C

    def gamma5_apply(self, psi):
        return np.einsum("st,nvtc->nvsc", self.g5, psi)
