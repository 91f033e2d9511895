"""Oracle: aggregation, restriction/prolongation, Galerkin coarse operators,
coarse stencil, SAP and MR smoothers.  Plain FP64 numpy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.

Every level is handled through the same flat vector shape [n][V_l][d_l]
(d = 12 spin-colour components on the fine lattice, d = 2N on a coarse
lattice).  On both kinds of level the first half of the components has
chirality +1 and the second half chirality -1 (fine: spins {0,1} vs {2,3} in
the chiral basis; coarse: gamma5_c = diag(1_N, -1_N)), so one
chirality-preserving construction serves every level transition.

Section 2 of the paper: the smoother is red-black SAP (chessboard blocks, local
block inversions), the coarse-grid correction is aggregation-based AMG whose
P and R = P^dagger are built from a few approximate low modes (test vectors),
and the coarse operator lives on the coarse lattice; the construction is
applied recursively.  Fig. 6 caption: the twist on a coarse level may carry
the multiplicative factor delta-mu.
"""
from __future__ import annotations

import numpy as np

from .dirac import WilsonTM, lattice_shape

__all__ = ["Blocking", "FineLevel", "CoarseOp", "build_prolongator", "restrict", "prolong",
           "galerkin", "sap", "mr_smoother", "block_mr"]


def _axis(mu):
    return 3 - mu


# ---------------------------------------------------------------------------
# blockings (SAP blocks and aggregates)
# ---------------------------------------------------------------------------
class Blocking:
    """Partition of a lattice into equal rectangular blocks."""

    def __init__(self, dims, block):
        self.dims = tuple(int(d) for d in dims)
        self.block = tuple(int(b) for b in block)
        for d, b in zip(self.dims, self.block):
            if d % b != 0:
                raise ValueError(f"block {block} does not tile lattice {dims}")
        self.cdims = tuple(d // b for d, b in zip(self.dims, self.block))
        self.V = int(np.prod(self.dims))
        self.nblocks = int(np.prod(self.cdims))
        self.bsize = self.V // self.nblocks
        Lx, Ly, Lz, Lt = self.dims
        t, z, y, x = np.meshgrid(np.arange(Lt), np.arange(Lz), np.arange(Ly), np.arange(Lx),
                                 indexing="ij")
        bx, by, bz, bt = x // self.block[0], y // self.block[1], z // self.block[2], t // self.block[3]
        Cx, Cy, Cz, Ct = self.cdims
        self.id_lat = bx + Cx * (by + Cy * (bz + Cz * bt))      # (Lt, Lz, Ly, Lx)
        self.colour_of_block = np.zeros(self.nblocks, dtype=np.int64)
        ids = np.arange(self.nblocks)
        cx = ids % Cx; cy = (ids // Cx) % Cy; cz = (ids // (Cx * Cy)) % Cz; ct = ids // (Cx * Cy * Cz)
        self.colour_of_block = (cx + cy + cz + ct) % 2
        self.id = self.id_lat.reshape(-1)                         # per site
        self.perm = np.argsort(self.id, kind="stable")            # sites grouped by block

    def internal_mask(self, mu, forward):
        """1 where the hop x -> x +- mu stays inside the block of x."""
        nb = np.roll(self.id_lat, -1 if forward else 1, axis=_axis(mu))
        return (nb == self.id_lat).astype(np.float64)

    def block_sum(self, a):
        """a: [n][V][...] -> [n][nblocks][...] (sum over the sites of each block)."""
        n = a.shape[0]
        g = a[:, self.perm]
        return g.reshape((n, self.nblocks, self.bsize) + a.shape[2:]).sum(axis=2)

    def per_site(self, b):
        """b: [n][nblocks][...] -> [n][V][...] (broadcast block value to its sites)."""
        return b[:, self.id]


# ---------------------------------------------------------------------------
# level operators with a common interface
# ---------------------------------------------------------------------------
class FineLevel:
    """The fine twisted-mass Wilson operator seen through flat [n][V][12] vectors."""

    def __init__(self, op: WilsonTM):
        self.op = op
        self.dims = op.dims
        self.V = op.V
        self.d = 12

    def _lat(self, x):
        return self.op.to_lat(x.reshape(x.shape[0], self.V, 4, 3))

    def _flat(self, y_lat):
        return y_lat.reshape(y_lat.shape[0], self.V, 12)

    def apply(self, x, mus):
        return self.op.apply(x.reshape(x.shape[0], self.V, 4, 3), mus).reshape(x.shape[0], self.V, 12)

    def diag0(self, x):
        """The mu-independent site term (4 + m0) x, plus the clover term when
        the operator has one."""
        if self.op.clover is None:
            return (4.0 + self.op.m0) * x
        return self._flat(self.op.site_term(self._lat(x)))

    def twist(self, x):
        """gamma5 x (the twist is i*mu times this)."""
        y = x.copy()
        y[:, :, 6:] *= -1.0
        return y

    def hop(self, x, mu, forward):
        p = self._lat(x)
        h = self.op.hop_forward(p, mu) if forward else self.op.hop_backward(p, mu)
        return self._flat(h)

    def masked_hop(self, x, mu, forward, mask_lat):
        h = self.hop(x, mu, forward)
        return h * mask_lat.reshape(-1)[None, :, None]

    def apply_block_diag(self, x, mus, blocking: Blocking):
        """D with every hop that leaves its block removed (Dirichlet blocks)."""
        y = self.diag0(x) + 1j * np.asarray(mus).reshape(-1, 1, 1) * self.twist(x)
        for mu in range(4):
            for fw in (True, False):
                y = y + self.masked_hop(x, mu, fw, blocking.internal_mask(mu, fw))
        return y


class CoarseOp:
    """Coarse stencil: per coarse site a self block and eight hop blocks, each
    d x d complex (d = 2N):

        y(a) = A0(a) phi(a) + i*dmu*mu gamma5_c phi(a)
               + sum_nu [ F_nu(a) phi(a + nu) + B_nu(a) phi(a - nu) ]

    blocks: complex128 [Vc][9][d][d], slot 0 = A0, 1+nu = F_nu, 5+nu = B_nu.
    Boundary signs of the fine hops are contained in the blocks."""

    def __init__(self, blocks, dims, mu_factor=1.0):
        self.blocks = np.asarray(blocks, dtype=np.complex128)
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.d = self.blocks.shape[-1]
        assert self.blocks.shape == (self.V, 9, self.d, self.d)
        self.lat = lattice_shape(self.dims)
        self.mu_factor = float(mu_factor)

    def _lat(self, x):
        return x.reshape((x.shape[0],) + self.lat + (self.d,))

    def _mat(self, slot):
        return self.blocks[:, slot].reshape(self.lat + (self.d, self.d))

    def diag0(self, x):
        return np.einsum("vij,nvj->nvi", self.blocks[:, 0], x)

    def twist(self, x):
        y = x.copy()
        y[:, :, self.d // 2:] *= -1.0
        return y

    def hop(self, x, mu, forward):
        p = self._lat(x)
        nb = np.roll(p, -1 if forward else 1, axis=1 + _axis(mu))
        M = self._mat(1 + mu if forward else 5 + mu)
        y = np.einsum("...ij,n...j->n...i", M, nb)
        return y.reshape(x.shape)

    def masked_hop(self, x, mu, forward, mask_lat):
        return self.hop(x, mu, forward) * mask_lat.reshape(-1)[None, :, None]

    def apply(self, x, mus):
        mus = np.asarray(mus, dtype=np.float64).reshape(-1, 1, 1)
        y = self.diag0(x) + 1j * self.mu_factor * mus * self.twist(x)
        for mu in range(4):
            y = y + self.hop(x, mu, True) + self.hop(x, mu, False)
        return y

    def apply_block_diag(self, x, mus, blocking: Blocking):
        mus = np.asarray(mus, dtype=np.float64).reshape(-1, 1, 1)
        y = self.diag0(x) + 1j * self.mu_factor * mus * self.twist(x)
        for mu in range(4):
            for fw in (True, False):
                y = y + self.masked_hop(x, mu, fw, blocking.internal_mask(mu, fw))
        return y


# ---------------------------------------------------------------------------
# prolongation / restriction
# ---------------------------------------------------------------------------
def build_prolongator(tv, aggs: Blocking):
    """Orthonormalise test vectors per (aggregate, chirality).

    tv: [N][V][d] test vectors.  Returns P as [V][d][N]: for a site x in
    aggregate a and a component k of chirality s, P[x, k, j] is entry (x, k)
    of coarse basis vector (a, s, j).  QR with R_ii > 0 (unique for full
    rank), so every orthonormalisation method gives the same P."""
    N, V, d = tv.shape
    h = d // 2
    P = np.zeros((V, d, N), dtype=np.complex128)
    for s in range(2):
        comp = slice(s * h, (s + 1) * h)
        # M[a] = stack over (site in aggregate, component of chirality s) x N
        sub = tv[:, :, comp]                                  # [N][V][h]
        grouped = sub[:, aggs.perm].reshape(N, aggs.nblocks, aggs.bsize * h)
        M = np.transpose(grouped, (1, 2, 0))                  # [nagg][bsize*h][N]
        Q, R = np.linalg.qr(M)
        ph = np.diagonal(R, axis1=-2, axis2=-1)
        ph = ph / np.abs(ph)
        Q = Q * ph[:, None, :]                                 # makes R_ii > 0
        Qs = Q.reshape(aggs.nblocks * aggs.bsize, h, N)
        P[aggs.perm, comp, :] = Qs
    return P


def restrict(P, aggs: Blocking, x):
    """(R x)[n, a, s*N + j] = sum_{y in A_a} sum_{k of chirality s} conj(P[y,k,j]) x[n,y,k]."""
    V, d, N = P.shape
    h = d // 2
    out = []
    for s in range(2):
        comp = slice(s * h, (s + 1) * h)
        per_site = np.einsum("vkj,nvk->nvj", np.conj(P[:, comp, :]), x[:, :, comp])
        out.append(aggs.block_sum(per_site))
    return np.concatenate(out, axis=2)                      # [n][nagg][2N]


def prolong(P, aggs: Blocking, xc):
    """(P xc)[n, y, k] = sum_j P[y, k, j] xc[n, a(y), s(k)*N + j]."""
    V, d, N = P.shape
    h = d // 2
    per_site = aggs.per_site(xc)                            # [n][V][2N]
    y = np.empty((xc.shape[0], V, d), dtype=np.complex128)
    for s in range(2):
        comp = slice(s * h, (s + 1) * h)
        y[:, :, comp] = np.einsum("vkj,nvj->nvk", P[:, comp, :], per_site[:, :, s * N:(s + 1) * N])
    return y


def galerkin(level, P, aggs: Blocking, mu_factor=1.0):
    """D_c(0) = P^dagger D(0) P assembled blockwise on the coarse lattice.

    The basis field X[s*N + j] holds P[:, comp of chirality s, j] on every
    aggregate.  A hop term restricted to links that cross from A_a into
    A_{a +- nu} and then restricted by R gives the hop block of aggregate a;
    the diagonal plus the hops internal to each aggregate give its self block.
    """
    V, d, N = P.shape
    h = d // 2
    X = np.zeros((2 * N, V, d), dtype=np.complex128)
    for s in range(2):
        comp = slice(s * h, (s + 1) * h)
        X[s * N:(s + 1) * N, :, comp] = np.transpose(P[:, comp, :], (2, 0, 1))
    nagg = aggs.nblocks
    blocks = np.zeros((nagg, 9, 2 * N, 2 * N), dtype=np.complex128)
    self_part = level.diag0(X)
    for mu in range(4):
        for fw in (True, False):
            inner = aggs.internal_mask(mu, fw)
            self_part = self_part + level.masked_hop(X, mu, fw, inner)
            cross = level.masked_hop(X, mu, fw, 1.0 - inner)
            Rc = restrict(P, aggs, cross)                      # [2N cols][nagg][2N rows]
            blocks[:, (1 if fw else 5) + mu] = np.transpose(Rc, (1, 2, 0))
    R0 = restrict(P, aggs, self_part)
    blocks[:, 0] = np.transpose(R0, (1, 2, 0))
    return CoarseOp(blocks, aggs.cdims, mu_factor=mu_factor)


# ---------------------------------------------------------------------------
# smoothers
# ---------------------------------------------------------------------------
def _dot_block(blocking: Blocking, a, b):
    """per (column, block): sum over the block's sites of conj(a) b."""
    return blocking.block_sum(np.sum(np.conj(a) * b, axis=2))     # [n][nblocks]


def block_mr(level, blocking: Blocking, r, mus, iters):
    """Minimal-residual iterations on every block at once, from zero:
    alpha = <D_BB rho, rho> / <D_BB rho, D_BB rho>;  delta += alpha rho;
    rho -= alpha D_BB rho   (alpha per column and per block)."""
    delta = np.zeros_like(r)
    rho = r.copy()
    for _ in range(iters):
        q = level.apply_block_diag(rho, mus, blocking)
        num = _dot_block(blocking, q, rho)
        den = _dot_block(blocking, q, q).real
        alpha = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        a = blocking.per_site(alpha)[:, :, None]
        delta = delta + a * rho
        rho = rho - a * q
    return delta


def site_parity(dims):
    """(x + y + z + t) mod 2 per site (lexicographic site order)."""
    Lx, Ly, Lz, Lt = dims
    i = np.arange(int(np.prod(dims)))
    return ((i % Lx) + (i // Lx) % Ly + (i // (Lx * Ly)) % Lz + i // (Lx * Ly * Lz)) % 2


def block_mr_oddeven(level, blocking: Blocking, r, mus, iters):
    """Block solves by minimal residual on the odd-even reduced block systems.

    Inside a block with even extents every hop joins an even and an odd site,
    so with the site term D_ee (on even sites) and D_oo (odd sites) and the
    hop parts D_eo, D_oe of D_BB:
        D_BB x = r  <=>  S x_o = r_o - D_oe D_ee^{-1} r_e,   S = D_oo - D_oe D_ee^{-1} D_eo,
                         x_e = D_ee^{-1} (r_e - D_eo x_o).
    `iters` MR steps on S from zero (alpha per column and block), then the
    even half by back substitution.  D_ee = (4 + m0) + i mu gamma5 is
    inverted per chirality (no clover term)."""
    assert getattr(level.op, "clover", None) is None, "odd-even block solves are for the clover-free operator"
    mus = np.asarray(mus, dtype=np.float64).reshape(-1, 1, 1)
    odd = site_parity(level.dims)[None, :, None].astype(np.float64)
    even = 1.0 - odd
    d0 = 4.0 + level.op.m0
    g5 = np.concatenate([np.ones(6), -np.ones(6)])[None, None, :]

    def site(v):               # D_ee or D_oo on a vector (site-local)
        return (d0 + 1j * mus * g5) * v

    def site_inv(v):
        return v / (d0 + 1j * mus * g5)

    def hops(v):               # the hop part of D_BB (in-block hops only)
        return level.apply_block_diag(v, mus.reshape(-1), blocking) - site(v)

    r_e, r_o = r * even, r * odd
    rhs = r_o - odd * hops(site_inv(r_e))

    def schur(v):
        return odd * (site(v) - hops(site_inv(even * hops(v))))

    x_o = np.zeros_like(r)
    rho = rhs.copy()
    for _ in range(iters):
        q = schur(rho)
        num = _dot_block(blocking, q, rho)
        den = _dot_block(blocking, q, q).real
        alpha = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)
        a = blocking.per_site(alpha)[:, :, None]
        x_o = x_o + a * rho
        rho = rho - a * q
    x_e = even * site_inv(r_e - even * hops(x_o))
    return x_o + x_e


def sap(level, blocking: Blocking, f, mus, cycles, mr_iters, x0=None, oddeven=False):
    """Red-black Schwarz alternating procedure (paper section 2): for each
    colour in turn, the residual on that colour's blocks is reduced by an
    approximate local inversion (block MR, on the plain or the odd-even
    reduced block systems), all blocks of one colour at once."""
    x = np.zeros_like(f) if x0 is None else x0.copy()
    solve = block_mr_oddeven if oddeven else block_mr
    for _ in range(cycles):
        for colour in (0, 1):
            on = (blocking.colour_of_block[blocking.id] == colour).astype(np.float64)
            r = (f - level.apply(x, mus)) * on[None, :, None]
            x = x + solve(level, blocking, r, mus, mr_iters)
    return x


def mr_smoother(level, f, mus, iters, x0=None):
    """Global minimal-residual steps per column (coarse-level smoother)."""
    x = np.zeros_like(f) if x0 is None else x0.copy()
    r = f - level.apply(x, mus)
    for _ in range(iters):
        q = level.apply(r, mus)
        num = np.sum(np.conj(q) * r, axis=(1, 2))
        den = np.sum(np.abs(q) ** 2, axis=(1, 2))
        alpha = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)[:, None, None]
        x = x + alpha * r
        r = r - alpha * q
    return x
