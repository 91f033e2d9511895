"""Seeded synthetic inputs for the twisted-mass multigrid workloads.

This module only *draws* inputs: gauge links, right-hand sides, twisted-mass
shifts and the random starting vectors of the multigrid setup.  It contains
none of the solver's arithmetic (no Dirac operator, no projection, no Krylov
step), so that both the FP64 oracle and the GPU library can be fed the same
arrays without sharing any computational code.

Canonical array layouts (the C-ABI layouts):

* site index ``i = x + Lx*(y + Ly*(z + Lz*t))``; directions ``mu = 0..3 = x,y,z,t``
* gauge: complex128 ``[V][mu][row 3][col 3]``; ``U[x][mu]`` connects ``x`` to
  ``x + mu``.  No boundary phase is folded into the links.
* spinor multivector: complex128 ``[col][V][spin 4][colour 3]``; for a batch of
  ``n_rhs`` right-hand sides and ``n_shift`` shifts the column index is
  ``col = r*n_shift + k``.
* coarse multivector: complex128 ``[col][Vc][2N]``.

The gauge recipe ``U = exp(i*eps*H)`` with ``H`` a Gaussian traceless Hermitian
3x3 matrix, re-unitarised, follows the workload definitions of the multi-shift
twisted-mass study (the paper itself uses dynamical ensembles, which are not
available here; these seeded fields stand in for them).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "workload", "gell_mann", "gauge_field", "random_su3",
    "gaussian_spinors", "z2_spinors", "gaussian_coarse", "shifts_for", "c3_solve_counts",
    "volume", "site_index", "site_coords",
]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    dims: Tuple[int, int, int, int]          # (Lx, Ly, Lz, Lt)
    eps: float                               # gauge disorder
    kappa: float                             # hopping parameter, m0 = 1/(2 kappa) - 4
    n_rhs: int
    mus: Tuple[float, ...]                   # twisted-mass shifts
    rhs_kind: str                            # "gauss" | "z2"
    agg: Tuple[Tuple[int, int, int, int], ...]  # aggregate extents per level transition
    n_tv: Tuple[int, ...]                    # test vectors per level transition
    sap_block: Tuple[int, int, int, int]
    seed_gauge: int
    seed_rhs: int
    seed_tv: int

    @property
    def m0(self) -> float:
        return 1.0 / (2.0 * self.kappa) - 4.0

    @property
    def n_levels(self) -> int:
        return 1 + len(self.agg)

    @property
    def n_col(self) -> int:
        return self.n_rhs * len(self.mus)

    @property
    def volume(self) -> int:
        return volume(self.dims)


def _logspace(lo: float, hi: float, n: int) -> Tuple[float, ...]:
    if n == 1:
        return (lo,)
    return tuple(float(lo * (hi / lo) ** (j / (n - 1))) for j in range(n))


WORKLOADS = {
    # plain FP64 method, two-level, runs in seconds on a CPU
    "tm_4x4x4x4_2rhs_3shift": Workload(
        name="tm_4x4x4x4_2rhs_3shift", dims=(4, 4, 4, 4), eps=0.3, kappa=0.14,
        n_rhs=2, mus=(0.01, 0.05, 0.1), rhs_kind="gauss",
        agg=((2, 2, 2, 2),), n_tv=(8,), sap_block=(2, 2, 2, 2),
        seed_gauge=101, seed_rhs=201, seed_tv=301),
    # precision study: 16^3x32, 12 Z2 rhs x 4 shifts, three levels
    "tm_16x16x16x32_12rhs_4shift": Workload(
        name="tm_16x16x16x32_12rhs_4shift", dims=(16, 16, 16, 32), eps=0.3, kappa=0.150,
        n_rhs=12, mus=(0.002, 0.01, 0.03, 0.1), rhs_kind="z2",
        agg=((4, 4, 4, 4), (2, 2, 2, 2)), n_tv=(24, 32), sap_block=(4, 4, 4, 4),
        seed_gauge=102, seed_rhs=202, seed_tv=302),
    # batching study: one 32^3x64 field, uneven solves (counts drawn separately)
    "tm_32x32x32x64_batched": Workload(
        name="tm_32x32x32x64_batched", dims=(32, 32, 32, 64), eps=0.3, kappa=0.150,
        n_rhs=1, mus=(1e-3,), rhs_kind="gauss",
        agg=((4, 4, 4, 4), (2, 2, 2, 2)), n_tv=(24, 32), sap_block=(4, 4, 4, 4),
        seed_gauge=103, seed_rhs=203, seed_tv=303),
    # large volume: one GPU's share of an 80^3x160 run
    "tm_40x40x40x80_4rhs_8shift": Workload(
        name="tm_40x40x40x80_4rhs_8shift", dims=(40, 40, 40, 80), eps=0.35, kappa=0.152,
        n_rhs=4, mus=_logspace(7e-4, 0.5, 8), rhs_kind="gauss",
        agg=((4, 4, 4, 4), (2, 2, 2, 2)), n_tv=(24, 32), sap_block=(4, 4, 4, 4),
        seed_gauge=105, seed_rhs=205, seed_tv=305),
    # small three-level case used by tests (8^4, cheap on CPU)
    "tm_8x8x8x8_3level": Workload(
        name="tm_8x8x8x8_3level", dims=(8, 8, 8, 8), eps=0.3, kappa=0.150,
        n_rhs=2, mus=(0.002, 0.05), rhs_kind="z2",
        agg=((2, 2, 2, 2), (2, 2, 2, 2)), n_tv=(8, 12), sap_block=(2, 2, 2, 2),
        seed_gauge=107, seed_rhs=207, seed_tv=307),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def shifts_for(w: Workload) -> np.ndarray:
    return np.asarray(w.mus, dtype=np.float64)


def c3_solve_counts(n_solves: int = 24, seed: int = 403):
    """Uneven batch of independent solves: column counts c_i ~ U{1..16};
    n_shift drawn uniformly from the divisors of c_i, n_rhs = c_i / n_shift;
    the shifts of a solve are log-spaced in [1e-3, 1] (1e-3 when n_shift = 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n_solves):
        c = int(rng.integers(1, 17))
        divs = [d for d in range(1, c + 1) if c % d == 0]
        ns = int(divs[int(rng.integers(0, len(divs)))])
        mus = _logspace(1e-3, 1.0, ns)
        out.append((c // ns, np.asarray(mus)))
    return out


# ---------------------------------------------------------------------------
# lattice indexing
# ---------------------------------------------------------------------------
def volume(dims: Sequence[int]) -> int:
    return int(np.prod(dims))


def site_index(x, y, z, t, dims):
    Lx, Ly, Lz, Lt = dims
    return x + Lx * (y + Ly * (z + Lz * t))


def site_coords(i, dims):
    Lx, Ly, Lz, Lt = dims
    x = i % Lx
    y = (i // Lx) % Ly
    z = (i // (Lx * Ly)) % Lz
    t = i // (Lx * Ly * Lz)
    return x, y, z, t


# ---------------------------------------------------------------------------
# gauge links
# ---------------------------------------------------------------------------
def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j; l[1][1, 0] = 1j
    l[2][0, 0] = 1; l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j; l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j; l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / math.sqrt(3); l[7][2, 2] = -2 / math.sqrt(3)
    return l


def _reunitarise(U: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 1 and 2, row 3 = conj(row1 x row2): det = 1."""
    r1 = U[..., 0, :]
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = U[..., 1, :]
    r2 = r2 - np.sum(np.conj(r1) * r2, axis=-1, keepdims=True) * r1
    r2 = r2 / np.linalg.norm(r2, axis=-1, keepdims=True)
    r3 = np.conj(np.cross(r1, r2))
    return np.stack([r1, r2, r3], axis=-2)


def _exp_i_eps_h(h: np.ndarray, eps: float) -> np.ndarray:
    """exp(i eps H) for H = sum_a h_a lambda_a / 2, batched over leading dims."""
    H = np.einsum("...a,aij->...ij", h, gell_mann()) * 0.5
    w, Q = np.linalg.eigh(H)
    return np.einsum("...ij,...j,...kj->...ik", Q, np.exp(1j * eps * w), np.conj(Q))


def gauge_field(dims: Sequence[int], eps: float, seed: int, chunk: int = 1 << 18) -> np.ndarray:
    """Seeded SU(3) links, complex128 [V][4][3][3]."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    for s0 in range(0, V, chunk):
        s1 = min(V, s0 + chunk)
        h = rng.standard_normal((s1 - s0, 4, 8))
        U[s0:s1] = _reunitarise(_exp_i_eps_h(h, eps))
    return U


def random_su3(n: int, seed: int) -> np.ndarray:
    """n Haar-ish random SU(3) matrices (QR of a complex Gaussian, det fixed to 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, 3, 3)) + 1j * rng.standard_normal((n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return _reunitarise(q)


# ---------------------------------------------------------------------------
# vectors
# ---------------------------------------------------------------------------
def gaussian_spinors(n: int, V: int, seed: int) -> np.ndarray:
    """complex128 [n][V][4][3], real and imaginary parts i.i.d. N(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((n, V, 4, 3))
    im = rng.standard_normal((n, V, 4, 3))
    return re + 1j * im


def z2_spinors(n: int, V: int, seed: int) -> np.ndarray:
    """complex128 [n][V][4][3], entries (+-1 +-i)/sqrt(2) with independent signs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = rng.integers(0, 2, size=(2, n, V, 4, 3)) * 2 - 1
    return (s[0] + 1j * s[1]) / math.sqrt(2.0)


def gaussian_coarse(n: int, Vc: int, dof: int, seed: int) -> np.ndarray:
    """complex128 [n][Vc][dof]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal((n, Vc, dof)) + 1j * rng.standard_normal((n, Vc, dof))


def rhs_for(w: Workload, V: Optional[int] = None) -> np.ndarray:
    V = w.volume if V is None else V
    if w.rhs_kind == "z2":
        return z2_spinors(w.n_rhs, V, w.seed_rhs)
    return gaussian_spinors(w.n_rhs, V, w.seed_rhs)


def setup_start_vectors(w: Workload):
    """Random starting vectors of the adaptive setup, one array per level
    transition: level 0 -> [N0][V][4][3]; level l>0 -> [N_l][Vc_l][2 N_{l-1}]."""
    out = []
    dims = list(w.dims)
    for l, (agg, n) in enumerate(zip(w.agg, w.n_tv)):
        V = volume(dims)
        if l == 0:
            out.append(gaussian_spinors(n, V, w.seed_tv + 1000 * l))
        else:
            out.append(gaussian_coarse(n, V, 2 * w.n_tv[l - 1], w.seed_tv + 1000 * l))
        dims = [d // a for d, a in zip(dims, agg)]
    return out
