"""The seeded input recipe (standing in for the paper's gauge ensembles and
sources) has the properties both implementations rely on:

* links are SU(3): unitary and of determinant 1, so the third row is
  conj(row 1 x row 2), which is what the 2-row link storage of the FP32
  stencil rebuilds; U = exp(i eps H) departs from 1 by O(eps), so the mean
  plaquette falls as eps grows;
* a seed gives the same field every time, and the generation in chunks does
  not change it;
* Z2 sources have entries (+-1 +- i)/sqrt 2; Gaussian ones unit variance per
  real component;
* the uneven batches: column counts in 1..16, shift counts dividing them,
  shifts log-spaced in [1e-3, 1] (1e-3 alone for one shift);
* the 40^3x80 shifts: 8 values log-spaced in [7e-4, 0.5].
"""
import numpy as np
import pytest

import synthetic as S


def _plaquette(U, dims):
    Lx, Ly, Lz, Lt = dims
    lat = U.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
    ax = {0: 3, 1: 2, 2: 1, 3: 0}
    tot, n = 0.0, 0
    for mu in range(4):
        for nu in range(mu + 1, 4):
            Umu, Unu = lat[..., mu, :, :], lat[..., nu, :, :]
            Unu_xmu = np.roll(Unu, -1, axis=ax[mu])
            Umu_xnu = np.roll(Umu, -1, axis=ax[nu])
            P = Umu @ Unu_xmu @ np.conj(np.swapaxes(Umu_xnu, -1, -2)) @ np.conj(np.swapaxes(Unu, -1, -2))
            tot += np.trace(P, axis1=-2, axis2=-1).real.sum() / 3
            n += P.shape[0] * P.shape[1] * P.shape[2] * P.shape[3]
    return tot / n


@pytest.mark.parametrize("eps", [0.3, 0.35])
def test_links_are_su3_with_the_two_row_form(eps):
    U = S.gauge_field((4, 4, 4, 4), eps, 101)
    M = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(M @ np.conj(np.swapaxes(M, -1, -2)) - eye)) < 1e-14
    assert np.max(np.abs(np.linalg.det(M) - 1)) < 1e-14
    third = np.conj(np.cross(M[:, 0], M[:, 1]))
    assert np.max(np.abs(M[:, 2] - third)) < 1e-14


def test_eps_sets_the_distance_from_the_free_field():
    dims = (4, 4, 4, 4)
    p = [_plaquette(S.gauge_field(dims, eps, 7), dims) for eps in (0.0, 0.1, 0.3, 0.35)]
    assert abs(p[0] - 1) < 1e-14
    assert p[0] > p[1] > p[2] > p[3] > 0
    # distance of the links from 1 grows linearly in eps at small eps
    d = [np.mean(np.abs(S.gauge_field(dims, eps, 7) - np.eye(3))) for eps in (0.01, 0.02)]
    assert abs(d[1] / d[0] - 2) < 0.01


def test_fields_are_reproducible_and_chunk_independent():
    a = S.gauge_field((4, 4, 4, 8), 0.3, 55)
    b = S.gauge_field((4, 4, 4, 8), 0.3, 55)
    c = S.gauge_field((4, 4, 4, 8), 0.3, 55, chunk=100)
    assert np.array_equal(a, b)
    assert np.array_equal(a, c)
    assert not np.array_equal(a, S.gauge_field((4, 4, 4, 8), 0.3, 56))


def test_sources():
    z = S.z2_spinors(3, 64, 1)
    assert np.allclose(np.abs(z.real), 1 / np.sqrt(2)) and np.allclose(np.abs(z.imag), 1 / np.sqrt(2))
    assert {1, -1} <= set(np.sign(z.real).ravel().astype(int).tolist())
    g = S.gaussian_spinors(4, 4096, 2)
    assert abs(g.real.var() - 1) < 0.02 and abs(g.imag.var() - 1) < 0.02 and abs(g.mean()) < 0.02
    assert np.array_equal(S.gaussian_spinors(1, 16, 9), S.gaussian_spinors(1, 16, 9))


def test_uneven_batches():
    counts = S.c3_solve_counts(24, 403)
    assert len(counts) == 24
    for n_rhs, mus in counts:
        c = n_rhs * len(mus)
        assert 1 <= c <= 16 and n_rhs >= 1
        if len(mus) == 1:
            assert mus[0] == 1e-3
        else:
            assert abs(mus[0] - 1e-3) < 1e-15 and abs(mus[-1] - 1.0) < 1e-12
            r = mus[1:] / mus[:-1]
            assert np.allclose(r, r[0])
    assert sum(n * len(m) for n, m in counts) == 211          # the 32^3x64 set of the full-size test
    again = S.c3_solve_counts(24, 403)
    assert all(a[0] == b[0] and np.array_equal(a[1], b[1]) for a, b in zip(counts, again))


def test_headline_shifts():
    w = S.workload("tm_40x40x40x80_4rhs_8shift")
    mus = np.array(w.mus)
    assert len(mus) == 8 and abs(mus[0] - 7e-4) < 1e-15 and abs(mus[-1] - 0.5) < 1e-12
    assert np.allclose(mus[1:] / mus[:-1], (0.5 / 7e-4) ** (1 / 7))
    assert w.dims == (40, 40, 40, 80) and w.n_rhs == 4 and abs(w.kappa - 0.152) < 1e-15 and abs(w.eps - 0.35) < 1e-15
