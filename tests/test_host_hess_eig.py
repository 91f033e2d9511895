"""Host logic: the small complex Hessenberg eigensolver that the GPU GMRES-DR
uses for its harmonic Ritz pairs (csrc/hess_eig.h), compiled with g++ into a
tiny driver and checked against numpy on Hessenberg matrices of the sizes the
solver meets (restart lengths up to 63), including the rank-one-updated form
H_m + |h|^2 f e_m^T of the harmonic Ritz problem; every check runs on a
plain build and on one under the host address and undefined-behaviour
sanitizers."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2201_03872_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "hess_eig.h"
int main() {
  int n;
  if (std::scanf("%d", &n) != 1) return 2;
  std::vector<ddamg::hcd> a((size_t)n * n), w, v;
  for (auto& x : a) { double re, im; std::scanf("%lf %lf", &re, &im); x = {re, im}; }
  if (!ddamg::hess_eig(n, a, w, v)) { std::printf("FAIL\n"); return 1; }
  for (auto& x : w) std::printf("%.17g %.17g\n", x.real(), x.imag());
  for (auto& x : v) std::printf("%.17g %.17g\n", x.real(), x.imag());
  return 0;
}
"""


# the same driver built plainly and with the host AddressSanitizer and
# UndefinedBehaviorSanitizer (any out-of-bounds access, use of freed memory or
# undefined arithmetic in the solver ends the run with an error)
BUILDS = {"plain": ["-O2"],
          "asan_ubsan": ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                         "-fno-sanitize-recover=all"]}


@pytest.fixture(scope="module", params=sorted(BUILDS))
def driver(request):
    d = tempfile.mkdtemp()
    src = os.path.join(d, "drv.cpp")
    exe = os.path.join(d, "drv")
    open(src, "w").write(DRIVER)
    r = subprocess.run(["g++", *BUILDS[request.param], "-std=c++17", "-I", CSRC, src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        if request.param == "plain":
            raise RuntimeError(r.stderr)
        pytest.skip("host sanitizer runtime not available: " + r.stderr[-200:])
    return exe


def run(exe, H):
    n = H.shape[0]
    inp = f"{n}\n" + "\n".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in H.reshape(-1))
    out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    vals = np.array([complex(*map(float, l.split())) for l in out[:n]])
    vecs = np.array([complex(*map(float, l.split())) for l in out[n:n + n * n]]).reshape(n, n)
    return vals, vecs


def _check(exe, H):
    w, V = run(exe, H)
    ref = np.linalg.eigvals(H)
    scale = np.max(np.abs(ref))
    for z in ref:            # multiset match
        assert np.min(np.abs(w - z)) < 1e-9 * scale
    for i in range(H.shape[0]):
        assert abs(np.linalg.norm(V[:, i]) - 1) < 1e-12
        assert np.linalg.norm(H @ V[:, i] - w[i] * V[:, i]) < 1e-8 * scale


@pytest.mark.parametrize("n", [1, 2, 5, 17, 40, 63])
def test_random_hessenberg(driver, n):
    rng = np.random.default_rng(n)
    H = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    _check(driver, H)


def test_harmonic_ritz_form_of_an_arnoldi_relation(driver):
    rng = np.random.default_rng(9)
    n, m = 200, 40
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 3 * np.eye(n)
    V = np.zeros((n, m + 1), dtype=complex)
    H = np.zeros((m + 1, m), dtype=complex)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    V[:, 0] = v / np.linalg.norm(v)
    for j in range(m):
        wv = A @ V[:, j]
        for i in range(j + 1):
            H[i, j] = np.vdot(V[:, i], wv)
            wv = wv - H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(wv)
        V[:, j + 1] = wv / H[j + 1, j]
    em = np.zeros(m)
    em[-1] = 1
    f = np.linalg.solve(H[:m, :m].conj().T, em)
    T = H[:m, :m] + abs(H[m, m - 1]) ** 2 * np.outer(f, em)
    assert np.allclose(np.tril(T, -2), 0)          # still upper Hessenberg
    _check(driver, T)
    # the k smallest in modulus agree with the oracle's harmonic Ritz values
    w, _ = run(driver, T)
    th, _ = O.harmonic_ritz(H, 8)
    assert np.max(np.abs(np.sort_complex(w[np.argsort(np.abs(w))][:8]) - np.sort_complex(th))) < 1e-9


@pytest.mark.parametrize("n", [3, 12, 30])
def test_general_matrix_with_a_full_leading_block(driver, n):
    """After a deflated restart H_m is Hessenberg except for a full leading
    block: the solver reduces any square matrix to Hessenberg form first."""
    rng = np.random.default_rng(100 + n)
    H = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), -1)
    k = n // 3 + 1
    H[:k + 1, :k] = rng.standard_normal((k + 1, k)) + 1j * rng.standard_normal((k + 1, k))
    _check(driver, H)
    _check(driver, rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))


def test_degenerate_and_diagonal(driver):
    _check(driver, np.diag([1.0, 1.0, 2.0, 2.0 + 1e-3j]).astype(complex))
    J = np.eye(6, k=1) * 0.5 + np.diag(np.full(6, 0.3 - 0.2j))     # defective Jordan-like block, values only
    w, _ = run(driver, J)
    assert np.max(np.abs(w - (0.3 - 0.2j))) < 1e-2
