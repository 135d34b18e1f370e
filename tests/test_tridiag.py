"""The host step of the natural-frequency solver: smallest eigenvalues of a symmetric
tridiagonal matrix by Sturm bisection, and the last entries of their eigenvectors (the
Lanczos residual estimate), against closed forms and LAPACK."""
import math

import numpy as np
import pytest

from paper_2207_09334_amd import cronos as CR


@pytest.mark.parametrize("k", [1, 2, 7, 200, 5000])
def test_discrete_laplacian_closed_form(k):
    """tridiag(-1, 2, -1) of order k: eigenvalues 2 - 2 cos(j pi / (k + 1)), eigenvectors
    sqrt(2 / (k + 1)) sin(i j pi / (k + 1))."""
    count = min(k, 6)
    theta, last = CR.cronos_tridiag_smallest(np.full(k, 2.0), np.full(k - 1, -1.0), count)
    j = np.arange(1, count + 1)
    assert theta == pytest.approx(2.0 - 2.0 * np.cos(j * math.pi / (k + 1)), rel=1e-9, abs=1e-14)
    want = np.abs(math.sqrt(2.0 / (k + 1)) * np.sin(k * j * math.pi / (k + 1)))
    assert last == pytest.approx(want, rel=1e-6, abs=1e-12)


def test_random_matrices_against_lapack():
    rng = np.random.default_rng(3)
    for k in (3, 40, 400):
        a = rng.normal(size=k) * 10.0
        b = rng.normal(size=k - 1)
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        w, v = np.linalg.eigh(T)
        count = min(k, 8)
        theta, last = CR.cronos_tridiag_smallest(a, b, count)
        assert theta == pytest.approx(w[:count], abs=1e-12 * np.abs(w).max())
        gaps = np.minimum(np.diff(np.r_[-np.inf, w]), np.diff(np.r_[w, np.inf]))[:count]
        ok = gaps > 1e-3
        assert last[ok] == pytest.approx(np.abs(v[-1, :count])[ok], rel=1e-6, abs=1e-10)


def test_stiff_spectrum_resolves_the_small_end():
    """A graded spectrum like the Lanczos matrices of a stiff lattice (1 to 1e9): the small
    eigenvalues come out to about 1e-16 of the largest."""
    rng = np.random.default_rng(5)
    lam = np.sort(np.r_[1.0, 1.7, 40.0, np.exp(rng.uniform(math.log(50.0), math.log(1e9), 120))])
    # orthogonal similarity to tridiagonal form with a Householder-free route: Lanczos in
    # exact-enough arithmetic on the diagonal matrix, full reorthogonalisation
    n = len(lam)
    q = rng.normal(size=n)
    q /= np.linalg.norm(q)
    Q = [q]
    a, b = [], []
    for i in range(n):
        w = lam * Q[-1]
        a.append(Q[-1] @ w)
        w -= a[-1] * Q[-1] + (b[-1] * Q[-2] if b else 0.0)
        for p in Q:
            w -= (p @ w) * p
        if i + 1 < n:
            b.append(np.linalg.norm(w))
            Q.append(w / b[-1])
    theta, _ = CR.cronos_tridiag_smallest(np.array(a), np.array(b), 3)
    assert theta == pytest.approx(lam[:3], abs=5e-16 * 1e9 * 8)


def test_bad_arguments():
    with pytest.raises(CR.CronosError):
        CR.cronos_tridiag_smallest(np.ones(3), np.ones(2), 4)
    with pytest.raises(CR.CronosError):
        CR.cronos_tridiag_smallest(np.array([1.0, np.nan]), np.ones(1), 1)
