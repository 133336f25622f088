"""Pins for the oracle's one-dimensional pieces: Gauss-Legendre rule, Cox-de Boor basis and
derivatives (Sec. 2.1), and the adjacency stencil of Algorithm 2 (Sec. 2.5)."""
import math

import numpy as np
import pytest

import inputs
import oracle


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8, 11])
def test_gauss_legendre_matches_library_and_is_exact(n):
    x, w = oracle.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xr, atol=1e-15, rtol=0)
    assert np.allclose(w, wr, atol=1e-15, rtol=0)
    # exact for monomials of degree <= 2n-1: int_{-1}^{1} t^k dt = 2/(k+1) for even k, 0 otherwise
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.dot(w, x ** k) - exact) < 1e-14
    # and not exact at degree 2n
    assert abs(np.dot(w, x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-8


def _random_knots(p, seed):
    u = inputs.uniform(seed, 0, 6)
    inner = np.sort(np.round(u * 8) / 8)                 # rounded -> some repeated knots
    inner = inner[(inner > 0) & (inner < 1)]
    # keep multiplicity <= p
    kv = [0.0] * (p + 1)
    for x in inner:
        if kv.count(x) < p:
            kv.append(x)
    kv += [1.0] * (p + 1)
    return np.array(kv)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_partition_of_unity_and_derivative_sum(p, seed):
    U = _random_knots(p, seed)
    n = len(U) - p - 1
    for xi in np.linspace(0, 1, 41):
        vals = [oracle.basis_1d(p, U, i, xi) for i in range(n)]
        B = np.array([v for v, _ in vals])
        D = np.array([d for _, d in vals])
        assert np.all(B >= -1e-15)
        assert abs(B.sum() - 1.0) < 1e-14
        assert abs(D.sum()) < 1e-10 * max(1.0, np.abs(D).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_bernstein_special_case(p):
    U = np.array([0.0] * (p + 1) + [1.0] * (p + 1))
    for t in np.linspace(0, 1, 17):
        for i in range(p + 1):
            v, d = oracle.basis_1d(p, U, i, t)
            b = math.comb(p, i) * t ** i * (1 - t) ** (p - i)
            db = math.comb(p, i) * ((i * t ** (i - 1) if i > 0 else 0.0) * (1 - t) ** (p - i)
                                    - (t ** i) * ((p - i) * (1 - t) ** (p - i - 1) if i < p else 0.0))
            assert abs(v - b) < 1e-14
            assert abs(d - db) < 1e-12


@pytest.mark.parametrize("p", [2, 3, 4])
def test_derivative_matches_central_difference(p):
    U = _random_knots(p, 7)
    n = len(U) - p - 1
    h = 1e-6
    for xi in np.linspace(0.013, 0.987, 23):
        if np.min(np.abs(U - xi)) < 3 * h:
            continue
        for i in range(n):
            _, d = oracle.basis_1d(p, U, i, xi)
            fp, _ = oracle.basis_1d(p, U, i, xi + h)
            fm, _ = oracle.basis_1d(p, U, i, xi - h)
            assert abs(d - (fp - fm) / (2 * h)) < 1e-7 * max(1.0, abs(d))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_integral_closed_form(p):
    # int B_{i,p} = (xi_{i+p+1} - xi_i) / (p+1), integrated span by span with numpy's rule
    U = _random_knots(p, 11)
    n = len(U) - p - 1
    t, w = np.polynomial.legendre.leggauss(p + 1)
    for i in range(n):
        tot = 0.0
        for s in range(len(U) - 1):
            a, b = U[s], U[s + 1]
            if b <= a:
                continue
            xs = 0.5 * (a + b) + 0.5 * (b - a) * t
            tot += 0.5 * (b - a) * sum(wk * oracle.basis_1d(p, U, i, xk)[0] for xk, wk in zip(xs, w))
        assert abs(tot - (U[i + p + 1] - U[i]) / (p + 1)) < 1e-15


def test_right_end_convention():
    # the last non-empty span is closed: B_{n-1,p}(1) = 1 for an open knot vector
    for p in (1, 2, 3):
        U = inputs.open_uniform_knots(4, p)
        n = len(U) - p - 1
        assert oracle.basis_1d(p, U, n - 1, 1.0)[0] == 1.0
        assert all(oracle.basis_1d(p, U, i, 1.0)[0] == 0.0 for i in range(n - 1))


def _support_overlap_bruteforce(U, p, i, j):
    """Open supports (xi_i, xi_{i+p+1}) and (xi_j, xi_{j+p+1}) intersect."""
    return max(U[i], U[j]) < min(U[i + p + 1], U[j + p + 1])


@pytest.mark.parametrize("U,p", [
    # knot vector of the cubic example whose continuity decreases element by element
    # (Sec. 2.5, caption of the adjacency figure)
    (np.array([0, 0, 0, 0, 2, 4, 4, 6, 6, 6, 8, 8, 8, 8], dtype=float), 3),
    (inputs.open_uniform_knots(6, 2), 2),
    (inputs.open_uniform_knots(5, 3, cont=1), 3),
    (inputs.open_uniform_knots(7, 4), 4),
])
def test_stencil_matches_support_overlap(U, p):
    n = len(U) - p - 1
    for i in range(n):
        l, r = oracle.stencil(p, U, i)
        js = [j for j in range(n) if _support_overlap_bruteforce(U, p, i, j)]
        assert (l, r) == (min(js), max(js)), (i, l, r, js)


def test_stencil_fig3_widths():
    # For the cubic example the stencil widths follow from the knot multiplicities:
    # the functions at the C^0 knot (6, multiplicity 3) couple only to their own side.
    U = np.array([0, 0, 0, 0, 2, 4, 4, 6, 6, 6, 8, 8, 8, 8], dtype=float)
    got = [oracle.stencil(3, U, i) for i in range(10)]
    assert got[0] == (0, 3)
    assert got[6] == (3, 9)     # the function interpolating at x=6 spans both sides
    assert got[9] == (6, 9)
