"""Pins of the oracle's periodic axes (Sec. 2.4: unclamping by eq:unclamp-left/right, index
wrapping by eq:map-wrap), against the paper's printed knot vectors and against properties that a
wrong unclamping or wrap would break."""
import os

import numpy as np
import pytest

import inputs
import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden", "unclamp_fig1.txt")


def test_unclamp_matches_the_papers_figure():
    rows = np.loadtxt(GOLD)
    open_kv = [0, 0, 0, 0, 0.2, 0.4, 0.6, 0.8, 1, 1, 1, 1]
    for r in rows:
        k = int(r[0])
        assert np.allclose(oracle.unclamp(open_kv, 3, k), r[1:], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p,k", [(1, 0), (2, 0), (2, 1), (3, 0), (3, 1), (3, 2)])
def test_periodic_function_is_ck_across_the_seam(p, k):
    """u = sum_i U_{mod(i, n-k)} B_i on the unclamped knots has equal value (and, k >= 1, slope)
    at both ends of the domain."""
    U0 = inputs.open_uniform_knots(7, p)
    U = oracle.unclamp(U0, p, k)
    n = len(U) - p - 1          # functions of the open vector (the paper's n is n - 1)
    nper = n - 1 - k
    c = inputs.uniform(3, 4, nper, -1.0, 1.0)

    def ev(xi):
        v = d = 0.0
        for i in range(n):
            b, db = oracle.basis_1d(p, U, i, xi)
            v += c[i % nper] * b
            d += c[i % nper] * db
        return v, d
    v0, d0 = ev(U0[p])
    v1, d1 = ev(U0[-p - 1] - 1e-15)
    assert abs(v0 - v1) < 1e-12
    if k >= 1:
        assert abs(d0 - d1) < 1e-10 * max(1.0, abs(d0))
    # an open (clamped) axis would not be continuous across the seam for random coefficients
    assert abs(v0 - v1) < 1e-3 * np.max(np.abs(c))


@pytest.mark.parametrize("dim,p,k", [(2, 2, 1), (2, 3, 0), (2, 3, 2), (3, 2, 1), (3, 2, 0)])
def test_fully_periodic_stiffness_has_zero_row_sums(dim, p, k):
    patch = inputs.unit_box(dim, [9, 8, 6][:dim], p)
    o = oracle.Oracle(patch.knots, patch.degree, lam=0.0, periodic=[k] * dim)
    nper = [len(U) - p - 2 - k for U in patch.knots]
    assert o.N == int(np.prod(nper))
    J = o.jacobian_csr(inputs.uniform(5, 1, o.N, 0.0, 0.3))
    assert np.max(np.abs(J @ np.ones(o.N))) < 1e-12 * abs(J).max()
    assert abs(J - J.T).max() < 1e-14 * abs(J).max()
    # at most 2p+1 distinct wrapped columns per periodic axis; exactly that everywhere when the
    # seam has the interior continuity (a C^k seam with k < p-1 is a repeated knot)
    rp, _ = o.pattern()
    lens = set(int(x) for x in np.diff(rp))
    assert max(lens) == (2 * p + 1) ** dim
    if k == p - 1:
        assert lens == {(2 * p + 1) ** dim}


@pytest.mark.parametrize("p", [2, 3])
def test_translation_invariance_with_maximal_seam_continuity(p):
    """Uniform knots and C^(p-1) across the seam: every periodic function is a translate of one
    another, so shifting the coefficients along the periodic axis shifts the residual."""
    patch = inputs.unit_box(2, [9, 5], p)
    o = oracle.Oracle(patch.knots, patch.degree, lam=3.0, periodic=[p - 1, None])
    n0 = len(patch.knots[0]) - p - 2 - (p - 1)
    n1 = len(patch.knots[1]) - p - 1
    U = inputs.uniform(6, 2, o.N, 0.0, 0.4).reshape(n1, n0)
    U[0, :] = U[-1, :] = 0.0
    R = o.residual(U.reshape(-1)).reshape(n1, n0)
    Rs = o.residual(np.roll(U, 1, axis=1).reshape(-1)).reshape(n1, n0)
    assert np.max(np.abs(Rs - np.roll(R, 1, axis=1))) < 1e-13 * np.max(np.abs(R))


def test_periodic_bratu_reduces_to_the_1d_problem():
    """With u = 0 at y = 0, 1 and periodicity in x, the problem is x-invariant; since the periodic
    functions sum to one, the 2D Newton solution is the 1D Bratu solution in y broadcast along x."""
    p, lam = 3, 2.5
    patch = inputs.unit_box(2, [6, 8], p)
    o2 = oracle.Oracle(patch.knots, patch.degree, lam=lam, periodic=[1, None])
    o1 = oracle.Oracle([patch.knots[1]], [p], lam=lam)
    U1, _, rc1 = o1.newton(np.zeros(o1.N), atol=1e-13)
    n0 = o2.N // o1.N
    U2, _, rc2 = o2.newton(inputs.uniform(7, 1, o2.N, 0.0, 0.05) * 0.0, atol=1e-13)
    assert rc1 == 0 and rc2 == 0
    U2 = U2.reshape(o1.N, n0)
    assert np.max(np.abs(U2 - U1[:, None])) < 1e-10 * np.max(np.abs(U1))
