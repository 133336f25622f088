"""Pins of the oracle's third derivatives (Sec. 2.1 derivative formula applied three times;
eq:dddrational; App. A eq:dddimap, eq:dddspatial) and of the operator built from them,
R_A = sum W grad N_A . grad(Lap u_h):

* 1D: third derivatives sum to zero; the polar-form (Marsden) coefficients of xi^3 give exactly 6,
  those of xi^2 and xi give 0;
* mapped NURBS (quarter annulus, quarter cylinder): sum_A x_{A,k} N_{A,ijk'} = 0 (the isoparametric
  map reproduces linear functions of x) and sum_A N_{A,ijk} = 0 (partition of unity); a sign slip in
  eq:dddimap or a dropped term of eq:dddspatial breaks the first on a curved map;
* symmetry of N_{A,ijk} in (i, j, k) (eq:dddspatial is written without that symmetry);
* the spatial third derivatives against central differences of the pinned spatial Hessian along the
  parameters, mapped (the whole chain) and with x = xi and rational weights (eq:dddrational alone);
* the operator: with every axis periodic and C^(p-1) continuity (p >= 3, so Lap u_h is continuous),
  integrating by parts once more gives sum W grad N_A . grad(Lap u_h) = - sum W Lap N_A Lap u_h
  exactly (the quadrature integrates both exactly on x = xi), i.e. minus the pinned fourth-order
  operator; on curved maps it vanishes for u linear in x and its rows sum to zero."""
import itertools

import numpy as np
import pytest

import inputs
import oracle


def polar(U, p, deg):
    """Coefficients of xi^deg in the B-spline basis: the polar form (elementary symmetric polynomial of
    degree deg of the knots t_{i+1..i+p}, divided by C(p, deg))."""
    from math import comb
    n = len(U) - p - 1
    c = np.zeros(n)
    for i in range(n):
        t = U[i + 1:i + p + 1]
        c[i] = sum(np.prod([t[j] for j in sub]) for sub in itertools.combinations(range(p), deg)) / comb(p, deg)
    return c


@pytest.mark.parametrize("p", [3, 4, 5, 6])
def test_1d_third_derivatives_reproduce_cubics(p):
    rng = np.random.default_rng(30 + p)
    inner = np.sort(rng.uniform(0.1, 0.9, 6))
    inner = np.concatenate([inner, inner[:2]]) if p >= 4 else inner      # double knots (C^{p-2}) for p >= 4
    U = np.concatenate([[0.0] * (p + 1), np.sort(inner), [1.0] * (p + 1)])
    n = len(U) - p - 1
    c3, c2, c1 = polar(U, p, 3), polar(U, p, 2), polar(U, p, 1)
    for xi in rng.uniform(0.0, 1.0, 25):
        v = np.array([oracle.basis_1d(p, U, i, xi)[0] for i in range(n)])
        d3 = np.array([oracle.basis_1d_d3(p, U, i, xi) for i in range(n)])
        assert abs(v @ c3 - xi ** 3) < 1e-13                         # the coefficients are right
        scale = np.abs(d3).sum()
        assert abs(d3.sum()) < 1e-9 * scale
        assert abs(d3 @ c3 - 6.0) < 1e-9 * max(1.0, np.abs(d3 * c3).sum())
        assert abs(d3 @ c2) < 1e-9 * max(1.0, np.abs(d3 * c2).sum())
        assert abs(d3 @ c1) < 1e-9 * max(1.0, np.abs(d3 * c1).sum())


def curved(dim, p):
    patch = inputs.quarter_cylinder([3, 4, 2][:dim], p, dim=dim)
    o = oracle.Oracle(patch.knots, patch.degree, ctrl=patch.ctrl, weights=patch.weights)
    return patch, o


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_third_derivatives_reproduce_linear_functions_on_curved_maps(dim, p):
    patch, o = curved(dim, p)
    rng = np.random.default_rng(40 + 10 * dim + p)
    nelem = int(np.prod([len(k) - 2 * p - 1 for k in patch.knots]))
    for e in rng.integers(0, nelem, 6):
        t = rng.uniform(-1, 1, dim)
        A, d3 = o.basis_third(int(e), t)
        d3 = d3[:, :dim, :dim, :dim]
        X = patch.ctrl[A]
        scale = np.abs(d3).sum(axis=0).max()
        lin = np.einsum("aijk,am->mijk", d3, X)
        assert np.abs(lin).max() < 1e-11 * scale, np.abs(lin).max()
        assert np.abs(d3.sum(axis=0)).max() < 1e-11 * scale
        for perm in itertools.permutations(range(3)):
            assert np.abs(d3 - d3.transpose((0,) + tuple(1 + q for q in perm))).max() < 1e-11 * scale


@pytest.mark.parametrize("dim,p,mapped", [(2, 2, True), (2, 3, True), (3, 3, True), (2, 3, False), (3, 2, False)])
def test_third_derivatives_match_differences_of_the_hessian(dim, p, mapped):
    """d/dt_b N_{A,ij}(x(t)) = N_{A,ijk} dx_k/dt_b, with both derivatives along t by central differences
    of the (pinned) spatial Hessian and of the map."""
    patch, o = curved(dim, p)
    if not mapped:
        o = oracle.Oracle(patch.knots, patch.degree, weights=patch.weights)
    h = 1e-5
    for e, t in [(1, np.array([0.2, -0.4, 0.1])[:dim]), (5, np.array([-0.7, 0.3, 0.6])[:dim])]:
        _, d3 = o.basis_third(e, t)
        for b in range(dim):
            tp, tm = t.copy(), t.copy()
            tp[b] += h
            tm[b] -= h
            _, _, _, Hp, xp = o.basis_hessian(e, tp)
            _, _, _, Hm, xm = o.basis_hessian(e, tm)
            dH = (Hp - Hm)[:, :dim, :dim] / (2 * h)
            dx = (xp - xm)[:dim] / (2 * h)
            pred = np.einsum("aijk,k->aij", d3[:, :dim, :dim, :dim], dx)
            assert np.abs(pred - dH).max() < 1e-5 * np.abs(dH).max(), (e, b, np.abs(pred - dH).max())


@pytest.mark.parametrize("dim,nel,p", [(2, [8, 7], 3), (2, [9, 10], 4), (3, [7, 7, 8], 3)])
def test_grad_laplacian_operator_equals_minus_fourth_order_operator_on_periodic_patches(dim, nel, p):
    patch = inputs.unit_box(dim, nel, p)
    per = [p - 1] * dim
    o = oracle.Oracle(patch.knots, patch.degree, periodic=per)
    U = inputs.uniform(51, 0, o.N, -1.0, 1.0)
    G = o.grad_laplacian_residual(U)
    B = o.biharmonic_residual(U)
    assert np.abs(G + B).max() < 1e-10 * np.abs(B).max()
    assert abs(G.sum()) < 1e-10 * np.abs(G).sum()               # sum_A grad N_A = 0


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_grad_laplacian_operator_on_curved_maps(dim, p):
    patch, o = curved(dim, p)
    rng = np.random.default_rng(60 + dim + 7 * p)
    ulin = patch.ctrl @ rng.normal(size=dim) + 0.3
    Ur = rng.normal(size=o.N)
    Gr = o.grad_laplacian_residual(Ur)
    assert np.abs(o.grad_laplacian_residual(ulin)).max() < 1e-10 * np.abs(Gr).max()   # Lap of linear = 0
    assert abs(Gr.sum()) < 1e-10 * np.abs(Gr).sum()
