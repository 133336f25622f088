"""Pins of the oracle's second derivatives and fourth-order operator (Sec. 2.1 derivative formula
applied twice; eq:ddrational; App. A eq:identity, eq:ddimap, eq:ddspatial):

* 1D: second derivatives sum to zero; quadratic and linear reproduction through the polar-form
  (Marsden) coefficients give exactly 2 and 0;
* mapped NURBS (quarter annulus, quarter cylinder): the isoparametric map reproduces linear
  functions of x, so sum_A x_{A,k} N_{A,ij} = 0 and sum_A x_{A,k} N_{A,i} = delta_ki; partition
  of unity gives sum_A N_{A,ij} = 0 (a sign slip in eq:ddimap breaks the first on a curved map);
* the spatial Hessian against central differences of the spatial gradient along the parameters,
  mapped and (for eq:ddrational alone) with x = xi and rational weights;
* the operator sum W Lap N_A Lap u_h: zero for u linear in x on curved maps; 8 int N_A for
  u = x^2 y^2 on the unit square and every function whose value and normal derivative vanish on
  the boundary (Green's second identity, with Lap^2 u = 8); symmetric; rows sum to zero."""
import itertools

import numpy as np
import pytest

import inputs
import oracle



def polar_quadratic(U, p):
    """Coefficients of xi^2 in the B-spline basis: the polar form 2/(p(p-1)) sum_{j<k} t_j t_k
    over the knots t_{i+1..i+p} of each function."""
    n = len(U) - p - 1
    c = np.zeros(n)
    for i in range(n):
        t = U[i + 1:i + p + 1]
        c[i] = sum(t[j] * t[k] for j in range(p) for k in range(j + 1, p)) * 2.0 / (p * (p - 1))
    return c


def basis_all(U, p, xi):
    n = len(U) - p - 1
    L = oracle.lib()
    v, d, d2 = np.zeros(n), np.zeros(n), np.zeros(n)
    Uc = np.ascontiguousarray(U, dtype=np.float64)
    for i in range(n):
        a, b, c = (oracle.C.c_double() for _ in range(3))
        assert L.orc_basis_1d(p, oracle._ptr(Uc), len(Uc), i, xi, oracle.C.byref(a), oracle.C.byref(b)) == 0
        assert L.orc_basis_1d_d2(p, oracle._ptr(Uc), len(Uc), i, xi, oracle.C.byref(c)) == 0
        v[i], d[i], d2[i] = a.value, b.value, c.value
    return v, d, d2


@pytest.mark.parametrize("p", [2, 3, 4, 5])
def test_1d_second_derivatives_reproduce_quadratics(p):
    rng = np.random.default_rng(p)
    inner = np.sort(rng.uniform(0.1, 0.9, 6))
    inner = np.concatenate([inner, inner[:2]]) if p >= 3 else inner      # double knots (C^{p-2}) for p >= 3
    U = np.concatenate([[0.0] * (p + 1), np.sort(inner), [1.0] * (p + 1)])
    c2 = polar_quadratic(U, p)
    c1 = inputs.greville(U, p)
    for xi in rng.uniform(0.0, 1.0, 25):
        v, d, d2 = basis_all(U, p, xi)
        assert abs(v @ c2 - xi * xi) < 1e-13
        assert abs(d2.sum()) < 1e-9 * np.abs(d2).sum()
        assert abs(d2 @ c2 - 2.0) < 1e-9 * max(1.0, np.abs(d2 * c2).sum())
        assert abs(d2 @ c1) < 1e-9 * max(1.0, np.abs(d2 * c1).sum())


def curved(dim, p):
    patch = inputs.quarter_cylinder([3, 4, 2][:dim], p, dim=dim)
    o = oracle.Oracle(patch.knots, patch.degree, ctrl=patch.ctrl, weights=patch.weights)
    return patch, o


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_spatial_hessian_reproduces_linear_functions_on_curved_maps(dim, p):
    patch, o = curved(dim, p)
    rng = np.random.default_rng(10 * dim + p)
    nelem = int(np.prod([len(k) - 2 * p - 1 for k in patch.knots]))
    for e in rng.integers(0, nelem, 6):
        t = rng.uniform(-1, 1, dim)
        A, N, dN, d2N, x = o.basis_hessian(int(e), t)
        X = patch.ctrl[A]                                        # [nloc, dim]
        scale = np.abs(d2N[:, :dim, :dim]).sum(axis=0).max()
        assert np.allclose(N @ X, x[:dim], atol=1e-13)
        assert np.allclose(dN[:, :dim].T @ X, np.eye(dim), atol=1e-12)
        lin = np.einsum("aij,ak->kij", d2N[:, :dim, :dim], X)
        assert np.abs(lin).max() < 1e-12 * scale, np.abs(lin).max()
        assert np.abs(d2N.sum(axis=0)).max() < 1e-12 * scale


@pytest.mark.parametrize("dim,p,mapped", [(2, 2, True), (3, 3, True), (2, 3, False), (3, 2, False)])
def test_spatial_hessian_matches_differences_of_the_gradient(dim, p, mapped):
    """Mapped: the full chain (eq:ddrational, eq:ddimap, eq:ddspatial).  Unmapped (x = xi with
    the cylinder's weights): the spatial Hessian is the parametric one of eq:ddrational itself,
    which a mapped case cannot see (an error in it that is consistent with the weights cancels
    through x_{,alpha beta} in eq:ddimap)."""
    patch, o = curved(dim, p)
    if not mapped:
        o = oracle.Oracle(patch.knots, patch.degree, weights=patch.weights)
    h = 1e-5
    for e, t in [(1, np.array([0.2, -0.4, 0.1])[:dim]), (5, np.array([-0.7, 0.3, 0.6])[:dim])]:
        A, N, dN, d2N, x = o.basis_hessian(e, t)
        for b in range(dim):
            tp, tm = t.copy(), t.copy()
            tp[b] += h
            tm[b] -= h
            _, _, dNp, _, xp = o.basis_hessian(e, tp)
            _, _, dNm, _, xm = o.basis_hessian(e, tm)
            dgrad = (dNp - dNm)[:, :dim] / (2 * h)               # d N_{A,i} / d t_b
            dx = (xp - xm)[:dim] / (2 * h)                       # d x_j / d t_b
            pred = np.einsum("aij,j->ai", d2N[:, :dim, :dim], dx)
            assert np.abs(pred - dgrad).max() < 1e-6 * np.abs(dgrad).max()


def test_biharmonic_residual_closed_form_on_the_unit_square():
    for p in (2, 3):
        patch = inputs.unit_box(2, [6, 7], p)
        o = oracle.Oracle(patch.knots, patch.degree)
        c2 = [polar_quadratic(U, p) for U in patch.knots]
        U = np.outer(c2[1], c2[0]).ravel()                      # x^2 y^2, natural order (axis 0 fastest)
        R = o.biharmonic_residual(U)
        n0, n1 = len(c2[0]), len(c2[1])
        ints = [np.array([(K[i + p + 1] - K[i]) / (p + 1) for i in range(len(K) - p - 1)]) for K in patch.knots]
        for i1, i0 in itertools.product(range(2, n1 - 2), range(2, n0 - 2)):
            exact = 8.0 * ints[0][i0] * ints[1][i1]
            assert abs(R[i0 + n0 * i1] - exact) < 1e-12 * max(1.0, abs(exact)), (p, i0, i1)


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_biharmonic_residual_invariants_on_curved_maps(dim, p):
    patch, o = curved(dim, p)
    rng = np.random.default_rng(dim + 7 * p)
    a = rng.normal(size=dim)
    ulin = patch.ctrl @ a + 0.3
    Rlin = o.biharmonic_residual(ulin)
    Ur, Vr = rng.normal(size=o.N), rng.normal(size=o.N)
    Rr, Rv = o.biharmonic_residual(Ur), o.biharmonic_residual(Vr)
    scale = np.abs(Rr).max()
    assert np.abs(Rlin).max() < 1e-11 * scale                   # Lap of a linear function of x is 0
    assert abs(Rr.sum()) < 1e-11 * np.abs(Rr).sum()            # sum_A Lap N_A = 0
    assert abs(Vr @ Rr - Ur @ Rv) < 1e-11 * abs(Ur @ Rr)      # symmetric
    assert Ur @ Rr > 0                                         # integral of (Lap u_h)^2
