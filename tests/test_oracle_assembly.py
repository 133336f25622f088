"""Pins for the oracle's assembly (Algorithm 3 with eq:residual / eq:jacobian), geometry
(Sec. 2.3, App. A) and Newton solver against values fixed by the paper and by mathematics."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import inputs
import oracle
from conftest import golden


def _greville_nd(patch):
    g = [inputs.greville(U, p) for U, p in zip(patch.knots, patch.degree)]
    grids = np.meshgrid(*g[::-1], indexing="ij")
    return [grids[patch.dim - 1 - d].reshape(-1) for d in range(patch.dim)]


def _int_b(U, p):
    n = len(U) - p - 1
    return np.array([(U[i + p + 1] - U[i]) / (p + 1) for i in range(n)])


# ------------------------------------------------------------------------------------------
# R(0) closed form and the paper's printed initial residual
# ------------------------------------------------------------------------------------------

def test_paper_initial_residual_pin():
    """2D Bratu tutorial, 128^2 quadratic C^1, lambda = 6.80, U = 0: the printed first SNES
    function norm (App. B) must be reproduced to all printed digits."""
    hist = np.loadtxt(golden("bratu2d_tutorial_history.txt"))
    patch = inputs.unit_box(2, 128, 2)
    o = oracle.Oracle(patch.knots, patch.degree, lam=6.80)
    r = np.linalg.norm(o.residual(np.zeros(o.N)))
    assert abs(r - hist[0, 1]) < 0.6e-14
    # and the closed form lambda * sum_{interior i} (int B_i)^2 (2D)
    ib = _int_b(patch.knots[0], 2)[1:-1]
    assert abs(r - 6.80 * np.sum(ib ** 2)) < 1e-16


@pytest.mark.parametrize("dim,nel,p,lam", [(2, 16, 2, 6.0), (2, 9, 3, 2.5), (3, 5, 2, 5.0), (3, 4, 3, 1.5)])
def test_residual_at_zero_closed_form(dim, nel, p, lam):
    patch = inputs.unit_box(dim, nel, p)
    o = oracle.Oracle(patch.knots, patch.degree, lam=lam)
    R = o.residual(np.zeros(o.N))
    ib = _int_b(patch.knots[0], p)
    full = ib
    for _ in range(dim - 1):
        full = np.multiply.outer(ib, full).reshape(-1) if False else np.kron(ib, full)
    expect = -lam * full
    expect[inputs.boundary_mask(patch.shape)] = 0.0
    assert np.allclose(R, expect, atol=1e-16, rtol=1e-13)


# ------------------------------------------------------------------------------------------
# Geometry: volumes, exact circle, NURBS with equal weights
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("dim,nel,p,vol", [
    (2, 4, 2, 1.0), (3, 3, 3, 1.0),
    (2, 16, 2, 3 * math.pi / 4), (2, 16, 3, 3 * math.pi / 4), (3, 16, 2, 3 * math.pi / 4),
])
def test_volume(dim, nel, p, vol):
    if vol == 1.0:
        patch = inputs.unit_box(dim, nel, p)
    else:
        patch = inputs.quarter_cylinder(nel, p, dim=dim)
    # the rational map makes det J a rational function: over-integrate so the quadrature
    # error of the NURBS cases sits below rounding
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, nquad=[p + 4] * dim)
    _, W, _, _ = o.qp_data()
    assert abs(W.sum() - vol) < 1e-13


def test_quarter_annulus_points_on_circles():
    """Radial coordinate of the exact NURBS annulus is 1 + xi_0 at every quadrature point."""
    patch = inputs.quarter_cylinder(6, 3, dim=2)
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights)
    x, _, _, _ = o.qp_data()
    t, _ = np.polynomial.legendre.leggauss(4)
    # quadrature points in oracle order: element-major (axis 0 fastest), then qp (axis 0 fastest)
    U0 = np.unique(patch.knots[0])
    xi0 = []
    for e1 in range(6):
        for e0 in range(6):
            a, b = U0[e0], U0[e0 + 1]
            for g1 in range(4):
                for g0 in range(4):
                    xi0.append(0.5 * (a + b) + 0.5 * (b - a) * t[g0])
    r = np.hypot(x[:, 0], x[:, 1])
    assert np.allclose(r, 1.0 + np.array(xi0), atol=2e-15, rtol=0)


def test_equal_weights_reduce_to_bsplines():
    patch = inputs.unit_box(2, 5, 3)
    U = inputs.uniform(9, 0, patch.ndof, -0.2, 0.4)
    o1 = oracle.Oracle(patch.knots, patch.degree, lam=2.0)
    o2 = oracle.Oracle(patch.knots, patch.degree, weights=np.full(patch.ndof, 2.5), lam=2.0)
    assert np.allclose(o1.residual(U), o2.residual(U), atol=1e-15, rtol=1e-13)
    assert np.allclose(o1.jacobian(U), o2.jacobian(U), atol=1e-15, rtol=1e-13)


# ------------------------------------------------------------------------------------------
# Stiffness and mass invariants
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("geom", ["box2", "box3", "ann2", "cyl3"])
def test_laplacian_rows_sum_to_zero_and_symmetric(geom):
    if geom.startswith("box"):
        patch = inputs.unit_box(int(geom[-1]), 4, 2)
    else:
        patch = inputs.quarter_cylinder(3, 3 if geom == "ann2" else 2, dim=int(geom[-1]))
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=0.0, dirichlet_mask=0)
    K = o.jacobian_csr(np.zeros(patch.ndof))
    assert np.abs(K.sum(axis=1)).max() < 1e-13 * abs(K).max()
    assert abs(K - K.T).max() < 1e-14 * abs(K).max()
    # positive semi-definite with a one-dimensional kernel (constants)
    ev = np.linalg.eigvalsh(K.toarray())
    assert ev[0] > -1e-12 and ev[1] > 1e-6


@pytest.mark.parametrize("geom,vol", [("box2", 1.0), ("box3", 1.0), ("ann2", 3 * math.pi / 4),
                                      ("cyl3", 3 * math.pi / 4)])
def test_mass_total_through_jacobian(geom, vol):
    """J(U=0) with kappa = 0 is -lambda times the mass matrix, whose entries sum to vol(Omega)."""
    if geom.startswith("box"):
        patch = inputs.unit_box(int(geom[-1]), 6, 2)
    else:
        patch = inputs.quarter_cylinder(16 if geom == "ann2" else 6, 2, dim=int(geom[-1]))
    E = int(np.prod([len(np.unique(U)) - 1 for U in patch.knots]))
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=1.7, kappa_mode=2,
                      kappa=np.zeros(E), dirichlet_mask=0, nquad=[6] * patch.dim)
    v = o.jacobian(np.zeros(patch.ndof))
    assert abs(v.sum() + 1.7 * vol) < 1e-12


# ------------------------------------------------------------------------------------------
# Brute force: exact rational integration of piecewise polynomials on tiny meshes
# ------------------------------------------------------------------------------------------

def _poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _poly_add(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def _poly_der(a):
    return [i * a[i] for i in range(1, len(a))] or [Fraction(0)]


def _poly_int(a, lo, hi):
    return sum(c * (hi ** (i + 1) - lo ** (i + 1)) / (i + 1) for i, c in enumerate(a))


def _bspline_polys(U, p):
    """Exact polynomial pieces of every B_{i,p} on every span (Fraction coefficients)."""
    U = [Fraction(u) for u in U]
    nk = len(U)
    spans = [s for s in range(nk - 1) if U[s] < U[s + 1]]
    # B[i][s] = coefficient list on span s
    B = {(i, s): ([Fraction(1)] if i == s else [Fraction(0)]) for i in range(nk - 1) for s in spans}
    for q in range(1, p + 1):
        NB = {}
        for i in range(nk - 1 - q):
            for s in spans:
                acc = [Fraction(0)]
                a = U[i + q] - U[i]
                if a != 0:
                    acc = _poly_add(acc, _poly_mul([-U[i] / a, 1 / a], B[(i, s)]))
                b = U[i + q + 1] - U[i + 1]
                if b != 0:
                    acc = _poly_add(acc, _poly_mul([U[i + q + 1] / b, -1 / b], B[(i + 1, s)]))
                NB[(i, s)] = acc
        B = NB
    return B, spans, U


def _exact_1d(U, p):
    B, spans, Uf = _bspline_polys(U, p)
    n = len(U) - p - 1
    M = [[Fraction(0)] * n for _ in range(n)]
    A = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            for s in spans:
                lo, hi = Uf[s], Uf[s + 1]
                M[i][j] += _poly_int(_poly_mul(B[(i, s)], B[(j, s)]), lo, hi)
                A[i][j] += _poly_int(_poly_mul(_poly_der(B[(i, s)]), _poly_der(B[(j, s)])), lo, hi)
    return np.array(M, dtype=float), np.array(A, dtype=float)


@pytest.mark.parametrize("nel,p,cont", [(1, 2, None), (2, 2, None), (2, 3, None), (3, 2, 0), (2, 4, 2)])
def test_bruteforce_exact_stiffness_and_mass_2d(nel, p, cont):
    U = inputs.open_uniform_knots(nel, p, cont)
    M1, A1 = _exact_1d(U, p)
    K_exact = np.kron(M1, A1) + np.kron(A1, M1)    # axis 0 fastest: index i0 + n0*i1
    M_exact = np.kron(M1, M1)
    o = oracle.Oracle([U, U], [p, p], lam=0.0, dirichlet_mask=0)
    K = o.jacobian_csr(np.zeros(o.N)).toarray()
    assert np.abs(K - K_exact).max() < 2e-15 * max(1, np.abs(K_exact).max())
    E = nel * nel
    om = oracle.Oracle([U, U], [p, p], lam=-1.0, kappa_mode=2, kappa=np.zeros(E), dirichlet_mask=0)
    Mo = om.jacobian_csr(np.zeros(o.N)).toarray()
    assert np.abs(Mo - M_exact).max() < 1e-16


# ------------------------------------------------------------------------------------------
# Jacobian against finite differences of the residual; patch test
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("case", ["box2", "ann2_nodal", "cyl3_nodal", "box3_elem"])
def test_jacobian_matches_central_differences(case):
    if case == "box2":
        patch, km, kap = inputs.unit_box(2, 5, 3), 0, None
    elif case == "ann2_nodal":
        patch = inputs.quarter_cylinder(4, 2, dim=2)
        km, kap = 1, np.exp(inputs.grf_rff(patch.ctrl, 3, 1))
    elif case == "cyl3_nodal":
        patch = inputs.quarter_cylinder(2, 2, dim=3)
        km, kap = 1, np.exp(inputs.grf_rff(patch.ctrl, 3, 1))
    else:
        patch = inputs.unit_box(3, 3, 2)
        km, kap = 2, inputs.uniform(4, 4, 27, 0.5, 2.0)
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=3.0, kappa_mode=km,
                      kappa=kap)
    U = inputs.initial_guess(patch.shape, 5, 0, 0.0, 0.5)
    J = o.jacobian_csr(U)
    v = inputs.uniform(6, 0, o.N, -1, 1)
    v[inputs.boundary_mask(patch.shape)] = 0.0
    h = 1e-5
    fd = (o.residual(U + h * v) - o.residual(U - h * v)) / (2 * h)
    assert np.linalg.norm(J @ v - fd) < 1e-8 * np.linalg.norm(fd)


@pytest.mark.parametrize("geom,dim,p", [("box", 2, 2), ("box", 3, 3), ("nurbs", 2, 2), ("nurbs", 2, 3),
                                        ("nurbs", 3, 2)])
def test_patch_test_linear_field(geom, dim, p):
    """A linear field is reproduced exactly (Greville abscissae on the box; the isoparametric
    U_A = x_{A,0} on the NURBS patch), so with lambda = 0 and kappa = 1 the residual vanishes for
    every function whose support stays inside the domain.  On the NURBS patch the integrand is
    rational, so the rule is raised until its error is below rounding."""
    if geom == "box":
        patch = inputs.unit_box(dim, 6, p)
        U = _greville_nd(patch)[0]
        nq = None
    else:
        patch = inputs.quarter_cylinder(6, p, dim=dim)
        U = patch.ctrl[:, 0].copy()
        nq = [10] * dim
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=0.0, dirichlet_mask=0,
                      nquad=nq)
    R = o.residual(U)
    idx = np.indices(patch.shape[::-1]).reshape(dim, -1)[::-1]
    inner = np.ones(o.N, dtype=bool)
    for d in range(dim):
        n = patch.shape[d]
        inner &= (idx[d] >= p + 1) & (idx[d] <= n - p - 2)
    assert inner.sum() > 0
    assert np.abs(R[inner]).max() < 1e-13
    assert np.abs(R[~inner]).max() > 1e-3      # boundary rows carry the flux


# ------------------------------------------------------------------------------------------
# Newton
# ------------------------------------------------------------------------------------------

@pytest.mark.slow
def test_tutorial_newton_history_pin():
    """App. B history: iteration 0 exact; iterations 1-6 agree to 1e-5 relative (the paper's
    CG tolerance is unstated, so later digits differ); the last step lands below 1e-10."""
    hist = np.loadtxt(golden("bratu2d_tutorial_history.txt"))[:, 1]
    patch = inputs.unit_box(2, 128, 2)
    o = oracle.Oracle(patch.knots, patch.degree, lam=6.80)
    _, h, rc = o.newton(np.zeros(o.N), atol=1e-10, maxit=12)
    assert rc == 0 and len(h) == len(hist)
    assert abs(h[0] - hist[0]) < 1e-14
    assert np.all(np.abs(h[1:7] - hist[1:7]) / hist[1:7] < 1e-5)
    assert h[7] < 1e-10 and hist[7] < 1e-10


def test_newton_small_config_quadratic_and_symmetric():
    w = inputs.config_2d_small()
    o = oracle.Oracle.from_workload(w)
    U, h, rc = o.newton(w.U0, atol=1e-10)
    assert rc == 0 and h[-1] < 1e-10
    # quadratic convergence in the last steps
    assert h[-1] < 10 * h[-2] ** 2 / h[-3] ** 0 + 1e-13
    assert np.log(h[-2]) / np.log(h[-3]) > 1.6
    # the converged solution is invariant under x <-> 1-x and x <-> y
    n = w.patch.shape[0]
    G = U.reshape(n, n)
    assert np.abs(G - G[:, ::-1]).max() < 1e-9
    assert np.abs(G - G.T).max() < 1e-9
    # lower branch: max u is small for lambda = 6 (the upper branch has max u > 2)
    assert 0 < G.max() < 2.0


def test_newton_lower_branch_by_continuation():
    """max u grows monotonically with lambda along the lower branch reached from U = 0."""
    patch = inputs.unit_box(2, 8, 2)
    prev = 0.0
    for lam in (1.0, 3.0, 5.0, 6.5):
        o = oracle.Oracle(patch.knots, patch.degree, lam=lam)
        U, h, rc = o.newton(np.zeros(o.N), atol=1e-12)
        assert rc == 0
        assert U.max() > prev
        prev = U.max()


@pytest.mark.slow
@pytest.mark.parametrize("p", [2, 3])
def test_manufactured_solution_convergence_rate(p):
    """u* = sin(pi x) sin(pi y), f = 2 pi^2 u* - lambda e^{u*}: the L2 error decays like
    h^(p+1) (f is passed as its L2 projection onto the spline space)."""
    lam = 1.0
    errs = []
    hs = [1 / 4, 1 / 8, 1 / 16]
    for h in hs:
        nel = int(round(1 / h))
        patch = inputs.unit_box(2, nel, p)
        o_proj = oracle.Oracle(patch.knots, patch.degree, lam=0.0, dirichlet_mask=0, nquad=[p + 3] * 2)
        xq, Wq, _, _ = o_proj.qp_data()
        us = np.sin(np.pi * xq[:, 0]) * np.sin(np.pi * xq[:, 1])
        fq = 2 * np.pi ** 2 * us - lam * np.exp(us)
        M = o_proj.mass_matrix()
        f = spla.spsolve(M.tocsc(), o_proj.load_vector(fq))
        o = oracle.Oracle(patch.knots, patch.degree, lam=lam, source=f)
        U, hist, rc = o.newton(np.zeros(o.N), atol=1e-12)
        assert rc == 0
        oe = oracle.Oracle(patch.knots, patch.degree, lam=lam, nquad=[p + 3] * 2)
        xq, Wq, uq, _ = oe.qp_data(U)
        us = np.sin(np.pi * xq[:, 0]) * np.sin(np.pi * xq[:, 1])
        errs.append(math.sqrt(np.sum(Wq * (uq - us) ** 2)))
    rates = [math.log(errs[i] / errs[i + 1], 2) for i in range(len(errs) - 1)]
    assert rates[-1] > p + 1 - 0.3, (errs, rates)


# ------------------------------------------------------------------------------------------
# Consistency of the oracle's partial entry points with its full assembly
# ------------------------------------------------------------------------------------------

def _tensor_support_pattern(patch):
    """Brute force: (A, B) interact iff the open supports overlap on every axis."""
    dim = patch.dim
    sup = []
    for U, p in zip(patch.knots, patch.degree):
        n = len(U) - p - 1
        sup.append(np.array([[max(U[i], U[j]) < min(U[i + p + 1], U[j + p + 1]) for j in range(n)]
                             for i in range(n)]))
    M = sup[0]
    for d in range(1, dim):
        M = np.kron(sup[d], M)
    return M


@pytest.mark.parametrize("kind", ["box2", "box3c1", "c0"])
def test_csr_pattern_bruteforce(kind):
    if kind == "box2":
        patch = inputs.unit_box(2, [4, 3], 3)
    elif kind == "box3c1":
        patch = inputs.unit_box(3, [3, 2, 2], 2, cont=0)
    else:
        patch = inputs.Patch([inputs.open_uniform_knots(4, 3, cont=1), inputs.open_uniform_knots(3, 2)], [3, 2])
    o = oracle.Oracle(patch.knots, patch.degree)
    rp, ci = o.pattern()
    M = np.zeros((o.N, o.N), dtype=bool)
    for A in range(o.N):
        cols = ci[rp[A]:rp[A + 1]]
        assert np.all(np.diff(cols) > 0)
        M[A, cols] = True
    assert np.array_equal(M, _tensor_support_pattern(patch))


def test_partial_entry_points_agree_with_full_assembly():
    patch = inputs.quarter_cylinder([3, 4], 2, dim=2)
    kap = np.exp(inputs.grf_rff(patch.ctrl, 3, 1))
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=2.0, kappa_mode=1, kappa=kap)
    U = inputs.initial_guess(patch.shape, 7, 0, 0.0, 0.4)
    R, J = o.residual(U), o.jacobian(U)
    rp, ci = o.pattern()
    rows = np.array([0, 5, 7, 13, o.N - 1])
    assert np.allclose(o.residual_rows(U, rows), R[rows], rtol=1e-13, atol=1e-16)
    JR = o.jacobian_rows(U, rows)
    ref = np.concatenate([J[rp[r]:rp[r + 1]] for r in rows])
    assert np.allclose(JR, ref, rtol=1e-13, atol=1e-16)
    # all element matrices scattered == the Jacobian without Dirichlet rows
    o0 = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=2.0, kappa_mode=1, kappa=kap,
                       dirichlet_mask=0)
    J0 = o0.jacobian(U)
    v = np.zeros(o0.nnz)
    o0.jacobian_elements(U, np.arange(o0.E), v)
    assert np.allclose(v, J0, rtol=1e-13, atol=1e-15)
    K, Re = o0.element_matrix(U, 4)
    assert np.allclose(K, K.T, rtol=1e-13, atol=1e-15)
    # SpMV against scipy
    x = inputs.uniform(1, 1, o.N, -1, 1)
    y = np.zeros(o.N)
    oracle.lib().orc_spmv(o.N, rp.ctypes.data_as(oracle._i64p), ci.ctypes.data_as(oracle._i32p),
                          J.ctypes.data_as(oracle._dp), x.ctypes.data_as(oracle._dp), y.ctypes.data_as(oracle._dp))
    assert np.allclose(y, o.jacobian_csr(U) @ x, rtol=1e-14, atol=1e-15)


def test_mass_matrix_and_load_vector():
    patch = inputs.quarter_cylinder(4, 2, dim=2)
    E = 16
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=-1.0, kappa_mode=2,
                      kappa=np.zeros(E), dirichlet_mask=0)
    M = o.mass_matrix()
    assert np.allclose(M.toarray(), o.jacobian_csr(np.zeros(o.N)).toarray(), rtol=1e-14, atol=1e-17)
    xq, Wq, _, _ = o.qp_data()
    b = o.load_vector(np.ones(len(Wq)))
    assert np.allclose(b, np.asarray(M.sum(axis=1)).ravel(), rtol=1e-13)
    assert abs(b.sum() - Wq.sum()) < 1e-13
