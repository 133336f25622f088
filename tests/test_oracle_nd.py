"""Pins of the oracle's local numerical-differentiation Jacobian (Sec. 2.8, eq:fdjac).

The finite-difference Jacobian is checked against what fixes it independently of the oracle's
own code: the exact Jacobian (itself pinned elsewhere) within the first-order error bound, the
linear case (no truncation error), the first-order scaling of the error with the step, and a
single bilinear element computed here from scratch with numpy's Gauss-Legendre rule, which fixes
the step delta = eta sqrt(1 + ||U_e||_2)."""
import numpy as np
import pytest

import inputs
import oracle


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def cases():
    cyl = inputs.quarter_cylinder(4, 2, dim=2)
    return {
        "box2_p3": (inputs.unit_box(2, [5, 4], 3), 4.0, 0, None, None),
        "annulus_p2_nodal": (cyl, 1.0, 1, np.exp(inputs.grf_rff(cyl.ctrl, 3, 1)), None),
        "box3_p2_mask": (inputs.unit_box(3, 3, 2), 5.0, 0, None, 0b010110),
        "box2_p2_kel_src": (inputs.unit_box(2, [4, 3], 2), 2.0, 2, inputs.uniform(8, 1, 12, 0.5, 2.0), "src"),
    }


def build(name, lam=None):
    patch, lm, km, kap, extra = cases()[name]
    src = inputs.uniform(8, 2, patch.ndof, -1.0, 1.0) if extra == "src" else None
    mask = extra if isinstance(extra, int) else None
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, lam=lm if lam is None else lam,
                      kappa_mode=km, kappa=kap, source=src, dirichlet_mask=mask)
    return o, inputs.uniform(11, 3, patch.ndof, 0.0, 0.3)


@pytest.mark.parametrize("name", list(cases()))
def test_nd_within_first_order_bound_of_exact(name):
    o, U = build(name)
    J = o.jacobian(U)
    e = rel(o.jacobian_nd(U), J)
    # default step ~1.5e-8: truncation O(delta) plus rounding O(eps / delta), both ~1e-8 relative
    assert 0.0 < e < 1e-7


@pytest.mark.parametrize("name", list(cases()))
def test_nd_error_is_first_order_in_the_step(name):
    o, U = build(name)
    J = o.jacobian(U)
    e4, e6 = rel(o.jacobian_nd(U, 1e-4), J), rel(o.jacobian_nd(U, 1e-6), J)
    assert 80.0 < e4 / e6 < 120.0


def test_nd_exact_for_a_linear_problem():
    # lambda = 0: F_q is linear in U_e, the difference quotient has no truncation error
    o, U = build("box2_p3", lam=0.0)
    assert rel(o.jacobian_nd(U, 1e-3), o.jacobian(U)) < 1e-11


def bilinear_nd(U, lam, delta):
    """Local-ND matrix of one bilinear element on [0,1]^2 with step delta, from scratch."""
    x, w = np.polynomial.legendre.leggauss(2)
    x, w = 0.5 * (x + 1.0), 0.5 * w
    N1 = lambda t: np.array([1.0 - t, t])
    D1 = lambda t: np.array([-1.0, 1.0])
    K = np.zeros((4, 4))
    for i, xi in enumerate(x):
        for j, yj in enumerate(x):
            W = w[i] * w[j]
            N = np.kron(N1(yj), N1(xi))                 # local a = a0 + 2 a1 (axis 0 fastest)
            G = np.stack([np.kron(N1(yj), D1(xi)), np.kron(D1(yj), N1(xi))], axis=1)

            def F(Ue):
                u, gu = N @ Ue, G.T @ Ue
                return W * (G @ gu - N * lam * np.exp(u))
            F0 = F(U)
            for k in range(4):
                Up = U.copy()
                Up[k] += delta
                K[:, k] += (F(Up) - F0) / delta
    return K


def test_nd_single_bilinear_element_from_scratch():
    """One bilinear element, no Dirichlet faces: the four columns by hand, with the step
    delta = eta sqrt(1 + ||U_e||_2)."""
    lam, eta = 3.0, 1e-3
    patch = inputs.unit_box(2, 1, 1)
    o = oracle.Oracle(patch.knots, patch.degree, None, None, lam=lam, dirichlet_mask=0)
    U = np.array([0.3, -0.2, 0.5, 0.1])
    rp, ci = o.pattern()
    dense = np.zeros((4, 4))
    vals = o.jacobian_nd(U, eta)
    for A in range(4):
        for s in range(rp[A], rp[A + 1]):
            dense[A, ci[s]] = vals[s]
    K = bilinear_nd(U, lam, eta * np.sqrt(1.0 + np.linalg.norm(U)))
    assert np.max(np.abs(dense - K)) < 1e-12 * np.max(np.abs(K))
    # the check resolves the step: the squared norm in place of the norm gives another matrix
    K2 = bilinear_nd(U, lam, eta * np.sqrt(1.0 + np.linalg.norm(U) ** 2))
    assert np.max(np.abs(dense - K2)) > 1e-8 * np.max(np.abs(K))
