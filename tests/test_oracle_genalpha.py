"""Pins of the oracle's generalized-alpha step (eq:ga) for M0 Udot + R(U) = 0:

* the parameters at rho_inf = 1 are 1/2, 1/2, 1/2 and the step is the implicit midpoint rule, as the paper
  states: with lambda = 0 (R = K U) one step equals (M0 + dt/2 K)^{-1} (M0 - dt/2 K) U_n for any Udot_n;
* second-order accuracy in time (rho_inf = 0.5) against the exact solution exp(-M0^{-1} K t) U_0 of the
  linear system (scipy expm);
* the steady Bratu solution with zero rate is a fixed point of a nonlinear step;
* rho_inf = 0 damps: the M0-norm of a rough start decays step after step at a large dt."""
import numpy as np
import pytest
import scipy.linalg as sla

import inputs
import oracle


def free_mask(patch):
    """True on functions that are not on a Dirichlet face (every face of the unit box)."""
    shape = [len(k) - p - 1 for k, p in zip(patch.knots, patch.degree)]
    return ~inputs.boundary_mask(shape)


def dense_ops(patch, o):
    """Dense mass matrix and lambda = 0 Jacobian (the stiffness) on the free functions."""
    f = free_mask(patch)
    M = o.mass_matrix().toarray()
    K = o.jacobian_csr(np.zeros(o.N)).toarray()
    return M[np.ix_(f, f)], K[np.ix_(f, f)], f


def test_parameters():
    assert np.allclose(oracle.gen_alpha_params(1.0), (0.5, 0.5, 0.5))
    assert np.allclose(oracle.gen_alpha_params(0.0), (1.5, 1.0, 1.0))
    am, af, g = oracle.gen_alpha_params(0.3)
    assert abs(g - (0.5 + am - af)) < 1e-15 and am > af


@pytest.mark.parametrize("p", [2, 3])
def test_midpoint_rule_at_rho_one(p):
    patch = inputs.unit_box(2, [6, 5], p)
    o = oracle.Oracle(patch.knots, patch.degree, lam=0.0)
    M, K, f = dense_ops(patch, o)
    rng = np.random.default_rng(p)
    U0 = np.where(f, rng.uniform(-1, 1, o.N), 0.0)
    V0 = np.where(f, rng.uniform(-1, 1, o.N), 0.0)          # any rate: the midpoint update ignores it
    dt = 0.01
    U1, V1, it = o.gen_alpha_step(U0, V0, dt, 1.0)
    ref = np.linalg.solve(M + 0.5 * dt * K, (M - 0.5 * dt * K) @ U0[f])
    assert np.abs(U1[f] - ref).max() < 1e-11 * np.abs(ref).max()
    assert np.all(U1[~f] == 0.0)


def test_second_order_in_time():
    p = 2
    patch = inputs.unit_box(2, [5, 4], p)
    o = oracle.Oracle(patch.knots, patch.degree, lam=0.0)
    M, K, f = dense_ops(patch, o)
    rng = np.random.default_rng(7)
    u0 = rng.uniform(-1, 1, f.sum())
    T = 0.02
    exact = sla.expm(-np.linalg.solve(M, K) * T) @ u0
    errs = []
    for nsteps in (8, 16, 32):
        dt = T / nsteps
        U = np.zeros(o.N)
        U[f] = u0
        V = np.zeros(o.N)
        V[f] = -np.linalg.solve(M, K @ u0)                   # consistent initial rate
        for _ in range(nsteps):
            U, V, _ = o.gen_alpha_step(U, V, dt, 0.5)
        errs.append(np.linalg.norm(U[f] - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_steady_solution_is_a_fixed_point():
    patch = inputs.unit_box(2, [8, 7], 3)
    o = oracle.Oracle(patch.knots, patch.degree, lam=4.0)
    U, _, rc = o.newton(np.zeros(o.N), atol=1e-13)
    assert rc == 0
    U1, V1, it = o.gen_alpha_step(U, np.zeros(o.N), 0.05, 0.5, atol=1e-11)
    assert np.abs(U1 - U).max() < 1e-11 and np.abs(V1).max() < 1e-9


def test_rho_zero_damps_at_large_steps():
    patch = inputs.unit_box(2, [6, 6], 2)
    o = oracle.Oracle(patch.knots, patch.degree, lam=0.0)
    M, K, f = dense_ops(patch, o)
    rng = np.random.default_rng(3)
    U = np.where(f, rng.uniform(-1, 1, o.N), 0.0)
    V = np.zeros(o.N)
    norms = []
    for _ in range(6):
        U, V, _ = o.gen_alpha_step(U, V, 10.0, 0.0)
        norms.append(float(U[f] @ M @ U[f]))
    assert all(b < a for a, b in zip(norms, norms[1:]))
