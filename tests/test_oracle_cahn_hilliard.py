"""Pins of the oracle's Cahn-Hilliard residual (the paper's strong form with D = 1, primal weak form
obtained by integrating by parts twice; periodic axes as in the paper's example):

* a uniform state: R = M_mass Cdot exactly (every gradient and Laplacian vanishes);
* conservation on a fully periodic patch: sum_A R_A = integral of cdot = sum_B Cdot_B int N_B;
* linearisation about c = 1/2: for c = 1/2 + d phi, R(Cdot = 0)/d tends to
  (1/(2 theta) - 1/2) K phi + (lam/4) B phi with an O(d^2) error, K the stiffness (the Jacobian at
  lambda = 0, pinned elsewhere) and B the pinned fourth-order operator: this ties the mobility,
  the chemical-potential derivative and both lam terms to independently checked pieces.

Pins of the oracle's generalized-alpha step of the Cahn-Hilliard system (eq:ga and the parameter
formulas after it), through the same linearisation: for c = 1/2 + d phi the system is, up to O(d^2),
M phi' + L phi = 0 with L = (1/(2 theta) - 1/2) K + (lam/4) B, whose exact solution is
exp(-M^{-1} L t) phi_0 (scipy expm):

* at rho_inf = 1 one step is the implicit midpoint rule (M + dt/2 L)^{-1} (M - dt/2 L) phi_n for any
  rate, as the paper states;
* at rho_inf = 0.5 the step is second order in dt against the exact solution;
* the same checks fail when alpha_m and alpha_f are swapped (first order) or when the c stage is taken
  at t_{n+1} instead of t_{n+alpha_f} (not the midpoint rule): both mistakes are planted in the oracle's
  parameters here, on the CPU."""
import numpy as np
import pytest
import scipy.linalg as sla

import inputs
import oracle


def periodic_patch(dim, p):
    nel = [8, 7, 7][:dim]
    patch = inputs.unit_box(dim, nel, p)
    per = [p - 1] * dim
    return patch, per


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_uniform_state_gives_the_mass_term(dim, p):
    patch, per = periodic_patch(dim, p)
    o = oracle.Oracle(patch.knots, patch.degree, periodic=per)
    rng = np.random.default_rng(dim + p)
    Cd = rng.uniform(-1, 1, o.N)
    R = o.cahn_hilliard_residual(np.full(o.N, 0.3), Cd, 0.7, 0.01)
    ref = o.mass_matrix() @ Cd
    assert np.abs(R - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("dim,p", [(2, 2), (3, 2)])
def test_conservation_on_a_periodic_patch(dim, p):
    patch, per = periodic_patch(dim, p)
    o = oracle.Oracle(patch.knots, patch.degree, periodic=per)
    rng = np.random.default_rng(11)
    C = rng.uniform(0.2, 0.8, o.N)
    Cd = rng.uniform(-1, 1, o.N)
    R = o.cahn_hilliard_residual(C, Cd, 0.667, 0.02)
    integ = np.asarray(o.mass_matrix().sum(axis=0)).ravel()      # int N_B over the periodic domain
    assert abs(R.sum() - integ @ Cd) < 1e-12 * np.abs(R).sum()


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_linearisation_about_one_half(dim, p):
    patch, per = periodic_patch(dim, p)
    o = oracle.Oracle(patch.knots, patch.degree, periodic=per, lam=0.0)
    rng = np.random.default_rng(5 * dim + p)
    phi = rng.uniform(-1, 1, o.N)
    theta, lam = 0.8, 0.05
    K = o.jacobian_csr(np.zeros(o.N))
    ref = (1.0 / (2 * theta) - 0.5) * (K @ phi) + lam / 4.0 * o.biharmonic_residual(phi)
    errs = []
    for d in (1e-3, 5e-4):
        R = o.cahn_hilliard_residual(0.5 + d * phi, np.zeros(o.N), theta, lam) / d
        errs.append(np.linalg.norm(R - ref) / np.linalg.norm(ref))
    assert errs[0] < 1e-4 and 3.0 < errs[0] / errs[1] < 5.0, errs      # O(d^2)


def polar_quadratic(U, p):
    n = len(U) - p - 1
    return np.array([sum(U[i + 1 + j] * U[i + 1 + k] for j in range(p) for k in range(j + 1, p)) * 2.0 / (p * (p - 1))
                     for i in range(n)])


@pytest.mark.parametrize("dim,p", [(2, 2), (2, 3), (3, 2)])
def test_fourth_order_term_vanishes_for_a_constant_laplacian(dim, p):
    """lam (M Lap N_A + M' grad c . grad N_A) Lap c = lam div(M grad N_A) Lap c; for c = 0.3 + s |x|^2
    (Lap c = 2 dim s) its integral is a boundary term, zero for every function that vanishes with its
    gradient on the boundary: the lam-part of R (R at lam = 1 minus R at lam = 0) is zero there."""
    patch = inputs.unit_box(dim, [6, 7, 5][:dim], p)
    o = oracle.Oracle(patch.knots, patch.degree)
    q = [polar_quadratic(K, p) for K in patch.knots]
    n = [len(c) for c in q]
    C = 0.3 * np.ones(o.N)
    for ax in range(dim):
        shape = [1] * dim
        shape[dim - 1 - ax] = n[ax]
        C = C + 0.1 * np.broadcast_to(q[ax].reshape(shape), tuple(n[::-1])).ravel()
    Z = np.zeros(o.N)
    lam_part = o.cahn_hilliard_residual(C, Z, 0.7, 1.0) - o.cahn_hilliard_residual(C, Z, 0.7, 0.0)
    idx = np.stack(np.unravel_index(np.arange(o.N), tuple(n[::-1]))[::-1], -1)
    interior = np.all((idx >= 2) & (idx <= np.array(n) - 3), axis=1)
    assert interior.sum() > 0
    scale = np.abs(lam_part).max()
    assert np.abs(lam_part[interior]).max() < 1e-11 * scale, np.abs(lam_part[interior]).max() / scale


def test_generalized_alpha_step_conserves_mass_and_keeps_uniform_states():
    """With every axis periodic the residual's rows sum to the integral of cdot, so a step that starts
    from a zero-mean rate keeps the integral of c; a uniform state at rest stays put."""
    patch, per = periodic_patch(2, 2)
    o = oracle.Oracle(patch.knots, patch.degree, periodic=per)
    m = np.asarray(o.mass_matrix().sum(axis=0)).ravel()
    C0 = 0.5 + 0.05 * np.random.default_rng(2).uniform(-1, 1, o.N)
    C1, V1, it = o.ch_gen_alpha_step(C0, np.zeros(o.N), 1e-3, 0.5, 1.5, 0.01)
    assert it >= 1
    assert abs(m @ C1 - m @ C0) < 1e-12 * abs(m @ C0)
    assert abs(m @ V1) < 1e-9 * np.abs(V1).max() * m.sum()
    Cu, Vu, _ = o.ch_gen_alpha_step(np.full(o.N, 0.4), np.zeros(o.N), 1e-3, 0.5, 1.5, 0.01)
    assert np.abs(Cu - 0.4).max() < 1e-14 and np.abs(Vu).max() < 1e-12


def linearised_ch_system(theta, lam):
    """Periodic 6x6 C^1 quadratic patch: the oracle, its mass matrix M and the operator L of the
    Cahn-Hilliard residual linearised about c = 1/2 (K: Jacobian at lambda = 0, B: fourth-order
    operator column by column; both pinned above and in the fourth-order tests)."""
    patch = inputs.unit_box(2, [6, 6], 2)
    o = oracle.Oracle(patch.knots, patch.degree, periodic=[1, 1], lam=0.0)
    K = o.jacobian_csr(np.zeros(o.N)).toarray()
    B = np.column_stack([o.biharmonic_residual(e) for e in np.eye(o.N)])
    M = o.mass_matrix().toarray()
    return o, M, (1.0 / (2 * theta) - 0.5) * K + lam / 4.0 * B


CH_THETA, CH_LAM, CH_AMP = 0.8, 0.01, 1e-5


def midpoint_error(o, M, L):
    """Relative distance of one rho_inf = 1 step (from c = 1/2 + d phi with a random rate) to the
    implicit midpoint rule of the linearised system."""
    rng = np.random.default_rng(21)
    phi = rng.uniform(-1, 1, o.N)
    V0 = CH_AMP * rng.uniform(-50, 50, o.N)          # any rate: the midpoint update ignores it
    dt = 1e-3
    C1, _, _ = o.ch_gen_alpha_step(0.5 + CH_AMP * phi, V0, dt, 1.0, CH_THETA, CH_LAM, atol=1e-14)
    ref = np.linalg.solve(M + 0.5 * dt * L, (M - 0.5 * dt * L) @ phi)
    return np.linalg.norm((C1 - 0.5) / CH_AMP - ref) / np.linalg.norm(ref)


def time_error_ratios(o, M, L, T=2e-3):
    """Errors against exp(-M^{-1} L T) phi after 4, 8, 16 steps of rho_inf = 0.5 from a consistent rate,
    and the ratios of successive errors (4 for a second-order method)."""
    phi = np.random.default_rng(3).uniform(-1, 1, o.N)
    exact = sla.expm(-np.linalg.solve(M, L) * T) @ phi
    errs = []
    for nsteps in (4, 8, 16):
        dt = T / nsteps
        C = 0.5 + CH_AMP * phi
        V = -CH_AMP * np.linalg.solve(M, L @ phi)
        for _ in range(nsteps):
            C, V, _ = o.ch_gen_alpha_step(C, V, dt, 0.5, CH_THETA, CH_LAM, atol=1e-14)
        errs.append(np.linalg.norm((C - 0.5) / CH_AMP - exact) / np.linalg.norm(exact))
    return errs, errs[0] / errs[1], errs[1] / errs[2]


def test_ch_generalized_alpha_is_the_midpoint_rule_at_rho_one():
    o, M, L = linearised_ch_system(CH_THETA, CH_LAM)
    err = midpoint_error(o, M, L)
    assert err < 1e-4, err                        # O(d) from the nonlinearity, d = 1e-5


def test_ch_generalized_alpha_is_second_order_in_time():
    o, M, L = linearised_ch_system(CH_THETA, CH_LAM)
    errs, r1, r2 = time_error_ratios(o, M, L)
    assert errs[0] < 1e-2 and 3.5 < r1 < 4.6 and 3.5 < r2 < 4.6, errs


def test_ch_generalized_alpha_pins_catch_planted_parameter_mistakes(monkeypatch):
    o, M, L = linearised_ch_system(CH_THETA, CH_LAM)
    good = oracle.gen_alpha_params
    # alpha_m and alpha_f swapped: gamma = 1/2 + alpha_m - alpha_f no longer holds, first order
    monkeypatch.setattr(oracle, "gen_alpha_params", lambda r: (good(r)[1], good(r)[0], good(r)[2]))
    errs, r1, r2 = time_error_ratios(o, M, L)
    assert r1 < 2.5 and r2 < 2.5, errs
    # the c stage at t_{n+1} (alpha_f = 1) instead of t_{n+1/2}: no longer the midpoint rule
    monkeypatch.setattr(oracle, "gen_alpha_params", lambda r: (good(r)[0], 1.0, good(r)[2]))
    assert midpoint_error(o, M, L) > 1e-2
