"""Batched Newton (iga_batch_*) against per-instance Newton and the oracle."""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1305_4452_amd as iga  # noqa: E402


def mixed_workloads():
    """Instances given in mixed degree/size order (exercises the internal regrouping)."""
    ws = []
    specs = [(12, 3, 2.0), (8, 2, 6.0), (20, 4, 1.0), (9, 2, 4.5), (16, 3, 6.4), (8, 4, 3.3), (33, 2, 5.0),
             (10, 3, 1.2)]
    for i, (nel, p, lam) in enumerate(specs):
        ws.append(inputs.bratu_box(2, nel, p, lam, seed=4, stream=i))
    # one element-wise kappa instance (p = 3, 8x8 elements, kappa constant on 2x2 blocks)
    _, lam, w = inputs.learned_instance(3, nel=8, p=3, ncell=4)
    w.lam = 1.5          # sub-critical for this kappa draw (lambda = 5 has no solution here)
    w.U0 = inputs.initial_guess(w.patch.shape, 4, 99)
    ws.append(w)
    return ws


def test_batch_matches_per_instance_and_oracle():
    ws = mixed_workloads()
    b = iga.IGABatch(ws)
    U = torch.as_tensor(b.pack([w.U0 for w in ws]), device="cuda")
    per, summ = b.newton_solve(U, atol=1e-10)
    assert summ["all_converged"] and all(p["converged"] for p in per)
    assert all(p["res_norm"] < 1e-10 for p in per)
    # one graph replay per Newton step (and the final convergence test), plus any extra CG chunks
    assert summ["graph_launches"] >= summ["newton_steps"] + 1
    assert max(p["newton_iters"] for p in per) == summ["newton_steps"]
    sols = b.unpack(U.cpu().numpy())
    for i, w in enumerate(ws):
        g = iga.IGA.from_workload(w)
        Ui = torch.as_tensor(w.U0, device="cuda")
        g.newton_solve(Ui, atol=1e-10)
        ref = Ui.cpu().numpy()
        assert np.linalg.norm(sols[i] - ref) <= 1e-8 * np.linalg.norm(ref), i
    for i in (1, 4, 8):
        o = oracle.Oracle.from_workload(ws[i])
        Uo, _, rc = o.newton(ws[i].U0, atol=1e-13)
        assert rc == 0
        assert np.linalg.norm(sols[i] - Uo) <= 1e-9 * np.linalg.norm(Uo), i


def test_batch_fp32_jacobian_and_determinism():
    ws = mixed_workloads()[:6]
    b = iga.IGABatch(ws)
    U0 = b.pack([w.U0 for w in ws])
    U1 = torch.as_tensor(U0, device="cuda")
    U2 = torch.as_tensor(U0, device="cuda")
    b.newton_solve(U1, atol=1e-10)
    b.newton_solve(U2, atol=1e-10)
    # the Jacobian and the CG reductions are order-fixed; the residual scatter uses FP64 atomics,
    # so two runs agree to rounding, not bit for bit
    assert torch.allclose(U1, U2, rtol=0, atol=1e-12 * float(U1.abs().max()))
    U3 = torch.as_tensor(U0, device="cuda")
    per, summ = b.newton_solve(U3, atol=1e-10, jac_prec=iga.IGA_FP32)
    assert all(p["converged"] for p in per)
    assert torch.allclose(U3, U1, rtol=0, atol=1e-9)


def test_batch_seeded_configuration_subset():
    ws = inputs.batched_instances(24)
    b = iga.IGABatch(ws)
    U = torch.as_tensor(b.pack([w.U0 for w in ws]), device="cuda")
    per, summ = b.newton_solve(U, atol=1e-10)
    assert summ["all_converged"]
    sols = b.unpack(U.cpu().numpy())
    for i in (0, 7, 13):
        g = iga.IGA.from_workload(ws[i])
        Ui = torch.as_tensor(ws[i].U0, device="cuda")
        g.newton_solve(Ui, atol=1e-10)
        ref = Ui.cpu().numpy()
        assert np.linalg.norm(sols[i] - ref) <= 1e-8 * np.linalg.norm(ref)


def test_batch_rejects_unsupported():
    w3 = inputs.bratu_box(3, 3, 2, 1.0, seed=1)
    with pytest.raises(iga.IGAError) as e:
        iga.IGABatch([w3])
    assert e.value.status == iga.IGA_EUNSUPPORTED


def test_batch_fdm_and_jacobi_agree():
    """The batched fast-diagonalisation preconditioner (the default) and Jacobi reach the same
    solutions; the former in far fewer CG iterations (one element-wise kappa instance included)."""
    ws = mixed_workloads()
    b = iga.IGABatch(ws)
    U0 = b.pack([w.U0 for w in ws])
    Uf = torch.as_tensor(U0, device="cuda")
    per_f, _ = b.newton_solve(Uf, atol=1e-10)
    b.set_option(iga.IGA_OPT_PRECOND, iga.IGA_PRECOND_JACOBI)
    Uj = torch.as_tensor(U0, device="cuda")
    per_j, _ = b.newton_solve(Uj, atol=1e-10)
    assert all(p["converged"] for p in per_f + per_j)
    assert float((Uf - Uj).norm()) <= 1e-8 * float(Uj.norm())
    kf = sum(p["krylov_iters"] for p in per_f)
    kj = sum(p["krylov_iters"] for p in per_j)
    assert kf < 0.5 * kj, (kf, kj)
    b.set_option(iga.IGA_OPT_PRECOND, iga.IGA_PRECOND_FDM)
    U2 = torch.as_tensor(U0, device="cuda")
    per2, summ2 = b.newton_solve(U2, atol=1e-10, check_every=2)
    assert summ2["all_converged"]
    assert float((U2 - Uj).norm()) <= 1e-8 * float(Uj.norm())


def test_batch_fdm_unavailable_for_long_axes():
    ws = [inputs.bratu_box(2, 140, 2, 1.0, seed=4, stream=0), inputs.bratu_box(2, 8, 3, 2.0, seed=4, stream=1)]
    b = iga.IGABatch(ws)
    with pytest.raises(iga.IGAError) as e:
        b.set_option(iga.IGA_OPT_PRECOND, iga.IGA_PRECOND_FDM)
    assert e.value.status == iga.IGA_EUNSUPPORTED
    U = torch.as_tensor(b.pack([w.U0 for w in ws]), device="cuda")
    per, summ = b.newton_solve(U, atol=1e-10)
    assert summ["all_converged"]


def _interior(shape, u):
    """u with the entries of the Dirichlet faces (every face of the unit box) set to zero."""
    g = np.array(u, dtype=np.float64).reshape(shape[::-1])
    g[0, :] = g[-1, :] = 0.0
    g[:, 0] = g[:, -1] = 0.0
    return g.ravel()


def test_batch_error_estimates_exact_for_the_linear_problem():
    """With lambda = 0 and kappa = 1 the fast-diagonalisation operator is the Jacobian itself and
    R(U) = J U, so ||P^{-1} R(U)|| equals ||U|| for any U that vanishes on the Dirichlet faces."""
    print("[case] batched error estimates, linear problem", flush=True)
    ws = [inputs.bratu_box(2, nel, p, 0.0, seed=7, stream=i) for i, (nel, p) in enumerate([(12, 2), (20, 3), (9, 4),
                                                                                          (31, 2)])]
    b = iga.IGABatch(ws)
    us = [_interior(w.patch.shape, inputs.uniform(40 + i, 0, w.patch.ndof, -1.0, 1.0)) for i, w in enumerate(ws)]
    est = b.error_estimates(torch.as_tensor(b.pack(us), device="cuda"))
    ref = np.array([np.linalg.norm(u) for u in us])
    assert np.allclose(est, ref, rtol=1e-10, atol=0.0), (est, ref)
    b.close()


def test_batch_error_estimates_track_the_error():
    """At the converged solution the estimate is at rounding level; from the zero guess (error
    ||U*||) it is within a factor two of ||U*||, for every instance of the mixed batch."""
    print("[case] batched error estimates, Bratu and kappa instances", flush=True)
    ws = mixed_workloads()
    b = iga.IGABatch(ws)
    U = torch.as_tensor(b.pack([np.zeros(w.patch.ndof) for w in ws]), device="cuda")
    est0 = b.error_estimates(U)
    per, summ = b.newton_solve(U, atol=1e-12)
    assert summ["all_converged"]
    sols = b.unpack(U.cpu().numpy())
    nrm = np.array([np.linalg.norm(s) for s in sols])
    assert np.all(est0 > 0.5 * nrm) and np.all(est0 < 2.0 * nrm), (est0, nrm)
    est1 = b.error_estimates(U)
    assert np.all(est1 < 1e-8 * nrm), (est1, nrm)
    b.close()
