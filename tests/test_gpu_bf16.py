"""BF16 matrix-core Jacobians (iga_assemble_jacobian with IGA_BF16 / IGA_BF16X3) against the FP64 oracle.

The contraction over axis 2 runs on v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Bars (relative
Frobenius error of the CSR values against the oracle's FP64 Jacobian, the metric the FP32 path uses
for element matrices, here over every assembled value): BF16 5e-3 (a BF16 operand keeps 8 significant
bits, unit roundoff 2^-9 ~ 2e-3, times the few roundings of one product), split BF16 1e-5 (each FP32
operand as hi + lo BF16, three products).  Newton with either Jacobian keeps the FP64 residual and must
reach the FP64 oracle's solution (relative 1e-9).  Cases span several 2 x 2 pencil blocks, ragged at
the far ends, on NURBS geometry with nodal kappa (the general metric, 16 terms) and on x = xi with
element kappa (4 terms)."""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1305_4452_amd as iga  # noqa: E402

BARS = {iga.IGA_BF16: 5e-3, iga.IGA_BF16X3: 1e-5}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def make_case(name):
    if name == "cyl3_p2_nodal":
        p = inputs.quarter_cylinder([7, 6, 5], 2, dim=3)
        return p, 1.0, 1, np.exp(inputs.grf_rff(p.ctrl, 3, 1)), None
    if name == "cyl3_p3_nodal":
        p = inputs.quarter_cylinder([5, 5, 4], 3, dim=3)
        return p, 1.0, 1, np.exp(inputs.grf_rff(p.ctrl, 3, 1)), None
    if name == "cyl3_p4_nodal":
        p = inputs.quarter_cylinder([4, 5, 3], 4, dim=3)
        return p, 1.0, 1, np.exp(inputs.grf_rff(p.ctrl, 3, 1)), None
    if name == "box3_p3_kel":
        p = inputs.unit_box(3, [5, 6, 4], 3)
        return p, 3.0, 2, inputs.uniform(8, 2, 120, 0.5, 2.0), None
    if name == "box3_p2":
        return inputs.unit_box(3, [5, 4, 3], 2), 5.0, 0, None, None
    if name == "box3_p4_mask":
        return inputs.unit_box(3, [4, 3, 5], 4), 1.0, 0, None, 0b010110
    raise KeyError(name)


CASES = ["cyl3_p2_nodal", "cyl3_p3_nodal", "cyl3_p4_nodal", "box3_p3_kel", "box3_p2", "box3_p4_mask"]


def pair(name):
    patch, lam, km, kap, mask = make_case(name)
    kw = dict(lam=lam, kappa_mode=km, kappa=kap, dirichlet_mask=mask)
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, **kw)
    g = iga.IGA(patch.knots, patch.degree, patch.ctrl, patch.weights, **kw)
    return patch, o, g


@pytest.mark.parametrize("prec", [iga.IGA_BF16, iga.IGA_BF16X3])
@pytest.mark.parametrize("name", CASES)
def test_bf16_jacobian_matches_oracle(name, prec):
    print(f"[case] BF16 jacobian {name} prec={prec}", flush=True)
    patch, o, g = pair(name)
    U = inputs.uniform(11, 3, patch.ndof, 0.0, 0.3)
    vals = torch.full((g.nnz,), float("nan"), dtype=torch.float32, device="cuda")
    g.assemble_jacobian(torch.as_tensor(U, device="cuda"), vals, prec)
    torch.cuda.synchronize()
    got = vals.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got)), "some CSR value was never written"
    ref = o.jacobian(U)
    err = rel(got, ref)
    rp, _ = o.pattern()
    rows = [rel(got[rp[A]:rp[A + 1]], ref[rp[A]:rp[A + 1]]) for A in range(o.N)]
    print(f"  relative Frobenius error {err:.2e}, worst row {max(rows):.2e}", flush=True)
    assert err < BARS[prec]


@pytest.mark.parametrize("prec", [iga.IGA_BF16, iga.IGA_BF16X3])
@pytest.mark.parametrize("p,nel", [(3, [13, 5, 4]), (4, [11, 4, 3]), (2, [9, 5, 4])])
def test_bf16_segments_along_axis0(p, nel, prec):
    """Pencils split into segments along axis 0 (IGA_OPT_ROW_SEGMENTS; ragged last segments, segments
    shorter than the p warm-up columns): every row sums the same element columns in the same order,
    so the values equal the unsplit ones bit for bit, and meet the oracle's bar."""
    print(f"[case] BF16 segments p={p} nel={nel} prec={prec}", flush=True)
    patch = inputs.quarter_cylinder(nel, p, dim=3)
    kap = np.exp(inputs.grf_rff(patch.ctrl, 3, 1))
    kw = dict(lam=1.0, kappa_mode=1, kappa=kap)
    o = oracle.Oracle(patch.knots, patch.degree, patch.ctrl, patch.weights, **kw)
    g = iga.IGA(patch.knots, patch.degree, patch.ctrl, patch.weights, **kw)
    U = torch.as_tensor(inputs.uniform(11, 3, patch.ndof, 0.0, 0.3), device="cuda")
    ref = o.jacobian(U.cpu().numpy())
    base = None
    for nseg in (1, 2, 3, 5, nel[0], 0):
        g.set_option(iga.IGA_OPT_ROW_SEGMENTS, nseg)
        vals = torch.full((g.nnz,), float("nan"), dtype=torch.float32, device="cuda")
        g.assemble_jacobian(U, vals, prec)
        torch.cuda.synchronize()
        got = vals.cpu().numpy()
        assert np.all(np.isfinite(got)), nseg
        if base is None:
            base = got
        assert np.array_equal(got, base), nseg
        assert rel(got, ref) < BARS[prec], nseg


@pytest.mark.parametrize("prec", [iga.IGA_BF16, iga.IGA_BF16X3])
@pytest.mark.parametrize("name", ["cyl3_p3_nodal", "box3_p3_kel"])
def test_newton_with_bf16_jacobian_reaches_fp64_solution(name, prec):
    print(f"[case] Newton with BF16 jacobian {name} prec={prec}", flush=True)
    patch, o, g = pair(name)
    U0 = inputs.uniform(12, 0, patch.ndof, 0.0, 0.1)
    ref, _, rc = o.newton(U0, atol=1e-13)
    assert rc == 0
    U = torch.as_tensor(U0, device="cuda")
    rep = g.newton_solve(U, atol=0.0, rtol=1e-12, jac_prec=prec, max_newton=40)
    assert rep["converged"] and rep["res_norm"] <= 1e-12 * rep["res_norm0"]
    torch.cuda.synchronize()
    assert rel(U.cpu().numpy(), ref) < 1e-9


def test_bf16_rejections():
    patch = inputs.unit_box(2, 6, 2)
    g = iga.IGA(patch.knots, patch.degree, lam=1.0)
    x = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IGAError) as ei:
        g.assemble_jacobian(x, torch.empty(g.nnz, dtype=torch.float32, device="cuda"), iga.IGA_BF16)
    assert ei.value.status == iga.IGA_EUNSUPPORTED
