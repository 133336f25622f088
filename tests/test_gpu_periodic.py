"""Periodic axes (Sec. 2.4) on the GPU against the oracle: both unclamp the open knots
(eq:unclamp-left/right) and wrap indices (eq:map-wrap) with code of their own.  Same bars as the
other parity tests: identical CSR pattern, 1e-12 relative for FP64 residuals, Jacobians, applies
and SpMV, 1e-7 for the local numerical-differentiation Jacobian, 1e-9 for Newton solutions."""
import numpy as np
import pytest

import inputs
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1305_4452_amd as iga  # noqa: E402

TOL64 = 1e-12

# name: (dim, nel, p, periodic continuity per axis (None: open), lambda, kappa element-wise)
CASES = {
    "per2_p2_c1_x": (2, [9, 7], 2, [1, None], 3.0, False),
    "per2_p3_c0_x_kel": (2, [10, 8], 3, [0, None], 2.0, True),
    "per2_p2_full": (2, [8, 9], 2, [1, 0], 1.0, False),
    "per3_p2_xz": (3, [7, 6, 7], 2, [1, None, 0], 2.5, False),   # y-only Dirichlet: 1D-like fold near 3.5
    "per3_p3_c2_x": (3, [8, 5, 6], 3, [2, None, None], 3.0, False),
    # three functions per periodic axis: a residual tile covers the axis and wraps onto itself
    "per3_p1_tiny": (3, [3, 3, 5], 1, [0, 0, None], 1.0, False),
    # periodic axis 2 walked by runs of chunks (residual and apply for every run length)
    "per3_p2_z_long": (3, [5, 4, 18], 2, [None, None, 1], 2.0, True),
    "per3_p2_z_wrap": (3, [6, 5, 5], 2, [None, 1, 1], 1.5, False),   # the first chunk wraps onto itself
}


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def build(name):
    dim, nel, p, per, lam, kel = CASES[name]
    patch = inputs.unit_box(dim, nel, p)
    ne = [n - p for n in patch.shape]
    kap = inputs.uniform(9, 5, int(np.prod(ne)), 0.5, 2.0) if kel else None
    km = iga.IGA_KAPPA_ELEMENT if kel else iga.IGA_KAPPA_ONE
    o = oracle.Oracle(patch.knots, patch.degree, lam=lam, kappa_mode=km, kappa=kap, periodic=per)
    g = iga.IGA(patch.knots, patch.degree, lam=lam, kappa_mode=km, kappa=kap, periodic=per)
    U = inputs.uniform(11, 3, o.N, 0.0, 0.3)
    return o, g, U


@pytest.mark.parametrize("name", list(CASES))
def test_periodic_pattern_residual_jacobians(name):
    print(f"[case] periodic {name}", flush=True)
    o, g, U = build(name)
    assert (g.N, g.nnz) == (o.N, o.nnz)
    rp, ci = g.csr_pattern()
    orp, oci = o.pattern()
    assert np.array_equal(host(rp), orp) and np.array_equal(host(ci), oci)
    R = torch.full((g.N,), np.nan, dtype=torch.float64, device="cuda")
    g.assemble_residual(dev(U), R)
    assert rel(host(R), o.residual(U)) < TOL64
    ref = o.jacobian(U)
    for algo in (iga.IGA_JAC_AUTO, iga.IGA_JAC_ATOMIC):
        g.set_option(iga.IGA_OPT_JAC_ALGO, algo)
        vals = torch.full((g.nnz,), np.nan, dtype=torch.float64, device="cuda")
        g.assemble_jacobian(dev(U), vals)
        got = host(vals)
        assert np.all(np.isfinite(got))
        assert rel(got, ref) < TOL64
    g.set_option(iga.IGA_OPT_JAC_ALGO, iga.IGA_JAC_LOCAL_ND)
    vals = torch.full((g.nnz,), np.nan, dtype=torch.float64, device="cuda")
    g.assemble_jacobian(dev(U), vals)
    assert rel(host(vals), o.jacobian_nd(U)) < 1e-7
    # matrix-free apply and the CSR SpMV with column indices
    v = inputs.uniform(12, 4, g.N, -1.0, 1.0)
    y = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    g.apply(dev(U), dev(v), y)
    Jv = o.jacobian_csr(U) @ v
    assert rel(host(y), Jv) < TOL64
    if len(CASES[name][1]) == 3:
        Rref = o.residual(U)
        for zrun in (1, 2, 3, 4):
            g.set_option(iga.IGA_OPT_RES_ZRUN, zrun)
            R = torch.full((g.N,), np.nan, dtype=torch.float64, device="cuda")
            g.assemble_residual(dev(U), R)
            y = torch.full((g.N,), np.nan, dtype=torch.float64, device="cuda")
            g.apply(dev(U), dev(v), y)
            assert rel(host(R), Rref) < TOL64 and rel(host(y), Jv) < TOL64, zrun
        g.set_option(iga.IGA_OPT_RES_ZRUN, 0)
    g.set_option(iga.IGA_OPT_JAC_ALGO, iga.IGA_JAC_AUTO)
    vals = torch.zeros(g.nnz, dtype=torch.float64, device="cuda")
    g.assemble_jacobian(dev(U), vals)
    y2 = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    g.spmv(vals, dev(v), y2)
    assert rel(host(y2), Jv) < TOL64


@pytest.mark.parametrize("p,nel,cont", [(1, [6, 7, 5], 0), (2, [9, 5, 6], 1), (2, [5, 4, 3], 1), (3, [12, 4, 5], 2),
                                        (3, [7, 6, 5], 2), (4, [10, 3, 4], 3), (4, [9, 4, 3], 3), (3, [8, 5, 4], 0)])
def test_periodic_axis0_separable_jacobian(p, nel, cont):
    """A periodic axis 0 with C^(p-1) across the seam on the separable row-gather (x = xi, kappa one,
    axes 1 and 2 open): warm-up columns from the far end of the axis, rows at the seam listed in sorted
    column order.  FP64 against the oracle at 1e-12 and FP32 at 1e-5, for every segment count along axis 0
    (values identical to the unsplit pencils); the kernel that ran is the separable one, and a lower
    continuity across the seam (more functions than elements) takes the element path (atomic adds, so
    only the oracle's bar applies)."""
    print(f"[case] periodic axis-0 separable jacobian p={p} nel={nel} C^{cont}", flush=True)
    patch = inputs.unit_box(3, nel, p)
    per = [cont, None, None]
    o = oracle.Oracle(patch.knots, patch.degree, lam=2.0, periodic=per)
    g = iga.IGA(patch.knots, patch.degree, lam=2.0, periodic=per)
    U = inputs.uniform(13, 1, o.N, 0.0, 0.3)
    ref = o.jacobian(U)
    g.set_option(iga.IGA_OPT_KERNEL_TIMING, 1)
    base = None
    for nseg in (0, 1, 2, 3, nel[0]):
        g.set_option(iga.IGA_OPT_ROW_SEGMENTS, nseg)
        vals = torch.full((g.nnz,), np.nan, dtype=torch.float64, device="cuda")
        g.assemble_jacobian(dev(U), vals)
        got = host(vals)
        assert np.all(np.isfinite(got)), nseg
        assert rel(got, ref) < TOL64, nseg
        if base is None:
            base = got
        # the row-gather writes each value once in a fixed order; the element path adds atomically
        assert np.array_equal(got, base) or cont != p - 1, nseg
    assert any(name.startswith("k_rgsep3") for name, _ in g.kernel_times()) == (cont == p - 1)
    v32 = torch.full((g.nnz,), np.nan, dtype=torch.float32, device="cuda")
    g.assemble_jacobian(dev(U), v32, iga.IGA_FP32)
    assert rel(host(v32), ref) < 1e-5


@pytest.mark.parametrize("name", ["per2_p2_c1_x", "per2_p3_c0_x_kel", "per3_p2_xz", "per3_p3_c2_x"])
@pytest.mark.parametrize("mf", [False, True])
def test_periodic_newton_matches_oracle(name, mf):
    print(f"[case] periodic newton {name} matrix_free={mf}", flush=True)
    o, g, _ = build(name)
    U0 = np.zeros(o.N)
    ref, _, rc = o.newton(U0, atol=1e-13)
    assert rc == 0
    Ug = dev(U0)
    rep = g.newton_solve(Ug, atol=1e-11, matrix_free=mf)
    assert rep["converged"]
    assert rel(host(Ug), ref) < 1e-9


def test_periodic_fast_diagonalisation_preconditioner():
    """With a Dirichlet axis left, the 1D eigendecompositions of the periodic axes (wrapped band
    matrices) give the fast-diagonalisation preconditioner: same solution, far fewer CG steps."""
    o, g, _ = build("per3_p3_c2_x")
    ref, _, rc = o.newton(np.zeros(o.N), atol=1e-13)
    its = {}
    for pc in (iga.IGA_PRECOND_JACOBI, iga.IGA_PRECOND_FDM):
        g.set_option(iga.IGA_OPT_PRECOND, pc)
        Ug = dev(np.zeros(o.N))
        rep = g.newton_solve(Ug, atol=1e-11)
        assert rep["converged"] and rel(host(Ug), ref) < 1e-9
        its[pc] = rep["krylov_iters_total"]
    assert its[iga.IGA_PRECOND_FDM] < 0.5 * its[iga.IGA_PRECOND_JACOBI], its
    # fully periodic, no Dirichlet face: the stiffness has a kernel, the preconditioner is refused
    _, gf, _ = build("per2_p2_full")
    with pytest.raises(iga.IGAError) as e:
        gf.set_option(iga.IGA_OPT_PRECOND, iga.IGA_PRECOND_FDM)
    assert e.value.status == iga.IGA_EUNSUPPORTED


def test_periodic_rejections():
    patch = inputs.unit_box(2, [9, 7], 2)
    with pytest.raises(iga.IGAError) as e:       # a Dirichlet face on a periodic axis
        iga.IGA(patch.knots, patch.degree, periodic=[1, None], dirichlet_mask=0b1111)
    assert e.value.status == iga.IGA_EINVAL
    with pytest.raises(iga.IGAError) as e:       # too few functions left after wrapping
        small = inputs.unit_box(2, [3, 7], 2)
        iga.IGA(small.knots, small.degree, periodic=[1, None])
    assert e.value.status == iga.IGA_EINVAL
    g = iga.IGA(patch.knots, patch.degree, periodic=[1, None])
    g.set_option(iga.IGA_OPT_JAC_ALGO, iga.IGA_JAC_COLOR)
    vals = torch.zeros(g.nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IGAError) as e:
        g.assemble_jacobian(dev(np.zeros(g.N)), vals)
    assert e.value.status == iga.IGA_EUNSUPPORTED
