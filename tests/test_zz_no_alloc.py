"""The allocation-free Jacobian entry point (iga_assemble_jacobian_noalloc) against iga_assemble_jacobian
through the C ABI: the same kernels with the reaction field in the library's static per-GPU array, so
the values must be identical.  Two calls in a row on one GPU, the second on a smaller mesh (the array
keeps the first call's field), FP64 and FP32 values, a 2D problem (no scratch path), and the size
limit refused with IGA_EINVAL before any kernel runs."""
import pytest

import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1305_4452_amd as iga  # noqa: E402


def both(g, U, prec):
    dt = torch.float64 if prec == iga.IGA_FP64 else torch.float32
    ref = torch.full((g.nnz,), float("nan"), dtype=dt, device="cuda")
    out = torch.full((g.nnz,), float("nan"), dtype=dt, device="cuda")
    g.assemble_jacobian(U, ref, prec)
    g.assemble_jacobian_noalloc(U, out, prec)
    torch.cuda.synchronize()
    return ref, out


@pytest.mark.parametrize("prec", [iga.IGA_FP64, iga.IGA_FP32])
def test_noalloc_jacobian_matches_in_two_calls(prec):
    assert torch.cuda.is_available()
    for nel, seed in ((40, 21), (24, 22)):           # second call on a smaller mesh
        print(f"noalloc jacobian: 3D Bratu {nel}^3 p=3 prec={prec}", flush=True)
        w = inputs.config_3d_bratu(nel=nel)
        g = iga.IGA.from_workload(w)
        U = torch.as_tensor(inputs.uniform(seed, 0, g.N, 0.0, 0.1), device="cuda")
        ref, out = both(g, U, prec)
        assert not torch.isnan(ref).any()
        assert torch.equal(ref, out)
        g.close()


def test_noalloc_jacobian_fp32_at_the_limit():
    # 64^3 elements at p = 3: 16,777,216 quadrature points, exactly 64 MiB of FP32 field
    print("noalloc jacobian: 3D Bratu 64^3 p=3 FP32 (64 MiB field)", flush=True)
    w = inputs.config_3d_bratu(nel=64)
    g = iga.IGA.from_workload(w)
    U = torch.as_tensor(w.U0, device="cuda")
    ref, out = both(g, U, iga.IGA_FP32)
    assert torch.equal(ref, out)
    # FP64 needs twice the limit: refused before any launch, the values left as they were
    vals = torch.zeros(g.nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IGAError) as ei:
        g.assemble_jacobian_noalloc(U, vals, iga.IGA_FP64)
    assert "IGA_EINVAL" in str(ei.value) and "exceeds" in str(ei.value)
    torch.cuda.synchronize()
    assert float(vals.abs().max()) == 0.0
    g.close()


def test_noalloc_jacobian_2d_path():
    print("noalloc jacobian: 2D Bratu 16^2 p=2", flush=True)
    w = inputs.config_2d_small()
    g = iga.IGA.from_workload(w)
    U = torch.as_tensor(w.U0, device="cuda")
    ref, out = both(g, U, iga.IGA_FP64)
    assert torch.equal(ref, out)
    g.close()
