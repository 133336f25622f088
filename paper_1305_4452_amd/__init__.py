"""MI355X isogeometric assembly and Newton-Krylov library: Python binding of libiga.so.

The binding only marshals arguments: every step of assembly, apply and solve runs in the HIP
kernels of libiga.so.  PyTorch supplies device memory and the stream.  Importing works without
a GPU (so the ABI can be inspected), but every call that computes needs the built library and a
GPU, and fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiga.so")

IGA_OK, IGA_EINVAL, IGA_ENOMEM, IGA_EHIP, IGA_ENOCONV, IGA_EUNSUPPORTED, IGA_ESTATE = range(7)
IGA_FP64, IGA_FP32, IGA_BF16, IGA_BF16X3 = 0, 1, 2, 3
IGA_KAPPA_ONE, IGA_KAPPA_NODAL, IGA_KAPPA_ELEMENT = 0, 1, 2
IGA_JAC_AUTO, IGA_JAC_ROWGATHER, IGA_JAC_ATOMIC, IGA_JAC_COLOR, IGA_JAC_ROWGATHER_GENERAL, IGA_JAC_LOCAL_ND = 0, 1, 2, 3, 4, 5
IGA_OPT_JAC_ALGO, IGA_OPT_ROW_BLOCK, IGA_OPT_LAMBDA_BITS, IGA_OPT_ROW_SEGMENTS, IGA_OPT_KERNEL_TIMING = 1, 2, 3, 4, 5
IGA_OPT_PRECOND = 6
IGA_OPT_ND_SCATTER = 7
IGA_OPT_TILED_3D = 8
IGA_OPT_RES_ZRUN = 9
IGA_OPT_FDM_KERNEL = 10
IGA_PRECOND_AUTO, IGA_PRECOND_JACOBI, IGA_PRECOND_FDM = 0, 1, 2

_STATUS = {0: "IGA_OK", 1: "IGA_EINVAL", 2: "IGA_ENOMEM", 3: "IGA_EHIP", 4: "IGA_ENOCONV",
           5: "IGA_EUNSUPPORTED", 6: "IGA_ESTATE"}

_dp = C.POINTER(C.c_double)


class iga_desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("degree", C.c_int * 3),
        ("nknots", C.c_int * 3),
        ("knots", _dp * 3),
        ("ctrl", _dp),
        ("weights", _dp),
        ("nquad", C.c_int * 3),
        ("lam", C.c_double),
        ("kappa_mode", C.c_int),
        ("kappa", _dp),
        ("source", _dp),
        ("dirichlet_mask", C.c_uint),
        ("periodic", C.c_int * 3),
    ]


class iga_newton_opts(C.Structure):
    _fields_ = [
        ("atol", C.c_double),
        ("rtol", C.c_double),
        ("max_newton", C.c_int),
        ("max_krylov", C.c_int),
        ("matrix_free", C.c_int),
        ("jac_prec", C.c_int),
        ("forcing_max", C.c_double),
        ("check_every", C.c_int),
    ]


class iga_newton_report(C.Structure):
    _fields_ = [
        ("converged", C.c_int),
        ("newton_iters", C.c_int),
        ("krylov_iters_total", C.c_int),
        ("res_norm0", C.c_double),
        ("res_norm", C.c_double),
        ("hist", C.c_double * 65),
        ("krylov_iters", C.c_int * 64),
        ("t_total_ms", C.c_double),
        ("t_residual_ms", C.c_double),
        ("t_jacobian_ms", C.c_double),
        ("t_krylov_ms", C.c_double),
    ]

    def as_dict(self):
        k = self.newton_iters
        return dict(converged=bool(self.converged), newton_iters=k, krylov_iters_total=self.krylov_iters_total,
                    res_norm0=self.res_norm0, res_norm=self.res_norm, hist=list(self.hist[:k + 1]),
                    krylov_iters=list(self.krylov_iters[:k]), t_total_ms=self.t_total_ms,
                    t_residual_ms=self.t_residual_ms, t_jacobian_ms=self.t_jacobian_ms,
                    t_krylov_ms=self.t_krylov_ms)


class iga_batch_item_report(C.Structure):
    _fields_ = [
        ("converged", C.c_int),
        ("newton_iters", C.c_int),
        ("krylov_iters", C.c_int),
        ("res_norm0", C.c_double),
        ("res_norm", C.c_double),
    ]


class iga_batch_report(C.Structure):
    _fields_ = [
        ("all_converged", C.c_int),
        ("newton_steps", C.c_int),
        ("graph_launches", C.c_int),
        ("krylov_iters_max", C.c_int),
        ("t_total_ms", C.c_double),
        ("t_residual_ms", C.c_double),
        ("t_jacobian_ms", C.c_double),
        ("t_krylov_ms", C.c_double),
        ("t_tune_ms", C.c_double),
    ]


# name -> (argtypes, restype): mirrors include/iga.h
_SIGNATURES = {
    "iga_create": ([C.POINTER(iga_desc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "iga_destroy": ([C.c_void_p], C.c_int),
    "iga_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "iga_set_option": ([C.c_void_p, C.c_int, C.c_int64], C.c_int),
    "iga_csr_pattern": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "iga_assemble_residual": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "iga_biharmonic_residual": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "iga_cahn_hilliard_residual": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p], C.c_int),
    "iga_ch_gen_alpha_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                               C.POINTER(iga_newton_opts), C.c_void_p, C.c_void_p, C.POINTER(iga_newton_report)], C.c_int),
    "iga_gen_alpha_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.POINTER(iga_newton_opts),
                            C.c_void_p, C.c_void_p, C.POINTER(iga_newton_report)], C.c_int),
    "iga_assemble_jacobian": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "iga_grad_laplacian_residual": ([C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "iga_assemble_jacobian_noalloc": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int], C.c_int),
    "iga_apply": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p], C.c_int),
    "iga_spmv": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p], C.c_int),
    "iga_newton_solve": ([C.c_void_p, C.c_void_p, C.POINTER(iga_newton_opts), C.POINTER(iga_newton_report)],
                         C.c_int),
    "iga_element_matrices": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_int32), C.c_int, C.c_int, _dp], C.c_int),
    "iga_kernel_times": ([C.c_void_p, C.c_int, _dp, C.POINTER(C.c_char_p), C.POINTER(C.c_int)], C.c_int),
    "iga_batch_create": ([C.c_int, C.POINTER(iga_desc), C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "iga_batch_info": ([C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "iga_batch_newton_solve": ([C.c_void_p, C.c_void_p, C.POINTER(iga_newton_opts), C.POINTER(iga_batch_item_report),
                                C.POINTER(iga_batch_report)], C.c_int),
    "iga_batch_set_option": ([C.c_void_p, C.c_int, C.c_int64], C.c_int),
    "iga_batch_error_estimates": ([C.c_void_p, C.c_void_p, C.POINTER(C.c_double)], C.c_int),
    "iga_batch_destroy": ([C.c_void_p], C.c_int),
    "igann_num_params": ([], C.c_int64),
    "igann_create": ([C.c_int, C.c_void_p, C.POINTER(C.c_void_p)], C.c_int),
    "igann_set_weights": ([C.c_void_p, C.POINTER(C.c_float), C.c_int64], C.c_int),
    "igann_get_weights": ([C.c_void_p, C.POINTER(C.c_float), C.c_int64], C.c_int),
    "igann_forward": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p], C.c_int),
    "igann_set_loss": ([C.c_void_p, C.c_float], C.c_int),
    "igann_postprocess": ([C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_float, C.c_void_p, C.c_int], C.c_int),
    "igann_gradients": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_float)],
                        C.c_int),
    "igann_train_step": ([C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_float, C.POINTER(C.c_float)], C.c_int),
    "igann_destroy": ([C.c_void_p], C.c_int),
    "iga_last_error": ([], C.c_char_p),
}

_lib = None


class IGAError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


def load():
    """Load libiga.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_1305_4452_amd.build` first")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGNATURES)


def _check(st, where):
    if st != IGA_OK:
        msg = load().iga_last_error()
        raise IGAError(st, where, msg.decode() if msg else "")


def _dev_ptr(t, dtype, n, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


def make_desc(keep, knots, degree, ctrl=None, weights=None, lam=1.0, kappa_mode=IGA_KAPPA_ONE, kappa=None,
              source=None, dirichlet_mask=None, d=None, periodic=None):
    """Fill an iga_desc; the numpy arrays backing its pointers are appended to `keep`.  periodic:
    per axis None (open) or the continuity k across the seam; the default Dirichlet mask then
    leaves the periodic axes' faces free."""
    dim = len(knots)

    def arr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data_as(_dp)

    if d is None:
        d = iga_desc()
    d.dim = dim
    for a in range(dim):
        d.degree[a] = int(degree[a])
        k = np.ascontiguousarray(knots[a], dtype=np.float64)
        keep.append(k)
        d.nknots[a] = len(k)
        d.knots[a] = k.ctypes.data_as(_dp)
        d.nquad[a] = 0
    d.ctrl = arr(ctrl)
    d.weights = arr(weights)
    d.lam = float(lam)
    d.kappa_mode = int(kappa_mode)
    d.kappa = arr(kappa)
    d.source = arr(source)
    per = [None] * 3 if periodic is None else list(periodic) + [None] * (3 - len(periodic))
    for a in range(3):
        d.periodic[a] = 0 if per[a] is None else int(per[a]) + 1
    if dirichlet_mask is None:
        dirichlet_mask = sum(3 << (2 * a) for a in range(dim) if per[a] is None)
    d.dirichlet_mask = int(dirichlet_mask)
    return d


class IGA:
    """One problem (handle) bound to the current torch stream at creation."""

    def __init__(self, knots, degree, ctrl=None, weights=None, lam=1.0, kappa_mode=IGA_KAPPA_ONE, kappa=None,
                 source=None, dirichlet_mask=None, stream=None, periodic=None):
        import torch
        L = load()
        dim = len(knots)
        self._keep = []
        d = make_desc(self._keep, knots, degree, ctrl, weights, lam, kappa_mode, kappa, source, dirichlet_mask,
                      periodic=periodic)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(L.iga_create(C.byref(d), C.c_void_p(stream.cuda_stream), C.byref(h)), "iga_create")
        self.h = h
        N, nnz, E = C.c_int64(), C.c_int64(), C.c_int64()
        _check(L.iga_info(h, C.byref(N), C.byref(nnz), C.byref(E)), "iga_info")
        self.N, self.nnz, self.E = N.value, nnz.value, E.value
        self.dim = dim
        self.p = int(degree[0])
        self._keep = []

    @classmethod
    def from_workload(cls, w, **kw):
        p = w.patch
        args = dict(lam=w.lam, kappa_mode=w.kappa_mode, kappa=w.kappa)
        args.update(kw)
        return cls(p.knots, p.degree, p.ctrl, p.weights, **args)

    def close(self):
        if getattr(self, "h", None):
            load().iga_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- calls -----------------------------------------------------------------------------
    def set_option(self, key, value):
        _check(load().iga_set_option(self.h, int(key), int(value)), "iga_set_option")

    def set_lambda(self, lam):
        bits = int(np.array([lam], dtype=np.float64).view(np.int64)[0])
        self.set_option(IGA_OPT_LAMBDA_BITS, bits)

    def csr_pattern(self, row_ptr=None, col_idx=None):
        import torch
        if row_ptr is None:
            row_ptr = torch.empty(self.N + 1, dtype=torch.int64, device="cuda")
            col_idx = torch.empty(self.nnz, dtype=torch.int32, device="cuda")
        _check(load().iga_csr_pattern(self.h, _dev_ptr(row_ptr, torch.int64, self.N + 1, "row_ptr"),
                                      _dev_ptr(col_idx, torch.int32, self.nnz, "col_idx")), "iga_csr_pattern")
        return row_ptr, col_idx

    def assemble_residual(self, U, R):
        import torch
        _check(load().iga_assemble_residual(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                            _dev_ptr(R, torch.float64, self.N, "R")), "iga_assemble_residual")
        return R

    def gen_alpha_step(self, U0, V0, dt, rho_inf, U1, V1, atol=1e-10, max_newton=30, max_krylov=5000):
        """One generalized-alpha step of M0 Udot + R(U) = 0 (iga_gen_alpha_step); returns the report."""
        import torch
        o = iga_newton_opts(atol, 0.0, max_newton, max_krylov, 0, IGA_FP64, 1e-2, 0)
        rep = iga_newton_report()
        _check(load().iga_gen_alpha_step(self.h, _dev_ptr(U0, torch.float64, self.N, "U0"),
                                         _dev_ptr(V0, torch.float64, self.N, "V0"), float(dt), float(rho_inf),
                                         C.byref(o), _dev_ptr(U1, torch.float64, self.N, "U1"),
                                         _dev_ptr(V1, torch.float64, self.N, "V1"), C.byref(rep)), "iga_gen_alpha_step")
        return dict(converged=bool(rep.converged), newton_iters=rep.newton_iters,
                    krylov_iters_total=rep.krylov_iters_total, res_norm=rep.res_norm)

    def ch_gen_alpha_step(self, C0, V0, dt, rho_inf, theta, lam, C1, V1, atol=1e-10, max_newton=30, max_krylov=2000):
        """One generalized-alpha step of the Cahn-Hilliard system (iga_ch_gen_alpha_step); returns the report."""
        import torch
        o = iga_newton_opts(atol, 0.0, max_newton, max_krylov, 0, IGA_FP64, 1e-2, 0)
        rep = iga_newton_report()
        _check(load().iga_ch_gen_alpha_step(self.h, _dev_ptr(C0, torch.float64, self.N, "C0"),
                                            _dev_ptr(V0, torch.float64, self.N, "V0"), float(dt), float(rho_inf),
                                            float(theta), float(lam), C.byref(o),
                                            _dev_ptr(C1, torch.float64, self.N, "C1"),
                                            _dev_ptr(V1, torch.float64, self.N, "V1"), C.byref(rep)),
               "iga_ch_gen_alpha_step")
        return dict(converged=bool(rep.converged), newton_iters=rep.newton_iters,
                    krylov_iters_total=rep.krylov_iters_total, res_norm=rep.res_norm)

    def cahn_hilliard_residual(self, Cv, Cd, theta, lam, R):
        """Cahn-Hilliard residual for coefficients Cv of c and Cd of its rate (iga_cahn_hilliard_residual)."""
        import torch
        _check(load().iga_cahn_hilliard_residual(self.h, _dev_ptr(Cv, torch.float64, self.N, "C"),
                                                 _dev_ptr(Cd, torch.float64, self.N, "Cdot"), float(theta), float(lam),
                                                 _dev_ptr(R, torch.float64, self.N, "R")), "iga_cahn_hilliard_residual")
        return R

    def grad_laplacian_residual(self, U, R):
        """R_A = sum W grad N_A . grad(Lap u_h) over every function (iga_grad_laplacian_residual)."""
        import torch
        _check(load().iga_grad_laplacian_residual(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                                  _dev_ptr(R, torch.float64, self.N, "R")),
               "iga_grad_laplacian_residual")
        return R

    def biharmonic_residual(self, U, R):
        """R_A = sum W (Lap N_A)(Lap u_h) over every function (iga_biharmonic_residual)."""
        import torch
        _check(load().iga_biharmonic_residual(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                              _dev_ptr(R, torch.float64, self.N, "R")), "iga_biharmonic_residual")
        return R

    def assemble_jacobian(self, U, vals, prec=IGA_FP64):
        import torch
        vt = torch.float64 if prec == IGA_FP64 else torch.float32
        _check(load().iga_assemble_jacobian(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                            _dev_ptr(vals, vt, self.nnz, "vals"), int(prec)),
               "iga_assemble_jacobian")
        return vals

    def assemble_jacobian_noalloc(self, U, vals, prec=IGA_FP64):
        """iga_assemble_jacobian_noalloc: the same values without any allocation (static scratch)."""
        import torch
        vt = torch.float64 if prec == IGA_FP64 else torch.float32
        _check(load().iga_assemble_jacobian_noalloc(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                                    _dev_ptr(vals, vt, self.nnz, "vals"), int(prec)),
               "iga_assemble_jacobian_noalloc")
        return vals

    def apply(self, U, v, y):
        import torch
        _check(load().iga_apply(self.h, _dev_ptr(U, torch.float64, self.N, "U"), _dev_ptr(v, torch.float64, self.N, "v"),
                                _dev_ptr(y, torch.float64, self.N, "y")), "iga_apply")
        return y

    def spmv(self, vals, x, y, prec=IGA_FP64):
        import torch
        vt = torch.float64 if prec == IGA_FP64 else torch.float32
        _check(load().iga_spmv(self.h, _dev_ptr(vals, vt, self.nnz, "vals"), int(prec),
                               _dev_ptr(x, torch.float64, self.N, "x"), _dev_ptr(y, torch.float64, self.N, "y")),
               "iga_spmv")
        return y

    def newton_solve(self, U, atol=1e-10, rtol=0.0, max_newton=30, max_krylov=5000, matrix_free=False,
                     jac_prec=IGA_FP64, forcing_max=1e-2, check_every=0, raise_on_fail=True):
        import torch
        o = iga_newton_opts(atol, rtol, max_newton, max_krylov, int(matrix_free), int(jac_prec), forcing_max,
                            check_every)
        rep = iga_newton_report()
        st = load().iga_newton_solve(self.h, _dev_ptr(U, torch.float64, self.N, "U"), C.byref(o), C.byref(rep))
        if raise_on_fail:
            _check(st, "iga_newton_solve")
        out = rep.as_dict()
        out["status"] = st
        return out

    def kernel_times(self):
        """[(kernel name, ms)] of the last Jacobian assembly made with IGA_OPT_KERNEL_TIMING = 1."""
        ms = (C.c_double * 8)()
        names = (C.c_char_p * 8)()
        n = C.c_int(0)
        _check(load().iga_kernel_times(self.h, 8, ms, names, C.byref(n)), "iga_kernel_times")
        return [(names[i].decode(), ms[i]) for i in range(min(n.value, 8))]

    def element_matrices(self, U, elems, prec=IGA_FP64):
        import torch
        elems = np.ascontiguousarray(elems, dtype=np.int32)
        nloc = (self.p + 1) ** self.dim
        out = np.zeros((len(elems), nloc, nloc))
        _check(load().iga_element_matrices(self.h, _dev_ptr(U, torch.float64, self.N, "U"),
                                           elems.ctypes.data_as(C.POINTER(C.c_int32)), len(elems), int(prec),
                                           out.ctypes.data_as(_dp)), "iga_element_matrices")
        return out


class IGABatch:
    """Many independent 2D problems solved together (iga_batch_*)."""

    def __init__(self, workloads, stream=None):
        import torch
        L = load()
        self.n = len(workloads)
        keep = []
        descs = (iga_desc * self.n)()
        for i, w in enumerate(workloads):
            p = w.patch
            make_desc(keep, p.knots, p.degree, p.ctrl, p.weights, w.lam, w.kappa_mode, w.kappa, None, None, descs[i])
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        _check(L.iga_batch_create(self.n, descs, C.c_void_p(stream.cuda_stream), C.byref(h)), "iga_batch_create")
        self.h = h
        tot, nnz = C.c_int64(), C.c_int64()
        offs = (C.c_int64 * (self.n + 1))()
        _check(L.iga_batch_info(h, C.byref(tot), C.byref(nnz), offs), "iga_batch_info")
        self.N, self.nnz = tot.value, nnz.value
        self.offsets = np.array(offs[:], dtype=np.int64)

    def close(self):
        if getattr(self, "h", None):
            load().iga_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, arrays):
        out = np.zeros(self.N)
        for i, a in enumerate(arrays):
            out[self.offsets[i]:self.offsets[i + 1]] = a
        return out

    def unpack(self, x):
        x = np.asarray(x)
        return [x[self.offsets[i]:self.offsets[i + 1]] for i in range(self.n)]

    def set_option(self, key, value):
        _check(load().iga_batch_set_option(self.h, int(key), int(value)), "iga_batch_set_option")

    def error_estimates(self, U):
        """Per instance ||P^{-1} R(U)||_2 (iga_batch_error_estimates): the first Newton correction as the
        fast-diagonalisation preconditioner approximates it."""
        import torch
        est = (C.c_double * self.n)()
        _check(load().iga_batch_error_estimates(self.h, _dev_ptr(U, torch.float64, self.N, "U"), est),
               "iga_batch_error_estimates")
        return np.array(est[:], dtype=np.float64)

    def newton_solve(self, U, atol=1e-10, rtol=0.0, max_newton=30, max_krylov=5000, jac_prec=IGA_FP64,
                     forcing_max=1e-2, raise_on_fail=True, check_every=0):
        import torch
        o = iga_newton_opts(atol, rtol, max_newton, max_krylov, 0, int(jac_prec), forcing_max, int(check_every))
        items = (iga_batch_item_report * self.n)()
        rep = iga_batch_report()
        st = load().iga_batch_newton_solve(self.h, _dev_ptr(U, torch.float64, self.N, "U"), C.byref(o), items,
                                           C.byref(rep))
        if raise_on_fail:
            _check(st, "iga_batch_newton_solve")
        per = [dict(converged=bool(it.converged), newton_iters=it.newton_iters, krylov_iters=it.krylov_iters,
                    res_norm0=it.res_norm0, res_norm=it.res_norm) for it in items]
        summary = {k: getattr(rep, k) for k, _ in iga_batch_report._fields_}
        summary["status"] = st
        return per, summary


class GuessNet:
    """Device network of the learned initial guess (igann_*)."""

    def __init__(self, batch_max=256, stream=None):
        import torch
        L = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.bmax = batch_max
        self.nparam = int(L.igann_num_params())
        h = C.c_void_p()
        _check(L.igann_create(int(batch_max), C.c_void_p(stream.cuda_stream), C.byref(h)), "igann_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            load().igann_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(load().igann_set_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), "igann_set_weights")

    def get_weights(self):
        w = np.zeros(self.nparam, dtype=np.float32)
        _check(load().igann_get_weights(self.h, w.ctypes.data_as(C.POINTER(C.c_float)), w.size), "igann_get_weights")
        return w

    def forward(self, x, y=None):
        import torch
        B = x.shape[0]
        if y is None:
            y = torch.empty((B, 65 * 65), dtype=torch.float32, device="cuda")
        _check(load().igann_forward(self.h, _dev_ptr(x, torch.float32, B * 2 * 32 * 32, "x"), B,
                                    _dev_ptr(y, torch.float32, B * 65 * 65, "y")), "igann_forward")
        return y

    def set_loss(self, laplacian_weight):
        _check(load().igann_set_loss(self.h, float(laplacian_weight)), "igann_set_loss")

    def postprocess(self, y, mean=None, scale=1.0, sample_scale=None, passes=0):
        import torch
        B = y.shape[0]
        mp = None if mean is None else _dev_ptr(mean, torch.float32, 65 * 65, "mean")
        sp = None if sample_scale is None else _dev_ptr(sample_scale, torch.float32, B, "sample_scale")
        _check(load().igann_postprocess(self.h, _dev_ptr(y, torch.float32, B * 65 * 65, "y"), B, mp, float(scale),
                                        sp, int(passes)), "igann_postprocess")
        return y

    def gradients(self, x, t):
        import torch
        B = x.shape[0]
        g = np.zeros(self.nparam, dtype=np.float32)
        loss = C.c_float()
        _check(load().igann_gradients(self.h, _dev_ptr(x, torch.float32, B * 2 * 32 * 32, "x"),
                                      _dev_ptr(t, torch.float32, B * 65 * 65, "t"), B, C.byref(loss),
                                      g.ctypes.data_as(C.POINTER(C.c_float))), "igann_gradients")
        return loss.value, g

    def train_step(self, x, t, lr, want_loss=True):
        import torch
        B = x.shape[0]
        loss = C.c_float()
        _check(load().igann_train_step(self.h, _dev_ptr(x, torch.float32, B * 2 * 32 * 32, "x"),
                                       _dev_ptr(t, torch.float32, B * 65 * 65, "t"), B, float(lr),
                                       C.byref(loss) if want_loss else None), "igann_train_step")
        return loss.value if want_loss else None
