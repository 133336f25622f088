"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the benchmark's
CPU-baseline leg, never by the library.  `build()` compiles oracle.c with gcc into
liboracle.so next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(opt: str = "-O2", out: str | None = None) -> str:
    """Compile oracle.c into `out` (default: liboracle.so next to this file).  `opt` is one string
    of gcc flags, e.g. "-O3 -march=native" for a timing copy built on the host that runs it."""
    src = os.path.join(_HERE, "oracle.c")
    out = out or os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", *opt.split(), "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def use_library(path: str) -> None:
    """Load the oracle from another build of the same source (e.g. a -O3 -march=native copy for
    timing); every Oracle call made afterwards goes through it."""
    global _lib, _LIB_PATH
    _LIB_PATH = path
    _lib = None
    lib()


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("degree", C.c_int * 3),
        ("nknots", C.c_int * 3),
        ("knots", C.POINTER(C.c_double) * 3),
        ("ctrl", C.POINTER(C.c_double)),
        ("weights", C.POINTER(C.c_double)),
        ("nquad", C.c_int * 3),
        ("lam", C.c_double),
        ("kappa_mode", C.c_int),
        ("kappa", C.POINTER(C.c_double)),
        ("source", C.POINTER(C.c_double)),
        ("dirichlet_mask", C.c_uint),
        ("periodic", C.c_int * 3),
    ]


_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER(Problem)
        sig = {
            "orc_gauss_legendre": [C.c_int, _dp, _dp],
            "orc_unclamp": [C.c_int, C.c_int, C.c_int, _dp],
            "orc_basis_1d": [C.c_int, _dp, C.c_int, C.c_int, C.c_double, _dp, _dp],
            "orc_stencil": [C.c_int, _dp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)],
            "orc_sizes": [P, _i64p, _i64p, _i64p],
            "orc_csr_pattern": [P, _i64p, _i32p],
            "orc_residual": [P, _dp, _dp],
            "orc_jacobian": [P, _dp, _i64p, _i32p, _dp],
            "orc_jacobian_nd": [P, _dp, _i64p, _i32p, C.c_double, _dp],
            "orc_residual_rows": [P, _dp, _i64p, C.c_int64, _dp],
            "orc_jacobian_rows": [P, _dp, _i64p, C.c_int64, _i64p, _i32p, _dp],
            "orc_element_matrix": [P, _dp, C.c_int64, _dp, _dp],
            "orc_jacobian_elements": [P, _dp, _i64p, C.c_int64, _i64p, _i32p, _dp],
            "orc_spmv": [C.c_int64, _i64p, _i32p, _dp, _dp, _dp],
            "orc_newton": [P, _dp, C.c_double, C.c_double, C.c_int, C.c_int, C.c_double, _dp,
                           C.POINTER(C.c_int)],
            "orc_qp_data": [P, _dp, _dp, _dp, _dp, _dp],
            "orc_load_vector": [P, _dp, _dp],
            "orc_mass_matrix": [P, _i64p, _i32p, _dp],
            "orc_basis_1d_d2": [C.c_int, _dp, C.c_int, C.c_int, C.c_double, _dp],
            "orc_basis_hessian": [P, C.c_int64, _dp, _i64p, _dp, _dp, _dp, _dp],
            "orc_basis_1d_d3": [C.c_int, _dp, C.c_int, C.c_int, C.c_double, _dp],
            "orc_basis_third": [P, C.c_int64, _dp, _i64p, _dp],
            "orc_grad_laplacian_residual": [P, _dp, _dp],
            "orc_biharmonic_residual": [P, _dp, _dp],
            "orc_gen_alpha_params": [C.c_double, _dp, _dp, _dp],
            "orc_cahn_hilliard_residual": [P, _dp, _dp, C.c_double, C.c_double, _dp],
            "orc_gen_alpha_step": [P, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int, _dp, _dp,
                                   C.POINTER(C.c_int)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.orc_nqp.argtypes = [P]
        L.orc_nqp.restype = C.c_int64
        _lib = L
    return _lib


def gen_alpha_params(rho):
    """(alpha_m, alpha_f, gamma) of generalized-alpha from the spectral radius at infinity."""
    am, af, g = C.c_double(), C.c_double(), C.c_double()
    if lib().orc_gen_alpha_params(float(rho), C.byref(am), C.byref(af), C.byref(g)):
        raise ValueError("rho must be in [0, 1]")
    return am.value, af.value, g.value


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


class Oracle:
    """Holds one problem description (knots, geometry, parameters) and keeps the numpy arrays
    that back its pointers alive."""

    def __init__(self, knots, degree, ctrl=None, weights=None, lam=1.0, kappa_mode=0, kappa=None,
                 source=None, dirichlet_mask=None, nquad=None, periodic=None):
        """periodic: per axis None (open) or the continuity k across the seam (Sec. 2.4); the
        default Dirichlet mask then leaves the periodic axes' faces free."""
        dim = len(knots)
        self.dim = dim
        self._keep = []
        pb = Problem()
        pb.dim = dim
        for d in range(dim):
            k = np.ascontiguousarray(knots[d], dtype=np.float64)
            self._keep.append(k)
            pb.degree[d] = int(degree[d])
            pb.nknots[d] = len(k)
            pb.knots[d] = _ptr(k)
            pb.nquad[d] = 0 if nquad is None else int(nquad[d])

        def keep(a):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dtype=np.float64)
            self._keep.append(a)
            return _ptr(a)

        pb.ctrl = keep(ctrl)
        pb.weights = keep(weights)
        pb.lam = float(lam)
        pb.kappa_mode = int(kappa_mode)
        pb.kappa = keep(kappa)
        pb.source = keep(source)
        per = [None] * 3 if periodic is None else list(periodic) + [None] * (3 - len(periodic))
        for d in range(3):
            pb.periodic[d] = 0 if per[d] is None else int(per[d]) + 1
        if dirichlet_mask is None:
            dirichlet_mask = sum(3 << (2 * d) for d in range(dim) if per[d] is None)
        pb.dirichlet_mask = int(dirichlet_mask)
        self.pb = pb
        N, E, nnz = C.c_int64(), C.c_int64(), C.c_int64()
        rc = lib().orc_sizes(C.byref(pb), C.byref(N), C.byref(E), C.byref(nnz))
        if rc:
            raise ValueError(f"oracle rejected the problem (code {rc})")
        self.N, self.E, self.nnz = N.value, E.value, nnz.value
        self._pattern = None

    @classmethod
    def from_workload(cls, w, **kw):
        p = w.patch
        args = dict(lam=w.lam, kappa_mode=w.kappa_mode, kappa=w.kappa)
        args.update(kw)
        return cls(p.knots, p.degree, p.ctrl, p.weights, **args)

    def _chk(self, rc, what):
        if rc:
            raise RuntimeError(f"oracle {what} failed (code {rc})")

    def pattern(self):
        if self._pattern is None:
            rp = np.zeros(self.N + 1, dtype=np.int64)
            ci = np.zeros(self.nnz, dtype=np.int32)
            self._chk(lib().orc_csr_pattern(C.byref(self.pb), _ptr(rp, _i64p), _ptr(ci, _i32p)), "pattern")
            self._pattern = (rp, ci)
        return self._pattern

    def basis_hessian(self, elem, t):
        """Local functions of element `elem` at local coordinates t in [-1,1]^dim: global indices,
        values, spatial gradients [nloc, 3], spatial Hessians [nloc, 3, 3] (eq:ddrational,
        eq:ddimap, eq:ddspatial) and the point x [3]."""
        nloc = int(np.prod([self.pb.degree[d] + 1 for d in range(self.dim)]))
        tt = np.zeros(3)
        tv = np.atleast_1d(np.asarray(t, dtype=np.float64))
        tt[:len(tv)] = tv
        A = np.zeros(nloc, dtype=np.int64)
        N = np.zeros(nloc)
        dN = np.zeros(nloc * 3)
        d2N = np.zeros(nloc * 9)
        x = np.zeros(3)
        self._chk(lib().orc_basis_hessian(C.byref(self.pb), int(elem), _ptr(tt), _ptr(A, _i64p), _ptr(N), _ptr(dN),
                                          _ptr(d2N), _ptr(x)), "basis_hessian")
        return A, N, dN.reshape(nloc, 3), d2N.reshape(nloc, 3, 3), x

    def basis_third(self, elem, t):
        """Spatial third derivatives [nloc, 3, 3, 3] of the local functions of element `elem` at local
        coordinates t (eq:dddrational, eq:dddimap, eq:dddspatial), with their global indices."""
        nloc = int(np.prod([self.pb.degree[d] + 1 for d in range(self.dim)]))
        tt = np.zeros(3)
        tv = np.atleast_1d(np.asarray(t, dtype=np.float64))
        tt[:len(tv)] = tv
        A = np.zeros(nloc, dtype=np.int64)
        d3N = np.zeros(nloc * 27)
        self._chk(lib().orc_basis_third(C.byref(self.pb), int(elem), _ptr(tt), _ptr(A, _i64p), _ptr(d3N)),
                  "basis_third")
        return A, d3N.reshape(nloc, 3, 3, 3)

    def grad_laplacian_residual(self, U):
        """R_A = sum_e sum_q W grad N_A . grad(Lap u_h) for every function (no boundary rows)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.zeros(self.N)
        self._chk(lib().orc_grad_laplacian_residual(C.byref(self.pb), _ptr(U), _ptr(R)), "grad_laplacian_residual")
        return R

    def biharmonic_residual(self, U):
        """R_A = sum_e sum_q W (Lap N_A)(Lap u_h) for every function (no boundary rows)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.zeros(self.N)
        self._chk(lib().orc_biharmonic_residual(C.byref(self.pb), _ptr(U), _ptr(R)), "biharmonic_residual")
        return R

    def cahn_hilliard_residual(self, Cv, Cd, theta, lam):
        """Cahn-Hilliard residual (primal weak form, D = 1) for coefficients C of c and Cdot of its rate."""
        Cv = np.ascontiguousarray(Cv, dtype=np.float64)
        Cd = np.ascontiguousarray(Cd, dtype=np.float64)
        R = np.zeros(self.N)
        self._chk(lib().orc_cahn_hilliard_residual(C.byref(self.pb), _ptr(Cv), _ptr(Cd), float(theta), float(lam),
                                                   _ptr(R)), "cahn_hilliard_residual")
        return R

    def ch_gen_alpha_step(self, C0, V0, dt, rho, theta, lam, atol=1e-12, maxit=30):
        """One generalized-alpha step (eq:ga) of the Cahn-Hilliard system R_CH(cdot, c) = 0: Newton on
        cdot_{n+1} from cdot_n with a dense Jacobian of G by central differences (columns), linear
        systems by LU; returns (C1, V1, Newton iterations).  Small problems only."""
        am, af, gm = gen_alpha_params(rho)
        C0 = np.asarray(C0, dtype=np.float64)
        V0 = np.asarray(V0, dtype=np.float64)
        V1 = V0.copy()

        def G(V):
            Ca = C0 + af * dt * (gm * V + (1.0 - gm) * V0)
            Va = V0 + am * (V - V0)
            return self.cahn_hilliard_residual(Ca, Va, theta, lam)

        for k in range(maxit + 1):
            g = G(V1)
            if np.linalg.norm(g) < atol:
                return C0 + dt * (gm * V1 + (1.0 - gm) * V0), V1, k
            if k == maxit:
                break
            J = np.empty((self.N, self.N))
            for j in range(self.N):
                h = 1e-6 * (1.0 + abs(V1[j]))
                e = np.zeros(self.N)
                e[j] = h
                J[:, j] = (G(V1 + e) - G(V1 - e)) / (2.0 * h)
            V1 = V1 - np.linalg.solve(J, g)
        raise RuntimeError("oracle Cahn-Hilliard generalized-alpha Newton did not converge")

    def gen_alpha_step(self, U0, V0, dt, rho, atol=1e-12, maxit=30):
        """One generalized-alpha step (eq:ga) of M0 Udot + R(U) = 0: returns (U1, V1, Newton iterations)."""
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        V0 = np.ascontiguousarray(V0, dtype=np.float64)
        U1, V1 = np.zeros(self.N), np.zeros(self.N)
        it = C.c_int(0)
        self._chk(lib().orc_gen_alpha_step(C.byref(self.pb), _ptr(U0), _ptr(V0), float(dt), float(rho), float(atol),
                                           int(maxit), _ptr(U1), _ptr(V1), C.byref(it)), "gen_alpha_step")
        return U1, V1, it.value

    def residual(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.zeros(self.N)
        self._chk(lib().orc_residual(C.byref(self.pb), _ptr(U), _ptr(R)), "residual")
        return R

    def jacobian(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        rp, ci = self.pattern()
        v = np.zeros(self.nnz)
        self._chk(lib().orc_jacobian(C.byref(self.pb), _ptr(U), _ptr(rp, _i64p), _ptr(ci, _i32p), _ptr(v)),
                  "jacobian")
        return v

    def jacobian_nd(self, U, eta=0.0):
        """Local numerical-differentiation Jacobian (Sec. 2.8, eq:fdjac), CSR values; eta <= 0
        selects the default step factor sqrt(machine epsilon)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        rp, ci = self.pattern()
        v = np.zeros(self.nnz)
        self._chk(lib().orc_jacobian_nd(C.byref(self.pb), _ptr(U), _ptr(rp, _i64p), _ptr(ci, _i32p), float(eta),
                                        _ptr(v)), "jacobian_nd")
        return v

    def jacobian_csr(self, U):
        import scipy.sparse as sp
        rp, ci = self.pattern()
        return sp.csr_matrix((self.jacobian(U), ci, rp), shape=(self.N, self.N))

    def residual_rows(self, U, rows):
        U = np.ascontiguousarray(U, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(len(rows))
        self._chk(lib().orc_residual_rows(C.byref(self.pb), _ptr(U), _ptr(rows, _i64p), len(rows), _ptr(out)),
                  "residual_rows")
        return out

    def jacobian_rows(self, U, rows, row_ptr=None, col_idx=None):
        """Values of the listed rows, concatenated in CSR order (pattern rows may be passed in
        to avoid building the whole pattern for large problems)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        if row_ptr is None:
            row_ptr, col_idx = self.pattern()
        n = int(sum(row_ptr[r + 1] - row_ptr[r] for r in rows))
        out = np.zeros(n)
        self._chk(lib().orc_jacobian_rows(C.byref(self.pb), _ptr(U), _ptr(rows, _i64p), len(rows),
                                          _ptr(row_ptr, _i64p), _ptr(col_idx, _i32p), _ptr(out)),
                  "jacobian_rows")
        return out

    def element_matrix(self, U, e):
        U = np.ascontiguousarray(U, dtype=np.float64)
        nloc = int(np.prod([self.pb.degree[d] + 1 for d in range(self.dim)]))
        K = np.zeros(nloc * nloc)
        Rv = np.zeros(nloc)
        self._chk(lib().orc_element_matrix(C.byref(self.pb), _ptr(U), int(e), _ptr(K), _ptr(Rv)), "element")
        return K.reshape(nloc, nloc), Rv

    def jacobian_elements(self, U, elems, vals):
        U = np.ascontiguousarray(U, dtype=np.float64)
        elems = np.ascontiguousarray(elems, dtype=np.int64)
        rp, ci = self.pattern()
        self._chk(lib().orc_jacobian_elements(C.byref(self.pb), _ptr(U), _ptr(elems, _i64p), len(elems),
                                              _ptr(rp, _i64p), _ptr(ci, _i32p), _ptr(vals)), "jac_elems")
        return vals

    def newton(self, U0, atol=1e-10, rtol=0.0, maxit=50, linear_solver=0, cg_rtol=1e-13):
        U = np.array(U0, dtype=np.float64, copy=True)
        hist = np.zeros(maxit + 1)
        it = C.c_int()
        rc = lib().orc_newton(C.byref(self.pb), _ptr(U), atol, rtol, maxit, linear_solver, cg_rtol,
                              _ptr(hist), C.byref(it))
        return U, hist[:it.value + 1].copy(), rc

    def qp_data(self, U=None):
        nqp = lib().orc_nqp(C.byref(self.pb))
        x = np.zeros(nqp * self.dim)
        W = np.zeros(nqp)
        u = np.zeros(nqp)
        g = np.zeros(nqp * self.dim)
        Uc = None if U is None else np.ascontiguousarray(U, dtype=np.float64)
        self._chk(lib().orc_qp_data(C.byref(self.pb), _ptr(Uc), _ptr(x), _ptr(W), _ptr(u), _ptr(g)), "qp")
        return x.reshape(nqp, self.dim), W, u, g.reshape(nqp, self.dim)

    def load_vector(self, fq):
        fq = np.ascontiguousarray(fq, dtype=np.float64)
        b = np.zeros(self.N)
        self._chk(lib().orc_load_vector(C.byref(self.pb), _ptr(fq), _ptr(b)), "load")
        return b

    def mass_matrix(self):
        import scipy.sparse as sp
        rp, ci = self.pattern()
        v = np.zeros(self.nnz)
        self._chk(lib().orc_mass_matrix(C.byref(self.pb), _ptr(rp, _i64p), _ptr(ci, _i32p), _ptr(v)), "mass")
        return sp.csr_matrix((v, ci, rp), shape=(self.N, self.N))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(n, _ptr(x), _ptr(w)):
        raise ValueError("bad n")
    return x, w


def basis_1d(p, U, i, xi):
    U = np.ascontiguousarray(U, dtype=np.float64)
    v, d = C.c_double(), C.c_double()
    if lib().orc_basis_1d(p, _ptr(U), len(U), i, float(xi), C.byref(v), C.byref(d)):
        raise ValueError("bad basis index")
    return v.value, d.value


def basis_1d_d3(p, U, i, xi):
    U = np.ascontiguousarray(U, dtype=np.float64)
    d = C.c_double()
    if lib().orc_basis_1d_d3(p, _ptr(U), len(U), i, float(xi), C.byref(d)):
        raise ValueError("bad basis index")
    return d.value


def stencil(p, U, i):
    U = np.ascontiguousarray(U, dtype=np.float64)
    l, r = C.c_int(), C.c_int()
    if lib().orc_stencil(p, _ptr(U), len(U), i, C.byref(l), C.byref(r)):
        raise ValueError("bad index")
    return l.value, r.value


def unclamp(U, p, k):
    """Knot vector unclamped for C^k periodicity (Sec. 2.4, eq:unclamp-left/right)."""
    U = np.array(U, dtype=np.float64, copy=True)
    n = len(U) - p - 2
    if lib().orc_unclamp(n, p, k, _ptr(U)):
        raise ValueError("bad continuity")
    return U
