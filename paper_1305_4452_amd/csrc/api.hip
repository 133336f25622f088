// extern "C" entry points of libiga (declared in include/iga.h) and the Newton driver.
#include <chrono>
#include <cmath>
#include <cstring>

#include "iga_impl.h"

namespace iga {
iga_status create_impl(const iga_desc *d, void *stream, Handle **out);
iga_status launch_norm(Handle &h, const double *x, double *out_dev);
iga_status launch_diag_inv(Handle &h, const void *vals, int prec, double *dinv);
iga_status launch_axpy(Handle &h, double a, const double *x, double *y);
iga_status launch_dot(Handle &h, const double *x, const double *y, double *out_dev);
iga_status cg_solve(Handle &h, const double *R, double *d, double rtol, int maxit, int check_every,
                    const void *vals, int prec, bool matrix_free, bool fdm, int *iters_out, double *rel_out);

static iga_status alloc_owned(Handle &h, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(IGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h.owned.push_back(*p);
  return IGA_OK;
}

static void pick_block(const Handle &h, int prec, int *b1, int *b2) {
  if (h.row_b1 > 0 && rowgather_supported(h, prec, h.row_b1, h.row_b2 > 0 ? h.row_b2 : 1)) {
    *b1 = h.row_b1;
    *b2 = h.row_b2 > 0 ? h.row_b2 : 1;
    return;
  }
  if (h.pb.dim == 3) {
    // measured on the 48^3 quarter cylinder (table mode): p = 3 FP64 2x1 10.9 ms (2x2 16.4),
    // p = 4 FP64 1x1 33.4 ms (2x1 63.0), p = 4 FP32 2x1 21.4 ms (1x1 29.3)
    *b1 = 2;
    *b2 = (h.pb.P <= 4) ? 2 : 1;
    if (h.pb.table && h.pb.P == 4 && prec == IGA_FP64) *b2 = 1;
    if (h.pb.table && h.pb.P >= 5 && prec == IGA_FP64) *b1 = 1;
  } else {
    *b1 = h.pb.n[1] >= 256 ? 8 : 4;
    *b2 = 1;
  }
}

// Separable row-gather pencil block, from a sweep at 64^3 p = 3 on MI355X: 2x2 for FP64
// (0.52 ms; 4x4 0.58, 8x2 0.61, 4x2 0.63) and FP32 (0.34 ms; 4x4 0.37, 4x2 0.39).
static void pick_sep_block(const Handle &h, int *b1, int *b2) {
  if (h.row_b1 > 0 && rgsep_supported(h, h.row_b1, h.row_b2 > 0 ? h.row_b2 : 1)) {
    *b1 = h.row_b1;
    *b2 = h.row_b2 > 0 ? h.row_b2 : 1;
    return;
  }
  *b1 = 2;
  *b2 = 2;
}

// storage precision of the Jacobian values for a contraction precision (BF16 contractions write FP32)
static int value_prec(int prec) { return prec == IGA_FP64 ? IGA_FP64 : IGA_FP32; }

static iga_status assemble_jacobian(Handle &h, const double *U, void *vals, int prec) {
  if (prec == IGA_BF16 || prec == IGA_BF16X3) return launch_jac_mma(h, U, (float *)vals, prec == IGA_BF16X3);
  int algo = h.jac_algo;
  int b1 = 0, b2 = 0;
  if (algo == IGA_JAC_AUTO || algo == IGA_JAC_ROWGATHER) {
    int s1 = 0, s2 = 0;
    pick_sep_block(h, &s1, &s2);
    if (rgsep_supported(h, s1, s2)) return launch_jac_rgsep(h, U, vals, prec, s1, s2);
    if (rgt2_supported(h.pb) && h.row_b1 == 0) return launch_jac_rgt2(h, U, vals, prec);
  }
  pick_block(h, prec, &b1, &b2);
  if (algo == IGA_JAC_AUTO) algo = rowgather_supported(h, prec, b1, b2) ? IGA_JAC_ROWGATHER : IGA_JAC_ATOMIC;
  iga_status st;
  if (algo == IGA_JAC_ROWGATHER || algo == IGA_JAC_ROWGATHER_GENERAL) {
    kt_begin(h, "k_rowgather (general)");
    st = launch_jac_rowgather(h, U, vals, prec, b1, b2);
  } else if (algo == IGA_JAC_LOCAL_ND) {
    kt_begin(h, "k_elem_nd (local numerical differentiation)");
    // colours assume no function is shared across the ends of an axis
    st = launch_jac_nd(h, U, vals, prec, h.pb.periodic ? 0 : h.nd_color);
  } else if (algo == IGA_JAC_COLOR && h.pb.periodic) {
    return fail(IGA_EUNSUPPORTED, "colour scatter needs open axes (elements share functions across the seam)");
  } else if (algo == IGA_JAC_ATOMIC || algo == IGA_JAC_COLOR) {
    kt_begin(h, algo == IGA_JAC_ATOMIC ? "k_elem_mat (atomic scatter)" : "k_elem_mat (colour scatter)");
    st = launch_jac_scatter(h, U, vals, prec, algo == IGA_JAC_COLOR ? 1 : 0);
  } else {
    return fail(IGA_EINVAL, "unknown Jacobian algorithm");
  }
  kt_end(h);
  return st;
}

static iga_status ensure_newton_ws(Handle &h, bool need_vals, int prec) {
  iga_status st;
  const size_t N = (size_t)h.pb.N;
  if (!h.nw && (st = alloc_owned(h, (void **)&h.nw, 6 * N * sizeof(double)))) return st;
  if (!h.dinv && (st = alloc_owned(h, (void **)&h.dinv, N * sizeof(double)))) return st;
  if (!h.scal && (st = alloc_owned(h, (void **)&h.scal, 1100 * sizeof(double)))) return st;
  if (h.fdm.ok && !h.fdm_w && (st = alloc_owned(h, (void **)&h.fdm_w, 2 * N * sizeof(double)))) return st;
  if (need_vals && (h.jvals == nullptr || h.jvals_prec != prec)) {
    size_t bytes = (size_t)h.pb.nnz * (prec == IGA_FP64 ? 8 : 4);
    if (h.jvals) {
      for (auto &q : h.owned)
        if (q == h.jvals) q = nullptr;
      (void)hipFree(h.jvals);
      h.jvals = nullptr;
    }
    if ((st = alloc_owned(h, &h.jvals, bytes))) return st;
    h.jvals_prec = prec;
  }
  return IGA_OK;
}

static float ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0;
  return ms;
}

static iga_status newton(Handle &h, double *U, const iga_newton_opts *o_in, iga_newton_report *rep) {
  iga_newton_opts o{};
  o.atol = 1e-10;
  o.rtol = 0;
  o.max_newton = 30;
  o.max_krylov = 5000;
  o.matrix_free = 0;
  o.jac_prec = IGA_FP64;
  o.forcing_max = 1e-2;
  o.check_every = 0;
  if (o_in) o = *o_in;
  if (o.max_newton < 0 || o.max_newton > 64) return fail(IGA_EINVAL, "max_newton must be in 0..64");
  if (o.max_krylov < 1) return fail(IGA_EINVAL, "max_krylov must be positive");
  if (o.jac_prec != IGA_FP64 && o.jac_prec != IGA_FP32 && o.jac_prec != IGA_BF16 && o.jac_prec != IGA_BF16X3)
    return fail(IGA_EUNSUPPORTED, "Jacobian precision");
  if ((o.jac_prec == IGA_BF16 || o.jac_prec == IGA_BF16X3) && !o.matrix_free && !mma_supported(h.pb))
    return fail(IGA_EUNSUPPORTED, "BF16 Jacobians need the matrix-core row-gather (3D, open axes, simple knots, p 2..4)");
  const int vprec = value_prec(o.jac_prec);
  if (o.forcing_max <= 0) o.forcing_max = 1e-2;
  if (h.precond != IGA_PRECOND_JACOBI) {
    iga_status sf = ensure_fdm(h);
    if (sf) return sf;
  }
  const bool fdm = h.precond != IGA_PRECOND_JACOBI && h.fdm.ok;
  if (h.precond == IGA_PRECOND_FDM && !fdm)
    return fail(IGA_EUNSUPPORTED, "the FDM preconditioner needs at most 512 unknowns per axis");
  if (o.check_every <= 0) o.check_every = fdm ? 4 : 16;
  if (o.check_every > 1024) o.check_every = 1024;
  iga_newton_report r{};
  iga_status st = ensure_newton_ws(h, !o.matrix_free, vprec);
  if (st) return st;
  const int64_t N = h.pb.N;
  double *R = h.nw, *dvec = h.nw + N;
  auto t0 = std::chrono::steady_clock::now();
  hipEvent_t ev[4];
  for (auto &e : ev)
    if (hipEventCreate(&e) != hipSuccess) return fail(IGA_EHIP, "hipEventCreate");
  double nr = 0, nr_prev = 0, r0 = -1, eta = o.forcing_max;
  int k = 0;
  st = IGA_OK;
  for (k = 0;; ++k) {
    hipEventRecord(ev[0], h.stream);
    if ((st = launch_residual(h, U, R))) break;
    if ((st = launch_norm(h, R, h.scal))) break;
    if (hipMemcpyAsync(&nr, h.scal, sizeof(double), hipMemcpyDeviceToHost, h.stream) != hipSuccess ||
        hipEventRecord(ev[1], h.stream) != hipSuccess || hipStreamSynchronize(h.stream) != hipSuccess) {
      st = fail(IGA_EHIP, "residual norm");
      break;
    }
    r.t_residual_ms += ev_ms(ev[0], ev[1]);
    r.hist[k] = nr;
    if (r0 < 0) r0 = nr;
    if (!std::isfinite(nr)) { st = fail(IGA_ENOCONV, "residual is not finite"); break; }
    if (nr < o.atol || (o.rtol > 0 && nr <= o.rtol * r0)) { r.converged = 1; break; }
    if (k >= o.max_newton) { st = fail(IGA_ENOCONV, "Newton did not converge"); break; }
    // forcing term (Eisenstat-Walker, second choice) with a floor that avoids over-solving
    if (k > 0) {
      double ratio = nr / nr_prev;
      eta = fmin(o.forcing_max, 0.9 * ratio * ratio);
    }
    double target = fmax(o.atol, o.rtol * r0);
    eta = fmax(eta, 0.1 * target / nr);
    eta = fmin(eta, o.forcing_max);
    nr_prev = nr;
    hipEventRecord(ev[0], h.stream);
    if (o.matrix_free) {
      if ((st = launch_linearize(h, U))) break;
      if (!fdm && (st = launch_diag_mf(h, h.dinv))) break;
    } else {
      if ((st = assemble_jacobian(h, U, h.jvals, o.jac_prec))) break;
      if (!fdm && (st = launch_diag_inv(h, h.jvals, vprec, h.dinv))) break;
    }
    if (fdm && (st = launch_fdm_shift(h, U))) break;
    hipEventRecord(ev[1], h.stream);
    int its = 0;
    double rel = 0;
    if ((st = cg_solve(h, R, dvec, eta, o.max_krylov, o.check_every, h.jvals, vprec, o.matrix_free != 0, fdm,
                       &its, &rel)))
      break;
    hipEventRecord(ev[2], h.stream);
    if ((st = launch_axpy(h, 1.0, dvec, U))) break;
    if (hipStreamSynchronize(h.stream) != hipSuccess) { st = fail(IGA_EHIP, "sync"); break; }
    r.t_jacobian_ms += ev_ms(ev[0], ev[1]);
    r.t_krylov_ms += ev_ms(ev[1], ev[2]);
    r.krylov_iters[k] = its;
    r.krylov_iters_total += its;
  }
  for (auto &e : ev) hipEventDestroy(e);
  r.newton_iters = k;
  r.res_norm0 = r0;
  r.res_norm = nr;
  r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = r;
  return st;
}

// ------------------------------------------------------------------------------------------
// Generalized-alpha time stepping (eq:ga) of M0 Udot + R(U) = 0, R the residual of eq:residual
// (Dirichlet rows U_A) and M0 the mass matrix without Dirichlet rows and columns.
// ------------------------------------------------------------------------------------------
static unsigned ga_blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// U_{n+af} = U0 + c1 V1 + c0 V0, Udot_{n+am} = (1 - am) V0 + am V1
__global__ void k_ga_stage(int64_t n, const double *__restrict__ U0, const double *__restrict__ V0,
                           const double *__restrict__ V1, double c1, double c0, double am, double *__restrict__ Ua,
                           double *__restrict__ Va) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  Ua[i] = U0[i] + c1 * V1[i] + c0 * V0[i];
  Va[i] = (1.0 - am) * V0[i] + am * V1[i];
}

// y = a x + b y over n values
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

// M0 = J(0; lambda = -1) - J(0; lambda = 0): the reaction term -lambda W e^u N_A N_B at u = 0 and
// lambda = -1 is the mass matrix, the stiffness cancels, and the Dirichlet identity rows of the
// two Jacobians cancel too (their columns are zero in both)
static iga_status ensure_mass(Handle &h) {
  if (h.massv) return IGA_OK;
  const int64_t N = h.pb.N, nnz = h.pb.nnz;
  iga_status st;
  double *mv = nullptr;
  if ((st = alloc_owned(h, (void **)&mv, (size_t)nnz * sizeof(double)))) return st;
  if ((st = ensure_newton_ws(h, true, IGA_FP64))) return st;
  double *zero = h.nw + 2 * N;
  if ((st = launch_fill(h, zero, N, 0.0))) return st;
  const double lam = h.pb.lambda;
  h.pb.lambda = -1.0;
  st = assemble_jacobian(h, zero, mv, IGA_FP64);
  h.pb.lambda = 0.0;
  if (!st) st = assemble_jacobian(h, zero, h.jvals, IGA_FP64);
  h.pb.lambda = lam;
  if (st) return st;
  hipLaunchKernelGGL(k_axpby, dim3(ga_blocks(nnz)), dim3(256), 0, h.stream, nnz, -1.0, (const double *)h.jvals,
                     1.0, mv);
  IGA_HIP_CHECK(hipGetLastError());
  h.massv = mv;
  return IGA_OK;
}

static iga_status gen_alpha_step(Handle &h, const double *U0, const double *V0, double dt, double rho,
                                 const iga_newton_opts *o_in, double *U1, double *V1, iga_newton_report *rep) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(IGA_EINVAL, "dt must be positive");
  if (!(rho >= 0.0 && rho <= 1.0)) return fail(IGA_EINVAL, "rho_inf must be in [0, 1]");
  iga_newton_opts o{};
  o.atol = 1e-10;
  o.max_newton = 30;
  o.max_krylov = 5000;
  o.jac_prec = IGA_FP64;
  o.forcing_max = 1e-2;
  if (o_in) o = *o_in;
  if (o.matrix_free || o.jac_prec != IGA_FP64) return fail(IGA_EUNSUPPORTED, "generalized-alpha uses the assembled FP64 Jacobian");
  if (o.max_newton < 0 || o.max_newton > 64) return fail(IGA_EINVAL, "max_newton must be in 0..64");
  if (o.max_krylov < 1) return fail(IGA_EINVAL, "max_krylov must be positive");
  if (o.forcing_max <= 0) o.forcing_max = 1e-2;
  // parameters from the spectral radius at infinity (after eq:ga)
  const double am = 0.5 * (3.0 - rho) / (1.0 + rho), af = 1.0 / (1.0 + rho), gm = 0.5 + am - af;
  // fast diagonalisation of K + (am / (af gamma dt) - lambda mean(e^u)) M when it is built (the
  // step's operator divided by af gamma dt), Jacobi otherwise
  iga_status st = IGA_OK;
  if (h.precond != IGA_PRECOND_JACOBI && (st = ensure_fdm(h))) return st;
  const bool fdm = h.precond != IGA_PRECOND_JACOBI && h.fdm.ok;
  if ((st = ensure_mass(h)) || (st = ensure_newton_ws(h, true, IGA_FP64))) return st;
  const int64_t N = h.pb.N, nnz = h.pb.nnz;
  if (!h.gaw && (st = alloc_owned(h, (void **)&h.gaw, (size_t)3 * N * sizeof(double)))) return st;
  double *G = h.nw, *dvec = h.nw + N, *Ua = h.gaw, *Va = h.gaw + N, *MV = h.gaw + 2 * N;
  const unsigned nb = (unsigned)ga_blocks(N);
  iga_newton_report r{};
  auto t0 = std::chrono::steady_clock::now();
  // start from Udot_{n+1} = Udot_n
  IGA_HIP_CHECK(hipMemcpyAsync(V1, V0, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
  double nr = 0, r0 = -1;
  int k;
  for (k = 0;; ++k) {
    hipLaunchKernelGGL(k_ga_stage, dim3(nb), dim3(256), 0, h.stream, N, U0, V0, (const double *)V1, af * dt * gm,
                       af * dt * (1.0 - gm), am, Ua, Va);
    IGA_HIP_CHECK(hipGetLastError());
    if ((st = launch_residual(h, Ua, G))) break;
    if ((st = launch_spmv(h, h.massv, IGA_FP64, Va, MV, nullptr, h.npartials))) break;
    if ((st = launch_axpy(h, 1.0, MV, G))) break;
    if ((st = launch_norm(h, G, h.scal))) break;
    if (hipMemcpyAsync(&nr, h.scal, sizeof(double), hipMemcpyDeviceToHost, h.stream) != hipSuccess ||
        hipStreamSynchronize(h.stream) != hipSuccess) {
      st = fail(IGA_EHIP, "stage residual norm");
      break;
    }
    r.hist[k] = nr;
    if (r0 < 0) r0 = nr;
    if (!std::isfinite(nr)) { st = fail(IGA_ENOCONV, "stage residual is not finite"); break; }
    if (nr < o.atol || (o.rtol > 0 && nr <= o.rtol * r0)) { r.converged = 1; break; }
    if (k >= o.max_newton) { st = fail(IGA_ENOCONV, "generalized-alpha Newton did not converge"); break; }
    // dG/dUdot_{n+1} = am M0 + af gamma dt J(U_{n+af}) on the Jacobian's CSR pattern
    if ((st = assemble_jacobian(h, Ua, h.jvals, IGA_FP64))) break;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)ga_blocks(nnz)), dim3(256), 0, h.stream, nnz, am,
                       (const double *)h.massv, af * gm * dt, (double *)h.jvals);
    IGA_HIP_CHECK(hipGetLastError());
    if (fdm) {
      if ((st = launch_fdm_shift(h, Ua, am / (af * gm * dt)))) break;
    } else if ((st = launch_diag_inv(h, h.jvals, IGA_FP64, h.dinv))) {
      break;
    }
    const double eta = fmin(o.forcing_max, fmax(1e-12, 0.1 * o.atol / nr));
    int its = 0;
    double rel = 0;
    if ((st = cg_solve(h, G, dvec, eta, o.max_krylov, o.check_every > 0 ? o.check_every : (fdm ? 4 : 16), h.jvals,
                       IGA_FP64, false, fdm, &its, &rel)))
      break;
    if ((st = launch_axpy(h, 1.0, dvec, V1))) break;
    r.krylov_iters[k] = its;
    r.krylov_iters_total += its;
  }
  if (!st) {
    // U_{n+1} = U_n + dt (gamma Udot_{n+1} + (1 - gamma) Udot_n)
    IGA_HIP_CHECK(hipMemcpyAsync(U1, U0, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    if (!(st = launch_axpy(h, dt * gm, V1, U1))) st = launch_axpy(h, dt * (1.0 - gm), V0, U1);
    if (!st && hipStreamSynchronize(h.stream) != hipSuccess) st = fail(IGA_EHIP, "sync");
  }
  r.newton_iters = k;
  r.res_norm0 = r0;
  r.res_norm = nr;
  r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = r;
  return st;
}

// ------------------------------------------------------------------------------------------
// Generalized-alpha step of the Cahn-Hilliard system R_CH(cdot, c) = 0 (the Cahn-Hilliard residual
// is linear in cdot): Newton on cdot_{n+1}, each linear system solved by BiCGStab (the Jacobian is
// not symmetric) with Jacobian-vector products by a forward difference of the residual along the
// stage direction (the matrix-free approach of Sec. 2.8): J x ~ (G(V1 + eps x) - G(V1)) / eps with
// eps = sqrt(eps_machine) (1 + ||c_{n+af}||) / ||x||.
// ------------------------------------------------------------------------------------------

// BiCGStab scalars kept on the device, in the handle's scalar block: the residual norm, the count of
// iterations taken, rho = (rh, r) and the rest of the recurrence.  Every update kernel is a no-op once
// the residual norm is at or below tol, so the host reads the norm back only every few iterations.
enum { kRes = 8, kIts, kRho, kRhoOld, kAlpha, kOmega, kRhv, kTs, kTt, kYn, kSn };

__global__ void k_bcg_init(double *S, double res) {
  S[kRes] = res;
  S[kIts] = 0;
  S[kRhoOld] = 1;
  S[kAlpha] = 1;
  S[kOmega] = 1;
}

// Grid-stride update kernels that also leave one partial sum per block of the reductions the next
// step needs (reduced by launch_reduce, in a fixed order).
// p = r + beta (p - omega v), beta = (rho / rho_old) (alpha / omega); partials of ||p||^2
__global__ void __launch_bounds__(256) k_bcg_p(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                               double *__restrict__ p, const double *__restrict__ S, double tol,
                                               double *__restrict__ part) {
  __shared__ double sh[4];
  const bool live = !(S[kRes] <= tol);
  const double beta = (S[kRho] / S[kRhoOld]) * (S[kAlpha] / S[kOmega]), om = S[kOmega];
  double acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double pi = p[i];
    if (live) {
      pi = r[i] + beta * (pi - om * v[i]);
      p[i] = pi;
    }
    acc += pi * pi;
  }
  const double b = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// s = r - alpha v, alpha = rho / (rh, v); partials of ||s||^2
__global__ void __launch_bounds__(256) k_bcg_s(int64_t n, const double *__restrict__ r, const double *__restrict__ v,
                                               double *__restrict__ s, double *__restrict__ S, double tol,
                                               double *__restrict__ part) {
  __shared__ double sh[4];
  const bool live = !(S[kRes] <= tol);
  const double alpha = S[kRho] / S[kRhv];
  double acc = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double si = s[i];
    if (live) {
      si = r[i] - alpha * v[i];
      s[i] = si;
    }
    acc += si * si;
  }
  const double b = block_sum(acc, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = b;
    if (blockIdx.x == 0 && live) S[kAlpha] = alpha;   // no lane of this launch reads it
  }
}

// x += alpha ph + omega sh, r = s - omega t, omega = (t, s) / (t, t) (0 when t = 0, i.e. s = 0);
// partials of ||r||^2 and (rh, r).  ph, sh: the preconditioned p and s (p and s without one)
__global__ void __launch_bounds__(256) k_bcg_xr(int64_t n, const double *__restrict__ p, const double *__restrict__ s,
                                                const double *__restrict__ t, const double *__restrict__ rh,
                                                double *__restrict__ x, double *__restrict__ r, double *__restrict__ S,
                                                double tol, double *__restrict__ part, double *__restrict__ part2,
                                                const double *__restrict__ ph, const double *__restrict__ sh_) {
  __shared__ double sh[4];
  const bool live = !(S[kRes] <= tol);
  const double tt = S[kTt], om = tt > 0 ? S[kTs] / tt : 0.0, al = S[kAlpha];
  double a1 = 0, a2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double ri = r[i];
    if (live) {
      x[i] += al * ph[i] + om * sh_[i];
      ri = s[i] - om * t[i];
      r[i] = ri;
    }
    a1 += ri * ri;
    a2 += rh[i] * ri;
  }
  const double b1 = block_sum(a1, sh), b2 = block_sum(a2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = b1;
    part2[blockIdx.x] = b2;
    if (blockIdx.x == 0 && live) {   // no lane of this launch reads these
      S[kOmega] = om;
      S[kRhoOld] = S[kRho];
      S[kIts] += 1.0;
    }
  }
}

// the perturbed stage along x with step K / ||x|| (||x|| = *yn on the device; 0 leaves the stage as is):
// o1 = a1 + (c1 / yn) x, o2 = a2 + (c2 / yn) x; z = 0 (the residual of the stage is added into it)
__global__ void k_lin2_dev(int64_t n, const double *__restrict__ a1, double c1, const double *__restrict__ a2, double c2,
                           const double *__restrict__ x, const double *__restrict__ yn, double *__restrict__ o1,
                           double *__restrict__ o2, double *__restrict__ z) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double y = *yn, s = y > 0 ? 1.0 / y : 0.0;
  o1[i] = a1[i] + (c1 * s) * x[i];
  o2[i] = a2[i] + (c2 * s) * x[i];
  z[i] = 0.0;
}

// out = (Gp - G) / eps, eps = K / yn (0 when yn = 0); partials of (a, out) and, with part2, of (out, out)
__global__ void __launch_bounds__(256) k_diffq(int64_t n, const double *__restrict__ G, const double *__restrict__ Gp,
                                               double K, const double *__restrict__ yn, double *__restrict__ out,
                                               const double *__restrict__ a, double *__restrict__ part,
                                               double *__restrict__ part2) {
  __shared__ double sh[4];
  const double y = *yn, f = y > 0 ? y / K : 0.0;
  double a1 = 0, a2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double o = y > 0 ? (Gp[i] - G[i]) * f : 0.0;
    out[i] = o;
    a1 += a[i] * o;
    a2 += o * o;
  }
  const double b1 = block_sum(a1, sh);
  const double b2 = part2 ? block_sum(a2, sh) : 0.0;
  if (threadIdx.x == 0) {
    part[blockIdx.x] = b1;
    if (part2) part2[blockIdx.x] = b2;
  }
}

// partials of sum x and sum x^2
__global__ void __launch_bounds__(256) k_moments(int64_t n, const double *__restrict__ x, double *__restrict__ part,
                                                 double *__restrict__ part2) {
  __shared__ double sh[4];
  double a1 = 0, a2 = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    a1 += x[i];
    a2 += x[i] * x[i];
  }
  const double b1 = block_sum(a1, sh), b2 = block_sum(a2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = b1;
    part2[blockIdx.x] = b2;
  }
}

static iga_status host_scalar(Handle &h, const double *dev, double *out, int n = 1) {
  if (hipMemcpyAsync(out, dev, n * sizeof(double), hipMemcpyDeviceToHost, h.stream) != hipSuccess ||
      hipStreamSynchronize(h.stream) != hipSuccess)
    return fail(IGA_EHIP, "scalar read-back");
  return IGA_OK;
}

static iga_status ch_gen_alpha_step(Handle &h, const double *C0, const double *V0, double dt, double rho,
                                    double theta, double lam, const iga_newton_opts *o_in, double *C1, double *V1,
                                    iga_newton_report *rep) {
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(IGA_EINVAL, "dt must be positive");
  if (!(rho >= 0.0 && rho <= 1.0)) return fail(IGA_EINVAL, "rho_inf must be in [0, 1]");
  iga_newton_opts o{};
  o.atol = 1e-10;
  o.max_newton = 30;
  o.max_krylov = 2000;
  o.forcing_max = 1e-2;
  if (o_in) o = *o_in;
  if (o.max_newton < 0 || o.max_newton > 64) return fail(IGA_EINVAL, "max_newton must be in 0..64");
  if (o.max_krylov < 1) return fail(IGA_EINVAL, "max_krylov must be positive");
  if (o.forcing_max <= 0) o.forcing_max = 1e-2;
  const double am = 0.5 * (3.0 - rho) / (1.0 + rho), af = 1.0 / (1.0 + rho), gm = 0.5 + am - af;
  iga_status st;
  if ((st = ensure_newton_ws(h, false, IGA_FP64))) return st;
  const int64_t N = h.pb.N;
  if ((st = ensure_chfdm(h))) return st;
  const bool pc = h.chfdm_ok && h.precond != IGA_PRECOND_JACOBI;
  if (!h.chw && (st = alloc_owned(h, (void **)&h.chw, (size_t)13 * N * sizeof(double)))) return st;
  if (pc && !h.chw_pc && (st = alloc_owned(h, (void **)&h.chw_pc, (size_t)4 * N * sizeof(double)))) return st;
  double *Ca = h.chw, *Va = Ca + N, *G = Va + N, *Gp = G + N, *tC = Gp + N, *tV = tC + N;
  double *x = tV + N, *r = x + N, *rh = r + N, *p = rh + N, *v = p + N, *sv = v + N;
  double *t = sv + N;
  // right preconditioning: the iteration runs on A P^-1 with ph = P^-1 p and sh = P^-1 s
  double *ph = pc ? h.chw_pc : p, *sh = pc ? h.chw_pc + N : sv, *w1 = pc ? h.chw_pc + 2 * N : nullptr,
         *w2 = pc ? w1 + N : nullptr;
  const unsigned nb = ga_blocks(N);
  iga_newton_report rr{};
  auto t0 = std::chrono::steady_clock::now();
  IGA_HIP_CHECK(hipMemcpyAsync(V1, V0, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
  double ca_norm = 0, cmom[2] = {0, 0};
  // A y: forward difference of the stage residual along y (writes out; uses Gp, tC, tV).  The
  // residual is linear in cdot, so only the change of c needs a small step: c moves by
  // sqrt(eps_machine) (1 + ||c_{n+af}||) along y / ||y|| (||y|| = *yn on the device), which is
  // a step K / ||y|| in cdot with K = sqrt(eps_machine) (1 + ||c_{n+af}||) / (af gamma dt).
  double K = 0;
  // with the partials of (a, out) in P1 and, when both is set, of (out, out) in P2
  const int nbv = vec_blocks(N, h.npartials);
  double *P1 = h.partials, *P2 = h.partials + h.npartials;
  auto apply = [&](const double *y, double *out, const double *yn, const double *a, bool both) -> iga_status {
    iga_status s2;
    hipLaunchKernelGGL(k_lin2_dev, dim3(nb), dim3(256), 0, h.stream, N, (const double *)Ca, K * af * gm * dt,
                       (const double *)Va, K * am, y, yn, tC, tV, Gp);
    if ((s2 = launch_cahn_hilliard(h, tC, tV, theta, lam, Gp, false))) return s2;
    hipLaunchKernelGGL(k_diffq, dim3(nbv), dim3(256), 0, h.stream, N, (const double *)G, (const double *)Gp, K, yn, out,
                       a, P1, both ? P2 : nullptr);
    IGA_HIP_CHECK(hipGetLastError());
    return IGA_OK;
  };
  double *S = h.scal;
  // iterations between read-backs of the residual norm: preconditioned solves take a few long
  // iterations, so each is checked (a converged chunk still runs its launches as no-ops)
  const int kCheck = pc ? 1 : 4;
  double nr = 0, r0 = -1;
  int k;
  st = IGA_OK;
  for (k = 0;; ++k) {
    hipLaunchKernelGGL(k_ga_stage, dim3(nb), dim3(256), 0, h.stream, N, C0, V0, (const double *)V1, af * dt * gm,
                       af * dt * (1.0 - gm), am, Ca, Va);
    IGA_HIP_CHECK(hipGetLastError());
    if ((st = launch_cahn_hilliard(h, Ca, Va, theta, lam, G))) break;
    if ((st = launch_norm(h, G, h.scal)) || (st = host_scalar(h, h.scal, &nr))) break;
    rr.hist[k] = nr;
    if (r0 < 0) r0 = nr;
    if (!std::isfinite(nr)) { st = fail(IGA_ENOCONV, "stage residual is not finite"); break; }
    if (nr < o.atol || (o.rtol > 0 && nr <= o.rtol * r0)) { rr.converged = 1; break; }
    if (k >= o.max_newton) { st = fail(IGA_ENOCONV, "Cahn-Hilliard Newton did not converge"); break; }
    if ((st = launch_norm(h, Ca, h.scal)) || (st = host_scalar(h, h.scal, &ca_norm))) break;
    // preconditioner coefficients from the means of c and c^2 over the coefficients: linearised
    // about a uniform state the Jacobian is am M + af gamma dt ((M mu')(c) K + lam M(c) B), with
    // M mu' = 1 / (2 theta) - 2 c (1 - c); the state's mean of c (1 - c) stands in for c (1 - c)
    double sa = 0, sb = 0;
    if (pc) {
      hipLaunchKernelGGL(k_moments, dim3(nbv), dim3(256), 0, h.stream, N, (const double *)Ca, P1, P2);
      if ((st = launch_reduce(h, P1, nbv, S + kYn, 0)) || (st = launch_reduce(h, P2, nbv, S + kSn, 0)) ||
          (st = host_scalar(h, S + kYn, cmom, 2)))
        break;
      const double mc = cmom[0] / N, m2 = fmax(0.0, mc - cmom[1] / N);
      sa = af * gm * dt * (0.5 / theta - 2.0 * m2);
      sb = af * gm * dt * lam * m2;
    }
    // BiCGStab on A x = -G from x = 0
    const double tol = fmin(o.forcing_max, fmax(1e-12, 0.1 * o.atol / nr)) * nr;
    if ((st = launch_fill(h, x, N, 0.0)) || (st = launch_fill(h, p, N, 0.0)) || (st = launch_fill(h, v, N, 0.0))) break;
    hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(256), 0, h.stream, N, -1.0, (const double *)G, 0.0, r);
    hipLaunchKernelGGL(k_axpby, dim3(nb), dim3(256), 0, h.stream, N, 1.0, (const double *)r, 0.0, rh);
    K = 1.4901161193847656e-8 * (1.0 + ca_norm) / (af * gm * dt);
    hipLaunchKernelGGL(k_bcg_init, dim3(1), dim3(1), 0, h.stream, S, nr);
    if ((st = launch_dot(h, rh, r, S + kRho))) break;
    double chk[3] = {nr, 0, 0};   // residual norm, iterations taken, rho
    for (int launched = 0; launched < o.max_krylov;) {
      for (int j = 0; j < kCheck && launched < o.max_krylov; ++j, ++launched) {
        hipLaunchKernelGGL(k_bcg_p, dim3(nbv), dim3(256), 0, h.stream, N, (const double *)r, (const double *)v, p,
                           (const double *)S, tol, P1);
        if (pc) {
          if ((st = launch_chfdm_apply(h, p, ph, w1, w2, am, sa, sb)) || (st = launch_norm(h, ph, S + kYn))) break;
        } else if ((st = launch_reduce(h, P1, nbv, S + kYn, 1))) {
          break;
        }
        if ((st = apply(ph, v, S + kYn, rh, false)) || (st = launch_reduce(h, P1, nbv, S + kRhv, 0))) break;
        hipLaunchKernelGGL(k_bcg_s, dim3(nbv), dim3(256), 0, h.stream, N, (const double *)r, (const double *)v, sv, S,
                           tol, P1);
        if (pc) {
          if ((st = launch_chfdm_apply(h, sv, sh, w1, w2, am, sa, sb)) || (st = launch_norm(h, sh, S + kSn))) break;
        } else if ((st = launch_reduce(h, P1, nbv, S + kSn, 1))) {
          break;
        }
        if ((st = apply(sh, t, S + kSn, sv, true)) || (st = launch_reduce(h, P1, nbv, S + kTs, 0)) ||
            (st = launch_reduce(h, P2, nbv, S + kTt, 0)))
          break;
        hipLaunchKernelGGL(k_bcg_xr, dim3(nbv), dim3(256), 0, h.stream, N, (const double *)p, (const double *)sv,
                           (const double *)t, (const double *)rh, x, r, S, tol, P1, P2, (const double *)ph,
                           (const double *)sh);
        if ((st = launch_reduce(h, P1, nbv, S + kRes, 1)) || (st = launch_reduce(h, P2, nbv, S + kRho, 0))) break;
      }
      if (st) break;
      IGA_HIP_CHECK(hipGetLastError());
      if ((st = host_scalar(h, S + kRes, chk, 3))) break;
      if (!std::isfinite(chk[0]) || chk[0] <= tol) break;
      if (chk[2] == 0.0) { st = fail(IGA_ENOCONV, "BiCGStab breakdown"); break; }
    }
    if (st) break;
    const int it = (int)chk[1];
    if (!(chk[0] <= tol)) { st = fail(IGA_ENOCONV, "BiCGStab did not reach its tolerance"); break; }
    if ((st = launch_axpy(h, 1.0, x, V1))) break;
    if (k < 64) rr.krylov_iters[k] = it;
    rr.krylov_iters_total += it;
  }
  if (!st) {
    IGA_HIP_CHECK(hipMemcpyAsync(C1, C0, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, h.stream));
    if (!(st = launch_axpy(h, dt * gm, V1, C1))) st = launch_axpy(h, dt * (1.0 - gm), V0, C1);
    if (!st && hipStreamSynchronize(h.stream) != hipSuccess) st = fail(IGA_EHIP, "sync");
  }
  rr.newton_iters = k;
  rr.res_norm0 = r0;
  rr.res_norm = nr;
  rr.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = rr;
  return st;
}

}  // namespace iga

using namespace iga;

extern "C" {

iga_status iga_create(const iga_desc *desc, void *hip_stream, iga_t *out) {
  if (!out) return fail(IGA_EINVAL, "null output handle");
  *out = nullptr;
  Handle *h = nullptr;
  iga_status st = create_impl(desc, hip_stream, &h);
  if (st) return st;
  // the preconditioner's 1D eigendecompositions are set-up work, like the pattern
  if ((st = ensure_fdm(*h))) {
    iga_destroy((iga_t)h);
    return st;
  }
  *out = (iga_t)h;
  set_error("");
  return IGA_OK;
}

iga_status iga_destroy(iga_t hh) {
  if (!hh) return IGA_OK;
  Handle *h = (Handle *)hh;
  hipStreamSynchronize(h->stream);
  for (void *p : h->owned)
    if (p) hipFree(p);
  for (auto &call : h->kt_ev)
    for (auto &pair : call)
      for (auto &e : pair)
        if (e) hipEventDestroy(e);
  delete h;
  return IGA_OK;
}

iga_status iga_info(iga_t hh, int64_t *ndof, int64_t *nnz, int64_t *nelem) {
  if (!hh) return fail(IGA_EINVAL, "null handle");
  Handle *h = (Handle *)hh;
  if (ndof) *ndof = h->pb.N;
  if (nnz) *nnz = h->pb.nnz;
  if (nelem) *nelem = h->pb.E;
  return IGA_OK;
}

iga_status iga_set_option(iga_t hh, int key, int64_t value) {
  if (!hh) return fail(IGA_EINVAL, "null handle");
  Handle *h = (Handle *)hh;
  switch (key) {
    case IGA_OPT_JAC_ALGO:
      if (value < IGA_JAC_AUTO || value > IGA_JAC_LOCAL_ND) return fail(IGA_EINVAL, "bad Jacobian algorithm");
      h->jac_algo = (int)value;
      return IGA_OK;
    case IGA_OPT_ROW_BLOCK:
      h->row_b1 = (int)((value >> 8) & 0xff);
      h->row_b2 = (int)(value & 0xff);
      return IGA_OK;
    case IGA_OPT_ROW_SEGMENTS:
      if (value < 0 || value > 64) return fail(IGA_EINVAL, "row segments must be in 0..64");
      h->row_segments = (int)value;
      return IGA_OK;
    case IGA_OPT_KERNEL_TIMING:
      if (value != 0 && value != 1) return fail(IGA_EINVAL, "kernel timing must be 0 or 1");
      h->ktiming = (int)value;
      h->kt_calls = 0;   // (re)starts the averaging window
      h->kt_n = 0;
      return IGA_OK;
    case IGA_OPT_TILED_3D:
      if (value < 0 || value > 3) return fail(IGA_EINVAL, "IGA_OPT_TILED_3D is 0, 1, 2 or 3");
      h->tiled_3d = (int)value;
      return IGA_OK;
    case IGA_OPT_FDM_KERNEL:
      if (value < 0 || value > 2) return fail(IGA_EINVAL, "IGA_OPT_FDM_KERNEL is 0, 1 or 2");
      h->fdm_kernel = (int)value;
      return IGA_OK;
    case IGA_OPT_RES_ZRUN:
      if (value < 0 || value > 8) return fail(IGA_EINVAL, "IGA_OPT_RES_ZRUN is 0..8");
      h->res_zrun = (int)value;
      return IGA_OK;
    case IGA_OPT_ND_SCATTER:
      if (value != 0 && value != 1) return fail(IGA_EINVAL, "IGA_OPT_ND_SCATTER is 0 or 1");
      h->nd_color = (int)value;
      return IGA_OK;
    case IGA_OPT_PRECOND:
      if (value < IGA_PRECOND_AUTO || value > IGA_PRECOND_FDM) return fail(IGA_EINVAL, "bad preconditioner");
      if (value == IGA_PRECOND_FDM && !fdm_possible(*h))
        return fail(IGA_EUNSUPPORTED, "the FDM preconditioner needs at most 512 unknowns per axis and a Dirichlet face");
      h->precond = (int)value;
      return IGA_OK;
    case IGA_OPT_LAMBDA_BITS: {
      double lam;
      std::memcpy(&lam, &value, sizeof(double));
      if (!std::isfinite(lam)) return fail(IGA_EINVAL, "lambda must be finite");
      h->pb.lambda = lam;
      return IGA_OK;
    }
  }
  return fail(IGA_EINVAL, "unknown option");
}

iga_status iga_csr_pattern(iga_t hh, int64_t *row_ptr_dev, int32_t *col_idx_dev) {
  if (!hh || !row_ptr_dev || !col_idx_dev) return fail(IGA_EINVAL, "null argument");
  Handle *h = (Handle *)hh;
  IGA_HIP_CHECK(hipMemcpyAsync(row_ptr_dev, h->row_ptr, sizeof(int64_t) * (h->pb.N + 1), hipMemcpyDeviceToDevice,
                               h->stream));
  IGA_HIP_CHECK(hipMemcpyAsync(col_idx_dev, h->col_idx, sizeof(int32_t) * h->pb.nnz, hipMemcpyDeviceToDevice,
                               h->stream));
  return IGA_OK;
}

iga_status iga_assemble_residual(iga_t hh, const double *U, double *R) {
  if (!hh || !U || !R) return fail(IGA_EINVAL, "null argument");
  return launch_residual(*(Handle *)hh, U, R);
}

iga_status iga_gen_alpha_step(iga_t hh, const double *U0, const double *V0, double dt, double rho_inf,
                              const iga_newton_opts *opts, double *U1, double *V1, iga_newton_report *report) {
  if (!hh || !U0 || !V0 || !U1 || !V1) return fail(IGA_EINVAL, "null argument");
  if (U1 == U0 || U1 == V0 || V1 == U0 || V1 == V0 || U1 == V1) return fail(IGA_EINVAL, "outputs must not alias inputs");
  return gen_alpha_step(*(Handle *)hh, U0, V0, dt, rho_inf, opts, U1, V1, report);
}

iga_status iga_ch_gen_alpha_step(iga_t hh, const double *C0, const double *V0, double dt, double rho_inf,
                                 double theta, double lambda_ch, const iga_newton_opts *opts, double *C1, double *V1,
                                 iga_newton_report *report) {
  if (!hh || !C0 || !V0 || !C1 || !V1) return fail(IGA_EINVAL, "null argument");
  if (C1 == C0 || C1 == V0 || V1 == C0 || V1 == V0 || C1 == V1) return fail(IGA_EINVAL, "outputs must not alias inputs");
  return ch_gen_alpha_step(*(Handle *)hh, C0, V0, dt, rho_inf, theta, lambda_ch, opts, C1, V1, report);
}

iga_status iga_cahn_hilliard_residual(iga_t hh, const double *C, const double *Cdot, double theta, double lambda_ch,
                                      double *R) {
  if (!hh || !C || !Cdot || !R) return fail(IGA_EINVAL, "null argument");
  return launch_cahn_hilliard(*(Handle *)hh, C, Cdot, theta, lambda_ch, R);
}

iga_status iga_grad_laplacian_residual(iga_t hh, const double *U, double *R) {
  if (!hh || !U || !R) return fail(IGA_EINVAL, "null argument");
  return launch_grad_laplacian(*(Handle *)hh, U, R);
}

iga_status iga_biharmonic_residual(iga_t hh, const double *U, double *R) {
  if (!hh || !U || !R) return fail(IGA_EINVAL, "null argument");
  return launch_biharmonic(*(Handle *)hh, U, R);
}

iga_status iga_assemble_jacobian(iga_t hh, const double *U, void *vals, int prec) {
  if (!hh || !U || !vals) return fail(IGA_EINVAL, "null argument");
  if (prec != IGA_FP64 && prec != IGA_FP32 && prec != IGA_BF16 && prec != IGA_BF16X3)
    return fail(IGA_EUNSUPPORTED, "unknown Jacobian precision");
  Handle &h = *(Handle *)hh;
  kt_reset(h);
  return assemble_jacobian(h, U, vals, prec);
}

iga_status iga_assemble_jacobian_noalloc(iga_t hh, const double *U, void *vals, int prec) {
  if (!hh || !U || !vals) return fail(IGA_EINVAL, "null argument");
  if (prec != IGA_FP64 && prec != IGA_FP32) return fail(IGA_EUNSUPPORTED, "Jacobian values are FP64 or FP32");
  Handle &h = *(Handle *)hh;
  const int algo = h.jac_algo;
  if (algo == IGA_JAC_AUTO || algo == IGA_JAC_ROWGATHER) {
    int s1 = 0, s2 = 0;
    pick_sep_block(h, &s1, &s2);
    if (rgsep_supported(h, s1, s2)) return launch_jac_rgsep_scratch(h, U, vals, prec, s1, s2);
    if (rgt2_supported(h.pb) && h.row_b1 == 0) return launch_jac_rgt2(h, U, vals, prec);
  }
  if (algo == IGA_JAC_AUTO || algo == IGA_JAC_ROWGATHER || algo == IGA_JAC_ROWGATHER_GENERAL) {
    int b1 = 0, b2 = 0;
    pick_block(h, prec, &b1, &b2);
    if (rowgather_supported(h, prec, b1, b2)) return launch_jac_rowgather(h, U, vals, prec, b1, b2);
  }
  return fail(IGA_EUNSUPPORTED, "the allocation-free Jacobian covers the row-gather paths only (element-matrix "
                                "and local-ND assembly keep a per-point cache in the handle)");
}

iga_status iga_kernel_times(iga_t hh, int cap, double *ms, const char **names, int *count) {
  if (!hh) return fail(IGA_EINVAL, "null handle");
  Handle &h = *(Handle *)hh;
  if (h.kt_calls == 0 || h.kt_n == 0) return fail(IGA_ESTATE, "no timed Jacobian assembly recorded");
  const int64_t ncalls = h.kt_calls < Handle::kTimedCalls ? h.kt_calls : Handle::kTimedCalls;
  const int last = (int)((h.kt_calls - 1) % Handle::kTimedCalls);
  IGA_HIP_CHECK(hipEventSynchronize(h.kt_ev[last][h.kt_n - 1][1]));
  for (int i = 0; i < h.kt_n && i < cap; ++i) {
    // kernel i of the latest call, averaged over the kept calls that timed the same kernel there
    // (calls made with another algorithm launch other kernels)
    double sum = 0;
    int64_t used = 0;
    for (int64_t c = 0; c < ncalls; ++c) {
      const int slot = (int)((h.kt_calls - 1 - c) % Handle::kTimedCalls);
      if (h.kt_cnt[slot] <= i || h.kt_name[slot][i] != h.kt_name[last][i]) continue;
      float t = 0;
      IGA_HIP_CHECK(hipEventElapsedTime(&t, h.kt_ev[slot][i][0], h.kt_ev[slot][i][1]));
      sum += t;
      ++used;
    }
    if (ms) ms[i] = sum / (double)used;
    if (names) names[i] = h.kt_name[last][i];
  }
  if (count) *count = h.kt_n;
  return IGA_OK;
}

iga_status iga_apply(iga_t hh, const double *U, const double *v, double *y) {
  if (!hh || !U || !v || !y) return fail(IGA_EINVAL, "null argument");
  Handle &h = *(Handle *)hh;
  iga_status st = launch_linearize(h, U);
  if (st) return st;
  return launch_apply(h, v, y);
}

iga_status iga_spmv(iga_t hh, const void *vals, int prec, const double *x, double *y) {
  if (!hh || !vals || !x || !y) return fail(IGA_EINVAL, "null argument");
  if (prec != IGA_FP64 && prec != IGA_FP32) return fail(IGA_EUNSUPPORTED, "values are FP64 or FP32");
  Handle &h = *(Handle *)hh;
  return launch_spmv(h, vals, prec, x, y, nullptr, h.npartials);
}

iga_status iga_newton_solve(iga_t hh, double *U, const iga_newton_opts *opts, iga_newton_report *report) {
  if (!hh || !U) return fail(IGA_EINVAL, "null argument");
  return newton(*(Handle *)hh, U, opts, report);
}

iga_status iga_element_matrices(iga_t hh, const double *U, const int32_t *elems, int n, int prec, double *out) {
  if (!hh || !U || !elems || !out || n < 0) return fail(IGA_EINVAL, "bad argument");
  if (prec != IGA_FP64 && prec != IGA_FP32) return fail(IGA_EUNSUPPORTED, "element matrices in FP64 or FP32");
  Handle &h = *(Handle *)hh;
  if (n == 0) return IGA_OK;
  for (int i = 0; i < n; ++i)
    if (elems[i] < 0 || elems[i] >= h.pb.E) return fail(IGA_EINVAL, "element index out of range");
  const int L = ipow(h.pb.P, h.pb.dim);
  int32_t *d_el = nullptr;
  double *d_out = nullptr;
  IGA_HIP_CHECK(hipMalloc(&d_el, sizeof(int32_t) * n));
  if (hipMalloc(&d_out, sizeof(double) * (size_t)n * L * L) != hipSuccess) {
    hipFree(d_el);
    return fail(IGA_ENOMEM, "element matrix buffer");
  }
  iga_status st = IGA_OK;
  if (hipMemcpyAsync(d_el, elems, sizeof(int32_t) * n, hipMemcpyHostToDevice, h.stream) != hipSuccess)
    st = fail(IGA_EHIP, "copy");
  if (!st) st = launch_elem_matrices(h, U, d_el, n, prec, d_out);
  if (!st && hipMemcpyAsync(out, d_out, sizeof(double) * (size_t)n * L * L, hipMemcpyDeviceToHost, h.stream) != hipSuccess)
    st = fail(IGA_EHIP, "copy back");
  if (!st && hipStreamSynchronize(h.stream) != hipSuccess) st = fail(IGA_EHIP, "sync");
  hipFree(d_el);
  hipFree(d_out);
  return st;
}

}  // extern "C"
