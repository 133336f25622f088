/*
 * iga.h -- C ABI of the MI355X (gfx950) isogeometric assembly and Newton-Krylov library.
 *
 * Problem class: tensor-product NURBS patches in 2D or 3D, scalar unknown u, Galerkin form of
 *     -div(kappa grad u) = lambda exp(u) + f,   u = 0 on the faces selected by dirichlet_mask,
 * i.e. the Bratu problem of the paper's Sec. 3 (eq:strong, eq:dirichlet) with its residual
 * eq:residual and Jacobian eq:jacobian, generalised by a diffusion coefficient kappa and an
 * optional source f.  The discretisation follows Sec. 2: B-spline bases from knot vectors
 * (Sec. 2.1), tensor products with lexicographic numbering A = i0 + n0*(i1 + n1*i2) (Sec. 2.2),
 * the rational basis of eq:rational, the geometry map and spatial gradients of App. A
 * (eq:identity, eq:dspatial), Gauss-Legendre quadrature with p+1 points per axis (Sec. 2.9),
 * the CSR pattern of Algorithm 2 (Sec. 2.5) and assembly as in Algorithm 3 (Sec. 2.7).
 *
 * Conventions for every call:
 *  - Vectors are FP64, contiguous, in the natural (lexicographic) order, and are DEVICE
 *    pointers owned by the caller.  Host arrays passed to iga_create are copied; the caller
 *    may free them afterwards.
 *  - Work is enqueued on the HIP stream given to iga_create and is asynchronous, except
 *    iga_create, iga_info, iga_element_matrices and iga_newton_solve, which synchronise.
 *  - Every call returns an iga_status; nothing is thrown and nothing is printed.  On failure
 *    iga_last_error() returns a message for the calling thread.
 *  - A handle must not be used from two threads at once.
 */
#ifndef IGA_H
#define IGA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct iga_s *iga_t;

typedef enum {
  IGA_OK = 0,
  IGA_EINVAL = 1,        /* invalid argument or problem description */
  IGA_ENOMEM = 2,        /* device or host allocation failed */
  IGA_EHIP = 3,          /* a HIP runtime call failed */
  IGA_ENOCONV = 4,       /* Newton or Krylov did not converge (or produced NaN/Inf) */
  IGA_EUNSUPPORTED = 5,  /* valid description outside what the GPU kernels implement */
  IGA_ESTATE = 6         /* call not valid in the handle's current state */
} iga_status;

/* Precision of the element contractions of a Jacobian (eq:jacobian).  FP64 and FP32 contract in that
 * precision and write values of that type.  BF16 and BF16X3 run the axis-2 contraction of the
 * row-gather on the BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) and write FP32
 * values: BF16 rounds both operands to BF16 (relative error of the values ~1e-3), BF16X3 splits each
 * FP32 operand x into hi = bf16(x) and lo = bf16(x - hi) and sums lo*hi + hi*lo + hi*hi (~1e-5).
 * The geometry, u and e^u stay FP64 and the other contraction levels FP32.  Newton with a BF16 or
 * BF16X3 Jacobian keeps the FP64 residual, so it converges to the FP64 solution (a refinement). */
typedef enum { IGA_FP64 = 0, IGA_FP32 = 1, IGA_BF16 = 2, IGA_BF16X3 = 3 } iga_prec;

typedef enum { IGA_KAPPA_ONE = 0, IGA_KAPPA_NODAL = 1, IGA_KAPPA_ELEMENT = 2 } iga_kappa_mode;

/* Jacobian assembly algorithm (iga_set_option(IGA_OPT_JAC_ALGO)):
 *   ROWGATHER: each workgroup owns a block of row pencils and sums element contributions
 *              itself; every CSR value is written exactly once (no atomics, deterministic).
 *              With identity geometry, no weights and kappa = 1 the stiffness is a Kronecker
 *              sum of 1D band matrices and only the reaction term is contracted in 3D;
 *   ATOMIC:    element matrices by sum factorisation, scattered with FP64 atomic adds;
 *   COLOR:     element matrices scattered colour by colour ((p+1)^d colours, no atomics);
 *   ROWGATHER_GENERAL: the row-gather kernel with every term contracted (never the
 *              Kronecker-sum shortcut), for comparison;
 *   LOCAL_ND:  local numerical differentiation (Sec. 2.8, eq:fdjac): column k of each element
 *              matrix is sum_q (F_q(U_e + delta e_k) - F_q(U_e)) / delta with
 *              delta = eta sqrt(1 + ||U_e||_2), eta = sqrt(DBL_EPSILON); an approximation of the
 *              same matrix (relative error ~1e-8), added colour by colour or with FP64 atomics
 *              (IGA_OPT_ND_SCATTER; p <= 4 in 3D). */
typedef enum {
  IGA_JAC_AUTO = 0, IGA_JAC_ROWGATHER = 1, IGA_JAC_ATOMIC = 2, IGA_JAC_COLOR = 3, IGA_JAC_ROWGATHER_GENERAL = 4,
  IGA_JAC_LOCAL_ND = 5
} iga_jac_algo;

typedef enum {
  IGA_OPT_JAC_ALGO = 1,      /* iga_jac_algo */
  IGA_OPT_ROW_BLOCK = 2,     /* row-gather pencil block: (b1 << 8) | b2, 0 = autotuned */
  IGA_OPT_LAMBDA_BITS = 3,   /* replace lambda: value is the IEEE-754 bit pattern of a double */
  IGA_OPT_ROW_SEGMENTS = 4,  /* separable and BF16 matrix-core row-gathers: split each pencil into this
                                many segments along axis 0 (each a workgroup; 0 = planned from the
                                occupancy), 0..64 */
  IGA_OPT_KERNEL_TIMING = 5, /* 1: record a HIP event pair around each kernel of iga_assemble_jacobian
                                (read back with iga_kernel_times); 0: off (default) */
  IGA_OPT_PRECOND = 6,       /* CG preconditioner of iga_newton_solve: iga_precond */
  IGA_OPT_ND_SCATTER = 7,    /* IGA_JAC_LOCAL_ND: 0 FP64 atomics in one launch (default), 1 colour
                                by colour with plain adds ((p+1)^d launches, no two workgroups of a
                                launch share a value) */
  IGA_OPT_TILED_3D = 8,      /* 3D residual and matrix-free apply with x = xi, no weights, no source:
                                1 by tiles of elements (default: (16/Q)^2 elements in x-y with one lane per
                                Gauss-point column, streamed along axis 2 in chunks of 4 elements that
                                keep the open function planes in registers), 3 the same tiles with a
                                fixed depth of 4 elements (3 at p = 4), 2 by cubic tiles of elements, 0 one
                                element per workgroup; 1, 2 and 3 also select tiles for the 3D
                                fourth-order operator on x = xi without weights and the 2D and 3D
                                Cahn-Hilliard residual */
  IGA_OPT_RES_ZRUN = 9,      /* IGA_OPT_TILED_3D = 1: chunks per run along axis 2 (one workgroup's
                                work), 1..8, capped at a kernel's longest run (4 chunks of 4 elements for
                                the residual and apply, 8 chunks of 2 elements for the 3D Cahn-Hilliard
                                residual of C^1 quadratics); 0 (default) plans it from the mesh size */
  IGA_OPT_FDM_KERNEL = 10    /* dense 1D transforms of the fast-diagonalisation preconditioners: 0
                                (default) matrix cores for boxes that give 1024 tiles of 128 x 64, the
                                vector units otherwise; 1 always the vector units; 2 always the FP64
                                matrix cores */
} iga_option;

/* CG preconditioner (iga_set_option(IGA_OPT_PRECOND)):
 *   AUTO:   FDM when every axis has at most 512 non-Dirichlet coefficients, Jacobi otherwise;
 *   JACOBI: the inverse diagonal of the Jacobian;
 *   FDM:    fast diagonalisation of a0 A0(x)M1(x)M2 + a1 M0(x)A1(x)M2 + a2 M0(x)M1(x)A2 + c M, the
 *           parametric 1D stiffness / mass matrices of the tensor-product B-spline basis (Sec. 2.1),
 *           a_d the quadrature average of kappa W (J^-1 J^-T)_dd per unit parametric volume (1 for
 *           x = xi, kappa = 1, where this is the exact stiffness), c = -lambda times the
 *           integral-weighted mean of e^U times the mean det J, set at each Newton step;
 *           IGA_EUNSUPPORTED if an axis is larger. */
typedef enum { IGA_PRECOND_AUTO = 0, IGA_PRECOND_JACOBI = 1, IGA_PRECOND_FDM = 2 } iga_precond;

typedef struct {
  int dim;                       /* 2 or 3 */
  int degree[3];                 /* p_d, 1..6; the GPU kernels require equal degrees */
  int nknots[3];
  const double *knots[3];        /* host; open (p+1 equal end knots), non-decreasing */
  const double *ctrl;            /* host, N*dim control points, natural order; NULL: x = xi */
  const double *weights;         /* host, N positive weights; NULL: non-rational */
  int nquad[3];                  /* 0 or p+1 (Gauss-Legendre points per axis) */
  double lambda;
  int kappa_mode;                /* iga_kappa_mode */
  const double *kappa;           /* host: N nodal values or E element values (natural order) */
  const double *source;          /* host, N spline coefficients of f, or NULL */
  unsigned dirichlet_mask;       /* bit 2*axis+side set: u = 0 on that face */
  int periodic[3];               /* 0: open axis; k + 1: periodic with C^k continuity across the seam
                                    (Sec. 2.4).  The open knots given are unclamped by
                                    eq:unclamp-left/right and functions are wrapped by eq:map-wrap,
                                    leaving n - k per axis (n: index of the last open function;
                                    at least 2p+1 must remain).  Needs x = xi, no weights, kappa one or
                                    element-wise, no Dirichlet face on that axis; the assembly then
                                    uses element kernels (IGA_JAC_ATOMIC or IGA_JAC_LOCAL_ND), CSR
                                    SpMV with column indices and Jacobi-CG. */
} iga_desc;

typedef struct {
  double atol;                   /* stop when ||R||_2 < atol ... */
  double rtol;                   /* ... or ||R||_2 <= rtol * ||R(U0)||_2 (0 disables) */
  int max_newton;                /* Newton steps (<= 64) */
  int max_krylov;                /* CG iterations per Newton step */
  int matrix_free;               /* 0: assembled CSR Jacobian; 1: iga_apply inside CG */
  int jac_prec;                  /* iga_prec of the Jacobian contraction (assembled mode) */
  double forcing_max;            /* cap of the CG relative tolerance (Eisenstat-Walker); 0: 1e-2 */
  int check_every;               /* CG iterations between convergence checks; 0: automatic (4 with the
                                    fast-diagonalisation preconditioner, 16 with Jacobi) */
} iga_newton_opts;

typedef struct {
  int converged;                 /* 1 if the Newton stopping test was met */
  int newton_iters;
  int krylov_iters_total;
  double res_norm0, res_norm;
  double hist[65];               /* ||R|| before each Newton step and at the end */
  int krylov_iters[64];
  double t_total_ms, t_residual_ms, t_jacobian_ms, t_krylov_ms;
} iga_newton_report;

/* Create a handle: validates the description (open non-decreasing knots, degrees, sizes,
 * positive weights, det J > 0 at every quadrature point), builds the quadrature rule, the 1D
 * basis tables, the Algorithm 2 CSR pattern and the geometry data on the device.
 * Errors: IGA_EINVAL (bad description), IGA_EUNSUPPORTED (unequal degrees, nquad != p+1,
 * interior knot multiplicity > 1 for the row-gather path is handled by falling back to ATOMIC),
 * IGA_ENOMEM, IGA_EHIP.  Synchronous.  hip_stream may be NULL (the null stream). */
iga_status iga_create(const iga_desc *desc, void *hip_stream, iga_t *out);
iga_status iga_destroy(iga_t h);
iga_status iga_info(iga_t h, int64_t *ndof, int64_t *nnz, int64_t *nelem);
iga_status iga_set_option(iga_t h, int key, int64_t value);

/* Copy the CSR pattern (row_ptr: N+1 int64, col_idx: nnz int32, both caller-owned device
 * buffers).  Columns of a row are ascending; row A holds the tensor product of the per-axis
 * Algorithm 2 ranges [l_d(i_d), r_d(i_d)]. */
iga_status iga_csr_pattern(iga_t h, int64_t *row_ptr_dev, int32_t *col_idx_dev);

/* R = R(U) (eq:residual): Dirichlet rows hold R_A = U_A. */
iga_status iga_assemble_residual(iga_t h, const double *U_dev, double *R_dev);

/* vals = J(U) (eq:jacobian) on the iga_csr_pattern pattern; prec IGA_FP64 writes double,
 * IGA_FP32 writes float (FP32 element contractions with FP32 accumulation), IGA_BF16 and
 * IGA_BF16X3 write float from the BF16 matrix-core row-gather (iga_prec; 3D, open axes, simple
 * interior knots, degree 2..4, IGA_EUNSUPPORTED otherwise).  Dirichlet rows are identity rows and
 * Dirichlet columns of the other rows are zero (symmetric elimination).  Every entry is written: no
 * zeroing is needed. */
iga_status iga_assemble_jacobian(iga_t h, const double *U_dev, void *vals_dev, int prec);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): iga_assemble_jacobian without any allocation and without
 * the handle's reaction-field buffer.  Same arguments, values and errors as iga_assemble_jacobian
 * (the handle itself is created beforehand by iga_create, which allocates).  On the separable
 * row-gather path (3D, x = xi, no weights, kappa = 1, simple knots) the per-point reaction field
 * -lambda W e^u the kernels pass between them lives in a static device array of 64 MiB per GPU,
 * part of the library's code object and held until the process ends: at most 64 MiB /
 * sizeof(value) quadrature points (FP64: 8,388,608, e.g. 50^3 elements at p = 3; FP32: 16,777,216,
 * i.e. 64^3 at p = 3); a larger mesh is refused with IGA_EINVAL and a message naming both sizes.
 * The 2D tiled and general row-gather paths use no scratch memory and run as in
 * iga_assemble_jacobian; the element-matrix and local-ND algorithms (IGA_OPT_JAC_ALGO) are refused
 * with IGA_EUNSUPPORTED.  Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other handles, other host threads) race and must be serialised by the caller.
 * No kernel-timing events are recorded.  Asynchronous on the handle's stream. */
iga_status iga_assemble_jacobian_noalloc(iga_t h, const double *U_dev, void *vals_dev, int prec);

/* Cahn-Hilliard residual (the Cahn-Hilliard example: the paper's strong form with D = 1, in the
 * primal weak form obtained by integrating by parts twice, boundary terms dropped as on periodic
 * axes): R_A = sum_e sum_q W [N_A cdot + (M mu' + lambda_ch M' Lap c) grad N_A . grad c
 * + lambda_ch M Lap c Lap N_A], M = c(1-c), M' = 1-2c, mu' = 1/(2 theta c(1-c)) - 2.  C_dev, Cdot_dev:
 * coefficients of c and of its rate (N doubles, device); R_dev overwritten, every function (no
 * Dirichlet rows).  c must lie in (0, 1) at the Gauss points.  Needs x = xi without weights, p >= 2,
 * p <= 6 in 2D and p <= 3 in 3D (IGA_EUNSUPPORTED otherwise); theta > 0 (IGA_EINVAL).
 * Asynchronous on the handle's stream. */
iga_status iga_cahn_hilliard_residual(iga_t h, const double *C_dev, const double *Cdot_dev, double theta,
                                      double lambda_ch, double *R_dev);

/* One generalized-alpha step (eq:ga) of the Cahn-Hilliard system R_CH(cdot, c) = 0 (the residual of
 * iga_cahn_hilliard_residual; theta, lambda_ch as there).  C0_dev, V0_dev: c and its rate at t_n;
 * C1_dev, V1_dev (outputs, not aliasing the inputs): at t_n + dt.  Newton on cdot_{n+1} from
 * cdot_n; each linear system by BiCGStab (the Jacobian is not symmetric) on Jacobian-vector products
 * by a forward difference of the residual (the matrix-free approach of Sec. 2.8): the residual is
 * linear in cdot, so the step moves c by sqrt(eps) (1 + ||c_{n+af}||) along the direction.  Stops
 * when ||G||_2 < opts->atol.  opts: atol, rtol, max_newton, max_krylov (BiCGStab iterations per
 * Newton step), forcing_max; NULL: defaults.  BiCGStab keeps its scalars on the device and the host
 * tests its residual norm every 4 iterations (every iteration when preconditioned); the report
 * counts the iterations that changed the iterate.  With every axis periodic on uniform knots and at
 * most 512 functions per axis, BiCGStab is right-preconditioned by fast diagonalisation of
 * am M + af gamma dt (a K + lambda_ch b B) (M, K the mass and stiffness matrices,
 * B = int Lap N_A Lap N_B, a = 1/(2 theta) - 2 b and b the mean of c (1 - c) over the
 * coefficients: the Jacobian linearised about a uniform state), its 1D eigenbases built at the
 * first call; IGA_OPT_PRECOND = IGA_PRECOND_JACOBI turns it off (the difference products give no
 * diagonal, so no other preconditioner is used).
 * Same geometry limits as iga_cahn_hilliard_residual.  IGA_ENOCONV if Newton or BiCGStab fails.
 * Synchronous. */
iga_status iga_ch_gen_alpha_step(iga_t h, const double *C0_dev, const double *V0_dev, double dt, double rho_inf,
                                 double theta, double lambda_ch, const iga_newton_opts *opts, double *C1_dev,
                                 double *V1_dev, iga_newton_report *report);

/* One generalized-alpha step (eq:ga, parameters from rho_inf in [0, 1] by the formulas after it)
 * of the first-order system M0 Udot + R(U) = 0: R the residual of eq:residual (Dirichlet rows
 * U_A), M0 the mass matrix without Dirichlet rows and columns.  U0_dev, V0_dev: state and rate at
 * t_n; U1_dev, V1_dev (outputs, not aliasing the inputs): at t_n + dt.  Newton on Udot_{n+1} from
 * Udot_n, each step solving (am M0 + af gamma dt J(U_{n+af})) d = -G by CG on the assembled FP64
 * Jacobian's pattern, preconditioned by fast diagonalisation of K + (am/(af gamma dt) - lambda
 * mean(e^u)) M where it is built (IGA_OPT_PRECOND as for Newton), Jacobi otherwise; stops when
 * ||G||_2 < opts->atol (or the rtol test).  opts as
 * for iga_newton_solve (matrix_free must be 0, jac_prec FP64; NULL: defaults); report may be NULL.
 * The mass matrix is assembled at the first call and kept.  IGA_ENOCONV if Newton did not
 * converge.  Synchronous. */
iga_status iga_gen_alpha_step(iga_t h, const double *U0_dev, const double *V0_dev, double dt, double rho_inf,
                              const iga_newton_opts *opts, double *U1_dev, double *V1_dev,
                              iga_newton_report *report);

/* Fourth-order operator from second spatial derivatives: R_A = sum_e sum_q W (Lap N_A)(Lap u_h)
 * for every function A (no Dirichlet rows), W the Gauss weight times the span factors and det J,
 * Lap N_A the trace of eq:ddspatial with the rational second derivatives of eq:ddrational and
 * the inverse-map derivatives of eq:ddimap (read with the minus sign that differentiating
 * eq:identity gives).  This is the principal part of a primal biharmonic / Cahn-Hilliard weak
 * form (the Cahn-Hilliard example).  U_dev, R_dev: N doubles on the device, natural order; R is
 * overwritten.
 * Needs p >= 2; p <= 6 in 2D and p <= 3 in 3D, p <= 4 in 3D on x = xi without weights
 * (IGA_EUNSUPPORTED otherwise).  Asynchronous on the handle's stream. */
iga_status iga_biharmonic_residual(iga_t h, const double *U_dev, double *R_dev);

/* The fourth-order operator integrated by parts once, from third spatial derivatives:
 * R_A = sum_e sum_q W grad N_A . grad(Lap u_h), d_i Lap u_h = sum_B U_B sum_j N_{B,ijj}, for every
 * function A (no Dirichlet rows), with the rational third derivatives of eq:dddrational, the
 * inverse-map derivatives of eq:ddimap (the sign of reading eq:identity) and eq:dddimap, and the
 * spatial third derivatives of eq:dddspatial (App. A).  On periodic axes with C^(p-1) continuity,
 * p >= 3, it equals minus iga_biharmonic_residual.  U_dev, R_dev: N doubles on the device; R is
 * overwritten.  Needs p >= 2; p <= 6 in 2D, p <= 3 in 3D (IGA_EUNSUPPORTED otherwise).  Asynchronous
 * on the handle's stream. */
iga_status iga_grad_laplacian_residual(iga_t h, const double *U_dev, double *R_dev);

/* y = J(U) v without forming J (exact linearisation, same Dirichlet convention). */
iga_status iga_apply(iga_t h, const double *U_dev, const double *v_dev, double *y_dev);

/* y = A x for CSR values on the handle's pattern (prec IGA_FP64: double vals, IGA_FP32: float). */
iga_status iga_spmv(iga_t h, const void *vals_dev, int prec, const double *x_dev, double *y_dev);

/* Newton's method on R(U) = 0 (Sec. 3: the residual eq:residual and Jacobian eq:jacobian of the
 * Bratu problem, solved by Newton as in the tutorial run of App. B) starting from U (updated in
 * place): each step assembles R and J (or uses iga_apply) and solves J d = -R by CG with an
 * Eisenstat-Walker forcing term, preconditioned as IGA_OPT_PRECOND selects (fast diagonalisation
 * or Jacobi).  The residual is always FP64, so an FP32, BF16 or BF16X3 Jacobian (opts->jac_prec)
 * gives an FP64-accurate fixed point.  Returns IGA_ENOCONV when the test is not met or on NaN/Inf.
 * opts may be NULL (defaults); report may be NULL.  Synchronous. */
iga_status iga_newton_solve(iga_t h, double *U_dev, const iga_newton_opts *opts, iga_newton_report *report);

/* Test hook: element matrices K_e (local order a = a0 + P*(a1 + P*a2), row-major K[a*nloc+b])
 * of the listed elements (host int32 indices, natural element order), without Dirichlet
 * conditions, computed by the GPU contraction kernels in precision prec; out_host receives
 * n * nloc * nloc doubles.  Synchronous. */
iga_status iga_element_matrices(iga_t h, const double *U_dev, const int32_t *elems_host, int n,
                                int prec, double *out_host);

/* Tracing aid: per-kernel device times of iga_assemble_jacobian.  With IGA_OPT_KERNEL_TIMING = 1
 * (setting the option starts a new averaging window) every call records a HIP event pair on the
 * handle's stream around each kernel it launches; the events of the last 64 calls are kept.
 * iga_kernel_times waits for the latest call's last event, then writes up to cap entries:
 * ms[i] the mean elapsed milliseconds of the latest call's i-th kernel over the kept calls that
 * launched the same kernel in that position (calls made with another algorithm are left out),
 * and names[i] a static string naming it (either array may be NULL); *count receives the number
 * of kernels of the latest call (at most 4).  IGA_ESTATE if no timed call has been made. */
iga_status iga_kernel_times(iga_t h, int cap, double *ms, const char **names, int *count);

/* ---- batched solves ------------------------------------------------------------------------
 * Many independent 2D problems (identity geometry, kappa one or element-wise, simple interior
 * knots; degrees and sizes may differ) solved together: every kernel of the Newton step covers
 * all instances in one launch over per-instance work lists, and per-instance CG scalars, Newton
 * stopping tests and forcing terms stay on the device.  A whole Newton step (the previous
 * correction, residual and norms, the Newton control, Jacobian, preconditioner set-up and one
 * chunk of CG iterations) is one replay of a captured hipGraph; further chunks of CG iterations,
 * when some instance needs them, are replays of a second graph.  Launch shapes (pencils per
 * row-gather block, SpMV lanes per row, and the tile shapes of the tiled row-gather and residual)
 * are autotuned per (degree, size class) when the batch is created, cached for the process and,
 * when the environment variable IGA_TUNE_CACHE names a file, kept there as JSON.  The CG preconditioner is the fast diagonalisation of each
 * instance (two 1D eigendecompositions per distinct 1D problem, computed at creation) when every
 * axis of every instance has at most 136 free coefficients, Jacobi otherwise.  Callers that need
 * many solves of small 2D problems (parameter sweeps, training-data generation) use this instead
 * of iga_newton_solve per instance. */
typedef struct iga_batch_s *iga_batch_t;

typedef struct {
  int converged;
  int newton_iters;
  int krylov_iters;
  double res_norm0, res_norm;
} iga_batch_item_report;

typedef struct {
  int all_converged;
  int newton_steps;              /* Newton steps of the slowest instance */
  int graph_launches;            /* graph replays in total (Newton steps and extra CG chunks) */
  int krylov_iters_max;          /* CG iterations run (chunks x chunk length) */
  double t_total_ms, t_residual_ms, t_jacobian_ms, t_krylov_ms, t_tune_ms;   /* t_jacobian_ms: the
                                    Newton-step graphs (residual, Jacobian, first CG chunk); t_krylov_ms:
                                    the extra CG chunks; t_residual_ms: 0 (inside the step graphs) */
} iga_batch_report;

/* n descriptions (host array); copied.  Errors as iga_create, plus IGA_EUNSUPPORTED for 3D,
 * NURBS geometry or repeated interior knots.  Synchronous. */
iga_status iga_batch_create(int n, const iga_desc *descs, void *hip_stream, iga_batch_t *out);
/* Sizes of the concatenated unknown vector; dof_offsets (host, n+1, may be NULL) receives the
 * offset of each instance's coefficients in the caller's order. */
iga_status iga_batch_info(iga_batch_t b, int64_t *total_ndof, int64_t *total_nnz, int64_t *dof_offsets);
/* Newton on every instance; U_dev is the concatenation (device, FP64) in the caller's order,
 * updated in place.  opts as for iga_newton_solve (matrix_free must be 0; check_every, rounded up
 * to even, is the CG chunk of one graph replay, 0: 8 with fast diagonalisation, 16 with Jacobi); items (host, n, may
 * be NULL) gets the per-instance result.  Returns IGA_ENOCONV if any instance did not converge.
 * Synchronous. */
iga_status iga_batch_newton_solve(iga_batch_t b, double *U_dev, const iga_newton_opts *opts,
                                  iga_batch_item_report *items, iga_batch_report *report);
/* Error estimate of a state, per instance: ||P^{-1} R(U)||_2, with R the residual of eq:residual
 * (Dirichlet rows U_A) and P the fast-diagonalisation operator with its reaction shift taken at U,
 * i.e. the first Newton correction as the preconditioner approximates it (close to ||U - U*|| for
 * U near the solution U*; no solve).  It judges an initial guess by its error where the residual
 * norm would mostly weigh the guess's high-frequency error.  U_dev as for iga_batch_newton_solve
 * (read only); est_host (host, n) gets the estimates in the caller's order.  IGA_EUNSUPPORTED when
 * the fast-diagonalisation data was not built (an axis longer than 136 coefficients).  Uses the
 * solve workspace; synchronous. */
iga_status iga_batch_error_estimates(iga_batch_t b, const double *U_dev, double *est_host);
/* key IGA_OPT_PRECOND only: IGA_PRECOND_AUTO (fast diagonalisation when built, the default),
 * IGA_PRECOND_JACOBI, or IGA_PRECOND_FDM (IGA_EUNSUPPORTED when it was not built).  Takes effect
 * at the next iga_batch_newton_solve. */
iga_status iga_batch_set_option(iga_batch_t b, int key, int64_t value);
iga_status iga_batch_destroy(iga_batch_t b);

/* ---- learned initial guess ---------------------------------------------------------------
 * A 4-layer convolutional encoder-decoder (conv 3x3 2->64, conv 3x3 stride 2 64->64, then the
 * per-channel mean over the 16x16 pixels added back as global context, transposed conv 4x4
 * stride 4 64->64, transposed conv 2x2 64->1; ReLU between layers) mapping
 * a [2][32][32] input (log kappa on the 32x32 cells, lambda broadcast) to the 65x65 interior
 * coefficients of the 64x64-element degree-3 problem.  BF16 weights and activations, FP32
 * accumulation, FP32 master weights, Adam (beta 0.9/0.999, eps 1e-8), mean-squared-error loss.
 * Parameters are one flat FP32 vector [W0 b0 W1 b1 W2 b2 W3 b3] (W0, W1: [co][ci][ky][kx];
 * W2, W3: [ci][co][ky][kx]).  Inputs/outputs are caller-owned FP32 device buffers, batch-major. */
typedef struct igann_s *igann_t;
int64_t igann_num_params(void);
/* Allocates weights, optimiser state and activations for batches of up to batch_max. */
iga_status igann_create(int batch_max, void *hip_stream, igann_t *out);
/* Host FP32 weights in and out (count must equal igann_num_params()); set also resets Adam. */
iga_status igann_set_weights(igann_t net, const float *host, int64_t count);
iga_status igann_get_weights(igann_t net, float *host, int64_t count);
/* y[B][4225] = net(x[B][2][32][32]). */
iga_status igann_forward(igann_t net, const float *x_dev, int B, float *y_dev);
/* Loss = mean((y-t)^2) + w * mean((L(y-t))^2) with L the 5-point Laplacian on the 65x65 grid
 * (zero outside); w = 0 (the default) is the plain mean squared error. */
iga_status igann_set_loss(igann_t net, float laplacian_weight);
/* In place on y[B][4225]: y = (scale * y + mean) * sample_scale[n] (mean: device [4225], may be
 * NULL; sample_scale: device [B], may be NULL), then `passes` times the separable [1 2 1]/4
 * filter along each axis of the 65x65 coefficient grid with zero (the Dirichlet value) outside. */
iga_status igann_postprocess(igann_t net, float *y_dev, int B, const float *mean_dev, float scale,
                             const float *sample_scale_dev, int passes);
/* Loss (as set by igann_set_loss, against t[B][4225]) and its gradient w.r.t. all parameters (host,
 * igann_num_params() floats; may be NULL) without updating the weights.  Synchronous. */
iga_status igann_gradients(igann_t net, const float *x_dev, const float *t_dev, int B, float *loss,
                           float *grad_host);
/* One Adam step with learning rate lr; *loss (may be NULL) gets the batch loss.  Synchronous
 * when loss is non-NULL. */
iga_status igann_train_step(igann_t net, const float *x_dev, const float *t_dev, int B, float lr,
                            float *loss);
iga_status igann_destroy(igann_t net);

/* Message describing the last failure on the calling thread ("" if none). */
const char *iga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
