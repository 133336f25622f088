/*
 * Plain FP64 CPU oracle for tensor-product NURBS isogeometric assembly (Bratu-type
 * problems -div(kappa grad u) = lambda exp(u) + f with u = 0 on chosen faces).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header, table or helper
 * with the HIP library; it is written to be checked against the paper by eye:
 *   - B-splines by the literal Cox-de Boor recursion (Sec. 2.1),
 *   - tensor product and lexicographic numbering (Sec. 2.2),
 *   - rational basis and its first derivatives (Sec. 2.3, eq:rational, eq:drational),
 *   - geometry Jacobian, inverse and spatial gradients (App. A, eq:identity, eq:dspatial),
 *   - second derivatives: of B-splines (the derivative formula applied twice), rational
 *     (eq:ddrational), of the inverse map (eq:ddimap) and spatial (eq:ddspatial), and the
 *     fourth-order operator sum W (Lap N_A)(Lap u_h) built from them,
 *   - generalized-alpha time stepping (eq:ga) of M Udot + R(U) = 0 with Newton on Udot_{n+1},
 *   - the Cahn-Hilliard residual (primal weak form of the paper's strong form),
 *   - the adjacency stencil of Algorithm 2 (Sec. 2.5),
 *   - periodic axes by unclamping (Sec. 2.4, eq:unclamp-left/right) and index wrapping (eq:map-wrap),
 *   - naive per-quadrature-point residual/Jacobian assembly as in Algorithm 3 (Sec. 2.7)
 *     with the Bratu integrands eq:residual and eq:jacobian (Sec. 3.1),
 *   - the local numerical-differentiation Jacobian of Sec. 2.8 (eq:fdjac),
 *   - Newton's method with exact (direct banded or tight CG) linear solves.
 * Every function returns 0 on success and a nonzero code on bad input.
 */
#ifndef IGA_ORACLE_H
#define IGA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int dim;                   /* 1, 2 or 3 */
  int degree[3];
  int nknots[3];
  const double *knots[3];
  const double *ctrl;        /* N*dim control points (natural order) or NULL: x = xi */
  const double *weights;     /* N weights or NULL: non-rational */
  int nquad[3];              /* 0 => degree+1 Gauss-Legendre points */
  double lambda;
  int kappa_mode;            /* 0: kappa = 1, 1: nodal N values, 2: one value per element */
  const double *kappa;
  const double *source;      /* N spline coefficients of f, or NULL */
  unsigned dirichlet_mask;   /* bit 2*axis+side: u = 0 on that face */
  int periodic[3];           /* 0: open axis; k + 1: periodic with C^k across the seam (Sec. 2.4):
                                the open knots given are unclamped and n - k functions remain,
                                n being the index of the last open function */
} orc_problem;

int orc_gauss_legendre(int n, double *x, double *w);
/* eq:unclamp-left / eq:unclamp-right in place; n = index of the last basis function */
int orc_unclamp(int n, int p, int k, double *U);
int orc_basis_1d(int p, const double *U, int nk, int i, double xi, double *val, double *der);
/* second derivative of B_{i,p} at xi (the derivative formula of Sec. 2.1 applied twice) */
int orc_basis_1d_d2(int p, const double *U, int nk, int i, double xi, double *d2);
int orc_stencil(int p, const double *U, int nk, int i, int *l, int *r);
int orc_sizes(const orc_problem *pb, int64_t *ndof, int64_t *nelem, int64_t *nnz);
int orc_csr_pattern(const orc_problem *pb, int64_t *row_ptr, int32_t *col_idx);
int orc_residual(const orc_problem *pb, const double *U, double *R);
int orc_jacobian(const orc_problem *pb, const double *U, const int64_t *row_ptr,
                 const int32_t *col_idx, double *vals);
/* Local numerical-differentiation Jacobian (Sec. 2.8, eq:fdjac); eta <= 0: sqrt(epsilon). */
int orc_jacobian_nd(const orc_problem *pb, const double *U, const int64_t *row_ptr,
                    const int32_t *col_idx, double eta, double *vals);
int orc_residual_rows(const orc_problem *pb, const double *U, const int64_t *rows, int64_t nrows,
                      double *out);
int orc_jacobian_rows(const orc_problem *pb, const double *U, const int64_t *rows, int64_t nrows,
                      const int64_t *row_ptr, const int32_t *col_idx, double *out);
int orc_element_matrix(const orc_problem *pb, const double *U, int64_t elem, double *Ke, double *Re);
int orc_jacobian_elements(const orc_problem *pb, const double *U, const int64_t *elems, int64_t n,
                          const int64_t *row_ptr, const int32_t *col_idx, double *vals);
int orc_spmv(int64_t n, const int64_t *row_ptr, const int32_t *col_idx, const double *vals,
             const double *x, double *y);
int orc_newton(const orc_problem *pb, double *U, double atol, double rtol, int maxit,
               int linear_solver, double cg_rtol, double *hist, int *iters);
int64_t orc_nqp(const orc_problem *pb);
int orc_qp_data(const orc_problem *pb, const double *U, double *xq, double *Wq, double *uq,
                double *gradu);
int orc_load_vector(const orc_problem *pb, const double *fq, double *b);
int orc_mass_matrix(const orc_problem *pb, const int64_t *row_ptr, const int32_t *col_idx,
                    double *vals);
/* At local coordinates t in [-1,1]^dim of element elem: the nloc = prod(p_d+1) local functions'
 * global indices A, values N, spatial gradients dN [nloc][3] and spatial Hessians d2N [nloc][3][3]
 * (eq:ddrational, eq:ddimap read with the sign that differentiating eq:identity gives,
 * eq:ddspatial), and the point x [3].  Any output may be NULL. */
int orc_basis_hessian(const orc_problem *pb, int64_t elem, const double *t, int64_t *A, double *N,
                      double *dN, double *d2N, double *x);
/* Third derivative of B_{i,p} at xi (the derivative formula of Sec. 2.1 applied three times). */
int orc_basis_1d_d3(int p, const double *U, int nk, int i, double xi, double *d3);
/* Spatial third derivatives d3N [nloc][3][3][3] of the local functions of element elem at local
 * coordinates t (eq:dddrational, eq:dddimap, eq:dddspatial) and their global indices A. */
int orc_basis_third(const orc_problem *pb, int64_t elem, const double *t, int64_t *A, double *d3N);
/* R_A = sum_e sum_q W grad N_A . grad(Lap u_h) over every function (no boundary rows): the
 * fourth-order operator integrated by parts once, from third spatial derivatives. */
int orc_grad_laplacian_residual(const orc_problem *pb, const double *U, double *R);
/* R_A = sum_e sum_q W (Lap N_A)(Lap u_h) over every function (no boundary rows). */
int orc_biharmonic_residual(const orc_problem *pb, const double *U, double *R);
/* Cahn-Hilliard residual of the paper's strong form (D = 1) in primal weak form: R_A = sum W [N_A cdot
 * + M mu' grad N_A . grad c + lam (M Lap N_A + M' grad c . grad N_A) Lap c], M = c(1-c), M' = 1-2c,
 * mu' = 1/(2 theta c(1-c)) - 2; C, Cdot: coefficients of c and its rate; no boundary terms. */
int orc_cahn_hilliard_residual(const orc_problem *pb, const double *C, const double *Cdot, double theta,
                               double lam, double *R);
/* Generalized-alpha parameters from the spectral radius at infinity rho in [0, 1] (after eq:ga). */
int orc_gen_alpha_params(double rho, double *am, double *af, double *gamma);
/* One generalized-alpha step (eq:ga) of M0 Udot + R(U) = 0 (M0: mass matrix without Dirichlet rows and
 * columns; R: eq:residual with its Dirichlet rows).  U0, V0: state and rate at t_n; U1, V1 at t_n + dt.
 * Newton on Udot_{n+1} from Udot_n to ||G||_2 < atol, exact linear solves.  Returns 0 when converged. */
int orc_gen_alpha_step(const orc_problem *pb, const double *U0, const double *V0, double dt, double rho,
                       double atol, int maxit, double *U1, double *V1, int *iters);

#ifdef __cplusplus
}
#endif
#endif
