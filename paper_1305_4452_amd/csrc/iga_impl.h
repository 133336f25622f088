// Internal definitions shared by the HIP translation units of libiga (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "iga.h"

namespace iga {

constexpr int kMaxP = 7;       // functions per element per axis (degree <= 6)
constexpr int kWave = 64;      // CDNA wavefront

// Number of per-quadrature-point geometry streams of the table mode.
//  3D: D'00 D'11 D'22 D'01 D'02 D'12 | g0 g1 g2 | W/w | 1/w     (11)
//  2D: D'00 D'11 D'01 | g0 g1 | W/w | 1/w                      (7)
// D' = kappa * W * Jinv Jinv^T / w^2 (parametric-gradient metric with the weight w of the
// rational basis divided out twice), g = grad_xi(w) / w, W = quadrature weight * det J.
__host__ __device__ constexpr int geo_streams(int dim) { return dim == 3 ? 11 : 7; }

struct AxisDev {
  const double *B;     // [ne][Q][P]   B-spline values at the Gauss points of each element
  const double *dB;    // [ne][Q][P]   d/dxi
  const double *wq;    // [ne][Q]      Gauss weight * (xi_{s+1} - xi_s) / 2
  const int *efirst;   // [ne]         index of the first non-zero function of each element
  const int *stl;      // [n]          Algorithm 2 left index
  const int *stw;      // [n]          Algorithm 2 width r - l + 1
  int nper;            // periodic axis: its number of functions (indices wrap); 0 on an open axis
  const int *nbr;      // periodic axis: [n][2p+1] sorted functions sharing an element with each one
  const double *d2B;   // [ne][Q][P]   d2/dxi2 (the fourth-order operator)
  const double *d3B;   // [ne][Q][P]   d3/dxi3 (the fourth-order operator integrated by parts once)
};

// eq:map-wrap for the local-to-global index of an element function (i < 2 nper here)
__host__ __device__ inline int wrap_fn(const AxisDev &ax, int i) { return (ax.nper && i >= ax.nper) ? i - ax.nper : i; }

// Plain-old-data view of a problem passed by value to kernels.
struct DevProblem {
  int dim, p, P, Q;
  int n[3], ne[3];
  int64_t N, E, nnz;
  AxisDev ax[3];
  const int64_t *row_ptr;
  const int32_t *col_idx;
  double lambda;
  int table;           // 0: identity geometry, kappa one/element (analytic metric); 1: geo table
  int rational;        // weights present
  int kappa_mode;
  const double *kel;   // element kappa (analytic mode, kappa_mode ELEMENT)
  const double *geo;   // table mode: [E][geo_streams][Q^dim]
  const double *wts;   // [N] or null
  const double *ctrl;  // [N][dim] control points (kept when given) or null: x = xi
  const double *src;   // [N] or null
  unsigned dmask;
  int simple_knots;    // every element's first function equals its span counter (max continuity)
  int separable;       // identity geometry, no weights, kappa = 1: stiffness is a Kronecker sum
  int periodic;        // some axis is periodic (element kernels and CSR SpMV only)
  // 1D Galerkin matrices per axis, band storage [n][2p+1] (offset o = j - i + p):
  //   M_d[i][o] = sum_g w(g) B_i(g) B_j(g),  A_d[i][o] = sum_g w(g) B'_i(g) B'_j(g)
  const double *sepM[3], *sepA[3];
  // the same per element: elM_d[e][a][b] = sum_q w(q) B_a(q) B_b(q) over element e (local a, b < P)
  const double *elM[3], *elA[3];
};

__host__ __device__ inline int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

__device__ inline bool is_dirichlet_idx(const DevProblem &pb, int i0, int i1, int i2) {
  unsigned m = pb.dmask;
  if (((m >> 0) & 1u) && i0 == 0) return true;
  if (((m >> 1) & 1u) && i0 == pb.n[0] - 1) return true;
  if (((m >> 2) & 1u) && i1 == 0) return true;
  if (((m >> 3) & 1u) && i1 == pb.n[1] - 1) return true;
  if (pb.dim == 3) {
    if (((m >> 4) & 1u) && i2 == 0) return true;
    if (((m >> 5) & 1u) && i2 == pb.n[2] - 1) return true;
  }
  return false;
}

__device__ inline bool is_dirichlet(const DevProblem &pb, int64_t A) {
  int i0 = (int)(A % pb.n[0]);
  int64_t r = A / pb.n[0];
  int i1 = (int)(r % pb.n[1]);
  int i2 = (int)(r / pb.n[1]);
  return is_dirichlet_idx(pb, i0, i1, i2);
}

// Offset of column (j0,j1,j2) inside row (i0,i1,i2): the row holds the tensor product of the
// per-axis stencils, ordered with axis 0 fastest, so no search is needed.
// position of column j in row i's list along one axis (a periodic axis searches its sorted list)
__device__ inline int axis_rank(const AxisDev &ax, int W, int i, int j) {
  if (!ax.nper) return j - ax.stl[i];
  const int *l = ax.nbr + (size_t)i * W;
  int r = 0;
  while (r < W - 1 && l[r] != j) ++r;
  return r;
}

__device__ inline int64_t csr_slot(const DevProblem &pb, int i0, int i1, int i2, int j0, int j1, int j2) {
  int64_t A = i0 + (int64_t)pb.n[0] * (i1 + (int64_t)pb.n[1] * i2);
  const int W = 2 * pb.p + 1;
  int w0 = pb.ax[0].stw[i0], w1 = pb.ax[1].stw[i1];
  int o0 = axis_rank(pb.ax[0], W, i0, j0), o1 = axis_rank(pb.ax[1], W, i1, j1);
  int o2 = pb.dim == 3 ? axis_rank(pb.ax[2], W, i2, j2) : 0;
  return pb.row_ptr[A] + ((int64_t)o2 * w1 + o1) * w0 + o0;
}

// Fast-diagonalisation preconditioner data (see precond.hip): per axis the non-Dirichlet index
// range [lo, lo + m), the forward / backward transforms V^T and V (m x m, row-major), the
// generalised eigenvalues times the axis coefficient a_d, and the 1D basis integrals (row sums
// of the mass matrix).
constexpr int kFdmMax = 512;      // longest axis (non-Dirichlet coefficients) of the FDM preconditioner
struct FdmData {
  int ok;
  int lo[3], m[3];
  const double *Tf[3], *Tb[3], *mu[3], *rs[3];
  double mu_min;
  double mscale;   // mass scale of the shift (mean det J per unit parametric volume; 1 for x = xi)
};

// ------------------------------------------------------------------------------------------
// Host-side handle
// ------------------------------------------------------------------------------------------
struct Handle {
  DevProblem pb{};
  hipStream_t stream = nullptr;
  int device = 0;
  // owned device buffers
  std::vector<void *> owned;
  int64_t *row_ptr = nullptr;
  int32_t *col_idx = nullptr;
  double *geo = nullptr;
  double *lin = nullptr;          // [E][Q^d] per-point linearisation coefficient (m'')
  double *partials = nullptr;     // reduction scratch
  int npartials = 0;
  // Newton workspace (lazily allocated)
  double *nw = nullptr;           // 6 * N doubles: R, d, r, z, p, q
  double *dinv = nullptr;
  double *scal = nullptr;         // device scalars
  void *jvals = nullptr;          // Jacobian values owned by Newton
  int jvals_prec = -1;
  // generalized-alpha (lazily allocated): mass matrix without Dirichlet rows and columns (CSR
  // values), and the stage vectors U_{n+af}, Udot_{n+am} and a product
  double *massv = nullptr;
  double *gaw = nullptr;          // 3 * N doubles
  double *chw = nullptr;          // Cahn-Hilliard generalized-alpha: 13 * N doubles
  // options
  int jac_algo = IGA_JAC_AUTO;
  int nd_color = 0;   // local-ND scatter: 0 atomics (default), 1 colour-ordered plain adds
  int tiled_3d = 1;   // 3D residual / apply by element tiles where supported (0: one element per workgroup;
                      // 1: column tiles streamed along axis 2; 2: cube tiles; 3: column tiles of fixed depth)
  int res_zrun = 0;   // streamed column tiles: chunks of 4 elements per run along axis 2 (0 = planned)
  int fdm_kernel = 0; // dense 1D transforms of the fast diagonalisation: 0 planned, 1 vector units, 2 matrix cores
  int row_b1 = 0, row_b2 = 0;
  int row_segments = 0;           // separable row-gather: segments along axis 0 (0 = planned)
  // separable row-gather tables (3D, identity geometry, kappa = 1, simple knots)
  void *mfield = nullptr;         // [ne0 Q][ne2 Q][ne1 Q] reaction coefficient, FP64 or FP32
  // BF16 matrix-core Jacobian (lazily): FP32 coefficient streams [ne0 Q][stream][ne1 Q][ne2 Q + pad]
  float *mma_cs = nullptr;
  size_t mma_cs_bytes = 0;
  const void *sep_phi[2][3] = {}; // [FP64, FP32][axis] band products [n][2p+1][(p+1)^2]
  const void *sep_b0[2] = {};     // [FP64, FP32] axis-0 basis table [ne0][Q][P]
  const int64_t *sep_cw = nullptr; // prefix sums of the stencil widths, [n0+1 | n1+1 | n2+1]
  // fast-diagonalisation preconditioner (built at creation when the problem is separable)
  FdmData fdm{};
  double *fdm_part = nullptr;     // 2 x 256 shift partial sums
  double *fdm_shift = nullptr;    // device scalar c
  double *fdm_w = nullptr;        // 2 x N scratch of the transforms (lazily, with the Newton workspace)
  int precond = IGA_PRECOND_AUTO;
  int fdm_tried = 0;              // build attempted (lazily, by the first Newton solve that uses it)
  std::vector<double> hsepM[3], hsepA[3];   // host copies of the 1D band matrices
  std::vector<double> hsepH[3];              // ... and of the second-derivative one, sum w B_i'' B_j''
  // Cahn-Hilliard fast diagonalisation (every axis periodic on uniform knots): per axis the
  // transforms V^T, V of A V = M V diag(mu), V^T M V = I, and eta = diag(V^T H V) (H is diagonal in
  // the same basis on uniform periodic knots, where A, M and H are circulant); built lazily
  int chfdm_tried = 0, chfdm_ok = 0;
  const double *ch_Tf[3] = {}, *ch_Tb[3] = {}, *ch_mu[3] = {}, *ch_eta[3] = {};
  double *chw_pc = nullptr;                  // 2 N scratch of its transforms
  // per-kernel timing (IGA_OPT_KERNEL_TIMING): event pairs of up to kMaxTimed kernels for each
  // of the last kTimedCalls Jacobian assemblies (a ring)
  static constexpr int kMaxTimed = 4, kTimedCalls = 64;
  int ktiming = 0, kt_n = 0;
  int64_t kt_calls = 0;           // timed calls since timing was switched on
  hipEvent_t kt_ev[kTimedCalls][kMaxTimed][2] = {};
  const char *kt_name[kTimedCalls][kMaxTimed] = {};   // per kept call: the kernel each event pair timed
  int kt_cnt[kTimedCalls] = {};                        // per kept call: timed kernels
  // host copies
  std::vector<double> hknots[3];
  int nb_colors = 0;
};

// Error reporting (thread-local message)
void set_error(const std::string &msg);
iga_status fail(iga_status st, const std::string &msg);

#define IGA_HIP_CHECK(expr)                                                          \
  do {                                                                               \
    hipError_t _e = (expr);                                                          \
    if (_e != hipSuccess)                                                            \
      return ::iga::fail(IGA_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

// Per-kernel timing: kt_reset at the start of a timed entry point, kt_begin / kt_end around
// each launch (events on the handle's stream; no-ops unless IGA_OPT_KERNEL_TIMING is set).
inline void kt_reset(Handle &h) {
  if (!h.ktiming) return;
  h.kt_n = 0;
  ++h.kt_calls;
  h.kt_cnt[(h.kt_calls - 1) % Handle::kTimedCalls] = 0;
}
inline void kt_begin(Handle &h, const char *name) {
  if (!h.ktiming || h.kt_n >= Handle::kMaxTimed) return;
  const int slot = (int)((h.kt_calls - 1) % Handle::kTimedCalls);
  hipEvent_t *ev = h.kt_ev[slot][h.kt_n];
  for (int k = 0; k < 2; ++k)
    if (!ev[k]) (void)hipEventCreate(&ev[k]);
  h.kt_name[slot][h.kt_n] = name;
  (void)hipEventRecord(ev[0], h.stream);
}
inline void kt_end(Handle &h) {
  if (!h.ktiming || h.kt_n >= Handle::kMaxTimed) return;
  const int slot = (int)((h.kt_calls - 1) % Handle::kTimedCalls);
  (void)hipEventRecord(h.kt_ev[slot][h.kt_n][1], h.stream);
  h.kt_cnt[slot] = ++h.kt_n;
}

// A v = mu M v for dense symmetric A, M (n x n, row-major): V (column i = vector i, V^T M V = I)
// and mu; false if M is not positive definite or the factorisation fails its check.
bool gen_eigen(const std::vector<double> &A, const std::vector<double> &M, int n, std::vector<double> &V,
               std::vector<double> &mu);
iga_status upload_owned(Handle &h, double **dst, const double *src, size_t count);
bool fdm_possible(const Handle &h);
iga_status ensure_fdm(Handle &h);   // builds on first use; h.fdm.ok tells whether it succeeded
// shift of K + shift M for the Jacobian at U (-lambda times the weighted mean of e^U), plus
// mass_coef for operators with an added mass term (generalized-alpha: am / (af gamma dt))
iga_status launch_fdm_shift(Handle &h, const double *U, double mass_coef = 0.0);
iga_status launch_fdm_apply(Handle &h, const double *r, double *z, double *w1, double *w2);

// Launchers implemented in the kernel translation units.
iga_status launch_geometry(Handle &h, const double *ctrl, const double *wts, const double *kappa_nodal,
                           int *bad_det);
iga_status launch_pattern(Handle &h);
iga_status launch_residual(Handle &h, const double *U, double *R);
iga_status launch_linearize(Handle &h, const double *U);
iga_status launch_biharmonic(Handle &h, const double *U, double *R);
iga_status launch_grad_laplacian(Handle &h, const double *U, double *R);
// Cahn-Hilliard preconditioner: z = P^{-1} r with P = am M + s (a K + b B) (see precond.hip)
iga_status ensure_chfdm(Handle &h);
iga_status launch_chfdm_apply(Handle &h, const double *r, double *z, double *w1, double *w2, double am, double sa,
                              double sb);
// sum over `width` lanes of a wavefront (all of them get it)
__device__ inline double warp_sum(double v, int width) {
  for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
  return v;
}

// block-wide sum of a 64-lane-multiple block, sh[blockDim.x / 64] in LDS; all threads get the result
__device__ inline double block_sum(double v, double *sh) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = warp_sum(v, 64);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// blocks for a grid-stride vector kernel with at most maxb partial sums; *out = sum of n partials
// (square root when do_sqrt)
int vec_blocks(int64_t N, int maxb);
iga_status launch_reduce(Handle &h, const double *part, int n, double *out, int do_sqrt);

// zero_out = false: R is already zero (the kernels add into it)
iga_status launch_cahn_hilliard(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R,
                                bool zero_out = true);
iga_status launch_apply(Handle &h, const double *v, double *y);
iga_status launch_diag_mf(Handle &h, double *diag);
iga_status launch_elem_matrices(Handle &h, const double *U, const int32_t *elems, int n, int prec,
                                double *out);
iga_status launch_jac_scatter(Handle &h, const double *U, void *vals, int prec, int color_mode);
iga_status launch_jac_rowgather(Handle &h, const double *U, void *vals, int prec, int b1, int b2);
bool rowgather_supported(const Handle &h, int prec, int b1, int b2);
iga_status launch_jac_rgsep(Handle &h, const double *U, void *vals, int prec, int b1, int b2);
iga_status launch_jac_nd(Handle &h, const double *U, void *vals, int prec, int color_mode);
bool rgt2_supported(const DevProblem &pb);
bool res2_supported(const DevProblem &pb);
bool res3_supported(const DevProblem &pb);
iga_status launch_res3(Handle &h, const double *X, double *Y, int op);
iga_status launch_res2(Handle &h, const double *U, double *R);
iga_status launch_jac_rgt2(Handle &h, const double *U, void *vals, int prec);
bool rgsep_supported(const Handle &h, int b1, int b2);
// BF16 matrix-core row-gather Jacobian (FP32 values; split: three BF16 products per operand pair)
bool mma_supported(const DevProblem &pb);
iga_status launch_jac_mma(Handle &h, const double *U, float *vals, bool split);
// allocation-free Jacobian: the separable path with its reaction field in a static per-device array
#define NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
iga_status noalloc_scratch_init(int device);
size_t rgsep_field_bytes(const Handle &h, int prec);
iga_status launch_jac_rgsep_scratch(Handle &h, const double *U, void *vals, int prec, int b1, int b2);
iga_status launch_spmv(Handle &h, const void *vals, int prec, const double *x, double *y,
                       double *partial_dot, int npart);
iga_status launch_fill(Handle &h, double *x, int64_t n, double v);

}  // namespace iga
