// Element-by-element kernels (Algorithm 3 organised for the GPU): one 64-lane wavefront per
// element for the residual, the linearisation and the matrix-free apply, and one 256-thread
// workgroup per element for element matrices.  All contractions between the P^d element
// coefficients and the Q^d quadrature points are sum-factorised axis by axis through LDS.
#include "iga_impl.h"
#include "kern_elem.h"

namespace iga {

namespace {
using namespace ek;

template <int DIM, int P, bool TABLE, int OP>
__global__ void __launch_bounds__(64) k_elem_op(DevProblem pb, const double *__restrict__ X,
                                                double *__restrict__ lin, double *__restrict__ Y) {
  elem_op_body<DIM, P, TABLE, OP>(pb, (int64_t)blockIdx.x, X, lin, Y);
}

// Dirichlet rows: R_A = U_A (u = 0 data) for the residual; y_A = v_A for the apply.
__global__ void k_bc_copy(DevProblem pb, const double *__restrict__ X, double *__restrict__ Y) {
  int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (A >= pb.N) return;
  if (is_dirichlet(pb, A)) Y[A] = X[A];
}

__global__ void k_fill(double *x, int64_t n, double v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_fill_f(float *x, int64_t n, float v) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// ------------------------------------------------------------------------------------------
// Element matrices K_e[a][b] = sum_q sum_terms coef_t(q) prod_d X_d(a_d,q_d) Y_d(b_d,q_d)
// ------------------------------------------------------------------------------------------
// A term selects, per axis, the value (0) or derivative (1) table on the test (x) and trial
// (y) side, and one per-point coefficient stream:
//   3D streams: 0..5 D' (00 11 22 01 02 12), 6..8 h = -D' g, 9 m'' = g.D'g + m'
//   2D streams: 0..2 D' (00 11 01), 3..4 h, 5 m''
struct Term {
  int coef;
  int x[3];
  int y[3];
};

__constant__ Term c_terms3_full[16] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {0, 0, 1}, {0, 0, 1}},
    {3, {1, 0, 0}, {0, 1, 0}}, {3, {0, 1, 0}, {1, 0, 0}}, {4, {1, 0, 0}, {0, 0, 1}},
    {4, {0, 0, 1}, {1, 0, 0}}, {5, {0, 1, 0}, {0, 0, 1}}, {5, {0, 0, 1}, {0, 1, 0}},
    {6, {0, 0, 0}, {1, 0, 0}}, {7, {0, 0, 0}, {0, 1, 0}}, {8, {0, 0, 0}, {0, 0, 1}},
    {6, {1, 0, 0}, {0, 0, 0}}, {7, {0, 1, 0}, {0, 0, 0}}, {8, {0, 0, 1}, {0, 0, 0}},
    {9, {0, 0, 0}, {0, 0, 0}}};
__constant__ Term c_terms2_full[9] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {1, 0, 0}, {0, 1, 0}},
    {2, {0, 1, 0}, {1, 0, 0}}, {3, {0, 0, 0}, {1, 0, 0}}, {4, {0, 0, 0}, {0, 1, 0}},
    {3, {1, 0, 0}, {0, 0, 0}}, {4, {0, 1, 0}, {0, 0, 0}}, {5, {0, 0, 0}, {0, 0, 0}}};
// identity geometry, no rational weights: only the diagonal metric and the mass term
__constant__ Term c_terms3_diag[4] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {0, 0, 1}, {0, 0, 1}}, {9, {0, 0, 0}, {0, 0, 0}}};
__constant__ Term c_terms2_diag[3] = {{0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {5, {0, 0, 0}, {0, 0, 0}}};

enum { EM_OUT = 0, EM_ATOMIC = 1, EM_COLOR = 2 };

template <int DIM, bool TABLE>
__device__ inline void point_coefs(const DevProblem &pb, int64_t e, int q, int L, const double *sW0,
                                   const double *sW1, const double *sW2, const double *lin, double *cs) {
  // cs[k] for the streams used by the term tables above
  constexpr int NG = geo_streams(DIM);
  const int P = pb.P;
  if constexpr (!TABLE) {
    int q0 = q % P, q1 = (q / P) % P, q2 = DIM == 3 ? q / (P * P) : 0;
    double W = sW0[q0] * sW1[q1] * (DIM == 3 ? sW2[q2] : 1.0);
    double kw = (pb.kappa_mode == IGA_KAPPA_ELEMENT ? pb.kel[e] : 1.0) * W;
    if (DIM == 3) { cs[0] = cs[1] = cs[2] = kw; cs[9] = lin[e * L + q]; }
    else { cs[0] = cs[1] = kw; cs[5] = lin[e * L + q]; }
  } else {
    const double *G = pb.geo + (size_t)e * NG * L + q;
    double m = lin[e * L + q];
    if (DIM == 3) {
      double D[3][3];
      D[0][0] = G[0]; D[1][1] = G[L]; D[2][2] = G[2 * L];
      D[0][1] = D[1][0] = G[3 * L]; D[0][2] = D[2][0] = G[4 * L]; D[1][2] = D[2][1] = G[5 * L];
      double g[3] = {G[6 * L], G[7 * L], G[8 * L]};
      double Dg[3];
      for (int k = 0; k < 3; ++k) Dg[k] = D[k][0] * g[0] + D[k][1] * g[1] + D[k][2] * g[2];
      cs[0] = D[0][0]; cs[1] = D[1][1]; cs[2] = D[2][2]; cs[3] = D[0][1]; cs[4] = D[0][2]; cs[5] = D[1][2];
      cs[6] = -Dg[0]; cs[7] = -Dg[1]; cs[8] = -Dg[2];
      cs[9] = g[0] * Dg[0] + g[1] * Dg[1] + g[2] * Dg[2] + m;
    } else {
      double D00 = G[0], D11 = G[L], D01 = G[2 * L], g0 = G[3 * L], g1 = G[4 * L];
      double Dg0 = D00 * g0 + D01 * g1, Dg1 = D01 * g0 + D11 * g1;
      cs[0] = D00; cs[1] = D11; cs[2] = D01; cs[3] = -Dg0; cs[4] = -Dg1;
      cs[5] = g0 * Dg0 + g1 * Dg1 + m;
    }
  }
}

// One workgroup (256 threads) per element; the element matrix is accumulated in registers,
// each thread owning NOWN entries, over the four test/trial combinations of axis 0.
template <int DIM, int P, bool TABLE, typename CT, int MODE>
__global__ void __launch_bounds__(256) k_elem_mat(DevProblem pb, const double *__restrict__ lin,
                                                  const int32_t *__restrict__ elems, int color,
                                                  void *__restrict__ outp) {
  constexpr int L = Shp<DIM, P>::L, PP = P * P;
  constexpr int NT = 256;
  constexpr int NOWN = (L * L + NT - 1) / NT;
  constexpr int NCS = DIM == 3 ? 10 : 6;
  __shared__ CT tab[2][3][PP];             // [value/deriv][axis][q*P+a]
  __shared__ CT cs[NCS][L];
  __shared__ CT T1[4][DIM == 3 ? PP * PP : 1];   // [x1y1][q0 q1][a2 b2] (3D)
  __shared__ CT T2[DIM == 3 ? P * PP * PP : P * PP];
  const int t = threadIdx.x;
  int64_t e;
  if (MODE == EM_COLOR) {
    // color = (c0, c1, c2) with c_d in [0, P); element (c0 + P k0, c1 + P k1, c2 + P k2)
    int c0 = color % P, c1 = (color / P) % P, c2 = color / PP;
    int k0n = (pb.ne[0] - c0 + P - 1) / P, k1n = (pb.ne[1] - c1 + P - 1) / P;
    int64_t k = blockIdx.x;
    int k0 = (int)(k % k0n);
    int64_t r = k / k0n;
    int k1 = (int)(r % k1n);
    int k2 = (int)(r / k1n);
    int e0 = c0 + P * k0, e1 = c1 + P * k1, e2 = DIM == 3 ? c2 + P * k2 : 0;
    if (e0 >= pb.ne[0] || e1 >= pb.ne[1] || (DIM == 3 && e2 >= pb.ne[2])) return;
    e = e0 + (int64_t)pb.ne[0] * (e1 + (int64_t)pb.ne[1] * e2);
  } else if (elems) {
    e = elems[blockIdx.x];
  } else {
    e = blockIdx.x;
  }
  int em[3], f[3];
  elem_coords(pb, e, em);
  __shared__ double sW[3][P];
  for (int d = 0; d < DIM; ++d) {
    const double *B = pb.ax[d].B + (size_t)em[d] * PP, *D = pb.ax[d].dB + (size_t)em[d] * PP;
    for (int i = t; i < PP; i += NT) { tab[0][d][i] = (CT)B[i]; tab[1][d][i] = (CT)D[i]; }
    if (t < P) sW[d][t] = pb.ax[d].wq[(size_t)em[d] * P + t];
    f[d] = pb.ax[d].efirst[em[d]];
  }
  if (DIM == 2) f[2] = 0;
  __syncthreads();
  for (int q = t; q < L; q += NT) {
    double cv[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    point_coefs<DIM, TABLE>(pb, e, q, L, sW[0], sW[1], sW[2], lin, cv);
    for (int k = 0; k < NCS; ++k) cs[k][q] = (CT)cv[k];
  }
  const Term *terms = DIM == 3 ? (TABLE ? c_terms3_full : c_terms3_diag) : (TABLE ? c_terms2_full : c_terms2_diag);
  const int nterms = DIM == 3 ? (TABLE ? 16 : 4) : (TABLE ? 9 : 3);
  CT acc[NOWN];
#pragma unroll
  for (int k = 0; k < NOWN; ++k) acc[k] = 0;
  for (int c0 = 0; c0 < 4; ++c0) {
    const int x0 = c0 >> 1, y0 = c0 & 1;
    int any = 0;
    for (int ti = 0; ti < nterms; ++ti) any |= (terms[ti].x[0] == x0 && terms[ti].y[0] == y0);
    if (!any) continue;
    __syncthreads();
    if constexpr (DIM == 3) {
      // level 1: contract axis 2 -> T1[x1y1][q0 q1][a2 b2]
      for (int idx = t; idx < 4 * PP * PP; idx += NT) {
        int k1 = idx / (PP * PP), rem = idx % (PP * PP);
        int qq = rem / PP, ab = rem % PP, a2 = ab / P, b2 = ab % P;
        int x1 = k1 >> 1, y1 = k1 & 1;
        CT s = 0;
        for (int ti = 0; ti < nterms; ++ti) {
          const Term &T = terms[ti];
          if (T.x[0] != x0 || T.y[0] != y0 || T.x[1] != x1 || T.y[1] != y1) continue;
          const CT *X = tab[T.x[2]][2], *Yt = tab[T.y[2]][2];
          const CT *cc = cs[T.coef] + qq;
#pragma unroll
          for (int q2 = 0; q2 < P; ++q2) s += cc[q2 * PP] * X[q2 * P + a2] * Yt[q2 * P + b2];
        }
        T1[k1][rem] = s;
      }
      __syncthreads();
      // level 2: contract axis 1 -> T2[q0][a1 b1][a2 b2]
      int mask1 = 0;
      for (int ti = 0; ti < nterms; ++ti)
        if (terms[ti].x[0] == x0 && terms[ti].y[0] == y0) mask1 |= 1 << (terms[ti].x[1] * 2 + terms[ti].y[1]);
      for (int idx = t; idx < P * PP * PP; idx += NT) {
        int q0 = idx / (PP * PP), rem = idx % (PP * PP);
        int a1b1 = rem / PP, a2b2 = rem % PP, a1 = a1b1 / P, b1 = a1b1 % P;
        CT s = 0;
        for (int k1 = 0; k1 < 4; ++k1) {
          if (!((mask1 >> k1) & 1)) continue;
          const CT *X = tab[k1 >> 1][1], *Yt = tab[k1 & 1][1];
#pragma unroll
          for (int q1 = 0; q1 < P; ++q1)
            s += X[q1 * P + a1] * Yt[q1 * P + b1] * T1[k1][(q0 + P * q1) * PP + a2b2];
        }
        T2[idx] = s;
      }
      __syncthreads();
      // level 3: contract axis 0 into the owned entries
      const CT *X = tab[x0][0], *Yt = tab[y0][0];
#pragma unroll
      for (int k = 0; k < NOWN; ++k) {
        int idx = t + k * NT;
        if (idx < L * L) {
          int a = idx / L, b = idx % L;
          int a0 = a % P, a1 = (a / P) % P, a2 = a / PP;
          int b0 = b % P, b1 = (b / P) % P, b2 = b / PP;
          int off = (a1 * P + b1) * PP + a2 * P + b2;
          CT s = 0;
#pragma unroll
          for (int q0 = 0; q0 < P; ++q0) s += X[q0 * P + a0] * Yt[q0 * P + b0] * T2[q0 * PP * PP + off];
          acc[k] += s;
        }
      }
    } else {
      // level 1: contract axis 1 -> T2[q0][a1 b1]
      for (int idx = t; idx < P * PP; idx += NT) {
        int q0 = idx / PP, ab = idx % PP, a1 = ab / P, b1 = ab % P;
        CT s = 0;
        for (int ti = 0; ti < nterms; ++ti) {
          const Term &T = terms[ti];
          if (T.x[0] != x0 || T.y[0] != y0) continue;
          const CT *X = tab[T.x[1]][1], *Yt = tab[T.y[1]][1];
#pragma unroll
          for (int q1 = 0; q1 < P; ++q1) s += cs[T.coef][q0 + P * q1] * X[q1 * P + a1] * Yt[q1 * P + b1];
        }
        T2[idx] = s;
      }
      __syncthreads();
      const CT *X = tab[x0][0], *Yt = tab[y0][0];
#pragma unroll
      for (int k = 0; k < NOWN; ++k) {
        int idx = t + k * NT;
        if (idx < L * L) {
          int a = idx / L, b = idx % L;
          int a0 = a % P, a1 = a / P, b0 = b % P, b1 = b / P;
          CT s = 0;
#pragma unroll
          for (int q0 = 0; q0 < P; ++q0) s += X[q0 * P + a0] * Yt[q0 * P + b0] * T2[q0 * PP + a1 * P + b1];
          acc[k] += s;
        }
      }
    }
  }
  // ---- output ----
#pragma unroll
  for (int k = 0; k < NOWN; ++k) {
    int idx = t + k * NT;
    if (idx >= L * L) continue;
    int a = idx / L, b = idx % L;
    int64_t A = local_to_global<DIM, P>(pb, f, a), Bg = local_to_global<DIM, P>(pb, f, b);
    double v = (double)acc[k];
    if (TABLE && pb.rational) v *= pb.wts[A] * pb.wts[Bg];
    if (MODE == EM_OUT) {
      ((double *)outp)[(size_t)blockIdx.x * L * L + idx] = v;
      continue;
    }
    int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / PP : 0;
    int b0 = b % P, b1 = (b / P) % P, b2 = DIM == 3 ? b / PP : 0;
    int i0 = wrap_fn(pb.ax[0], f[0] + a0), i1 = wrap_fn(pb.ax[1], f[1] + a1), i2 = DIM == 3 ? wrap_fn(pb.ax[2], f[2] + a2) : 0;
    int j0 = wrap_fn(pb.ax[0], f[0] + b0), j1 = wrap_fn(pb.ax[1], f[1] + b1), j2 = DIM == 3 ? wrap_fn(pb.ax[2], f[2] + b2) : 0;
    if (is_dirichlet_idx(pb, i0, i1, i2) || is_dirichlet_idx(pb, j0, j1, j2)) continue;
    int64_t slot = csr_slot(pb, i0, i1, i2, j0, j1, j2);
    if (MODE == EM_ATOMIC) {
      if (std::is_same<CT, float>::value) atomicAdd(&((float *)outp)[slot], (float)v);
      else atomicAdd(&((double *)outp)[slot], v);
    } else {
      if (std::is_same<CT, float>::value) ((float *)outp)[slot] += (float)v;
      else ((double *)outp)[slot] += v;
    }
  }
}

// ------------------------------------------------------------------------------------------
// Local numerical differentiation (Sec. 2.8, eq:fdjac).  Column k of element e's matrix is
// sum_q (F_q(U_e + delta e_k) - F_q(U_e)) / delta with delta = eta sqrt(1 + ||U_e||_2), where
// F_q is the point's contribution to the element residual (the integrand of eq:residual tested
// with every local function).  The difference is taken on the point flux and source before the
// test functions are applied (the same sum in exact arithmetic); the perturbed state is
// u + delta N_k (its exponential from the base point's, exp_near), and the column is contracted
// by the transposed sum factorisation of the residual
// kernel.  One workgroup per element, four columns in flight (one wave each).  Columns are kept
// in LDS in chunks of KC and each chunk is added into the CSR values with FP64 atomics (FP32
// values: FP32 atomics of the FP64 result) in one pass, so the workgroup barriers inside the
// column loop never wait for outstanding atomics.
// ------------------------------------------------------------------------------------------
// exp(arg) from exp(arg0): the perturbed exponent differs by x = arg - arg0, exactly
// representable, |x| <~ 1e-7 here, so e^x = 1 + x + x^2/2 + x^3/6 to within x^4/24; a larger x
// (huge ||U_e||) takes the library exp
__device__ inline double exp_near(double arg, double arg0, double e0) {
  const double x = arg - arg0;
  if (fabs(x) > 1e-3) return exp(arg);
  return e0 + e0 * (x * (1.0 + x * (0.5 + x * (1.0 / 6.0))));
}

// point flux F and source term S of eq:residual at state (val, gu); with arg0 / e0 given, the
// exponential is formed from the base point's (exp_near)
template <int DIM, bool TABLE>
__device__ inline void nd_point(const DevProblem &pb, int64_t e, int q, int L, const double *sW0, const double *sW1,
                                const double *sW2, double kap_e, double val, const double gu[3], double f,
                                double Fv[3], double &Sv, bool near = false, double arg0 = 0.0, double e0 = 0.0,
                                double *arg_out = nullptr) {
  const double lam = pb.lambda;
  const bool src = pb.src != nullptr;
  if constexpr (!TABLE) {
    const int Q = pb.Q;
    const int q0 = q % Q, q1 = (q / Q) % Q, q2 = DIM == 3 ? q / (Q * Q) : 0;
    const double W = sW0[q0] * sW1[q1] * (DIM == 3 ? sW2[q2] : 1.0);
    const double kw = kap_e * W;
    for (int k = 0; k < DIM; ++k) Fv[k] = kw * gu[k];
    if (arg_out) *arg_out = val;
    Sv = -W * (lam * (near ? exp_near(val, arg0, e0) : exp(val)) + (src ? f : 0.0));
  } else {
    constexpr int NG = geo_streams(DIM);
    const double *G = pb.geo + (size_t)e * NG * L + q;
    double Dm[3][3], g[3] = {0, 0, 0}, Wow, iw;
    if (DIM == 3) {
      Dm[0][0] = G[0]; Dm[1][1] = G[L]; Dm[2][2] = G[2 * L];
      Dm[0][1] = Dm[1][0] = G[3 * L]; Dm[0][2] = Dm[2][0] = G[4 * L]; Dm[1][2] = Dm[2][1] = G[5 * L];
      g[0] = G[6 * L]; g[1] = G[7 * L]; g[2] = G[8 * L];
      Wow = G[9 * L]; iw = G[10 * L];
    } else {
      Dm[0][0] = G[0]; Dm[1][1] = G[L]; Dm[0][1] = Dm[1][0] = G[2 * L];
      g[0] = G[3 * L]; g[1] = G[4 * L];
      Wow = G[5 * L]; iw = G[6 * L];
    }
    double gv[3];
    for (int k = 0; k < DIM; ++k) gv[k] = gu[k] - val * g[k];
    double gF = 0;
    for (int k = 0; k < DIM; ++k) {
      double s = 0;
      for (int m = 0; m < DIM; ++m) s += Dm[k][m] * gv[m];
      Fv[k] = s;
      gF += g[k] * s;
    }
    const double arg = val * iw;
    if (arg_out) *arg_out = arg;
    Sv = -Wow * (lam * (near ? exp_near(arg, arg0, e0) : exp(arg)) + (src ? f * iw : 0.0)) - gF;
  }
}

template <int DIM, int P, bool TABLE>
__global__ void __launch_bounds__(256) k_elem_nd(DevProblem pb, const double *__restrict__ U, double eta,
                                                 void *__restrict__ vals, int f32, int color) {
  constexpr int L = Shp<DIM, P>::L, PP = P * P;
  constexpr int NGRP = 4;   // columns in flight, one wave each
  constexpr int L4 = (L + 3) / 4 * 4, KCM = (4096 / L) / 4 * 4;
  constexpr int KC = L4 < KCM ? L4 : KCM;   // columns per LDS chunk (multiple of 4)
  __shared__ double Ke[L * KC];
  __shared__ double sB[3][PP], sD[3][PP], sW[3][P];
  __shared__ double c[L], cf[L], su[L], sg[3][L], sfq[L], Fb[3][L], Sb[L], sA[L], sE[L];
  __shared__ double buf[NGRP][7][L];
  __shared__ double sh[4];
  const int t = threadIdx.x, grp = t >> 6, lane = t & 63;
  int64_t e = blockIdx.x;
  if (color >= 0) {
    // colour (c0, c1, c2), c_d < P: elements (c0 + P k0, c1 + P k1, c2 + P k2) share no function
    const int c0 = color % P, c1 = (color / P) % P, c2 = color / PP;
    const int k0n = (pb.ne[0] - c0 + P - 1) / P, k1n = (pb.ne[1] - c1 + P - 1) / P;
    const int64_t kk = blockIdx.x;
    const int k0 = (int)(kk % k0n);
    const int64_t r = kk / k0n;
    const int e0 = c0 + P * k0, e1 = c1 + P * (int)(r % k1n), e2 = DIM == 3 ? c2 + P * (int)(r / k1n) : 0;
    if (e0 >= pb.ne[0] || e1 >= pb.ne[1] || (DIM == 3 && e2 >= pb.ne[2])) return;
    e = e0 + (int64_t)pb.ne[0] * (e1 + (int64_t)pb.ne[1] * e2);
  }
  int em[3], f[3];
  elem_coords(pb, e, em);
  for (int d = 0; d < DIM; ++d) {
    const double *B = pb.ax[d].B + (size_t)em[d] * PP, *D = pb.ax[d].dB + (size_t)em[d] * PP;
    for (int i = t; i < PP; i += 256) { sB[d][i] = B[i]; sD[d][i] = D[i]; }
    if (t < P) sW[d][t] = pb.ax[d].wq[(size_t)em[d] * P + t];
    f[d] = pb.ax[d].efirst[em[d]];
  }
  if (DIM == 2) f[2] = 0;
  const bool src = pb.src != nullptr;
  double nrm = 0;
  for (int a = t; a < L; a += 256) {
    const int64_t A = local_to_global<DIM, P>(pb, f, a);
    const double wa = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
    const double x = U[A];
    nrm += x * x;
    c[a] = x * wa;
    cf[a] = src ? pb.src[A] * wa : 0.0;
  }
  for (int o = 32; o > 0; o >>= 1) nrm += __shfl_xor(nrm, o, 64);
  if (lane == 0) sh[grp] = nrm;
  __syncthreads();
  const double delta = eta * sqrt(1.0 + sqrt(sh[0] + sh[1] + sh[2] + sh[3]));
  // state at the points: value and parametric gradient of the (homogeneous) field, source
  double *y0 = buf[0][0], *y1 = buf[0][1], *y2 = buf[0][2], *y3 = buf[0][3], *y4 = buf[0][4], *y5 = buf[0][5];
  if constexpr (DIM == 3) {
    fwd<PP, 1, P>(c, y0, sB[0], t, 256);
    fwd<PP, 1, P>(c, y1, sD[0], t, 256);
    fwd<PP, 1, P>(cf, y5, sB[0], t, 256);
    __syncthreads();
    fwd<P, P, P>(y0, y2, sB[1], t, 256);
    fwd<P, P, P>(y1, y3, sB[1], t, 256);
    fwd<P, P, P>(y0, y4, sD[1], t, 256);
    fwd<P, P, P>(y5, buf[1][0], sB[1], t, 256);
    __syncthreads();
    fwd<1, PP, P>(y2, su, sB[2], t, 256);
    fwd<1, PP, P>(y3, sg[0], sB[2], t, 256);
    fwd<1, PP, P>(y4, sg[1], sB[2], t, 256);
    fwd<1, PP, P>(y2, sg[2], sD[2], t, 256);
    fwd<1, PP, P>(buf[1][0], sfq, sB[2], t, 256);
  } else {
    fwd<P, 1, P>(c, y0, sB[0], t, 256);
    fwd<P, 1, P>(c, y1, sD[0], t, 256);
    fwd<P, 1, P>(cf, y5, sB[0], t, 256);
    __syncthreads();
    fwd<1, P, P>(y0, su, sB[1], t, 256);
    fwd<1, P, P>(y1, sg[0], sB[1], t, 256);
    fwd<1, P, P>(y0, sg[1], sD[1], t, 256);
    fwd<1, P, P>(y5, sfq, sB[1], t, 256);
  }
  __syncthreads();
  const double kap_e = (!TABLE && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
  for (int q = t; q < L; q += 256) {
    double gq[3] = {sg[0][q], sg[1][q], DIM == 3 ? sg[2][q] : 0.0}, Fv[3] = {0, 0, 0}, Sv = 0, arg = 0;
    nd_point<DIM, TABLE>(pb, e, q, L, sW[0], sW[1], sW[2], kap_e, su[q], gq, sfq[q], Fv, Sv, false, 0.0, 0.0, &arg);
    for (int k = 0; k < DIM; ++k) Fb[k][q] = Fv[k];
    Sb[q] = Sv;
    sA[q] = arg;
    sE[q] = exp(arg);
  }
  __syncthreads();
  for (int cs = 0; cs < L; cs += KC) {
  const int ce = min(L, cs + KC);
  for (int kb = cs; kb < ce; kb += NGRP) {
    const int k = kb + grp;
    const bool ok = k < ce;
    double *dF0 = buf[grp][0], *dF1 = buf[grp][1], *dF2 = buf[grp][2], *dS = buf[grp][3];
    if (ok) {
      const int k0 = k % P, k1 = (k / P) % P, k2 = DIM == 3 ? k / PP : 0;
      const int64_t Ak = local_to_global<DIM, P>(pb, f, k);
      const double dc = delta * ((TABLE && pb.rational) ? pb.wts[Ak] : 1.0);
      for (int q = lane; q < L; q += 64) {
        const int q0 = q % P, q1 = (q / P) % P, q2 = DIM == 3 ? q / PP : 0;
        const double b0 = sB[0][q0 * P + k0], b1 = sB[1][q1 * P + k1], b2 = DIM == 3 ? sB[2][q2 * P + k2] : 1.0;
        const double d0 = sD[0][q0 * P + k0], d1 = sD[1][q1 * P + k1], d2 = DIM == 3 ? sD[2][q2 * P + k2] : 0.0;
        double gq[3] = {sg[0][q] + dc * d0 * b1 * b2, sg[1][q] + dc * b0 * d1 * b2,
                        DIM == 3 ? sg[2][q] + dc * b0 * b1 * d2 : 0.0};
        double Fv[3] = {0, 0, 0}, Sv = 0;
        nd_point<DIM, TABLE>(pb, e, q, L, sW[0], sW[1], sW[2], kap_e, su[q] + dc * b0 * b1 * b2, gq, sfq[q], Fv,
                             Sv, true, sA[q], sE[q]);
        dF0[q] = (Fv[0] - Fb[0][q]) / delta;
        dF1[q] = (Fv[1] - Fb[1][q]) / delta;
        if (DIM == 3) dF2[q] = (Fv[2] - Fb[2][q]) / delta;
        dS[q] = (Sv - Sb[q]) / delta;
      }
    }
    __syncthreads();
    double *Re;
    if constexpr (DIM == 3) {
      double *Sa = buf[grp][4], *S0 = buf[grp][5], *S1 = buf[grp][6];
      if (ok) {
        bwd2<1, PP, P>(dF2, sD[2], dS, sB[2], Sa, lane, 64);
        bwd2<1, PP, P>(dF0, sB[2], (const double *)nullptr, sB[2], S0, lane, 64);
        bwd2<1, PP, P>(dF1, sB[2], (const double *)nullptr, sB[2], S1, lane, 64);
      }
      __syncthreads();
      double *VB = buf[grp][0], *V0 = buf[grp][1];
      if (ok) {
        bwd2<P, P, P>(S1, sD[1], Sa, sB[1], VB, lane, 64);
        bwd2<P, P, P>(S0, sB[1], (const double *)nullptr, sB[1], V0, lane, 64);
      }
      __syncthreads();
      Re = buf[grp][2];
      if (ok) bwd2<PP, 1, P>(V0, sD[0], VB, sB[0], Re, lane, 64);
    } else {
      double *Sa = buf[grp][4], *S0 = buf[grp][5];
      if (ok) {
        bwd2<1, P, P>(dF1, sD[1], dS, sB[1], Sa, lane, 64);
        bwd2<1, P, P>(dF0, sB[1], (const double *)nullptr, sB[1], S0, lane, 64);
      }
      __syncthreads();
      Re = buf[grp][2];
      if (ok) bwd2<P, 1, P>(S0, sD[0], Sa, sB[0], Re, lane, 64);
    }
    __syncthreads();
    if (ok)
      for (int a = lane; a < L; a += 64) Ke[a * KC + (k - cs)] = Re[a];
    __syncthreads();
  }
  // add the chunk's columns: consecutive threads on consecutive columns of one row
  const int nc = ce - cs;
  for (int i = t; i < L * nc; i += 256) {
    const int a = i / nc, k = cs + i % nc;
    const int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / PP : 0;
    const int k0 = k % P, k1 = (k / P) % P, k2 = DIM == 3 ? k / PP : 0;
    const int i0 = wrap_fn(pb.ax[0], f[0] + a0), i1 = wrap_fn(pb.ax[1], f[1] + a1);
    const int i2 = DIM == 3 ? wrap_fn(pb.ax[2], f[2] + a2) : 0;
    const int j0 = wrap_fn(pb.ax[0], f[0] + k0), j1 = wrap_fn(pb.ax[1], f[1] + k1);
    const int j2 = DIM == 3 ? wrap_fn(pb.ax[2], f[2] + k2) : 0;
    if (is_dirichlet_idx(pb, i0, i1, i2) || is_dirichlet_idx(pb, j0, j1, j2)) continue;
    double v = Ke[a * KC + (k - cs)];
    if (TABLE && pb.rational) v *= pb.wts[local_to_global<DIM, P>(pb, f, a)];
    const int64_t slot = csr_slot(pb, i0, i1, i2, j0, j1, j2);
    if (color >= 0) {
      // no other workgroup of this launch touches the slot
      if (f32) ((float *)vals)[slot] += (float)v;
      else ((double *)vals)[slot] += v;
    } else {
      if (f32) atomicAdd(&((float *)vals)[slot], (float)v);
      else atomicAdd(&((double *)vals)[slot], v);
    }
  }
  if (ce < L) __syncthreads();
  }
}

// Dirichlet rows of an assembled Jacobian become identity rows (entries were never written).
template <typename VT>
__global__ void k_bc_diag(DevProblem pb, VT *vals) {
  int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (A >= pb.N) return;
  int i0 = (int)(A % pb.n[0]);
  int64_t r = A / pb.n[0];
  int i1 = (int)(r % pb.n[1]);
  int i2 = (int)(r / pb.n[1]);
  if (is_dirichlet_idx(pb, i0, i1, i2)) vals[csr_slot(pb, i0, i1, i2, i0, i1, i2)] = (VT)1;
}

// Diagonal of the Jacobian for the matrix-free Jacobi preconditioner: per element,
// diag_a = sum_terms sum_q coef_t(q) prod_d X_d(a_d,q_d) Y_d(a_d,q_d), sum-factorised.
template <int DIM, int P, bool TABLE>
__global__ void __launch_bounds__(64) k_elem_diag(DevProblem pb, const double *__restrict__ lin,
                                                  double *__restrict__ diag) {
  constexpr int L = Shp<DIM, P>::L, PP = P * P;
  constexpr int NCS = DIM == 3 ? 10 : 6;
  __shared__ double tab[2][3][PP], sW[3][P];
  __shared__ double cs[NCS][L];
  __shared__ double t1[L], t2[L], acc[L];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  int em[3], f[3];
  elem_coords(pb, e, em);
  for (int d = 0; d < DIM; ++d) {
    const double *B = pb.ax[d].B + (size_t)em[d] * PP, *D = pb.ax[d].dB + (size_t)em[d] * PP;
    for (int i = t; i < PP; i += 64) { tab[0][d][i] = B[i]; tab[1][d][i] = D[i]; }
    if (t < P) sW[d][t] = pb.ax[d].wq[(size_t)em[d] * P + t];
    f[d] = pb.ax[d].efirst[em[d]];
  }
  if (DIM == 2) f[2] = 0;
  __syncthreads();
  for (int q = t; q < L; q += 64) {
    double cv[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    point_coefs<DIM, TABLE>(pb, e, q, L, sW[0], sW[1], sW[2], lin, cv);
    for (int k = 0; k < NCS; ++k) cs[k][q] = cv[k];
    acc[q] = 0;
  }
  __syncthreads();
  const Term *terms = DIM == 3 ? (TABLE ? c_terms3_full : c_terms3_diag) : (TABLE ? c_terms2_full : c_terms2_diag);
  const int nterms = DIM == 3 ? (TABLE ? 16 : 4) : (TABLE ? 9 : 3);
  for (int ti = 0; ti < nterms; ++ti) {
    const Term T = terms[ti];
    if constexpr (DIM == 3) {
      // [q2][q1][q0] -> [a2][q1][q0] -> [a2][a1][q0] -> [a2][a1][a0]
      for (int idx = t; idx < L; idx += 64) {
        int l = idx % PP, a2 = idx / PP;
        double s = 0;
        for (int q2 = 0; q2 < P; ++q2) s += tab[T.x[2]][2][q2 * P + a2] * tab[T.y[2]][2][q2 * P + a2] * cs[T.coef][q2 * PP + l];
        t1[idx] = s;
      }
      __syncthreads();
      for (int idx = t; idx < L; idx += 64) {
        int q0 = idx % P, a1 = (idx / P) % P, a2 = idx / PP;
        double s = 0;
        for (int q1 = 0; q1 < P; ++q1) s += tab[T.x[1]][1][q1 * P + a1] * tab[T.y[1]][1][q1 * P + a1] * t1[a2 * PP + q1 * P + q0];
        t2[idx] = s;
      }
      __syncthreads();
      for (int idx = t; idx < L; idx += 64) {
        int a0 = idx % P, rest = idx / P;
        double s = 0;
        for (int q0 = 0; q0 < P; ++q0) s += tab[T.x[0]][0][q0 * P + a0] * tab[T.y[0]][0][q0 * P + a0] * t2[rest * P + q0];
        acc[idx] += s;
      }
      __syncthreads();
    } else {
      for (int idx = t; idx < L; idx += 64) {
        int q0 = idx % P, a1 = idx / P;
        double s = 0;
        for (int q1 = 0; q1 < P; ++q1) s += tab[T.x[1]][1][q1 * P + a1] * tab[T.y[1]][1][q1 * P + a1] * cs[T.coef][q1 * P + q0];
        t1[idx] = s;
      }
      __syncthreads();
      for (int idx = t; idx < L; idx += 64) {
        int a0 = idx % P, a1 = idx / P;
        double s = 0;
        for (int q0 = 0; q0 < P; ++q0) s += tab[T.x[0]][0][q0 * P + a0] * tab[T.y[0]][0][q0 * P + a0] * t1[a1 * P + q0];
        acc[idx] += s;
      }
      __syncthreads();
    }
  }
  for (int a = t; a < L; a += 64) {
    int64_t A = local_to_global<DIM, P>(pb, f, a);
    double wa = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
    atomicAdd(&diag[A], acc[a] * wa * wa);
  }
}

__global__ void k_diag_bc_invert(DevProblem pb, double *d) {
  int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (A >= pb.N) return;
  d[A] = is_dirichlet(pb, A) ? 1.0 : 1.0 / d[A];
}

// ------------------------------------------------------------------------------------------
// Dispatch helpers
// ------------------------------------------------------------------------------------------
template <template <int, int, bool> class F, typename... Args>
iga_status dispatch_dpt(const Handle &h, Args &&...args) {
  const DevProblem &pb = h.pb;
  const bool T = pb.table != 0;
#define IGA_CASE(D, PP_)                                                   \
  if (pb.dim == D && pb.P == PP_) {                                        \
    if (T) F<D, PP_, true>::run(h, args...);                               \
    else F<D, PP_, false>::run(h, args...);                                \
    return IGA_OK;                                                         \
  }
  IGA_CASE(3, 2) IGA_CASE(3, 3) IGA_CASE(3, 4) IGA_CASE(3, 5)
  IGA_CASE(2, 2) IGA_CASE(2, 3) IGA_CASE(2, 4) IGA_CASE(2, 5) IGA_CASE(2, 6) IGA_CASE(2, 7)
#undef IGA_CASE
  return fail(IGA_EUNSUPPORTED, "degree/dimension combination not compiled (3D needs p <= 4)");
}

template <int D, int P, bool T>
struct RunRes {
  static void run(const Handle &h, const double *U, double *R) {
    hipLaunchKernelGGL((k_elem_op<D, P, T, OP_RES>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, U,
                       (double *)nullptr, R);
  }
};
template <int D, int P, bool T>
struct RunLin {
  static void run(const Handle &h, const double *U) {
    hipLaunchKernelGGL((k_elem_op<D, P, T, OP_LIN>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, U, h.lin,
                       (double *)nullptr);
  }
};
template <int D, int P, bool T>
struct RunApply {
  static void run(const Handle &h, const double *v, double *y) {
    hipLaunchKernelGGL((k_elem_op<D, P, T, OP_APPLY>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, v,
                       h.lin, y);
  }
};
template <int D, int P, bool T>
struct RunDiag {
  static void run(const Handle &h, double *dg) {
    hipLaunchKernelGGL((k_elem_diag<D, P, T>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, h.lin, dg);
  }
};
template <int D, int P, bool T>
struct RunElemMat {
  static void run(const Handle &h, const int32_t *elems, int n, int prec, int mode, int color, unsigned nblk,
                  void *out) {
    if constexpr (D == 3 && P > 5) {
      return;
    } else {
      if (prec == IGA_FP32) {
        if (mode == EM_OUT)
          hipLaunchKernelGGL((k_elem_mat<D, P, T, float, EM_OUT>), dim3(nblk), dim3(256), 0, h.stream, h.pb, h.lin,
                             elems, color, out);
        else if (mode == EM_ATOMIC)
          hipLaunchKernelGGL((k_elem_mat<D, P, T, float, EM_ATOMIC>), dim3(nblk), dim3(256), 0, h.stream, h.pb,
                             h.lin, elems, color, out);
        else
          hipLaunchKernelGGL((k_elem_mat<D, P, T, float, EM_COLOR>), dim3(nblk), dim3(256), 0, h.stream, h.pb,
                             h.lin, elems, color, out);
      } else {
        if (mode == EM_OUT)
          hipLaunchKernelGGL((k_elem_mat<D, P, T, double, EM_OUT>), dim3(nblk), dim3(256), 0, h.stream, h.pb, h.lin,
                             elems, color, out);
        else if (mode == EM_ATOMIC)
          hipLaunchKernelGGL((k_elem_mat<D, P, T, double, EM_ATOMIC>), dim3(nblk), dim3(256), 0, h.stream, h.pb,
                             h.lin, elems, color, out);
        else
          hipLaunchKernelGGL((k_elem_mat<D, P, T, double, EM_COLOR>), dim3(nblk), dim3(256), 0, h.stream, h.pb,
                             h.lin, elems, color, out);
      }
    }
    (void)n;
  }
};

template <int D, int P, bool T>
struct RunElemND {
  static void run(const Handle &h, const double *U, double eta, void *vals, int f32, int color, unsigned nblk) {
    if constexpr (D == 3 && P > 5) {
      return;
    } else {
      hipLaunchKernelGGL((k_elem_nd<D, P, T>), dim3(nblk), dim3(256), 0, h.stream, h.pb, U, eta, vals, f32, color);
    }
  }
};

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

iga_status launch_fill(Handle &h, double *x, int64_t n, double v) {
  if (n <= 0) return IGA_OK;
  hipLaunchKernelGGL(k_fill, dim3(blocks_for(n, 256)), dim3(256), 0, h.stream, x, n, v);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_residual(Handle &h, const double *U, double *R) {
  iga_status st = launch_fill(h, R, h.pb.N, 0.0);
  if (st) return st;
  if (res2_supported(h.pb)) st = launch_res2(h, U, R);
  else if (res3_supported(h.pb) && h.tiled_3d) st = launch_res3(h, U, R, 0);
  else st = dispatch_dpt<RunRes>(h, U, R);
  if (st) return st;
  hipLaunchKernelGGL(k_bc_copy, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb, U, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_linearize(Handle &h, const double *U) {
  iga_status st = (res3_supported(h.pb) && h.tiled_3d) ? launch_res3(h, U, h.lin, 2) : dispatch_dpt<RunLin>(h, U);
  if (st) return st;
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_apply(Handle &h, const double *v, double *y) {
  iga_status st = launch_fill(h, y, h.pb.N, 0.0);
  if (st) return st;
  if (res3_supported(h.pb) && h.tiled_3d) st = launch_res3(h, v, y, 1);
  else st = dispatch_dpt<RunApply>(h, v, y);
  if (st) return st;
  hipLaunchKernelGGL(k_bc_copy, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb, v, y);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_diag_mf(Handle &h, double *diag) {
  iga_status st = launch_fill(h, diag, h.pb.N, 0.0);
  if (st) return st;
  if ((st = dispatch_dpt<RunDiag>(h, diag))) return st;
  hipLaunchKernelGGL(k_diag_bc_invert, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb, diag);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_elem_matrices(Handle &h, const double *U, const int32_t *elems, int n, int prec, double *out) {
  if (h.pb.dim == 3 && h.pb.P > 5) return fail(IGA_EUNSUPPORTED, "element matrices need p <= 4 in 3D");
  iga_status st = launch_linearize(h, U);
  if (st) return st;
  if ((st = dispatch_dpt<RunElemMat>(h, elems, n, prec, (int)EM_OUT, 0, (unsigned)n, (void *)out))) return st;
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_jac_scatter(Handle &h, const double *U, void *vals, int prec, int color_mode) {
  if (h.pb.dim == 3 && h.pb.P > 5) return fail(IGA_EUNSUPPORTED, "element matrices need p <= 4 in 3D");
  iga_status st = launch_linearize(h, U);
  if (st) return st;
  const int64_t nnz = h.pb.nnz;
  if (prec == IGA_FP32)
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(nnz, 256)), dim3(256), 0, h.stream, (float *)vals, nnz, 0.0f);
  else
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(nnz, 256)), dim3(256), 0, h.stream, (double *)vals, nnz, 0.0);
  if (!color_mode) {
    if ((st = dispatch_dpt<RunElemMat>(h, (const int32_t *)nullptr, 0, prec, (int)EM_ATOMIC, 0,
                                       (unsigned)h.pb.E, vals)))
      return st;
  } else {
    const int P = h.pb.P, ncol = ipow(P, h.pb.dim);
    for (int c = 0; c < ncol; ++c) {
      int c0 = c % P, c1 = (c / P) % P, c2 = c / (P * P);
      int64_t k0 = (h.pb.ne[0] - c0 + P - 1) / P, k1 = (h.pb.ne[1] - c1 + P - 1) / P;
      int64_t k2 = h.pb.dim == 3 ? (h.pb.ne[2] - c2 + P - 1) / P : 1;
      if (k0 <= 0 || k1 <= 0 || k2 <= 0) continue;
      if ((st = dispatch_dpt<RunElemMat>(h, (const int32_t *)nullptr, 0, prec, (int)EM_COLOR, c,
                                         (unsigned)(k0 * k1 * k2), vals)))
        return st;
    }
  }
  if (prec == IGA_FP32)
    hipLaunchKernelGGL(k_bc_diag<float>, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb, (float *)vals);
  else
    hipLaunchKernelGGL(k_bc_diag<double>, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb,
                       (double *)vals);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// Jacobian by local numerical differentiation: zero the values, add every element's difference
// columns, then the identity Dirichlet rows.
iga_status launch_jac_nd(Handle &h, const double *U, void *vals, int prec, int color_mode) {
  if (h.pb.dim == 3 && h.pb.P > 5) return fail(IGA_EUNSUPPORTED, "local numerical differentiation needs p <= 4 in 3D");
  const int64_t nnz = h.pb.nnz;
  const int f32 = prec == IGA_FP32 ? 1 : 0;
  if (f32)
    hipLaunchKernelGGL(k_fill_f, dim3(blocks_for(nnz, 256)), dim3(256), 0, h.stream, (float *)vals, nnz, 0.0f);
  else
    hipLaunchKernelGGL(k_fill, dim3(blocks_for(nnz, 256)), dim3(256), 0, h.stream, (double *)vals, nnz, 0.0);
  // eta = sqrt(machine epsilon), the default of Sec. 2.8
  const double eta = 1.4901161193847656e-08;
  iga_status st;
  if (!color_mode) {
    if ((st = dispatch_dpt<RunElemND>(h, U, eta, vals, f32, -1, (unsigned)h.pb.E))) return st;
  } else {
    const int P = h.pb.P, ncol = ipow(P, h.pb.dim);
    for (int c = 0; c < ncol; ++c) {
      const int c0 = c % P, c1 = (c / P) % P, c2 = c / (P * P);
      const int64_t k0 = (h.pb.ne[0] - c0 + P - 1) / P, k1 = (h.pb.ne[1] - c1 + P - 1) / P;
      const int64_t k2 = h.pb.dim == 3 ? (h.pb.ne[2] - c2 + P - 1) / P : 1;
      if (k0 <= 0 || k1 <= 0 || k2 <= 0) continue;
      if ((st = dispatch_dpt<RunElemND>(h, U, eta, vals, f32, c, (unsigned)(k0 * k1 * k2)))) return st;
    }
  }
  if (f32)
    hipLaunchKernelGGL(k_bc_diag<float>, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb, (float *)vals);
  else
    hipLaunchKernelGGL(k_bc_diag<double>, dim3(blocks_for(h.pb.N, 256)), dim3(256), 0, h.stream, h.pb,
                       (double *)vals);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

}  // namespace iga
