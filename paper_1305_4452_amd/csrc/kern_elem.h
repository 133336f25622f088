// Element-operator kernel bodies shared by the single-problem and batched launchers.
#pragma once

#include "iga_impl.h"

namespace iga {
namespace ek {

template <int DIM, int P>
struct Shp {
  static constexpr int Q = P;
  static constexpr int L = DIM == 3 ? P * P * P : P * P;   // functions = points per element
};

__device__ inline void elem_coords(const DevProblem &pb, int64_t e, int em[3]) {
  em[0] = (int)(e % pb.ne[0]);
  int64_t r = e / pb.ne[0];
  em[1] = (int)(r % pb.ne[1]);
  em[2] = (int)(r / pb.ne[1]);
}

template <int DIM, int P>
__device__ inline int64_t local_to_global(const DevProblem &pb, const int f[3], int a) {
  int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / (P * P) : 0;
  int64_t A = wrap_fn(pb.ax[0], f[0] + a0) +
              (int64_t)pb.n[0] * (wrap_fn(pb.ax[1], f[1] + a1) + (int64_t)pb.n[1] * (DIM == 3 ? wrap_fn(pb.ax[2], f[2] + a2) : 0));
  return A;
}

// out[h][q][l] = sum_a T[q][a] in[h][a][l]   (interpolation along one axis)
template <int NH, int NL, int P, typename T>
__device__ inline void fwd(const T *__restrict__ in, T *__restrict__ out, const T *__restrict__ tab, int t, int nt) {
  constexpr int NO = NH * P * NL;
  for (int idx = t; idx < NO; idx += nt) {
    int l = idx % NL, q = (idx / NL) % P, hh = idx / (NL * P);
    const T *x = in + hh * P * NL + l;
    const T *w = tab + q * P;
    T s = 0;
#pragma unroll
    for (int a = 0; a < P; ++a) s += w[a] * x[a * NL];
    out[idx] = s;
  }
}

// out[h][a][l] = sum_q T1[q][a] in1[h][q][l] + T2[q][a] in2[h][q][l]   (test functions)
template <int NH, int NL, int P, typename T>
__device__ inline void bwd2(const T *__restrict__ in1, const T *__restrict__ t1, const T *__restrict__ in2,
                            const T *__restrict__ t2, T *__restrict__ out, int t, int nt) {
  constexpr int NO = NH * P * NL;
  for (int idx = t; idx < NO; idx += nt) {
    int l = idx % NL, a = (idx / NL) % P, hh = idx / (NL * P);
    const T *x1 = in1 + hh * P * NL + l;
    T s = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) s += t1[q * P + a] * x1[q * NL];
    if (in2) {
      const T *x2 = in2 + hh * P * NL + l;
#pragma unroll
      for (int q = 0; q < P; ++q) s += t2[q * P + a] * x2[q * NL];
    }
    out[idx] = s;
  }
}

enum { OP_RES = 0, OP_APPLY = 1, OP_LIN = 2 };

// Residual (OP_RES), matrix-free Jacobian apply (OP_APPLY) and per-point linearisation
// coefficient (OP_LIN).  Rational bases are handled on the B-spline tensor structure:
// coefficients are multiplied by w_A, the geometry table supplies D' = kappa W Jinv Jinv^T/w^2,
// g = grad w / w, W/w and 1/w, and the tested result is multiplied by w_A again.
template <int DIM, int P, bool TABLE, int OP>
__device__ inline void elem_op_body(const DevProblem &pb, const int64_t e, const double *__restrict__ X,
                                    double *__restrict__ lin, double *__restrict__ Y) {
  constexpr int L = Shp<DIM, P>::L, PP = P * P;
  constexpr int NG = geo_streams(DIM);
  __shared__ double sB[3][PP], sD[3][PP], sW[3][P];
  __shared__ double buf[12][L];
  const int t = threadIdx.x;
  int em[3], f[3];
  elem_coords(pb, e, em);
  for (int d = 0; d < DIM; ++d) {
    const double *B = pb.ax[d].B + (size_t)em[d] * PP, *D = pb.ax[d].dB + (size_t)em[d] * PP;
    for (int i = t; i < PP; i += 64) { sB[d][i] = B[i]; sD[d][i] = D[i]; }
    if (t < P) sW[d][t] = pb.ax[d].wq[(size_t)em[d] * P + t];
    f[d] = pb.ax[d].efirst[em[d]];
  }
  if (DIM == 2) f[2] = 0;
  double *c = buf[0], *cf = buf[1];
  const bool want_src = (OP == OP_RES) && pb.src;
  for (int a = t; a < L; a += 64) {
    int64_t A = local_to_global<DIM, P>(pb, f, a);
    double wa = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
    double x = X[A];
    if (OP == OP_APPLY && is_dirichlet(pb, A)) x = 0.0;
    c[a] = x * wa;
    if (want_src) cf[a] = pb.src[A] * wa;
  }
  __syncthreads();
  // ---- interpolate to the quadrature points: value (and gradient) ----
  double *u = buf[2], *u0 = buf[3], *u1 = buf[4], *u2 = buf[5], *fq = buf[6];
  const bool grads = (OP != OP_LIN);
  if constexpr (DIM == 3) {
    double *yB = buf[7], *yD = buf[8], *zBB = buf[9], *zDB = buf[10], *zBD = buf[11];
    fwd<PP, 1, P>(c, yB, sB[0], t, 64);
    if (grads) fwd<PP, 1, P>(c, yD, sD[0], t, 64);
    __syncthreads();
    fwd<P, P, P>(yB, zBB, sB[1], t, 64);
    if (grads) {
      fwd<P, P, P>(yD, zDB, sB[1], t, 64);
      fwd<P, P, P>(yB, zBD, sD[1], t, 64);
    }
    __syncthreads();
    fwd<1, PP, P>(zBB, u, sB[2], t, 64);
    if (grads) {
      fwd<1, PP, P>(zDB, u0, sB[2], t, 64);
      fwd<1, PP, P>(zBD, u1, sB[2], t, 64);
      fwd<1, PP, P>(zBB, u2, sD[2], t, 64);
    }
    __syncthreads();
    if (want_src) {
      fwd<PP, 1, P>(cf, yB, sB[0], t, 64);
      __syncthreads();
      fwd<P, P, P>(yB, zBB, sB[1], t, 64);
      __syncthreads();
      fwd<1, PP, P>(zBB, fq, sB[2], t, 64);
      __syncthreads();
    }
  } else {
    double *yB = buf[7], *yD = buf[8];
    fwd<P, 1, P>(c, yB, sB[0], t, 64);
    if (grads) fwd<P, 1, P>(c, yD, sD[0], t, 64);
    __syncthreads();
    fwd<1, P, P>(yB, u, sB[1], t, 64);
    if (grads) {
      fwd<1, P, P>(yD, u0, sB[1], t, 64);
      fwd<1, P, P>(yB, u1, sD[1], t, 64);
    }
    __syncthreads();
    if (want_src) {
      fwd<P, 1, P>(cf, yB, sB[0], t, 64);
      __syncthreads();
      fwd<1, P, P>(yB, fq, sB[1], t, 64);
      __syncthreads();
    }
  }
  // ---- pointwise integrand ----
  double *F0 = buf[7], *F1 = buf[8], *F2 = buf[9], *S = buf[10];
  const double lam = pb.lambda;
  const double kap_e = (!TABLE && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
  for (int q = t; q < L; q += 64) {
    int q0 = q % P, q1 = (q / P) % P, q2 = DIM == 3 ? q / PP : 0;
    double gu[3] = {u0[q], u1[q], DIM == 3 ? u2[q] : 0.0};
    double val = u[q];
    double Fv[3] = {0, 0, 0}, Sv = 0;
    if constexpr (!TABLE) {
      double W = sW[0][q0] * sW[1][q1] * (DIM == 3 ? sW[2][q2] : 1.0);
      if (OP == OP_LIN) {
        lin[e * L + q] = -lam * W * exp(val);
        continue;
      }
      double kw = kap_e * W;
      for (int k = 0; k < DIM; ++k) Fv[k] = kw * gu[k];
      if (OP == OP_RES) Sv = -W * (lam * exp(val) + (want_src ? fq[q] : 0.0));
      else Sv = lin[e * L + q] * val;
    } else {
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
      if (OP == OP_LIN) {
        lin[e * L + q] = -lam * Wow * iw * exp(val * iw);
        continue;
      }
      double gv[3];
      for (int k = 0; k < DIM; ++k) gv[k] = gu[k] - val * g[k];
      for (int k = 0; k < DIM; ++k) {
        double s = 0;
        for (int m = 0; m < DIM; ++m) s += Dm[k][m] * gv[m];
        Fv[k] = s;
      }
      double gF = 0;
      for (int k = 0; k < DIM; ++k) gF += g[k] * Fv[k];
      if (OP == OP_RES) Sv = -Wow * (lam * exp(val * iw) + (want_src ? fq[q] * iw : 0.0)) - gF;
      else Sv = lin[e * L + q] * val - gF;
    }
    F0[q] = Fv[0];
    F1[q] = Fv[1];
    if (DIM == 3) F2[q] = Fv[2];
    S[q] = Sv;
  }
  if (OP == OP_LIN) return;
  __syncthreads();
  // ---- test with the basis (transposed sum factorisation) ----
  double *Re;
  if constexpr (DIM == 3) {
    double *Sa = buf[0], *S0 = buf[1], *S1 = buf[2], *VB = buf[3], *V0 = buf[4];
    bwd2<1, PP, P>(F2, sD[2], S, sB[2], Sa, t, 64);
    bwd2<1, PP, P>(F0, sB[2], (const double *)nullptr, sB[2], S0, t, 64);
    bwd2<1, PP, P>(F1, sB[2], (const double *)nullptr, sB[2], S1, t, 64);
    __syncthreads();
    bwd2<P, P, P>(S1, sD[1], Sa, sB[1], VB, t, 64);
    bwd2<P, P, P>(S0, sB[1], (const double *)nullptr, sB[1], V0, t, 64);
    __syncthreads();
    Re = buf[5];
    bwd2<PP, 1, P>(V0, sD[0], VB, sB[0], Re, t, 64);
  } else {
    double *Sa = buf[0], *S0 = buf[1];
    bwd2<1, P, P>(F1, sD[1], S, sB[1], Sa, t, 64);
    bwd2<1, P, P>(F0, sB[1], (const double *)nullptr, sB[1], S0, t, 64);
    __syncthreads();
    Re = buf[2];
    bwd2<P, 1, P>(S0, sD[0], Sa, sB[0], Re, t, 64);
  }
  __syncthreads();
  for (int a = t; a < L; a += 64) {
    int64_t A = local_to_global<DIM, P>(pb, f, a);
    double wa = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
    atomicAdd(&Y[A], Re[a] * wa);
  }
}

}  // namespace ek
}  // namespace iga
