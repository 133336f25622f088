// Tiled 3D residual and matrix-free Jacobian apply for the identity map (no weights, kappa one or
// element-wise, every interior knot simple, no source term; periodic axes wrap their indices).
//
// A workgroup owns TE^3 elements.  Over the whole tile, sum factorisation takes the coefficients
// of the tile's (TE + p)^3 functions to the value and gradient at its (TE Q)^3 Gauss points (three
// 1D contractions), forms the point flux F and source S of the weak form (Sec. 3):
//   residual: F = kappa W grad u, S = -lambda W e^u;
//   apply:    F = kappa W grad v, S = m v with m = -lambda W e^u cached per point,
// and the three transposed contractions give the tile's contribution to each of its functions,
//   R_A += sum_g F . grad N_A + S N_A,
// added to the output with one FP64 atomic per function (border functions are shared with the
// neighbouring tiles).  The output must be zeroed before and the Dirichlet rows set afterwards, as
// for the element-by-element kernel; for the apply, Dirichlet coefficients of v count as zero.
// The linearisation (OP3_LIN) stops after the forward contractions of u (values only) and writes
// m = -lambda W e^u at every Gauss point, layout [element][q0 + Q (q1 + Q q2)], into Y.
#pragma once

#include "iga_impl.h"

namespace iga {
namespace rs3 {

constexpr int kThreads = 256;
enum { OP3_RES = 0, OP3_APPLY = 1, OP3_LIN = 2 };

// elements per tile side (TE Q = 8 or 9 Gauss points per axis: measured at 64^3, larger tiles run one
// workgroup per CU and lose to the element-by-element kernel) and the LDS plan in doubles:
// c [NI^3]; A0, D0 [NI^2 G]; U1, U01, U10 [NI G^2] (reused for Y0, Y1, Y2); F0, F1, F2, S [G^3]
// (A0 / D0 reused for Za / Zb); the tile's basis values and derivatives [axis][B|dB][G][P] and
// quadrature weights [axis][G].
template <int P>
struct Res3 {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TE = P == 2 ? 4 : P == 3 ? 3 : 2;
  static constexpr int NI = TE + p, G = TE * Q;
  static constexpr int n_c = NI * NI * NI, n_a = NI * NI * G, n_u = NI * G * G, n_f = G * G * G;
  static constexpr int n_b = 6 * G * P + 3 * G;
  static constexpr size_t total = (size_t)(n_c + 2 * n_a + 3 * n_u + 4 * n_f + n_b) * sizeof(double);
};

__host__ __device__ inline int res3_tiles(int ne0, int ne1, int ne2, int TE) {
  return ((ne0 + TE - 1) / TE) * ((ne1 + TE - 1) / TE) * ((ne2 + TE - 1) / TE);
}

// Every stage runs over the full tile extents (compile-time strides); a tile cut by the end of the
// mesh skips the entries past its NE_d elements.
template <int P, int OP>
__device__ inline void res3_body(const DevProblem &pb, const int tile, const double *__restrict__ X,
                                 const double *__restrict__ lin, double *__restrict__ Y, double *__restrict__ lds) {
  using S_ = Res3<P>;
  constexpr int p = S_::p, Q = S_::Q, TE = S_::TE, NI = S_::NI, G = S_::G;
  constexpr int NT = kThreads, L = P * P * P, GP = G * P;
  constexpr bool LIN = OP == OP3_LIN;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TE - 1) / TE, nt1 = (ne1 + TE - 1) / TE;
  const int E0 = (tile % nt0) * TE, E1 = ((tile / nt0) % nt1) * TE, E2 = (tile / (nt0 * nt1)) * TE;
  const int NE0 = min(TE, ne0 - E0), NE1 = min(TE, ne1 - E1), NE2 = min(TE, ne2 - E2);
  const int G0 = NE0 * Q, G1 = NE1 * Q, G2 = NE2 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p, NI2 = NE2 + p;
  double *c = lds;                                       // [k2][k1][k0]
  double *A0 = c + S_::n_c, *D0 = A0 + S_::n_a;          // [k2][k1][g0]
  double *U1 = D0 + S_::n_a, *U01 = U1 + S_::n_u, *U10 = U01 + S_::n_u;   // [k2][g1][g0]
  double *F0 = U10 + S_::n_u, *F1 = F0 + S_::n_f, *F2 = F1 + S_::n_f, *Sg = F2 + S_::n_f;   // [g2][g1][g0]
  double *Y0 = U1, *Y1 = U01, *Y2 = U10, *Za = A0, *Zb = D0;
  double *sB = Sg + S_::n_f, *sW = sB + 6 * GP;
  const double *B0 = sB, *dB0 = sB + GP, *B1 = sB + 2 * GP, *dB1 = sB + 3 * GP, *B2 = sB + 4 * GP,
               *dB2 = sB + 5 * GP;
  const double *W0 = sW, *W1 = sW + G, *W2 = sW + 2 * G;
  const int t = threadIdx.x;
  const bool kel = pb.kappa_mode == IGA_KAPPA_ELEMENT;

  // the tile's rows of the basis tables (point g of axis d is global point E_d Q + g)
  auto stage_axis = [&](const AxisDev &ax, int E, int Gd, double *dst, double *wdst) {
    for (int i = t; i < GP; i += NT) {
      if (i / P < Gd) {
        dst[i] = ax.B[(size_t)E * Q * P + i];
        dst[GP + i] = ax.dB[(size_t)E * Q * P + i];
      }
    }
    for (int i = t; i < G; i += NT)
      if (i < Gd) wdst[i] = ax.wq[(size_t)E * Q + i];
  };
  stage_axis(pb.ax[0], E0, G0, sB, sW);
  stage_axis(pb.ax[1], E1, G1, sB + 2 * GP, sW + G);
  stage_axis(pb.ax[2], E2, G2, sB + 4 * GP, sW + 2 * G);
  for (int i = t; i < NI * NI * NI; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    // functions past the end of a periodic axis wrap (eq:map-wrap)
    const int i0 = wrap_fn(pb.ax[0], E0 + k0), i1 = wrap_fn(pb.ax[1], E1 + k1), i2 = wrap_fn(pb.ax[2], E2 + k2);
    double x = X[i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2)];
    if (OP == OP3_APPLY && is_dirichlet_idx(pb, i0, i1, i2)) x = 0.0;
    c[i] = x;
  }
  __syncthreads();
  // axis 0: value and derivative per function pair (k1, k2)
  for (int i = t; i < NI * NI * G; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), el0 = g0 / Q;
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    const double *cc = c + (k2 * NI + k1) * NI + el0;
    double a = 0, d = 0;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) {
      a += B0[g0 * P + a0] * cc[a0];
      if constexpr (!LIN) d += dB0[g0 * P + a0] * cc[a0];
    }
    A0[i] = a;
    if constexpr (!LIN) D0[i] = d;
  }
  __syncthreads();
  // axis 1
  for (int i = t; i < NI * G * G; i += NT) {
    const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G), el1 = g1 / Q;
    if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
    double u = 0, u01 = 0, u10 = 0;
#pragma unroll
    for (int a1 = 0; a1 < P; ++a1) {
      const int r = (k2 * NI + el1 + a1) * G + g0;
      const double b = B1[g1 * P + a1];
      u += b * A0[r];
      if constexpr (!LIN) {
        u01 += b * D0[r];
        u10 += dB1[g1 * P + a1] * A0[r];
      }
    }
    U1[i] = u;
    if constexpr (!LIN) {
      U01[i] = u01;
      U10[i] = u10;
    }
  }
  __syncthreads();
  // axis 2 and the point integrands
  {
    const double lam = pb.lambda;
    for (int i = t; i < G * G * G; i += NT) {
      const int g0 = i % G, g1 = (i / G) % G, g2 = i / (G * G), el2 = g2 / Q;
      if (g0 >= G0 || g1 >= G1 || g2 >= G2) continue;
      double u = 0, d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) {
        const int r = ((el2 + a2) * G + g1) * G + g0;
        const double b = B2[g2 * P + a2];
        u += b * U1[r];
        if constexpr (!LIN) {
          d0 += b * U01[r];
          d1 += b * U10[r];
          d2 += dB2[g2 * P + a2] * U1[r];
        }
      }
      const int el0 = g0 / Q, el1 = g1 / Q;
      const double W = W0[g0] * W1[g1] * W2[g2];
      const int64_t e = (E0 + el0) + (int64_t)ne0 * ((E1 + el1) + (int64_t)ne1 * (E2 + el2));
      if constexpr (LIN) {
        const int q = (g0 % Q) + Q * ((g1 % Q) + Q * (g2 % Q));
        Y[e * L + q] = -lam * W * exp(u);
        continue;
      }
      const double kw = (kel ? pb.kel[e] : 1.0) * W;
      F0[i] = kw * d0;
      F1[i] = kw * d1;
      F2[i] = kw * d2;
      if (OP == OP3_RES) {
        Sg[i] = -W * lam * exp(u);
      } else {
        const int q = (g0 % Q) + Q * ((g1 % Q) + Q * (g2 % Q));
        Sg[i] = lin[e * L + q] * u;
      }
    }
  }
  if constexpr (LIN) return;
  __syncthreads();
  // transposed axis 2: Y0 = sum B2 F0, Y1 = sum B2 F1, Y2 = sum dB2 F2 + B2 S
  for (int i = t; i < NI * G * G; i += NT) {
    const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G);
    if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
    double y0 = 0, y1 = 0, y2 = 0;
#pragma unroll
    for (int a2 = 0; a2 <= p; ++a2) {
      const int el2 = k2 - a2;
      if (el2 < 0 || el2 >= NE2) continue;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const int g2 = el2 * Q + q2, w = (g2 * G + g1) * G + g0;
        const double b = B2[g2 * P + a2];
        y0 += b * F0[w];
        y1 += b * F1[w];
        y2 += dB2[g2 * P + a2] * F2[w] + b * Sg[w];
      }
    }
    Y0[i] = y0;
    Y1[i] = y1;
    Y2[i] = y2;
  }
  __syncthreads();
  // transposed axis 1: Za = sum B1 Y0, Zb = sum dB1 Y1 + B1 Y2
  for (int i = t; i < NI * NI * G; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI);
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    double za = 0, zb = 0;
#pragma unroll
    for (int a1 = 0; a1 <= p; ++a1) {
      const int el1 = k1 - a1;
      if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const int g1 = el1 * Q + q1, w = (k2 * G + g1) * G + g0;
        const double b = B1[g1 * P + a1];
        za += b * Y0[w];
        zb += dB1[g1 * P + a1] * Y1[w] + b * Y2[w];
      }
    }
    Za[i] = za;
    Zb[i] = zb;
  }
  __syncthreads();
  // transposed axis 0 and the scatter of the tile's contributions
  for (int i = t; i < NI * NI * NI; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    double r = 0;
#pragma unroll
    for (int a0 = 0; a0 <= p; ++a0) {
      const int el0 = k0 - a0;
      if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        const int g0 = el0 * Q + q0, w = (k2 * NI + k1) * G + g0;
        r += dB0[g0 * P + a0] * Za[w] + B0[g0 * P + a0] * Zb[w];
      }
    }
    atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                 (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2))],
              r);
  }
}

// Fourth-order operator on x = xi without weights (tiles as above): R_A = sum_q W (Lap N_A)(Lap u_h)
// with Lap N_A = N''_{a0} N_{a1} N_{a2} + N_{a0} N''_{a1} N_{a2} + N_{a0} N_{a1} N''_{a2}.  Forward:
// axis 0 gives B.c and B''.c, axis 1 the three products needed, axis 2 the Laplacian at every
// point, S = W Lap u_h; transposed: axis 2 gives B.S and B''.S, axis 1 the two sums that axis 0
// closes with B'' and B.  One FP64 atomic per tile function; the output must be zeroed before.
template <int P>
__device__ inline void bih3_body(const DevProblem &pb, const int tile, const double *__restrict__ X,
                                 double *__restrict__ Y, double *__restrict__ lds) {
  using S_ = Res3<P>;
  constexpr int p = S_::p, Q = S_::Q, TE = S_::TE, NI = S_::NI, G = S_::G;
  constexpr int NT = kThreads, GP = G * P;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TE - 1) / TE, nt1 = (ne1 + TE - 1) / TE;
  const int E0 = (tile % nt0) * TE, E1 = ((tile / nt0) % nt1) * TE, E2 = (tile / (nt0 * nt1)) * TE;
  const int NE0 = min(TE, ne0 - E0), NE1 = min(TE, ne1 - E1), NE2 = min(TE, ne2 - E2);
  const int G0 = NE0 * Q, G1 = NE1 * Q, G2 = NE2 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p, NI2 = NE2 + p;
  double *c = lds;                                       // [k2][k1][k0]
  double *A0 = c + S_::n_c, *D0 = A0 + S_::n_a;          // [k2][k1][g0]: B.c, B''.c along axis 0
  double *V1 = D0 + S_::n_a, *W1 = V1 + S_::n_u, *X1 = W1 + S_::n_u;   // [k2][g1][g0]
  double *Sg = X1 + S_::n_u;                             // [g2][g1][g0]
  double *YB = V1, *YD = W1, *Z1 = A0, *Z2 = D0;
  double *sB = Sg + 4 * S_::n_f, *sW = sB + 6 * GP;      // the residual's table slots: [axis][B|B''][G][P]
  const double *B0 = sB, *C0 = sB + GP, *B1 = sB + 2 * GP, *C1 = sB + 3 * GP, *B2 = sB + 4 * GP,
               *C2 = sB + 5 * GP;
  const double *Wq0 = sW, *Wq1 = sW + G, *Wq2 = sW + 2 * G;
  const int t = threadIdx.x;

  auto stage_axis = [&](const AxisDev &ax, int E, int Gd, double *dst, double *wdst) {
    for (int i = t; i < GP; i += NT) {
      if (i / P < Gd) {
        dst[i] = ax.B[(size_t)E * Q * P + i];
        dst[GP + i] = ax.d2B[(size_t)E * Q * P + i];
      }
    }
    for (int i = t; i < G; i += NT)
      if (i < Gd) wdst[i] = ax.wq[(size_t)E * Q + i];
  };
  stage_axis(pb.ax[0], E0, G0, sB, sW);
  stage_axis(pb.ax[1], E1, G1, sB + 2 * GP, sW + G);
  stage_axis(pb.ax[2], E2, G2, sB + 4 * GP, sW + 2 * G);
  for (int i = t; i < NI * NI * NI; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    const int i0 = wrap_fn(pb.ax[0], E0 + k0), i1 = wrap_fn(pb.ax[1], E1 + k1), i2 = wrap_fn(pb.ax[2], E2 + k2);
    c[i] = X[i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2)];
  }
  __syncthreads();
  for (int i = t; i < NI * NI * G; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), el0 = g0 / Q;
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    const double *cc = c + (k2 * NI + k1) * NI + el0;
    double a = 0, d = 0;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) {
      a += B0[g0 * P + a0] * cc[a0];
      d += C0[g0 * P + a0] * cc[a0];
    }
    A0[i] = a;
    D0[i] = d;
  }
  __syncthreads();
  for (int i = t; i < NI * G * G; i += NT) {
    const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G), el1 = g1 / Q;
    if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
    double v = 0, w = 0, x = 0;
#pragma unroll
    for (int a1 = 0; a1 < P; ++a1) {
      const int r = (k2 * NI + el1 + a1) * G + g0;
      v += B1[g1 * P + a1] * A0[r];
      w += C1[g1 * P + a1] * A0[r];
      x += B1[g1 * P + a1] * D0[r];
    }
    V1[i] = v;    // B B
    W1[i] = w;    // B B''  (second derivative along axis 1)
    X1[i] = x;    // B'' B  (second derivative along axis 0)
  }
  __syncthreads();
  for (int i = t; i < G * G * G; i += NT) {
    const int g0 = i % G, g1 = (i / G) % G, g2 = i / (G * G), el2 = g2 / Q;
    if (g0 >= G0 || g1 >= G1 || g2 >= G2) continue;
    double lap = 0;
#pragma unroll
    for (int a2 = 0; a2 < P; ++a2) {
      const int r = ((el2 + a2) * G + g1) * G + g0;
      lap += B2[g2 * P + a2] * (X1[r] + W1[r]) + C2[g2 * P + a2] * V1[r];
    }
    Sg[i] = Wq0[g0] * Wq1[g1] * Wq2[g2] * lap;
  }
  __syncthreads();
  for (int i = t; i < NI * G * G; i += NT) {
    const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G);
    if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
    double yb = 0, yd = 0;
#pragma unroll
    for (int a2 = 0; a2 <= p; ++a2) {
      const int el2 = k2 - a2;
      if (el2 < 0 || el2 >= NE2) continue;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const int g2 = el2 * Q + q2, w = (g2 * G + g1) * G + g0;
        yb += B2[g2 * P + a2] * Sg[w];
        yd += C2[g2 * P + a2] * Sg[w];
      }
    }
    YB[i] = yb;
    YD[i] = yd;
  }
  __syncthreads();
  for (int i = t; i < NI * NI * G; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI);
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    double z1 = 0, z2 = 0;
#pragma unroll
    for (int a1 = 0; a1 <= p; ++a1) {
      const int el1 = k1 - a1;
      if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const int g1 = el1 * Q + q1, w = (k2 * G + g1) * G + g0;
        z1 += B1[g1 * P + a1] * YB[w];
        z2 += C1[g1 * P + a1] * YB[w] + B1[g1 * P + a1] * YD[w];
      }
    }
    Z1[i] = z1;
    Z2[i] = z2;
  }
  __syncthreads();
  for (int i = t; i < NI * NI * NI; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    double r = 0;
#pragma unroll
    for (int a0 = 0; a0 <= p; ++a0) {
      const int el0 = k0 - a0;
      if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        const int g0 = el0 * Q + q0, w = (k2 * NI + k1) * G + g0;
        r += C0[g0 * P + a0] * Z1[w] + B0[g0 * P + a0] * Z2[w];
      }
    }
    atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                 (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2))],
              r);
  }
}

// Cahn-Hilliard residual on x = xi without weights, by the tiles above (see the element kernel for the
// form): forward, axis 0 gives B.c, B'.c, B''.c and B.cdot, axis 1 the six products that c, its
// gradient, its Laplacian and cdot need, axis 2 those at every point; the point terms are
// S0 = W cdot, F = W (M mu' + lam M' Lap c) grad c and S2 = W lam M Lap c; transposed, the terms
// B0 B1 (B2 S0 + B2' F2 + B2'' S2) + B0' B1 B2 F0 + B0 B1' B2 F1 + (B0'' B1 + B0 B1'') B2 S2 are
// contracted axis by axis.  One FP64 atomic per tile function; the output must be zeroed before.
template <int P>
struct Ch3 {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TE = P == 2 ? 4 : P == 3 ? 3 : 2;
  static constexpr int NI = TE + p, G = TE * Q, GP = G * P;
  static constexpr int n_c = NI * NI * NI, n_a = NI * NI * G, n_u = NI * G * G, n_f = G * G * G;
  static constexpr int n_b = 9 * GP + 3 * G;
  static constexpr size_t total = (size_t)(2 * n_c + 4 * n_a + 6 * n_u + 5 * n_f + n_b) * sizeof(double);
};

template <int P>
__device__ inline void ch3_body(const DevProblem &pb, const int tile, const double *__restrict__ Cv,
                                const double *__restrict__ Cd, double theta, double lam, double *__restrict__ Y,
                                double *__restrict__ lds) {
  using S_ = Ch3<P>;
  constexpr int p = S_::p, Q = S_::Q, TE = S_::TE, NI = S_::NI, G = S_::G, GP = S_::GP;
  constexpr int NT = kThreads;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TE - 1) / TE, nt1 = (ne1 + TE - 1) / TE;
  const int E0 = (tile % nt0) * TE, E1 = ((tile / nt0) % nt1) * TE, E2 = (tile / (nt0 * nt1)) * TE;
  const int NE0 = min(TE, ne0 - E0), NE1 = min(TE, ne1 - E1), NE2 = min(TE, ne2 - E2);
  const int G0 = NE0 * Q, G1 = NE1 * Q, G2 = NE2 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p, NI2 = NE2 + p;
  double *c = lds, *cd = c + S_::n_c;                                      // [k2][k1][k0]
  double *aB = cd + S_::n_c, *aD = aB + S_::n_a, *aE = aD + S_::n_a, *aR = aE + S_::n_a;   // [k2][k1][g0]
  double *bBB = aR + S_::n_a, *bDB = bBB + S_::n_u, *bBE = bDB + S_::n_u;   // [k2][g1][g0]
  double *bEB = bBE + S_::n_u, *bBD = bEB + S_::n_u, *bRB = bBD + S_::n_u;
  double *F0 = bRB + S_::n_u, *F1 = F0 + S_::n_f, *F2 = F1 + S_::n_f, *S0 = F2 + S_::n_f, *S2 = S0 + S_::n_f;
  double *tb = S2 + S_::n_f, *tw = tb + 9 * GP;                             // [axis][B|B'|B''][G][P], [axis][G]
  // transposed stage arrays reuse the forward ones
  double *Ybb = bBB, *Yf0 = bDB, *Yf1 = bBE, *Ys = bEB;                    // [k2][g1][g0]
  double *Zb = aB, *Zd = aD, *Ze = aE;                                      // [k2][k1][g0]
  const int t = threadIdx.x;
  auto T = [&](int d, int kind) { return tb + (d * 3 + kind) * GP; };
  const int Ed[3] = {E0, E1, E2}, Gd[3] = {G0, G1, G2};
  for (int d = 0; d < 3; ++d) {
    const AxisDev &ax = pb.ax[d];
    for (int i = t; i < GP; i += NT) {
      if (i / P < Gd[d]) {
        const size_t o = (size_t)Ed[d] * Q * P + i;
        T(d, 0)[i] = ax.B[o];
        T(d, 1)[i] = ax.dB[o];
        T(d, 2)[i] = ax.d2B[o];
      }
    }
    for (int i = t; i < G; i += NT)
      if (i < Gd[d]) tw[d * G + i] = ax.wq[(size_t)Ed[d] * Q + i];
  }
  for (int i = t; i < NI * NI * NI; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    const int64_t A = wrap_fn(pb.ax[0], E0 + k0) +
                      (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2));
    c[i] = Cv[A];
    cd[i] = Cd[A];
  }
  __syncthreads();
  {
    const double *B = T(0, 0), *D = T(0, 1), *E = T(0, 2);
    for (int i = t; i < NI * NI * G; i += NT) {
      const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), el0 = g0 / Q;
      if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
      const int o = (k2 * NI + k1) * NI + el0;
      double vb = 0, vd = 0, ve = 0, vr = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        vb += B[g0 * P + a0] * c[o + a0];
        vd += D[g0 * P + a0] * c[o + a0];
        ve += E[g0 * P + a0] * c[o + a0];
        vr += B[g0 * P + a0] * cd[o + a0];
      }
      aB[i] = vb;
      aD[i] = vd;
      aE[i] = ve;
      aR[i] = vr;
    }
  }
  __syncthreads();
  {
    const double *B = T(1, 0), *D = T(1, 1), *E = T(1, 2);
    for (int i = t; i < NI * G * G; i += NT) {
      const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G), el1 = g1 / Q;
      if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
      double bb = 0, db = 0, be = 0, eb = 0, bd = 0, rb = 0;
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) {
        const int r = (k2 * NI + el1 + a1) * G + g0;
        const double b = B[g1 * P + a1];
        bb += b * aB[r];
        db += b * aD[r];               // d/dxi0
        be += E[g1 * P + a1] * aB[r];  // d2/dxi1^2
        eb += b * aE[r];               // d2/dxi0^2
        bd += D[g1 * P + a1] * aB[r];  // d/dxi1
        rb += b * aR[r];               // rate
      }
      bBB[i] = bb;
      bDB[i] = db;
      bBE[i] = be;
      bEB[i] = eb;
      bBD[i] = bd;
      bRB[i] = rb;
    }
  }
  __syncthreads();
  {
    const double *B = T(2, 0), *D = T(2, 1), *E = T(2, 2);
    for (int i = t; i < G * G * G; i += NT) {
      const int g0 = i % G, g1 = (i / G) % G, g2 = i / (G * G), el2 = g2 / Q;
      if (g0 >= G0 || g1 >= G1 || g2 >= G2) continue;
      double cv = 0, c0 = 0, c1 = 0, c2 = 0, lc = 0, cr = 0;
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) {
        const int r = ((el2 + a2) * G + g1) * G + g0;
        const double b = B[g2 * P + a2];
        cv += b * bBB[r];
        c0 += b * bDB[r];
        c1 += b * bBD[r];
        c2 += D[g2 * P + a2] * bBB[r];
        lc += b * (bEB[r] + bBE[r]) + E[g2 * P + a2] * bBB[r];
        cr += b * bRB[r];
      }
      const double W = tw[g0] * tw[G + g1] * tw[2 * G + g2];
      const double M = cv * (1.0 - cv), dM = 1.0 - 2.0 * cv, dmu = 1.0 / (2.0 * theta * cv * (1.0 - cv)) - 2.0;
      const double sg = W * (M * dmu + lam * dM * lc);
      F0[i] = sg * c0;
      F1[i] = sg * c1;
      F2[i] = sg * c2;
      S0[i] = W * cr;
      S2[i] = W * lam * M * lc;
    }
  }
  __syncthreads();
  {
    const double *B = T(2, 0), *D = T(2, 1), *E = T(2, 2);
    for (int i = t; i < NI * G * G; i += NT) {
      const int g0 = i % G, g1 = (i / G) % G, k2 = i / (G * G);
      if (g0 >= G0 || g1 >= G1 || k2 >= NI2) continue;
      double ybb = 0, yf0 = 0, yf1 = 0, ys = 0;
#pragma unroll
      for (int a2 = 0; a2 <= p; ++a2) {
        const int el2 = k2 - a2;
        if (el2 < 0 || el2 >= NE2) continue;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const int g2 = el2 * Q + q2, w = (g2 * G + g1) * G + g0, o = g2 * P + a2;
          ybb += B[o] * S0[w] + D[o] * F2[w] + E[o] * S2[w];
          yf0 += B[o] * F0[w];
          yf1 += B[o] * F1[w];
          ys += B[o] * S2[w];
        }
      }
      Ybb[i] = ybb;
      Yf0[i] = yf0;
      Yf1[i] = yf1;
      Ys[i] = ys;
    }
  }
  __syncthreads();
  {
    const double *B = T(1, 0), *D = T(1, 1), *E = T(1, 2);
    for (int i = t; i < NI * NI * G; i += NT) {
      const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI);
      if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
      double zb = 0, zd = 0, ze = 0;
#pragma unroll
      for (int a1 = 0; a1 <= p; ++a1) {
        const int el1 = k1 - a1;
        if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          const int g1 = el1 * Q + q1, w = (k2 * G + g1) * G + g0, o = g1 * P + a1;
          zb += B[o] * Ybb[w] + D[o] * Yf1[w] + E[o] * Ys[w];
          zd += B[o] * Yf0[w];
          ze += B[o] * Ys[w];
        }
      }
      Zb[i] = zb;
      Zd[i] = zd;
      Ze[i] = ze;
    }
  }
  __syncthreads();
  {
    const double *B = T(0, 0), *D = T(0, 1), *E = T(0, 2);
    for (int i = t; i < NI * NI * NI; i += NT) {
      const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
      if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
      double r = 0;
#pragma unroll
      for (int a0 = 0; a0 <= p; ++a0) {
        const int el0 = k0 - a0;
        if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          const int g0 = el0 * Q + q0, w = (k2 * NI + k1) * G + g0, o = g0 * P + a0;
          r += B[o] * Zb[w] + D[o] * Zd[w] + E[o] * Ze[w];
        }
      }
      atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                   (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2))],
                r);
    }
  }
}

// ------------------------------------------------------------------------------------------
// Column-register variant of the residual, the apply and the point linearisation.  The x-y extent of a tile
// is TEX = 16 / Q elements, so its TEX Q x TEX Q Gauss-point columns (g0, g1) are one lane each, and
// a tile is TEZ elements deep.  The axis-0 contraction goes through LDS; then every lane holds the
// axis-1 results of its column for all NZ = TEZ + p function planes in registers and runs the axis-2
// contraction, the point integrands and the transposed axis-2 contraction for all of its column's
// points in registers (the axis-2 basis rows are the same for every lane: uniform loads).  Only the
// transposed axis-1 and axis-0 contractions go through LDS again.  Compared with res3_body this
// removes the point arrays from LDS and most of the LDS reads per multiply-add; it adds
// (TEX + p)^2 / TEX^2 of x-y halo work instead of (TE + p)^3 / TE^3.  Border functions are shared
// with neighbouring tiles: one FP64 atomic per tile function, the output zeroed before.  OP3_LIN
// stops after the point values and writes m = -lambda W e^u per point, layout [element][q].
template <int P, int TEZ>
struct Res3R {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TEX = 16 / Q, G = TEX * Q;
  static constexpr int NI = TEX + p, NZ = TEZ + p;
  static constexpr int GS = G % 2 ? G : G + 1;   // LDS row stride along g0 (odd: rows fall in different banks)
  static constexpr int n_c = NZ * NI * NI, n_a = NZ * NI * GS, n_y = NZ * G * GS;
  static constexpr int n_b = 4 * G * P + 2 * G + 2 * TEZ * Q * P + TEZ * Q;
  static constexpr size_t total = (size_t)(n_c + 2 * n_a + 3 * n_y + n_b) * sizeof(double);
  static_assert(G * G <= kThreads, "one lane per Gauss-point column");
  static_assert(total <= 65536, "static LDS");
};

template <int P>
struct Res3RDepth {
  static constexpr int TEZ = P == 5 ? 3 : 4;
};

__host__ __device__ inline int res3r_tiles(int ne0, int ne1, int ne2, int TEX, int TEZ) {
  return ((ne0 + TEX - 1) / TEX) * ((ne1 + TEX - 1) / TEX) * ((ne2 + TEZ - 1) / TEZ);
}

template <int P, int TEZ, int OP>
__device__ inline void res3r_body(const DevProblem &pb, const int tile, const double *__restrict__ X,
                                  const double *__restrict__ lin, double *__restrict__ Y, double *__restrict__ lds) {
  constexpr bool LIN = OP == OP3_LIN;
  using S_ = Res3R<P, TEZ>;
  constexpr int p = S_::p, Q = S_::Q, TEX = S_::TEX, G = S_::G, GS = S_::GS, NI = S_::NI, NZ = S_::NZ;
  constexpr int NT = kThreads, L = P * P * P, GP = G * P, NA = NZ * NI * G;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TEX - 1) / TEX, nt1 = (ne1 + TEX - 1) / TEX;
  const int E0 = (tile % nt0) * TEX, E1 = ((tile / nt0) % nt1) * TEX, E2 = (tile / (nt0 * nt1)) * TEZ;
  const int NE0 = min(TEX, ne0 - E0), NE1 = min(TEX, ne1 - E1), NE2 = min(TEZ, ne2 - E2);
  const int G0 = NE0 * Q, G1 = NE1 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p, NI2 = NE2 + p;
  double *c = lds;                                     // [k2][k1][k0]
  double *A0 = c + S_::n_c, *D0 = A0 + S_::n_a;        // [k2][k1][g0] (row stride GS); later Za, Zb
  double *Ys = D0 + S_::n_a;                           // [3][k2][g1][g0] (row stride GS)
  double *sB = Ys + 3 * S_::n_y, *sW = sB + 4 * GP;
  double *sB2 = sW + 2 * G, *sW2 = sB2 + 2 * TEZ * Q * P;   // axis-2 rows of the tile: [B|dB][z point][a], weights
  const double *B0 = sB, *dB0 = sB + GP, *B1 = sB + 2 * GP, *dB1 = sB + 3 * GP, *W0 = sW, *W1 = sW + G;
  double *Za = A0, *Zb = D0;
  const int t = threadIdx.x;
  const bool kel = pb.kappa_mode == IGA_KAPPA_ELEMENT;

  for (int i = t; i < GP; i += NT)
    if (i / P < G0) {
      sB[i] = pb.ax[0].B[(size_t)E0 * Q * P + i];
      sB[GP + i] = pb.ax[0].dB[(size_t)E0 * Q * P + i];
    }
  for (int i = t; i < GP; i += NT)
    if (i / P < G1) {
      sB[2 * GP + i] = pb.ax[1].B[(size_t)E1 * Q * P + i];
      sB[3 * GP + i] = pb.ax[1].dB[(size_t)E1 * Q * P + i];
    }
  for (int i = t; i < G; i += NT) {
    if (i < G0) sW[i] = pb.ax[0].wq[(size_t)E0 * Q + i];
    if (i < G1) sW[G + i] = pb.ax[1].wq[(size_t)E1 * Q + i];
  }
  for (int i = t; i < TEZ * Q * P; i += NT)
    if (i / (Q * P) < NE2) {
      sB2[i] = pb.ax[2].B[(size_t)E2 * Q * P + i];
      sB2[TEZ * Q * P + i] = pb.ax[2].dB[(size_t)E2 * Q * P + i];
    }
  for (int i = t; i < TEZ * Q; i += NT)
    if (i / Q < NE2) sW2[i] = pb.ax[2].wq[(size_t)E2 * Q + i];
  for (int i = t; i < S_::n_c; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    const int i0 = wrap_fn(pb.ax[0], E0 + k0), i1 = wrap_fn(pb.ax[1], E1 + k1), i2 = wrap_fn(pb.ax[2], E2 + k2);
    double x = X[i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2)];
    if (OP == OP3_APPLY && is_dirichlet_idx(pb, i0, i1, i2)) x = 0.0;
    c[i] = x;
  }
  __syncthreads();
  // axis 0: value and derivative per function pair (k1, k2)
  for (int i = t; i < NA; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), el0 = g0 / Q;
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    const double *cc = c + (k2 * NI + k1) * NI + el0;
    double a = 0, d = 0;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) {
      a += B0[g0 * P + a0] * cc[a0];
      if constexpr (!LIN) d += dB0[g0 * P + a0] * cc[a0];
    }
    const int o = (k2 * NI + k1) * GS + g0;
    A0[o] = a;
    if constexpr (!LIN) D0[o] = d;
  }
  __syncthreads();
  // one lane per Gauss-point column: axis 1, axis 2, the point integrands and the transposed axis 2
  const int g0 = t % G, g1 = t / G;
  const bool act = t < G * G && g0 < G0 && g1 < G1;
  double Y0[NZ], Y1[NZ], Y2[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) Y0[k] = Y1[k] = Y2[k] = 0.0;
  if (act) {
    const int el0 = g0 / Q, el1 = g1 / Q, q0 = g0 % Q, q1 = g1 % Q;
    // the apply's point factors of this column, loaded before the axis-1 work so that they arrive
    // while it runs
    double lv[OP == OP3_APPLY ? TEZ * Q : 1];
    if constexpr (OP == OP3_APPLY) {
#pragma unroll
      for (int el2 = 0; el2 < TEZ; ++el2) {
        const int64_t e = (E0 + el0) + (int64_t)ne0 * ((E1 + el1) + (int64_t)ne1 * (E2 + min(el2, NE2 - 1)));
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) lv[el2 * Q + q2] = lin[e * L + q0 + Q * (q1 + Q * q2)];
      }
    }
    double b1[P], db1[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      b1[a] = B1[g1 * P + a];
      db1[a] = dB1[g1 * P + a];
    }
    double U[NZ], U01[NZ], U10[NZ];
#pragma unroll
    for (int k2 = 0; k2 < NZ; ++k2) {
      double u = 0, u01 = 0, u10 = 0;
      if (k2 < NI2) {
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) {
          const int r = (k2 * NI + el1 + a1) * GS + g0;
          u += b1[a1] * A0[r];
          if constexpr (!LIN) {
            u01 += b1[a1] * D0[r];
            u10 += db1[a1] * A0[r];
          }
        }
      }
      U[k2] = u;
      U01[k2] = u01;
      U10[k2] = u10;
    }
    const double w01 = W0[g0] * W1[g1], lam = pb.lambda;
#pragma unroll
    for (int el2 = 0; el2 < TEZ; ++el2) {
      if (el2 >= NE2) break;
      const int e2 = E2 + el2;
      const int64_t e = (E0 + el0) + (int64_t)ne0 * ((E1 + el1) + (int64_t)ne1 * e2);
      const double kap = kel ? pb.kel[e] : 1.0;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const int o = (el2 * Q + q2) * P;
        double b2[P], db2[P];
#pragma unroll
        for (int a = 0; a < P; ++a) {
          b2[a] = sB2[o + a];
          db2[a] = sB2[TEZ * Q * P + o + a];
        }
        double u = 0, d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) {
          u += b2[a2] * U[el2 + a2];
          d0 += b2[a2] * U01[el2 + a2];
          d1 += b2[a2] * U10[el2 + a2];
          d2 += db2[a2] * U[el2 + a2];
        }
        const double W = w01 * sW2[el2 * Q + q2], kw = kap * W;
        if constexpr (LIN) {
          Y[e * L + q0 + Q * (q1 + Q * q2)] = -lam * W * exp(u);
          continue;
        }
        const double F0 = kw * d0, F1 = kw * d1, F2 = kw * d2;
        double S;
        if constexpr (OP == OP3_RES) S = -W * lam * exp(u);
        else S = lv[el2 * Q + q2] * u;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) {
          Y0[el2 + a2] += b2[a2] * F0;
          Y1[el2 + a2] += b2[a2] * F1;
          Y2[el2 + a2] += db2[a2] * F2 + b2[a2] * S;
        }
      }
    }
    if constexpr (LIN) return;
#pragma unroll
    for (int k2 = 0; k2 < NZ; ++k2) {
      if (k2 < NI2) {
        const int w = (k2 * G + g1) * GS + g0;
        Ys[w] = Y0[k2];
        Ys[S_::n_y + w] = Y1[k2];
        Ys[2 * S_::n_y + w] = Y2[k2];
      }
    }
  }
  if constexpr (LIN) return;
  __syncthreads();
  // transposed axis 1: Za = sum B1 Y0, Zb = sum dB1 Y1 + B1 Y2 (over A0 / D0, whose reads are done)
  for (int i = t; i < NA; i += NT) {
    const int gg0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI);
    if (gg0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    double za = 0, zb = 0;
#pragma unroll
    for (int a1 = 0; a1 <= p; ++a1) {
      const int el1 = k1 - a1;
      if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const int gg1 = el1 * Q + q1, w = (k2 * G + gg1) * GS + gg0;
        const double b = B1[gg1 * P + a1];
        za += b * Ys[w];
        zb += dB1[gg1 * P + a1] * Ys[S_::n_y + w] + b * Ys[2 * S_::n_y + w];
      }
    }
    Za[(k2 * NI + k1) * GS + gg0] = za;
    Zb[(k2 * NI + k1) * GS + gg0] = zb;
  }
  __syncthreads();
  // transposed axis 0 and the scatter of the tile's contributions
  for (int i = t; i < S_::n_c; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    double r = 0;
#pragma unroll
    for (int a0 = 0; a0 <= p; ++a0) {
      const int el0 = k0 - a0;
      if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        const int gg0 = el0 * Q + q0, w = (k2 * NI + k1) * GS + gg0;
        r += dB0[gg0 * P + a0] * Za[w] + B0[gg0 * P + a0] * Zb[w];
      }
    }
    atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                 (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2))],
              r);
  }
}

// ------------------------------------------------------------------------------------------
// Streaming column tiles for the residual and the apply: the x-y extent and the lane layout of
// res3r_body, but a workgroup walks a run of chunks of TEZ elements along axis 2.  A function plane
// k2 receives contributions from elements k2 - p .. k2 only, so after a chunk its first TEZ planes
// are complete and go out (transposed axis 1 and axis 0 through LDS, one FP64 atomic per function:
// the x-y borders are still shared with neighbouring tiles), while the last p planes stay open in
// registers and become the first p planes of the next chunk, together with their axis-1 results of
// the forward pass.  Per chunk only TEZ new coefficient planes are loaded and contracted, so the
// axis-2 halo work ((TEZ + p) / TEZ in res3r_body) and the atomics on the planes that two z tiles
// share are paid once per run instead of once per chunk.  The run's last chunk flushes all of its
// open planes.  Runs of zc <= kRes3sRunMax chunks start every zc TEZ elements; the last run ends with
// the mesh.
template <int P, int TEZ>
struct Res3S {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TEX = 16 / Q, G = TEX * Q;
  static constexpr int NI = TEX + p, NZ = TEZ + p;
  static constexpr int GS = G % 2 ? G : G + 1;
  static constexpr int n_c = NZ * NI * NI, n_a = NZ * NI * GS, n_y = TEZ * G * GS;
  static constexpr int n_b = 4 * G * P + 2 * G + 2 * TEZ * Q * P + TEZ * Q;
  static constexpr size_t total = (size_t)(n_c + 2 * n_a + 3 * n_y + n_b) * sizeof(double);
  static_assert(G * G <= kThreads, "one lane per Gauss-point column");
  static_assert(TEZ >= p, "the planes left open by a chunk fit one emission");
  static_assert(total <= 65536, "static LDS");
};

constexpr int kRes3sRunMax = 4;   // chunks per run, at most

__host__ __device__ inline int res3s_blocks(int ne0, int ne1, int ne2, int TEX, int TEZ, int zc) {
  return ((ne0 + TEX - 1) / TEX) * ((ne1 + TEX - 1) / TEX) * ((ne2 + TEZ * zc - 1) / (TEZ * zc));
}

template <int P, int TEZ, int OP>
__device__ inline void res3s_body(const DevProblem &pb, const int blk, const int zc, const double *__restrict__ X,
                                  const double *__restrict__ lin, double *__restrict__ Y, double *__restrict__ lds) {
  static_assert(OP == OP3_RES || OP == OP3_APPLY, "residual or apply");
  using S_ = Res3S<P, TEZ>;
  constexpr int p = S_::p, Q = S_::Q, TEX = S_::TEX, G = S_::G, GS = S_::GS, NI = S_::NI, NZ = S_::NZ;
  constexpr int NT = kThreads, L = P * P * P, GP = G * P;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TEX - 1) / TEX, nt1 = (ne1 + TEX - 1) / TEX;
  const int E0 = (blk % nt0) * TEX, E1 = ((blk / nt0) % nt1) * TEX;
  const int Zlo = (blk / (nt0 * nt1)) * zc * TEZ, Zhi = min(ne2, Zlo + zc * TEZ);
  const int NE0 = min(TEX, ne0 - E0), NE1 = min(TEX, ne1 - E1);
  const int G0 = NE0 * Q, G1 = NE1 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p;
  double *c = lds;                                     // [k2][k1][k0], plane k2 = function Ez + k2
  double *A0 = c + S_::n_c, *D0 = A0 + S_::n_a;        // [k2][k1][g0] (row stride GS); later Za, Zb
  double *Ys = D0 + S_::n_a;                           // [3][slot][g1][g0] (row stride GS)
  double *sB = Ys + 3 * S_::n_y, *sW = sB + 4 * GP;
  double *sB2 = sW + 2 * G, *sW2 = sB2 + 2 * TEZ * Q * P;   // the chunk's axis-2 rows [B|dB][z point][a], weights
  const double *B0 = sB, *dB0 = sB + GP, *B1 = sB + 2 * GP, *dB1 = sB + 3 * GP, *W0 = sW, *W1 = sW + G;
  double *Za = A0, *Zb = D0;
  const int t = threadIdx.x;
  const bool kel = pb.kappa_mode == IGA_KAPPA_ELEMENT;

  for (int i = t; i < GP; i += NT)
    if (i / P < G0) {
      sB[i] = pb.ax[0].B[(size_t)E0 * Q * P + i];
      sB[GP + i] = pb.ax[0].dB[(size_t)E0 * Q * P + i];
    }
  for (int i = t; i < GP; i += NT)
    if (i / P < G1) {
      sB[2 * GP + i] = pb.ax[1].B[(size_t)E1 * Q * P + i];
      sB[3 * GP + i] = pb.ax[1].dB[(size_t)E1 * Q * P + i];
    }
  for (int i = t; i < G; i += NT) {
    if (i < G0) sW[i] = pb.ax[0].wq[(size_t)E0 * Q + i];
    if (i < G1) sW[G + i] = pb.ax[1].wq[(size_t)E1 * Q + i];
  }

  // open planes: the axis-1 results of the forward pass and the transposed axis-2 sums
  double U[NZ], U01[NZ], U10[NZ], Y0[NZ], Y1[NZ], Y2[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) U[k] = U01[k] = U10[k] = Y0[k] = Y1[k] = Y2[k] = 0.0;

  // planes [pl0, pl1) of the chunk at Ez (pl1 - pl0 <= TEZ): transposed axes 1 and 0, then the atomics
  auto emit = [&](int Ez, int pl0, int pl1, int ti, int g0, int g1, bool act) {
    if (act) {
#pragma unroll
      for (int k2 = 0; k2 < NZ; ++k2)
        if (k2 >= pl0 && k2 < pl1) {
          const int w = ((k2 - pl0) * G + g1) * GS + g0;
          Ys[w] = Y0[k2];
          Ys[S_::n_y + w] = Y1[k2];
          Ys[2 * S_::n_y + w] = Y2[k2];
        }
    }
    __syncthreads();
    const int ns = pl1 - pl0;
    for (int i = ti; i < TEZ * NI * G; i += NT) {
      const int gg0 = i % G, k1 = (i / G) % NI, s = i / (G * NI);
      if (gg0 >= G0 || k1 >= NI1 || s >= ns) continue;
      double za = 0, zb = 0;
#pragma unroll
      for (int a1 = 0; a1 <= p; ++a1) {
        const int e1 = k1 - a1;
        if (e1 < 0 || e1 >= NE1) continue;
#pragma unroll
        for (int r1 = 0; r1 < Q; ++r1) {
          const int gg1 = e1 * Q + r1, w = (s * G + gg1) * GS + gg0;
          const double b = B1[gg1 * P + a1];
          za += b * Ys[w];
          zb += dB1[gg1 * P + a1] * Ys[S_::n_y + w] + b * Ys[2 * S_::n_y + w];
        }
      }
      Za[(s * NI + k1) * GS + gg0] = za;
      Zb[(s * NI + k1) * GS + gg0] = zb;
    }
    __syncthreads();
    for (int i = ti; i < TEZ * NI * NI; i += NT) {
      const int k0 = i % NI, k1 = (i / NI) % NI, s = i / (NI * NI);
      if (k0 >= NI0 || k1 >= NI1 || s >= ns) continue;
      double r = 0;
#pragma unroll
      for (int a0 = 0; a0 <= p; ++a0) {
        const int e0 = k0 - a0;
        if (e0 < 0 || e0 >= NE0) continue;
#pragma unroll
        for (int r0 = 0; r0 < Q; ++r0) {
          const int gg0 = e0 * Q + r0, w = (s * NI + k1) * GS + gg0;
          r += dB0[gg0 * P + a0] * Za[w] + B0[gg0 * P + a0] * Zb[w];
        }
      }
      atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                   (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], Ez + pl0 + s))],
                r);
    }
  };

  // the chunks of a run are unrolled: carried through a runtime loop, the open planes and everything the
  // compiler hoists out of it exceed the register budget of three waves per SIMD
#pragma unroll
  for (int ch = 0; ch < kRes3sRunMax; ++ch) {
    const int Ez = Zlo + ch * TEZ;
    if (Ez >= Zhi) break;
    const int NE2 = min(TEZ, Zhi - Ez), NI2 = NE2 + p;
    const bool last = Ez + TEZ >= Zhi;
    const int kf = Ez == Zlo ? 0 : p;                  // planes below kf are open from the previous chunk
    // the lane's column and strided indices, re-derived in every chunk from an opaque copy of the thread
    // index (otherwise the compiler keeps every address it can share between chunks live in registers)
    int tt = t;
    asm volatile("" : "+v"(tt));
    const int g0 = tt % G, g1 = tt / G;
    const bool act = tt < G * G && g0 < G0 && g1 < G1;
    const int el0 = g0 / Q, el1 = g1 / Q, q0 = g0 % Q, q1 = g1 % Q;
    // (1) coefficients of the new planes and the chunk's axis-2 rows.  The previous chunk's readers of
    // c and sB2 finished before its emission; its transposed axis 0 may still read Za / Zb (= A0 / D0),
    // which the barrier below separates from the axis-0 writes.
    for (int i = tt; i < S_::n_c; i += NT) {
      const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
      if (k0 >= NI0 || k1 >= NI1 || k2 < kf || k2 >= NI2) continue;
      const int i0 = wrap_fn(pb.ax[0], E0 + k0), i1 = wrap_fn(pb.ax[1], E1 + k1), i2 = wrap_fn(pb.ax[2], Ez + k2);
      double x = X[i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2)];
      if (OP == OP3_APPLY && is_dirichlet_idx(pb, i0, i1, i2)) x = 0.0;
      c[i] = x;
    }
    for (int i = tt; i < TEZ * Q * P; i += NT)
      if (i / (Q * P) < NE2) {
        sB2[i] = pb.ax[2].B[(size_t)Ez * Q * P + i];
        sB2[TEZ * Q * P + i] = pb.ax[2].dB[(size_t)Ez * Q * P + i];
      }
    for (int i = tt; i < TEZ * Q; i += NT)
      if (i / Q < NE2) sW2[i] = pb.ax[2].wq[(size_t)Ez * Q + i];
    __syncthreads();
    // (2) axis 0 on the new planes
    for (int i = tt; i < NZ * NI * G; i += NT) {
      const int gg0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), e0 = gg0 / Q;
      if (gg0 >= G0 || k1 >= NI1 || k2 < kf || k2 >= NI2) continue;
      const double *cc = c + (k2 * NI + k1) * NI + e0;
      double a = 0, d = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        a += B0[gg0 * P + a0] * cc[a0];
        d += dB0[gg0 * P + a0] * cc[a0];
      }
      const int o = (k2 * NI + k1) * GS + gg0;
      A0[o] = a;
      D0[o] = d;
    }
    __syncthreads();
    // (3) one lane per Gauss-point column: axis 1 on the new planes, axis 2, the point integrands and
    // the transposed axis 2 into the open planes
    if (act) {
      double b1[P], db1[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        b1[a] = B1[g1 * P + a];
        db1[a] = dB1[g1 * P + a];
      }
#pragma unroll
      for (int k2 = 0; k2 < NZ; ++k2) {
        if (k2 < kf) continue;
        double u = 0, u01 = 0, u10 = 0;
        if (k2 < NI2) {
#pragma unroll
          for (int a1 = 0; a1 < P; ++a1) {
            const int r = (k2 * NI + el1 + a1) * GS + g0;
            u += b1[a1] * A0[r];
            u01 += b1[a1] * D0[r];
            u10 += db1[a1] * A0[r];
          }
        }
        U[k2] = u;
        U01[k2] = u01;
        U10[k2] = u10;
      }
      const double w01 = W0[g0] * W1[g1], lam = pb.lambda;
#pragma unroll
      for (int el2 = 0; el2 < TEZ; ++el2) {
        if (el2 >= NE2) break;
        const int64_t e = (E0 + el0) + (int64_t)ne0 * ((E1 + el1) + (int64_t)ne1 * (Ez + el2));
        const double kap = kel ? pb.kel[e] : 1.0;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const int o = (el2 * Q + q2) * P;
          double b2[P], db2[P];
#pragma unroll
          for (int a = 0; a < P; ++a) {
            b2[a] = sB2[o + a];
            db2[a] = sB2[TEZ * Q * P + o + a];
          }
          double u = 0, d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
          for (int a2 = 0; a2 < P; ++a2) {
            u += b2[a2] * U[el2 + a2];
            d0 += b2[a2] * U01[el2 + a2];
            d1 += b2[a2] * U10[el2 + a2];
            d2 += db2[a2] * U[el2 + a2];
          }
          const double W = w01 * sW2[el2 * Q + q2], kw = kap * W;
          const double F0 = kw * d0, F1 = kw * d1, F2 = kw * d2;
          double S;
          if constexpr (OP == OP3_RES) S = -W * lam * exp(u);
          else S = lin[e * L + q0 + Q * (q1 + Q * q2)] * u;
#pragma unroll
          for (int a2 = 0; a2 < P; ++a2) {
            Y0[el2 + a2] += b2[a2] * F0;
            Y1[el2 + a2] += b2[a2] * F1;
            Y2[el2 + a2] += db2[a2] * F2 + b2[a2] * S;
          }
        }
      }
    }
    // (4) the complete planes go out (the run's last chunk: all of them, in passes of at most TEZ
    // planes); the open ones move down to the first p planes
    const int npass = (last && NI2 > TEZ) ? 2 : 1;
    for (int ps = 0; ps < npass; ++ps) emit(Ez, ps * TEZ, last ? min(ps * TEZ + TEZ, NI2) : TEZ, tt, g0, g1, act);
    if (!last) {
#pragma unroll
      for (int k = 0; k < NZ; ++k) {
        if (k < p) {
          U[k] = U[k + TEZ];
          U01[k] = U01[k + TEZ];
          U10[k] = U10[k + TEZ];
          Y0[k] = Y0[k + TEZ];
          Y1[k] = Y1[k + TEZ];
          Y2[k] = Y2[k + TEZ];
        } else {
          Y0[k] = Y1[k] = Y2[k] = 0.0;
        }
      }
    }
  }
}

// Column-register variant of the Cahn-Hilliard residual (the arithmetic of ch3_body, regrouped):
// tiles of TEX x TEX x TEZ elements with TEX Q <= 16, one lane per Gauss-point column (g0, g1).  The
// axis-0 contraction (B.c, B'.c, B''.c, B.cdot) goes through LDS; each lane then holds the six axis-1
// products of its column for all NZ = TEZ + p function planes in registers, forms c, grad c, Lap c and
// cdot at its points, the point terms S0, F, S2 and the four transposed axis-2 sums in registers; the
// transposed axis-1 and axis-0 contractions go through LDS.  One FP64 atomic per tile function, the
// output zeroed before.
template <int P, int TEZ>
struct Chr3 {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TEX = 16 / Q, G = TEX * Q, GS = G % 2 ? G : G + 1;
  static constexpr int NI = TEX + p, NZ = TEZ + p;
  static constexpr int n_c = NZ * NI * NI, n_a = NZ * NI * GS, n_y = NZ * G * GS;
  static constexpr int n_b = 6 * G * P + 2 * G + 3 * TEZ * Q * P + TEZ * Q;
  static constexpr size_t total = (size_t)(2 * n_c + 4 * n_a + 4 * n_y + n_b) * sizeof(double);
  static_assert(G * G <= kThreads, "one lane per Gauss-point column");
  static_assert(total <= 65536, "static LDS");
};

template <int P, int TEZ>
__device__ inline void chr3_body(const DevProblem &pb, const int tile, const double *__restrict__ Cv,
                                 const double *__restrict__ Cd, double theta, double lam, double *__restrict__ Y,
                                 double *__restrict__ lds) {
  using S_ = Chr3<P, TEZ>;
  constexpr int p = S_::p, Q = S_::Q, TEX = S_::TEX, G = S_::G, GS = S_::GS, NI = S_::NI, NZ = S_::NZ;
  constexpr int NT = kThreads, GP = G * P, NA = NZ * NI * G, ZP = TEZ * Q * P;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TEX - 1) / TEX, nt1 = (ne1 + TEX - 1) / TEX;
  const int E0 = (tile % nt0) * TEX, E1 = ((tile / nt0) % nt1) * TEX, E2 = (tile / (nt0 * nt1)) * TEZ;
  const int NE0 = min(TEX, ne0 - E0), NE1 = min(TEX, ne1 - E1), NE2 = min(TEZ, ne2 - E2);
  const int G0 = NE0 * Q, G1 = NE1 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p, NI2 = NE2 + p;
  double *c = lds, *cd = c + S_::n_c;                                       // [k2][k1][k0]
  double *aB = cd + S_::n_c, *aD = aB + S_::n_a, *aE = aD + S_::n_a, *aR = aE + S_::n_a;   // [k2][k1][g0]
  double *Yb = aR + S_::n_a, *Y0 = Yb + S_::n_y, *Y1 = Y0 + S_::n_y, *Ysl = Y1 + S_::n_y;   // [k2][g1][g0]
  double *tb = Ysl + S_::n_y, *tw = tb + 6 * GP, *t2 = tw + 2 * G, *w2 = t2 + 3 * ZP;
  double *Zb = aB, *Zd = aD, *Ze = aE;                                      // transposed axis 1, [k2][k1][g0]
  const double *B0 = tb, *D0 = tb + GP, *E0t = tb + 2 * GP, *B1 = tb + 3 * GP, *D1 = tb + 4 * GP, *E1t = tb + 5 * GP;
  const int t = threadIdx.x;
  for (int i = t; i < GP; i += NT) {
    if (i / P < G0) {
      const size_t o = (size_t)E0 * Q * P + i;
      tb[i] = pb.ax[0].B[o];
      tb[GP + i] = pb.ax[0].dB[o];
      tb[2 * GP + i] = pb.ax[0].d2B[o];
    }
    if (i / P < G1) {
      const size_t o = (size_t)E1 * Q * P + i;
      tb[3 * GP + i] = pb.ax[1].B[o];
      tb[4 * GP + i] = pb.ax[1].dB[o];
      tb[5 * GP + i] = pb.ax[1].d2B[o];
    }
  }
  for (int i = t; i < G; i += NT) {
    if (i < G0) tw[i] = pb.ax[0].wq[(size_t)E0 * Q + i];
    if (i < G1) tw[G + i] = pb.ax[1].wq[(size_t)E1 * Q + i];
  }
  for (int i = t; i < ZP; i += NT)
    if (i / (Q * P) < NE2) {
      const size_t o = (size_t)E2 * Q * P + i;
      t2[i] = pb.ax[2].B[o];
      t2[ZP + i] = pb.ax[2].dB[o];
      t2[2 * ZP + i] = pb.ax[2].d2B[o];
    }
  for (int i = t; i < TEZ * Q; i += NT)
    if (i / Q < NE2) w2[i] = pb.ax[2].wq[(size_t)E2 * Q + i];
  for (int i = t; i < S_::n_c; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    const int64_t A = wrap_fn(pb.ax[0], E0 + k0) +
                      (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2));
    c[i] = Cv[A];
    cd[i] = Cd[A];
  }
  __syncthreads();
  for (int i = t; i < NA; i += NT) {
    const int g0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), el0 = g0 / Q;
    if (g0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    const int o = (k2 * NI + k1) * NI + el0;
    double vb = 0, vd = 0, ve = 0, vr = 0;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) {
      vb += B0[g0 * P + a0] * c[o + a0];
      vd += D0[g0 * P + a0] * c[o + a0];
      ve += E0t[g0 * P + a0] * c[o + a0];
      vr += B0[g0 * P + a0] * cd[o + a0];
    }
    const int w = (k2 * NI + k1) * GS + g0;
    aB[w] = vb;
    aD[w] = vd;
    aE[w] = ve;
    aR[w] = vr;
  }
  __syncthreads();
  const int g0 = t % G, g1 = t / G;
  const bool act = t < G * G && g0 < G0 && g1 < G1;
  if (act) {
    const int el1 = g1 / Q;
    double b1[P], d1[P], e1[P];
#pragma unroll
    for (int a = 0; a < P; ++a) {
      b1[a] = B1[g1 * P + a];
      d1[a] = D1[g1 * P + a];
      e1[a] = E1t[g1 * P + a];
    }
    // axis 1: bb = B1 B0 c, db = B1 B0' c, be = B1'' B0 c, eb = B1 B0'' c, bd = B1' B0 c, rb = B1 B0 cdot
    double bb[NZ], db[NZ], be[NZ], eb[NZ], bd[NZ], rb[NZ];
#pragma unroll
    for (int k2 = 0; k2 < NZ; ++k2) {
      double x0 = 0, x1 = 0, x2 = 0, x3 = 0, x4 = 0, x5 = 0;
      if (k2 < NI2) {
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) {
          const int r = (k2 * NI + el1 + a1) * GS + g0;
          x0 += b1[a1] * aB[r];
          x1 += b1[a1] * aD[r];
          x2 += e1[a1] * aB[r];
          x3 += b1[a1] * aE[r];
          x4 += d1[a1] * aB[r];
          x5 += b1[a1] * aR[r];
        }
      }
      bb[k2] = x0;
      db[k2] = x1;
      be[k2] = x2;
      eb[k2] = x3;
      bd[k2] = x4;
      rb[k2] = x5;
    }
    double yb[NZ], y0[NZ], y1[NZ], ys[NZ];
#pragma unroll
    for (int k = 0; k < NZ; ++k) yb[k] = y0[k] = y1[k] = ys[k] = 0.0;
    const double w01 = tw[g0] * tw[G + g1];
#pragma unroll
    for (int el2 = 0; el2 < TEZ; ++el2) {
      if (el2 >= NE2) break;
#pragma unroll
      for (int q2 = 0; q2 < Q; ++q2) {
        const int o = (el2 * Q + q2) * P;
        double cv = 0, c0 = 0, c1 = 0, c2 = 0, lc = 0, cr = 0;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) {
          const double b = t2[o + a2], d = t2[ZP + o + a2], e = t2[2 * ZP + o + a2];
          const int k = el2 + a2;
          cv += b * bb[k];
          c0 += b * db[k];
          c1 += b * bd[k];
          c2 += d * bb[k];
          lc += b * (eb[k] + be[k]) + e * bb[k];
          cr += b * rb[k];
        }
        const double W = w01 * w2[el2 * Q + q2];
        const double M = cv * (1.0 - cv), dM = 1.0 - 2.0 * cv, dmu = 1.0 / (2.0 * theta * cv * (1.0 - cv)) - 2.0;
        const double sg = W * (M * dmu + lam * dM * lc);
        const double F0 = sg * c0, F1 = sg * c1, F2 = sg * c2, S0 = W * cr, S2 = W * lam * M * lc;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) {
          const double b = t2[o + a2], d = t2[ZP + o + a2], e = t2[2 * ZP + o + a2];
          const int k = el2 + a2;
          yb[k] += b * S0 + d * F2 + e * S2;
          y0[k] += b * F0;
          y1[k] += b * F1;
          ys[k] += b * S2;
        }
      }
    }
#pragma unroll
    for (int k2 = 0; k2 < NZ; ++k2) {
      if (k2 < NI2) {
        const int w = (k2 * G + g1) * GS + g0;
        Yb[w] = yb[k2];
        Y0[w] = y0[k2];
        Y1[w] = y1[k2];
        Ysl[w] = ys[k2];
      }
    }
  }
  __syncthreads();
  for (int i = t; i < NA; i += NT) {
    const int gg0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI);
    if (gg0 >= G0 || k1 >= NI1 || k2 >= NI2) continue;
    double zb = 0, zd = 0, ze = 0;
#pragma unroll
    for (int a1 = 0; a1 <= p; ++a1) {
      const int el1 = k1 - a1;
      if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const int gg1 = el1 * Q + q1, w = (k2 * G + gg1) * GS + gg0, o = gg1 * P + a1;
        zb += B1[o] * Yb[w] + D1[o] * Y1[w] + E1t[o] * Ysl[w];
        zd += B1[o] * Y0[w];
        ze += B1[o] * Ysl[w];
      }
    }
    const int w = (k2 * NI + k1) * GS + gg0;
    Zb[w] = zb;
    Zd[w] = zd;
    Ze[w] = ze;
  }
  __syncthreads();
  for (int i = t; i < S_::n_c; i += NT) {
    const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
    if (k0 >= NI0 || k1 >= NI1 || k2 >= NI2) continue;
    double r = 0;
#pragma unroll
    for (int a0 = 0; a0 <= p; ++a0) {
      const int el0 = k0 - a0;
      if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        const int gg0 = el0 * Q + q0, w = (k2 * NI + k1) * GS + gg0, o = gg0 * P + a0;
        r += B0[o] * Zb[w] + D0[o] * Zd[w] + E0t[o] * Ze[w];
      }
    }
    atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                 (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], E2 + k2))],
              r);
  }
}

// Streamed variant of chr3_body: the x-y tiles and lanes of chr3_body, walking a run of chunks of TEZ
// elements along axis 2 with the p open function planes (their six axis-1 products and four transposed
// axis-2 sums) carried in registers from chunk to chunk, as res3s_body does for the Bratu residual.
template <int P, int TEZ>
struct Chr3S {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TEX = 16 / Q, G = TEX * Q, GS = G % 2 ? G : G + 1;
  static constexpr int NI = TEX + p, NZ = TEZ + p;
  static constexpr int n_c = NZ * NI * NI, n_a = NZ * NI * GS, n_y = TEZ * G * GS;
  static constexpr int n_b = 6 * G * P + 2 * G + 3 * TEZ * Q * P + TEZ * Q;
  static constexpr size_t total = (size_t)(2 * n_c + 4 * n_a + 4 * n_y + n_b) * sizeof(double);
  static_assert(G * G <= kThreads, "one lane per Gauss-point column");
  static_assert(TEZ >= p, "the planes left open by a chunk fit one emission");
  static_assert(total <= 65536, "static LDS");
};

template <int P, int TEZ, int RUNMAX>
__device__ inline void chr3s_body(const DevProblem &pb, const int blk, const int zc, const double *__restrict__ Cv,
                                  const double *__restrict__ Cd, double theta, double lam, double *__restrict__ Y,
                                  double *__restrict__ lds) {
  using S_ = Chr3S<P, TEZ>;
  constexpr int p = S_::p, Q = S_::Q, TEX = S_::TEX, G = S_::G, GS = S_::GS, NI = S_::NI, NZ = S_::NZ;
  constexpr int NT = kThreads, GP = G * P, ZP = TEZ * Q * P;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nt0 = (ne0 + TEX - 1) / TEX, nt1 = (ne1 + TEX - 1) / TEX;
  const int E0 = (blk % nt0) * TEX, E1 = ((blk / nt0) % nt1) * TEX;
  const int Zlo = (blk / (nt0 * nt1)) * zc * TEZ, Zhi = min(ne2, Zlo + zc * TEZ);
  const int NE0 = min(TEX, ne0 - E0), NE1 = min(TEX, ne1 - E1);
  const int G0 = NE0 * Q, G1 = NE1 * Q;
  const int NI0 = NE0 + p, NI1 = NE1 + p;
  double *c = lds, *cd = c + S_::n_c;                                       // [k2][k1][k0], plane k2 = Ez + k2
  double *aB = cd + S_::n_c, *aD = aB + S_::n_a, *aE = aD + S_::n_a, *aR = aE + S_::n_a;   // [k2][k1][g0]
  double *Yb = aR + S_::n_a, *Y0 = Yb + S_::n_y, *Y1 = Y0 + S_::n_y, *Ysl = Y1 + S_::n_y;   // [slot][g1][g0]
  double *tb = Ysl + S_::n_y, *tw = tb + 6 * GP, *t2 = tw + 2 * G, *w2 = t2 + 3 * ZP;
  double *Zb = aB, *Zd = aD, *Ze = aE;                                      // transposed axis 1, [slot][k1][g0]
  const double *B0 = tb, *D0 = tb + GP, *E0t = tb + 2 * GP, *B1 = tb + 3 * GP, *D1 = tb + 4 * GP, *E1t = tb + 5 * GP;
  const int t = threadIdx.x;
  for (int i = t; i < GP; i += NT) {
    if (i / P < G0) {
      const size_t o = (size_t)E0 * Q * P + i;
      tb[i] = pb.ax[0].B[o];
      tb[GP + i] = pb.ax[0].dB[o];
      tb[2 * GP + i] = pb.ax[0].d2B[o];
    }
    if (i / P < G1) {
      const size_t o = (size_t)E1 * Q * P + i;
      tb[3 * GP + i] = pb.ax[1].B[o];
      tb[4 * GP + i] = pb.ax[1].dB[o];
      tb[5 * GP + i] = pb.ax[1].d2B[o];
    }
  }
  for (int i = t; i < G; i += NT) {
    if (i < G0) tw[i] = pb.ax[0].wq[(size_t)E0 * Q + i];
    if (i < G1) tw[G + i] = pb.ax[1].wq[(size_t)E1 * Q + i];
  }
  // open planes: axis-1 products bb = B1 B0 c, db = B1 B0' c, bd = B1' B0 c, rb = B1 B0 cdot and
  // le = (B1'' B0 + B1 B0'') c (the two enter only as a sum, in the Laplacian), and the transposed
  // axis-2 sums yb, y0, y1, ys
  double bb[NZ], db[NZ], le[NZ], bd[NZ], rb[NZ], yb[NZ], y0[NZ], y1[NZ], ys[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) bb[k] = db[k] = le[k] = bd[k] = rb[k] = yb[k] = y0[k] = y1[k] = ys[k] = 0.0;

  // planes [pl0, pl1) of the chunk at Ez (pl1 - pl0 <= TEZ): transposed axes 1 and 0, then the atomics
  auto emit = [&](int Ez, int pl0, int pl1, int ti, int g0, int g1, bool act) {
    if (act) {
#pragma unroll
      for (int k2 = 0; k2 < NZ; ++k2)
        if (k2 >= pl0 && k2 < pl1) {
          const int w = ((k2 - pl0) * G + g1) * GS + g0;
          Yb[w] = yb[k2];
          Y0[w] = y0[k2];
          Y1[w] = y1[k2];
          Ysl[w] = ys[k2];
        }
    }
    __syncthreads();
    const int ns = pl1 - pl0;
    for (int i = ti; i < TEZ * NI * G; i += NT) {
      const int gg0 = i % G, k1 = (i / G) % NI, s = i / (G * NI);
      if (gg0 >= G0 || k1 >= NI1 || s >= ns) continue;
      double zb = 0, zd = 0, ze = 0;
#pragma unroll
      for (int a1 = 0; a1 <= p; ++a1) {
        const int e1 = k1 - a1;
        if (e1 < 0 || e1 >= NE1) continue;
#pragma unroll
        for (int r1 = 0; r1 < Q; ++r1) {
          const int gg1 = e1 * Q + r1, w = (s * G + gg1) * GS + gg0, o = gg1 * P + a1;
          zb += B1[o] * Yb[w] + D1[o] * Y1[w] + E1t[o] * Ysl[w];
          zd += B1[o] * Y0[w];
          ze += B1[o] * Ysl[w];
        }
      }
      const int w = (s * NI + k1) * GS + gg0;
      Zb[w] = zb;
      Zd[w] = zd;
      Ze[w] = ze;
    }
    __syncthreads();
    for (int i = ti; i < TEZ * NI * NI; i += NT) {
      const int k0 = i % NI, k1 = (i / NI) % NI, s = i / (NI * NI);
      if (k0 >= NI0 || k1 >= NI1 || s >= ns) continue;
      double r = 0;
#pragma unroll
      for (int a0 = 0; a0 <= p; ++a0) {
        const int e0 = k0 - a0;
        if (e0 < 0 || e0 >= NE0) continue;
#pragma unroll
        for (int r0 = 0; r0 < Q; ++r0) {
          const int gg0 = e0 * Q + r0, w = (s * NI + k1) * GS + gg0, o = gg0 * P + a0;
          r += B0[o] * Zb[w] + D0[o] * Zd[w] + E0t[o] * Ze[w];
        }
      }
      atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) +
                   (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], Ez + pl0 + s))],
                r);
    }
  };

  // the chunks of a run (at most RUNMAX) are unrolled (see res3s_body)
#pragma unroll
  for (int ch = 0; ch < RUNMAX; ++ch) {
    const int Ez = Zlo + ch * TEZ;
    if (Ez >= Zhi) break;
    const int NE2 = min(TEZ, Zhi - Ez), NI2 = NE2 + p;
    const bool last = Ez + TEZ >= Zhi;
    const int kf = Ez == Zlo ? 0 : p;                  // planes below kf are open from the previous chunk
    int tt = t;                                        // opaque copy of the thread index (see res3s_body)
    asm volatile("" : "+v"(tt));
    const int g0 = tt % G, g1 = tt / G;
    const bool act = tt < G * G && g0 < G0 && g1 < G1;
    // (1) coefficients of the new planes and the chunk's axis-2 rows
    for (int i = tt; i < ZP; i += NT)
      if (i / (Q * P) < NE2) {
        const size_t o = (size_t)Ez * Q * P + i;
        t2[i] = pb.ax[2].B[o];
        t2[ZP + i] = pb.ax[2].dB[o];
        t2[2 * ZP + i] = pb.ax[2].d2B[o];
      }
    for (int i = tt; i < TEZ * Q; i += NT)
      if (i / Q < NE2) w2[i] = pb.ax[2].wq[(size_t)Ez * Q + i];
    for (int i = tt; i < S_::n_c; i += NT) {
      const int k0 = i % NI, k1 = (i / NI) % NI, k2 = i / (NI * NI);
      if (k0 >= NI0 || k1 >= NI1 || k2 < kf || k2 >= NI2) continue;
      const int64_t A = wrap_fn(pb.ax[0], E0 + k0) +
                        (int64_t)n0 * (wrap_fn(pb.ax[1], E1 + k1) + (int64_t)n1 * wrap_fn(pb.ax[2], Ez + k2));
      c[i] = Cv[A];
      cd[i] = Cd[A];
    }
    __syncthreads();
    // (2) axis 0 on the new planes
    for (int i = tt; i < NZ * NI * G; i += NT) {
      const int gg0 = i % G, k1 = (i / G) % NI, k2 = i / (G * NI), e0 = gg0 / Q;
      if (gg0 >= G0 || k1 >= NI1 || k2 < kf || k2 >= NI2) continue;
      const int o = (k2 * NI + k1) * NI + e0;
      double vb = 0, vd = 0, ve = 0, vr = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        vb += B0[gg0 * P + a0] * c[o + a0];
        vd += D0[gg0 * P + a0] * c[o + a0];
        ve += E0t[gg0 * P + a0] * c[o + a0];
        vr += B0[gg0 * P + a0] * cd[o + a0];
      }
      const int w = (k2 * NI + k1) * GS + gg0;
      aB[w] = vb;
      aD[w] = vd;
      aE[w] = ve;
      aR[w] = vr;
    }
    __syncthreads();
    // (3) one lane per Gauss-point column: axis 1 on the new planes, axis 2, the point terms of the
    // Cahn-Hilliard weak form and the transposed axis 2 into the open planes
    if (act) {
      const int el1 = g1 / Q;
      double b1[P], d1[P], e1[P];
#pragma unroll
      for (int a = 0; a < P; ++a) {
        b1[a] = B1[g1 * P + a];
        d1[a] = D1[g1 * P + a];
        e1[a] = E1t[g1 * P + a];
      }
#pragma unroll
      for (int k2 = 0; k2 < NZ; ++k2) {
        if (k2 < kf) continue;
        double x0 = 0, x1 = 0, x2 = 0, x4 = 0, x5 = 0;
        if (k2 < NI2) {
#pragma unroll
          for (int a1 = 0; a1 < P; ++a1) {
            const int r = (k2 * NI + el1 + a1) * GS + g0;
            x0 += b1[a1] * aB[r];
            x1 += b1[a1] * aD[r];
            x2 += e1[a1] * aB[r] + b1[a1] * aE[r];
            x4 += d1[a1] * aB[r];
            x5 += b1[a1] * aR[r];
          }
        }
        bb[k2] = x0;
        db[k2] = x1;
        le[k2] = x2;
        bd[k2] = x4;
        rb[k2] = x5;
      }
      const double w01 = tw[g0] * tw[G + g1];
#pragma unroll
      for (int el2 = 0; el2 < TEZ; ++el2) {
        if (el2 >= NE2) break;
#pragma unroll
        for (int q2 = 0; q2 < Q; ++q2) {
          const int o = (el2 * Q + q2) * P;
          double cv = 0, c0 = 0, c1 = 0, c2 = 0, lc = 0, cr = 0;
#pragma unroll
          for (int a2 = 0; a2 < P; ++a2) {
            const double b = t2[o + a2], d = t2[ZP + o + a2], e = t2[2 * ZP + o + a2];
            const int k = el2 + a2;
            cv += b * bb[k];
            c0 += b * db[k];
            c1 += b * bd[k];
            c2 += d * bb[k];
            lc += b * le[k] + e * bb[k];
            cr += b * rb[k];
          }
          const double W = w01 * w2[el2 * Q + q2];
          const double M = cv * (1.0 - cv), dM = 1.0 - 2.0 * cv, dmu = 1.0 / (2.0 * theta * cv * (1.0 - cv)) - 2.0;
          const double sg = W * (M * dmu + lam * dM * lc);
          const double F0 = sg * c0, F1 = sg * c1, F2 = sg * c2, S0 = W * cr, S2 = W * lam * M * lc;
#pragma unroll
          for (int a2 = 0; a2 < P; ++a2) {
            const double b = t2[o + a2], d = t2[ZP + o + a2], e = t2[2 * ZP + o + a2];
            const int k = el2 + a2;
            yb[k] += b * S0 + d * F2 + e * S2;
            y0[k] += b * F0;
            y1[k] += b * F1;
            ys[k] += b * S2;
          }
        }
      }
    }
    // (4) the complete planes go out; the open ones move down to the first p planes
    const int npass = (last && NI2 > TEZ) ? 2 : 1;
    for (int ps = 0; ps < npass; ++ps) emit(Ez, ps * TEZ, last ? min(ps * TEZ + TEZ, NI2) : TEZ, tt, g0, g1, act);
    if (!last) {
#pragma unroll
      for (int k = 0; k < NZ; ++k) {
        if (k < p) {
          bb[k] = bb[k + TEZ];
          db[k] = db[k + TEZ];
          le[k] = le[k + TEZ];
          bd[k] = bd[k + TEZ];
          rb[k] = rb[k + TEZ];
          yb[k] = yb[k + TEZ];
          y0[k] = y0[k + TEZ];
          y1[k] = y1[k + TEZ];
          ys[k] = ys[k + TEZ];
        } else {
          yb[k] = y0[k] = y1[k] = ys[k] = 0.0;
        }
      }
    }
  }
}

}  // namespace rs3
}  // namespace iga
