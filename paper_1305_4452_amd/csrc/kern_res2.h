// Tiled 2D residual for the analytic metric (identity geometry, no weights, kappa one or
// element-wise; every interior knot simple, so element e carries functions e .. e + p, wrapped on a
// periodic axis).  Shared by the single-problem and batched launchers.
//
// A workgroup owns TE x TE elements.  The weak-form residual of Sec. 3,
//   R_A = sum_g [ kappa W grad N_A . grad u  -  W N_A (lambda e^u + f) ],
// is evaluated by sum factorisation over the whole tile: the coefficients of the tile's
// (TE + p)^2 functions are contracted to u, du/dxi0, du/dxi1 (and f) at its (TE Q)^2 Gauss
// points, the point integrands are formed, and the transposed contractions give the tile's
// contribution to each of those functions, added to R with one FP64 atomic per function (the
// functions on the tile border are shared with neighbouring tiles).  R must be zeroed before and
// the Dirichlet rows set afterwards, as for the element-by-element kernel.
#pragma once

#include "iga_impl.h"

namespace iga {
namespace rst {

constexpr int kThreads = 256;

// elements per tile side: TE * Q = 40 Gauss points per axis (V = 0), or about 20 (V = 1: less idle work
// on small meshes; the batched solver picks per degree and size class by timing both)
template <int P, int VS = 0>
struct Res2 {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TE = (VS ? 20 : 40) / Q;
  static constexpr int NI = TE + p, G = TE * Q;
  // doubles: sU, sF [NI][NI]; V, D, VF [NI][G]; F0, F1, S [G][G]; the tile's basis values and
  // derivatives [axis][B|dB][G][P] and quadrature weights [axis][G]
  static constexpr int n_u = NI * NI, n_v = NI * G, n_f = G * G, n_b = 4 * G * P + 2 * G;
  static constexpr size_t total = (size_t)(2 * n_u + 3 * n_v + 3 * n_f + n_b) * sizeof(double);
};

// i / d for 0 <= i < 2^16 and 1 <= d <= 64 from inv = 1/d in FP32: (i + 1/2) / d lies at least 1/(2d)
// from an integer, and the two roundings move it by less than 2^16 * 2^-23 / d, so the truncation is exact.
__device__ inline int small_div(int i, float inv) { return (int)(((float)i + 0.5f) * inv); }

__host__ __device__ inline int res2_tiles(int ne0, int ne1, int TE) {
  return ((ne0 + TE - 1) / TE) * ((ne1 + TE - 1) / TE);
}

template <int P, int VS = 0>
__device__ inline void res2_body(const DevProblem &pb, const int tile, const double *__restrict__ U,
                                 double *__restrict__ R, double *__restrict__ lds) {
  using S_ = Res2<P, VS>;
  constexpr int p = S_::p, Q = S_::Q, TE = S_::TE, NI = S_::NI, G = S_::G;
  const int n0 = pb.n[0], ne0 = pb.ne[0], ne1 = pb.ne[1];
  const int nt0 = (ne0 + TE - 1) / TE;
  const int E0 = (tile % nt0) * TE, E1 = (tile / nt0) * TE;
  const int NE0 = min(TE, ne0 - E0), NE1 = min(TE, ne1 - E1);
  const int G0 = NE0 * Q, G1 = NE1 * Q;
  // the tile's functions: f0 .. f0 + NI0 - 1 along axis 0 (likewise axis 1)
  const int f0 = E0, f1 = E1, NI0 = NE0 + p, NI1 = NE1 + p;
  double *sU = lds, *sF = sU + S_::n_u;
  double *V = sF + S_::n_u, *D = V + S_::n_v, *VF = D + S_::n_v;
  double *F0 = VF + S_::n_v, *F1 = F0 + S_::n_f, *Sg = F1 + S_::n_f;
  double *Ya = V, *Yb = D;   // reused once the point integrands are formed
  constexpr int GP = G * P;
  double *sB = Sg + S_::n_f, *sW = sB + 4 * GP;
  const double *B0 = sB, *dB0 = sB + GP, *B1 = sB + 2 * GP, *dB1 = sB + 3 * GP, *W0 = sW, *W1 = sW + G;
  const int t = threadIdx.x;
  const bool src = pb.src != nullptr;
  const bool kel = pb.kappa_mode == IGA_KAPPA_ELEMENT;
  const float iNI0 = 1.0f / NI0, iG0 = 1.0f / G0;

  // the tile's rows of the basis tables (point g of axis d is global point E_d Q + g)
  for (int i = t; i < G0 * P; i += kThreads) {
    sB[i] = pb.ax[0].B[(size_t)E0 * Q * P + i];
    sB[GP + i] = pb.ax[0].dB[(size_t)E0 * Q * P + i];
  }
  for (int i = t; i < G1 * P; i += kThreads) {
    sB[2 * GP + i] = pb.ax[1].B[(size_t)E1 * Q * P + i];
    sB[3 * GP + i] = pb.ax[1].dB[(size_t)E1 * Q * P + i];
  }
  for (int i = t; i < G0; i += kThreads) sW[i] = pb.ax[0].wq[(size_t)E0 * Q + i];
  for (int i = t; i < G1; i += kThreads) sW[G + i] = pb.ax[1].wq[(size_t)E1 * Q + i];
  for (int i = t; i < NI0 * NI1; i += kThreads) {
    const int k1 = small_div(i, iNI0), k0 = i - k1 * NI0;
    const int64_t A = wrap_fn(pb.ax[0], f0 + k0) + (int64_t)n0 * wrap_fn(pb.ax[1], f1 + k1);   // eq:map-wrap
    sU[k1 * NI + k0] = U[A];
    if (src) sF[k1 * NI + k0] = pb.src[A];
  }
  __syncthreads();
  // axis 0: coefficients -> (value, derivative) at the Gauss points, per function row k1
  for (int i = t; i < NI1 * G0; i += kThreads) {
    const int k1 = small_div(i, iG0), g0 = i - k1 * G0, el0 = g0 / Q;
    double v = 0, d = 0, vf = 0;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) {
      const double c = sU[k1 * NI + el0 + a0];
      v += B0[g0 * P + a0] * c;
      d += dB0[g0 * P + a0] * c;
      if (src) vf += B0[g0 * P + a0] * sF[k1 * NI + el0 + a0];
    }
    V[k1 * G + g0] = v;
    D[k1 * G + g0] = d;
    VF[k1 * G + g0] = vf;
  }
  __syncthreads();
  // axis 1 and the point integrands
  {
    const double lam = pb.lambda;
    for (int i = t; i < G1 * G0; i += kThreads) {
      const int g1 = small_div(i, iG0), g0 = i - g1 * G0, el1 = g1 / Q, el0 = g0 / Q;
      double u = 0, u0 = 0, u1 = 0, f = 0;
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) {
        const double b = B1[g1 * P + a1], db = dB1[g1 * P + a1];
        const int r = (el1 + a1) * G + g0;
        u += b * V[r];
        u0 += b * D[r];
        u1 += db * V[r];
        f += b * VF[r];
      }
      const double W = W0[g0] * W1[g1];
      const double kw = (kel ? pb.kel[(E0 + el0) + (int64_t)ne0 * (E1 + el1)] : 1.0) * W;
      F0[g1 * G + g0] = kw * u0;
      F1[g1 * G + g0] = kw * u1;
      Sg[g1 * G + g0] = -W * (lam * exp(u) + (src ? f : 0.0));
    }
  }
  __syncthreads();
  // transposed axis 1: Ya[k1][g0] = sum F0 N_k1, Yb[k1][g0] = sum F1 N'_k1 + S N_k1
  for (int i = t; i < NI1 * G0; i += kThreads) {
    const int k1 = small_div(i, iG0), g0 = i - k1 * G0;
    double ya = 0, yb = 0;
#pragma unroll
    for (int a1 = 0; a1 <= p; ++a1) {
      const int el1 = k1 - a1;
      if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
      for (int q1 = 0; q1 < Q; ++q1) {
        const int g1 = el1 * Q + q1, r = g1 * G + g0;
        const double b = B1[g1 * P + a1];
        ya += F0[r] * b;
        yb += F1[r] * dB1[g1 * P + a1] + Sg[r] * b;
      }
    }
    Ya[k1 * G + g0] = ya;
    Yb[k1 * G + g0] = yb;
  }
  __syncthreads();
  // transposed axis 0 and the scatter of the tile's contributions
  for (int i = t; i < NI0 * NI1; i += kThreads) {
    const int k1 = small_div(i, iNI0), k0 = i - k1 * NI0;
    double r = 0;
#pragma unroll
    for (int a0 = 0; a0 <= p; ++a0) {
      const int el0 = k0 - a0;
      if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        const int g0 = el0 * Q + q0;
        r += Ya[k1 * G + g0] * dB0[g0 * P + a0] + Yb[k1 * G + g0] * B0[g0 * P + a0];
      }
    }
    atomicAdd(&R[wrap_fn(pb.ax[0], f0 + k0) + (int64_t)n0 * wrap_fn(pb.ax[1], f1 + k1)], r);
  }
}

// Cahn-Hilliard residual on x = xi without weights by 2D tiles (the form of the element kernel):
// forward, axis 0 gives B.c, B'.c, B''.c and B.cdot per function row, axis 1 the value, gradient,
// Laplacian and rate at every point; the point terms are S0 = W cdot, F = W (M mu' + lam M' Lap c)
// grad c and S2 = W lam M Lap c; transposed, B0 (B1 S0 + B1' F1 + B1'' S2) + B0' B1 F0 + B0'' B1 S2
// is contracted axis by axis.  Tiles of about 24 Gauss points per side keep four workgroups or more
// per CU on a 256^2 mesh.  One FP64 atomic per tile function; the output must be zeroed before.
template <int P>
struct Ch2 {
  static constexpr int p = P - 1, Q = P;
  static constexpr int TE = 24 / Q > 2 ? 24 / Q : 2;
  static constexpr int NI = TE + p, G = TE * Q, GP = G * P;
  static constexpr int n_c = NI * NI, n_a = NI * G, n_f = G * G, n_b = 6 * GP + 2 * G;
  static constexpr size_t total = (size_t)(2 * n_c + 4 * n_a + 4 * n_f + n_b) * sizeof(double);
};

template <int P>
__device__ inline void ch2_body(const DevProblem &pb, const int tile, const double *__restrict__ Cv,
                                const double *__restrict__ Cd, double theta, double lam, double *__restrict__ Y,
                                double *__restrict__ lds) {
  using S_ = Ch2<P>;
  constexpr int p = S_::p, Q = S_::Q, TE = S_::TE, NI = S_::NI, G = S_::G, GP = S_::GP;
  const int n0 = pb.n[0], ne0 = pb.ne[0], ne1 = pb.ne[1];
  const int nt0 = (ne0 + TE - 1) / TE;
  const int E0 = (tile % nt0) * TE, E1 = (tile / nt0) * TE;
  const int NE0 = min(TE, ne0 - E0), NE1 = min(TE, ne1 - E1);
  const int G0 = NE0 * Q, G1 = NE1 * Q, NI0 = NE0 + p, NI1 = NE1 + p;
  double *c = lds, *cd = c + S_::n_c;                                                    // [k1][k0]
  double *aB = cd + S_::n_c, *aD = aB + S_::n_a, *aE = aD + S_::n_a, *aR = aE + S_::n_a;  // [k1][g0]
  double *F0 = aR + S_::n_a, *F1 = F0 + S_::n_f, *S0 = F1 + S_::n_f, *S2 = S0 + S_::n_f;  // [g1][g0]
  double *tb = S2 + S_::n_f, *tw = tb + 6 * GP;   // [axis][B|B'|B''][G][P], [axis][G]
  double *Zb = aB, *Zd = aD, *Ze = aE;            // [k1][g0], once the point terms are formed
  const int t = threadIdx.x;
  const int Ed[2] = {E0, E1}, Gd[2] = {G0, G1};
  for (int d = 0; d < 2; ++d) {
    const AxisDev &ax = pb.ax[d];
    double *T = tb + d * 3 * GP;
    for (int i = t; i < Gd[d] * P; i += kThreads) {
      const size_t o = (size_t)Ed[d] * Q * P + i;
      T[i] = ax.B[o];
      T[GP + i] = ax.dB[o];
      T[2 * GP + i] = ax.d2B[o];
    }
    for (int i = t; i < Gd[d]; i += kThreads) tw[d * G + i] = ax.wq[(size_t)Ed[d] * Q + i];
  }
  for (int i = t; i < NI * NI; i += kThreads) {
    const int k0 = i % NI, k1 = i / NI;
    if (k0 >= NI0 || k1 >= NI1) continue;
    const int64_t A = wrap_fn(pb.ax[0], E0 + k0) + (int64_t)n0 * wrap_fn(pb.ax[1], E1 + k1);   // eq:map-wrap
    c[i] = Cv[A];
    cd[i] = Cd[A];
  }
  __syncthreads();
  {
    const double *B = tb, *D = tb + GP, *E = tb + 2 * GP;
    for (int i = t; i < NI * G; i += kThreads) {
      const int g0 = i % G, k1 = i / G, el0 = g0 / Q;
      if (g0 >= G0 || k1 >= NI1) continue;
      const int o = k1 * NI + el0;
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
    const double *B = tb + 3 * GP, *D = tb + 4 * GP, *E = tb + 5 * GP;
    for (int i = t; i < G * G; i += kThreads) {
      const int g0 = i % G, g1 = i / G, el1 = g1 / Q;
      if (g0 >= G0 || g1 >= G1) continue;
      double cv = 0, c0 = 0, c1 = 0, lc = 0, cr = 0;
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) {
        const int r = (el1 + a1) * G + g0, o = g1 * P + a1;
        const double b = B[o];
        cv += b * aB[r];
        c0 += b * aD[r];
        c1 += D[o] * aB[r];
        lc += b * aE[r] + E[o] * aB[r];
        cr += b * aR[r];
      }
      const double W = tw[g0] * tw[G + g1];
      const double M = cv * (1.0 - cv), dM = 1.0 - 2.0 * cv, dmu = 1.0 / (2.0 * theta * cv * (1.0 - cv)) - 2.0;
      const double sg = W * (M * dmu + lam * dM * lc);
      F0[i] = sg * c0;
      F1[i] = sg * c1;
      S0[i] = W * cr;
      S2[i] = W * lam * M * lc;
    }
  }
  __syncthreads();
  {
    const double *B = tb + 3 * GP, *D = tb + 4 * GP, *E = tb + 5 * GP;
    for (int i = t; i < NI * G; i += kThreads) {
      const int g0 = i % G, k1 = i / G;
      if (g0 >= G0 || k1 >= NI1) continue;
      double zb = 0, zd = 0, ze = 0;
#pragma unroll
      for (int a1 = 0; a1 <= p; ++a1) {
        const int el1 = k1 - a1;
        if (el1 < 0 || el1 >= NE1) continue;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          const int g1 = el1 * Q + q1, w = g1 * G + g0, o = g1 * P + a1;
          zb += B[o] * S0[w] + D[o] * F1[w] + E[o] * S2[w];
          zd += B[o] * F0[w];
          ze += B[o] * S2[w];
        }
      }
      Zb[i] = zb;
      Zd[i] = zd;
      Ze[i] = ze;
    }
  }
  __syncthreads();
  {
    const double *B = tb, *D = tb + GP, *E = tb + 2 * GP;
    for (int i = t; i < NI * NI; i += kThreads) {
      const int k0 = i % NI, k1 = i / NI;
      if (k0 >= NI0 || k1 >= NI1) continue;
      double r = 0;
#pragma unroll
      for (int a0 = 0; a0 <= p; ++a0) {
        const int el0 = k0 - a0;
        if (el0 < 0 || el0 >= NE0) continue;
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          const int g0 = el0 * Q + q0, w = k1 * G + g0, o = g0 * P + a0;
          r += B[o] * Zb[w] + D[o] * Zd[w] + E[o] * Ze[w];
        }
      }
      atomicAdd(&Y[wrap_fn(pb.ax[0], E0 + k0) + (int64_t)n0 * wrap_fn(pb.ax[1], E1 + k1)], r);
    }
  }
}

}  // namespace rst
}  // namespace iga
