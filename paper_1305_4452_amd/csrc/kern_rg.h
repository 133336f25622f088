// Row-gather helpers and the 2D row-gather body, shared by the single-problem and batched
// launchers.
#pragma once

#include "iga_impl.h"

namespace iga {
namespace rgk {

struct Term {
  int coef;
  int x[3];
  int y[3];
};
// Term tables (same stream numbering as the element-matrix kernels).
static __constant__ Term r_terms3_full[16] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {0, 0, 1}, {0, 0, 1}},
    {3, {1, 0, 0}, {0, 1, 0}}, {3, {0, 1, 0}, {1, 0, 0}}, {4, {1, 0, 0}, {0, 0, 1}},
    {4, {0, 0, 1}, {1, 0, 0}}, {5, {0, 1, 0}, {0, 0, 1}}, {5, {0, 0, 1}, {0, 1, 0}},
    {6, {0, 0, 0}, {1, 0, 0}}, {7, {0, 0, 0}, {0, 1, 0}}, {8, {0, 0, 0}, {0, 0, 1}},
    {6, {1, 0, 0}, {0, 0, 0}}, {7, {0, 1, 0}, {0, 0, 0}}, {8, {0, 0, 1}, {0, 0, 0}},
    {9, {0, 0, 0}, {0, 0, 0}}};
static __constant__ Term r_terms3_diag[4] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {0, 0, 1}, {0, 0, 1}}, {9, {0, 0, 0}, {0, 0, 0}}};
static __constant__ Term r_terms2_full[9] = {
    {0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {2, {1, 0, 0}, {0, 1, 0}},
    {2, {0, 1, 0}, {1, 0, 0}}, {3, {0, 0, 0}, {1, 0, 0}}, {4, {0, 0, 0}, {0, 1, 0}},
    {3, {1, 0, 0}, {0, 0, 0}}, {4, {0, 1, 0}, {0, 0, 0}}, {5, {0, 0, 0}, {0, 0, 0}}};
static __constant__ Term r_terms2_diag[3] = {{0, {1, 0, 0}, {1, 0, 0}}, {1, {0, 1, 0}, {0, 1, 0}}, {5, {0, 0, 0}, {0, 0, 0}}};

constexpr int rg_threads(int nown) { return nown <= 256 ? 256 : ((nown + 63) / 64) * 64; }

// Per-point coefficient streams at one quadrature point (see the element kernels):
//  analytic metric: stream 0 = kappa W (all diagonal D' entries), stream 9/5 = m = -lambda W e^u
//  geometry table:  D' (6|3), h = -D' g (3|2), m'' = g.D'g + m'  with m' = -lambda (W/w)(1/w) e^{u}
template <int DIM, bool TABLE>
__device__ inline void rg_coefs(const DevProblem &pb, int64_t e, int q, int QD, double W, double kap, double ut,
                                double *cs) {
  const double lam = pb.lambda;
  if constexpr (!TABLE) {
    cs[0] = kap * W;
    cs[1] = -lam * W * exp(ut);
  } else {
    constexpr int NG = geo_streams(DIM);
    const double *G = pb.geo + (size_t)e * NG * QD + q;
    if (DIM == 3) {
      double D[3][3];
      D[0][0] = G[0]; D[1][1] = G[QD]; D[2][2] = G[2 * QD];
      D[0][1] = D[1][0] = G[3 * QD]; D[0][2] = D[2][0] = G[4 * QD]; D[1][2] = D[2][1] = G[5 * QD];
      double g[3] = {G[6 * QD], G[7 * QD], G[8 * QD]}, Wow = G[9 * QD], iw = G[10 * QD];
      double Dg[3];
      for (int k = 0; k < 3; ++k) Dg[k] = D[k][0] * g[0] + D[k][1] * g[1] + D[k][2] * g[2];
      double m = -lam * Wow * iw * exp(ut * iw);
      cs[0] = D[0][0]; cs[1] = D[1][1]; cs[2] = D[2][2]; cs[3] = D[0][1]; cs[4] = D[0][2]; cs[5] = D[1][2];
      cs[6] = -Dg[0]; cs[7] = -Dg[1]; cs[8] = -Dg[2];
      cs[9] = g[0] * Dg[0] + g[1] * Dg[1] + g[2] * Dg[2] + m;
    } else {
      double D00 = G[0], D11 = G[QD], D01 = G[2 * QD], g0 = G[3 * QD], g1 = G[4 * QD];
      double Wow = G[5 * QD], iw = G[6 * QD];
      double Dg0 = D00 * g0 + D01 * g1, Dg1 = D01 * g0 + D11 * g1;
      double m = -lam * Wow * iw * exp(ut * iw);
      cs[0] = D00; cs[1] = D11; cs[2] = D01; cs[3] = -Dg0; cs[4] = -Dg1;
      cs[5] = g0 * Dg0 + g1 * Dg1 + m;
    }
  }
  (void)W;
  (void)kap;
}

// maps a term's coefficient index to the compact analytic stream index
template <bool TABLE, int DIM>
__device__ inline int stream_of(int coef) {
  if (TABLE) return coef;
  return (coef == (DIM == 3 ? 9 : 5)) ? 1 : 0;
}

template <typename OT>
__device__ inline void store_val(OT *vals, int64_t slot, double v) {
  vals[slot] = (OT)v;
}

// ------------------------------------------------------------------------------------------
// 2D: pencils are rows with fixed i1; level 1 contracts axis 1, level 2 streams axis 0.
// ------------------------------------------------------------------------------------------
template <int P, bool TABLE, int B1, typename CT, typename OT>
__device__ inline void rowgather2_body(const DevProblem &pb, const int bid, const double *__restrict__ U,
                                       OT *__restrict__ vals) {
  constexpr int p = P - 1, Q = P, W7 = 2 * p + 1;
  constexpr int NOWN = B1 * W7;
  constexpr int NT = rg_threads(NOWN);
  constexpr int ME1 = B1 + p, MG1 = ME1 * Q, MI1 = ME1 + p;
  constexpr int NCS = TABLE ? 6 : 2;
  constexpr int NC0 = TABLE ? 4 : 2;
  __shared__ CT tX1[2][ME1][Q][P];
  __shared__ double tB1d[ME1][Q][P], tW1[ME1][Q];
  __shared__ CT tX0[2][Q][P];
  __shared__ double tB0d[Q][P], tW0[Q];
  __shared__ double sU[P][MI1], V0[MI1];
  __shared__ CT cs[NCS][MG1];
  __shared__ CT T1[NC0][B1][W7];
  __shared__ int c0Code[4], nC0;

  const int t = threadIdx.x;
  const int I1 = bid * B1;
  const int E1lo = max(0, I1 - p), E1hi = min(pb.ne[1] - 1, I1 + B1 - 1);
  const int NE1 = E1hi - E1lo + 1, G1 = NE1 * Q, NI1 = NE1 + p;
  const int n0 = pb.n[0], n1 = pb.n[1];
  const Term *terms = TABLE ? r_terms2_full : r_terms2_diag;
  const int nterms = TABLE ? 9 : 3;
  if (t == 0) {
    int n0c = 0;
    for (int ti = 0; ti < nterms; ++ti) {
      int c0 = (terms[ti].x[0] << 1) | terms[ti].y[0], j = 0;
      while (j < n0c && c0Code[j] != c0) ++j;
      if (j == n0c) c0Code[n0c++] = c0;
    }
    nC0 = n0c;
  }
  for (int i = t; i < ME1 * Q * P; i += NT) {
    int el = i / (Q * P), r = i % (Q * P);
    int e1 = min(E1lo + el, pb.ne[1] - 1);
    size_t o = (size_t)e1 * Q * P + r;
    (&tX1[0][0][0][0])[i] = (CT)pb.ax[1].B[o];
    (&tX1[1][0][0][0])[i] = (CT)pb.ax[1].dB[o];
    (&tB1d[0][0][0])[i] = pb.ax[1].B[o];
  }
  for (int i = t; i < ME1 * Q; i += NT) {
    int e1 = min(E1lo + i / Q, pb.ne[1] - 1);
    (&tW1[0][0])[i] = pb.ax[1].wq[(size_t)e1 * Q + i % Q];
  }
  __syncthreads();
  const bool owner = t < NOWN;
  int i1l = 0, o1 = 0;
  if (owner) { o1 = t % W7 - p; i1l = t / W7; }
  const int i1 = I1 + i1l, j1 = i1 + o1;
  const bool live = owner && i1 < n1 && j1 >= 0 && j1 < n1;
  CT acc[P][W7];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int k = 0; k < W7; ++k) acc[a][k] = 0;

  for (int e0 = 0; e0 < pb.ne[0]; ++e0) {
    for (int i = t; i < Q * P; i += NT) {
      size_t o = (size_t)e0 * Q * P + i;
      (&tX0[0][0][0])[i] = (CT)pb.ax[0].B[o];
      (&tX0[1][0][0])[i] = (CT)pb.ax[0].dB[o];
      (&tB0d[0][0])[i] = pb.ax[0].B[o];
    }
    if (t < Q) tW0[t] = pb.ax[0].wq[(size_t)e0 * Q + t];
    for (int i = t; i < P * NI1; i += NT) {
      int k1 = i % NI1, a0 = i / NI1;
      int64_t A = (e0 + a0) + (int64_t)n0 * (E1lo + k1);
      double v = U[A];
      if (TABLE && pb.rational) v *= pb.wts[A];
      sU[a0][k1] = v;
    }
    __syncthreads();
    for (int q0 = 0; q0 < Q; ++q0) {
      for (int i = t; i < NI1; i += NT) {
        double s = 0;
#pragma unroll
        for (int a0 = 0; a0 < P; ++a0) s += tB0d[q0][a0] * sU[a0][i];
        V0[i] = s;
      }
      __syncthreads();
      for (int g1 = t; g1 < G1; g1 += NT) {
        int el = g1 / Q, q1 = g1 % Q;
        double ut = 0;
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) ut += tB1d[el][q1][a1] * V0[el + a1];
        int64_t e = e0 + (int64_t)pb.ne[0] * (E1lo + el);
        double W = tW0[q0] * tW1[el][q1];
        double kap = (!TABLE && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
        double cv[10];
        rg_coefs<2, TABLE>(pb, e, q0 + Q * q1, Q * Q, W, kap, ut, cv);
#pragma unroll
        for (int k = 0; k < NCS; ++k) cs[k][g1] = (CT)cv[k];
      }
      __syncthreads();
      for (int i = t; i < nC0 * B1 * W7; i += NT) {
        int oo = i % W7, il = (i / W7) % B1, c = i / (W7 * B1);
        int ii1 = I1 + il, jj1 = ii1 + oo - p;
        CT s = 0;
        if (ii1 < n1 && jj1 >= 0 && jj1 < n1) {
          int elo = max(max(ii1, jj1) - p, E1lo), ehi = min(min(ii1, jj1), E1hi);
          for (int ti = 0; ti < nterms; ++ti) {
            const Term &T = terms[ti];
            if (((T.x[0] << 1) | T.y[0]) != c0Code[c]) continue;
            const int sidx = stream_of<TABLE, 2>(T.coef);
            for (int e1 = elo; e1 <= ehi; ++e1) {
              const int el = e1 - E1lo, a1 = ii1 - e1, b1 = jj1 - e1;
#pragma unroll
              for (int q1 = 0; q1 < Q; ++q1)
                s += cs[sidx][el * Q + q1] * tX1[T.x[1]][el][q1][a1] * tX1[T.y[1]][el][q1][b1];
            }
          }
        }
        T1[c][il][oo] = s;
      }
      __syncthreads();
      if (live) {
        for (int c = 0; c < nC0; ++c) {
          const int x0 = c0Code[c] >> 1, y0 = c0Code[c] & 1;
          const CT v = T1[c][i1l][o1 + p];
#pragma unroll
          for (int a0 = 0; a0 < P; ++a0) {
            const CT xa = tX0[x0][q0][a0] * v;
#pragma unroll
            for (int b0 = 0; b0 < P; ++b0) acc[a0][b0 - a0 + p] += xa * tX0[y0][q0][b0];
          }
        }
      }
      __syncthreads();
    }
    if (live) {
      const int last = (e0 == pb.ne[0] - 1) ? p : 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        if (a0 > last) break;
        const int i0 = e0 + a0;
        const bool rowDir = is_dirichlet_idx(pb, i0, i1, 0);
        const int64_t A = i0 + (int64_t)n0 * i1;
        const int64_t base = csr_slot(pb, i0, i1, 0, max(0, i0 - p), j1, 0);
        const double wA = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
#pragma unroll
        for (int k = 0; k < W7; ++k) {
          const int j0 = i0 + k - p;
          if (j0 < 0 || j0 >= n0) continue;
          double v;
          if (rowDir) v = (j0 == i0 && j1 == i1) ? 1.0 : 0.0;
          else if (is_dirichlet_idx(pb, j0, j1, 0)) v = 0.0;
          else {
            v = (double)acc[a0][k];
            if (TABLE && pb.rational) v *= wA * pb.wts[j0 + (int64_t)n0 * j1];
          }
          store_val(vals, base + (j0 - max(0, i0 - p)), v);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < P - 1; ++a)
#pragma unroll
      for (int k = 0; k < W7; ++k) acc[a][k] = acc[a + 1][k];
#pragma unroll
    for (int k = 0; k < W7; ++k) acc[P - 1][k] = 0;
    __syncthreads();
  }
}

}  // namespace rgk
}  // namespace iga
