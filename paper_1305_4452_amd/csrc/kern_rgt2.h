// Tiled 2D row-gather Jacobian for the analytic metric (identity geometry, no weights, kappa one or
// element-wise, every interior knot simple).  Shared by the single-problem and batched launchers.
//
// A workgroup owns a tile of T0 x B1 rows (i0 along axis 0, i1 along axis 1).  With
// c = kappa_e W and m = -lambda W e^u at the Gauss points (the Jacobian of the weak form, Sec. 3),
//   J[i][j] = sum_e kappa_e (A0_e M1_e + M0_e A1_e)[i][j]  +  sum_g m(g) N_i(g) N_j(g),
// where A_e / M_e are the 1D element stiffness / mass matrices; the first part is a sum of products
// of 1D element matrices (the global 1D band matrices when kappa = 1) and only the reaction part
// is contracted over Gauss points, by sum factorisation:
//   a. u at the tile's Gauss points (two 1D contractions of the coefficients), m into LDS;
//   b. level 1 (axis 1): Sm[i1, o1][g0] = sum_{g1} m(g0, g1) N_i1(g1) N_j1(g1)   (one wave per i1,
//      one lane per g0: the axis-1 basis values are wave-uniform);
//   c. level 2 (axis 0): J[(i0, i1)][(j0, j1)] += sum_{g0} Sm[i1, o1][g0] N_i0(g0) N_j0(g0) plus the
//      stiffness, one wave per row i0 and one lane per (i1, o1) pair; each lane stores its run of
//      2p + 1 consecutive CSR values (the lanes of one i1 together cover the whole row).
// Dirichlet rows become identity rows and Dirichlet columns zero, as in every assembly path.
#pragma once

#include "iga_impl.h"

namespace iga {
namespace rgt {

constexpr int kThreads = 256;

// Tile shape per P = p + 1: B1 * (2p + 1) <= 64 (one lane per pair) and (T0 + p) * Q <= 64 (one
// lane per Gauss point along axis 0).  V = 0: the largest such tiles; V = 1: tiles of about half the
// rows per axis (less idle work on small meshes; the batched solver picks per degree and size class
// by timing both).
template <int P, int VS = 0>
struct Shape2;
template <>
struct Shape2<2, 0> { static constexpr int B1 = 21, T0 = 24; };
template <>
struct Shape2<3, 0> { static constexpr int B1 = 12, T0 = 19; };
template <>
struct Shape2<4, 0> { static constexpr int B1 = 9, T0 = 12; };
template <>
struct Shape2<5, 0> { static constexpr int B1 = 7, T0 = 8; };
template <>
struct Shape2<2, 1> { static constexpr int B1 = 10, T0 = 12; };
template <>
struct Shape2<3, 1> { static constexpr int B1 = 6, T0 = 10; };
template <>
struct Shape2<4, 1> { static constexpr int B1 = 5, T0 = 6; };
template <>
struct Shape2<5, 1> { static constexpr int B1 = 4, T0 = 4; };

constexpr size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }

template <int P, typename CT, typename OT, int VS = 0>
struct Lds2 {
  static constexpr int p = P - 1, Q = P, W = 2 * p + 1;
  static constexpr int B1 = Shape2<P, VS>::B1, T0 = Shape2<P, VS>::T0;
  static constexpr int NPAIR = B1 * W;
  static constexpr int G0M = (T0 + p) * Q, G1M = (B1 + p) * Q;
  static constexpr int SP = G0M + 1;   // odd pitch of Sm rows (lanes = pairs read one column)
  static constexpr int NI0M = T0 + 2 * p, NI1M = B1 + 2 * p;
  // region A: m at the Gauss points
  static constexpr size_t bytes_a = align16((size_t)G1M * G0M * sizeof(CT));
  static constexpr size_t bytes_s = align16((size_t)NPAIR * SP * sizeof(CT));
  static constexpr size_t bytes_uv = align16((size_t)(NI0M * NI1M + NI1M * G0M) * sizeof(double));
  // region B: coefficients and their axis-0 contraction (phase a), then Sm
  static constexpr size_t bytes_b = bytes_s > bytes_uv ? bytes_s : bytes_uv;
  static constexpr size_t bytes_k = align16((size_t)(T0 + p) * (B1 + p) * sizeof(double));
  static constexpr size_t total = bytes_a + bytes_b + bytes_k;
  static_assert(NPAIR <= 64, "one lane per (i1, o1) pair");
};

// number of tiles of one problem
__host__ __device__ inline int rgt2_tiles_0(int n0, int T0) { return (n0 + T0 - 1) / T0; }

template <int P, typename CT, typename OT, int VS = 0>
__device__ inline void rgt2_body(const DevProblem &pb, const int tile, const double *__restrict__ U,
                                 OT *__restrict__ vals, char *__restrict__ lds) {
  using L = Lds2<P, CT, OT, VS>;
  constexpr int p = L::p, Q = L::Q, W = L::W, B1 = L::B1, T0 = L::T0;
  constexpr int NW = kThreads / 64;
  const int n0 = pb.n[0], n1 = pb.n[1], ne0 = pb.ne[0], ne1 = pb.ne[1];
  const int nt0 = rgt2_tiles_0(n0, T0);
  const int I0 = (tile % nt0) * T0, I1 = (tile / nt0) * B1;
  const int E0lo = max(0, I0 - p), E0hi = min(ne0 - 1, I0 + T0 - 1);
  const int E1lo = max(0, I1 - p), E1hi = min(ne1 - 1, I1 + B1 - 1);
  const int NE0 = E0hi - E0lo + 1, NE1 = E1hi - E1lo + 1;
  const int G0 = NE0 * Q, G1 = NE1 * Q, NI0 = NE0 + p, NI1 = NE1 + p;
  CT *mQ = (CT *)lds;                                   // [G1M][G0M]
  CT *Sm = (CT *)(lds + L::bytes_a);                    // [NPAIR][SP]
  double *sU = (double *)(lds + L::bytes_a);            // [NI1M][NI0M], phase a only
  double *V = sU + L::NI0M * L::NI1M;                   // [NI1M][G0M], phase a only
  double *kt = (double *)(lds + L::bytes_a + L::bytes_b);   // [NE0][NE1] element kappa
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const double *__restrict__ B0 = pb.ax[0].B;
  const double *__restrict__ B1t = pb.ax[1].B;
  const bool kel = pb.kappa_mode == IGA_KAPPA_ELEMENT;

  // ---- a. u and m at the tile's Gauss points -------------------------------------------
  for (int i = t; i < NI0 * NI1; i += kThreads) {
    const int k0 = i % NI0, k1 = i / NI0;
    sU[k1 * L::NI0M + k0] = U[(E0lo + k0) + (int64_t)n0 * (E1lo + k1)];
  }
  if (kel)
    for (int i = t; i < NE0 * NE1; i += kThreads) {
      const int el0 = i % NE0, el1 = i / NE0;
      kt[el0 * NE1 + el1] = pb.kel[(E0lo + el0) + (int64_t)ne0 * (E1lo + el1)];
    }
  __syncthreads();
  // one lane per axis-0 Gauss point (its basis values in registers), waves walk axis 1 (the
  // axis-1 basis values and weights are wave-uniform)
  for (int gb = 0; gb < G0; gb += 64) {
    const int g0 = gb + lane;
    const bool ok = g0 < G0;
    const int el0 = ok ? g0 / Q : 0;
    double b0[P];
    const double *Bq0 = B0 + ((size_t)(E0lo + el0) * Q + (ok ? g0 % Q : 0)) * P;
#pragma unroll
    for (int a0 = 0; a0 < P; ++a0) b0[a0] = Bq0[a0];
    for (int k1 = wave; k1 < NI1; k1 += NW) {
      double s = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) s += b0[a0] * sU[k1 * L::NI0M + el0 + a0];
      if (ok) V[k1 * L::G0M + g0] = s;
    }
  }
  __syncthreads();
  {
    const double lam = pb.lambda;
    const double *wq0 = pb.ax[0].wq + (size_t)E0lo * Q, *wq1 = pb.ax[1].wq + (size_t)E1lo * Q;
    for (int gb = 0; gb < G0; gb += 64) {
      const int g0 = gb + lane;
      const bool ok = g0 < G0;
      const double w0 = ok ? -lam * wq0[g0] : 0.0;
      for (int g1 = wave; g1 < G1; g1 += NW) {
        const int el1 = g1 / Q;
        const double *Bq = B1t + ((size_t)E1lo * Q + g1) * P;
        double u = 0;
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) u += Bq[a1] * V[(el1 + a1) * L::G0M + (ok ? g0 : 0)];
        if (ok) mQ[g1 * L::G0M + g0] = (CT)(w0 * wq1[g1] * exp(u));
      }
    }
  }
  __syncthreads();

  // ---- b. level 1: contract axis 1 (wave = i1, lane = g0) ------------------------------
  for (int i1l = wave; i1l < B1; i1l += NW) {
    const int i1 = I1 + i1l;
    if (i1 >= n1) break;
    for (int gb = 0; gb < G0; gb += 64) {
      const int g0 = gb + lane;
      const bool ok = g0 < G0;
      CT sm[W];
#pragma unroll
      for (int o = 0; o < W; ++o) sm[o] = 0;
#pragma unroll
      for (int a1 = 0; a1 <= p; ++a1) {
        const int e1 = i1 - a1;
        if (e1 < 0 || e1 >= ne1) continue;
        const int el1 = e1 - E1lo;
#pragma unroll
        for (int q1 = 0; q1 < Q; ++q1) {
          const double *Bq = B1t + ((size_t)e1 * Q + q1) * P;
          const CT m = ok ? mQ[(el1 * Q + q1) * L::G0M + g0] : CT(0);
          const CT mb = m * (CT)Bq[a1];
#pragma unroll
          for (int b1 = 0; b1 <= p; ++b1) sm[b1 - a1 + p] += mb * (CT)Bq[b1];
        }
      }
      if (ok)
#pragma unroll
        for (int o = 0; o < W; ++o) Sm[(i1l * W + o) * L::SP + g0] = sm[o];
    }
  }
  __syncthreads();

  // ---- c. level 2: contract axis 0 (wave = i0, lane = (i1, o1)) plus the stiffness -----
  {
    const int pair = lane;
    const int i1l = pair / W, o1 = pair % W - p;
    const int i1 = I1 + i1l, j1 = i1 + o1;
    const bool live = pair < L::NPAIR && i1 < n1 && j1 >= 0 && j1 < n1;
    // axis-1 factors of the stiffness, fixed per lane
    CT sM1 = 0, sA1 = 0;
    CT M1s[P], A1s[P];
#pragma unroll
    for (int a1 = 0; a1 < P; ++a1) { M1s[a1] = 0; A1s[a1] = 0; }
    if (live) {
      if (!kel) {
        sM1 = (CT)pb.sepM[1][(size_t)i1 * W + (o1 + p)];
        sA1 = (CT)pb.sepA[1][(size_t)i1 * W + (o1 + p)];
      } else {
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) {
          const int e1 = i1 - a1, b1 = j1 - e1;
          if (e1 >= 0 && e1 < ne1 && b1 >= 0 && b1 <= p) {
            M1s[a1] = (CT)pb.elM[1][((size_t)e1 * P + a1) * P + b1];
            A1s[a1] = (CT)pb.elA[1][((size_t)e1 * P + a1) * P + b1];
          }
        }
      }
    }
    const int l1 = max(0, i1 - p), w1 = min(n1 - 1, i1 + p) - l1 + 1;
    // CSR rows (I0 .. I0 + T0 - 1, i1) are consecutive: row (i0, i1) starts w1 * (sum of the
    // axis-0 widths of rows I0 .. i0 - 1) after row (I0, i1)
    const int64_t rp0 = live ? pb.row_ptr[I0 + (int64_t)n0 * i1] : 0;
    const unsigned dm = pb.dmask;
    const bool dirI1 = (((dm >> 2) & 1u) && i1 == 0) || (((dm >> 3) & 1u) && i1 == n1 - 1);
    const bool dirJ1 = (((dm >> 2) & 1u) && j1 == 0) || (((dm >> 3) & 1u) && j1 == n1 - 1);
    for (int i0l = wave; i0l < T0; i0l += NW) {
      const int i0 = I0 + i0l;
      if (i0 >= n0) break;
      CT out[W];
      if (!kel) {
        const double *M0r = pb.sepM[0] + (size_t)i0 * W, *A0r = pb.sepA[0] + (size_t)i0 * W;
#pragma unroll
        for (int o = 0; o < W; ++o) out[o] = (CT)A0r[o] * sM1 + (CT)M0r[o] * sA1;
      } else {
#pragma unroll
        for (int o = 0; o < W; ++o) out[o] = 0;
      }
#pragma unroll
      for (int a0 = 0; a0 <= p; ++a0) {
        const int e0 = i0 - a0;
        if (e0 < 0 || e0 >= ne0) continue;
        const int el0 = e0 - E0lo;
        if (kel) {
          CT kM = 0, kA = 0;
#pragma unroll
          for (int a1 = 0; a1 < P; ++a1) {
            const int el1 = min(max(i1 - a1 - E1lo, 0), NE1 - 1);
            const CT k = (CT)kt[el0 * NE1 + el1];
            kM += k * M1s[a1];
            kA += k * A1s[a1];
          }
          const double *eM = pb.elM[0] + ((size_t)e0 * P + a0) * P, *eA = pb.elA[0] + ((size_t)e0 * P + a0) * P;
#pragma unroll
          for (int b0 = 0; b0 <= p; ++b0) out[b0 - a0 + p] += (CT)eA[b0] * kM + (CT)eM[b0] * kA;
        }
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          const double *Bq = B0 + ((size_t)e0 * Q + q0) * P;
          const CT s = live ? Sm[pair * L::SP + el0 * Q + q0] : CT(0);
          const CT xb = s * (CT)Bq[a0];
#pragma unroll
          for (int b0 = 0; b0 <= p; ++b0) out[b0 - a0 + p] += xb * (CT)Bq[b0];
        }
      }
      int pre = 0;   // wave-uniform
      for (int i = I0; i < i0; ++i) pre += min(n0 - 1, i + p) - max(0, i - p) + 1;
      if (live) {
        const bool dir0i = ((dm & 1u) && i0 == 0) || (((dm >> 1) & 1u) && i0 == n0 - 1);
        const bool rowDir = dir0i || dirI1;
        const int l0 = max(0, i0 - p), w0 = min(n0 - 1, i0 + p) - l0 + 1;
        // CSR row (i0, i1): columns (j0, j1) with j1 - l1 major, j0 - l0 minor
        OT *srow = vals + rp0 + (int64_t)w1 * pre + (j1 - l1) * w0 - l0;
#pragma unroll
        for (int o = 0; o < W; ++o) {
          const int j0 = i0 + o - p;
          if (j0 < 0 || j0 >= n0) continue;
          const bool dir0j = ((dm & 1u) && j0 == 0) || (((dm >> 1) & 1u) && j0 == n0 - 1);
          double v = (double)out[o];
          if (rowDir) v = (o == p && o1 == 0) ? 1.0 : 0.0;
          else if (dir0j || dirJ1) v = 0.0;
          srow[j0] = (OT)v;
        }
      }
    }
  }
}

}  // namespace rgt
}  // namespace iga
