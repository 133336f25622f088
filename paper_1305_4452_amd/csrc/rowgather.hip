// Row-gather Jacobian assembly.
//
// The paper assembles element matrices and adds them into the global matrix (Algorithm 3 and
// "matrices are assembled in a similar fashion", Sec. 2.7), which on a GPU means up to
// (p+1)^d colliding read-modify-writes per CSR value.  Here a workgroup instead owns a block of
// row *pencils* (all rows i0 for a B1 x B2 block of (i1, i2)) and computes every value of
// those rows itself, so each CSR value is written exactly once, with no atomics and in a fixed
// summation order (bitwise reproducible).
//
// For a tensor-product basis every Jacobian entry is a sum over quadrature points of
// coefficient(q) * prod_d X_d(i_d, q_d) Y_d(j_d, q_d), where the 1D factors depend only on the
// global quadrature coordinate along axis d.  The sum over elements is therefore folded into
// the sum-factorised contraction:
//   level 1 (axis 2): T1[g1][i2][o2] = sum over the quadrature points g2 in supp(i2) n supp(i2+o2)
//   level 2 (axis 1): T2[i1][o1][i2][o2] = sum over g1 in supp(i1) n supp(i1+o1)
//   level 3 (axis 0): streamed element by element along axis 0; the rows i0 = e0..e0+p that
//                     element column e0 touches live in a register window per thread, and
//                     row e0 is complete (and written) once column e0 has been processed.
// Requires every interior knot to be simple (element e's first function is e).
#include <type_traits>

#include "iga_impl.h"
#include "kern_rg.h"

namespace iga {
namespace {
using namespace rgk;

// ------------------------------------------------------------------------------------------
// 3D
// ------------------------------------------------------------------------------------------
template <int P, bool TABLE, int B1, int B2, typename CT, typename OT>
__global__ void __launch_bounds__(rg_threads(B1 * B2 * (2 * P - 1) * (2 * P - 1)))
k_rowgather3(DevProblem pb, const double *__restrict__ U, OT *__restrict__ vals) {
  constexpr int p = P - 1, Q = P, W7 = 2 * p + 1;
  constexpr int NOWN = B1 * B2 * W7 * W7;
  constexpr int NT = rg_threads(NOWN);
  constexpr int ME1 = B1 + p, ME2 = B2 + p;           // elements per block along axes 1, 2
  constexpr int MG1 = ME1 * Q, MG2 = ME2 * Q;          // block quadrature points
  constexpr int MI1 = ME1 + p, MI2 = ME2 + p;          // coefficient indices
  constexpr int NCS = TABLE ? 10 : 2;
  constexpr int NCOMBO = TABLE ? 9 : 3;                // (c0, c1) combinations with terms
  constexpr int NC0 = TABLE ? 4 : 2;                   // active axis-0 combinations

  __shared__ CT tX1[2][ME1][Q][P], tX2[2][ME2][Q][P];  // [val/der][elem][q][a]
  __shared__ double tW1[ME1][Q], tW2[ME2][Q];
  // FP64 basis values for the interpolation of u: with FP64 contractions they are the value tables
  // themselves, so the copies (and their LDS) exist only for FP32 contractions
  constexpr bool F64 = std::is_same<CT, double>::value;
  __shared__ double tB1c[F64 ? 1 : ME1][Q][P], tB2c[F64 ? 1 : ME2][Q][P];
  __shared__ CT tX0[2][Q][P];
  __shared__ double tB0c[F64 ? 1 : Q][P], tW0[Q];
  const auto tB1d = [&](int el, int q, int a) -> double { return F64 ? (double)tX1[0][el][q][a] : tB1c[el][q][a]; };
  const auto tB2d = [&](int el, int q, int a) -> double { return F64 ? (double)tX2[0][el][q][a] : tB2c[el][q][a]; };
  const auto tB0d = [&](int q, int a) -> double { return F64 ? (double)tX0[0][q][a] : tB0c[q][a]; };
  __shared__ double sU[P][MI2][MI1];
  __shared__ double V0[MI2][MI1];
  __shared__ double V1[MI2][MG1];
  __shared__ CT cs[NCS][MG2][MG1];
  __shared__ CT T1[NCOMBO][MG1][B2][W7];
  __shared__ CT T2[NC0][B1][W7][B2][W7];
  __shared__ int comboCode[16], comboTerm[16][4], comboNT[16], nCombo;
  __shared__ int c0Code[4], nC0;

  const int t = threadIdx.x;
  const int nb1 = (pb.n[1] + B1 - 1) / B1;
  const int I1 = (blockIdx.x % nb1) * B1, I2 = (blockIdx.x / nb1) * B2;
  const int E1lo = max(0, I1 - p), E1hi = min(pb.ne[1] - 1, I1 + B1 - 1);
  const int E2lo = max(0, I2 - p), E2hi = min(pb.ne[2] - 1, I2 + B2 - 1);
  const int NE1 = E1hi - E1lo + 1, NE2 = E2hi - E2lo + 1;
  const int G1 = NE1 * Q, G2 = NE2 * Q, NI1 = NE1 + p, NI2 = NE2 + p;
  const int n0 = pb.n[0], n1 = pb.n[1], n2 = pb.n[2];

  // ---- combination lists (compile-time term table, built once per block) ----
  if (t == 0) {
    const Term *terms = TABLE ? r_terms3_full : r_terms3_diag;
    const int nterms = TABLE ? 16 : 4;
    int nc = 0, n0c = 0;
    for (int ti = 0; ti < nterms; ++ti) {
      int code = (terms[ti].x[0] << 3) | (terms[ti].y[0] << 2) | (terms[ti].x[1] << 1) | terms[ti].y[1];
      int k = 0;
      while (k < nc && comboCode[k] != code) ++k;
      if (k == nc) { comboCode[nc] = code; comboNT[nc] = 0; ++nc; }
      comboTerm[k][comboNT[k]++] = ti;
      int c0 = code >> 2, j = 0;
      while (j < n0c && c0Code[j] != c0) ++j;
      if (j == n0c) c0Code[n0c++] = c0;
    }
    nCombo = nc;
    nC0 = n0c;
  }
  // ---- per-block axis 1 and 2 tables ----
  for (int i = t; i < ME1 * Q * P; i += NT) {
    int el = i / (Q * P), r = i % (Q * P);
    int e1 = min(E1lo + el, pb.ne[1] - 1);
    size_t o = (size_t)e1 * Q * P + r;
    (&tX1[0][0][0][0])[i] = (CT)pb.ax[1].B[o];
    (&tX1[1][0][0][0])[i] = (CT)pb.ax[1].dB[o];
    if constexpr (!F64) (&tB1c[0][0][0])[i] = pb.ax[1].B[o];
  }
  for (int i = t; i < ME2 * Q * P; i += NT) {
    int el = i / (Q * P), r = i % (Q * P);
    int e2 = min(E2lo + el, pb.ne[2] - 1);
    size_t o = (size_t)e2 * Q * P + r;
    (&tX2[0][0][0][0])[i] = (CT)pb.ax[2].B[o];
    (&tX2[1][0][0][0])[i] = (CT)pb.ax[2].dB[o];
    if constexpr (!F64) (&tB2c[0][0][0])[i] = pb.ax[2].B[o];
  }
  for (int i = t; i < ME1 * Q; i += NT) {
    int e1 = min(E1lo + i / Q, pb.ne[1] - 1);
    (&tW1[0][0])[i] = pb.ax[1].wq[(size_t)e1 * Q + i % Q];
  }
  for (int i = t; i < ME2 * Q; i += NT) {
    int e2 = min(E2lo + i / Q, pb.ne[2] - 1);
    (&tW2[0][0])[i] = pb.ax[2].wq[(size_t)e2 * Q + i % Q];
  }
  __syncthreads();

  // ---- ownership for level 3: (i1l, i2l, o1, o2) ----
  const bool owner = t < NOWN;
  int i1l = 0, i2l = 0, o1 = 0, o2 = 0;
  if (owner) {
    o2 = t % W7 - p;
    o1 = (t / W7) % W7 - p;
    i2l = (t / (W7 * W7)) % B2;
    i1l = t / (W7 * W7 * B2);
  }
  const int i1 = I1 + i1l, i2 = I2 + i2l, j1 = i1 + o1, j2 = i2 + o2;
  const bool live = owner && i1 < n1 && i2 < n2 && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2;
  CT acc[P][W7];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int k = 0; k < W7; ++k) acc[a][k] = 0;

  for (int e0 = 0; e0 < pb.ne[0]; ++e0) {
    // axis 0 tables for this element column
    for (int i = t; i < Q * P; i += NT) {
      size_t o = (size_t)e0 * Q * P + i;
      (&tX0[0][0][0])[i] = (CT)pb.ax[0].B[o];
      (&tX0[1][0][0])[i] = (CT)pb.ax[0].dB[o];
      if constexpr (!F64) (&tB0c[0][0])[i] = pb.ax[0].B[o];
    }
    if (t < Q) tW0[t] = pb.ax[0].wq[(size_t)e0 * Q + t];
    // coefficient block U[e0 + a0, E1lo + k1, E2lo + k2] (weighted for rational bases)
    for (int i = t; i < P * NI2 * NI1; i += NT) {
      int k1 = i % NI1, k2 = (i / NI1) % NI2, a0 = i / (NI1 * NI2);
      int64_t A = (e0 + a0) + (int64_t)n0 * ((E1lo + k1) + (int64_t)n1 * (E2lo + k2));
      double v = U[A];
      if (TABLE && pb.rational) v *= pb.wts[A];
      sU[a0][k2][k1] = v;
    }
    __syncthreads();
    for (int q0 = 0; q0 < Q; ++q0) {
      // ---- interpolate u at (q0, g1, g2) by sum factorisation over the block ----
      for (int i = t; i < NI2 * NI1; i += NT) {
        int k1 = i % NI1, k2 = i / NI1;
        double s = 0;
#pragma unroll
        for (int a0 = 0; a0 < P; ++a0) s += tB0d(q0, a0) * sU[a0][k2][k1];
        V0[k2][k1] = s;
      }
      __syncthreads();
      for (int i = t; i < NI2 * G1; i += NT) {
        int g1 = i % G1, k2 = i / G1, el = g1 / Q, q1 = g1 % Q;
        double s = 0;
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) s += tB1d(el, q1, a1) * V0[k2][el + a1];
        V1[k2][g1] = s;
      }
      __syncthreads();
      for (int i = t; i < G2 * G1; i += NT) {
        int g1 = i % G1, g2 = i / G1, el1 = g1 / Q, q1 = g1 % Q, el2 = g2 / Q, q2 = g2 % Q;
        double ut = 0;
#pragma unroll
        for (int a2 = 0; a2 < P; ++a2) ut += tB2d(el2, q2, a2) * V1[el2 + a2][g1];
        int64_t e = e0 + (int64_t)pb.ne[0] * ((E1lo + el1) + (int64_t)pb.ne[1] * (E2lo + el2));
        double W = tW0[q0] * tW1[el1][q1] * tW2[el2][q2];
        double kap = (!TABLE && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
        double cv[10];
        rg_coefs<3, TABLE>(pb, e, q0 + Q * (q1 + Q * q2), Q * Q * Q, W, kap, ut, cv);
#pragma unroll
        for (int k = 0; k < NCS; ++k) cs[k][g2][g1] = (CT)cv[k];
      }
      __syncthreads();
      // ---- level 1: contract axis 2 for every (c0,c1) combination ----
      {
        const Term *terms = TABLE ? r_terms3_full : r_terms3_diag;
        const int nout = nCombo * G1 * B2 * W7;
        for (int i = t; i < nout; i += NT) {
          int oo = i % W7, il = (i / W7) % B2, g1 = (i / (W7 * B2)) % G1, k = i / (W7 * B2 * G1);
          int ii2 = I2 + il, jj2 = ii2 + oo - p;
          CT s = 0;
          if (ii2 < n2 && jj2 >= 0 && jj2 < n2) {
            int elo = max(max(ii2, jj2) - p, E2lo), ehi = min(min(ii2, jj2), E2hi);
            for (int m = 0; m < comboNT[k]; ++m) {
              const Term &T = terms[comboTerm[k][m]];
              const int sidx = stream_of<TABLE, 3>(T.coef);
              for (int e2 = elo; e2 <= ehi; ++e2) {
                const int el = e2 - E2lo, a2 = ii2 - e2, b2 = jj2 - e2;
#pragma unroll
                for (int q2 = 0; q2 < Q; ++q2)
                  s += cs[sidx][el * Q + q2][g1] * tX2[T.x[2]][el][q2][a2] * tX2[T.y[2]][el][q2][b2];
              }
            }
          }
          T1[k][g1][il][oo] = s;
        }
      }
      __syncthreads();
      // ---- level 2: contract axis 1 ----
      {
        const int nout = nC0 * B1 * W7 * B2 * W7;
        for (int i = t; i < nout; i += NT) {
          int oo2 = i % W7, il2 = (i / W7) % B2, oo1 = (i / (W7 * B2)) % W7, il1 = (i / (W7 * B2 * W7)) % B1;
          int c = i / (W7 * B2 * W7 * B1);
          int ii1 = I1 + il1, jj1 = ii1 + oo1 - p;
          CT s = 0;
          if (ii1 < n1 && jj1 >= 0 && jj1 < n1) {
            int elo = max(max(ii1, jj1) - p, E1lo), ehi = min(min(ii1, jj1), E1hi);
            for (int k = 0; k < nCombo; ++k) {
              int code = comboCode[k];
              if ((code >> 2) != c0Code[c]) continue;
              int x1 = (code >> 1) & 1, y1 = code & 1;
              for (int e1 = elo; e1 <= ehi; ++e1) {
                const int el = e1 - E1lo, a1 = ii1 - e1, b1 = jj1 - e1;
#pragma unroll
                for (int q1 = 0; q1 < Q; ++q1)
                  s += tX1[x1][el][q1][a1] * tX1[y1][el][q1][b1] * T1[k][el * Q + q1][il2][oo2];
              }
            }
          }
          T2[c][il1][oo1][il2][oo2] = s;
        }
      }
      __syncthreads();
      // ---- level 3: this quadrature point of axis 0 into the register window ----
      if (live) {
        for (int c = 0; c < nC0; ++c) {
          const int x0 = c0Code[c] >> 1, y0 = c0Code[c] & 1;
          const CT v = T2[c][i1l][o1 + p][i2l][o2 + p];
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
    // ---- emit the completed row(s) ----
    if (live) {
      const int last = (e0 == pb.ne[0] - 1) ? p : 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        if (a0 > last) break;
        const int i0 = e0 + a0;
        const bool rowDir = is_dirichlet_idx(pb, i0, i1, i2);
        const int64_t A = i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2);
        const int64_t base = csr_slot(pb, i0, i1, i2, max(0, i0 - p), j1, j2);
        const double wA = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
#pragma unroll
        for (int k = 0; k < W7; ++k) {
          const int j0 = i0 + k - p;
          if (j0 < 0 || j0 >= n0) continue;
          double v;
          if (rowDir) v = (j0 == i0 && j1 == i1 && j2 == i2) ? 1.0 : 0.0;
          else if (is_dirichlet_idx(pb, j0, j1, j2)) v = 0.0;
          else {
            v = (double)acc[a0][k];
            if (TABLE && pb.rational) v *= wA * pb.wts[j0 + (int64_t)n0 * (j1 + (int64_t)n1 * j2)];
          }
          store_val(vals, base + (j0 - max(0, i0 - p)), v);
        }
      }
    }
    // shift the window: row e0+1 becomes slot 0
#pragma unroll
    for (int a = 0; a < P - 1; ++a)
#pragma unroll
      for (int k = 0; k < W7; ++k) acc[a][k] = acc[a + 1][k];
#pragma unroll
    for (int k = 0; k < W7; ++k) acc[P - 1][k] = 0;
    __syncthreads();
  }
}

template <int P, bool TABLE, int B1, typename CT, typename OT>
__global__ void __launch_bounds__(rg_threads(B1 * (2 * P - 1)))
k_rowgather2(DevProblem pb, const double *__restrict__ U, OT *__restrict__ vals) {
  rowgather2_body<P, TABLE, B1, CT, OT>(pb, (int)blockIdx.x, U, vals);
}

template <int P, bool TABLE, int B1, int B2>
iga_status run3(const Handle &h, const double *U, void *vals, int prec) {
  constexpr int NT = rg_threads(B1 * B2 * (2 * P - 1) * (2 * P - 1));
  const int nb1 = (h.pb.n[1] + B1 - 1) / B1, nb2 = (h.pb.n[2] + B2 - 1) / B2;
  dim3 grid((unsigned)(nb1 * nb2)), block(NT);
  if (prec == IGA_FP32)
    hipLaunchKernelGGL((k_rowgather3<P, TABLE, B1, B2, float, float>), grid, block, 0, h.stream, h.pb, U,
                       (float *)vals);
  else
    hipLaunchKernelGGL((k_rowgather3<P, TABLE, B1, B2, double, double>), grid, block, 0, h.stream, h.pb, U,
                       (double *)vals);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P, bool TABLE, int B1>
iga_status run2(const Handle &h, const double *U, void *vals, int prec) {
  constexpr int NT = rg_threads(B1 * (2 * P - 1));
  dim3 grid((unsigned)((h.pb.n[1] + B1 - 1) / B1)), block(NT);
  if (prec == IGA_FP32)
    hipLaunchKernelGGL((k_rowgather2<P, TABLE, B1, float, float>), grid, block, 0, h.stream, h.pb, U, (float *)vals);
  else
    hipLaunchKernelGGL((k_rowgather2<P, TABLE, B1, double, double>), grid, block, 0, h.stream, h.pb, U,
                       (double *)vals);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// compiled pencil blocks: 3D (b1, b2) in {(1,1), (2,1), (2,2)}; 2D b1 in {1, 4, 8}
template <int P, bool T>
iga_status pick3(const Handle &h, const double *U, void *vals, int prec, int b1, int b2) {
  if (b1 == 1 && b2 == 1) return run3<P, T, 1, 1>(h, U, vals, prec);
  if (b1 == 2 && b2 == 1) return run3<P, T, 2, 1>(h, U, vals, prec);
  if constexpr (P <= 4) {
    if (b1 == 2 && b2 == 2) return run3<P, T, 2, 2>(h, U, vals, prec);
  }
  return fail(IGA_EUNSUPPORTED, "row-gather block shape not compiled");
}

template <int P, bool T>
iga_status pick2(const Handle &h, const double *U, void *vals, int prec, int b1) {
  if (b1 == 1) return run2<P, T, 1>(h, U, vals, prec);
  if (b1 == 4) return run2<P, T, 4>(h, U, vals, prec);
  if (b1 == 8) return run2<P, T, 8>(h, U, vals, prec);
  return fail(IGA_EUNSUPPORTED, "row-gather block shape not compiled");
}

}  // namespace

bool rowgather_supported(const Handle &h, int prec, int b1, int b2) {
  (void)prec;
  if (!h.pb.simple_knots || h.pb.periodic) return false;
  if (h.pb.dim == 3) {
    if (h.pb.P < 2 || h.pb.P > 5) return false;
    if (b1 == 1 && b2 == 1) return true;
    if (b1 == 2 && b2 == 1) return true;
    if (b1 == 2 && b2 == 2) return h.pb.P <= 4;
    return false;
  }
  if (h.pb.P < 2 || h.pb.P > 7) return false;
  return b1 == 1 || b1 == 4 || b1 == 8;
}

iga_status launch_jac_rowgather(Handle &h, const double *U, void *vals, int prec, int b1, int b2) {
  if (!rowgather_supported(h, prec, b1, b2)) return fail(IGA_EUNSUPPORTED, "row-gather configuration");
  const bool T = h.pb.table != 0;
  if (h.pb.dim == 3) {
    switch (h.pb.P) {
      case 2: return T ? pick3<2, true>(h, U, vals, prec, b1, b2) : pick3<2, false>(h, U, vals, prec, b1, b2);
      case 3: return T ? pick3<3, true>(h, U, vals, prec, b1, b2) : pick3<3, false>(h, U, vals, prec, b1, b2);
      case 4: return T ? pick3<4, true>(h, U, vals, prec, b1, b2) : pick3<4, false>(h, U, vals, prec, b1, b2);
      case 5: return T ? pick3<5, true>(h, U, vals, prec, b1, b2) : pick3<5, false>(h, U, vals, prec, b1, b2);
    }
  } else {
    switch (h.pb.P) {
      case 2: return T ? pick2<2, true>(h, U, vals, prec, b1) : pick2<2, false>(h, U, vals, prec, b1);
      case 3: return T ? pick2<3, true>(h, U, vals, prec, b1) : pick2<3, false>(h, U, vals, prec, b1);
      case 4: return T ? pick2<4, true>(h, U, vals, prec, b1) : pick2<4, false>(h, U, vals, prec, b1);
      case 5: return T ? pick2<5, true>(h, U, vals, prec, b1) : pick2<5, false>(h, U, vals, prec, b1);
      case 6: return T ? pick2<6, true>(h, U, vals, prec, b1) : pick2<6, false>(h, U, vals, prec, b1);
      case 7: return T ? pick2<7, true>(h, U, vals, prec, b1) : pick2<7, false>(h, U, vals, prec, b1);
    }
  }
  return fail(IGA_EUNSUPPORTED, "row-gather degree");
}

}  // namespace iga
