// Row-gather Jacobian for the separable case: identity geometry, no weights, kappa = 1.
//
// With x = xi and W = w0(g0) w1(g1) w2(g2) the stiffness part of eq:jacobian is the Kronecker
// sum A0 (x) M1 (x) M2 + M0 (x) A1 (x) M2 + M0 (x) M1 (x) A2 of 1D band matrices (built once at
// creation), so only the reaction term -lambda e^u N_A N_B needs a 3D contraction.  That term
// is contracted exactly like the general row-gather kernel (level 1 over the quadrature points
// of axis 2, level 2 over axis 1, axis 0 streamed element column by element column), but with
// fixed-size windows: the block's element window along axes 1 and 2 is always [I-p, I+B-1]
// (zero-padded outside the mesh), so every band contraction is a fixed-length, fully unrolled
// dot product over the (p+1)^2 quadrature points of one function's support, and each phase
// handles all p+1 quadrature points of axis 0 at once.
#include "iga_impl.h"

namespace iga {
namespace {

constexpr int rs_threads(int nown) { return ((nown + 63) / 64) * 64 < 256 ? 256 : ((nown + 63) / 64) * 64; }

template <typename CT>
__device__ inline CT exp_ct(double u);
template <>
__device__ inline double exp_ct<double>(double u) { return exp(u); }
template <>
__device__ inline float exp_ct<float>(double u) { return expf((float)u); }

template <int P, int B1, int B2, typename CT, typename OT>
__global__ void __launch_bounds__(rs_threads(B1 * (2 * P - 1) * B2 * (2 * P - 1)))
k_rgsep3(DevProblem pb, const double *__restrict__ U, OT *__restrict__ vals) {
  constexpr int p = P - 1, Q = P, W = 2 * p + 1, KM = P * Q;
  constexpr int ME1 = B1 + p, ME2 = B2 + p, G1 = ME1 * Q, G2 = ME2 * Q;
  constexpr int NI1 = ME1 + p, NI2 = ME2 + p;
  constexpr int R1 = B1 * W, R2 = B2 * W, NOWN = R1 * R2;
  constexpr int NT = rs_threads(NOWN);

  __shared__ double tB1[ME1][Q][P], tB2[ME2][Q][P], tw1[ME1][Q], tw2[ME2][Q];
  __shared__ CT phi1[B1][W][KM], phi2[B2][W][KM];
  __shared__ double tB0[Q][P], tw0[Q];
  __shared__ CT cB0[Q][P];
  __shared__ double sU[P][NI2][NI1];
  __shared__ double V0[Q][NI2][NI1];
  __shared__ double V1[Q][NI2][G1];
  __shared__ CT mq[Q][G2][G1];
  __shared__ CT T1[Q][R2][G1];
  __shared__ CT T2[Q][R1][R2];

  const int t = threadIdx.x;
  const int n0 = pb.n[0], n1 = pb.n[1], n2 = pb.n[2];
  const int ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nb1 = (n1 + B1 - 1) / B1;
  const int I1 = (blockIdx.x % nb1) * B1, I2 = (blockIdx.x / nb1) * B2;
  const int W1lo = I1 - p, W2lo = I2 - p;   // first window element (may be negative)

  // ---- window tables and band operators (once per block) ----
  for (int i = t; i < ME1 * Q * P; i += NT) {
    int el = i / (Q * P), r = i % (Q * P), e = W1lo + el;
    (&tB1[0][0][0])[i] = (e >= 0 && e < ne1) ? pb.ax[1].B[(size_t)e * Q * P + r] : 0.0;
  }
  for (int i = t; i < ME2 * Q * P; i += NT) {
    int el = i / (Q * P), r = i % (Q * P), e = W2lo + el;
    (&tB2[0][0][0])[i] = (e >= 0 && e < ne2) ? pb.ax[2].B[(size_t)e * Q * P + r] : 0.0;
  }
  for (int i = t; i < ME1 * Q; i += NT) {
    int e = W1lo + i / Q;
    (&tw1[0][0])[i] = (e >= 0 && e < ne1) ? pb.ax[1].wq[(size_t)e * Q + i % Q] : 0.0;
  }
  for (int i = t; i < ME2 * Q; i += NT) {
    int e = W2lo + i / Q;
    (&tw2[0][0])[i] = (e >= 0 && e < ne2) ? pb.ax[2].wq[(size_t)e * Q + i % Q] : 0.0;
  }
  __syncthreads();
  // phi_d[il][o][k] = B_i(g) B_j(g) over the support of i = I + il, g = element (i - p + k/Q), point k%Q
  for (int i = t; i < B1 * W * KM; i += NT) {
    int k = i % KM, o = (i / KM) % W, il = i / (KM * W);
    int ii = I1 + il, jj = ii + o - p, el = il + k / Q, q = k % Q, a = p - k / Q, b = jj - (W1lo + el);
    double v = 0.0;
    if (ii < n1 && jj >= 0 && jj < n1 && b >= 0 && b <= p) v = tB1[el][q][a] * tB1[el][q][b];
    (&phi1[0][0][0])[i] = (CT)v;
  }
  for (int i = t; i < B2 * W * KM; i += NT) {
    int k = i % KM, o = (i / KM) % W, il = i / (KM * W);
    int ii = I2 + il, jj = ii + o - p, el = il + k / Q, q = k % Q, a = p - k / Q, b = jj - (W2lo + el);
    double v = 0.0;
    if (ii < n2 && jj >= 0 && jj < n2 && b >= 0 && b <= p) v = tB2[el][q][a] * tB2[el][q][b];
    (&phi2[0][0][0])[i] = (CT)v;
  }

  // ---- owner of the register window: (il1, o1, il2, o2) ----
  const bool owner = t < NOWN;
  const int o2 = t % W, il2 = (t / W) % B2, o1 = (t / (W * B2)) % W, il1 = (t / (W * B2 * W)) % B1;
  const int r1 = il1 * W + o1, r2 = il2 * W + o2;
  const int i1 = I1 + il1, i2 = I2 + il2, j1 = i1 + o1 - p, j2 = i2 + o2 - p;
  const bool live = owner && i1 < n1 && i2 < n2 && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2;
  double M1v = 0, A1v = 0, M2v = 0, A2v = 0;
  int64_t off12 = 0;
  bool dirRow12 = false, dirCol12 = false;
  if (live) {
    M1v = pb.sepM[1][(size_t)i1 * W + o1];
    A1v = pb.sepA[1][(size_t)i1 * W + o1];
    M2v = pb.sepM[2][(size_t)i2 * W + o2];
    A2v = pb.sepA[2][(size_t)i2 * W + o2];
    int l1 = max(0, i1 - p), w1 = min(n1 - 1, i1 + p) - l1 + 1, l2 = max(0, i2 - p);
    off12 = (int64_t)(j2 - l2) * w1 + (j1 - l1);
    const unsigned m = pb.dmask;
    dirRow12 = (((m >> 2) & 1u) && i1 == 0) || (((m >> 3) & 1u) && i1 == n1 - 1) || (((m >> 4) & 1u) && i2 == 0) ||
               (((m >> 5) & 1u) && i2 == n2 - 1);
    dirCol12 = (((m >> 2) & 1u) && j1 == 0) || (((m >> 3) & 1u) && j1 == n1 - 1) || (((m >> 4) & 1u) && j2 == 0) ||
               (((m >> 5) & 1u) && j2 == n2 - 1);
  }
  CT acc[P][W];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int k = 0; k < W; ++k) acc[a][k] = 0;
  const double lam = pb.lambda;
  __syncthreads();

  for (int e0 = 0; e0 < pb.ne[0]; ++e0) {
    // (1) coefficient window and axis-0 tables
    for (int i = t; i < P * NI2 * NI1; i += NT) {
      int k1 = i % NI1, k2 = (i / NI1) % NI2, a0 = i / (NI1 * NI2);
      int g1 = W1lo + k1, g2 = W2lo + k2;
      double v = 0.0;
      if (g1 >= 0 && g1 < n1 && g2 >= 0 && g2 < n2) v = U[(e0 + a0) + (int64_t)n0 * (g1 + (int64_t)n1 * g2)];
      sU[a0][k2][k1] = v;
    }
    if (t < Q * P) {
      double b = pb.ax[0].B[(size_t)e0 * Q * P + t];
      (&tB0[0][0])[t] = b;
      (&cB0[0][0])[t] = (CT)b;
    }
    if (t < Q) tw0[t] = pb.ax[0].wq[(size_t)e0 * Q + t];
    __syncthreads();
    // (2) contract axis 0 of the coefficients
    for (int i = t; i < Q * NI2 * NI1; i += NT) {
      int k1 = i % NI1, k2 = (i / NI1) % NI2, q0 = i / (NI1 * NI2);
      double s = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) s += tB0[q0][a0] * sU[a0][k2][k1];
      V0[q0][k2][k1] = s;
    }
    __syncthreads();
    // (3) contract axis 1
    for (int i = t; i < Q * NI2 * G1; i += NT) {
      int g1 = i % G1, k2 = (i / G1) % NI2, q0 = i / (G1 * NI2), el = g1 / Q, q1 = g1 % Q;
      double s = 0;
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) s += tB1[el][q1][a1] * V0[q0][k2][el + a1];
      V1[q0][k2][g1] = s;
    }
    __syncthreads();
    // (4) u at the window's quadrature points -> reaction coefficient m = -lambda W e^u
    for (int i = t; i < Q * G2 * G1; i += NT) {
      int g1 = i % G1, g2 = (i / G1) % G2, q0 = i / (G1 * G2), el1 = g1 / Q, q1 = g1 % Q, el2 = g2 / Q, q2 = g2 % Q;
      double u = 0;
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) u += tB2[el2][q2][a2] * V1[q0][el2 + a2][g1];
      double Wq = tw0[q0] * tw1[el1][q1] * tw2[el2][q2];
      mq[q0][g2][g1] = (Wq != 0.0) ? (CT)(-lam * Wq) * exp_ct<CT>(u) : (CT)0;
    }
    __syncthreads();
    // (5) level 1: band contraction over the quadrature points of axis 2 in supp(i2)
    for (int i = t; i < Q * B2 * G1; i += NT) {
      int g1 = i % G1, il = (i / G1) % B2, q0 = i / (G1 * B2);
      CT m[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) m[k] = mq[q0][il * Q + k][g1];
#pragma unroll
      for (int o = 0; o < W; ++o) {
        CT s = 0;
#pragma unroll
        for (int k = 0; k < KM; ++k) s += phi2[il][o][k] * m[k];
        T1[q0][il * W + o][g1] = s;
      }
    }
    __syncthreads();
    // (6) level 2: band contraction over the quadrature points of axis 1 in supp(i1)
    for (int i = t; i < Q * B1 * R2; i += NT) {
      int rr = i % R2, il = (i / R2) % B1, q0 = i / (R2 * B1);
      CT v[KM];
#pragma unroll
      for (int k = 0; k < KM; ++k) v[k] = T1[q0][rr][il * Q + k];
#pragma unroll
      for (int o = 0; o < W; ++o) {
        CT s = 0;
#pragma unroll
        for (int k = 0; k < KM; ++k) s += phi1[il][o][k] * v[k];
        T2[q0][il * W + o][rr] = s;
      }
    }
    __syncthreads();
    // (7) level 3: axis 0 into the register window
    if (live) {
      CT y[Q][P];
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        CT tq = T2[q0][r1][r2];
#pragma unroll
        for (int b0 = 0; b0 < P; ++b0) y[q0][b0] = cB0[q0][b0] * tq;
      }
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0)
#pragma unroll
        for (int b0 = 0; b0 < P; ++b0) {
          CT s = 0;
#pragma unroll
          for (int q0 = 0; q0 < Q; ++q0) s += cB0[q0][a0] * y[q0][b0];
          acc[a0][b0 - a0 + p] += s;
        }
      // (8) emit the completed row(s)
      const int last = (e0 == pb.ne[0] - 1) ? p : 0;
      const unsigned msk = pb.dmask;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) {
        if (a0 > last) break;
        const int i0 = e0 + a0;
        const bool rowDir = dirRow12 || (((msk >> 0) & 1u) && i0 == 0) || (((msk >> 1) & 1u) && i0 == n0 - 1);
        const int l0 = max(0, i0 - p), w0 = min(n0 - 1, i0 + p) - l0 + 1;
        const int64_t A = i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2);
        const int64_t base = pb.row_ptr[A] + off12 * w0 - l0;
        const double *sM0 = pb.sepM[0] + (size_t)i0 * W, *sA0 = pb.sepA[0] + (size_t)i0 * W;
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int j0 = i0 + k - p;
          if (j0 < 0 || j0 >= n0) continue;
          double v;
          if (rowDir) {
            v = (k == p && o1 == p && o2 == p) ? 1.0 : 0.0;
          } else if (dirCol12 || (((msk >> 0) & 1u) && j0 == 0) || (((msk >> 1) & 1u) && j0 == n0 - 1)) {
            v = 0.0;
          } else {
            v = (double)acc[a0][k] + sA0[k] * M1v * M2v + sM0[k] * (A1v * M2v + M1v * A2v);
          }
          vals[base + j0] = (OT)v;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < P - 1; ++a)
#pragma unroll
      for (int k = 0; k < W; ++k) acc[a][k] = acc[a + 1][k];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[P - 1][k] = 0;
    __syncthreads();
  }
}

template <int P, int B1, int B2>
iga_status run_sep3(const Handle &h, const double *U, void *vals, int prec) {
  constexpr int W = 2 * P - 1;
  constexpr int NT = rs_threads(B1 * W * B2 * W);
  const int nb1 = (h.pb.n[1] + B1 - 1) / B1, nb2 = (h.pb.n[2] + B2 - 1) / B2;
  dim3 grid((unsigned)(nb1 * nb2)), block(NT);
  if (prec == IGA_FP32)
    hipLaunchKernelGGL((k_rgsep3<P, B1, B2, float, float>), grid, block, 0, h.stream, h.pb, U, (float *)vals);
  else
    hipLaunchKernelGGL((k_rgsep3<P, B1, B2, double, double>), grid, block, 0, h.stream, h.pb, U, (double *)vals);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

}  // namespace

bool rgsep_supported(const Handle &h, int b1, int b2) {
  if (!h.pb.separable || !h.pb.simple_knots || h.pb.dim != 3) return false;
  if (h.pb.P < 2 || h.pb.P > 5) return false;
  if (h.pb.P == 5) return (b1 == 2 && b2 == 2) || (b1 == 2 && b2 == 1);
  return (b1 == 4 && b2 == 2) || (b1 == 2 && b2 == 2) || (b1 == 4 && b2 == 4) || (b1 == 8 && b2 == 2);
}

iga_status launch_jac_rgsep(Handle &h, const double *U, void *vals, int prec, int b1, int b2) {
  if (!rgsep_supported(h, b1, b2)) return fail(IGA_EUNSUPPORTED, "separable row-gather configuration");
#define IGA_SEP(PP, X, Y) \
  if (h.pb.P == PP && b1 == X && b2 == Y) return run_sep3<PP, X, Y>(h, U, vals, prec);
  IGA_SEP(2, 4, 2) IGA_SEP(2, 2, 2) IGA_SEP(2, 4, 4) IGA_SEP(2, 8, 2)
  IGA_SEP(3, 4, 2) IGA_SEP(3, 2, 2) IGA_SEP(3, 4, 4) IGA_SEP(3, 8, 2)
  IGA_SEP(4, 4, 2) IGA_SEP(4, 2, 2) IGA_SEP(4, 4, 4) IGA_SEP(4, 8, 2)
  IGA_SEP(5, 2, 2) IGA_SEP(5, 2, 1)
#undef IGA_SEP
  return fail(IGA_EUNSUPPORTED, "separable row-gather block");
}

}  // namespace iga
