// Row-gather Jacobian for the separable case: identity geometry, no weights, kappa = 1.
//
// With x = xi and W = w0(g0) w1(g1) w2(g2) the stiffness part of eq:jacobian is the Kronecker
// sum A0 (x) M1 (x) M2 + M0 (x) A1 (x) M2 + M0 (x) M1 (x) A2 of 1D band matrices (built once at
// creation), so only the reaction term -lambda e^u N_A N_B needs a 3D contraction:
//
//   J_react[(i0,i1,i2),(j0,j1,j2)] = sum_g phi0[i0][j0-i0](g0) phi1[i1][j1-i1](g1) phi2[i2][j2-i2](g2) m(g)
//
// with m(g) = -lambda W(g) e^{u(g)} at the global Gauss point g and phi_d[i][o](g) = B_i(g) B_{i+o-p}(g)
// over the p+1 elements of supp(B_i).  Two kernels:
//
//  * k_mfield evaluates m at every Gauss point once (sum factorisation over an element row),
//    layout [g0][g2][g1];
//  * k_rgsep3 gives a workgroup B1 x B2 row pencils (i1, i2) and a segment of rows along axis 0.
//    It streams the element columns e0 of that segment; per column it stages the m window of
//    its (B1+p) x (B2+p) elements in LDS, contracts axis 2 (level 1) and axis 1 (level 2) with
//    fixed-length band dot products, and folds axis 0 into a per-thread register window of the
//    p+1 rows still open (level 3).  A row is complete when the column of its last supporting
//    element has been added; it is staged in LDS in CSR order and written once, by consecutive
//    lanes on consecutive entries, during the next column.  No atomics; every sum's order is fixed.
//
// The band operators phi1, phi2 are per-mesh tables indexed by a wave-uniform row, read through
// the scalar cache as SGPR operands of the FMAs.  Everything a column needs from memory (the m
// window, the axis-0 basis values, the 1D matrix rows and the row pointer, computed from
// per-axis prefix sums of the stencil widths) is loaded one column ahead, so no global-memory
// round trip sits on a column's critical path.
#include <mutex>
#include <utility>

#include "iga_impl.h"

namespace iga {
namespace {

template <typename CT>
__device__ inline CT exp_ct(double u);
template <>
__device__ inline double exp_ct<double>(double u) { return exp(u); }
template <>
__device__ inline float exp_ct<float>(double u) { return expf((float)u); }

// ---------------------------------------------------------------------------------------------
// m(g) = -lambda W(g) exp(u(g)) at every Gauss point, layout [g0][g2][g1], g_d = e_d * Q + q_d.
// Block (chunk of C1 elements along axis 1, e2, e0); u by sum factorisation: axes 0 and 2 on the
// coefficient block in LDS, then axis 1 per point.
// ---------------------------------------------------------------------------------------------
template <int P>
constexpr int mf_chunk() { return 256 / P; }

template <int P, typename CT>
__global__ void __launch_bounds__(256) k_mfield(DevProblem pb, const double *__restrict__ U, CT *__restrict__ mf) {
  constexpr int p = P - 1, Q = P, C1 = mf_chunk<P>(), NK = C1 + p;
  __shared__ double sU[P][P][NK];
  __shared__ double V[Q][Q][NK];
  __shared__ double b0[Q][P], b2[Q][P], w0[Q], w2[Q];
  const int t = threadIdx.x;
  const int e1s = blockIdx.x * C1, e2 = blockIdx.y, e0 = blockIdx.z;
  const int n0 = pb.n[0], n1 = pb.n[1], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nc = min(C1, ne1 - e1s), nk = nc + p;
  for (int i = t; i < P * P * nk; i += 256) {   // a0 fastest: runs of P consecutive coefficients of U
    const int a0 = i % P, k1 = (i / P) % nk, a2 = i / (nk * P);
    sU[a2][a0][k1] = U[wrap_fn(pb.ax[0], e0 + a0) + (int64_t)n0 * ((e1s + k1) + (int64_t)n1 * (e2 + a2))];
  }
  if (t < Q * P) {
    (&b0[0][0])[t] = pb.ax[0].B[(size_t)e0 * Q * P + t];
    (&b2[0][0])[t] = pb.ax[2].B[(size_t)e2 * Q * P + t];
  }
  if (t < Q) {
    w0[t] = pb.ax[0].wq[(size_t)e0 * Q + t];
    w2[t] = pb.ax[2].wq[(size_t)e2 * Q + t];
  }
  __syncthreads();
  for (int i = t; i < Q * Q * nk; i += 256) {
    const int k1 = i % nk, q0 = (i / nk) % Q, q2 = i / (nk * Q);
    double s = 0;
#pragma unroll
    for (int a2 = 0; a2 < P; ++a2) {
      double s0 = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) s0 += b0[q0][a0] * sU[a2][a0][k1];
      s += b2[q2][a2] * s0;
    }
    V[q2][q0][k1] = s;
  }
  __syncthreads();
  const double lam = pb.lambda;
  const size_t G1 = (size_t)ne1 * Q, G2 = (size_t)ne2 * Q;
  for (int g = t; g < nc * Q; g += 256) {
    const int el = g / Q, q1 = g % Q, e1 = e1s + el;
    double bb[P];
#pragma unroll
    for (int a1 = 0; a1 < P; ++a1) bb[a1] = pb.ax[1].B[((size_t)e1 * Q + q1) * P + a1];
    const double w1 = pb.ax[1].wq[(size_t)e1 * Q + q1];
#pragma unroll
    for (int q2 = 0; q2 < Q; ++q2)
#pragma unroll
      for (int q0 = 0; q0 < Q; ++q0) {
        double u = 0;
#pragma unroll
        for (int a1 = 0; a1 < P; ++a1) u += bb[a1] * V[q2][q0][el + a1];
        const double Wq = w0[q0] * w1 * w2[q2];
        mf[((size_t)(e0 * Q + q0) * G2 + (size_t)(e2 * Q + q2)) * G1 + (size_t)e1s * Q + g] =
            (CT)(-lam * Wq) * exp_ct<CT>(u);
      }
  }
}

// ---------------------------------------------------------------------------------------------
// Row-gather kernel.
// ---------------------------------------------------------------------------------------------
constexpr int rup64(int x) { return ((x + 63) / 64) * 64; }
constexpr int rs_threads(int nown) { return rup64(nown) < 256 ? 256 : rup64(nown); }

// Waves per SIMD the register budget is sized for (measured at 64^3, p = 3): FP64 4-wave
// blocks run best with up to 256 VGPRs (2 waves/SIMD: no spills), FP32 ones and the 7-wave
// blocks with <= 128 (4 waves/SIMD).
constexpr int sep_min_waves(int P, int B1, int B2, bool fp64) {
  return P > 4 || B1 * B2 > 8 ? 1 : (fp64 && B1 * B2 <= 4) ? 2 : 4;
}

template <class F, int... Rs>
__device__ __forceinline__ void unroll_seq(F &&f, std::integer_sequence<int, Rs...>) {
  (f(std::integral_constant<int, Rs>{}), ...);
}

// out[o] = sum_k ph[o][k] v[k] over the (p+1)^2 Gauss points of supp(B_i) (v in registers,
// ph wave-uniform).  Only k in the overlap of supp(B_i) and supp(B_{i+o-p}) can be non-zero:
// elements (o-p)..p of the support for o >= p, 0..(p+o-p) otherwise, so each dot product runs
// over that compile-time range; the 2p+1 dot products are independent FMA chains.
template <int P, typename CT, class Store>
__device__ __forceinline__ void band_dots(const CT *__restrict__ ph, const CT (&v)[P * P], Store &&store) {
  constexpr int p = P - 1, Q = P, W = 2 * p + 1, KM = P * Q;
  unroll_seq(
      [&](auto Oc) {
        constexpr int o = decltype(Oc)::value;
        constexpr int kl = o >= p ? (o - p) * Q : 0;
        constexpr int kh = o >= p ? KM : KM + (o - p) * Q;
        CT s0 = 0;
#pragma unroll
        for (int k = kl; k < kh; ++k) s0 += ph[o * KM + k] * v[k];
        store(o, s0);
      },
      std::make_integer_sequence<int, W>{});
}

template <int P, int B1, int B2, typename CT, typename OT, bool PER0>
__global__ void __launch_bounds__(rs_threads(B1 * (2 * P - 1) * B2 * (2 * P - 1)), sep_min_waves(P, B1, B2, sizeof(CT) == 8))
k_rgsep3(DevProblem pb, const CT *__restrict__ mf, const CT *__restrict__ phi1, const CT *__restrict__ phi2,
         const CT *__restrict__ b0t, const int64_t *__restrict__ cw0, const double *__restrict__ sepM0,
         const double *__restrict__ sepA0, OT *__restrict__ vals, int seg_len, int nseg, int nlogical) {
  constexpr int p = P - 1, Q = P, W = 2 * p + 1, KM = P * Q;
  constexpr int ME1 = B1 + p, ME2 = B2 + p, G1 = ME1 * Q, G2 = ME2 * Q;
  constexpr int G1P = G1 | 1;                 // odd row stride: conflict-free level-2 reads
  constexpr int R1 = B1 * W, R2 = B2 * W, NOWN = R1 * R2;
  constexpr int NT = rs_threads(NOWN);
  constexpr int NWIN = Q * G2 * G1, NLD = (NWIN + NT - 1) / NT;
  constexpr int L5 = Q * G1, NL5 = rup64(L5);   // level-1 lanes per pencil row il2
  constexpr int L6 = Q * R2, NL6 = rup64(L6);   // level-2 lanes per pencil row il1

  constexpr int NROW = B1 * B2, RLEN = W * W * W;   // rows emitted per column, values per row
  __shared__ CT mw[Q][G2][G1];
  __shared__ CT T1[Q][R2][G1P];
  __shared__ CT T2[Q][R1][R2];
  __shared__ OT stage[NROW][RLEN];      // completed rows in CSR order, written out coalesced
  __shared__ int64_t rstart[NROW];
  __shared__ int rlen[NROW];
  // per-column tables, double-buffered and loaded one column ahead: axis-0 basis values of
  // element e0, the 1D mass / stiffness rows and the width prefix sum of row i0 = e0
  constexpr int QP = Q * P, NTAB = QP + 2 * W + 1;
  static_assert(NTAB <= NT, "one table entry per thread");
  __shared__ CT tb0[2][QP];
  __shared__ double tsm[2][W], tsa[2][W];
  __shared__ int64_t tcw[2];

  // XCD-aware block order: consecutive dispatch slots go round-robin over the 8 XCDs, so
  // logical block L = (b mod 8) * C + b / 8 keeps neighbouring pencil blocks (which share m
  // windows) in one XCD's L2.  The grid is padded to 8 C blocks.
  const int nb8 = gridDim.x / 8;
  const int L = (int)(blockIdx.x % 8) * nb8 + (int)(blockIdx.x / 8);
  if (L >= nlogical) return;
  const int n0 = pb.n[0], n1 = pb.n[1], n2 = pb.n[2];
  const int ne0 = pb.ne[0], ne1 = pb.ne[1], ne2 = pb.ne[2];
  const int nb1 = (n1 + B1 - 1) / B1, nb2 = (n2 + B2 - 1) / B2;
  const int npb = nb1 * nb2;
  const int seg = L / npb, pbi = L % npb;
  const int I1 = (pbi % nb1) * B1, I2 = (pbi / nb1) * B2;
  const int W1lo = I1 - p, W2lo = I2 - p;   // first window element (may be negative)
  const int row_lo = seg * seg_len, row_hi = (seg == nseg - 1) ? n0 : (seg + 1) * seg_len;
  // a periodic axis 0 (PER0; C^(p-1) across the seam: n0 = ne0 functions, element e carries rows
  // e .. e + p mod n0) takes its warm-up columns from the far end of the axis (column e < 0 is element
  // e + ne0); an open one starts at column 0 and flushes its last p rows with columns past ne0.  A
  // template parameter, so that the open kernel carries none of the seam arithmetic.
  constexpr bool per0 = PER0;
  const int e_start = per0 ? row_lo - p : max(0, row_lo - p), e_end = row_hi;
  const int t = threadIdx.x;
  const size_t GG1 = (size_t)ne1 * Q, GG2 = (size_t)ne2 * Q;

  // ---- owner of the register window: (il1, o1, il2, o2) ----
  const bool owner = t < NOWN;
  const int r2 = t % R2, r1 = (t / R2) % R1;
  const int o2 = r2 % W, il2 = r2 / W, o1 = r1 % W, il1 = r1 / W;
  const int i1 = I1 + il1, i2 = I2 + il2, j1 = i1 + o1 - p, j2 = i2 + o2 - p;
  const bool live = owner && i1 < n1 && i2 < n2 && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2;
  double c1 = 0, c2 = 0;   // M1 M2 and A1 M2 + M1 A2 of this (i1,j1,i2,j2)
  int64_t off12 = 0;
  // row pointer of row (i0,i1,i2) = rp12 + m12 * cw0[i0], with cw_d the prefix sums of the
  // stencil widths w_d: rows with a smaller i2, then a smaller i1 at this i2, then a smaller i0
  int64_t rp12 = 0, m12 = 0;
  bool dirRow12 = false, dirCol12 = false;
  const unsigned msk = pb.dmask;
  if (live) {
    const double M1v = pb.sepM[1][(size_t)i1 * W + o1], A1v = pb.sepA[1][(size_t)i1 * W + o1];
    const double M2v = pb.sepM[2][(size_t)i2 * W + o2], A2v = pb.sepA[2][(size_t)i2 * W + o2];
    c1 = M1v * M2v;
    c2 = A1v * M2v + M1v * A2v;
    const int64_t *cw1 = cw0 + (n0 + 1), *cw2 = cw1 + (n1 + 1);
    const int64_t T0 = cw0[n0], T1w = cw1[n1];
    const int64_t w1i = cw1[i1 + 1] - cw1[i1], w2i = cw2[i2 + 1] - cw2[i2];
    rp12 = cw2[i2] * T1w * T0 + w2i * cw1[i1] * T0;
    m12 = w2i * w1i;
    const int l1 = max(0, i1 - p), w1 = min(n1 - 1, i1 + p) - l1 + 1, l2 = max(0, i2 - p);
    off12 = (int64_t)(j2 - l2) * w1 + (j1 - l1);
    dirRow12 = (((msk >> 2) & 1u) && i1 == 0) || (((msk >> 3) & 1u) && i1 == n1 - 1) ||
               (((msk >> 4) & 1u) && i2 == 0) || (((msk >> 5) & 1u) && i2 == n2 - 1);
    dirCol12 = (((msk >> 2) & 1u) && j1 == 0) || (((msk >> 3) & 1u) && j1 == n1 - 1) ||
               (((msk >> 4) & 1u) && j2 == 0) || (((msk >> 5) & 1u) && j2 == n2 - 1);
  }
  CT acc[P][W];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int k = 0; k < W; ++k) acc[a][k] = 0;

  // m window of element column e0 -> registers (zero outside the mesh).  The offset of each
  // loaded point inside the Q planes of a column is the same for every column: computed once.
  CT pre[NLD];
  int woff[NLD];
#pragma unroll
  for (int j = 0; j < NLD; ++j) {
    const int i = t + j * NT;
    woff[j] = -1;
    if (i < NWIN) {
      const int q0 = i / (G2 * G1), rr = i % (G2 * G1), g2l = rr / G1, g1l = rr % G1;
      const int el1 = W1lo + g1l / Q, el2 = W2lo + g2l / Q;
      if (el1 >= 0 && el1 < ne1 && el2 >= 0 && el2 < ne2)
        woff[j] = (int)(((size_t)q0 * GG2 + (size_t)(W2lo * Q + g2l)) * GG1 + (size_t)(W1lo * Q + g1l));
    }
  }
  // every lane loads (points outside the mesh read the column's first point and are zeroed when
  // stored), so no register is written while a load into it may still be in flight
  auto load_win = [&](int e0) {
    const CT *base = mf + (size_t)(PER0 && e0 < 0 ? e0 + ne0 : e0) * Q * GG2 * GG1;
#pragma unroll
    for (int j = 0; j < NLD; ++j) pre[j] = base[woff[j] >= 0 ? woff[j] : 0];
  };
  auto store_win = [&]() {
#pragma unroll
    for (int j = 0; j < NLD; ++j) {
      const int i = t + j * NT;
      if (i < NWIN) (&mw[0][0][0])[i] = woff[j] >= 0 ? pre[j] : (CT)0;
    }
  };

  double tv = 0;
  int64_t tc = 0;
  auto load_tab = [&](int e0) {
    if (PER0 && e0 < 0) e0 += ne0;   // a warm-up column of a periodic axis: its rows are not emitted
    if (t < QP) {
      if (e0 < ne0) tv = (double)b0t[(size_t)e0 * QP + t];
    } else if (t < QP + W) {
      tv = sepM0[(size_t)e0 * W + (t - QP)];
    } else if (t < QP + 2 * W) {
      tv = sepA0[(size_t)e0 * W + (t - QP - W)];
    } else if (t == QP + 2 * W) {
      tc = cw0[e0];
    }
  };
  auto store_tab = [&](int buf) {
    if (t < QP) tb0[buf][t] = (CT)tv;
    else if (t < QP + W) tsm[buf][t - QP] = tv;
    else if (t < QP + 2 * W) tsa[buf][t - QP - W] = tv;
    else if (t == QP + 2 * W) tcw[buf] = tc;
  };

  // rows staged by the previous column -> vals: one wave per row, consecutive lanes on
  // consecutive CSR entries
  auto copy_out = [&]() {
    const int wv = __builtin_amdgcn_readfirstlane(t / 64), lane = t % 64;
    for (int r = wv; r < NROW; r += NT / 64) {
      const int len = rlen[r];
      const int64_t start = rstart[r];
      // streamed once: non-temporal, so the values do not displace the m windows in L2
      for (int loc = lane; loc < len; loc += 64) __builtin_nontemporal_store(stage[r][loc], &vals[start + loc]);
    }
  };

  // one element column; R = rotation of the register window (slot of local function a0 is (a0+R) mod P).
  // Columns e0 >= ne0 contract nothing: they only emit the last p rows, one per column.
  auto step = [&](auto Rc, int e0) {
    constexpr int R = decltype(Rc)::value;
    const bool contract = e0 < ne0;
    const int buf = (e0 - e_start) & 1;
    if (e0 + 1 < ne0) load_win(e0 + 1);   // in flight during this column
    if (e0 + 1 < e_end) load_tab(e0 + 1);
    if (contract) {
      // (1) level 1: band contraction over the Gauss points of axis 2 in supp(i2)
      for (int it = t; it < B2 * NL5; it += NT) {
        const int jl2 = __builtin_amdgcn_readfirstlane(it / NL5);
        const int l = it % NL5;
        if (l < L5 && I2 + jl2 < n2) {
          const int q0 = l / G1, g1l = l % G1;
          CT m[KM];
#pragma unroll
          for (int k = 0; k < KM; ++k) m[k] = mw[q0][jl2 * Q + k][g1l];
          band_dots<P, CT>(phi2 + (size_t)(I2 + jl2) * W * KM, m,
                           [&](int o, CT val) { T1[q0][jl2 * W + o][g1l] = val; });
        }
      }
    }
    copy_out();
    __syncthreads();
    if (contract) {
      // (2) level 2: band contraction over the Gauss points of axis 1 in supp(i1)
      for (int it = t; it < B1 * NL6; it += NT) {
        const int jl1 = __builtin_amdgcn_readfirstlane(it / NL6);
        const int l = it % NL6;
        if (l < L6 && I1 + jl1 < n1) {
          const int q0 = l / R2, rr = l % R2;
          CT v[KM];
#pragma unroll
          for (int k = 0; k < KM; ++k) v[k] = T1[q0][rr][jl1 * Q + k];
          band_dots<P, CT>(phi1 + (size_t)(I1 + jl1) * W * KM, v,
                           [&](int o, CT val) { T2[q0][jl1 * W + o][rr] = val; });
        }
      }
      __syncthreads();
      // (3) level 3: axis 0 into the register window
      if (live) {
        CT t2[Q];
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) t2[q0] = T2[q0][r1][r2];
        const CT *bp = tb0[buf];
#pragma unroll
        for (int q0 = 0; q0 < Q; ++q0) {
          CT y[P];
#pragma unroll
          for (int b0 = 0; b0 < P; ++b0) y[b0] = bp[q0 * P + b0] * t2[q0];
#pragma unroll
          for (int a0 = 0; a0 < P; ++a0)
#pragma unroll
            for (int b0 = 0; b0 < P; ++b0) acc[(a0 + R) % P][b0 - a0 + p] += bp[q0 * P + a0] * y[b0];
        }
      }
    }
    // row i0 = e0 has received its last element column: stage it, then reuse its slot
    const int i0 = e0;
    const bool emit = e0 >= row_lo;
    // the row's axis-0 columns: an open axis stores column j0 at j0 - l0; on a periodic axis the 2p + 1
    // columns i0 - p .. i0 + p wrap, and a row at the seam lists them sorted: those at or below
    // (i0 + p) mod n0 first, the wrapped-around ones after (position j - (n0 - W))
    const int l0 = per0 ? 0 : max(0, i0 - p), w0 = per0 ? W : min(n0 - 1, i0 + p) - l0 + 1;
    const bool seam = per0 && (i0 < p || i0 + p >= n0);
    const int lowEnd = i0 + p >= n0 ? i0 + p - n0 : i0 + p;
    const int slot = il1 * B2 + il2;
    if (live && emit) {
      // the column range and the axis-0 Dirichlet tests depend on i0 and k only (wave-uniform)
      const bool rowDir = dirRow12 || (((msk >> 0) & 1u) && i0 == 0) || (((msk >> 1) & 1u) && i0 == n0 - 1);
      const bool diag = o1 == p && o2 == p;
      const double *sM0 = tsm[buf], *sA0 = tsa[buf];
      OT *dst = &stage[slot][off12 * w0];
#pragma unroll
      for (int k = 0; k < W; ++k) {
        int j0 = i0 + k - p;
        if (!per0 && (j0 < 0 || j0 >= n0)) continue;
        const bool colDir = dirCol12 || (((msk >> 0) & 1u) && j0 == 0) || (((msk >> 1) & 1u) && j0 == n0 - 1);
        double v = (double)acc[R][k] + sA0[k] * c1 + sM0[k] * c2;
        v = colDir ? 0.0 : v;
        v = rowDir ? ((k == p && diag) ? 1.0 : 0.0) : v;
        int pos = j0 - l0;
        if (per0) {
          j0 = j0 < 0 ? j0 + n0 : (j0 >= n0 ? j0 - n0 : j0);
          pos = !seam ? k : (j0 <= lowEnd ? j0 : j0 - (n0 - W));
        }
        dst[pos] = (OT)v;
      }
    }
    if (owner && o1 == p && o2 == p) {   // the diagonal window of each pencil row describes it
      const bool row = live && emit;
      rstart[slot] = row ? rp12 + m12 * tcw[buf] : 0;
      rlen[slot] = row ? (int)(m12 * w0) : 0;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) acc[R][k] = 0;   // slot R becomes local function p of the next column
    if (e0 + 1 < ne0) store_win();
    if (e0 + 1 < e_end) store_tab(buf ^ 1);
    __syncthreads();
  };

  if (t < NROW) rlen[t] = 0;
  load_win(e_start);
  store_win();
  load_tab(e_start);
  store_tab(0);
  __syncthreads();
  for (int e0 = e_start; e0 < e_end; e0 += P) {
    unroll_seq(
        [&](auto Rc) {
          constexpr int R = decltype(Rc)::value;
          if (e0 + R < e_end) step(Rc, e0 + R);
        },
        std::make_integer_sequence<int, P>{});
  }
  copy_out();
}

struct SepPlan {
  int nseg, seg_len, nlogical, grid;
};

template <int P, int B1, int B2, typename CT, typename OT, bool PER0>
SepPlan plan_sep3(const Handle &h) {
  constexpr int W = 2 * P - 1;
  constexpr int NT = rs_threads(B1 * W * B2 * W);
  const int nb1 = (h.pb.n[1] + B1 - 1) / B1, nb2 = (h.pb.n[2] + B2 - 1) / B2;
  const int npb = nb1 * nb2, ne0 = h.pb.ne[0], p = P - 1;
  int per_cu = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rgsep3<P, B1, B2, CT, OT, PER0>, NT, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h.device) != hipSuccess || ncu < 1)
    ncu = 256;
  const long slots = (long)per_cu * ncu;
  int nseg = h.row_segments;
  if (nseg <= 0) {
    // minimise (rounds of resident blocks) x (element columns per block, warm-up included); at 64^3,
    // p = 3 this picks 3 segments: 0.457 ms against 0.498 ms for unsplit pencils, whose second round
    // of blocks half fills the chip (measured over 1..16 segments)
    double best = 1e300;
    nseg = 1;
    for (int s = 1; s <= 16 && s <= ne0; ++s) {
      const int len = (ne0 + s - 1) / s;
      const int ns = (ne0 + len - 1) / len;
      const double rounds = (double)((npb * (long)ns + slots - 1) / slots);
      const double cost = rounds * (len + (ns > 1 ? p : 0));
      if (cost < best) { best = cost; nseg = s; }
    }
  }
  if (nseg > ne0) nseg = ne0;
  SepPlan pl;
  pl.seg_len = (ne0 + nseg - 1) / nseg;
  pl.nseg = (ne0 + pl.seg_len - 1) / pl.seg_len;
  pl.nlogical = npb * pl.nseg;
  pl.grid = ((pl.nlogical + 7) / 8) * 8;
  return pl;
}

// mf: the reaction field (the handle's, or the static scratch of the allocation-free entry point);
// timed: record the kernel-timing events (never for the allocation-free entry point)
template <int P, int B1, int B2, typename CT, typename OT>
iga_status run_sep3(Handle &h, const double *U, OT *vals, CT *mf, bool timed) {
  constexpr int W = 2 * P - 1;
  constexpr int NT = rs_threads(B1 * W * B2 * W);
  const int prec = sizeof(CT) == 8 ? 0 : 1;
  dim3 gm((unsigned)((h.pb.ne[1] + mf_chunk<P>() - 1) / mf_chunk<P>()), (unsigned)h.pb.ne[2], (unsigned)h.pb.ne[0]);
  if (timed) kt_begin(h, "k_mfield");
  hipLaunchKernelGGL((k_mfield<P, CT>), gm, dim3(256), 0, h.stream, h.pb, U, mf);
  if (timed) kt_end(h);
  IGA_HIP_CHECK(hipGetLastError());
  if (timed) kt_begin(h, "k_rgsep3");
  if (h.pb.ax[0].nper) {
    const SepPlan pl = plan_sep3<P, B1, B2, CT, OT, true>(h);
    hipLaunchKernelGGL((k_rgsep3<P, B1, B2, CT, OT, true>), dim3((unsigned)pl.grid), dim3(NT), 0, h.stream, h.pb, mf,
                       (const CT *)h.sep_phi[prec][1], (const CT *)h.sep_phi[prec][2], (const CT *)h.sep_b0[prec], h.sep_cw,
                       h.pb.sepM[0], h.pb.sepA[0], vals, pl.seg_len, pl.nseg, pl.nlogical);
  } else {
    const SepPlan pl = plan_sep3<P, B1, B2, CT, OT, false>(h);
    hipLaunchKernelGGL((k_rgsep3<P, B1, B2, CT, OT, false>), dim3((unsigned)pl.grid), dim3(NT), 0, h.stream, h.pb, mf,
                       (const CT *)h.sep_phi[prec][1], (const CT *)h.sep_phi[prec][2], (const CT *)h.sep_b0[prec], h.sep_cw,
                       h.pb.sepM[0], h.pb.sepA[0], vals, pl.seg_len, pl.nseg, pl.nlogical);
  }
  if (timed) kt_end(h);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P, int B1, int B2>
iga_status run_sep3_prec(Handle &h, const double *U, void *vals, int prec, void *field, bool timed) {
  if (prec == IGA_FP32) return run_sep3<P, B1, B2, float, float>(h, U, (float *)vals, (float *)field, timed);
  return run_sep3<P, B1, B2, double, double>(h, U, (double *)vals, (double *)field, timed);
}

// ------------------------------------------------------------------------------------------
// Reaction-field memory for callers that cannot allocate (iga_assemble_jacobian_noalloc): one
// 64 MiB array per GPU, part of the code object, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (in host code the name is a host-side stand-in); it uses
// the device address looked up once per device by noalloc_scratch_init.
// ------------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

iga_status noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(IGA_EUNSUPPORTED, "device ordinal above 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return IGA_OK;
  int cur = -1;
  IGA_HIP_CHECK(hipGetDevice(&cur));
  if (cur != device) IGA_HIP_CHECK(hipSetDevice(device));
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess || ptr == nullptr)
    return fail(IGA_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return IGA_OK;
}

bool rgsep_supported(const Handle &h, int b1, int b2) {
  if (!h.pb.separable || !h.pb.simple_knots || h.pb.dim != 3 || !h.mfield) return false;
  // a periodic axis 0: C^(p-1) across the seam (as many functions as elements, so element e carries
  // rows e .. e + p mod n0) and 2p + 1 distinct columns per row
  if (h.pb.ax[0].nper && (h.pb.n[0] != h.pb.ne[0] || h.pb.n[0] < 2 * h.pb.p + 1)) return false;
  // window offsets inside the Q point planes of one element column are 32-bit
  if ((double)h.pb.Q * h.pb.ne[1] * h.pb.Q * h.pb.ne[2] * h.pb.Q >= 2147483647.0) return false;
  if (h.pb.P < 2 || h.pb.P > 5) return false;
  if (h.pb.P == 5) return (b1 == 2 && b2 == 2) || (b1 == 2 && b2 == 1);
  return (b1 == 4 && b2 == 2) || (b1 == 2 && b2 == 2) || (b1 == 4 && b2 == 4) || (b1 == 8 && b2 == 2);
}

static iga_status launch_jac_rgsep_field(Handle &h, const double *U, void *vals, int prec, int b1, int b2,
                                         void *field, bool timed) {
  if (!rgsep_supported(h, b1, b2)) return fail(IGA_EUNSUPPORTED, "separable row-gather configuration");
#define IGA_SEP(PP, X, Y) \
  if (h.pb.P == PP && b1 == X && b2 == Y) return run_sep3_prec<PP, X, Y>(h, U, vals, prec, field, timed);
  IGA_SEP(2, 4, 2) IGA_SEP(2, 2, 2) IGA_SEP(2, 4, 4) IGA_SEP(2, 8, 2)
  IGA_SEP(3, 4, 2) IGA_SEP(3, 2, 2) IGA_SEP(3, 4, 4) IGA_SEP(3, 8, 2)
  IGA_SEP(4, 4, 2) IGA_SEP(4, 2, 2) IGA_SEP(4, 4, 4) IGA_SEP(4, 8, 2)
  IGA_SEP(5, 2, 2) IGA_SEP(5, 2, 1)
#undef IGA_SEP
  return fail(IGA_EUNSUPPORTED, "separable row-gather block");
}

iga_status launch_jac_rgsep(Handle &h, const double *U, void *vals, int prec, int b1, int b2) {
  return launch_jac_rgsep_field(h, U, vals, prec, b1, b2, h.mfield, true);
}

size_t rgsep_field_bytes(const Handle &h, int prec) {
  const size_t nqp = (size_t)h.pb.ne[0] * h.pb.Q * h.pb.ne[1] * h.pb.Q * h.pb.ne[2] * h.pb.Q;
  return nqp * (prec == IGA_FP32 ? sizeof(float) : sizeof(double));
}

iga_status launch_jac_rgsep_scratch(Handle &h, const double *U, void *vals, int prec, int b1, int b2) {
  void *ptr = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (h.device >= 0 && h.device < kMaxDevices) ptr = g_scratch_ptr[h.device];
  }
  if (!ptr) return fail(IGA_ESTATE, "scratch address of this device was not looked up (iga_create does it)");
  const size_t need = rgsep_field_bytes(h, prec);
  if (need > kScratchBytes)
    return fail(IGA_EINVAL, "reaction field of " + std::to_string(need) + " bytes exceeds the " +
                                std::to_string(kScratchBytes) + "-byte scratch of the allocation-free entry point");
  return launch_jac_rgsep_field(h, U, vals, prec, b1, b2, ptr, false);
}

}  // namespace iga
