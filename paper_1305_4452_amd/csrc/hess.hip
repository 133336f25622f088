// Fourth-order operator from second spatial derivatives (Sec. 2.3 eq:ddrational; App. A
// eq:identity, eq:ddimap, eq:ddspatial):
//
//   R_A = sum_e sum_q W (Lap N_A)(Lap u_h),   Lap u_h = sum_B U_B Lap N_B,
//
// W = Gauss weight x span factors x det J, over every function (no boundary rows): the principal
// part of a primal biharmonic / Cahn-Hilliard weak form.
//
// One 64-lane workgroup per element, one lane per Gauss point (Q^d <= 64).  A lane forms at its
// point, from the element's 1D value / first / second derivative tables staged in LDS:
//   * the weight w and its parametric derivatives (rational bases);
//   * the map's parametric derivatives x_{i,alpha} and x_{i,alpha beta} from the control points,
//     its inverse xi_{alpha,i} (eq:identity) and xi_{alpha,ij} = -xi_{alpha,m} x_{m,eps mu}
//     xi_{eps,i} xi_{mu,j} (eq:ddimap, with the sign that differentiating eq:identity gives);
//   * Lap N_A = N_{A,alpha beta} xi_{alpha,i} xi_{beta,i} + N_{A,alpha} xi_{alpha,ii} for every
//     local function (eq:ddspatial, traced), kept in LDS, and W Lap u_h.
// The element's contributions sum_q Lap N_A(q) W Lap u_h(q) are added with one FP64 atomic per
// local function.  Without control points x = xi (the inverse map is the identity).
//
// On x = xi without weights in 3D the Laplacian factorises axis by axis and the operator runs by
// tiles of elements with sum factorisation instead (bih3_body, the residual's tiles and LDS plan).
#include "iga_impl.h"
#include "kern_res2.h"
#include "kern_res3.h"

namespace iga {
namespace {

constexpr int hpow(int b, int e) { return e == 0 ? 1 : b * hpow(b, e - 1); }

template <int DIM, int P>
__global__ void __launch_bounds__(64) k_biharmonic(DevProblem pb, const double *__restrict__ U,
                                                   double *__restrict__ R) {
  constexpr int Q = P, L = hpow(P, DIM), QD = hpow(Q, DIM);
  static_assert(QD <= 64 && L <= 64, "one lane per Gauss point and per local function");
  __shared__ double tb[3][3][Q][P];   // [axis][value | d/dxi | d2/dxi2][q][a]
  __shared__ double tw[3][Q];
  __shared__ double sU[L], sW[L], sX[L][3];
  __shared__ int64_t sA[L];
  __shared__ double sLap[L][QD + 1];
  __shared__ double sLu[QD];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  int em[3] = {(int)(e % pb.ne[0]), (int)((e / pb.ne[0]) % pb.ne[1]), (int)(e / ((int64_t)pb.ne[0] * pb.ne[1]))};
  for (int d = 0; d < 3; ++d) {
    for (int i = t; i < 3 * Q * P; i += 64) {
      const int kind = i / (Q * P), r = i % (Q * P);
      double v = (kind == 0 && r % P == 0) ? 1.0 : 0.0;   // axes beyond dim: the constant function
      if (d < DIM) {
        const size_t o = (size_t)em[d] * Q * P + r;
        v = kind == 0 ? pb.ax[d].B[o] : kind == 1 ? pb.ax[d].dB[o] : pb.ax[d].d2B[o];
      }
      (&tb[d][0][0][0])[i] = v;
    }
    if (t < Q) tw[d][t] = d < DIM ? pb.ax[d].wq[(size_t)em[d] * Q + t] : (t == 0 ? 1.0 : 0.0);
  }
  for (int a = t; a < L; a += 64) {
    const int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / (P * P) : 0;
    const int i0 = wrap_fn(pb.ax[0], pb.ax[0].efirst[em[0]] + a0);
    const int i1 = wrap_fn(pb.ax[1], pb.ax[1].efirst[em[1]] + a1);
    const int i2 = DIM == 3 ? wrap_fn(pb.ax[2], pb.ax[2].efirst[em[2]] + a2) : 0;
    const int64_t A = i0 + (int64_t)pb.n[0] * (i1 + (int64_t)pb.n[1] * i2);
    sA[a] = A;
    sU[a] = U[A];
    sW[a] = pb.wts ? pb.wts[A] : 1.0;
    for (int i = 0; i < 3; ++i) sX[a][i] = (pb.ctrl && i < DIM) ? pb.ctrl[A * DIM + i] : 0.0;
  }
  __syncthreads();

  if (t < QD) {
    const int qi[3] = {t % Q, (t / Q) % Q, DIM == 3 ? t / (Q * Q) : 0};
    // tensor-product value, first and second parametric derivatives of local function a
    auto tens = [&](int a, double &m, double *dm, double (*d2m)[3]) {
      const int ai[3] = {a % P, (a / P) % P, DIM == 3 ? a / (P * P) : 0};
      double v[3][3];   // [axis][order]
      for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) v[d][k] = (d < DIM || k == 0) ? tb[d][k][qi[d]][ai[d]] : 0.0;
      m = v[0][0] * v[1][0] * v[2][0];
      for (int al = 0; al < 3; ++al) {
        double s = 1.0;
        for (int d = 0; d < 3; ++d) s *= v[d][d == al ? 1 : 0];
        dm[al] = s;
        for (int be = 0; be < 3; ++be) {
          double s2 = 1.0;
          for (int d = 0; d < 3; ++d) s2 *= v[d][(d == al) + (d == be)];
          d2m[al][be] = s2;
        }
      }
    };
    // weight function and its derivatives (eq:rational)
    double w = 1.0, dw[3] = {0, 0, 0}, d2w[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (pb.wts) {
      w = 0.0;
      for (int a = 0; a < L; ++a) {
        double m, dm[3], d2m[3][3];
        tens(a, m, dm, d2m);
        w += sW[a] * m;
        for (int al = 0; al < 3; ++al) {
          dw[al] += sW[a] * dm[al];
          for (int be = 0; be < 3; ++be) d2w[al][be] += sW[a] * d2m[al][be];
        }
      }
    }
    // rational value, first and second parametric derivatives (eq:rational, eq:drational,
    // eq:ddrational)
    auto rat = [&](int a, double &n, double *dn, double (*d2n)[3]) {
      double m, dm[3], d2m[3][3];
      tens(a, m, dm, d2m);
      const double wa = sW[a];
      n = wa * m / w;
      for (int al = 0; al < 3; ++al) dn[al] = (wa * dm[al] - n * dw[al]) / w;
      for (int al = 0; al < 3; ++al)
        for (int be = 0; be < 3; ++be)
          d2n[al][be] = (wa * d2m[al][be] - n * d2w[al][be]) / w - (dn[be] * dw[al] + dn[al] * dw[be]) / w;
    };
    // the map's parametric derivatives, its inverse (eq:identity) and eq:ddimap
    double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, H[3][3][3] = {};
    if (pb.ctrl) {
      for (int i = 0; i < DIM; ++i)
        for (int al = 0; al < DIM; ++al) J[i][al] = 0.0;
      for (int a = 0; a < L; ++a) {
        double n, dn[3], d2n[3][3];
        rat(a, n, dn, d2n);
        for (int i = 0; i < DIM; ++i)
          for (int al = 0; al < DIM; ++al) {
            J[i][al] += sX[a][i] * dn[al];
            for (int be = 0; be < DIM; ++be) H[i][al][be] += sX[a][i] * d2n[al][be];
          }
      }
    }
    double det, Ji[3][3] = {};
    if (DIM == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      Ji[0][0] = J[1][1] / det;
      Ji[0][1] = -J[0][1] / det;
      Ji[1][0] = -J[1][0] / det;
      Ji[1][1] = J[0][0] / det;
    } else {
      det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
          Ji[r][c] = (J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1]) / det;
        }
    }
    // only the trace over i is needed: G[al][be] = sum_i xi_{al,i} xi_{be,i} and
    // h[al] = xi_{al,ii} = - xi_{al,m} x_{m,eps mu} G[eps][mu]
    double G[3][3] = {}, hv[3] = {};
    for (int al = 0; al < DIM; ++al)
      for (int be = 0; be < DIM; ++be)
        for (int i = 0; i < DIM; ++i) G[al][be] += Ji[al][i] * Ji[be][i];
    for (int al = 0; al < DIM; ++al) {
      double s = 0.0;
      for (int m = 0; m < DIM; ++m)
        for (int ep = 0; ep < DIM; ++ep)
          for (int mu = 0; mu < DIM; ++mu) s += Ji[al][m] * H[m][ep][mu] * G[ep][mu];
      hv[al] = -s;
    }
    double lu = 0.0;
    for (int a = 0; a < L; ++a) {
      double n, dn[3], d2n[3][3];
      rat(a, n, dn, d2n);
      double lap = 0.0;
      for (int al = 0; al < DIM; ++al) {
        lap += dn[al] * hv[al];
        for (int be = 0; be < DIM; ++be) lap += d2n[al][be] * G[al][be];
      }
      sLap[a][t] = lap;
      lu += sU[a] * lap;
    }
    sLu[t] = tw[0][qi[0]] * tw[1][qi[1]] * tw[2][qi[2]] * det * lu;
  }
  __syncthreads();
  for (int a = t; a < L; a += 64) {
    double r = 0.0;
    for (int q = 0; q < QD; ++q) r += sLap[a][q] * sLu[q];
    atomicAdd(&R[sA[a]], r);
  }
}

// Cahn-Hilliard residual on x = xi without weights (periodic axes wrap): with M = c (1 - c),
// M' = 1 - 2c and mu' = 1 / (2 theta c (1 - c)) - 2,
//   R_A = sum_e sum_q W [N_A cdot + (M mu' + lam M' Lap c) grad N_A . grad c + lam M Lap c Lap N_A],
// the primal weak form of the paper's strong form (D = 1; the lam terms are
// lam div(M grad N_A) Lap c).  One 64-lane workgroup per element, one lane per Gauss point: the lane
// forms c, cdot, grad c and Lap c, then its point's contribution to every local function (kept in
// LDS); one FP64 atomic per local function.
template <int DIM, int P>
__global__ void __launch_bounds__(64) k_cahn_hilliard(DevProblem pb, const double *__restrict__ Cv,
                                                      const double *__restrict__ Cd, double theta, double lam,
                                                      double *__restrict__ R) {
  constexpr int Q = P, L = hpow(P, DIM), QD = hpow(Q, DIM);
  static_assert(QD <= 64 && L <= 64, "one lane per Gauss point and per local function");
  __shared__ double tb[3][3][Q][P];   // [axis][value | d/dxi | d2/dxi2][q][a]
  __shared__ double tw[3][Q];
  __shared__ double sC[L], sCd[L];
  __shared__ int64_t sA[L];
  __shared__ double sR[L][QD + 1];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  int em[3] = {(int)(e % pb.ne[0]), (int)((e / pb.ne[0]) % pb.ne[1]), (int)(e / ((int64_t)pb.ne[0] * pb.ne[1]))};
  for (int d = 0; d < 3; ++d) {
    for (int i = t; i < 3 * Q * P; i += 64) {
      const int kind = i / (Q * P), r = i % (Q * P);
      double v = (kind == 0 && r % P == 0) ? 1.0 : 0.0;
      if (d < DIM) {
        const size_t o = (size_t)em[d] * Q * P + r;
        v = kind == 0 ? pb.ax[d].B[o] : kind == 1 ? pb.ax[d].dB[o] : pb.ax[d].d2B[o];
      }
      (&tb[d][0][0][0])[i] = v;
    }
    if (t < Q) tw[d][t] = d < DIM ? pb.ax[d].wq[(size_t)em[d] * Q + t] : (t == 0 ? 1.0 : 0.0);
  }
  for (int a = t; a < L; a += 64) {
    const int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / (P * P) : 0;
    const int i0 = wrap_fn(pb.ax[0], pb.ax[0].efirst[em[0]] + a0);
    const int i1 = wrap_fn(pb.ax[1], pb.ax[1].efirst[em[1]] + a1);
    const int i2 = DIM == 3 ? wrap_fn(pb.ax[2], pb.ax[2].efirst[em[2]] + a2) : 0;
    const int64_t A = i0 + (int64_t)pb.n[0] * (i1 + (int64_t)pb.n[1] * i2);
    sA[a] = A;
    sC[a] = Cv[A];
    sCd[a] = Cd[A];
  }
  __syncthreads();
  if (t < QD) {
    const int qi[3] = {t % Q, (t / Q) % Q, DIM == 3 ? t / (Q * Q) : 0};
    // value, gradient and Laplacian of local function a at this point
    auto fn = [&](int a, double &n, double *g, double &lap) {
      const int ai[3] = {a % P, (a / P) % P, DIM == 3 ? a / (P * P) : 0};
      double v[3][3];
      for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 3; ++k) v[d][k] = (d < DIM || k == 0) ? tb[d][k][qi[d]][ai[d]] : 0.0;
      n = v[0][0] * v[1][0] * v[2][0];
      lap = 0.0;
      for (int al = 0; al < 3; ++al) {
        double s = 1.0, s2 = 1.0;
        for (int d = 0; d < 3; ++d) {
          s *= v[d][d == al ? 1 : 0];
          s2 *= v[d][d == al ? 2 : 0];
        }
        g[al] = s;
        if (al < DIM) lap += s2;
      }
    };
    double c = 0, cd = 0, gc[3] = {0, 0, 0}, lc = 0;
    for (int a = 0; a < L; ++a) {
      double n, g[3], lap;
      fn(a, n, g, lap);
      c += sC[a] * n;
      cd += sCd[a] * n;
      for (int i = 0; i < 3; ++i) gc[i] += sC[a] * g[i];
      lc += sC[a] * lap;
    }
    const double W = tw[0][qi[0]] * tw[1][qi[1]] * tw[2][qi[2]];
    const double M = c * (1.0 - c), dM = 1.0 - 2.0 * c, dmu = 1.0 / (2.0 * theta * c * (1.0 - c)) - 2.0;
    const double s0 = W * cd, sg = W * (M * dmu + lam * dM * lc), s2 = W * lam * M * lc;
    for (int a = 0; a < L; ++a) {
      double n, g[3], lap;
      fn(a, n, g, lap);
      sR[a][t] = n * s0 + sg * (g[0] * gc[0] + g[1] * gc[1] + g[2] * gc[2]) + s2 * lap;
    }
  }
  __syncthreads();
  for (int a = t; a < L; a += 64) {
    double r = 0.0;
    for (int q = 0; q < QD; ++q) r += sR[a][q];
    atomicAdd(&R[sA[a]], r);
  }
}

template <int DIM, int P>
iga_status run_ch(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R) {
  hipLaunchKernelGGL((k_cahn_hilliard<DIM, P>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, C, Cd, theta,
                     lam, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P>
__global__ void __launch_bounds__(rst::kThreads) k_ch2(DevProblem pb, const double *__restrict__ C,
                                                       const double *__restrict__ Cd, double theta, double lam,
                                                       double *__restrict__ R) {
  __shared__ double lds[rst::Ch2<P>::total / sizeof(double)];
  rst::ch2_body<P>(pb, (int)blockIdx.x, C, Cd, theta, lam, R, lds);
}

template <int P>
iga_status run_ch2(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R) {
  const unsigned nb = (unsigned)rst::res2_tiles(h.pb.ne[0], h.pb.ne[1], rst::Ch2<P>::TE);
  hipLaunchKernelGGL(k_ch2<P>, dim3(nb), dim3(rst::kThreads), 0, h.stream, h.pb, C, Cd, theta, lam, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P>
__global__ void __launch_bounds__(rs3::kThreads) k_ch3(DevProblem pb, const double *__restrict__ C,
                                                       const double *__restrict__ Cd, double theta, double lam,
                                                       double *__restrict__ R) {
  __shared__ double lds[rs3::Ch3<P>::total / sizeof(double)];
  rs3::ch3_body<P>(pb, (int)blockIdx.x, C, Cd, theta, lam, R, lds);
}

template <int P>
iga_status run_ch3(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R) {
  const unsigned nb = (unsigned)rs3::res3_tiles(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], rs3::Ch3<P>::TE);
  hipLaunchKernelGGL(k_ch3<P>, dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, C, Cd, theta, lam, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// Cahn-Hilliard residual on column tiles (C^1 quadratics): tile depth / chunk length along axis 2 and the
// longest run of the streamed tiles.  Measured at 256^3 (ms per residual): fixed-depth tiles 4.44 (depth
// 3), 4.13 (depth 2); streamed chunks of 3 at 184 VGPRs (2 waves per SIMD) 3.95, capped at 168 VGPRs (3
// waves, 44 spilled) 3.31; chunks of 2 (150 VGPRs, 3 waves) in runs of 4 / 6 / 8: 3.50 / 3.33 / 3.28.
constexpr int kChrTEZ = 2;
constexpr int kChrRunMax = 8;

template <int P>
__global__ void __launch_bounds__(rs3::kThreads) k_chr3(DevProblem pb, const double *__restrict__ C,
                                                        const double *__restrict__ Cd, double theta, double lam,
                                                        double *__restrict__ R) {
  __shared__ double lds[rs3::Chr3<P, kChrTEZ>::total / sizeof(double)];
  rs3::chr3_body<P, kChrTEZ>(pb, (int)blockIdx.x, C, Cd, theta, lam, R, lds);
}

template <int P>
__global__ void __launch_bounds__(rs3::kThreads) k_chr3s(DevProblem pb, const double *__restrict__ C,
                                                         const double *__restrict__ Cd, double theta, double lam,
                                                         double *__restrict__ R, int zc) {
  __shared__ double lds[rs3::Chr3S<P, kChrTEZ>::total / sizeof(double)];
  rs3::chr3s_body<P, kChrTEZ, kChrRunMax>(pb, (int)blockIdx.x, zc, C, Cd, theta, lam, R, lds);
}

// IGA_OPT_TILED_3D = 1: column tiles streamed along axis 2 in runs of zc chunks (the option value, else the
// longest run of at most kChrRunMax chunks that leaves 1024 workgroups); 3: column tiles of fixed depth
template <int P>
iga_status run_chr3(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R) {
  using S = rs3::Chr3<P, kChrTEZ>;
  if (h.tiled_3d == 1) {
    const int nz = (h.pb.ne[2] + kChrTEZ - 1) / kChrTEZ;
    const int64_t nxy = (int64_t)((h.pb.ne[0] + S::TEX - 1) / S::TEX) * ((h.pb.ne[1] + S::TEX - 1) / S::TEX);
    int zc = std::min(kChrRunMax, nz);
    if (h.res_zrun > 0) zc = std::max(1, std::min(std::min(h.res_zrun, kChrRunMax), nz));
    else
      while (zc > 1 && nxy * ((nz + zc - 1) / zc) < 1024) --zc;
    const unsigned nb = (unsigned)rs3::res3s_blocks(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], S::TEX, kChrTEZ, zc);
    hipLaunchKernelGGL(k_chr3s<P>, dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, C, Cd, theta, lam, R, zc);
  } else {
    const unsigned nb = (unsigned)rs3::res3r_tiles(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], S::TEX, kChrTEZ);
    hipLaunchKernelGGL(k_chr3<P>, dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, C, Cd, theta, lam, R);
  }
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P>
__global__ void __launch_bounds__(rs3::kThreads) k_bih3(DevProblem pb, const double *__restrict__ U,
                                                        double *__restrict__ R) {
  __shared__ double lds[rs3::Res3<P>::total / sizeof(double)];
  rs3::bih3_body<P>(pb, (int)blockIdx.x, U, R, lds);
}

template <int P>
iga_status run_bih3(Handle &h, const double *U, double *R) {
  const unsigned nb = (unsigned)rs3::res3_tiles(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], rs3::Res3<P>::TE);
  hipLaunchKernelGGL(k_bih3<P>, dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, U, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int DIM, int P>
iga_status run_bih(Handle &h, const double *U, double *R) {
  hipLaunchKernelGGL((k_biharmonic<DIM, P>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, U, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// The fourth-order operator integrated by parts once, from third spatial derivatives (Sec. 2.3
// eq:dddrational; App. A eq:dddimap, eq:dddspatial):
//
//   R_A = sum_e sum_q W grad N_A . grad(Lap u_h),   d_i Lap u_h = sum_B U_B sum_j N_{B,ijj},
//
// over every function (no boundary rows).  One 64-lane workgroup per element, one lane per Gauss
// point.  Only the traces the operator needs are formed: with G = xi_{b,j} xi_{c,j}, h_b = xi_{b,jj},
// C_{abi} = xi_{a,ij} xi_{b,j} and X_{ai} = xi_{a,ijj} (eq:dddimap traced over j = k),
//   sum_j N_{A,ijj} = N_{A,abc} xi_{a,i} G_{bc} + N_{A,ab} (2 C_{abi} + xi_{a,i} h_b) + N_{A,a} X_{ai}.
template <int DIM, int P>
__global__ void __launch_bounds__(64) k_gradlap(DevProblem pb, const double *__restrict__ U, double *__restrict__ R) {
  constexpr int Q = P, L = hpow(P, DIM), QD = hpow(Q, DIM);
  static_assert(QD <= 64 && L <= 64, "one lane per Gauss point and per local function");
  __shared__ double tb[3][4][Q][P];   // [axis][value | d | d2 | d3][q][a]
  __shared__ double tw[3][Q];
  __shared__ double sU[L], sW[L], sX[L][3];
  __shared__ int64_t sA[L];
  __shared__ double sR[L][QD + 1];
  const int t = threadIdx.x;
  const int64_t e = blockIdx.x;
  int em[3] = {(int)(e % pb.ne[0]), (int)((e / pb.ne[0]) % pb.ne[1]), (int)(e / ((int64_t)pb.ne[0] * pb.ne[1]))};
  for (int d = 0; d < 3; ++d) {
    for (int i = t; i < 4 * Q * P; i += 64) {
      const int kind = i / (Q * P), r = i % (Q * P);
      double v = (kind == 0 && r % P == 0) ? 1.0 : 0.0;   // axes beyond dim: the constant function
      if (d < DIM) {
        const size_t o = (size_t)em[d] * Q * P + r;
        v = kind == 0 ? pb.ax[d].B[o] : kind == 1 ? pb.ax[d].dB[o] : kind == 2 ? pb.ax[d].d2B[o] : pb.ax[d].d3B[o];
      }
      (&tb[d][0][0][0])[i] = v;
    }
    if (t < Q) tw[d][t] = d < DIM ? pb.ax[d].wq[(size_t)em[d] * Q + t] : (t == 0 ? 1.0 : 0.0);
  }
  for (int a = t; a < L; a += 64) {
    const int a0 = a % P, a1 = (a / P) % P, a2 = DIM == 3 ? a / (P * P) : 0;
    const int i0 = wrap_fn(pb.ax[0], pb.ax[0].efirst[em[0]] + a0);
    const int i1 = wrap_fn(pb.ax[1], pb.ax[1].efirst[em[1]] + a1);
    const int i2 = DIM == 3 ? wrap_fn(pb.ax[2], pb.ax[2].efirst[em[2]] + a2) : 0;
    const int64_t A = i0 + (int64_t)pb.n[0] * (i1 + (int64_t)pb.n[1] * i2);
    sA[a] = A;
    sU[a] = U[A];
    sW[a] = pb.wts ? pb.wts[A] : 1.0;
    for (int i = 0; i < 3; ++i) sX[a][i] = (pb.ctrl && i < DIM) ? pb.ctrl[A * DIM + i] : 0.0;
  }
  __syncthreads();

  if (t < QD) {
    const int qi[3] = {t % Q, (t / Q) % Q, DIM == 3 ? t / (Q * Q) : 0};
    // tensor-product value and parametric derivatives up to third order of local function a
    auto tens = [&](int a, double &m, double *dm, double (*d2m)[3], double (*d3m)[3][3]) {
      const int ai[3] = {a % P, (a / P) % P, DIM == 3 ? a / (P * P) : 0};
      double v[3][4];
      for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 4; ++k) v[d][k] = (d < DIM || k == 0) ? tb[d][k][qi[d]][ai[d]] : 0.0;
      m = v[0][0] * v[1][0] * v[2][0];
      for (int al = 0; al < DIM; ++al) {
        dm[al] = v[0][al == 0] * v[1][al == 1] * v[2][al == 2];
        for (int be = 0; be < DIM; ++be) {
          d2m[al][be] = v[0][(al == 0) + (be == 0)] * v[1][(al == 1) + (be == 1)] * v[2][(al == 2) + (be == 2)];
          for (int ga = 0; ga < DIM; ++ga)
            d3m[al][be][ga] = v[0][(al == 0) + (be == 0) + (ga == 0)] * v[1][(al == 1) + (be == 1) + (ga == 1)] *
                              v[2][(al == 2) + (be == 2) + (ga == 2)];
        }
      }
    };
    // weight function and its derivatives (eq:rational)
    double w = 1.0, dw[3] = {}, d2w[3][3] = {}, d3w[3][3][3] = {};
    if (pb.wts) {
      w = 0.0;
      for (int a = 0; a < L; ++a) {
        double m, dm[3], d2m[3][3], d3m[3][3][3];
        tens(a, m, dm, d2m, d3m);
        w += sW[a] * m;
        for (int al = 0; al < DIM; ++al) {
          dw[al] += sW[a] * dm[al];
          for (int be = 0; be < DIM; ++be) {
            d2w[al][be] += sW[a] * d2m[al][be];
            for (int ga = 0; ga < DIM; ++ga) d3w[al][be][ga] += sW[a] * d3m[al][be][ga];
          }
        }
      }
    }
    // rational basis and its parametric derivatives (eq:drational, eq:ddrational, eq:dddrational)
    auto rat = [&](int a, double *dn, double (*d2n)[3], double (*d3n)[3][3]) {
      double m, dm[3], d2m[3][3], d3m[3][3][3];
      tens(a, m, dm, d2m, d3m);
      const double wa = sW[a], n = wa * m / w;
      for (int al = 0; al < DIM; ++al) dn[al] = (wa * dm[al] - n * dw[al]) / w;
      for (int al = 0; al < DIM; ++al)
        for (int be = 0; be < DIM; ++be)
          d2n[al][be] = (wa * d2m[al][be] - n * d2w[al][be]) / w - (dn[be] * dw[al] + dn[al] * dw[be]) / w;
      for (int al = 0; al < DIM; ++al)
        for (int be = 0; be < DIM; ++be)
          for (int ga = 0; ga < DIM; ++ga)
            d3n[al][be][ga] = (wa * d3m[al][be][ga] - n * d3w[al][be][ga]) / w -
                              (dn[al] * d2w[be][ga] + dn[be] * d2w[al][ga] + dn[ga] * d2w[al][be]) / w -
                              (d2n[be][ga] * dw[al] + d2n[al][ga] * dw[be] + d2n[al][be] * dw[ga]) / w;
    };
    // the map's parametric derivatives up to third order
    double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, H[3][3][3] = {}, T3[3][3][3][3] = {};
    if (pb.ctrl) {
      for (int i = 0; i < DIM; ++i)
        for (int al = 0; al < DIM; ++al) J[i][al] = 0.0;
      for (int a = 0; a < L; ++a) {
        double dn[3], d2n[3][3], d3n[3][3][3];
        rat(a, dn, d2n, d3n);
        for (int i = 0; i < DIM; ++i)
          for (int al = 0; al < DIM; ++al) {
            J[i][al] += sX[a][i] * dn[al];
            for (int be = 0; be < DIM; ++be) {
              H[i][al][be] += sX[a][i] * d2n[al][be];
              for (int ga = 0; ga < DIM; ++ga) T3[i][al][be][ga] += sX[a][i] * d3n[al][be][ga];
            }
          }
      }
    }
    double det, Ji[3][3] = {};
    if (DIM == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      Ji[0][0] = J[1][1] / det;
      Ji[0][1] = -J[0][1] / det;
      Ji[1][0] = -J[1][0] / det;
      Ji[1][1] = J[0][0] / det;
    } else {
      det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
          Ji[r][c] = (J[r1][c1] * J[r2][c2] - J[r1][c2] * J[r2][c1]) / det;
        }
    }
    // eq:ddimap (with the sign that differentiating eq:identity gives) and the traces of eq:dddimap
    double X2[3][3][3] = {}, G[3][3] = {}, hv[3] = {}, Ct[3][3][3] = {}, Xt[3][3] = {};
    for (int al = 0; al < DIM; ++al)
      for (int i = 0; i < DIM; ++i)
        for (int j = 0; j < DIM; ++j) {
          double s = 0.0;
          for (int m = 0; m < DIM; ++m)
            for (int ep = 0; ep < DIM; ++ep)
              for (int mu = 0; mu < DIM; ++mu) s += Ji[al][m] * H[m][ep][mu] * Ji[ep][i] * Ji[mu][j];
          X2[al][i][j] = -s;
        }
    for (int al = 0; al < DIM; ++al) {
      for (int be = 0; be < DIM; ++be)
        for (int j = 0; j < DIM; ++j) G[al][be] += Ji[al][j] * Ji[be][j];
      for (int j = 0; j < DIM; ++j) hv[al] += X2[al][j][j];
      for (int be = 0; be < DIM; ++be)
        for (int i = 0; i < DIM; ++i)
          for (int j = 0; j < DIM; ++j) Ct[al][be][i] += X2[al][i][j] * Ji[be][j];
    }
    for (int al = 0; al < DIM; ++al)
      for (int i = 0; i < DIM; ++i) {
        double s = 0.0;
        for (int m = 0; m < DIM; ++m)
          for (int ep = 0; ep < DIM; ++ep)
            for (int mu = 0; mu < DIM; ++mu) {
              for (int om = 0; om < DIM; ++om) s += T3[m][ep][mu][om] * Ji[al][m] * Ji[ep][i] * G[mu][om];
              s += H[m][ep][mu] * (Ct[al][mu][m] * Ji[ep][i] + Ji[al][m] * Ct[ep][mu][i] + Ji[al][m] * Ji[ep][i] * hv[mu]);
            }
        Xt[al][i] = -s;
      }
    // spatial gradient and d_i Lap of local function a (eq:dspatial, eq:dddspatial traced)
    auto grads = [&](int a, double *g, double *gl) {
      double dn[3], d2n[3][3], d3n[3][3][3];
      rat(a, dn, d2n, d3n);
      for (int i = 0; i < DIM; ++i) {
        double s = 0.0, l = 0.0;
        for (int al = 0; al < DIM; ++al) {
          s += dn[al] * Ji[al][i];
          l += dn[al] * Xt[al][i];
          for (int be = 0; be < DIM; ++be) {
            l += d2n[al][be] * (2.0 * Ct[al][be][i] + Ji[al][i] * hv[be]);
            for (int ga = 0; ga < DIM; ++ga) l += d3n[al][be][ga] * Ji[al][i] * G[be][ga];
          }
        }
        g[i] = s;
        gl[i] = l;
      }
    };
    double glu[3] = {0, 0, 0};
    for (int a = 0; a < L; ++a) {
      double g[3], gl[3];
      grads(a, g, gl);
      for (int i = 0; i < DIM; ++i) glu[i] += sU[a] * gl[i];
    }
    const double W = tw[0][qi[0]] * tw[1][qi[1]] * tw[2][qi[2]] * det;
    for (int a = 0; a < L; ++a) {
      double g[3], gl[3];
      grads(a, g, gl);
      double s = 0.0;
      for (int i = 0; i < DIM; ++i) s += g[i] * glu[i];
      sR[a][t] = W * s;
    }
  }
  __syncthreads();
  for (int a = t; a < L; a += 64) {
    double r = 0.0;
    for (int q = 0; q < QD; ++q) r += sR[a][q];
    atomicAdd(&R[sA[a]], r);
  }
}

template <int DIM, int P>
iga_status run_gradlap(Handle &h, const double *U, double *R) {
  hipLaunchKernelGGL((k_gradlap<DIM, P>), dim3((unsigned)h.pb.E), dim3(64), 0, h.stream, h.pb, U, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

}  // namespace

iga_status launch_cahn_hilliard(Handle &h, const double *C, const double *Cd, double theta, double lam, double *R,
                                bool zero_out) {
  const int p = h.pb.p;
  if (h.pb.ctrl || h.pb.wts) return fail(IGA_EUNSUPPORTED, "the Cahn-Hilliard residual needs x = xi without weights");
  if (!(theta > 0.0) || !std::isfinite(theta) || !std::isfinite(lam)) return fail(IGA_EINVAL, "theta must be positive");
  if (p < 2) return fail(IGA_EUNSUPPORTED, "the Cahn-Hilliard residual needs p >= 2");
  iga_status st = zero_out ? launch_fill(h, R, h.pb.N, 0.0) : IGA_OK;
  if (st) return st;
  // simple knots: tiles with sum factorisation (IGA_OPT_TILED_3D = 0 keeps one element per workgroup,
  // for comparison)
  if (h.pb.simple_knots && h.tiled_3d) {
    if (h.pb.dim == 3) {
      if (p == 2) return h.tiled_3d != 2 ? run_chr3<3>(h, C, Cd, theta, lam, R) : run_ch3<3>(h, C, Cd, theta, lam, R);
      if (p == 3) return run_ch3<4>(h, C, Cd, theta, lam, R);
    } else {
      switch (p) {
        case 2: return run_ch2<3>(h, C, Cd, theta, lam, R);
        case 3: return run_ch2<4>(h, C, Cd, theta, lam, R);
        case 4: return run_ch2<5>(h, C, Cd, theta, lam, R);
        case 5: return run_ch2<6>(h, C, Cd, theta, lam, R);
        case 6: return run_ch2<7>(h, C, Cd, theta, lam, R);
      }
    }
  }
  if (h.pb.dim == 2) {
    switch (p) {
      case 2: return run_ch<2, 3>(h, C, Cd, theta, lam, R);
      case 3: return run_ch<2, 4>(h, C, Cd, theta, lam, R);
      case 4: return run_ch<2, 5>(h, C, Cd, theta, lam, R);
      case 5: return run_ch<2, 6>(h, C, Cd, theta, lam, R);
      case 6: return run_ch<2, 7>(h, C, Cd, theta, lam, R);
    }
  } else {
    switch (p) {
      case 2: return run_ch<3, 3>(h, C, Cd, theta, lam, R);
      case 3: return run_ch<3, 4>(h, C, Cd, theta, lam, R);
    }
  }
  return fail(IGA_EUNSUPPORTED, "the Cahn-Hilliard residual supports p <= 6 in 2D and p <= 3 in 3D");
}

iga_status launch_grad_laplacian(Handle &h, const double *U, double *R) {
  const int p = h.pb.p;
  if (p < 2) return fail(IGA_EUNSUPPORTED, "the once-integrated fourth-order operator needs p >= 2");
  iga_status st = launch_fill(h, R, h.pb.N, 0.0);
  if (st) return st;
  if (h.pb.dim == 2) {
    switch (p) {
      case 2: return run_gradlap<2, 3>(h, U, R);
      case 3: return run_gradlap<2, 4>(h, U, R);
      case 4: return run_gradlap<2, 5>(h, U, R);
      case 5: return run_gradlap<2, 6>(h, U, R);
      case 6: return run_gradlap<2, 7>(h, U, R);
    }
  } else {
    switch (p) {
      case 2: return run_gradlap<3, 3>(h, U, R);
      case 3: return run_gradlap<3, 4>(h, U, R);
    }
  }
  return fail(IGA_EUNSUPPORTED, "the once-integrated fourth-order operator supports p <= 6 in 2D and p <= 3 in 3D");
}

iga_status launch_biharmonic(Handle &h, const double *U, double *R) {
  const int p = h.pb.p;
  if (p < 2) return fail(IGA_EUNSUPPORTED, "the fourth-order operator needs p >= 2");
  iga_status st = launch_fill(h, R, h.pb.N, 0.0);
  if (st) return st;
  // x = xi, no weights, simple knots, 3D: tiles with sum factorisation (IGA_OPT_TILED_3D = 0 keeps
  // one element per workgroup, for comparison)
  if (h.pb.dim == 3 && !h.pb.ctrl && !h.pb.wts && h.pb.simple_knots && h.tiled_3d) {
    switch (p) {
      case 2: return run_bih3<3>(h, U, R);
      case 3: return run_bih3<4>(h, U, R);
      case 4: return run_bih3<5>(h, U, R);
    }
  }
  if (h.pb.dim == 2) {
    switch (p) {
      case 2: return run_bih<2, 3>(h, U, R);
      case 3: return run_bih<2, 4>(h, U, R);
      case 4: return run_bih<2, 5>(h, U, R);
      case 5: return run_bih<2, 6>(h, U, R);
      case 6: return run_bih<2, 7>(h, U, R);
    }
  } else {
    switch (p) {
      case 2: return run_bih<3, 3>(h, U, R);
      case 3: return run_bih<3, 4>(h, U, R);
    }
  }
  return fail(IGA_EUNSUPPORTED, "the fourth-order operator supports p <= 6 in 2D and p <= 3 in 3D (p <= 4 on x = xi)");
}

}  // namespace iga
