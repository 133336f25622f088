// Fast-diagonalisation preconditioner for the separable case (identity geometry, no weights,
// kappa = 1).  There the stiffness restricted to the non-Dirichlet coefficients is the Kronecker
// sum K = A0 (x) M1 (x) M2 + M0 (x) A1 (x) M2 + M0 (x) M1 (x) A2 of the 1D stiffness and mass
// matrices of each axis, and the reaction part of eq:jacobian is close to a multiple of the mass
// matrix M = M0 (x) M1 (x) M2, because e^u varies little.  With the 1D generalised eigenpairs
// A_d V_d = M_d V_d diag(mu_d), V_d^T M_d V_d = I (Lynch, Rice and Thomas's fast diagonalisation),
//
//   (K + c M)^{-1} = (V0 (x) V1 (x) V2) diag(1 / (mu0 + mu1 + mu2 + c)) (V0 (x) V1 (x) V2)^T,
//
// applied as three dense 1D transforms along the axes, a scaling and three more transforms.
// c = -lambda * (integral-weighted mean of e^U) is set before each linear solve.  Dirichlet rows
// are identity rows, so z = r there.
//
// For mapped (NURBS) geometry or variable kappa the Jacobian is spectrally equivalent to the
// parametric Kronecker sum with per-axis coefficients, a0 A0 (x) M1 (x) M2 + a1 M0 (x) A1 (x) M2 +
// a2 M0 (x) M1 (x) A2, where a_d is the quadrature average of the metric diagonal kappa W
// (J^-1 J^-T)_dd per unit parametric volume, and the mass shift is scaled by the mean det J; the
// same eigenvectors apply with eigenvalues a0 mu0 + a1 mu1 + a2 mu2.  Only the rate of CG depends
// on how good this approximation is, not the converged answer.
#include <cmath>
#include <vector>

#include "iga_impl.h"

namespace iga {

// ---------------------------------------------------------------------------------------------
// Host: generalised symmetric eigenproblem A v = mu M v (dense, row-major, FP64).
// M = L L^T by Cholesky; C = L^{-1} A L^{-T} is symmetric; cyclic Jacobi rotations give
// C = Q diag(mu) Q^T; V = L^{-T} Q.
// ---------------------------------------------------------------------------------------------
static bool cholesky_lower(std::vector<double> &a, int n) {
  for (int j = 0; j < n; ++j) {
    double d = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(d > 0)) return false;
    d = std::sqrt(d);
    a[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double s = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = s / d;
    }
    for (int k = j + 1; k < n; ++k) a[(size_t)j * n + k] = 0.0;
  }
  return true;
}

// symmetric C (overwritten) -> eigenvalues mu, eigenvectors in the columns of Q
static void jacobi_eigen(std::vector<double> &C, int n, std::vector<double> &mu, std::vector<double> &Q) {
  Q.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
  auto at = [&](int i, int j) -> double & { return C[(size_t)i * n + j]; };
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, diag = 0;
    for (int i = 0; i < n; ++i) {
      diag += at(i, i) * at(i, i);
      for (int j = i + 1; j < n; ++j) off += at(i, j) * at(i, j);
    }
    if (off <= 1e-30 * diag) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = at(p, q);
        if (std::fabs(apq) <= 1e-300) continue;
        // rotation in the (p, q) plane that zeroes C[p][q]: tan(phi) = t
        const double theta = (at(q, q) - at(p, p)) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          const double ckp = at(k, p), ckq = at(k, q);
          at(k, p) = c * ckp - s * ckq;
          at(k, q) = s * ckp + c * ckq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          const double cpk = at(p, k), cqk = at(q, k);
          at(p, k) = c * cpk - s * cqk;
          at(q, k) = s * cpk + c * cqk;
        }
        at(p, q) = at(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {
          const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
          Q[(size_t)k * n + p] = c * qkp - s * qkq;
          Q[(size_t)k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  mu.resize(n);
  for (int i = 0; i < n; ++i) mu[i] = at(i, i);
}

// A, M dense symmetric (n x n); on success V (row-major, V[k*n+i] = component k of vector i)
// and mu.  The factorisation is checked: V^T M V = I and V^T A V = diag(mu) to 1e-9 relative.
bool gen_eigen(const std::vector<double> &A, const std::vector<double> &M, int n, std::vector<double> &V,
               std::vector<double> &mu) {
  std::vector<double> L = M;
  if (!cholesky_lower(L, n)) return false;
  // C = L^{-1} A L^{-T}: solve L X = A (forward), then C^T = L^{-1} X^T
  std::vector<double> X = A;
  for (int col = 0; col < n; ++col)
    for (int i = 0; i < n; ++i) {
      double s = X[(size_t)i * n + col];
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * X[(size_t)k * n + col];
      X[(size_t)i * n + col] = s / L[(size_t)i * n + i];
    }
  std::vector<double> C((size_t)n * n);
  for (int row = 0; row < n; ++row)   // C[row][:] = L^{-1} (X[row][:])^T  (X = L^{-1} A, C = X L^{-T})
    for (int i = 0; i < n; ++i) {
      double s = X[(size_t)row * n + i];
      for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * C[(size_t)row * n + k];
      C[(size_t)row * n + i] = s / L[(size_t)i * n + i];
    }
  for (int i = 0; i < n; ++i)   // symmetrise against rounding
    for (int j = i + 1; j < n; ++j) C[(size_t)i * n + j] = C[(size_t)j * n + i] = 0.5 * (C[(size_t)i * n + j] + C[(size_t)j * n + i]);
  std::vector<double> Q;
  jacobi_eigen(C, n, mu, Q);
  // V = L^{-T} Q: back substitution with L^T, column by column
  V.assign((size_t)n * n, 0.0);
  for (int col = 0; col < n; ++col)
    for (int i = n - 1; i >= 0; --i) {
      double s = Q[(size_t)i * n + col];
      for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * V[(size_t)k * n + col];
      V[(size_t)i * n + col] = s / L[(size_t)i * n + i];
    }
  // check
  double amax = 0, err_m = 0, err_a = 0;
  for (double v : mu) amax = std::fmax(amax, std::fabs(v));
  std::vector<double> MV((size_t)n * n), AV((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int col = 0; col < n; ++col) {
      double sm = 0, sa = 0;
      for (int k = 0; k < n; ++k) {
        sm += M[(size_t)i * n + k] * V[(size_t)k * n + col];
        sa += A[(size_t)i * n + k] * V[(size_t)k * n + col];
      }
      MV[(size_t)i * n + col] = sm;
      AV[(size_t)i * n + col] = sa;
    }
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double sm = 0, sa = 0;
      for (int k = 0; k < n; ++k) {
        sm += V[(size_t)k * n + a] * MV[(size_t)k * n + b];
        sa += V[(size_t)k * n + a] * AV[(size_t)k * n + b];
      }
      err_m = std::fmax(err_m, std::fabs(sm - (a == b ? 1.0 : 0.0)));
      err_a = std::fmax(err_a, std::fabs(sa - (a == b ? mu[a] : 0.0)));
    }
  return err_m < 1e-9 && err_a < 1e-9 * std::fmax(amax, 1.0);
}

static void fdm_ranges(const DevProblem &pb, int *lo, int *m) {
  for (int d = 0; d < 3; ++d) {
    if (d >= pb.dim) {
      lo[d] = 0;
      m[d] = 1;
      continue;
    }
    lo[d] = ((pb.dmask >> (2 * d)) & 1u) ? 1 : 0;
    m[d] = pb.n[d] - (((pb.dmask >> (2 * d + 1)) & 1u) ? 1 : 0) - lo[d];
  }
}

bool fdm_possible(const Handle &h) {
  if (h.hsepM[0].empty()) return false;
  // with every axis periodic and no Dirichlet face the stiffness has the constants in its kernel
  if (h.pb.periodic && h.pb.dmask == 0) return false;
  int lo[3], m[3];
  fdm_ranges(h.pb, lo, m);
  for (int d = 0; d < h.pb.dim; ++d)
    if (m[d] < 1 || m[d] > kFdmMax) return false;
  return true;
}

// per-axis averages a_d and the mass scale: sums over all Gauss points of the metric diagonal,
// of the mass coefficient and of the parametric weight (one partial set per block)
__global__ void __launch_bounds__(256) k_fdm_coef_sums(DevProblem pb, double *__restrict__ part) {
  __shared__ double sh[5][4];
  const int Q = pb.Q, dim = pb.dim, L = dim == 3 ? Q * Q * Q : Q * Q, NG = geo_streams(dim);
  double s[5] = {0, 0, 0, 0, 0};
  for (int64_t e = blockIdx.x; e < pb.E; e += gridDim.x) {
    const int e0 = (int)(e % pb.ne[0]);
    const int64_t r = e / pb.ne[0];
    const int e1 = (int)(r % pb.ne[1]), e2 = (int)(r / pb.ne[1]);
    const double kap = (!pb.table && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
    for (int q = threadIdx.x; q < L; q += blockDim.x) {
      const int q0 = q % Q, q1 = (q / Q) % Q, q2 = dim == 3 ? q / (Q * Q) : 0;
      double wpar = pb.ax[0].wq[(size_t)e0 * Q + q0] * pb.ax[1].wq[(size_t)e1 * Q + q1];
      if (dim == 3) wpar *= pb.ax[2].wq[(size_t)e2 * Q + q2];
      if (pb.table) {
        const double *G = pb.geo + (size_t)e * NG * L + q;
        s[0] += G[0];
        s[1] += G[L];
        if (dim == 3) s[2] += G[2 * L];
        s[3] += G[(NG - 2) * L] * G[(NG - 1) * L];   // (W / w) (1 / w): the coefficient of M_A M_B
      } else {
        s[0] += kap * wpar;
        s[1] += kap * wpar;
        if (dim == 3) s[2] += kap * wpar;
        s[3] += wpar;
      }
      s[4] += wpar;
    }
  }
  for (int k = 0; k < 5; ++k) {
    double v = s[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    double v = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) v += sh[threadIdx.x][i];
    part[blockIdx.x * 5 + threadIdx.x] = v;
  }
}

static iga_status fdm_coefficients(Handle &h, double a[3], double *mscale) {
  a[0] = a[1] = a[2] = 1.0;
  *mscale = 1.0;
  if (h.pb.separable) return IGA_OK;
  const int nb = 256;
  double *part = nullptr;
  IGA_HIP_CHECK(hipMalloc(&part, nb * 5 * sizeof(double)));
  hipLaunchKernelGGL(k_fdm_coef_sums, dim3(nb), dim3(256), 0, h.stream, h.pb, part);
  std::vector<double> hp(nb * 5);
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, h.stream);
  hipError_t e3 = hipStreamSynchronize(h.stream);
  (void)hipFree(part);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(IGA_EHIP, "preconditioner coefficients");
  double sum[5] = {0, 0, 0, 0, 0};
  for (int b = 0; b < nb; ++b)
    for (int k = 0; k < 5; ++k) sum[k] += hp[b * 5 + k];
  if (!(sum[4] > 0)) return IGA_OK;
  for (int d = 0; d < h.pb.dim; ++d) a[d] = sum[d] / sum[4];
  *mscale = sum[3] / sum[4];
  return IGA_OK;
}

static iga_status build_fdm(Handle &h) {
  const std::vector<double> *bandM = h.hsepM, *bandA = h.hsepA;
  const DevProblem &pb = h.pb;
  const int p = pb.p, W = 2 * p + 1;
  FdmData f{};
  double mu_min = 0, mins[3] = {0, 0, 0};
  double acoef[3], mscale;
  {
    iga_status sc = fdm_coefficients(h, acoef, &mscale);
    if (sc) return sc;
    for (int d = 0; d < pb.dim; ++d)
      if (!(acoef[d] > 0) || !std::isfinite(acoef[d])) return IGA_OK;   // Jacobi stays in use
  }
  f.mscale = mscale;
  std::vector<double> hostV[3], hostMu[3];   // unscaled decompositions, for axis reuse
  for (int d = 0; d < 3; ++d) {
    if (d >= pb.dim) {
      f.lo[d] = 0;
      f.m[d] = 1;
      continue;
    }
    const int n = pb.n[d];
    int los[3], ms[3];
    fdm_ranges(pb, los, ms);
    const int lo = los[d], m = ms[d], hi = lo + m;
    if (m < 1 || m > kFdmMax) return IGA_OK;   // not applicable: Jacobi stays in use
    std::vector<double> A((size_t)m * m, 0.0), M((size_t)m * m, 0.0), rs(n, 0.0);
    const bool per = pb.ax[d].nper != 0;   // periodic axis: band columns wrap (eq:map-wrap)
    for (int i = 0; i < n; ++i)
      for (int o = 0; o < W; ++o) {
        int j = i + o - p;
        if (per) j = (j + n) % n;
        if (j < 0 || j >= n) continue;
        rs[i] += bandM[d][(size_t)i * W + o];
        if (i < lo || i >= hi || j < lo || j >= hi) continue;
        A[(size_t)(i - lo) * m + (j - lo)] += bandA[d][(size_t)i * W + o];
        M[(size_t)(i - lo) * m + (j - lo)] += bandM[d][(size_t)i * W + o];
      }
    // an axis with the same 1D problem as an earlier one reuses its decomposition
    int same = -1;
    for (int e = 0; e < d && same < 0; ++e)
      if (f.lo[e] == lo && f.m[e] == m && pb.n[e] == n && pb.ax[e].nper == pb.ax[d].nper && bandM[e] == bandM[d] &&
          bandA[e] == bandA[d])
        same = e;
    std::vector<double> V, mu;
    if (same >= 0) {
      V = hostV[same];
      mu = hostMu[same];
    } else if (!gen_eigen(A, M, m, V, mu)) {
      return IGA_OK;   // fall back to Jacobi
    }
    hostV[d] = V;
    hostMu[d] = mu;
    if (same >= 0) {
      std::vector<double> smu(mu);
      for (double &v : smu) v *= acoef[d];
      double *dmu;
      iga_status st;
      if ((st = upload_owned(h, &dmu, smu.data(), smu.size()))) return st;
      f.Tf[d] = f.Tf[same];
      f.Tb[d] = f.Tb[same];
      f.mu[d] = dmu;
      f.rs[d] = f.rs[same];
      f.lo[d] = lo;
      f.m[d] = m;
      mins[d] = mins[same] / acoef[same] * acoef[d];
      mu_min += mins[d];
      continue;
    }
    for (double &v : mu) v *= acoef[d];
    // device copies: T_fwd = V^T (row i = vector i), T_bwd = V (row k = components k)
    std::vector<double> Tf((size_t)m * m);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) Tf[(size_t)i * m + k] = V[(size_t)k * m + i];
    iga_status st;
    double *dTf, *dTb, *dmu, *drs;
    if ((st = upload_owned(h, &dTf, Tf.data(), Tf.size())) || (st = upload_owned(h, &dTb, V.data(), V.size())) ||
        (st = upload_owned(h, &dmu, mu.data(), mu.size())) || (st = upload_owned(h, &drs, rs.data(), rs.size())))
      return st;
    f.Tf[d] = dTf;
    f.Tb[d] = dTb;
    f.mu[d] = dmu;
    f.rs[d] = drs;
    f.lo[d] = lo;
    f.m[d] = m;
    double mn = mu[0];
    for (double v : mu) mn = std::fmin(mn, v);
    mu_min += mn;
    mins[d] = mn;
  }
  f.mu_min = mu_min;
  double *part, *shift;
  iga_status st;
  if ((st = upload_owned(h, &part, std::vector<double>(512, 0.0).data(), 512)) ||
      (st = upload_owned(h, &shift, std::vector<double>(1, 0.0).data(), 1)))
    return st;
  h.fdm_part = part;
  h.fdm_shift = shift;
  f.ok = 1;
  h.fdm = f;
  return IGA_OK;
}

iga_status ensure_fdm(Handle &h) {
  if (h.fdm_tried) return IGA_OK;
  h.fdm_tried = 1;
  if (!fdm_possible(h)) return IGA_OK;
  return build_fdm(h);
}

// ---------------------------------------------------------------------------------------------
// Device
// ---------------------------------------------------------------------------------------------
namespace {


// Eigenvalue of the Cahn-Hilliard preconditioner am M + sa K + sb B in the product basis: with
// V^T M V = I, V^T A V = diag(mu), V^T H V = diag(eta) per axis, M = M0 M1 M2, K = sum_d A_d (x) M (x) M
// and B = sum_d H_d (x) M (x) M + 2 sum_{d<e} A_d (x) A_e (x) M (Laplacians of tensor products; on
// periodic axes int B_i'' B_j = -A_ij), it is am + sa sum mu + sb (sum eta + 2 sum_{d<e} mu_d mu_e),
// kept at least 0.05 am (the linearisation about the mean can lose definiteness inside the spinodal).
struct ChScale {
  const double *eta0, *eta1, *eta2;
  double am, sa, sb;
};

struct BoxView {
  int64_t off, s0, s1, s2;   // element (i0,i1,i2) of the box at off + i0 s0 + i1 s1 + i2 s2
};

__global__ void k_copy(int64_t n, const double *__restrict__ a, double *__restrict__ b) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += gridDim.x * (int64_t)blockDim.x) b[i] = a[i];
}

// partial sums of w_A e^{U_A} and w_A with w_A = prod_d (integral of B_{i_d}) (a lumped mass)
__global__ void __launch_bounds__(256) k_fdm_shift_partial(DevProblem pb, FdmData f, const double *__restrict__ U,
                                                           double *__restrict__ part) {
  __shared__ double sh[2][8];
  double s1 = 0, s2 = 0;
  for (int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; A < pb.N; A += gridDim.x * (int64_t)blockDim.x) {
    const int i0 = (int)(A % pb.n[0]);
    const int64_t r = A / pb.n[0];
    const int i1 = (int)(r % pb.n[1]), i2 = (int)(r / pb.n[1]);
    double w = f.rs[0][i0] * f.rs[1][i1];
    if (pb.dim == 3) w *= f.rs[2][i2];
    s1 += w * exp(U[A]);
    s2 += w;
  }
  for (int o = 32; o > 0; o >>= 1) {
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = s1;
    sh[1][threadIdx.x >> 6] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      a += sh[0][i];
      b += sh[1][i];
    }
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// shift = max(-lambda mscale sum1 / sum2, -0.9 mu_min): K + shift M stays positive definite
__global__ void k_fdm_shift_final(const double *__restrict__ part, int nb, double lam, double mscale, double mu_min,
                                  double add, double *__restrict__ shift) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0, b = 0;
  for (int i = 0; i < nb; ++i) {
    a += part[2 * i];
    b += part[2 * i + 1];
  }
  double c = ((b > 0) ? -lam * mscale * a / b : 0.0) + add;
  *shift = fmax(c, -0.9 * mu_min);
}

template <int AX>
void launch_gemm_axis(Handle &h, const double *in, BoxView vi, double *out, BoxView vo, const double *T, const int *m,
                      const double *mu0, const double *mu1, const double *mu2, const double *shift, ChScale chs);

template <int AX>
void launch_axis(Handle &h, const double *in, BoxView vi, double *out, BoxView vo, const double *T, const int *m,
                 const double *mu0, const double *mu1, const double *mu2, const double *shift) {
  launch_gemm_axis<AX>(h, in, vi, out, vo, T, m, mu0, mu1, mu2, shift, ChScale{});
}

// One dense 1D transform along axis AX of the box m0 x m1 x m2 (element (i0, i1, i2) of a view at
// off + i0 s0 + i1 s1 + i2 s2) as a register-tiled product Y = T X (T: m x m row-major; X: the box with
// axis AX as the reduction index and the other two axes as columns).  A workgroup owns 16 R rows x
// 16 R columns (R = 8 for large boxes, 4 or 2 where larger tiles would leave the chip idle); per
// (64 / R)-deep step the T and X tiles are staged in LDS (each with its contiguous direction on
// consecutive lanes) and every lane accumulates an R x R block (2 R LDS reads per R^2 multiply-adds).
// The result is divided by the Cahn-Hilliard eigenvalue when chs.eta0 is set, else by
// mu0[i0] + mu1[i1] + mu2[i2] + shift when mu0 is set (the scaling of the third forward transform).

template <int AX>
__device__ inline void box_coords(int r, int64_t c, int m0, int m1, int &i0, int &i1, int &i2) {
  if (AX == 0) { i0 = r; i1 = (int)(c % m1); i2 = (int)(c / m1); }
  else if (AX == 1) { i0 = (int)(c % m0); i1 = r; i2 = (int)(c / m0); }
  else { i0 = (int)(c % m0); i1 = (int)(c / m0); i2 = r; }
}

template <int AX, int kGR>
__global__ void __launch_bounds__(256) k_fdm_gemm(const double *__restrict__ in, BoxView vi, double *__restrict__ out,
                                                  BoxView vo, const double *__restrict__ T, int m0, int m1, int m2,
                                                  const double *__restrict__ mu0, const double *__restrict__ mu1,
                                                  const double *__restrict__ mu2, const double *__restrict__ shift,
                                                  ChScale chs) {
  constexpr int kGM = 16 * kGR, kGN = 16 * kGR, kGK = 64 / kGR;   // 1024 entries per staged tile
  __shared__ __align__(16) double Ts[kGK][kGM + 2], Xs[kGK][kGN + 2];
  const int m = AX == 0 ? m0 : (AX == 1 ? m1 : m2);
  const int64_t ncol = AX == 0 ? (int64_t)m1 * m2 : (AX == 1 ? (int64_t)m0 * m2 : (int64_t)m0 * m1);
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15;
  const int nbr = (m + kGM - 1) / kGM;
  const int r0 = (blockIdx.x % nbr) * kGM;
  const int64_t c0 = (int64_t)(blockIdx.x / nbr) * kGN;
  double acc[kGR][kGR];
#pragma unroll
  for (int i = 0; i < kGR; ++i)
#pragma unroll
    for (int j = 0; j < kGR; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < m; k0 += kGK) {
    // T tile: kGK consecutive k per row on consecutive lanes
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = t % kGK, row = t / kGK + (256 / kGK) * j, gr = r0 + row, gk = k0 + k;
      Ts[k][row] = (gr < m && gk < m) ? T[(int64_t)gr * m + gk] : 0.0;
    }
    // X tile: consecutive lanes on the contiguous direction (k for axis 0, columns otherwise)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int k, col;
      if (AX == 0) {
        k = t % kGK;
        col = t / kGK + (256 / kGK) * j;
      } else {
        k = t / kGN + (256 / kGN) * j;
        col = t % kGN;
      }
      const int gk = k0 + k;
      const int64_t gc = c0 + col;
      double v = 0.0;
      if (gk < m && gc < ncol) {
        int i0, i1, i2;
        box_coords<AX>(gk, gc, m0, m1, i0, i1, i2);
        v = in[vi.off + i0 * vi.s0 + i1 * vi.s1 + i2 * vi.s2];
      }
      Xs[k][col] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGK; ++k) {
      double a[kGR], b[kGR];
#pragma unroll
      for (int i = 0; i < kGR; ++i) {
        a[i] = Ts[k][tr * kGR + i];
        b[i] = Xs[k][tc * kGR + i];
      }
#pragma unroll
      for (int i = 0; i < kGR; ++i)
#pragma unroll
        for (int j = 0; j < kGR; ++j) acc[i][j] += a[i] * b[j];
    }
    __syncthreads();
  }
  const double c_shift = (mu0 && shift) ? *shift : 0.0;
#pragma unroll
  for (int i = 0; i < kGR; ++i) {
    const int gr = r0 + tr * kGR + i;
    if (gr >= m) continue;
#pragma unroll
    for (int j = 0; j < kGR; ++j) {
      const int64_t gc = c0 + tc * kGR + j;
      if (gc >= ncol) continue;
      int i0, i1, i2;
      box_coords<AX>(gr, gc, m0, m1, i0, i1, i2);
      double v = acc[i][j];
      if (chs.eta0) {
        const double a0 = mu0[i0], a1 = mu1[i1], a2 = mu2[i2];
        const double lam = chs.am + chs.sa * (a0 + a1 + a2) +
                           chs.sb * (chs.eta0[i0] + chs.eta1[i1] + chs.eta2[i2] + 2.0 * (a0 * a1 + a0 * a2 + a1 * a2));
        v /= fmax(lam, 0.05 * chs.am);
      } else if (mu0) {
        v /= mu0[i0] + mu1[i1] + (mu2 ? mu2[i2] : 0.0) + c_shift;
      }
      out[vo.off + i0 * vo.s0 + i1 * vo.s1 + i2 * vo.s2] = v;
    }
  }
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// The same transform on the FP64 matrix cores (v_mfma_f64_16x16x4f64; lane l holds A[l % 16][l / 16],
// B[l / 16][l % 16] and receives D[l / 16 + 4 r][l % 16], r = 0..3, checked by an in-bounds probe).  A workgroup owns 128 rows x 64
// columns, each of its four waves 32 rows as 2 x 4 products of 16 x 16 tiles (32 accumulators per lane;
// 64 held the epilogue's copies in VGPRs as well and left one wave per SIMD); per 16-deep step the T and
// X tiles are staged in LDS with the reduction index fastest (row stride 17 doubles), so a wave reads 6
// operands per 8 products and the vector units only move data.  The next step's tiles are loaded into
// registers while the current step's products run: without that, every step waited for its own loads
// and the kernel ran no faster than the vector one.
template <int AX>
__global__ void __launch_bounds__(256) k_fdm_mfma(const double *__restrict__ in, BoxView vi, double *__restrict__ out,
                                                  BoxView vo, const double *__restrict__ T, int m0, int m1, int m2,
                                                  const double *__restrict__ mu0, const double *__restrict__ mu1,
                                                  const double *__restrict__ mu2, const double *__restrict__ shift,
                                                  ChScale chs) {
  constexpr int kM = 128, kN = 64, kK = 16, kS = kK + 1;
  __shared__ double Ts[kM * kS], Xs[kN * kS];   // [row][k], [column][k]
  const int m = AX == 0 ? m0 : (AX == 1 ? m1 : m2);
  const int64_t ncol = AX == 0 ? (int64_t)m1 * m2 : (AX == 1 ? (int64_t)m0 * m2 : (int64_t)m0 * m1);
  const int t = threadIdx.x, lane = t & 63, wr = t >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int nbr = (m + kM - 1) / kM;
  const int r0 = (blockIdx.x % nbr) * kM;
  const int64_t c0 = (int64_t)(blockIdx.x / nbr) * kN;
  const int64_t sin = AX == 0 ? vi.s0 : (AX == 1 ? vi.s1 : vi.s2), sout = AX == 0 ? vo.s0 : (AX == 1 ? vo.s1 : vo.s2);
  // the part of a column's address that does not depend on the reduction index (-1: past the box)
  auto col_part = [&](int64_t gc, const BoxView &v) -> int64_t {
    if (gc >= ncol) return -1;
    int i0, i1, i2;
    box_coords<AX>(0, gc, m0, m1, i0, i1, i2);
    return v.off + i0 * v.s0 + i1 * v.s1 + i2 * v.s2;
  };
  // X tile: consecutive lanes on the contiguous direction (k for axis 0: four columns per lane; the
  // columns otherwise: one column per lane, four k)
  constexpr int NXC = AX == 0 ? 4 : 1;
  int64_t xc[NXC];
#pragma unroll
  for (int j = 0; j < NXC; ++j) xc[j] = col_part(c0 + (AX == 0 ? (t >> 4) + 16 * j : (t & 63)), vi);
  f64x4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  // the tiles of step k0 are loaded into registers one step ahead (in flight while the previous step's
  // products run): T 16 consecutive k of a row on consecutive lanes; X as described above
  double tp[8], xp[4];
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = t & 15, gr = r0 + (t >> 4) + 16 * j, gk = k0 + k;
      tp[j] = (gr < m && gk < m) ? T[(int64_t)gr * m + gk] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = AX == 0 ? (t & 15) : (t >> 6) + 4 * j;
      const int64_t base = xc[AX == 0 ? j : 0];
      const int gk = k0 + k;
      xp[j] = (gk < m && base >= 0) ? in[base + gk * sin] : 0.0;
    }
  };
  load_tiles(0);
  for (int k0 = 0; k0 < m; k0 += kK) {
#pragma unroll
    for (int j = 0; j < 8; ++j) Ts[((t >> 4) + 16 * j) * kS + (t & 15)] = tp[j];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = AX == 0 ? (t & 15) : (t >> 6) + 4 * j, col = AX == 0 ? (t >> 4) + 16 * j : (t & 63);
      Xs[col * kS + k] = xp[j];
    }
    __syncthreads();
    if (k0 + kK < m) load_tiles(k0 + kK);
#pragma unroll
    for (int kk = 0; kk < kK; kk += 4) {
      double a[2], b[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = Ts[(wr * 32 + i * 16 + lr) * kS + kk + lk];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Xs[(j * 16 + lr) * kS + kk + lk];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  const double c_shift = (mu0 && shift) ? *shift : 0.0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t gc = c0 + j * 16 + lr, oc = col_part(gc, vo);
    if (oc < 0) continue;
    int c0i, c1i, c2i;
    box_coords<AX>(0, gc, m0, m1, c0i, c1i, c2i);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = r0 + wr * 32 + i * 16 + lk + 4 * r;
        if (gr >= m) continue;
        const int i0 = AX == 0 ? gr : c0i, i1 = AX == 1 ? gr : c1i, i2 = AX == 2 ? gr : c2i;
        double v = acc[i][j][r];
        if (chs.eta0) {
          const double a0 = mu0[i0], a1 = mu1[i1], a2 = mu2[i2];
          const double lam = chs.am + chs.sa * (a0 + a1 + a2) +
                             chs.sb * (chs.eta0[i0] + chs.eta1[i1] + chs.eta2[i2] + 2.0 * (a0 * a1 + a0 * a2 + a1 * a2));
          v /= fmax(lam, 0.05 * chs.am);
        } else if (mu0) {
          v /= mu0[i0] + mu1[i1] + (mu2 ? mu2[i2] : 0.0) + c_shift;
        }
        out[oc + gr * sout] = v;
      }
  }
}

template <int AX>
void launch_gemm_axis(Handle &h, const double *in, BoxView vi, double *out, BoxView vo, const double *T, const int *m,
                      const double *mu0, const double *mu1, const double *mu2, const double *shift, ChScale chs) {
  const int mm = m[AX];
  const int64_t ncol = AX == 0 ? (int64_t)m[1] * m[2] : (AX == 1 ? (int64_t)m[0] * m[2] : (int64_t)m[0] * m[1]);
  // the largest per-lane block that still gives at least 1024 workgroups (4 per CU); the matrix cores
  // take boxes whose 128 x 64 tiles reach that count too (IGA_OPT_FDM_KERNEL forces either kernel)
  auto blocks = [&](int R) { return (int64_t)((mm + 16 * R - 1) / (16 * R)) * ((ncol + 16 * R - 1) / (16 * R)); };
  const int64_t mblocks = (int64_t)((mm + 127) / 128) * ((ncol + 63) / 64);
  if (h.fdm_kernel == 2 || (h.fdm_kernel == 0 && mblocks >= 1024)) {
    hipLaunchKernelGGL((k_fdm_mfma<AX>), dim3((unsigned)mblocks), dim3(256), 0, h.stream, in, vi, out, vo, T, m[0],
                       m[1], m[2], mu0, mu1, mu2, shift, chs);
    return;
  }
  const int R = blocks(8) >= 1024 ? 8 : (blocks(4) >= 1024 ? 4 : 2);
  const unsigned nb = (unsigned)blocks(R);
  if (R == 8)
    hipLaunchKernelGGL((k_fdm_gemm<AX, 8>), dim3(nb), dim3(256), 0, h.stream, in, vi, out, vo, T, m[0], m[1], m[2], mu0,
                       mu1, mu2, shift, chs);
  else if (R == 4)
    hipLaunchKernelGGL((k_fdm_gemm<AX, 4>), dim3(nb), dim3(256), 0, h.stream, in, vi, out, vo, T, m[0], m[1], m[2], mu0,
                       mu1, mu2, shift, chs);
  else
    hipLaunchKernelGGL((k_fdm_gemm<AX, 2>), dim3(nb), dim3(256), 0, h.stream, in, vi, out, vo, T, m[0], m[1], m[2], mu0,
                       mu1, mu2, shift, chs);
}

template <int AX>
void launch_ch_axis(Handle &h, const double *in, double *out, const double *T, const int *m, const double *const *mu,
                    ChScale chs) {
  const BoxView box{0, 1, m[0], (int64_t)m[0] * m[1]};
  launch_gemm_axis<AX>(h, in, box, out, box, T, m, mu ? mu[0] : nullptr, mu ? mu[1] : nullptr, mu ? mu[2] : nullptr,
                       nullptr, chs);
}

}  // namespace

// Cahn-Hilliard fast diagonalisation: every axis periodic, x = xi without weights, at most kFdmMax
// functions per axis, and the second-derivative matrix diagonal in the (A, M) eigenbasis (uniform
// knots); otherwise chfdm_ok stays 0 and the Krylov solve runs without a preconditioner.  In 2D
// the third axis has one function with mu = eta = 0.
iga_status ensure_chfdm(Handle &h) {
  if (h.chfdm_tried) return IGA_OK;
  h.chfdm_tried = 1;
  const DevProblem &pb = h.pb;
  if (pb.dim < 2 || pb.ctrl || pb.wts) return IGA_OK;
  const int p = pb.p, W = 2 * p + 1;
  if (pb.dim == 2) {
    const double zero = 0.0;
    double *dz;
    iga_status st;
    if ((st = upload_owned(h, &dz, &zero, 1))) return st;
    h.ch_mu[2] = h.ch_eta[2] = dz;
  }
  for (int d = 0; d < pb.dim; ++d) {
    const int n = pb.n[d];
    if (!pb.ax[d].nper || n > kFdmMax || h.hsepH[d].empty()) return IGA_OK;
    std::vector<double> A((size_t)n * n, 0.0), M((size_t)n * n, 0.0), H((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int o = 0; o < W; ++o) {
        const int j = ((i + o - p) % n + n) % n;
        A[(size_t)i * n + j] += h.hsepA[d][(size_t)i * W + o];
        M[(size_t)i * n + j] += h.hsepM[d][(size_t)i * W + o];
        H[(size_t)i * n + j] += h.hsepH[d][(size_t)i * W + o];
      }
    int same = -1;
    for (int e = 0; e < d && same < 0; ++e)
      if (pb.n[e] == n && h.hsepM[e] == h.hsepM[d] && h.hsepA[e] == h.hsepA[d] && h.hsepH[e] == h.hsepH[d]) same = e;
    if (same >= 0) {
      h.ch_Tf[d] = h.ch_Tf[same];
      h.ch_Tb[d] = h.ch_Tb[same];
      h.ch_mu[d] = h.ch_mu[same];
      h.ch_eta[d] = h.ch_eta[same];
      continue;
    }
    std::vector<double> V, mu;
    if (!gen_eigen(A, M, n, V, mu)) return IGA_OK;
    // eta = diag(V^T H V); the off-diagonal part must vanish (relative to the largest eta)
    std::vector<double> HV((size_t)n * n, 0.0), eta(n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        const double hik = H[(size_t)i * n + k];
        if (hik == 0.0) continue;
        for (int c = 0; c < n; ++c) HV[(size_t)i * n + c] += hik * V[(size_t)k * n + c];
      }
    double emax = 0, off = 0;
    for (int a = 0; a < n; ++a)
      for (int c = 0; c < n; ++c) {
        double s = 0;
        for (int i = 0; i < n; ++i) s += V[(size_t)i * n + a] * HV[(size_t)i * n + c];
        if (a == c) { eta[a] = s; emax = fmax(emax, fabs(s)); }
        else off = fmax(off, fabs(s));
      }
    if (!(off <= 1e-8 * emax)) return IGA_OK;
    std::vector<double> Tf((size_t)n * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) Tf[(size_t)i * n + k] = V[(size_t)k * n + i];
    double *dTf, *dTb, *dmu, *deta;
    iga_status st;
    if ((st = upload_owned(h, &dTf, Tf.data(), Tf.size())) || (st = upload_owned(h, &dTb, V.data(), V.size())) ||
        (st = upload_owned(h, &dmu, mu.data(), mu.size())) || (st = upload_owned(h, &deta, eta.data(), eta.size())))
      return st;
    h.ch_Tf[d] = dTf;
    h.ch_Tb[d] = dTb;
    h.ch_mu[d] = dmu;
    h.ch_eta[d] = deta;
  }
  h.chfdm_ok = 1;
  return IGA_OK;
}

iga_status launch_chfdm_apply(Handle &h, const double *r, double *z, double *w1, double *w2, double am, double sa,
                              double sb) {
  const int m[3] = {h.pb.n[0], h.pb.n[1], h.pb.n[2]};
  const ChScale none{};
  const ChScale chs{h.ch_eta[0], h.ch_eta[1], h.ch_eta[2], am, sa, sb};
  if (h.pb.dim == 2) {
    launch_ch_axis<0>(h, r, w1, h.ch_Tf[0], m, nullptr, none);
    launch_ch_axis<1>(h, w1, w2, h.ch_Tf[1], m, h.ch_mu, chs);
    launch_ch_axis<1>(h, w2, w1, h.ch_Tb[1], m, nullptr, none);
    launch_ch_axis<0>(h, w1, z, h.ch_Tb[0], m, nullptr, none);
    IGA_HIP_CHECK(hipGetLastError());
    return IGA_OK;
  }
  launch_ch_axis<0>(h, r, w1, h.ch_Tf[0], m, nullptr, none);
  launch_ch_axis<1>(h, w1, w2, h.ch_Tf[1], m, nullptr, none);
  launch_ch_axis<2>(h, w2, w1, h.ch_Tf[2], m, h.ch_mu, chs);
  launch_ch_axis<2>(h, w1, w2, h.ch_Tb[2], m, nullptr, none);
  launch_ch_axis<1>(h, w2, w1, h.ch_Tb[1], m, nullptr, none);
  launch_ch_axis<0>(h, w1, z, h.ch_Tb[0], m, nullptr, none);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_fdm_shift(Handle &h, const double *U, double mass_coef) {
  const int nb = 256;
  hipLaunchKernelGGL(k_fdm_shift_partial, dim3(nb), dim3(256), 0, h.stream, h.pb, h.fdm, U, h.fdm_part);
  hipLaunchKernelGGL(k_fdm_shift_final, dim3(1), dim3(64), 0, h.stream, (const double *)h.fdm_part, nb, h.pb.lambda,
                     h.fdm.mscale, h.fdm.mu_min, h.fdm.mscale * mass_coef, h.fdm_shift);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// z = (K + shift M)^{-1} r on the non-Dirichlet coefficients, z = r on the Dirichlet ones.
// w1, w2: scratch of m0 m1 m2 doubles each.
iga_status launch_fdm_apply(Handle &h, const double *r, double *z, double *w1, double *w2) {
  const FdmData &f = h.fdm;
  const int dim = h.pb.dim;
  const int64_t n0 = h.pb.n[0], n1 = h.pb.n[1];
  const int *m = f.m;
  const BoxView full{f.lo[0] + n0 * (f.lo[1] + n1 * (int64_t)f.lo[2]), 1, n0, n0 * n1};
  const BoxView box{0, 1, m[0], (int64_t)m[0] * m[1]};
  const int64_t N = h.pb.N;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)((N + 255) / 256 < 2048 ? (N + 255) / 256 : 2048)), dim3(256), 0, h.stream,
                     N, r, z);
  const double *mu2 = dim == 3 ? f.mu[2] : nullptr;
  if (dim == 3) {
    launch_axis<0>(h, r, full, w1, box, f.Tf[0], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<1>(h, w1, box, w2, box, f.Tf[1], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<2>(h, w2, box, w1, box, f.Tf[2], m, f.mu[0], f.mu[1], mu2, h.fdm_shift);
    launch_axis<2>(h, w1, box, w2, box, f.Tb[2], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<1>(h, w2, box, w1, box, f.Tb[1], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<0>(h, w1, box, z, full, f.Tb[0], m, nullptr, nullptr, nullptr, nullptr);
  } else {
    launch_axis<0>(h, r, full, w1, box, f.Tf[0], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<1>(h, w1, box, w2, box, f.Tf[1], m, f.mu[0], f.mu[1], nullptr, h.fdm_shift);
    launch_axis<1>(h, w2, box, w1, box, f.Tb[1], m, nullptr, nullptr, nullptr, nullptr);
    launch_axis<0>(h, w1, box, z, full, f.Tb[0], m, nullptr, nullptr, nullptr, nullptr);
  }
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

}  // namespace iga
