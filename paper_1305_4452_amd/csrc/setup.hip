// Problem set-up: validation, Gauss-Legendre rule, 1D B-spline tables at the Gauss points of
// every element, the Algorithm 2 adjacency pattern and the per-point geometry table.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "iga_impl.h"

namespace iga {

// ------------------------------------------------------------------------------------------
// Gauss-Legendre nodes/weights on [-1,1] (Sec. 2.9 uses tensor Gauss-Legendre rules):
// Newton's method on P_n in extended precision, started from Tricomi's asymptotic estimate.
// ------------------------------------------------------------------------------------------
static void gauss_legendre(int n, double *x, double *w) {
  for (int k = 1; k <= n; ++k) {
    long double th = M_PI * (4.0L * k - 1.0L) / (4.0L * n + 2.0L);
    long double z = (1.0L - (n - 1.0L) / (8.0L * n * n * n)) * cosl(th);
    long double dp = 1.0L;
    for (int it = 0; it < 60; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int j = 2; j <= n; ++j) {
        long double p2 = ((2.0L * j - 1.0L) * z * p1 - (j - 1.0L) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0L; }
      dp = n * (p0 - z * p1) / (1.0L - z * z);
      long double step = p1 / dp;
      z -= step;
      if (fabsl(step) < 1e-21L) break;
    }
    // k-th largest root
    x[n - k] = (double)z;
    w[n - k] = (double)(2.0L / ((1.0L - z * z) * dp * dp));
  }
  if (n % 2) x[n / 2] = 0.0;
  for (int k = 0; k < n / 2; ++k) {   // enforce exact symmetry
    double a = 0.5 * (x[n - 1 - k] - x[k]);
    x[k] = -a;
    x[n - 1 - k] = a;
    double ww = 0.5 * (w[k] + w[n - 1 - k]);
    w[k] = w[n - 1 - k] = ww;
  }
}

// Values of the q+1 B-splines of degree q that are non-zero in span s (functions s-q..s),
// built up degree by degree: each degree-(k-1) function i feeds the left term of function i
// and the right term of function i-1, which share the denominator xi_{i+k} - xi_i.
static void nonzero_basis(const double *U, int s, int q, double xi, double *N) {
  double tmp[kMaxP + 1];
  N[0] = 1.0;
  for (int k = 1; k <= q; ++k) {
    double prev = 0.0;
    for (int j = 0; j < k; ++j) {
      int i = s - k + 1 + j;
      double t = N[j] / (U[i + k] - U[i]);
      tmp[j] = prev + (U[i + k] - xi) * t;
      prev = (xi - U[i]) * t;
    }
    tmp[k] = prev;
    for (int j = 0; j <= k; ++j) N[j] = tmp[j];
  }
}

// Values and first derivatives of the p+1 non-zero functions at xi in span s.
static void basis_and_derivative(const double *U, int s, int p, double xi, double *N, double *dN) {
  double low[kMaxP + 1];
  nonzero_basis(U, s, p - 1, xi, low);          // degree p-1: functions s-p+1..s
  nonzero_basis(U, s, p, xi, N);
  for (int j = 0; j <= p; ++j) {
    int m = s - p + j;
    double d = 0.0;
    if (j >= 1) d += low[j - 1] / (U[m + p] - U[m]);
    if (j <= p - 1) d -= low[j] / (U[m + p + 1] - U[m + 1]);
    dN[j] = p * d;
  }
}

// Second derivatives of the p+1 non-zero functions on span s: the derivative formula applied to
// the first derivatives of the degree p-1 functions (zero for p = 1).
static void basis_second_derivative(const double *U, int s, int p, double xi, double *d2N) {
  double low[kMaxP + 1] = {0}, dlow[kMaxP + 1] = {0};
  if (p >= 2) basis_and_derivative(U, s, p - 1, xi, low, dlow);
  for (int j = 0; j <= p; ++j) {
    int m = s - p + j;
    double d = 0.0;
    if (p >= 2) {
      if (j >= 1) d += dlow[j - 1] / (U[m + p] - U[m]);
      if (j <= p - 1) d -= dlow[j] / (U[m + p + 1] - U[m + 1]);
    }
    d2N[j] = p * d;
  }
}

// third derivatives of the p+1 functions of span s: the derivative formula of Sec. 2.1 applied to the
// second derivatives of the degree p-1 functions
static void basis_third_derivative(const double *U, int s, int p, double xi, double *d3N) {
  double low[kMaxP + 1] = {0};
  if (p >= 3) basis_second_derivative(U, s, p - 1, xi, low);
  for (int j = 0; j <= p; ++j) {
    int m = s - p + j;
    double d = 0.0;
    if (p >= 3) {
      if (j >= 1) d += low[j - 1] / (U[m + p] - U[m]);
      if (j <= p - 1) d -= low[j] / (U[m + p + 1] - U[m + 1]);
    }
    d3N[j] = p * d;
  }
}

// ------------------------------------------------------------------------------------------
// Device kernels used once at creation
// ------------------------------------------------------------------------------------------

// One thread per row: columns are the tensor product of the per-axis stencil ranges.
__global__ void k_pattern(DevProblem pb, int32_t *col_idx) {
  int64_t A = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (A >= pb.N) return;
  int i0 = (int)(A % pb.n[0]);
  int64_t r = A / pb.n[0];
  int i1 = (int)(r % pb.n[1]);
  int i2 = (int)(r / pb.n[1]);
  const int W = 2 * pb.p + 1;
  int l0 = pb.ax[0].stl[i0], w0 = pb.ax[0].stw[i0];
  int l1 = pb.ax[1].stl[i1], w1 = pb.ax[1].stw[i1];
  int l2 = 0, w2 = 1;
  if (pb.dim == 3) { l2 = pb.ax[2].stl[i2]; w2 = pb.ax[2].stw[i2]; }
  // column b of row i along an axis: l + b, or the b-th entry of a periodic axis' sorted list
  auto col = [&](int d, int i, int l, int b) { return pb.ax[d].nper ? pb.ax[d].nbr[(size_t)i * W + b] : l + b; };
  int64_t pos = pb.row_ptr[A];
  for (int b2 = 0; b2 < w2; ++b2)
    for (int b1 = 0; b1 < w1; ++b1)
      for (int b0 = 0; b0 < w0; ++b0)
        col_idx[pos++] = (int32_t)(col(0, i0, l0, b0) +
                                   (int64_t)pb.n[0] * (col(1, i1, l1, b1) + (int64_t)pb.n[1] * (pb.dim == 3 ? col(2, i2, l2, b2) : 0)));
}

// Geometry table, one thread per (element, quadrature point); naive sums over the element's
// functions (runs once).  Homogeneous coordinates: w = sum w_A M_A, X~ = sum w_A x_A M_A, so
// x = X~/w and dx/dxi = (dX~ - x dw)/w (eq:rational, eq:drational applied to the geometry map
// of App. A); D = kappa W Jinv Jinv^T with Jinv from eq:identity.
__global__ void k_geometry(DevProblem pb, const double *__restrict__ ctrl, const double *__restrict__ wts,
                           const double *__restrict__ kap_nodal, double *__restrict__ geo, int *bad) {
  const int dim = pb.dim, P = pb.P, Q = pb.Q;
  const int QD = dim == 3 ? Q * Q * Q : Q * Q;
  int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= pb.E * QD) return;
  int64_t e = gid / QD;
  int q = (int)(gid % QD);
  int em[3], qm[3] = {q % Q, (q / Q) % Q, dim == 3 ? q / (Q * Q) : 0};
  em[0] = (int)(e % pb.ne[0]);
  em[1] = (int)((e / pb.ne[0]) % pb.ne[1]);
  em[2] = dim == 3 ? (int)(e / ((int64_t)pb.ne[0] * pb.ne[1])) : 0;
  double w = 0, dw[3] = {0, 0, 0}, X[3] = {0, 0, 0}, dX[3][3] = {{0}}, kt = 0;
  double W = 1.0;
  for (int d = 0; d < dim; ++d) W *= pb.ax[d].wq[(size_t)em[d] * Q + qm[d]];
  const int P2 = dim == 3 ? P : 1;
  for (int a2 = 0; a2 < P2; ++a2)
    for (int a1 = 0; a1 < P; ++a1)
      for (int a0 = 0; a0 < P; ++a0) {
        int a[3] = {a0, a1, a2};
        double v = 1.0, g[3] = {1.0, 1.0, 1.0};
        int64_t A = 0, stride = 1;
        for (int d = 0; d < dim; ++d) {
          size_t o = ((size_t)em[d] * Q + qm[d]) * P + a[d];
          double b = pb.ax[d].B[o], db = pb.ax[d].dB[o];
          for (int k = 0; k < dim; ++k) g[k] *= (k == d) ? db : b;
          v *= b;
          A += stride * (pb.ax[d].efirst[em[d]] + a[d]);
          stride *= pb.n[d];
        }
        double wa = wts ? wts[A] : 1.0;
        w += wa * v;
        for (int k = 0; k < dim; ++k) dw[k] += wa * g[k];
        if (ctrl)
          for (int i = 0; i < dim; ++i) {
            double xa = ctrl[A * dim + i] * wa;
            X[i] += xa * v;
            for (int k = 0; k < dim; ++k) dX[i][k] += xa * g[k];
          }
        if (kap_nodal) kt += wa * kap_nodal[A] * v;
      }
  double J[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  if (ctrl)
    for (int i = 0; i < dim; ++i)
      for (int k = 0; k < dim; ++k) J[i][k] = (dX[i][k] - (X[i] / w) * dw[k]) / w;
  double det, Ji[3][3];
  if (dim == 2) {
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    Ji[0][0] = J[1][1] / det;  Ji[0][1] = -J[0][1] / det;
    Ji[1][0] = -J[1][0] / det; Ji[1][1] = J[0][0] / det;
  } else {
    double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    double id = 1.0 / det;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  if (!(det > 0.0)) atomicOr(bad, 1);
  W *= det;
  double kappa = 1.0;
  if (pb.kappa_mode == IGA_KAPPA_NODAL) kappa = kt / w;
  else if (pb.kappa_mode == IGA_KAPPA_ELEMENT) kappa = pb.kel[e];
  // Ji[alpha][i] = d xi_alpha / d x_i : D_ab = kappa W sum_i Ji[a][i] Ji[b][i]
  const int NG = geo_streams(dim);
  double *out = geo + (size_t)e * NG * QD + q;
  double s = kappa * W / (w * w);
  auto D = [&](int a, int b) {
    double r = 0.0;
    for (int i = 0; i < dim; ++i) r += Ji[a][i] * Ji[b][i];
    return s * r;
  };
  if (dim == 3) {
    out[0 * QD] = D(0, 0); out[1 * QD] = D(1, 1); out[2 * QD] = D(2, 2);
    out[3 * QD] = D(0, 1); out[4 * QD] = D(0, 2); out[5 * QD] = D(1, 2);
    out[6 * QD] = dw[0] / w; out[7 * QD] = dw[1] / w; out[8 * QD] = dw[2] / w;
    out[9 * QD] = W / w; out[10 * QD] = 1.0 / w;
  } else {
    out[0 * QD] = D(0, 0); out[1 * QD] = D(1, 1); out[2 * QD] = D(0, 1);
    out[3 * QD] = dw[0] / w; out[4 * QD] = dw[1] / w;
    out[5 * QD] = W / w; out[6 * QD] = 1.0 / w;
  }
}

iga_status launch_pattern(Handle &h) {
  int64_t N = h.pb.N;
  int blocks = (int)((N + 255) / 256);
  hipLaunchKernelGGL(k_pattern, dim3(blocks), dim3(256), 0, h.stream, h.pb, h.col_idx);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status launch_geometry(Handle &h, const double *ctrl, const double *wts, const double *kappa_nodal,
                           int *bad_det) {
  const int QD = ipow(h.pb.Q, h.pb.dim);
  int64_t tot = h.pb.E * QD;
  int blocks = (int)((tot + 255) / 256);
  hipLaunchKernelGGL(k_geometry, dim3(blocks), dim3(256), 0, h.stream, h.pb, ctrl, wts, kappa_nodal, h.geo,
                     bad_det);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

// ------------------------------------------------------------------------------------------
// Host-side creation
// ------------------------------------------------------------------------------------------
thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
iga_status fail(iga_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

template <typename T>
static iga_status dev_alloc(Handle &h, T **p, size_t count) {
  void *q = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(IGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  h.owned.push_back(q);
  *p = (T *)q;
  return IGA_OK;
}

template <typename T>
static iga_status dev_upload(Handle &h, T **p, const T *src, size_t count) {
  iga_status st = dev_alloc(h, p, count);
  if (st) return st;
  IGA_HIP_CHECK(hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, h.stream));
  return IGA_OK;
}

// Tables of the separable row-gather Jacobian (simple knots: element e carries functions e..e+p).
//  phi_d[i][o][k] = B_i(g) B_{i+o-p}(g) at the k-th Gauss point g of supp(B_i) (element i-p+k/Q,
//                   point k mod Q), zero where j = i+o-p is not a function or g is outside the mesh;
// and the axis-0 basis table [ne0][Q][P], both in FP64 and FP32; the prefix sums of the stencil widths (row pointers of the tensor-product pattern)
// and the per-point reaction-coefficient buffer.  Axes 1 and 2 are open; axis 0 may be periodic.
static iga_status build_separable_tables(Handle &h, const std::vector<double> *hostB, const std::vector<int> *stw) {
  const DevProblem &pb = h.pb;
  const int p = pb.p, P = pb.P, Q = pb.Q, W = 2 * p + 1, KM = P * Q;
  iga_status st;
  for (int a = 1; a < 3; ++a) {
    const int n = pb.n[a], ne = pb.ne[a];
    const std::vector<double> &B = hostB[a];
    std::vector<double> ph((size_t)n * W * KM, 0.0);
    for (int i = 0; i < n; ++i)
      for (int o = 0; o < W; ++o) {
        const int j = i + o - p;
        for (int k = 0; k < KM; ++k) {
          const int el = i - p + k / Q, q = k % Q, ia = i - el, ib = j - el;
          if (el < 0 || el >= ne || j < 0 || j >= n || ib < 0 || ib > p) continue;
          ph[((size_t)i * W + o) * KM + k] = B[((size_t)el * Q + q) * P + ia] * B[((size_t)el * Q + q) * P + ib];
        }
      }
    std::vector<float> phf(ph.begin(), ph.end());
    double *dd;
    float *df;
    if ((st = dev_upload(h, &dd, ph.data(), ph.size())) || (st = dev_upload(h, &df, phf.data(), phf.size())))
      return st;
    h.sep_phi[0][a] = dd;
    h.sep_phi[1][a] = df;
  }
  {
    std::vector<float> bf(hostB[0].begin(), hostB[0].end());
    double *dd;
    float *df;
    if ((st = dev_upload(h, &dd, hostB[0].data(), hostB[0].size())) || (st = dev_upload(h, &df, bf.data(), bf.size())))
      return st;
    h.sep_b0[0] = dd;
    h.sep_b0[1] = df;
  }
  {
    std::vector<int64_t> cw;
    for (int a = 0; a < 3; ++a) {
      int64_t c = 0;
      for (int i = 0; i < pb.n[a]; ++i) {
        cw.push_back(c);
        c += stw[a][i];
      }
      cw.push_back(c);
    }
    int64_t *dcw;
    if ((st = dev_upload(h, &dcw, cw.data(), cw.size()))) return st;
    h.sep_cw = dcw;
  }
  const size_t nqp = (size_t)pb.ne[0] * Q * pb.ne[1] * Q * pb.ne[2] * Q;
  double *mf;
  if ((st = dev_alloc(h, &mf, nqp))) return st;
  h.mfield = mf;
  return IGA_OK;
}

iga_status upload_owned(Handle &h, double **dst, const double *src, size_t count) {
  return dev_upload(h, dst, src, count);
}

iga_status create_impl(const iga_desc *d, void *stream, Handle **out) {
  if (!d || !out) return fail(IGA_EINVAL, "null descriptor or output");
  if (d->dim != 2 && d->dim != 3) return fail(IGA_EINVAL, "dim must be 2 or 3");
  const int dim = d->dim, p = d->degree[0];
  if (p < 1 || p > kMaxP - 1) return fail(IGA_EINVAL, "degree must be in 1..6");
  for (int a = 0; a < dim; ++a) {
    if (d->degree[a] < 1 || d->degree[a] > kMaxP - 1) return fail(IGA_EINVAL, "degree must be in 1..6");
    if (d->degree[a] != p) return fail(IGA_EUNSUPPORTED, "the GPU kernels need equal degrees on all axes");
    if (d->nquad[a] != 0 && d->nquad[a] != p + 1)
      return fail(IGA_EUNSUPPORTED, "the GPU kernels use p+1 Gauss points per axis");
    if (!d->knots[a] || d->nknots[a] < 2 * p + 2) return fail(IGA_EINVAL, "knot vector too short or NULL");
    const double *U = d->knots[a];
    int nk = d->nknots[a];
    for (int k = 0; k + 1 < nk; ++k)
      if (!(U[k] <= U[k + 1]) || !std::isfinite(U[k]) || !std::isfinite(U[k + 1]))
        return fail(IGA_EINVAL, "knot vector must be finite and non-decreasing");
    for (int k = 0; k < p; ++k)
      if (U[k] != U[k + 1] || U[nk - 1 - k] != U[nk - 2 - k])
        return fail(IGA_EINVAL, "knot vector must be open (p+1 equal end knots)");
    for (int k = p + 1; k + 1 < nk - p - 1; ++k) {
      int mult = 1;
      while (k + mult < nk - p - 1 && U[k + mult] == U[k]) ++mult;
      if (mult > p) return fail(IGA_EINVAL, "interior knot multiplicity must be <= p");
    }
  }
  bool any_periodic = false;
  for (int a = 0; a < dim; ++a) {
    const int pr = d->periodic[a];
    if (pr == 0) continue;
    any_periodic = true;
    if (pr < 1 || pr > p) return fail(IGA_EINVAL, "periodic[axis] must be 0 or k + 1 with 0 <= k <= p - 1");
    if ((d->dirichlet_mask >> (2 * a)) & 3u) return fail(IGA_EINVAL, "a periodic axis has no Dirichlet faces");
    if (d->nknots[a] - p - 2 - (pr - 1) < 2 * p + 1)
      return fail(IGA_EINVAL, "a periodic axis needs at least 2p+1 functions after wrapping");
  }
  for (int a = dim; a < 3; ++a)
    if (d->periodic[a] != 0) return fail(IGA_EINVAL, "periodic set on an axis beyond dim");
  if (any_periodic && (d->ctrl || d->weights || d->kappa_mode == IGA_KAPPA_NODAL))
    return fail(IGA_EUNSUPPORTED, "periodic axes need x = xi, no weights and kappa one or element-wise");
  if (d->kappa_mode < 0 || d->kappa_mode > 2) return fail(IGA_EINVAL, "bad kappa_mode");
  if (d->kappa_mode != IGA_KAPPA_ONE && !d->kappa) return fail(IGA_EINVAL, "kappa values missing");
  if (!std::isfinite(d->lambda)) return fail(IGA_EINVAL, "lambda must be finite");

  Handle *h = new Handle();
  h->stream = (hipStream_t)stream;
  if (hipGetDevice(&h->device) != hipSuccess) { delete h; return fail(IGA_EHIP, "hipGetDevice failed"); }
  // device address of the allocation-free Jacobian's scratch array, looked up once per device
  if (iga_status sst = noalloc_scratch_init(h->device)) { delete h; return sst; }
  DevProblem &pb = h->pb;
  pb.dim = dim;
  pb.p = p;
  pb.P = p + 1;
  pb.Q = p + 1;
  pb.lambda = d->lambda;
  pb.dmask = d->dirichlet_mask & ((1u << (2 * dim)) - 1u);
  pb.kappa_mode = d->kappa_mode;
  pb.N = 1;
  pb.E = 1;
  pb.simple_knots = 1;
  iga_status st = IGA_OK;
  double gx[kMaxP], gw[kMaxP];
  gauss_legendre(pb.Q, gx, gw);
  std::vector<int> stl[3], stw[3];
  std::vector<double> hostB[3], hostSM[3], hostSA[3], hostSH[3];
  std::vector<int> nbr[3];
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) { pb.n[a] = 1; pb.ne[a] = 1; continue; }
    int nk = d->nknots[a];
    h->hknots[a].assign(d->knots[a], d->knots[a] + nk);
    const int kper = d->periodic[a] - 1;   // -1: open axis
    if (kper >= 0) {
      // unclamp for C^k across the seam (eq:unclamp-left / eq:unclamp-right); the domain
      // [U_p, U_{n+1}] and its spans are unchanged, only the end knots move
      std::vector<double> &K = h->hknots[a];
      const int nl = nk - p - 2, m = nk - 1;   // index of the last function, of the last knot
      for (int i = 0; i <= kper; ++i) K[kper - i] = K[p] - K[nl + 1] + K[nl - i];
      for (int i = 0; i <= kper; ++i) K[m - kper + i] = K[nl + 1] - K[p] + K[p + i + 1];
    }
    const double *U = h->hknots[a].data();
    int n = nk - p - 1;
    std::vector<int> efirst;
    std::vector<double> B, dB, d2B, d3B, wq;
    for (int s = p; s < n; ++s) {
      if (!(U[s] < U[s + 1])) continue;
      int e = (int)efirst.size();
      efirst.push_back(s - p);
      if (s - p != e) pb.simple_knots = 0;
      double lo = U[s], hi = U[s + 1];
      for (int q = 0; q < pb.Q; ++q) {
        double xi = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[q];
        double N[kMaxP], dN[kMaxP];
        double d2N[kMaxP], d3N[kMaxP];
        basis_and_derivative(U, s, p, xi, N, dN);
        basis_second_derivative(U, s, p, xi, d2N);
        basis_third_derivative(U, s, p, xi, d3N);
        for (int j = 0; j <= p; ++j) {
          B.push_back(N[j]);
          dB.push_back(dN[j]);
          d2B.push_back(d2N[j]);
          d3B.push_back(d3N[j]);
        }
        wq.push_back(gw[q] * 0.5 * (hi - lo));
      }
    }
    const int nopen = n;
    if (kper >= 0) n = nopen - 1 - kper;   // eq:map-wrap leaves n - k functions
    pb.n[a] = n;
    pb.ne[a] = (int)efirst.size();
    hostB[a] = B;
    const int W = 2 * p + 1;
    stl[a].resize(n);
    stw[a].resize(n);
    if (kper < 0) {
      // Algorithm 2 ranges: function j overlaps function i iff their open supports intersect
      for (int i = 0; i < n; ++i) {
        int l = i, r = i;
        while (l - 1 >= 0 && U[l - 1 + p + 1] > U[i]) --l;
        while (r + 1 < n && U[r + 1] < U[i + p + 1]) ++r;
        stl[a][i] = l;
        stw[a][i] = r - l + 1;
      }
    } else {
      // periodic axis: the wrapped functions sharing an element with i, sorted
      std::vector<std::vector<int>> sets(n);
      for (size_t e = 0; e < efirst.size(); ++e)
        for (int ia = 0; ia <= p; ++ia)
          for (int ib = 0; ib <= p; ++ib) sets[(efirst[e] + ia) % n].push_back((efirst[e] + ib) % n);
      nbr[a].assign((size_t)n * W, -1);
      for (int i = 0; i < n; ++i) {
        std::sort(sets[i].begin(), sets[i].end());
        sets[i].erase(std::unique(sets[i].begin(), sets[i].end()), sets[i].end());
        stl[a][i] = sets[i][0];
        stw[a][i] = (int)sets[i].size();
        for (size_t r = 0; r < sets[i].size(); ++r) nbr[a][(size_t)i * W + r] = sets[i][r];
      }
    }
    // 1D mass and stiffness in band storage (row i, offset o: column i + o - p, wrapped on a
    // periodic axis), used by the separable kernels and the fast-diagonalisation set-up
    const int P1 = p + 1;
    std::vector<double> sM((size_t)n * W, 0.0), sA((size_t)n * W, 0.0), sH((size_t)n * W, 0.0);
    std::vector<double> eM(efirst.size() * P1 * P1, 0.0), eA(efirst.size() * P1 * P1, 0.0);
    for (size_t e = 0; e < efirst.size(); ++e)
      for (int q = 0; q < pb.Q; ++q) {
        const double *Bq = &B[(e * pb.Q + q) * (p + 1)], *dBq = &dB[(e * pb.Q + q) * (p + 1)];
        const double *d2Bq = &d2B[(e * pb.Q + q) * (p + 1)];
        double wgt = wq[e * pb.Q + q];
        for (int ia = 0; ia <= p; ++ia)
          for (int ib = 0; ib <= p; ++ib) {
            size_t o = (size_t)((efirst[e] + ia) % n) * W + (ib - ia + p);
            const double m = wgt * Bq[ia] * Bq[ib], k = wgt * dBq[ia] * dBq[ib];
            sM[o] += m;
            sA[o] += k;
            sH[o] += wgt * d2Bq[ia] * d2Bq[ib];
            eM[(e * P1 + ia) * P1 + ib] += m;
            eA[(e * P1 + ia) * P1 + ib] += k;
          }
      }
    double *d_sM, *d_sA, *d_eM, *d_eA;
    if ((st = dev_upload(*h, &d_sM, sM.data(), sM.size())) || (st = dev_upload(*h, &d_sA, sA.data(), sA.size())) ||
        (st = dev_upload(*h, &d_eM, eM.data(), eM.size())) || (st = dev_upload(*h, &d_eA, eA.data(), eA.size()))) {
      iga_destroy((iga_t)h);
      return st;
    }
    pb.sepM[a] = d_sM;
    pb.sepA[a] = d_sA;
    pb.elM[a] = d_eM;
    pb.elA[a] = d_eA;
    hostSM[a] = sM;
    hostSA[a] = sA;
    hostSH[a] = sH;
    int *d_ef, *d_stl, *d_stw;
    double *d_B, *d_dB, *d_wq;
    if ((st = dev_upload(*h, &d_ef, efirst.data(), efirst.size())) ||
        (st = dev_upload(*h, &d_B, B.data(), B.size())) || (st = dev_upload(*h, &d_dB, dB.data(), dB.size())) ||
        (st = dev_upload(*h, &d_wq, wq.data(), wq.size())) ||
        (st = dev_upload(*h, &d_stl, stl[a].data(), (size_t)n)) ||
        (st = dev_upload(*h, &d_stw, stw[a].data(), (size_t)n))) {
      iga_destroy((iga_t)h);
      return st;
    }
    double *d_d2B, *d_d3B;
    if ((st = dev_upload(*h, &d_d2B, d2B.data(), d2B.size())) || (st = dev_upload(*h, &d_d3B, d3B.data(), d3B.size()))) {
      iga_destroy((iga_t)h);
      return st;
    }
    pb.ax[a] = AxisDev{d_B, d_dB, d_wq, d_ef, d_stl, d_stw, 0, nullptr, d_d2B, d_d3B};
    if (kper >= 0) {
      int *d_nbr;
      if ((st = dev_upload(*h, &d_nbr, nbr[a].data(), nbr[a].size()))) {
        iga_destroy((iga_t)h);
        return st;
      }
      pb.ax[a].nper = n;
      pb.ax[a].nbr = d_nbr;
      pb.periodic = 1;
    }
  }
  for (int a = 0; a < 3; ++a) { pb.N *= pb.n[a]; pb.E *= pb.ne[a]; }
  // row pointer: prefix sum of the stencil-width products
  std::vector<int64_t> rp((size_t)pb.N + 1);
  rp[0] = 0;
  for (int64_t A = 0; A < pb.N; ++A) {
    int i0 = (int)(A % pb.n[0]);
    int64_t r = A / pb.n[0];
    int i1 = (int)(r % pb.n[1]);
    int i2 = (int)(r / pb.n[1]);
    int64_t w = (int64_t)stw[0][i0] * stw[1][i1] * (dim == 3 ? stw[2][i2] : 1);
    rp[A + 1] = rp[A] + w;
  }
  pb.nnz = rp[pb.N];
  if (pb.nnz > INT32_MAX * 16LL) { iga_destroy((iga_t)h); return fail(IGA_EUNSUPPORTED, "pattern too large"); }
  if ((st = dev_upload(*h, &h->row_ptr, rp.data(), rp.size())) ||
      (st = dev_alloc(*h, &h->col_idx, (size_t)pb.nnz))) {
    iga_destroy((iga_t)h);
    return st;
  }
  pb.row_ptr = h->row_ptr;
  pb.col_idx = h->col_idx;
  if (d->weights)
    for (int64_t A = 0; A < pb.N; ++A)
      if (!(d->weights[A] > 0.0) || !std::isfinite(d->weights[A])) {
        iga_destroy((iga_t)h);
        return fail(IGA_EINVAL, "weights must be positive and finite");
      }
  pb.rational = d->weights != nullptr;
  pb.table = (d->ctrl != nullptr || d->weights != nullptr || d->kappa_mode == IGA_KAPPA_NODAL) ? 1 : 0;
  // x = xi and kappa one; a periodic axis only as axis 0 (the streaming axis of the separable row-gather)
  pb.separable = (!pb.table && d->kappa_mode == IGA_KAPPA_ONE && !pb.ax[1].nper && !pb.ax[2].nper) ? 1 : 0;
  if (pb.separable && pb.simple_knots && dim == 3 && pb.P >= 2 && pb.P <= 5 &&
      (st = build_separable_tables(*h, hostB, stw))) {
    iga_destroy((iga_t)h);
    return st;
  }
  for (int a = 0; a < dim; ++a) {
    h->hsepM[a] = hostSM[a];
    h->hsepA[a] = hostSA[a];
    h->hsepH[a] = hostSH[a];
  }
  double *d_w = nullptr, *d_ctrl = nullptr, *d_kn = nullptr, *d_kel = nullptr, *d_src = nullptr;
  if (d->weights && (st = dev_upload(*h, &d_w, d->weights, (size_t)pb.N))) { iga_destroy((iga_t)h); return st; }
  if (d->kappa_mode == IGA_KAPPA_ELEMENT && (st = dev_upload(*h, &d_kel, d->kappa, (size_t)pb.E))) {
    iga_destroy((iga_t)h);
    return st;
  }
  if (d->source && (st = dev_upload(*h, &d_src, d->source, (size_t)pb.N))) { iga_destroy((iga_t)h); return st; }
  pb.wts = d_w;
  pb.kel = d_kel;
  pb.src = d_src;
  if ((st = launch_pattern(*h))) { iga_destroy((iga_t)h); return st; }
  const int QD = ipow(pb.Q, dim);
  if ((st = dev_alloc(*h, &h->lin, (size_t)pb.E * QD))) { iga_destroy((iga_t)h); return st; }
  h->npartials = 4096;
  if ((st = dev_alloc(*h, &h->partials, (size_t)h->npartials * 4))) { iga_destroy((iga_t)h); return st; }
  if (pb.table) {
    if (d->ctrl && (st = dev_upload(*h, &d_ctrl, d->ctrl, (size_t)pb.N * dim))) { iga_destroy((iga_t)h); return st; }
    pb.ctrl = d_ctrl;
    if (d->kappa_mode == IGA_KAPPA_NODAL && (st = dev_upload(*h, &d_kn, d->kappa, (size_t)pb.N))) {
      iga_destroy((iga_t)h);
      return st;
    }
    if ((st = dev_alloc(*h, &h->geo, (size_t)pb.E * QD * geo_streams(dim)))) { iga_destroy((iga_t)h); return st; }
    pb.geo = h->geo;
    int *d_bad;
    if ((st = dev_alloc(*h, &d_bad, 1))) { iga_destroy((iga_t)h); return st; }
    hipMemsetAsync(d_bad, 0, sizeof(int), h->stream);
    if ((st = launch_geometry(*h, d_ctrl, d_w, d_kn, d_bad))) { iga_destroy((iga_t)h); return st; }
    int bad = 0;
    hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (hipStreamSynchronize(h->stream) != hipSuccess) { iga_destroy((iga_t)h); return fail(IGA_EHIP, "geometry"); }
    if (bad) { iga_destroy((iga_t)h); return fail(IGA_EINVAL, "det J <= 0 at a quadrature point"); }
  }
  if (hipStreamSynchronize(h->stream) != hipSuccess) { iga_destroy((iga_t)h); return fail(IGA_EHIP, "setup sync"); }
  *out = h;
  return IGA_OK;
}

}  // namespace iga

extern "C" const char *iga_last_error(void) { return iga::g_err.c_str(); }
