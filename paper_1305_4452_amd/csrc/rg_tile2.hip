// Tiled 2D kernels (single problem): the row-gather Jacobian, one workgroup per T0 x B1 tile of
// rows, and the residual, one workgroup per TE x TE tile of elements; the bodies are shared with
// the batched solver.
#include "kern_res2.h"
#include "kern_res3.h"
#include "kern_rgt2.h"

namespace iga {
namespace {

template <int P, typename OT>
__global__ void __launch_bounds__(rgt::kThreads) k_rgt2(DevProblem pb, const double *__restrict__ U,
                                                        OT *__restrict__ vals) {
  __shared__ __align__(16) char lds[rgt::Lds2<P, OT, OT>::total];
  rgt::rgt2_body<P, OT, OT>(pb, (int)blockIdx.x, U, vals, lds);
}

template <int P>
iga_status run_rgt2(Handle &h, const double *U, void *vals, int prec) {
  using S = rgt::Shape2<P>;
  const unsigned nb = (unsigned)(rgt::rgt2_tiles_0(h.pb.n[0], S::T0) * ((h.pb.n[1] + S::B1 - 1) / S::B1));
  kt_begin(h, "k_rgt2");
  if (prec == IGA_FP32)
    hipLaunchKernelGGL((k_rgt2<P, float>), dim3(nb), dim3(rgt::kThreads), 0, h.stream, h.pb, U, (float *)vals);
  else
    hipLaunchKernelGGL((k_rgt2<P, double>), dim3(nb), dim3(rgt::kThreads), 0, h.stream, h.pb, U, (double *)vals);
  kt_end(h);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P>
__global__ void __launch_bounds__(rst::kThreads) k_res2(DevProblem pb, const double *__restrict__ U,
                                                        double *__restrict__ R) {
  __shared__ double lds[rst::Res2<P>::total / sizeof(double)];
  rst::res2_body<P>(pb, (int)blockIdx.x, U, R, lds);
}

template <int P>
iga_status run_res2(Handle &h, const double *U, double *R) {
  const unsigned nb = (unsigned)rst::res2_tiles(h.pb.ne[0], h.pb.ne[1], rst::Res2<P>::TE);
  hipLaunchKernelGGL(k_res2<P>, dim3(nb), dim3(rst::kThreads), 0, h.stream, h.pb, U, R);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P, int OP>
__global__ void __launch_bounds__(rs3::kThreads) k_res3(DevProblem pb, const double *__restrict__ X,
                                                        const double *__restrict__ lin, double *__restrict__ Y) {
  __shared__ double lds[rs3::Res3<P>::total / sizeof(double)];
  rs3::res3_body<P, OP>(pb, (int)blockIdx.x, X, lin, Y, lds);
}

template <int P, int OP>
__global__ void __launch_bounds__(rs3::kThreads) k_res3r(DevProblem pb, const double *__restrict__ X,
                                                         const double *__restrict__ lin, double *__restrict__ Y) {
  constexpr int TEZ = rs3::Res3RDepth<P>::TEZ;
  __shared__ double lds[rs3::Res3R<P, TEZ>::total / sizeof(double)];
  rs3::res3r_body<P, TEZ, OP>(pb, (int)blockIdx.x, X, lin, Y, lds);
}

template <int P, int OP>
__global__ void __launch_bounds__(rs3::kThreads) k_res3s(DevProblem pb, const double *__restrict__ X,
                                                         const double *__restrict__ lin, double *__restrict__ Y, int zc) {
  __shared__ double lds[rs3::Res3S<P, 4>::total / sizeof(double)];
  rs3::res3s_body<P, 4, OP>(pb, (int)blockIdx.x, zc, X, lin, Y, lds);
}

// chunks of 4 elements per run along axis 2: the option value, else the longest run of at most 3 chunks
// that still leaves 512 workgroups.  Measured at 64^3 (p = 1, 2, 3) and 48^3 (p = 4), residual in us for
// runs of 1 / 2 / 3 / 4 chunks: p = 3 125.7 / 107.5 / 102.7 / 105.9, p = 4 129.5 / 109.8 / 103.1 / 108.8,
// p = 2 57.7 / 53.0 / 54.4 / 52.0, p = 1 25.0 / 22.6 / 28.3 / 29.9 (fixed-depth tiles: 143.1, 144.2,
// 54.0, 22.0).
int res3s_run_chunks(const Handle &h, int TEX) {
  const int nz = (h.pb.ne[2] + 3) / 4;
  if (h.res_zrun > 0) return std::max(1, std::min(std::min(h.res_zrun, rs3::kRes3sRunMax), nz));
  const int64_t nxy = (int64_t)((h.pb.ne[0] + TEX - 1) / TEX) * ((h.pb.ne[1] + TEX - 1) / TEX);
  int zc = std::min(3, nz);
  while (zc > 1 && nxy * ((nz + zc - 1) / zc) < 512) --zc;
  return zc;
}

template <int P>
iga_status run_res3(Handle &h, const double *X, double *Y, int op) {
  const unsigned nb = (unsigned)rs3::res3_tiles(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], rs3::Res3<P>::TE);
  if (h.tiled_3d == 1 && op != rs3::OP3_LIN) {
    using R = rs3::Res3S<P, 4>;
    const int zc = res3s_run_chunks(h, R::TEX);
    const unsigned nr = (unsigned)rs3::res3s_blocks(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], R::TEX, 4, zc);
    if (op == rs3::OP3_APPLY)
      hipLaunchKernelGGL((k_res3s<P, rs3::OP3_APPLY>), dim3(nr), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                         (const double *)h.lin, Y, zc);
    else
      hipLaunchKernelGGL((k_res3s<P, rs3::OP3_RES>), dim3(nr), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                         (const double *)nullptr, Y, zc);
  } else if (h.tiled_3d == 1 || h.tiled_3d == 3) {
    using R = rs3::Res3R<P, rs3::Res3RDepth<P>::TEZ>;
    const unsigned nr = (unsigned)rs3::res3r_tiles(h.pb.ne[0], h.pb.ne[1], h.pb.ne[2], R::TEX, rs3::Res3RDepth<P>::TEZ);
    if (op == rs3::OP3_APPLY)
      hipLaunchKernelGGL((k_res3r<P, rs3::OP3_APPLY>), dim3(nr), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                         (const double *)h.lin, Y);
    else if (op == rs3::OP3_LIN)
      hipLaunchKernelGGL((k_res3r<P, rs3::OP3_LIN>), dim3(nr), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                         (const double *)nullptr, Y);
    else
      hipLaunchKernelGGL((k_res3r<P, rs3::OP3_RES>), dim3(nr), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                         (const double *)nullptr, Y);
  } else if (op == rs3::OP3_APPLY)
    hipLaunchKernelGGL((k_res3<P, rs3::OP3_APPLY>), dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                       (const double *)h.lin, Y);
  else if (op == rs3::OP3_LIN)
    hipLaunchKernelGGL((k_res3<P, rs3::OP3_LIN>), dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                       (const double *)nullptr, Y);
  else
    hipLaunchKernelGGL((k_res3<P, rs3::OP3_RES>), dim3(nb), dim3(rs3::kThreads), 0, h.stream, h.pb, X,
                       (const double *)nullptr, Y);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

}  // namespace

bool res3_supported(const DevProblem &pb) {
  // p <= 4 (measured at 64^3, p = 4: 0.78 ms against 0.95 ms for the element-by-element kernel)
  return pb.dim == 3 && !pb.table && !pb.rational && pb.simple_knots && !pb.src && pb.P >= 2 && pb.P <= 5 &&
         (pb.kappa_mode == IGA_KAPPA_ONE || pb.kappa_mode == IGA_KAPPA_ELEMENT);
}

// residual (op = 0), matrix-free Jacobian apply (op = 1, needs the point cache of the linearisation) or
// the linearisation itself (op = 2: X = U, Y = the point cache)
iga_status launch_res3(Handle &h, const double *X, double *Y, int op) {
  if (op < rs3::OP3_RES || op > rs3::OP3_LIN) return fail(IGA_EINVAL, "tiled 3D operation");
  switch (h.pb.P) {
    case 2: return run_res3<2>(h, X, Y, op);
    case 3: return run_res3<3>(h, X, Y, op);
    case 4: return run_res3<4>(h, X, Y, op);
    case 5: return run_res3<5>(h, X, Y, op);
  }
  return fail(IGA_EUNSUPPORTED, "tiled 3D residual degree");
}

bool res2_supported(const DevProblem &pb) {
  return pb.dim == 2 && !pb.table && !pb.rational && pb.simple_knots && pb.P >= 2 && pb.P <= 5 &&
         (pb.kappa_mode == IGA_KAPPA_ONE || pb.kappa_mode == IGA_KAPPA_ELEMENT);
}

iga_status launch_res2(Handle &h, const double *U, double *R) {
  switch (h.pb.P) {
    case 2: return run_res2<2>(h, U, R);
    case 3: return run_res2<3>(h, U, R);
    case 4: return run_res2<4>(h, U, R);
    case 5: return run_res2<5>(h, U, R);
  }
  return fail(IGA_EUNSUPPORTED, "tiled 2D residual degree");
}

bool rgt2_supported(const DevProblem &pb) {
  return pb.dim == 2 && !pb.table && !pb.rational && pb.simple_knots && !pb.periodic && pb.P >= 2 && pb.P <= 5 &&
         (pb.kappa_mode == IGA_KAPPA_ONE || pb.kappa_mode == IGA_KAPPA_ELEMENT);
}

iga_status launch_jac_rgt2(Handle &h, const double *U, void *vals, int prec) {
  if (!rgt2_supported(h.pb)) return fail(IGA_EUNSUPPORTED, "tiled 2D row-gather configuration");
  switch (h.pb.P) {
    case 2: return run_rgt2<2>(h, U, vals, prec);
    case 3: return run_rgt2<3>(h, U, vals, prec);
    case 4: return run_rgt2<4>(h, U, vals, prec);
    case 5: return run_rgt2<5>(h, U, vals, prec);
  }
  return fail(IGA_EUNSUPPORTED, "tiled 2D row-gather degree");
}

}  // namespace iga
