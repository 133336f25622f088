// Batched Newton-Krylov for many independent 2D problems of different sizes and degrees.
//
// Every kernel below covers all instances in one launch: a launch walks a work list of tiles
// (instance, rows) or (instance, element) / (instance, pencil block) and reads the instance's
// problem description from a device array.  Per-instance CG scalars never leave the device:
// each tile writes one partial sum, and every block of an instance reduces that instance's
// partials in the same order, so all blocks take bitwise-identical alpha/beta and the same
// converged/not-converged decision without flags or atomics.  One chunk of CG iterations is
// captured once into a hipGraph and replayed; the host only reads one counter per chunk and
// one vector of residual norms per Newton step.  Launch shapes (pencils per row-gather block
// and lanes per SpMV row) are chosen per (degree, size class) by timing the candidates on the
// device when the batch is created.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "iga_impl.h"
#include "kern_elem.h"
#include "kern_rg.h"
#include "kern_res2.h"
#include "kern_rgt2.h"

namespace iga {
iga_status create_impl(const iga_desc *d, void *stream, Handle **out);

namespace {

constexpr int kVT = 256;   // rows per vector tile
// CG iterations per captured graph with each preconditioner (even: the partial buffers alternate)
constexpr int kChunkJacobi = 16, kChunkFdm = 8;

struct Tile {
  int inst;
  int start;
  int count;
};
struct Pair {
  int inst;
  int idx;
};

__device__ inline double bsum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  __syncthreads();
  return s;
}

// sum of the partials of one instance (identical in every block of that instance)
__device__ inline double inst_sum(const double *__restrict__ part, const int *__restrict__ vt_start, int inst,
                                  double *sh) {
  double v = 0;
  for (int i = vt_start[inst] + threadIdx.x; i < vt_start[inst + 1]; i += blockDim.x) v += part[i];
  return bsum(v, sh);
}

__device__ inline bool cg_done(const double *rr_cur, const int *vt_start, const double *target, int inst,
                               double *sh) {
  double rr = inst_sum(rr_cur, vt_start, inst, sh);
  return !(sqrt(rr) > target[inst]);
}

__global__ void k_b_fill(const Tile *__restrict__ tl, const int64_t *__restrict__ off, const int *__restrict__ act,
                         double *__restrict__ x, double v) {
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst] || (int)threadIdx.x >= T.count) return;
  x[off[T.inst] + T.start + threadIdx.x] = v;
}

template <int P>
__global__ void __launch_bounds__(64) k_b_residual(const DevProblem *__restrict__ pbs, const Pair *__restrict__ work,
                                                   const int64_t *__restrict__ off, const int *__restrict__ act,
                                                   const double *__restrict__ U, double *__restrict__ R) {
  const Pair w = work[blockIdx.x];
  if (!act[w.inst]) return;
  const int64_t o = off[w.inst];
  ek::elem_op_body<2, P, false, ek::OP_RES>(pbs[w.inst], (int64_t)w.idx, U + o, (double *)nullptr, R + o);
}

__global__ void k_b_bc_copy(const DevProblem *__restrict__ pbs, const Tile *__restrict__ tl,
                            const int64_t *__restrict__ off, const int *__restrict__ act, const double *__restrict__ X,
                            double *__restrict__ Y) {
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst] || (int)threadIdx.x >= T.count) return;
  const int64_t A = T.start + threadIdx.x, o = off[T.inst];
  if (is_dirichlet(pbs[T.inst], A)) Y[o + A] = X[o + A];
}

__global__ void k_b_sq_partial(const Tile *__restrict__ tl, const int64_t *__restrict__ off,
                               const double *__restrict__ x, double *__restrict__ part) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  double v = 0;
  if ((int)threadIdx.x < T.count) {
    double a = x[off[T.inst] + T.start + threadIdx.x];
    v = a * a;
  }
  double s = bsum(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_b_inst_norms(int n, const int *__restrict__ vt_start, const double *__restrict__ part,
                               double *__restrict__ norms) {
  __shared__ double sh[4];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    double s = inst_sum(part, vt_start, i, sh);
    if (threadIdx.x == 0) norms[i] = sqrt(s);
  }
}

template <int P, int B1, typename OT>
__global__ void __launch_bounds__(rgk::rg_threads(B1 * (2 * P - 1)))
k_b_rowgather(const DevProblem *__restrict__ pbs, const Pair *__restrict__ work, const int64_t *__restrict__ off,
              const int64_t *__restrict__ noff, const int *__restrict__ act, const double *__restrict__ U,
              OT *__restrict__ vals) {
  const Pair w = work[blockIdx.x];
  if (!act[w.inst]) return;
  rgk::rowgather2_body<P, false, B1, OT, OT>(pbs[w.inst], w.idx, U + off[w.inst], vals + noff[w.inst]);
}

template <int P, int V>
__global__ void __launch_bounds__(rst::kThreads) k_b_res2(const DevProblem *__restrict__ pbs,
                                                          const Pair *__restrict__ work,
                                                          const int64_t *__restrict__ off,
                                                          const int *__restrict__ act, const double *__restrict__ U,
                                                          double *__restrict__ R) {
  __shared__ double lds[rst::Res2<P, V>::total / sizeof(double)];
  const Pair w = work[blockIdx.x];
  if (!act[w.inst]) return;
  rst::res2_body<P, V>(pbs[w.inst], w.idx, U + off[w.inst], R + off[w.inst], lds);
}

template <int P, typename OT, int V>
__global__ void __launch_bounds__(rgt::kThreads)
k_b_rgt2(const DevProblem *__restrict__ pbs, const Pair *__restrict__ work, const int64_t *__restrict__ off,
         const int64_t *__restrict__ noff, const int *__restrict__ act, const double *__restrict__ U,
         OT *__restrict__ vals) {
  __shared__ __align__(16) char lds[rgt::Lds2<P, OT, OT, V>::total];
  const Pair w = work[blockIdx.x];
  if (!act[w.inst]) return;
  rgt::rgt2_body<P, OT, OT, V>(pbs[w.inst], w.idx, U + off[w.inst], vals + noff[w.inst], lds);
}

template <typename VT>
__global__ void k_b_diag_inv(const DevProblem *__restrict__ pbs, const Tile *__restrict__ tl,
                             const int64_t *__restrict__ off, const int64_t *__restrict__ noff,
                             const int *__restrict__ act, const VT *__restrict__ vals, double *__restrict__ dinv) {
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst] || (int)threadIdx.x >= T.count) return;
  const DevProblem &pb = pbs[T.inst];
  const int64_t A = T.start + threadIdx.x;
  const int i0 = (int)(A % pb.n[0]), i1 = (int)(A / pb.n[0]);
  double d = (double)vals[noff[T.inst] + csr_slot(pb, i0, i1, 0, i0, i1, 0)];
  dinv[off[T.inst] + A] = d != 0.0 ? 1.0 / d : 1.0;
}

// x = 0, r = -R, z = Dinv r, p = z; partials of r.z and r.r
__global__ void k_b_cg_init(const Tile *__restrict__ tl, const int64_t *__restrict__ off, const int *__restrict__ act,
                            const double *__restrict__ R, const double *__restrict__ dinv, double *__restrict__ x,
                            double *__restrict__ r, double *__restrict__ z, double *__restrict__ p,
                            double *__restrict__ part_rz, double *__restrict__ part_rr) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  double a = 0, b = 0;
  if (act[T.inst] && (int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    double ri = -R[i];
    x[i] = 0;
    r[i] = ri;
    if (dinv) {   // Jacobi; otherwise z, p and r.z come from the preconditioner step
      const double zi = dinv[i] * ri;
      z[i] = zi;
      p[i] = zi;
      a = ri * zi;
    }
    b = ri * ri;
  }
  double sa = bsum(a, sh), sb = bsum(b, sh);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = sa;
    part_rr[blockIdx.x] = sb;
  }
}

// q = J p on the instance's CSR rows (LPR lanes per row); partial p.q per tile
template <typename VT, int LPR>
__global__ void __launch_bounds__(256) k_b_spmv(const DevProblem *__restrict__ pbs, const Tile *__restrict__ st,
                                                const int *__restrict__ vt_start, const int64_t *__restrict__ off,
                                                const int64_t *__restrict__ noff, const int *__restrict__ act,
                                                const double *__restrict__ target, const double *__restrict__ rr_cur,
                                                const VT *__restrict__ vals, const double *__restrict__ p,
                                                double *__restrict__ q, double *__restrict__ part_pq) {
  __shared__ double sh[4];
  const Tile T = st[blockIdx.x];
  if (!act[T.inst]) return;
  if (cg_done(rr_cur, vt_start, target, T.inst, sh)) return;
  const DevProblem &pb = pbs[T.inst];
  const int64_t o = off[T.inst];
  const VT *v = vals + noff[T.inst];
  const double *pp = p + o;
  const int sub = threadIdx.x % LPR, row = threadIdx.x / LPR;
  const int n0 = pb.n[0], n1 = pb.n[1], deg = pb.p;
  double dot = 0;
  for (int r = row; r < T.count; r += 256 / LPR) {
    const int64_t A = T.start + r;
    // tensor-product pattern (simple knots): row (i0, i1) couples (l0 .. l0 + w0 - 1) x
    // (l1 .. l1 + w1 - 1), stored with axis 0 fastest, so no column indices are read
    const int i0 = (int)(A % n0), i1 = (int)(A / n0);
    const int l0 = max(0, i0 - deg), w0 = min(n0 - 1, i0 + deg) - l0 + 1;
    const int l1 = max(0, i1 - deg), w1 = min(n1 - 1, i1 + deg) - l1 + 1;
    const int64_t b = pb.row_ptr[A];
    const double *xb = pp + l0 + (int64_t)n0 * l1;
    double s = 0;
    for (int k = sub; k < w0 * w1; k += LPR) {
      const int o1 = k / w0, o0 = k - o1 * w0;
      s += (double)v[b + k] * xb[o0 + (int64_t)n0 * o1];
    }
    for (int w = LPR / 2; w > 0; w >>= 1) s += __shfl_xor(s, w, LPR);
    if (sub == 0) {
      q[o + A] = s;
      dot += s * pp[A];
    }
  }
  double bs = bsum(dot, sh);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = bs;
}

// alpha = rz/pq; x += alpha p; r -= alpha q; z = Dinv r; partials of the new r.z and r.r.
// A converged instance carries its partials over unchanged, so the decision stays put.
__global__ void __launch_bounds__(256) k_b_cg_xr(const Tile *__restrict__ tl, const int *__restrict__ vt_start,
                                                 const int *__restrict__ st_start, const int64_t *__restrict__ off,
                                                 const int *__restrict__ act, const double *__restrict__ target,
                                                 const double *__restrict__ rz_cur, const double *__restrict__ rr_cur,
                                                 const double *__restrict__ part_pq, double *__restrict__ x,
                                                 double *__restrict__ r, double *__restrict__ z,
                                                 const double *__restrict__ p, const double *__restrict__ q,
                                                 const double *__restrict__ dinv, double *__restrict__ rz_new,
                                                 double *__restrict__ rr_new) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst]) return;
  if (cg_done(rr_cur, vt_start, target, T.inst, sh)) {
    if (threadIdx.x == 0) {
      rz_new[blockIdx.x] = rz_cur[blockIdx.x];
      rr_new[blockIdx.x] = rr_cur[blockIdx.x];
    }
    return;
  }
  const double rz = inst_sum(rz_cur, vt_start, T.inst, sh);
  double pq = 0;
  for (int i = st_start[T.inst] + threadIdx.x; i < st_start[T.inst + 1]; i += blockDim.x) pq += part_pq[i];
  pq = bsum(pq, sh);
  const double alpha = pq != 0.0 ? rz / pq : 0.0;
  double a = 0, b = 0;
  if ((int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    x[i] += alpha * p[i];
    double ri = r[i] - alpha * q[i];
    r[i] = ri;
    if (dinv) {
      const double zi = dinv[i] * ri;
      z[i] = zi;
      a = ri * zi;
    }
    b = ri * ri;
  }
  double sa = bsum(a, sh), sb = bsum(b, sh);
  if (threadIdx.x == 0) {
    if (dinv) rz_new[blockIdx.x] = sa;
    rr_new[blockIdx.x] = sb;
  }
}

// beta = rz_new/rz; p = z + beta p; the first tile of an instance counts its iterations
__global__ void __launch_bounds__(256) k_b_cg_p(const Tile *__restrict__ tl, const int *__restrict__ vt_start,
                                                const int64_t *__restrict__ off, const int *__restrict__ act,
                                                const double *__restrict__ target, const double *__restrict__ rz_cur,
                                                const double *__restrict__ rr_cur, const double *__restrict__ rz_new,
                                                const double *__restrict__ z, double *__restrict__ p,
                                                int *__restrict__ iters) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst]) return;
  if (cg_done(rr_cur, vt_start, target, T.inst, sh)) return;
  const double rz = inst_sum(rz_cur, vt_start, T.inst, sh);
  const double rzn = inst_sum(rz_new, vt_start, T.inst, sh);
  const double beta = rz != 0.0 ? rzn / rz : 0.0;
  if ((int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    p[i] = z[i] + beta * p[i];
  }
  if (threadIdx.x == 0 && (int)blockIdx.x == vt_start[T.inst]) iters[T.inst] += 1;
}

// number of Newton-active instances whose CG has not converged (single block)
// flags[i] = 1 if instance i is active and its CG has not converged (one wave per instance)
__global__ void __launch_bounds__(256) k_b_flags(int n, const int *__restrict__ vt_start, const int *__restrict__ act,
                                                 const double *__restrict__ target, const double *__restrict__ rr,
                                                 int *__restrict__ flags) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (i >= n) return;
  double v = 0;
  if (act[i])
    for (int k = vt_start[i] + lane; k < vt_start[i + 1]; k += 64) v += rr[k];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if (lane == 0) flags[i] = (act[i] && sqrt(v) > target[i] && v == v) ? 1 : 0;
}

// number of instances whose CG still runs
__global__ void __launch_bounds__(256) k_b_count(int n, const int *__restrict__ flags, int *__restrict__ out) {
  __shared__ double sh[4];
  double c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += flags[i];
  c = bsum(c, sh);
  if (threadIdx.x == 0) *out = (int)c;
}

__global__ void k_b_axpy(const Tile *__restrict__ tl, const int64_t *__restrict__ off, const int *__restrict__ act,
                         const double *__restrict__ d, double *__restrict__ U) {
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst] || (int)threadIdx.x >= T.count) return;
  const int64_t i = off[T.inst] + T.start + threadIdx.x;
  U[i] += d[i];
}

// Newton control of every instance on the device, after the residual norms of step k = *kstep:
// the stopping test (||R|| < atol, or ||R|| <= rtol ||R_0||, or k = max_newton, or a non-finite
// norm) ends an instance (act = 0); otherwise the Eisenstat-Walker forcing term (second choice,
// floor 0.1 target / ||R||, cap forcing_max) sets its CG target eta ||R||.  Also records the norm
// history.  One workgroup; *nact receives the number of instances still iterating.
// prm: atol, rtol, forcing_max, max_newton.
constexpr int kHist = 65;
__global__ void __launch_bounds__(1024) k_b_newton_ctl(int n, const double *__restrict__ norms, const double *__restrict__ prm,
                                                       int *__restrict__ act, double *__restrict__ target,
                                                       double *__restrict__ r0, double *__restrict__ nr_prev,
                                                       double *__restrict__ eta, int *__restrict__ conv,
                                                       int *__restrict__ hcount, double *__restrict__ hist,
                                                       int *__restrict__ kstep, int *__restrict__ nact) {
  __shared__ int cnt[16];
  const int k = *kstep, t = threadIdx.x;
  const double atol = prm[0], rtol = prm[1], fmax_ = prm[2];
  const int max_newton = (int)prm[3];
  int c = 0;
  for (int i = t; i < n; i += blockDim.x) {
    if (!act[i]) continue;
    const double nr = norms[i];
    if (k < kHist) hist[(size_t)i * kHist + k] = nr;
    hcount[i] = k + 1;
    if (r0[i] < 0) r0[i] = nr;
    if (!isfinite(nr)) { act[i] = 0; continue; }
    if (nr < atol || (rtol > 0 && nr <= rtol * r0[i])) { act[i] = 0; conv[i] = 1; continue; }
    if (k >= max_newton) { act[i] = 0; continue; }
    double e = eta[i];
    if (k > 0) {
      const double ratio = nr / nr_prev[i];
      e = fmin(fmax_, 0.9 * ratio * ratio);
    }
    const double tgt = fmax(atol, rtol * r0[i]);
    e = fmin(fmax_, fmax(e, 0.1 * tgt / nr));
    eta[i] = e;
    nr_prev[i] = nr;
    target[i] = e * nr;
    ++c;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((t & 63) == 0) cnt[t >> 6] = c;
  __syncthreads();
  if (t == 0) {
    int s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += cnt[w];
    *nact = s;
    *kstep = k + 1;
  }
}

// ------------------------------------------------------------------------------------------
// Batched fast-diagonalisation preconditioner.  Per instance (2D) z = (a0 A0 (x) M1 + a1 M0 (x) A1
// + c M)^{-1} r on the non-Dirichlet box, z = r elsewhere (the single-problem preconditioner of
// precond.hip, one box per instance): two 1D transforms, a scaling, two inverse transforms.
// A block handles kBfTC columns of one instance; instances whose CG has converged are skipped.
// ------------------------------------------------------------------------------------------
constexpr int kBfMax = 136, kBfTC = 16;
struct BfInst {
  int m0, m1, lo0, lo1, n0;
  int64_t tf0, tb0, tf1, tb1;   // V^T / V of each axis in the pool
  int64_t mu0, mu1;             // eigenvalues times the axis coefficient, in the pool
  int64_t rs0, rs1;             // 1D basis integrals, in the pool
  int64_t box;                  // offset of the m0 x m1 box in the scratch vectors
  double mu_min;
};

// shift c_k = max(-lambda_k * (integral-weighted mean of e^U), -0.9 min eigenvalue), per instance
__global__ void __launch_bounds__(256) k_bf_shift(const DevProblem *__restrict__ pbs, const BfInst *__restrict__ bf,
                                                  const double *__restrict__ pool, const int64_t *__restrict__ off,
                                                  const int *__restrict__ act, const double *__restrict__ U,
                                                  double *__restrict__ shift) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  if (!act[k]) return;
  const DevProblem &pb = pbs[k];
  const BfInst B = bf[k];
  double s1 = 0, s2 = 0;
  for (int64_t A = threadIdx.x; A < pb.N; A += blockDim.x) {
    const int i0 = (int)(A % pb.n[0]), i1 = (int)(A / pb.n[0]);
    const double w = pool[B.rs0 + i0] * pool[B.rs1 + i1];
    s1 += w * exp(U[off[k] + A]);
    s2 += w;
  }
  s1 = bsum(s1, sh);
  s2 = bsum(s2, sh);
  if (threadIdx.x == 0) {
    const double c = s2 > 0 ? -pb.lambda * s1 / s2 : 0.0;
    shift[k] = fmax(c, -0.9 * B.mu_min);
  }
}

template <int AX>
__global__ void __launch_bounds__(256) k_bf_axis(const Pair *__restrict__ work, const BfInst *__restrict__ bf,
                                                 const double *__restrict__ pool, const int64_t *__restrict__ off,
                                                 const int *__restrict__ act, const int *__restrict__ vt_start,
                                                 const double *__restrict__ target, const double *__restrict__ rr_cur,
                                                 const double *__restrict__ in, int in_full, double *__restrict__ out,
                                                 int out_full, int fwd, int scale, const double *__restrict__ shift) {
  __shared__ double x[kBfMax][kBfTC + 1], y[kBfMax][kBfTC + 1];
  __shared__ double sh[4];
  const Pair w = work[blockIdx.x];
  const int k = w.inst;
  if (!act[k]) return;
  if (rr_cur && cg_done(rr_cur, vt_start, target, k, sh)) return;
  const BfInst B = bf[k];
  const int m = AX == 0 ? B.m0 : B.m1, ncol = AX == 0 ? B.m1 : B.m0;
  const double *T = pool + (AX == 0 ? (fwd ? B.tf0 : B.tb0) : (fwd ? B.tf1 : B.tb1));
  const int c0 = w.idx, t = threadIdx.x;
  auto addr = [&](int full, int i0, int i1) -> int64_t {
    return full ? off[k] + (B.lo0 + i0) + (int64_t)B.n0 * (B.lo1 + i1) : B.box + i0 + (int64_t)B.m0 * i1;
  };
  // axis 0 walks the contracted index (contiguous) fastest, axis 1 the columns (i0)
  for (int e = t; e < m * kBfTC; e += 256) {
    const int kk = AX == 0 ? e % m : e / kBfTC, cl = AX == 0 ? e / m : e % kBfTC, c = c0 + cl;
    double v = 0;
    if (c < ncol) v = AX == 0 ? in[addr(in_full, kk, c)] : in[addr(in_full, c, kk)];
    x[kk][cl] = v;
  }
  __syncthreads();
  const int cl = t % kBfTC, g = t / kBfTC;
  for (int i = g; i < m; i += 256 / kBfTC) {
    const double *Ti = T + (size_t)i * m;
    double acc = 0;
    for (int kk = 0; kk < m; ++kk) acc += Ti[kk] * x[kk][cl];
    y[i][cl] = acc;
  }
  __syncthreads();
  const double c_shift = scale ? shift[k] : 0.0;
  for (int e = t; e < m * kBfTC; e += 256) {
    const int i = AX == 0 ? e % m : e / kBfTC, cl2 = AX == 0 ? e / m : e % kBfTC, c = c0 + cl2;
    if (c >= ncol) continue;
    const int i0 = AX == 0 ? i : c, i1 = AX == 0 ? c : i;
    double v = y[i][cl2];
    if (scale) v /= pool[B.mu0 + i0] + pool[B.mu1 + i1] + c_shift;
    out[addr(out_full, i0, i1)] = v;
  }
}

// z = r (the Dirichlet rows keep it; the transforms overwrite the box)
__global__ void k_b_copy_pc(const Tile *__restrict__ tl, const int *__restrict__ vt_start, const int64_t *__restrict__ off,
                            const int *__restrict__ act, const double *__restrict__ target,
                            const double *__restrict__ rr_cur, const double *__restrict__ r, double *__restrict__ z) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst]) return;
  if (rr_cur && cg_done(rr_cur, vt_start, target, T.inst, sh)) return;
  if ((int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    z[i] = r[i];
  }
}

// partial r.z per tile; a converged instance carries its partials over
__global__ void __launch_bounds__(256) k_b_rz(const Tile *__restrict__ tl, const int *__restrict__ vt_start,
                                              const int64_t *__restrict__ off, const int *__restrict__ act,
                                              const double *__restrict__ target, const double *__restrict__ rr_cur,
                                              const double *__restrict__ rz_cur, const double *__restrict__ r,
                                              const double *__restrict__ z, double *__restrict__ rz_new) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  if (!act[T.inst]) return;
  if (cg_done(rr_cur, vt_start, target, T.inst, sh)) {
    if (threadIdx.x == 0) rz_new[blockIdx.x] = rz_cur[blockIdx.x];
    return;
  }
  double a = 0;
  if ((int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    a = r[i] * z[i];
  }
  const double sa = bsum(a, sh);
  if (threadIdx.x == 0) rz_new[blockIdx.x] = sa;
}

// p = z; partial r.z (first CG iteration)
__global__ void __launch_bounds__(256) k_b_pz(const Tile *__restrict__ tl, const int64_t *__restrict__ off,
                                              const int *__restrict__ act, const double *__restrict__ r,
                                              const double *__restrict__ z, double *__restrict__ p,
                                              double *__restrict__ part_rz) {
  __shared__ double sh[4];
  const Tile T = tl[blockIdx.x];
  double a = 0;
  if (act[T.inst] && (int)threadIdx.x < T.count) {
    const int64_t i = off[T.inst] + T.start + threadIdx.x;
    p[i] = z[i];
    a = r[i] * z[i];
  }
  const double sa = bsum(a, sh);
  if (threadIdx.x == 0) part_rz[blockIdx.x] = sa;
}

// ------------------------------------------------------------------------------------------
// Autotuner cache: (degree, size class, kernel) -> chosen shape, kept for the process
// ------------------------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<long, int> g_tune;   // key = (kind << 16) | (p << 8) | size class
bool g_tune_loaded = false;

// The cache is also kept in the JSON file named by IGA_TUNE_CACHE (when set): an object whose
// keys are "kind:degree:size class" (kind 1: row-gather pencils per block, 2: SpMV lanes per row,
// 3: tiled row-gather shape, 4: tiled residual shape) and whose values are the chosen shapes.
// Read once per process before the first tuning, rewritten after each tuning.  Caller holds g_tune_mu.
void tune_cache_load() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *path = std::getenv("IGA_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  int c, kind, p, cls, v;
  while ((c = std::fgetc(f)) != EOF) {
    if (c != '"') continue;
    if (std::fscanf(f, "%d:%d:%d\": %d", &kind, &p, &cls, &v) == 4 && kind >= 1 && kind <= 4)
      g_tune[((long)kind << 16) | (p << 8) | cls] = v;
  }
  std::fclose(f);
}

void tune_cache_save() {
  const char *path = std::getenv("IGA_TUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  std::fprintf(f, "{");
  bool first = true;
  for (const auto &kv : g_tune) {
    std::fprintf(f, "%s\n  \"%ld:%ld:%ld\": %d", first ? "" : ",", kv.first >> 16, (kv.first >> 8) & 255, kv.first & 255,
                 kv.second);
    first = false;
  }
  std::fprintf(f, "\n}\n");
  std::fclose(f);
}

int size_class(int64_t N) { return N < 1500 ? 0 : (N < 5000 ? 1 : 2); }

}  // namespace

struct Group {
  int P;
  int cls;
  std::vector<int> insts;
  int b1 = 4;               // row-gather pencils per block, 0: tiled kernel (autotuned)
  int lpr = 8;              // SpMV lanes per row (autotuned)
  int rgt_v = 0;            // tiled row-gather tile shape (rgt::Shape2 variant, autotuned)
  int res_v = 0;            // tiled residual tile shape (rst::Res2 variant, autotuned)
  std::vector<Pair> pencils;
  Pair *d_pencils = nullptr;
  std::vector<Pair> tiles;   // (instance, tile) of the tiled row-gather
  Pair *d_tiles = nullptr;
  std::vector<Pair> elems;   // (instance, element), or (instance, element tile) when res_tiles
  Pair *d_elems = nullptr;
  bool res_tiles = false;
};

struct Batch {
  int n = 0;
  std::vector<Handle *> hs;
  hipStream_t user = nullptr, bs = nullptr;
  std::vector<void *> owned;
  DevProblem *d_pbs = nullptr;
  std::vector<int64_t> off, noff;
  int64_t *d_off = nullptr, *d_noff = nullptr;
  int64_t Ntot = 0, nnztot = 0;
  std::vector<Tile> vt;
  std::vector<int> vt_start;
  Tile *d_vt = nullptr;
  int *d_vt_start = nullptr;
  // SpMV tiles (per group shapes), concatenated; st_start per instance
  std::vector<Tile> st;
  std::vector<int> st_start;
  Tile *d_st = nullptr;
  int *d_st_start = nullptr;
  std::vector<std::pair<int, int>> st_group_range;   // [first tile, count) per group
  std::vector<Group> groups;
  // state
  double *ws = nullptr;        // R d r z p q : 6 * Ntot
  double *dinv = nullptr;
  void *vals = nullptr;
  int vals_prec = -1;
  double *partA = nullptr, *partB = nullptr, *partC = nullptr, *partD = nullptr, *part_pq = nullptr;
  double *norms = nullptr, *target = nullptr;
  int *act = nullptr, *iters = nullptr, *count = nullptr, *flags = nullptr;
  hipGraphExec_t graph = nullptr;
  // one Newton step as one graph (see batch_newton) and its device-side Newton state
  hipGraphExec_t step_graph = nullptr;
  const double *step_U = nullptr;
  int step_prec = -1, step_chunk = 0;
  bool step_fdm = false;
  double *nprm = nullptr, *r0 = nullptr, *nr_prev = nullptr, *eta = nullptr, *hist = nullptr;
  int *conv = nullptr, *hcount = nullptr, *kstep = nullptr, *nact = nullptr;
  // batched fast-diagonalisation preconditioner (bf_on: every instance has one)
  bool bf_on = false;
  int precond = IGA_PRECOND_AUTO;   // iga_precond chosen by the caller
  BfInst *d_bf = nullptr;
  double *bf_pool = nullptr, *bf_shift = nullptr, *bf_w = nullptr;
  std::vector<Pair> bf_w0, bf_w1;
  Pair *d_bf_w0 = nullptr, *d_bf_w1 = nullptr;
  int64_t bf_box_total = 0;
  int graph_prec = -1, graph_chunk = 0;
  bool graph_fdm = false;
  double t_tune_ms = 0;
  std::vector<int> perm_;
};

template <typename T>
static iga_status balloc(Batch &b, T **p, size_t n) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
  if (e != hipSuccess) return fail(IGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  b.owned.push_back(q);
  *p = (T *)q;
  return IGA_OK;
}

template <typename T>
static iga_status bupload(Batch &b, T **p, const std::vector<T> &v) {
  iga_status st = balloc(b, p, v.size());
  if (st) return st;
  IGA_HIP_CHECK(hipMemcpyAsync(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, b.bs));
  return IGA_OK;
}

static void batch_free(Batch *b) {
  if (!b) return;
  if (b->bs) (void)hipStreamSynchronize(b->bs);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->step_graph) (void)hipGraphExecDestroy(b->step_graph);
  for (void *p : b->owned)
    if (p) (void)hipFree(p);
  for (Handle *h : b->hs) iga_destroy((iga_t)h);
  if (b->bs) (void)hipStreamDestroy(b->bs);
  delete b;
}

// ---- launch helpers -----------------------------------------------------------------------
template <int P, int V>
static void launch_rgt_v(Batch &b, const Group &g, const double *U, void *vals, int prec, hipStream_t s) {
  dim3 grid((unsigned)g.tiles.size()), blk(rgt::kThreads);
  if (prec == IGA_FP32)
    hipLaunchKernelGGL((k_b_rgt2<P, float, V>), grid, blk, 0, s, b.d_pbs, g.d_tiles, b.d_off, b.d_noff, b.act, U,
                       (float *)vals);
  else
    hipLaunchKernelGGL((k_b_rgt2<P, double, V>), grid, blk, 0, s, b.d_pbs, g.d_tiles, b.d_off, b.d_noff, b.act, U,
                       (double *)vals);
}

template <int P>
static void launch_rgt_group(Batch &b, const Group &g, const double *U, void *vals, int prec, hipStream_t s) {
  if constexpr (P >= 2 && P <= 5) {
    if (g.rgt_v == 1) launch_rgt_v<P, 1>(b, g, U, vals, prec, s);
    else launch_rgt_v<P, 0>(b, g, U, vals, prec, s);
  }
}

template <int P>
static void launch_rg_group(Batch &b, const Group &g, int b1, const double *U, void *vals, int prec, hipStream_t s) {
  if (b1 == 0) {
    if (!g.tiles.empty()) launch_rgt_group<P>(b, g, U, vals, prec, s);
    return;
  }
  dim3 grid((unsigned)g.pencils.size());
#define IGA_RGB(BB)                                                                                          \
  if (b1 == BB) {                                                                                            \
    dim3 blk(rgk::rg_threads(BB * (2 * P - 1)));                                                             \
    if (prec == IGA_FP32)                                                                                    \
      hipLaunchKernelGGL((k_b_rowgather<P, BB, float>), grid, blk, 0, s, b.d_pbs, g.d_pencils, b.d_off,      \
                         b.d_noff, b.act, U, (float *)vals);                                                 \
    else                                                                                                     \
      hipLaunchKernelGGL((k_b_rowgather<P, BB, double>), grid, blk, 0, s, b.d_pbs, g.d_pencils, b.d_off,     \
                         b.d_noff, b.act, U, (double *)vals);                                                \
    return;                                                                                                  \
  }
  IGA_RGB(1) IGA_RGB(4) IGA_RGB(8)
#undef IGA_RGB
}

static void launch_rg(Batch &b, const Group &g, int b1, const double *U, void *vals, int prec, hipStream_t s) {
  if (b1 != 0 && g.pencils.empty()) return;
  switch (g.P) {
    case 3: launch_rg_group<3>(b, g, b1, U, vals, prec, s); break;
    case 4: launch_rg_group<4>(b, g, b1, U, vals, prec, s); break;
    case 5: launch_rg_group<5>(b, g, b1, U, vals, prec, s); break;
    case 2: launch_rg_group<2>(b, g, b1, U, vals, prec, s); break;
    case 6: launch_rg_group<6>(b, g, b1, U, vals, prec, s); break;
  }
}

static void launch_res(Batch &b, const Group &g, const double *U, double *R, hipStream_t s) {
  if (g.elems.empty()) return;
  dim3 grid((unsigned)g.elems.size()), blk(64);
  if (g.res_tiles) {
    dim3 bt(rst::kThreads);
#define IGA_BRES(PP, VV) \
  hipLaunchKernelGGL((k_b_res2<PP, VV>), grid, bt, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R)
    switch (g.P * 2 + g.res_v) {
      case 4: IGA_BRES(2, 0); break;
      case 5: IGA_BRES(2, 1); break;
      case 6: IGA_BRES(3, 0); break;
      case 7: IGA_BRES(3, 1); break;
      case 8: IGA_BRES(4, 0); break;
      case 9: IGA_BRES(4, 1); break;
      case 10: IGA_BRES(5, 0); break;
      case 11: IGA_BRES(5, 1); break;
    }
#undef IGA_BRES
    return;
  }
  switch (g.P) {
    case 2: hipLaunchKernelGGL(k_b_residual<2>, grid, blk, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R); break;
    case 3: hipLaunchKernelGGL(k_b_residual<3>, grid, blk, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R); break;
    case 4: hipLaunchKernelGGL(k_b_residual<4>, grid, blk, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R); break;
    case 5: hipLaunchKernelGGL(k_b_residual<5>, grid, blk, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R); break;
    case 6: hipLaunchKernelGGL(k_b_residual<6>, grid, blk, 0, s, b.d_pbs, g.d_elems, b.d_off, b.act, U, R); break;
  }
}

template <typename VT>
static void launch_spmv_group(Batch &b, size_t gi, const VT *vals, const double *p, double *q, const double *rr_cur,
                              hipStream_t s) {
  const Group &g = b.groups[gi];
  auto rng = b.st_group_range[gi];
  if (rng.second == 0) return;
  dim3 grid((unsigned)rng.second), blk(256);
  const Tile *tiles = b.d_st + rng.first;
  double *part = b.part_pq + rng.first;
#define IGA_SPM(L)                                                                                            \
  if (g.lpr == L) {                                                                                           \
    hipLaunchKernelGGL((k_b_spmv<VT, L>), grid, blk, 0, s, b.d_pbs, tiles, b.d_vt_start, b.d_off, b.d_noff,  \
                       b.act, b.target, rr_cur, vals, p, q, part);                                            \
    return;                                                                                                   \
  }
  IGA_SPM(4) IGA_SPM(8) IGA_SPM(16) IGA_SPM(32)
#undef IGA_SPM
}

// SpMV tiles: rows per tile = 256 / lpr of the instance's group.  Instances are numbered so
// that each group is contiguous; tile ranges are then contiguous per instance and per group.
static void build_spmv_tiles(Batch &b) {
  b.st.clear();
  b.st_start.assign(b.n + 1, 0);
  b.st_group_range.assign(b.groups.size(), {0, 0});
  for (size_t gi = 0; gi < b.groups.size(); ++gi) {
    const Group &g = b.groups[gi];
    const int rpt = 256 / g.lpr;
    b.st_group_range[gi].first = (int)b.st.size();
    for (int i : g.insts) {
      b.st_start[i] = (int)b.st.size();
      for (int64_t s0 = 0; s0 < b.hs[i]->pb.N; s0 += rpt)
        b.st.push_back(Tile{i, (int)s0, (int)std::min<int64_t>(rpt, b.hs[i]->pb.N - s0)});
    }
    b.st_group_range[gi].second = (int)b.st.size() - b.st_group_range[gi].first;
  }
  b.st_start[b.n] = (int)b.st.size();
}

static iga_status upload_spmv(Batch &b) {
  build_spmv_tiles(b);
  iga_status st;
  if ((st = bupload(b, &b.d_st, b.st)) || (st = bupload(b, &b.d_st_start, b.st_start))) return st;
  if ((st = balloc(b, &b.part_pq, b.st.size()))) return st;
  return IGA_OK;
}

// tiles of the tiled row-gather (degrees 1..4 with element-wise or unit kappa; every batched
// instance has the identity geometry and simple knots)
static bool tiles_supported(const Batch &b, const Group &g) {
  if (g.P < 2 || g.P > 5) return false;
  for (int i : g.insts)
    if (!rgt2_supported(b.hs[i]->pb)) return false;
  return true;
}

template <int P>
static void rgt_shape(int v, int *T0, int *B1) {
  if constexpr (P >= 2 && P <= 5) {
    *T0 = v ? rgt::Shape2<P, 1>::T0 : rgt::Shape2<P, 0>::T0;
    *B1 = v ? rgt::Shape2<P, 1>::B1 : rgt::Shape2<P, 0>::B1;
  }
}

static iga_status build_tiles(Batch &b, Group &g) {
  g.tiles.clear();
  int T0 = 0, B1 = 0;
  switch (g.P) {
    case 2: rgt_shape<2>(g.rgt_v, &T0, &B1); break;
    case 3: rgt_shape<3>(g.rgt_v, &T0, &B1); break;
    case 4: rgt_shape<4>(g.rgt_v, &T0, &B1); break;
    case 5: rgt_shape<5>(g.rgt_v, &T0, &B1); break;
    default: return IGA_OK;
  }
  for (int i : g.insts) {
    const DevProblem &pb = b.hs[i]->pb;
    const int nt = rgt::rgt2_tiles_0(pb.n[0], T0) * ((pb.n[1] + B1 - 1) / B1);
    for (int k = 0; k < nt; ++k) g.tiles.push_back(Pair{i, k});
  }
  return bupload(b, &g.d_tiles, g.tiles);
}

// (instance, element) or (instance, element tile) work list of the residual
static iga_status build_elems(Batch &b, Group &g) {
  g.elems.clear();
  int TE = 0;
  switch (g.P * 2 + g.res_v) {
    case 4: TE = rst::Res2<2, 0>::TE; break;
    case 5: TE = rst::Res2<2, 1>::TE; break;
    case 6: TE = rst::Res2<3, 0>::TE; break;
    case 7: TE = rst::Res2<3, 1>::TE; break;
    case 8: TE = rst::Res2<4, 0>::TE; break;
    case 9: TE = rst::Res2<4, 1>::TE; break;
    case 10: TE = rst::Res2<5, 0>::TE; break;
    case 11: TE = rst::Res2<5, 1>::TE; break;
  }
  for (int k : g.insts) {
    const DevProblem &pk = b.hs[k]->pb;
    const int64_t cnt = g.res_tiles ? rst::res2_tiles(pk.ne[0], pk.ne[1], TE) : pk.E;
    for (int64_t e = 0; e < cnt; ++e) g.elems.push_back(Pair{k, (int)e});
  }
  return bupload(b, &g.d_elems, g.elems);
}

static iga_status build_pencils(Batch &b, Group &g) {
  g.pencils.clear();
  for (int i : g.insts) {
    const int nb = (b.hs[i]->pb.n[1] + g.b1 - 1) / g.b1;
    for (int k = 0; k < nb; ++k) g.pencils.push_back(Pair{i, k});
  }
  iga_status st = bupload(b, &g.d_pencils, g.pencils);
  return st;
}

static float elapsed(hipEvent_t a, hipEvent_t c) {
  float ms = 0;
  (void)hipEventElapsedTime(&ms, a, c);
  return ms;
}

// Time every candidate shape of each group's row-gather and SpMV launches on the device and
// keep the fastest (cached per process by degree and size class).
static iga_status autotune(Batch &b) {
  auto t0 = std::chrono::steady_clock::now();
  hipEvent_t e0, e1;
  IGA_HIP_CHECK(hipEventCreate(&e0));
  IGA_HIP_CHECK(hipEventCreate(&e1));
  double *U = b.ws + 5 * b.Ntot;   // q slot as a zero state
  hipLaunchKernelGGL(k_b_fill, dim3((unsigned)b.vt.size()), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, U, 0.0);
  iga_status st = IGA_OK;
  for (Group &g : b.groups) {
    long key_rg = (1L << 16) | (g.P << 8) | g.cls, key_sp = (2L << 16) | (g.P << 8) | g.cls;
    bool have_rg, have_sp;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      tune_cache_load();
      have_rg = g_tune.count(key_rg);
      have_sp = g_tune.count(key_sp);
      if (have_rg) g.b1 = g_tune[key_rg];
      if (have_sp) g.lpr = g_tune[key_sp];
    }
    const bool tiles = tiles_supported(b, g);
    if (tiles && (st = build_tiles(b, g))) return st;
    if (have_rg && g.b1 == 0 && !tiles) have_rg = false;
    if (!have_rg && tiles) {
      // the tiled kernel wherever it applies (several times faster than any pencil shape)
      g.b1 = 0;
    } else if (!have_rg) {
      float best = 1e30f;
      int bestb = 4;
      for (int cand : {1, 4, 8}) {
        g.b1 = cand;
        if ((st = build_pencils(b, g))) return st;
        launch_rg(b, g, cand, U, b.vals, IGA_FP64, b.bs);
        hipEventRecord(e0, b.bs);
        for (int r = 0; r < 3; ++r) launch_rg(b, g, cand, U, b.vals, IGA_FP64, b.bs);
        hipEventRecord(e1, b.bs);
        IGA_HIP_CHECK(hipEventSynchronize(e1));
        float ms = elapsed(e0, e1);
        if (ms < best) { best = ms; bestb = cand; }
      }
      g.b1 = bestb;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[key_rg] = bestb;
    }
    if (g.b1 > 0 && (st = build_pencils(b, g))) return st;
    // tile shapes of the tiled row-gather and residual: time both variants (values are never read)
    const long key_rt = (3L << 16) | (g.P << 8) | g.cls, key_rs = (4L << 16) | (g.P << 8) | g.cls;
    int cached_rt = -1, cached_rs = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      if (g_tune.count(key_rt)) cached_rt = g_tune[key_rt];
      if (g_tune.count(key_rs)) cached_rs = g_tune[key_rs];
    }
    if (g.b1 == 0 && tiles) {
      if (cached_rt >= 0) {
        g.rgt_v = cached_rt;
      } else {
        float best = 1e30f;
        int bestv = 0;
        for (int v : {0, 1}) {
          g.rgt_v = v;
          if ((st = build_tiles(b, g))) return st;
          IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
          launch_rg(b, g, 0, U, b.vals, IGA_FP64, b.bs);
          hipEventRecord(e0, b.bs);
          for (int r = 0; r < 3; ++r) launch_rg(b, g, 0, U, b.vals, IGA_FP64, b.bs);
          hipEventRecord(e1, b.bs);
          IGA_HIP_CHECK(hipEventSynchronize(e1));
          const float ms = elapsed(e0, e1);
          if (ms < best) { best = ms; bestv = v; }
        }
        g.rgt_v = bestv;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key_rt] = bestv;
      }
      if ((st = build_tiles(b, g))) return st;
    }
    if (g.res_tiles) {
      if (cached_rs >= 0) {
        g.res_v = cached_rs;
      } else {
        double *R = b.ws;
        float best = 1e30f;
        int bestv = 0;
        for (int v : {0, 1}) {
          g.res_v = v;
          if ((st = build_elems(b, g))) return st;
          IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
          launch_res(b, g, U, R, b.bs);
          hipEventRecord(e0, b.bs);
          for (int r = 0; r < 3; ++r) launch_res(b, g, U, R, b.bs);
          hipEventRecord(e1, b.bs);
          IGA_HIP_CHECK(hipEventSynchronize(e1));
          const float ms = elapsed(e0, e1);
          if (ms < best) { best = ms; bestv = v; }
        }
        g.res_v = bestv;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key_rs] = bestv;
      }
      if ((st = build_elems(b, g))) return st;
    }
  }
  // SpMV lanes per row: tune each group with the others fixed
  for (size_t gi = 0; gi < b.groups.size(); ++gi) {
    Group &g = b.groups[gi];
    long key_sp = (2L << 16) | (g.P << 8) | g.cls;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      if (g_tune.count(key_sp)) { g.lpr = g_tune[key_sp]; continue; }
    }
    float best = 1e30f;
    int bestl = 8;
    for (int cand : {4, 8, 16, 32}) {
      g.lpr = cand;
      if ((st = upload_spmv(b))) return st;
      // all instances "not converged": target = -1 makes sqrt(rr) > target true
      hipLaunchKernelGGL(k_b_fill, dim3((unsigned)b.vt.size()), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act,
                         b.ws + 4 * b.Ntot, 1.0);
      launch_spmv_group<double>(b, gi, (const double *)b.vals, b.ws + 4 * b.Ntot, b.ws + 5 * b.Ntot, b.partA, b.bs);
      hipEventRecord(e0, b.bs);
      for (int r = 0; r < 5; ++r)
        launch_spmv_group<double>(b, gi, (const double *)b.vals, b.ws + 4 * b.Ntot, b.ws + 5 * b.Ntot, b.partA, b.bs);
      hipEventRecord(e1, b.bs);
      IGA_HIP_CHECK(hipEventSynchronize(e1));
      float ms = elapsed(e0, e1);
      if (ms < best) { best = ms; bestl = cand; }
    }
    g.lpr = bestl;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key_sp] = bestl;
  }
  if ((st = upload_spmv(b))) return st;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_cache_save();
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b.t_tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return IGA_OK;
}

// Fast-diagonalisation data of every instance: one generalised eigendecomposition per distinct
// 1D problem (knots, degree, Dirichlet range), computed on host threads; instances scale the
// eigenvalues by their axis coefficient (the mean kappa for element-wise kappa).  Leaves
// bf_on false (Jacobi) if an axis is longer than kBfMax or a decomposition fails.
static iga_status build_bfdm(Batch &b, const iga_desc *descs) {
  const int n = b.n;
  struct Prob {
    int n, p, lo, m;
    const std::vector<double> *bm, *ba;
  };
  std::map<std::vector<double>, int> keymap;
  std::vector<Prob> probs;
  std::vector<int> key(2 * n), lo(2 * n), mm(2 * n);
  for (int k = 0; k < n; ++k) {
    const Handle &h = *b.hs[k];
    const DevProblem &pb = h.pb;
    for (int d = 0; d < 2; ++d) {
      const int nn = pb.n[d];
      const int l = ((pb.dmask >> (2 * d)) & 1u) ? 1 : 0;
      const int m = nn - (((pb.dmask >> (2 * d + 1)) & 1u) ? 1 : 0) - l;
      if (m < 1 || m > kBfMax || h.hsepM[d].empty()) return IGA_OK;
      std::vector<double> sig = {(double)nn, (double)pb.p, (double)l, (double)m};
      sig.insert(sig.end(), h.hsepM[d].begin(), h.hsepM[d].end());
      sig.insert(sig.end(), h.hsepA[d].begin(), h.hsepA[d].end());
      auto it = keymap.find(sig);
      int id;
      if (it == keymap.end()) {
        id = (int)probs.size();
        keymap.emplace(std::move(sig), id);
        probs.push_back(Prob{nn, pb.p, l, m, &h.hsepM[d], &h.hsepA[d]});
      } else {
        id = it->second;
      }
      key[2 * k + d] = id;
      lo[2 * k + d] = l;
      mm[2 * k + d] = m;
    }
  }
  const int np = (int)probs.size();
  std::vector<std::vector<double>> V(np), mu(np), rs(np);
  std::vector<char> ok(np, 0);
  std::atomic<int> next(0);
  auto worker = [&]() {
    for (int j; (j = next++) < np;) {
      const Prob &q = probs[j];
      const int W = 2 * q.p + 1, m = q.m;
      std::vector<double> A((size_t)m * m, 0.0), M((size_t)m * m, 0.0), r(q.n, 0.0);
      for (int i = 0; i < q.n; ++i)
        for (int o = 0; o < W; ++o) {
          const int jj = i + o - q.p;
          if (jj < 0 || jj >= q.n) continue;
          r[i] += (*q.bm)[(size_t)i * W + o];
          if (i < q.lo || i >= q.lo + m || jj < q.lo || jj >= q.lo + m) continue;
          A[(size_t)(i - q.lo) * m + (jj - q.lo)] = (*q.ba)[(size_t)i * W + o];
          M[(size_t)(i - q.lo) * m + (jj - q.lo)] = (*q.bm)[(size_t)i * W + o];
        }
      rs[j] = r;
      ok[j] = gen_eigen(A, M, m, V[j], mu[j]) ? 1 : 0;
    }
  };
  const unsigned hw = std::thread::hardware_concurrency();
  const int nth = (int)std::min<unsigned>(8u, hw > 0 ? hw : 1u);
  std::vector<std::thread> th;
  for (int i = 1; i < nth; ++i) th.emplace_back(worker);
  worker();
  for (auto &t : th) t.join();
  for (int j = 0; j < np; ++j)
    if (!ok[j]) return IGA_OK;
  std::vector<double> pool;
  std::vector<int64_t> otf(np), otb(np), ors(np);
  for (int j = 0; j < np; ++j) {
    const int m = probs[j].m;
    otf[j] = (int64_t)pool.size();
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < m; ++k) pool.push_back(V[j][(size_t)k * m + i]);   // V^T
    otb[j] = (int64_t)pool.size();
    pool.insert(pool.end(), V[j].begin(), V[j].end());                      // V
    ors[j] = (int64_t)pool.size();
    pool.insert(pool.end(), rs[j].begin(), rs[j].end());
  }
  std::vector<BfInst> bf(n);
  int64_t box = 0;
  for (int k = 0; k < n; ++k) {
    const DevProblem &pb = b.hs[k]->pb;
    const iga_desc &dk = descs[b.perm_[k]];
    double a = 1.0;
    if (dk.kappa_mode == IGA_KAPPA_ELEMENT && dk.kappa) {
      double s = 0;
      for (int64_t e = 0; e < pb.E; ++e) s += dk.kappa[e];
      a = s / (double)pb.E;
      if (!(a > 0) || !std::isfinite(a)) return IGA_OK;
    }
    BfInst B{};
    const int j0 = key[2 * k], j1 = key[2 * k + 1];
    B.m0 = mm[2 * k];
    B.m1 = mm[2 * k + 1];
    B.lo0 = lo[2 * k];
    B.lo1 = lo[2 * k + 1];
    B.n0 = pb.n[0];
    B.tf0 = otf[j0];
    B.tb0 = otb[j0];
    B.tf1 = otf[j1];
    B.tb1 = otb[j1];
    B.rs0 = ors[j0];
    B.rs1 = ors[j1];
    double mn0 = mu[j0][0], mn1 = mu[j1][0];
    B.mu0 = (int64_t)pool.size();
    for (double v : mu[j0]) { pool.push_back(a * v); mn0 = std::min(mn0, v); }
    B.mu1 = (int64_t)pool.size();
    for (double v : mu[j1]) { pool.push_back(a * v); mn1 = std::min(mn1, v); }
    B.mu_min = a * (mn0 + mn1);
    B.box = box;
    box += (int64_t)B.m0 * B.m1;
    bf[k] = B;
    for (int c = 0; c < B.m1; c += kBfTC) b.bf_w0.push_back(Pair{k, c});
    for (int c = 0; c < B.m0; c += kBfTC) b.bf_w1.push_back(Pair{k, c});
  }
  iga_status st;
  if ((st = bupload(b, &b.d_bf, bf)) || (st = bupload(b, &b.bf_pool, pool)) || (st = bupload(b, &b.d_bf_w0, b.bf_w0)) ||
      (st = bupload(b, &b.d_bf_w1, b.bf_w1)) || (st = balloc(b, &b.bf_shift, (size_t)n)) ||
      (st = balloc(b, &b.bf_w, 2 * (size_t)box)))
    return st;
  b.bf_box_total = box;
  b.bf_on = true;
  return IGA_OK;
}

// z = P^{-1} r for every active instance (skipping those whose CG has converged when rr_cur is given)
static void launch_bf_apply(Batch &b, const double *r, double *z, const double *rr_cur, hipStream_t s) {
  double *w1 = b.bf_w, *w2 = b.bf_w + b.bf_box_total;
  const unsigned nvt = (unsigned)b.vt.size(), n0 = (unsigned)b.bf_w0.size(), n1 = (unsigned)b.bf_w1.size();
  hipLaunchKernelGGL(k_b_copy_pc, dim3(nvt), dim3(kVT), 0, s, b.d_vt, b.d_vt_start, b.d_off, b.act, b.target, rr_cur, r,
                     z);
  hipLaunchKernelGGL(k_bf_axis<0>, dim3(n0), dim3(256), 0, s, b.d_bf_w0, b.d_bf, b.bf_pool, b.d_off, b.act,
                     b.d_vt_start, b.target, rr_cur, r, 1, w1, 0, 1, 0, b.bf_shift);
  hipLaunchKernelGGL(k_bf_axis<1>, dim3(n1), dim3(256), 0, s, b.d_bf_w1, b.d_bf, b.bf_pool, b.d_off, b.act,
                     b.d_vt_start, b.target, rr_cur, (const double *)w1, 0, w2, 0, 1, 1, b.bf_shift);
  hipLaunchKernelGGL(k_bf_axis<1>, dim3(n1), dim3(256), 0, s, b.d_bf_w1, b.d_bf, b.bf_pool, b.d_off, b.act,
                     b.d_vt_start, b.target, rr_cur, (const double *)w2, 0, w1, 0, 0, 0, b.bf_shift);
  hipLaunchKernelGGL(k_bf_axis<0>, dim3(n0), dim3(256), 0, s, b.d_bf_w0, b.d_bf, b.bf_pool, b.d_off, b.act,
                     b.d_vt_start, b.target, rr_cur, (const double *)w1, 0, z, 1, 0, 0, b.bf_shift);
}

static iga_status batch_create(int n, const iga_desc *descs, void *stream, Batch **out) {
  if (n <= 0 || !descs || !out) return fail(IGA_EINVAL, "bad batch arguments");
  Batch *b = new Batch();
  b->n = n;
  b->user = (hipStream_t)stream;
  if (hipStreamCreateWithFlags(&b->bs, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return fail(IGA_EHIP, "stream creation failed");
  }
  iga_status st = IGA_OK;
  // instances sorted by (degree, size class) so that groups are contiguous; `perm[k]` is the
  // caller's index of internal instance k
  std::vector<Handle *> hs_user(n, nullptr);
  for (int i = 0; i < n; ++i) {
    if (descs[i].dim != 2) { st = fail(IGA_EUNSUPPORTED, "batched solves are 2D"); break; }
    if (descs[i].periodic[0] || descs[i].periodic[1] || descs[i].periodic[2]) {
      st = fail(IGA_EUNSUPPORTED, "batched solves use open axes");
      break;
    }
    if (descs[i].ctrl || descs[i].weights || descs[i].kappa_mode == IGA_KAPPA_NODAL) {
      st = fail(IGA_EUNSUPPORTED, "batched solves use the identity geometry without weights");
      break;
    }
    Handle *h = nullptr;
    if ((st = create_impl(&descs[i], b->bs, &h))) break;
    if (!h->pb.simple_knots) {
      iga_destroy((iga_t)h);
      st = fail(IGA_EUNSUPPORTED, "batched solves need simple interior knots");
      break;
    }
    hs_user[i] = h;
  }
  if (st) {
    for (Handle *h : hs_user)
      if (h) iga_destroy((iga_t)h);
    (void)hipStreamDestroy(b->bs);
    delete b;
    return st;
  }
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  std::stable_sort(perm.begin(), perm.end(), [&](int x, int y) {
    int px = hs_user[x]->pb.P, py = hs_user[y]->pb.P;
    if (px != py) return px < py;
    return size_class(hs_user[x]->pb.N) < size_class(hs_user[y]->pb.N);
  });
  b->hs.resize(n);
  std::vector<int64_t> uoff(n + 1, 0), unoff(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    uoff[i + 1] = uoff[i] + hs_user[i]->pb.N;
    unoff[i + 1] = unoff[i] + hs_user[i]->pb.nnz;
  }
  b->off.resize(n);
  b->noff.resize(n);
  std::vector<DevProblem> pbs(n);
  for (int k = 0; k < n; ++k) {
    b->hs[k] = hs_user[perm[k]];
    b->off[k] = uoff[perm[k]];
    b->noff[k] = unoff[perm[k]];
    pbs[k] = b->hs[k]->pb;
  }
  b->Ntot = uoff[n];
  b->nnztot = unoff[n];
  b->perm_ = perm;
  // groups
  for (int k = 0; k < n; ++k) {
    int P = b->hs[k]->pb.P, cls = size_class(b->hs[k]->pb.N);
    if (b->groups.empty() || b->groups.back().P != P || b->groups.back().cls != cls) {
      Group g;
      g.P = P;
      g.cls = cls;
      b->groups.push_back(g);
    }
    b->groups.back().insts.push_back(k);
  }
  // vector tiles
  b->vt_start.assign(n + 1, 0);
  for (int k = 0; k < n; ++k) {
    b->vt_start[k] = (int)b->vt.size();
    for (int64_t s0 = 0; s0 < b->hs[k]->pb.N; s0 += kVT)
      b->vt.push_back(Tile{k, (int)s0, (int)std::min<int64_t>(kVT, b->hs[k]->pb.N - s0)});
  }
  b->vt_start[n] = (int)b->vt.size();
  const size_t nvt = b->vt.size();
  if ((st = bupload(*b, &b->d_pbs, pbs)) || (st = bupload(*b, &b->d_off, b->off)) ||
      (st = bupload(*b, &b->d_noff, b->noff)) || (st = bupload(*b, &b->d_vt, b->vt)) ||
      (st = bupload(*b, &b->d_vt_start, b->vt_start)) || (st = balloc(*b, &b->ws, 6 * (size_t)b->Ntot)) ||
      (st = balloc(*b, &b->dinv, (size_t)b->Ntot)) || (st = balloc(*b, &b->partA, nvt)) ||
      (st = balloc(*b, &b->partB, nvt)) || (st = balloc(*b, &b->partC, nvt)) || (st = balloc(*b, &b->partD, nvt)) ||
      (st = balloc(*b, &b->norms, (size_t)n)) || (st = balloc(*b, &b->target, (size_t)n)) ||
      (st = balloc(*b, &b->act, (size_t)n)) || (st = balloc(*b, &b->iters, (size_t)n)) ||
      (st = balloc(*b, &b->count, 1)) || (st = balloc(*b, &b->flags, (size_t)n)) ||
      (st = balloc(*b, &b->nprm, 4)) || (st = balloc(*b, &b->r0, (size_t)n)) || (st = balloc(*b, &b->nr_prev, (size_t)n)) ||
      (st = balloc(*b, &b->eta, (size_t)n)) || (st = balloc(*b, &b->hist, (size_t)n * kHist)) ||
      (st = balloc(*b, &b->conv, (size_t)n)) || (st = balloc(*b, &b->hcount, (size_t)n)) ||
      (st = balloc(*b, &b->kstep, 1)) || (st = balloc(*b, &b->nact, 2))) {
    batch_free(b);
    return st;
  }
  void *vals = nullptr;
  if (hipMalloc(&vals, (size_t)b->nnztot * sizeof(double)) != hipSuccess) {
    batch_free(b);
    return fail(IGA_ENOMEM, "batch Jacobian values");
  }
  b->owned.push_back(vals);
  b->vals = vals;
  b->vals_prec = IGA_FP64;
  for (Group &g : b->groups) {
    g.res_tiles = g.P >= 2 && g.P <= 5;
    for (int k : g.insts) g.res_tiles = g.res_tiles && res2_supported(b->hs[k]->pb);
    if ((st = build_elems(*b, g))) {
      batch_free(b);
      return st;
    }
  }
  std::vector<int> ones(n, 1);
  std::vector<double> tz(n, -1.0);
  if ((st = [&]() -> iga_status {
        IGA_HIP_CHECK(hipMemcpyAsync(b->act, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, b->bs));
        IGA_HIP_CHECK(hipMemcpyAsync(b->target, tz.data(), n * sizeof(double), hipMemcpyHostToDevice, b->bs));
        // defined partials: the shape tuner runs the SpMV before any CG state exists
        IGA_HIP_CHECK(hipMemsetAsync(b->partA, 0, nvt * sizeof(double), b->bs));
        IGA_HIP_CHECK(hipMemsetAsync(b->partC, 0, nvt * sizeof(double), b->bs));
        return IGA_OK;
      }())) {
    batch_free(b);
    return st;
  }
  if ((st = build_bfdm(*b, descs))) {
    batch_free(b);
    return st;
  }
  if ((st = autotune(*b))) {
    batch_free(b);
    return st;
  }
  if (hipStreamSynchronize(b->bs) != hipSuccess) {
    batch_free(b);
    return fail(IGA_EHIP, "batch setup");
  }
  *out = b;
  return IGA_OK;
}

// `chunk` CG iterations of every instance, then the count of instances whose CG has not converged
// (recorded into the capturing stream)
static void record_cg_chunk(Batch &b, int prec, int chunk, bool fdm) {
  const int64_t N = b.Ntot;
  double *d = b.ws + N, *r = b.ws + 2 * N, *z = b.ws + 3 * N, *p = b.ws + 4 * N, *q = b.ws + 5 * N;
  const unsigned nvt = (unsigned)b.vt.size();
  // partial buffers: rz in A/B, rr in C/D; iteration k reads (A,C) or (B,D) alternately
  for (int it = 0; it < chunk; ++it) {
    double *rz_cur = (it % 2 == 0) ? b.partA : b.partB, *rz_new = (it % 2 == 0) ? b.partB : b.partA;
    double *rr_cur = (it % 2 == 0) ? b.partC : b.partD, *rr_new = (it % 2 == 0) ? b.partD : b.partC;
    for (size_t gi = 0; gi < b.groups.size(); ++gi) {
      if (prec == IGA_FP32) launch_spmv_group<float>(b, gi, (const float *)b.vals, p, q, rr_cur, b.bs);
      else launch_spmv_group<double>(b, gi, (const double *)b.vals, p, q, rr_cur, b.bs);
    }
    hipLaunchKernelGGL(k_b_cg_xr, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_vt_start, b.d_st_start, b.d_off, b.act,
                       b.target, rz_cur, rr_cur, b.part_pq, d, r, z, p, q, fdm ? nullptr : b.dinv, rz_new,
                       rr_new);
    if (fdm) {
      launch_bf_apply(b, r, z, rr_cur, b.bs);
      hipLaunchKernelGGL(k_b_rz, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_vt_start, b.d_off, b.act, b.target, rr_cur,
                         rz_cur, (const double *)r, (const double *)z, rz_new);
    }
    hipLaunchKernelGGL(k_b_cg_p, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_vt_start, b.d_off, b.act, b.target,
                       rz_cur, rr_cur, rz_new, z, p, b.iters);
  }
  hipLaunchKernelGGL(k_b_flags, dim3((unsigned)((b.n + 3) / 4)), dim3(256), 0, b.bs, b.n, b.d_vt_start, b.act,
                     b.target, b.partC, b.flags);
  hipLaunchKernelGGL(k_b_count, dim3(1), dim3(256), 0, b.bs, b.n, (const int *)b.flags, b.count);
}

static iga_status end_capture(Batch &b, hipGraphExec_t *out) {
  hipGraph_t g;
  hipError_t e = hipStreamEndCapture(b.bs, &g);
  if (e != hipSuccess) return fail(IGA_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(IGA_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
  return IGA_OK;
}

static iga_status capture_cg_graph(Batch &b, int prec, int chunk, bool fdm) {
  if (b.graph && b.graph_prec == prec && b.graph_chunk == chunk && b.graph_fdm == fdm) return IGA_OK;
  if (b.graph) {
    (void)hipGraphExecDestroy(b.graph);
    b.graph = nullptr;
  }
  IGA_HIP_CHECK(hipStreamBeginCapture(b.bs, hipStreamCaptureModeThreadLocal));
  record_cg_chunk(b, prec, chunk, fdm);
  iga_status st = end_capture(b, &b.graph);
  if (st) return st;
  b.graph_prec = prec;
  b.graph_chunk = chunk;
  b.graph_fdm = fdm;
  return IGA_OK;
}

// One whole Newton step of every instance as one graph: U += d (the previous step's correction, on
// the instances that solved for it), the residual and its norms, the device-side Newton control
// (stopping test and CG targets), the Jacobian, the preconditioner set-up, the CG start and one chunk
// of CG iterations.  Kernels skip instances that are done (act = 0), so the same graph serves every
// step; the host reads two counters per step.
static iga_status capture_step_graph(Batch &b, const double *Uc, int prec, int chunk, bool fdm) {
  if (b.step_graph && b.step_U == Uc && b.step_prec == prec && b.step_chunk == chunk && b.step_fdm == fdm)
    return IGA_OK;
  if (b.step_graph) {
    (void)hipGraphExecDestroy(b.step_graph);
    b.step_graph = nullptr;
  }
  double *U = const_cast<double *>(Uc);
  const int n = b.n;
  const int64_t N = b.Ntot;
  double *R = b.ws, *d = b.ws + N;
  const unsigned nvt = (unsigned)b.vt.size();
  IGA_HIP_CHECK(hipStreamBeginCapture(b.bs, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_b_axpy, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, (const double *)d, U);
  hipLaunchKernelGGL(k_b_fill, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, R, 0.0);
  for (const Group &g : b.groups) launch_res(b, g, U, R, b.bs);
  hipLaunchKernelGGL(k_b_bc_copy, dim3(nvt), dim3(kVT), 0, b.bs, b.d_pbs, b.d_vt, b.d_off, b.act, (const double *)U, R);
  hipLaunchKernelGGL(k_b_sq_partial, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, (const double *)R, b.partA);
  hipLaunchKernelGGL(k_b_inst_norms, dim3(std::min(n, 1024)), dim3(256), 0, b.bs, n, b.d_vt_start,
                     (const double *)b.partA, b.norms);
  hipLaunchKernelGGL(k_b_newton_ctl, dim3(1), dim3(1024), 0, b.bs, n, (const double *)b.norms,
                     (const double *)b.nprm, b.act, b.target, b.r0, b.nr_prev, b.eta, b.conv, b.hcount, b.hist,
                     b.kstep, b.nact);
  for (const Group &g : b.groups) launch_rg(b, g, g.b1, U, b.vals, prec, b.bs);
  if (fdm) {
    hipLaunchKernelGGL(k_bf_shift, dim3((unsigned)n), dim3(256), 0, b.bs, b.d_pbs, b.d_bf, (const double *)b.bf_pool,
                       b.d_off, b.act, (const double *)U, b.bf_shift);
  } else if (prec == IGA_FP32) {
    hipLaunchKernelGGL(k_b_diag_inv<float>, dim3(nvt), dim3(kVT), 0, b.bs, b.d_pbs, b.d_vt, b.d_off, b.d_noff, b.act,
                       (const float *)b.vals, b.dinv);
  } else {
    hipLaunchKernelGGL(k_b_diag_inv<double>, dim3(nvt), dim3(kVT), 0, b.bs, b.d_pbs, b.d_vt, b.d_off, b.d_noff,
                       b.act, (const double *)b.vals, b.dinv);
  }
  hipLaunchKernelGGL(k_b_cg_init, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, (const double *)R,
                     fdm ? nullptr : (const double *)b.dinv, d, b.ws + 2 * N, b.ws + 3 * N, b.ws + 4 * N,
                     b.partA, b.partC);
  if (fdm) {
    launch_bf_apply(b, b.ws + 2 * N, b.ws + 3 * N, nullptr, b.bs);
    hipLaunchKernelGGL(k_b_pz, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, (const double *)(b.ws + 2 * N),
                       (const double *)(b.ws + 3 * N), b.ws + 4 * N, b.partA);
  }
  record_cg_chunk(b, prec, chunk, fdm);
  iga_status st = end_capture(b, &b.step_graph);
  if (st) return st;
  b.step_U = Uc;
  b.step_prec = prec;
  b.step_chunk = chunk;
  b.step_fdm = fdm;
  return IGA_OK;
}

// Newton on every instance: one replay of the step graph per Newton step, plus replays of the
// CG-chunk graph while some instance's CG has not met its target; the host reads the number of
// active instances and of unconverged CG solves once per replay.
static iga_status batch_newton(Batch &b, double *U, const iga_newton_opts *o_in, iga_batch_item_report *items,
                               iga_batch_report *rep) {
  iga_newton_opts o{};
  o.atol = 1e-10;
  o.max_newton = 30;
  o.max_krylov = 5000;
  o.jac_prec = IGA_FP64;
  o.forcing_max = 1e-2;
  if (o_in) o = *o_in;
  if (o.matrix_free) return fail(IGA_EUNSUPPORTED, "batched solves use the assembled Jacobian");
  if (o.jac_prec != IGA_FP64 && o.jac_prec != IGA_FP32) return fail(IGA_EUNSUPPORTED, "Jacobian precision");
  if (o.max_newton < 0 || o.max_newton > 64) return fail(IGA_EINVAL, "max_newton must be in 0..64");
  if (o.forcing_max <= 0) o.forcing_max = 1e-2;
  const int n = b.n;
  const int64_t N = b.Ntot;
  const unsigned nvt = (unsigned)b.vt.size();
  iga_batch_report r{};
  r.t_tune_ms = b.t_tune_ms;
  auto t0 = std::chrono::steady_clock::now();
  IGA_HIP_CHECK(hipStreamSynchronize(b.user));
  const bool fdm = b.bf_on && b.precond != IGA_PRECOND_JACOBI;
  const int chunk = o.check_every > 0 ? std::min(64, (o.check_every + 1) & ~1) : (fdm ? kChunkFdm : kChunkJacobi);
  iga_status st = capture_cg_graph(b, o.jac_prec, chunk, fdm);
  if (st) return st;
  if ((st = capture_step_graph(b, U, o.jac_prec, chunk, fdm))) return st;
  // device-side Newton state: every instance active, zero correction, no history
  const double prm[4] = {o.atol, o.rtol, o.forcing_max, (double)o.max_newton};
  std::vector<int> ones(n, 1), zeros(n, 0);
  std::vector<double> mone(n, -1.0), fmx(n, o.forcing_max);
  IGA_HIP_CHECK(hipMemcpyAsync(b.nprm, prm, sizeof(prm), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.act, ones.data(), n * sizeof(int), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.conv, zeros.data(), n * sizeof(int), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.hcount, zeros.data(), n * sizeof(int), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.iters, zeros.data(), n * sizeof(int), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.r0, mone.data(), n * sizeof(double), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.eta, fmx.data(), n * sizeof(double), hipMemcpyHostToDevice, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(b.kstep, zeros.data(), sizeof(int), hipMemcpyHostToDevice, b.bs));
  hipLaunchKernelGGL(k_b_fill, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, b.ws + N, 0.0);   // d = 0
  IGA_HIP_CHECK(hipGetLastError());
  hipEvent_t ev[3];
  for (auto &e : ev) IGA_HIP_CHECK(hipEventCreate(&e));
  int k = 0;
  for (;; ++k) {
    int ctr[2] = {0, 0};   // active instances, unconverged CG solves
    (void)hipEventRecord(ev[0], b.bs);
    IGA_HIP_CHECK(hipGraphLaunch(b.step_graph, b.bs));
    (void)hipEventRecord(ev[1], b.bs);
    IGA_HIP_CHECK(hipMemcpyAsync(&ctr[0], b.nact, sizeof(int), hipMemcpyDeviceToHost, b.bs));
    IGA_HIP_CHECK(hipMemcpyAsync(&ctr[1], b.count, sizeof(int), hipMemcpyDeviceToHost, b.bs));
    IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
    r.graph_launches += 1;
    r.t_jacobian_ms += elapsed(ev[0], ev[1]);
    if (ctr[0] == 0) break;
    int done_iters = chunk, remaining = ctr[1];
    (void)hipEventRecord(ev[1], b.bs);
    while (done_iters < o.max_krylov && remaining > 0) {
      IGA_HIP_CHECK(hipGraphLaunch(b.graph, b.bs));
      IGA_HIP_CHECK(hipMemcpyAsync(&remaining, b.count, sizeof(int), hipMemcpyDeviceToHost, b.bs));
      IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
      done_iters += chunk;
      r.graph_launches += 1;
    }
    (void)hipEventRecord(ev[2], b.bs);
    IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
    r.t_krylov_ms += elapsed(ev[1], ev[2]);
    r.krylov_iters_max += done_iters;
  }
  std::vector<int> dev_iters(n), conv(n), hcount(n);
  std::vector<double> r0(n), hist((size_t)n * kHist);
  IGA_HIP_CHECK(hipMemcpyAsync(dev_iters.data(), b.iters, n * sizeof(int), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(conv.data(), b.conv, n * sizeof(int), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(hcount.data(), b.hcount, n * sizeof(int), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(r0.data(), b.r0, n * sizeof(double), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipMemcpyAsync(hist.data(), b.hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
  for (auto &e : ev) (void)hipEventDestroy(e);
  r.newton_steps = k;
  r.all_converged = 1;
  for (int kk = 0; kk < n; ++kk) {
    r.all_converged &= conv[kk];
    if (items) {
      iga_batch_item_report &it = items[b.perm_[kk]];
      it.converged = conv[kk];
      it.newton_iters = hcount[kk] - 1;
      it.krylov_iters = dev_iters[kk];
      it.res_norm0 = r0[kk];
      it.res_norm = hcount[kk] > 0 ? hist[(size_t)kk * kHist + std::min(hcount[kk], kHist) - 1] : 0.0;
    }
  }
  r.t_total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rep) *rep = r;
  return r.all_converged ? IGA_OK : fail(IGA_ENOCONV, "some batched instances did not converge");
}

// Per instance, ||P^{-1} R(U)||_2 with P the fast-diagonalisation operator whose reaction shift is
// taken at U: the first Newton correction as the preconditioner approximates it, an estimate of
// ||U - U*|| that needs no solve.  Used to judge an initial guess: its residual norm is dominated
// by the high-frequency part of its error, which the stiffness amplifies, while this estimate weighs
// every frequency of the error alike (exactly so where P is the exact Jacobian).  est_host gets one
// value per instance in the caller's order.  Uses the residual and correction slots of the solve
// workspace; runs on the batch stream after the caller's stream, and returns once done.
static iga_status batch_error_estimates(Batch &b, const double *U, double *est_host) {
  if (!b.bf_on) return fail(IGA_EUNSUPPORTED, "error estimates need the fast-diagonalisation preconditioner");
  const int n = b.n;
  const int64_t N = b.Ntot;
  double *R = b.ws, *z = b.ws + N;
  const unsigned nvt = (unsigned)b.vt.size();
  IGA_HIP_CHECK(hipStreamSynchronize(b.user));
  std::vector<int> act(n, 1);
  std::vector<double> nr(n);
  IGA_HIP_CHECK(hipMemcpyAsync(b.act, act.data(), n * sizeof(int), hipMemcpyHostToDevice, b.bs));
  hipLaunchKernelGGL(k_b_fill, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, b.act, R, 0.0);
  for (const Group &g : b.groups) launch_res(b, g, U, R, b.bs);
  hipLaunchKernelGGL(k_b_bc_copy, dim3(nvt), dim3(kVT), 0, b.bs, b.d_pbs, b.d_vt, b.d_off, b.act, U, R);
  hipLaunchKernelGGL(k_bf_shift, dim3((unsigned)n), dim3(256), 0, b.bs, b.d_pbs, b.d_bf, (const double *)b.bf_pool,
                     b.d_off, b.act, U, b.bf_shift);
  launch_bf_apply(b, R, z, nullptr, b.bs);
  hipLaunchKernelGGL(k_b_sq_partial, dim3(nvt), dim3(kVT), 0, b.bs, b.d_vt, b.d_off, (const double *)z, b.partA);
  hipLaunchKernelGGL(k_b_inst_norms, dim3(std::min(n, 1024)), dim3(256), 0, b.bs, n, b.d_vt_start,
                     (const double *)b.partA, b.norms);
  IGA_HIP_CHECK(hipGetLastError());
  IGA_HIP_CHECK(hipMemcpyAsync(nr.data(), b.norms, n * sizeof(double), hipMemcpyDeviceToHost, b.bs));
  IGA_HIP_CHECK(hipStreamSynchronize(b.bs));
  for (int k = 0; k < n; ++k) est_host[b.perm_[k]] = nr[k];
  return IGA_OK;
}

}  // namespace iga

using namespace iga;

extern "C" {

iga_status iga_batch_create(int n, const iga_desc *descs, void *hip_stream, iga_batch_t *out) {
  if (!out) return fail(IGA_EINVAL, "null output");
  *out = nullptr;
  Batch *b = nullptr;
  iga_status st = batch_create(n, descs, hip_stream, &b);
  if (st) return st;
  *out = (iga_batch_t)b;
  return IGA_OK;
}

iga_status iga_batch_info(iga_batch_t bb, int64_t *total_ndof, int64_t *total_nnz, int64_t *dof_offsets) {
  if (!bb) return fail(IGA_EINVAL, "null batch");
  Batch *b = (Batch *)bb;
  if (total_ndof) *total_ndof = b->Ntot;
  if (total_nnz) *total_nnz = b->nnztot;
  if (dof_offsets) {
    std::vector<int64_t> o(b->n + 1, 0);
    for (int k = 0; k < b->n; ++k) o[b->perm_[k]] = b->off[k];
    o[b->n] = b->Ntot;
    for (int i = 0; i <= b->n; ++i) dof_offsets[i] = o[i];
  }
  return IGA_OK;
}

iga_status iga_batch_newton_solve(iga_batch_t bb, double *U_dev, const iga_newton_opts *opts,
                                  iga_batch_item_report *items, iga_batch_report *report) {
  if (!bb || !U_dev) return fail(IGA_EINVAL, "null argument");
  return batch_newton(*(Batch *)bb, U_dev, opts, items, report);
}

iga_status iga_batch_error_estimates(iga_batch_t bb, const double *U_dev, double *est_host) {
  if (!bb || !U_dev || !est_host) return fail(IGA_EINVAL, "null argument");
  return batch_error_estimates(*(Batch *)bb, U_dev, est_host);
}

iga_status iga_batch_set_option(iga_batch_t bb, int key, int64_t value) {
  if (!bb) return fail(IGA_EINVAL, "null batch");
  Batch *b = (Batch *)bb;
  if (key != IGA_OPT_PRECOND) return fail(IGA_EINVAL, "batched solves take IGA_OPT_PRECOND only");
  if (value < IGA_PRECOND_AUTO || value > IGA_PRECOND_FDM) return fail(IGA_EINVAL, "bad preconditioner");
  if (value == IGA_PRECOND_FDM && !b->bf_on)
    return fail(IGA_EUNSUPPORTED, "fast diagonalisation needs every axis of every instance within 136 coefficients");
  b->precond = (int)value;
  return IGA_OK;
}

iga_status iga_batch_destroy(iga_batch_t bb) {
  batch_free((Batch *)bb);
  return IGA_OK;
}

}  // extern "C"
