// Learned initial guess: a 4-layer convolutional encoder-decoder that maps (log kappa, lambda)
// on a 32x32 grid to the 65x65 interior spline coefficients of the 64x64-element, degree-3
// problem.  BF16 weights and activations, FP32 accumulation, FP32 master weights, Adam.
//
//   x  [2][32][32]  -> conv 3x3 s1 p1 (2->64)   + ReLU -> a1 [64][32][32]
//                  -> conv 3x3 s2 p1 (64->64)  + ReLU -> a2 [64][16][16]
//                  -> global context: g = a2 + mean over the 16x16 pixels (per channel)
//                  -> convT 4x4 s4 (64->64)    + ReLU -> a3 [64][64][64]
//                  -> convT 2x2 s1 (64->1)            -> y  [65][65]
// Convolutions are cross-correlations; a transposed convolution adds W[ci][co][ky][kx] in
// at output (iy*s + ky, ix*s + kx).  Parameters are one flat FP32 vector
// [W0 b0 W1 b1 W2 b2 W3 b3] with W0, W1 as [co][ci][ky][kx] and W2, W3 as [ci][co][ky][kx].
#include <hip/hip_bfloat16.h>

#include <cmath>
#include <vector>

#include "iga_impl.h"

namespace iga {
namespace {

typedef unsigned short bf16_t;   // raw BF16 bits

__device__ inline float bf2f(bf16_t b) {
  unsigned u = ((unsigned)b) << 16;
  return __uint_as_float(u);
}
// round to nearest even (finite inputs)
__device__ inline bf16_t f2bf(float f) {
  unsigned u = __float_as_uint(f);
  unsigned r = ((u >> 16) & 1u) + 0x7fffu;
  return (bf16_t)((u + r) >> 16);
}

constexpr int C = 64;
constexpr int NP_W0 = C * 2 * 9, NP_W1 = C * C * 9, NP_W2 = C * C * 16, NP_W3 = C * 4;
constexpr int O_W0 = 0, O_B0 = O_W0 + NP_W0, O_W1 = O_B0 + C, O_B1 = O_W1 + NP_W1, O_W2 = O_B1 + C,
              O_B2 = O_W2 + NP_W2, O_W3 = O_B2 + C, O_B3 = O_W3 + NP_W3, NPARAM = O_B3 + 1;
constexpr int H0 = 32, H1 = 32, H2 = 16, H3 = 64, H4 = 65;

inline unsigned nblk(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_to_bf16(const float *__restrict__ x, bf16_t *__restrict__ y, long n) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// conv (stride S, pad PD), ReLU, BF16 out; one thread per output element
template <int CIN, int HIN, int HOUT, int S>
__global__ void k_conv_fwd(int B, const bf16_t *__restrict__ in, const bf16_t *__restrict__ W,
                           const float *__restrict__ bias, bf16_t *__restrict__ out) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * C * HOUT * HOUT) return;
  int ox = i % HOUT, oy = (i / HOUT) % HOUT, co = (i / (HOUT * HOUT)) % C;
  long n = i / ((long)C * HOUT * HOUT);
  float s = bias[co];
  for (int ci = 0; ci < CIN; ++ci) {
    const bf16_t *ip = in + ((n * CIN + ci) * HIN) * HIN;
    const bf16_t *wp = W + (co * CIN + ci) * 9;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      int iy = oy * S + ky - 1;
      if (iy < 0 || iy >= HIN) continue;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        int ix = ox * S + kx - 1;
        if (ix < 0 || ix >= HIN) continue;
        s += bf2f(wp[ky * 3 + kx]) * bf2f(ip[iy * HIN + ix]);
      }
    }
  }
  out[i] = f2bf(s > 0.f ? s : 0.f);
}

// transposed conv 4x4 stride 4 (64->64): each output pixel has exactly one source pixel
__global__ void k_convT4_fwd(int B, const bf16_t *__restrict__ in, const bf16_t *__restrict__ W,
                             const float *__restrict__ bias, bf16_t *__restrict__ out) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * C * H3 * H3) return;
  int ox = i % H3, oy = (i / H3) % H3, co = (i / (H3 * H3)) % C;
  long n = i / ((long)C * H3 * H3);
  int iy = oy >> 2, ix = ox >> 2, ky = oy & 3, kx = ox & 3;
  float s = bias[co];
  const bf16_t *ip = in + n * C * H2 * H2 + iy * H2 + ix;
  const bf16_t *wp = W + co * 16 + ky * 4 + kx;
  for (int ci = 0; ci < C; ++ci) s += bf2f(wp[ci * C * 16]) * bf2f(ip[ci * H2 * H2]);
  out[i] = f2bf(s > 0.f ? s : 0.f);
}

// transposed conv 2x2 stride 1 (64->1), FP32 output (no activation)
__global__ void k_convT2_fwd(int B, const bf16_t *__restrict__ in, const bf16_t *__restrict__ W,
                             const float *__restrict__ bias, float *__restrict__ out) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * H4 * H4) return;
  int ox = i % H4, oy = (i / H4) % H4;
  long n = i / (H4 * H4);
  float s = bias[0];
  for (int ky = 0; ky < 2; ++ky) {
    int iy = oy - ky;
    if (iy < 0 || iy >= H3) continue;
    for (int kx = 0; kx < 2; ++kx) {
      int ix = ox - kx;
      if (ix < 0 || ix >= H3) continue;
      const bf16_t *ip = in + n * C * H3 * H3 + iy * H3 + ix;
      for (int ci = 0; ci < C; ++ci) s += bf2f(W[ci * 4 + ky * 2 + kx]) * bf2f(ip[ci * H3 * H3]);
    }
  }
  out[i] = s;
}

// global context: out[n][c][:] = a[n][c][:] + mean(a[n][c][:]) over the 16x16 pixels
__global__ void k_gctx_fwd(const bf16_t *__restrict__ a, bf16_t *__restrict__ out) {
  __shared__ float sh[256];
  const long base = (long)blockIdx.x * H2 * H2;     // one block per (n, c), 256 threads = 256 pixels
  float v = bf2f(a[base + threadIdx.x]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  out[base + threadIdx.x] = f2bf(v + sh[0] * (1.f / (H2 * H2)));
}

// backward of the global context and the ReLU of layer 2:
// da2 = (dg + mean(dg)) * (a2 > 0)
__global__ void k_gctx_bwd(const float *__restrict__ dg, const bf16_t *__restrict__ a2, float *__restrict__ da2) {
  __shared__ float sh[256];
  const long base = (long)blockIdx.x * H2 * H2;
  float v = dg[base + threadIdx.x];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  float d = v + sh[0] * (1.f / (H2 * H2));
  da2[base + threadIdx.x] = bf2f(a2[base + threadIdx.x]) > 0.f ? d : 0.f;
}

// y = (scale * y + mean[pixel]) * sample_scale[n] (un-standardise the network output)
__global__ void k_affine_out(int B, float *__restrict__ y, const float *__restrict__ mean, float scale,
                             const float *__restrict__ sample_scale) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * H4 * H4) return;
  float v = scale * y[i] + (mean ? mean[i % (H4 * H4)] : 0.f);
  y[i] = sample_scale ? v * sample_scale[i / (H4 * H4)] : v;
}

// one pass of the separable [1 2 1]/4 filter on the 65x65 output, zero outside (the Dirichlet
// coefficients around the interior are zero)
__global__ void k_smooth(int B, const float *__restrict__ y, float *__restrict__ out, int axis) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * H4 * H4) return;
  int x = i % H4, yy = (i / H4) % H4;
  long n = i / (H4 * H4);
  const float *p = y + n * H4 * H4;
  float c = p[yy * H4 + x], l, r;
  if (axis == 0) {
    l = x > 0 ? p[yy * H4 + x - 1] : 0.f;
    r = x < H4 - 1 ? p[yy * H4 + x + 1] : 0.f;
  } else {
    l = yy > 0 ? p[(yy - 1) * H4 + x] : 0.f;
    r = yy < H4 - 1 ? p[(yy + 1) * H4 + x] : 0.f;
  }
  out[i] = 0.25f * l + 0.5f * c + 0.25f * r;
}

// Loss = mean((y-t)^2) + beta * mean((L e)^2), e = y - t, L the 5-point discrete Laplacian on the
// 65x65 grid with zero outside (the error vanishes on the Dirichlet coefficients).  The second
// term weighs rough errors the way the stiffness part of the residual does.
__device__ inline float lap_at(const float *__restrict__ y, const float *__restrict__ t, long n, int yy, int x) {
  auto e = [&](int a, int b) -> float {
    if (a < 0 || a >= H4 || b < 0 || b >= H4) return 0.f;
    long k = n * H4 * H4 + a * H4 + b;
    return y[k] - t[k];
  };
  return 4.f * e(yy, x) - e(yy - 1, x) - e(yy + 1, x) - e(yy, x - 1) - e(yy, x + 1);
}

__global__ void k_lap_err(int B, const float *__restrict__ y, const float *__restrict__ t, float *__restrict__ l) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * H4 * H4) return;
  int x = i % H4, yy = (i / H4) % H4;
  long n = i / (H4 * H4);
  l[i] = lap_at(y, t, n, yy, x);
}

// dy = 2 e / n + beta * 2 L(l) / n ; per-block partial sums of e^2 + beta l^2
__global__ void k_mse(int B, const float *__restrict__ y, const float *__restrict__ t, const float *__restrict__ l,
                      float beta, float *__restrict__ dy, float *__restrict__ part) {
  __shared__ float sh[256];
  long n = (long)B * H4 * H4;
  float acc = 0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    int x = i % H4, yy = (i / H4) % H4;
    long s0 = (i / (H4 * H4)) * H4 * H4;
    float d = y[i] - t[i];
    float g = 2.f * d;
    if (beta != 0.f) {
      auto L = [&](int a, int b) -> float { return (a < 0 || a >= H4 || b < 0 || b >= H4) ? 0.f : l[s0 + a * H4 + b]; };
      float lap = 4.f * L(yy, x) - L(yy - 1, x) - L(yy + 1, x) - L(yy, x - 1) - L(yy, x + 1);
      g += beta * 2.f * lap;
      acc += beta * l[i] * l[i];
    }
    dy[i] = g / (float)n;
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// ---- backward: data gradients (FP32), multiplied by the ReLU mask of the layer input ----
// convT2: da3[n][ci][iy][ix] = sum_{ky,kx} W3[ci][ky][kx] dy[n][iy+ky][ix+kx]
__global__ void k_convT2_bwd_data(int B, const float *__restrict__ dy, const bf16_t *__restrict__ W,
                                  const bf16_t *__restrict__ a3, float *__restrict__ da3) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * C * H3 * H3) return;
  int ix = i % H3, iy = (i / H3) % H3, ci = (i / (H3 * H3)) % C;
  long n = i / ((long)C * H3 * H3);
  float s = 0;
  for (int ky = 0; ky < 2; ++ky)
    for (int kx = 0; kx < 2; ++kx) s += bf2f(W[ci * 4 + ky * 2 + kx]) * dy[n * H4 * H4 + (iy + ky) * H4 + ix + kx];
  da3[i] = bf2f(a3[i]) > 0.f ? s : 0.f;
}

// convT4: da2[n][ci][iy][ix] = sum_{co,ky,kx} W2[ci][co][ky][kx] dz3[n][co][4iy+ky][4ix+kx]
__global__ void k_convT4_bwd_data(int B, const float *__restrict__ dz3, const bf16_t *__restrict__ W,
                                  float *__restrict__ dg) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * C * H2 * H2) return;
  int ix = i % H2, iy = (i / H2) % H2, ci = (i / (H2 * H2)) % C;
  long n = i / ((long)C * H2 * H2);
  float s = 0;
  for (int co = 0; co < C; ++co) {
    const float *dp = dz3 + ((n * C + co) * H3 + 4 * iy) * H3 + 4 * ix;
    const bf16_t *wp = W + (ci * C + co) * 16;
#pragma unroll
    for (int ky = 0; ky < 4; ++ky)
#pragma unroll
      for (int kx = 0; kx < 4; ++kx) s += bf2f(wp[ky * 4 + kx]) * dp[ky * H3 + kx];
  }
  dg[i] = s;
}

// conv (3x3, stride S, pad 1): din[n][ci][iy][ix] = sum_{co,ky,kx} W[co][ci][ky][kx] dout[n][co][oy][ox]
// with iy = oy*S + ky - 1
template <int CIN, int HIN, int HOUT, int S>
__global__ void k_conv_bwd_data(int B, const float *__restrict__ dout, const bf16_t *__restrict__ W,
                                const bf16_t *__restrict__ ain, float *__restrict__ din) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= (long)B * CIN * HIN * HIN) return;
  int ix = i % HIN, iy = (i / HIN) % HIN, ci = (i / (HIN * HIN)) % CIN;
  long n = i / ((long)CIN * HIN * HIN);
  float s = 0;
  for (int ky = 0; ky < 3; ++ky) {
    int t = iy + 1 - ky;
    if (t < 0 || t % S) continue;
    int oy = t / S;
    if (oy >= HOUT) continue;
    for (int kx = 0; kx < 3; ++kx) {
      int u = ix + 1 - kx;
      if (u < 0 || u % S) continue;
      int ox = u / S;
      if (ox >= HOUT) continue;
      const float *dp = dout + (n * C * HOUT + oy) * HOUT + ox;
      const bf16_t *wp = W + ci * 9 + ky * 3 + kx;
      for (int co = 0; co < C; ++co) s += bf2f(wp[co * CIN * 9]) * dp[(long)co * HOUT * HOUT];
    }
  }
  din[i] = bf2f(ain[i]) > 0.f ? s : 0.f;
}

// ---- weight gradients: one block per weight, reduction over (n, output pixels) ----
__device__ inline float block_reduce(float v, float *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

template <int CIN, int HIN, int HOUT, int S>
__global__ void k_conv_bwd_w(int B, const float *__restrict__ dout, const bf16_t *__restrict__ ain,
                             float *__restrict__ dW, float *__restrict__ db) {
  __shared__ float sh[256];
  const int w = blockIdx.x;                 // [co][ci][ky][kx]
  const int kx = w % 3, ky = (w / 3) % 3, ci = (w / 9) % CIN, co = w / (9 * CIN);
  const long tot = (long)B * HOUT * HOUT;
  float s = 0, sb = 0;
  for (long j = threadIdx.x; j < tot; j += blockDim.x) {
    int ox = j % HOUT, oy = (j / HOUT) % HOUT;
    long n = j / (HOUT * HOUT);
    float d = dout[((n * C + co) * HOUT + oy) * HOUT + ox];
    int iy = oy * S + ky - 1, ix = ox * S + kx - 1;
    if (iy >= 0 && iy < HIN && ix >= 0 && ix < HIN) s += d * bf2f(ain[((n * CIN + ci) * HIN + iy) * HIN + ix]);
    sb += d;
  }
  float r = block_reduce(s, sh);
  if (threadIdx.x == 0) dW[w] = r;
  __syncthreads();
  if (ci == 0 && ky == 0 && kx == 0) {
    float rb = block_reduce(sb, sh);
    if (threadIdx.x == 0) db[co] = rb;
  }
}

// convT4: dW2[ci][co][ky][kx] = sum_{n,iy,ix} a2[n][ci][iy][ix] dz3[n][co][4iy+ky][4ix+kx]
__global__ void k_convT4_bwd_w(int B, const float *__restrict__ dz3, const bf16_t *__restrict__ a2,
                               float *__restrict__ dW, float *__restrict__ db) {
  __shared__ float sh[256];
  const int w = blockIdx.x;
  const int kx = w % 4, ky = (w / 4) % 4, co = (w / 16) % C, ci = w / (16 * C);
  const long tot = (long)B * H2 * H2;
  float s = 0;
  for (long j = threadIdx.x; j < tot; j += blockDim.x) {
    int ix = j % H2, iy = (j / H2) % H2;
    long n = j / (H2 * H2);
    s += bf2f(a2[((n * C + ci) * H2 + iy) * H2 + ix]) * dz3[((n * C + co) * H3 + 4 * iy + ky) * H3 + 4 * ix + kx];
  }
  float r = block_reduce(s, sh);
  if (threadIdx.x == 0) dW[w] = r;
  __syncthreads();
  if (ci == 0 && ky == 0 && kx == 0) {
    float sb = 0;
    const long tb = (long)B * H3 * H3;
    for (long j = threadIdx.x; j < tb; j += blockDim.x) {
      long n = j / (H3 * H3);
      sb += dz3[(n * C + co) * H3 * H3 + j % (H3 * H3)];
    }
    float rb = block_reduce(sb, sh);
    if (threadIdx.x == 0) db[co] = rb;
  }
}

// convT2: dW3[ci][ky][kx] = sum_{n,iy,ix} a3[n][ci][iy][ix] dy[n][iy+ky][ix+kx]
__global__ void k_convT2_bwd_w(int B, const float *__restrict__ dy, const bf16_t *__restrict__ a3,
                               float *__restrict__ dW, float *__restrict__ db) {
  __shared__ float sh[256];
  const int w = blockIdx.x;
  const int kx = w % 2, ky = (w / 2) % 2, ci = w / 4;
  const long tot = (long)B * H3 * H3;
  float s = 0;
  for (long j = threadIdx.x; j < tot; j += blockDim.x) {
    int ix = j % H3, iy = (j / H3) % H3;
    long n = j / (H3 * H3);
    s += bf2f(a3[((n * C + ci) * H3 + iy) * H3 + ix]) * dy[(n * H4 + iy + ky) * H4 + ix + kx];
  }
  float r = block_reduce(s, sh);
  if (threadIdx.x == 0) dW[w] = r;
  __syncthreads();
  if (w == 0) {
    float sb = 0;
    for (long j = threadIdx.x; j < (long)B * H4 * H4; j += blockDim.x) sb += dy[j];
    float rb = block_reduce(sb, sh);
    if (threadIdx.x == 0) db[0] = rb;
  }
}

// Adam on the FP32 master weights, then refresh the BF16 copy
__global__ void k_adam(long n, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, bf16_t *__restrict__ pb, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  pb[i] = f2bf(pi);
}

}  // namespace

struct Net {
  hipStream_t stream = nullptr;
  int bmax = 0;
  long step = 0;
  float beta = 0.f;           // weight of the Laplacian term of the loss
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr, *part = nullptr;
  bf16_t *pb = nullptr;
  bf16_t *x = nullptr, *a1 = nullptr, *a2 = nullptr, *a2g = nullptr, *a3 = nullptr;
  float *y = nullptr, *dy = nullptr, *lap = nullptr, *d3 = nullptr, *dg = nullptr, *d2 = nullptr, *d1 = nullptr;
  std::vector<void *> owned;
};

template <typename T>
static iga_status nalloc(Net &n, T **q, size_t count) {
  void *r = nullptr;
  hipError_t e = hipMalloc(&r, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) return fail(IGA_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  n.owned.push_back(r);
  *q = (T *)r;
  return IGA_OK;
}

static void net_free(Net *n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  for (void *q : n->owned) (void)hipFree(q);
  delete n;
}

static iga_status forward(Net &n, const float *x, int B) {
  hipStream_t s = n.stream;
  const bf16_t *pb = n.pb;
  const float *p = n.p;
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk((long)B * 2 * H0 * H0)), dim3(256), 0, s, x, n.x, (long)B * 2 * H0 * H0);
  hipLaunchKernelGGL((k_conv_fwd<2, H0, H1, 1>), dim3(nblk((long)B * C * H1 * H1)), dim3(256), 0, s, B, n.x,
                     pb + O_W0, p + O_B0, n.a1);
  hipLaunchKernelGGL((k_conv_fwd<C, H1, H2, 2>), dim3(nblk((long)B * C * H2 * H2)), dim3(256), 0, s, B, n.a1,
                     pb + O_W1, p + O_B1, n.a2);
  hipLaunchKernelGGL(k_gctx_fwd, dim3((unsigned)(B * C)), dim3(256), 0, s, (const bf16_t *)n.a2, n.a2g);
  hipLaunchKernelGGL(k_convT4_fwd, dim3(nblk((long)B * C * H3 * H3)), dim3(256), 0, s, B, n.a2g, pb + O_W2, p + O_B2,
                     n.a3);
  hipLaunchKernelGGL(k_convT2_fwd, dim3(nblk((long)B * H4 * H4)), dim3(256), 0, s, B, n.a3, pb + O_W3, p + O_B3, n.y);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

static iga_status backward(Net &n, const float *target, int B) {
  hipStream_t s = n.stream;
  const bf16_t *pb = n.pb;
  float *g = n.g;
  if (n.beta != 0.f)
    hipLaunchKernelGGL(k_lap_err, dim3(nblk((long)B * H4 * H4)), dim3(256), 0, s, B, (const float *)n.y, target, n.lap);
  hipLaunchKernelGGL(k_mse, dim3(256), dim3(256), 0, s, B, (const float *)n.y, target, (const float *)n.lap, n.beta,
                     n.dy, n.part);
  hipLaunchKernelGGL(k_convT2_bwd_w, dim3(NP_W3), dim3(256), 0, s, B, n.dy, n.a3, g + O_W3, g + O_B3);
  hipLaunchKernelGGL(k_convT2_bwd_data, dim3(nblk((long)B * C * H3 * H3)), dim3(256), 0, s, B, n.dy, pb + O_W3, n.a3,
                     n.d3);
  hipLaunchKernelGGL(k_convT4_bwd_w, dim3(NP_W2), dim3(256), 0, s, B, n.d3, n.a2g, g + O_W2, g + O_B2);
  hipLaunchKernelGGL(k_convT4_bwd_data, dim3(nblk((long)B * C * H2 * H2)), dim3(256), 0, s, B, n.d3, pb + O_W2, n.dg);
  hipLaunchKernelGGL(k_gctx_bwd, dim3((unsigned)(B * C)), dim3(256), 0, s, (const float *)n.dg, (const bf16_t *)n.a2,
                     n.d2);
  hipLaunchKernelGGL((k_conv_bwd_w<C, H1, H2, 2>), dim3(NP_W1), dim3(256), 0, s, B, n.d2, n.a1, g + O_W1, g + O_B1);
  hipLaunchKernelGGL((k_conv_bwd_data<C, H1, H2, 2>), dim3(nblk((long)B * C * H1 * H1)), dim3(256), 0, s, B, n.d2,
                     pb + O_W1, n.a1, n.d1);
  hipLaunchKernelGGL((k_conv_bwd_w<2, H0, H1, 1>), dim3(NP_W0), dim3(256), 0, s, B, n.d1, n.x, g + O_W0, g + O_B0);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

static iga_status read_loss(Net &n, int B, float *loss) {
  float part[256];
  IGA_HIP_CHECK(hipMemcpyAsync(part, n.part, sizeof(part), hipMemcpyDeviceToHost, n.stream));
  IGA_HIP_CHECK(hipStreamSynchronize(n.stream));
  double s = 0;
  for (float q : part) s += q;
  *loss = (float)(s / ((double)B * H4 * H4));
  return IGA_OK;
}

}  // namespace iga

using namespace iga;

extern "C" {

int64_t igann_num_params(void) { return NPARAM; }

iga_status igann_create(int batch_max, void *hip_stream, igann_t *out) {
  if (!out || batch_max < 1) return fail(IGA_EINVAL, "bad arguments");
  *out = nullptr;
  Net *n = new Net();
  n->stream = (hipStream_t)hip_stream;
  n->bmax = batch_max;
  const size_t B = (size_t)batch_max;
  iga_status st;
  if ((st = nalloc(*n, &n->p, NPARAM)) || (st = nalloc(*n, &n->g, NPARAM)) || (st = nalloc(*n, &n->m, NPARAM)) ||
      (st = nalloc(*n, &n->v, NPARAM)) || (st = nalloc(*n, &n->pb, NPARAM)) || (st = nalloc(*n, &n->part, 256)) ||
      (st = nalloc(*n, &n->x, B * 2 * H0 * H0)) || (st = nalloc(*n, &n->a1, B * C * H1 * H1)) ||
      (st = nalloc(*n, &n->a2, B * C * H2 * H2)) || (st = nalloc(*n, &n->a2g, B * C * H2 * H2)) ||
      (st = nalloc(*n, &n->dg, B * C * H2 * H2)) || (st = nalloc(*n, &n->a3, B * C * H3 * H3)) ||
      (st = nalloc(*n, &n->y, B * H4 * H4)) || (st = nalloc(*n, &n->dy, B * H4 * H4)) ||
      (st = nalloc(*n, &n->lap, B * H4 * H4)) ||
      (st = nalloc(*n, &n->d3, B * C * H3 * H3)) || (st = nalloc(*n, &n->d2, B * C * H2 * H2)) ||
      (st = nalloc(*n, &n->d1, B * C * H1 * H1))) {
    net_free(n);
    return st;
  }
  *out = (igann_t)n;
  return IGA_OK;
}

iga_status igann_set_weights(igann_t nn, const float *host, int64_t count) {
  if (!nn || !host || count != NPARAM) return fail(IGA_EINVAL, "weights must have igann_num_params() values");
  Net &n = *(Net *)nn;
  IGA_HIP_CHECK(hipMemcpyAsync(n.p, host, NPARAM * sizeof(float), hipMemcpyHostToDevice, n.stream));
  IGA_HIP_CHECK(hipMemsetAsync(n.m, 0, NPARAM * sizeof(float), n.stream));
  IGA_HIP_CHECK(hipMemsetAsync(n.v, 0, NPARAM * sizeof(float), n.stream));
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(NPARAM)), dim3(256), 0, n.stream, (const float *)n.p, n.pb, (long)NPARAM);
  IGA_HIP_CHECK(hipStreamSynchronize(n.stream));
  n.step = 0;
  return IGA_OK;
}

iga_status igann_get_weights(igann_t nn, float *host, int64_t count) {
  if (!nn || !host || count != NPARAM) return fail(IGA_EINVAL, "weights must have igann_num_params() values");
  Net &n = *(Net *)nn;
  IGA_HIP_CHECK(hipMemcpyAsync(host, n.p, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n.stream));
  IGA_HIP_CHECK(hipStreamSynchronize(n.stream));
  return IGA_OK;
}

iga_status igann_forward(igann_t nn, const float *x_dev, int B, float *y_dev) {
  if (!nn || !x_dev || !y_dev) return fail(IGA_EINVAL, "null argument");
  Net &n = *(Net *)nn;
  if (B < 1 || B > n.bmax) return fail(IGA_EINVAL, "batch larger than the network was created for");
  iga_status st = forward(n, x_dev, B);
  if (st) return st;
  IGA_HIP_CHECK(hipMemcpyAsync(y_dev, n.y, (size_t)B * H4 * H4 * sizeof(float), hipMemcpyDeviceToDevice, n.stream));
  return IGA_OK;
}

iga_status igann_set_loss(igann_t nn, float laplacian_weight) {
  if (!nn || !(laplacian_weight >= 0.f)) return fail(IGA_EINVAL, "weight must be >= 0");
  ((Net *)nn)->beta = laplacian_weight;
  return IGA_OK;
}

iga_status igann_postprocess(igann_t nn, float *y_dev, int B, const float *mean_dev, float scale,
                             const float *sample_scale_dev, int passes) {
  if (!nn || !y_dev || passes < 0) return fail(IGA_EINVAL, "bad argument");
  Net &n = *(Net *)nn;
  if (B < 1 || B > n.bmax) return fail(IGA_EINVAL, "batch larger than the network was created for");
  const unsigned g = nblk((long)B * H4 * H4);
  hipLaunchKernelGGL(k_affine_out, dim3(g), dim3(256), 0, n.stream, B, y_dev, mean_dev, scale, sample_scale_dev);
  for (int k = 0; k < passes; ++k) {
    hipLaunchKernelGGL(k_smooth, dim3(g), dim3(256), 0, n.stream, B, (const float *)y_dev, n.dy, 0);
    hipLaunchKernelGGL(k_smooth, dim3(g), dim3(256), 0, n.stream, B, (const float *)n.dy, y_dev, 1);
  }
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

iga_status igann_gradients(igann_t nn, const float *x_dev, const float *t_dev, int B, float *loss, float *grad_host) {
  if (!nn || !x_dev || !t_dev) return fail(IGA_EINVAL, "null argument");
  Net &n = *(Net *)nn;
  if (B < 1 || B > n.bmax) return fail(IGA_EINVAL, "batch larger than the network was created for");
  iga_status st;
  if ((st = forward(n, x_dev, B)) || (st = backward(n, t_dev, B))) return st;
  if (grad_host)
    IGA_HIP_CHECK(hipMemcpyAsync(grad_host, n.g, NPARAM * sizeof(float), hipMemcpyDeviceToHost, n.stream));
  float l = 0;
  if ((st = read_loss(n, B, &l))) return st;
  if (loss) *loss = l;
  return IGA_OK;
}

iga_status igann_train_step(igann_t nn, const float *x_dev, const float *t_dev, int B, float lr, float *loss) {
  if (!nn || !x_dev || !t_dev) return fail(IGA_EINVAL, "null argument");
  Net &n = *(Net *)nn;
  if (B < 1 || B > n.bmax) return fail(IGA_EINVAL, "batch larger than the network was created for");
  iga_status st;
  if ((st = forward(n, x_dev, B)) || (st = backward(n, t_dev, B))) return st;
  n.step += 1;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)n.step), c2 = 1.f - powf(b2, (float)n.step);
  hipLaunchKernelGGL(k_adam, dim3(nblk(NPARAM)), dim3(256), 0, n.stream, (long)NPARAM, n.p, (const float *)n.g, n.m,
                     n.v, n.pb, lr, b1, b2, eps, c1, c2);
  IGA_HIP_CHECK(hipGetLastError());
  if (loss) return read_loss(n, B, loss);
  return IGA_OK;
}

iga_status igann_destroy(igann_t nn) {
  net_free((Net *)nn);
  return IGA_OK;
}

}  // extern "C"
