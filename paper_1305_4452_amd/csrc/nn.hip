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
// Activations are [sample][channel][y][x].  The two 64 -> 64 layers (forward, data gradient, weight
// gradient) run on the BF16 matrix cores (k_nn_gemm); the thin first and last layers (2 -> 64,
// 64 -> 1) and the elementwise steps run on the vector units.
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

// ---- weight and bias gradients of the thin layers: a block per (channel, chunk of kSampChunk samples)
// forms every sum of its channel in one pass and leaves them as a partial row; k_sum_parts adds the
// chunks in order ----
constexpr int kSampChunk = 4;

template <int NV>
__device__ inline void block_sum_n(float (&v)[NV], float (*sh)[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    float x = v[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    if (lane == 0) sh[j][w] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = sh[j][0] + sh[j][1] + sh[j][2] + sh[j][3];
}

// conv 3x3 2 -> 64 (stride 1, pad 1): dW0[co][ci][ky][kx] = sum dz1[n][co][oy][ox] x[n][ci][oy+ky-1][ox+kx-1]
// and db0[co] = sum dz1[n][co][:]; partial row [chunk][co 18 weights ..., 1152 + co bias]
__global__ void __launch_bounds__(256) k_conv0_wgrad(int B, const float *__restrict__ dz, const bf16_t *__restrict__ x,
                                                     float *__restrict__ part) {
  __shared__ float sh[19][4];
  const int co = blockIdx.x, n0 = blockIdx.y * kSampChunk, n1 = min(B, n0 + kSampChunk);
  float acc[19];
#pragma unroll
  for (int j = 0; j < 19; ++j) acc[j] = 0.f;
  for (long j = threadIdx.x; j < (long)(n1 - n0) * H1 * H1; j += 256) {
    const long n = n0 + j / (H1 * H1);
    const int oy = (int)(j / H1) % H1, ox = (int)(j % H1);
    const float d = dz[(n * C + co) * H1 * H1 + oy * H1 + ox];
#pragma unroll
    for (int ci = 0; ci < 2; ++ci)
#pragma unroll
      for (int ky = 0; ky < 3; ++ky)
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int iy = oy + ky - 1, ix = ox + kx - 1;
          if (iy >= 0 && iy < H0 && ix >= 0 && ix < H0) acc[ci * 9 + ky * 3 + kx] += d * bf2f(x[((n * 2 + ci) * H0 + iy) * H0 + ix]);
        }
    acc[18] += d;
  }
  block_sum_n<19>(acc, sh);
  if (threadIdx.x == 0) {
    float *row = part + (long)blockIdx.y * (NP_W0 + C);
#pragma unroll
    for (int j = 0; j < 18; ++j) row[co * 18 + j] = acc[j];
    row[NP_W0 + co] = acc[18];
  }
}

// transposed conv 2x2 64 -> 1: dW3[ci][ky][kx] = sum a3[n][ci][iy][ix] dy[n][iy+ky][ix+kx], db3 = sum dy;
// partial row [chunk][ci 4 weights ..., 256 bias] (the bias by the ci = 0 blocks)
__global__ void __launch_bounds__(256) k_convT2_wgrad(int B, const float *__restrict__ dy, const bf16_t *__restrict__ a3,
                                                      float *__restrict__ part) {
  __shared__ float sh[5][4];
  const int ci = blockIdx.x, n0 = blockIdx.y * kSampChunk, n1 = min(B, n0 + kSampChunk);
  float acc[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  for (long j = threadIdx.x; j < (long)(n1 - n0) * H3 * H3; j += 256) {
    const long n = n0 + j / (H3 * H3);
    const int iy = (int)(j / H3) % H3, ix = (int)(j % H3);
    const float a = bf2f(a3[((n * C + ci) * H3 + iy) * H3 + ix]);
    const float *d = dy + (n * H4 + iy) * H4 + ix;
    acc[0] += a * d[0];
    acc[1] += a * d[1];
    acc[2] += a * d[H4];
    acc[3] += a * d[H4 + 1];
  }
  if (ci == 0)
    for (long j = threadIdx.x; j < (long)(n1 - n0) * H4 * H4; j += 256) acc[4] += dy[(long)n0 * H4 * H4 + j];
  block_sum_n<5>(acc, sh);
  if (threadIdx.x == 0) {
    float *row = part + (long)blockIdx.y * (NP_W3 + 1);
#pragma unroll
    for (int j = 0; j < 4; ++j) row[ci * 4 + j] = acc[j];
    if (ci == 0) row[NP_W3] = acc[4];
  }
}

// bias gradient of a 64-channel layer: partial row [chunk][c] = sum over the chunk's samples of d[n][c][:]
__global__ void __launch_bounds__(256) k_bias_part(int B, const float *__restrict__ d, int hw, float *__restrict__ part) {
  __shared__ float sh[1][4];
  const int c = blockIdx.x, n0 = blockIdx.y * kSampChunk, n1 = min(B, n0 + kSampChunk);
  float acc[1] = {0.f};
  for (long j = threadIdx.x; j < (long)(n1 - n0) * hw; j += 256) acc[0] += d[((n0 + j / hw) * C + c) * hw + j % hw];
  block_sum_n<1>(acc, sh);
  if (threadIdx.x == 0) part[(long)blockIdx.y * C + c] = acc[0];
}

// ---- matrix-core layers ------------------------------------------------------------------
// The six large contractions of the network (conv 3x3 s2 and transposed conv 4x4 s4: forward, data
// gradient, weight gradient) run as implicit GEMMs C[M][N] = sum_k A[m][k] B[k][n] on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  A workgroup of four waves owns a 64 x 64 tile of C
// and a range of k (the weight gradients split their long k = (sample, pixel) reduction over
// workgroups and add the partial tiles in a fixed order afterwards).  Per 32-deep step the tile's A
// and B operands are gathered from the activation / gradient / weight layouts by the layer's loader
// (zero padding included) into LDS as BF16, A as [m][k] and B as [n][k], so each lane reads its 8
// consecutive k of one row with one 16-byte load.  Weights and activations are BF16 already;
// gradients are FP32 and enter as hi = bf16(g), lo = bf16(g - hi) with two products (about 16
// significant bits, as exact as the FP32 kernels they replace to within the FP32 accumulation).
// Lane l of a 16 x 16 x 32 product holds A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16] (j < 8)
// and receives D[4 (l / 16) + i][l % 16] (i < 4).
typedef __bf16 nbf16x8 __attribute__((ext_vector_type(8)));
typedef float nf32x4 __attribute__((ext_vector_type(4)));
constexpr int kGT = 64, kGK = 32, kGLD = 40;   // tile side, reduction step, LDS row stride (bf16)

__device__ inline __bf16 raw_bf(bf16_t b) { return __builtin_bit_cast(__bf16, b); }

// gather one 8-deep k segment of a row (A: row m, B: column n) into LDS as hi (and lo) BF16
template <bool SPLIT, typename F>
__device__ inline void gather8(F &&get, __bf16 *hi, __bf16 *lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if constexpr (SPLIT) {
      const float v = get(j);
      const __bf16 h = (__bf16)v;
      hi[j] = h;
      lo[j] = (__bf16)(v - (float)h);
    } else {
      hi[j] = get(j);
    }
  }
}

// Op: static SPLIT_A / SPLIT_B (the operand is FP32 and split), a(m, k) / b(k, n) returning float
// (split) or __bf16, and out(m, n, value, kz).  M, N multiples of 64, K and kchunk multiples of 32.
template <class Op>
__global__ void __launch_bounds__(256) k_nn_gemm(Op op, int M, int N, int K, int kchunk) {
  constexpr bool SA = Op::SPLIT_A, SB = Op::SPLIT_B;
  __shared__ __align__(16) __bf16 sA[SA ? 2 : 1][kGT][kGLD];
  __shared__ __align__(16) __bf16 sB[SB ? 2 : 1][kGT][kGLD];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, wm = w >> 1, wn = w & 1;
  const int ntn = N / kGT;
  const int m0 = (blockIdx.x / ntn) * kGT, n0 = (blockIdx.x % ntn) * kGT;
  const int kz = blockIdx.y, kb = kz * kchunk, ke = min(K, kb + kchunk);
  nf32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = nf32x4{0.f, 0.f, 0.f, 0.f};
  const int lr = t >> 2, lk = (t & 3) * 8;   // this thread's loader row and k segment
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    gather8<SA>([&](int j) { return op.a(m0 + lr, k0 + lk + j); }, &sA[0][lr][lk], &sA[SA ? 1 : 0][lr][lk]);
    gather8<SB>([&](int j) { return op.b(k0 + lk + j, n0 + lr); }, &sB[0][lr][lk], &sB[SB ? 1 : 0][lr][lk]);
    __syncthreads();
    const int r = lane & 15, kk = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ra = wm * 32 + i * 16 + r;
      const nbf16x8 ah = *(const nbf16x8 *)&sA[0][ra][kk];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rb = wn * 32 + j * 16 + r;
        const nbf16x8 bh = *(const nbf16x8 *)&sB[0][rb][kk];
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc[i][j], 0, 0, 0);
        if constexpr (SA) {
          const nbf16x8 al = *(const nbf16x8 *)&sA[1][ra][kk];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc[i][j], 0, 0, 0);
        }
        if constexpr (SB) {
          const nbf16x8 bl = *(const nbf16x8 *)&sB[1][rb][kk];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc[i][j], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        op.out(m0 + wm * 32 + i * 16 + 4 * (lane >> 4) + q, n0 + wn * 32 + j * 16 + (lane & 15), acc[i][j][q], kz);
}

// conv 3x3 s2 p1 (64 -> 64), 32^2 -> 16^2: m = (n, oy, ox), n = co, k = (ci, ky, kx); ReLU, BF16 out
struct OpConv1Fwd {
  static constexpr bool SPLIT_A = false, SPLIT_B = false;
  const bf16_t *in, *W;
  const float *bias;
  bf16_t *out_;
  __device__ __bf16 a(int m, int k) const {
    const int s = m >> 8, oy = (m >> 4) & 15, ox = m & 15, ci = k / 9, r = k - 9 * ci, ky = r / 3, kx = r - 3 * ky;
    const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
    if (iy < 0 || iy >= H1 || ix < 0 || ix >= H1) return raw_bf(0);
    return raw_bf(in[(((long)s * C + ci) * H1 + iy) * H1 + ix]);
  }
  __device__ __bf16 b(int k, int n) const { return raw_bf(W[n * C * 9 + k]); }
  __device__ void out(int m, int n, float v, int) const {
    v += bias[n];
    out_[((long)(m >> 8) * C + n) * (H2 * H2) + (m & 255)] = f2bf(v > 0.f ? v : 0.f);
  }
};

// transposed conv 4x4 s4 (64 -> 64), 16^2 -> 64^2: m = (n, iy, ix), n = (co, ky, kx), k = ci; ReLU
struct OpConvT4Fwd {
  static constexpr bool SPLIT_A = false, SPLIT_B = false;
  const bf16_t *in, *W;
  const float *bias;
  bf16_t *out_;
  __device__ __bf16 a(int m, int k) const { return raw_bf(in[((long)(m >> 8) * C + k) * (H2 * H2) + (m & 255)]); }
  __device__ __bf16 b(int k, int n) const { return raw_bf(W[k * C * 16 + n]); }
  __device__ void out(int m, int n, float v, int) const {
    const int co = n >> 4, ky = (n >> 2) & 3, kx = n & 3, iy = (m >> 4) & 15, ix = m & 15;
    v += bias[co];
    out_[(((long)(m >> 8) * C + co) * H3 + 4 * iy + ky) * H3 + 4 * ix + kx] = f2bf(v > 0.f ? v : 0.f);
  }
};

// its data gradient: dg[n][ci][iy][ix] = sum_{co,ky,kx} W2[ci][co][ky][kx] dz3[n][co][4iy+ky][4ix+kx]
// m = (n, iy, ix), n = ci, k = (co, ky, kx)
struct OpConvT4Data {
  static constexpr bool SPLIT_A = true, SPLIT_B = false;
  const float *dz;
  const bf16_t *W;
  float *out_;
  __device__ float a(int m, int k) const {
    const int co = k >> 4, ky = (k >> 2) & 3, kx = k & 3, iy = (m >> 4) & 15, ix = m & 15;
    return dz[(((long)(m >> 8) * C + co) * H3 + 4 * iy + ky) * H3 + 4 * ix + kx];
  }
  __device__ __bf16 b(int k, int n) const { return raw_bf(W[n * C * 16 + k]); }
  __device__ void out(int m, int n, float v, int) const { out_[((long)(m >> 8) * C + n) * (H2 * H2) + (m & 255)] = v; }
};

// its weight gradient: dW2[ci][(co,ky,kx)] = sum_{(n,iy,ix)} g[n][ci][iy][ix] dz3[n][co][4iy+ky][4ix+kx];
// m = ci, n = (co, ky, kx), k = (n, iy, ix); partial tiles per k chunk
struct OpConvT4W {
  static constexpr bool SPLIT_A = false, SPLIT_B = true;
  const bf16_t *g;
  const float *dz;
  float *part;
  __device__ __bf16 a(int m, int k) const { return raw_bf(g[((long)(k >> 8) * C + m) * (H2 * H2) + (k & 255)]); }
  __device__ float b(int k, int n) const {
    const int co = n >> 4, ky = (n >> 2) & 3, kx = n & 3, iy = (k >> 4) & 15, ix = k & 15;
    return dz[(((long)(k >> 8) * C + co) * H3 + 4 * iy + ky) * H3 + 4 * ix + kx];
  }
  __device__ void out(int m, int n, float v, int kz) const { part[((long)kz * C + m) * (C * 16) + n] = v; }
};

// conv 3x3 s2 data gradient: din[n][ci][iy][ix] = sum_{co,ky,kx} W1[co][ci][ky][kx] dz2[n][co][oy][ox]
// over 2 oy + ky - 1 = iy, 2 ox + kx - 1 = ix; m = (n, iy, ix), n = ci, k = (co, ky, kx); ReLU mask of a1
struct OpConv1Data {
  static constexpr bool SPLIT_A = true, SPLIT_B = false;
  const float *dz;
  const bf16_t *W, *ain;
  float *out_;
  __device__ float a(int m, int k) const {
    const int iy = (m >> 5) & 31, ix = m & 31, co = k / 9, r = k - 9 * co, ky = r / 3, kx = r - 3 * ky;
    const int ty = iy + 1 - ky, tx = ix + 1 - kx;
    if (ty < 0 || tx < 0 || (ty & 1) || (tx & 1) || ty >= 2 * H2 || tx >= 2 * H2) return 0.f;
    return dz[(((long)(m >> 10) * C + co) * H2 + (ty >> 1)) * H2 + (tx >> 1)];
  }
  __device__ __bf16 b(int k, int n) const {
    const int co = k / 9, r = k - 9 * co;
    return raw_bf(W[(co * C + n) * 9 + r]);
  }
  __device__ void out(int m, int n, float v, int) const {
    const long i = ((long)(m >> 10) * C + n) * (H1 * H1) + (m & 1023);
    out_[i] = bf2f(ain[i]) > 0.f ? v : 0.f;
  }
};

// conv 3x3 s2 weight gradient: dW1[co][(ci,ky,kx)] = sum_{(n,oy,ox)} dz2[n][co][oy][ox] a1[n][ci][2oy+ky-1][2ox+kx-1];
// m = co, n = (ci, ky, kx), k = (n, oy, ox); partial tiles per k chunk
struct OpConv1W {
  static constexpr bool SPLIT_A = true, SPLIT_B = false;
  const float *dz;
  const bf16_t *ain;
  float *part;
  __device__ float a(int m, int k) const { return dz[((long)(k >> 8) * C + m) * (H2 * H2) + (k & 255)]; }
  __device__ __bf16 b(int k, int n) const {
    const int oy = (k >> 4) & 15, ox = k & 15, ci = n / 9, r = n - 9 * ci, ky = r / 3, kx = r - 3 * ky;
    const int iy = 2 * oy + ky - 1, ix = 2 * ox + kx - 1;
    if (iy < 0 || iy >= H1 || ix < 0 || ix >= H1) return raw_bf(0);
    return raw_bf(ain[(((long)(k >> 8) * C + ci) * H1 + iy) * H1 + ix]);
  }
  __device__ void out(int m, int n, float v, int kz) const { part[((long)kz * C + m) * (C * 9) + n] = v; }
};

// dW[i] = sum over the nz partial tiles, in order
__global__ void k_sum_parts(const float *__restrict__ part, int nz, long nw, float *__restrict__ dW) {
  long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (i >= nw) return;
  float s = 0.f;
  for (int z = 0; z < nz; ++z) s += part[z * nw + i];
  dW[i] = s;
}

constexpr int kWChunk = 512;   // k = (sample, pixel) per partial tile of the weight gradients

template <class Op>
void launch_gemm(hipStream_t s, const Op &op, int M, int N, int K, int kchunk) {
  const dim3 grid((unsigned)((M / kGT) * (N / kGT)), (unsigned)((K + kchunk - 1) / kchunk));
  hipLaunchKernelGGL(k_nn_gemm<Op>, grid, dim3(256), 0, s, op, M, N, K, kchunk);
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
  float *wpart = nullptr;     // partial tiles of the split weight-gradient reductions
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
  launch_gemm(s, OpConv1Fwd{n.a1, pb + O_W1, p + O_B1, n.a2}, B * H2 * H2, C, C * 9, C * 9);
  hipLaunchKernelGGL(k_gctx_fwd, dim3((unsigned)(B * C)), dim3(256), 0, s, (const bf16_t *)n.a2, n.a2g);
  launch_gemm(s, OpConvT4Fwd{n.a2g, pb + O_W2, p + O_B2, n.a3}, B * H2 * H2, C * 16, C, C);
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
  const int nch = (B + kSampChunk - 1) / kSampChunk;
  hipLaunchKernelGGL(k_convT2_wgrad, dim3(C, nch), dim3(256), 0, s, B, (const float *)n.dy, (const bf16_t *)n.a3,
                     n.wpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(NP_W3 + 1)), dim3(256), 0, s, (const float *)n.wpart, nch,
                     (long)(NP_W3 + 1), g + O_W3);   // W3 then b3 (contiguous)
  hipLaunchKernelGGL(k_convT2_bwd_data, dim3(nblk((long)B * C * H3 * H3)), dim3(256), 0, s, B, n.dy, pb + O_W3, n.a3,
                     n.d3);
  const int KW = B * H2 * H2, nz = (KW + kWChunk - 1) / kWChunk;
  launch_gemm(s, OpConvT4W{n.a2g, n.d3, n.wpart}, C, C * 16, KW, kWChunk);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(NP_W2)), dim3(256), 0, s, (const float *)n.wpart, nz, (long)NP_W2, g + O_W2);
  hipLaunchKernelGGL(k_bias_part, dim3(C, nch), dim3(256), 0, s, B, (const float *)n.d3, H3 * H3, n.wpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const float *)n.wpart, nch, (long)C, g + O_B2);
  launch_gemm(s, OpConvT4Data{n.d3, pb + O_W2, n.dg}, B * H2 * H2, C, C * 16, C * 16);
  hipLaunchKernelGGL(k_gctx_bwd, dim3((unsigned)(B * C)), dim3(256), 0, s, (const float *)n.dg, (const bf16_t *)n.a2,
                     n.d2);
  launch_gemm(s, OpConv1W{n.d2, n.a1, n.wpart}, C, C * 9, KW, kWChunk);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(NP_W1)), dim3(256), 0, s, (const float *)n.wpart, nz, (long)NP_W1, g + O_W1);
  hipLaunchKernelGGL(k_bias_part, dim3(C, nch), dim3(256), 0, s, B, (const float *)n.d2, H2 * H2, n.wpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, (const float *)n.wpart, nch, (long)C, g + O_B1);
  launch_gemm(s, OpConv1Data{n.d2, pb + O_W1, n.a1, n.d1}, B * H1 * H1, C, C * 9, C * 9);
  hipLaunchKernelGGL(k_conv0_wgrad, dim3(C, nch), dim3(256), 0, s, B, (const float *)n.d1, (const bf16_t *)n.x,
                     n.wpart);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(NP_W0 + C)), dim3(256), 0, s, (const float *)n.wpart, nch,
                     (long)(NP_W0 + C), g + O_W0);   // W0 then b0 (contiguous)
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
      (st = nalloc(*n, &n->d1, B * C * H1 * H1)) ||
      (st = nalloc(*n, &n->wpart, (B * H2 * H2 + kWChunk - 1) / kWChunk * (size_t)NP_W2))) {
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
