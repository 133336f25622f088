// Row-gather Jacobian of eq:jacobian with its axis-2 and axis-1 contractions on the BF16 matrix cores
// of gfx950 (FP32 accumulation): iga_assemble_jacobian with prec IGA_BF16 or IGA_BF16X3, FP32 values.
//
// Two launches:
//   k_cs3     the per-point coefficient streams of eq:jacobian (the metric D', the rational
//             corrections and the reaction coefficient, or kappa W and the reaction coefficient on
//             x = xi), in FP64 arithmetic from the FP64 geometry table and u by sum factorisation, once
//             per Gauss point, stored FP32 as cs[e0 q0][stream][g1][g2] (g = global Gauss-point index
//             along an axis; every row padded with zeros);
//   k_rgmma3  the row-gather of rowgather.hip: a workgroup owns a 2 x 2 block of row pencils (i1, i2)
//             and streams element columns e0 along axis 0.  For each Gauss point q0 of a column:
//     level 1 (matrix cores) contracts axis 2: T1_k[g1][n] = sum_t sum_g2 cs_s(t)[g1][g2] Z2_f(t)[g2][n],
//             n = (pencil i2, offset o2), Z2_f[g2][n] = X(i2, g2) Y(i2 + o2, g2) the product of the two
//             1D axis-2 factors of term t (zero outside the support overlap); the terms of one
//             combination k of axis-0/axis-1 factors share an accumulator (concatenated along the
//             reduction).  The A operand comes straight from cs in global memory (L2), the B operand
//             from LDS;
//     level 2 (matrix cores) contracts axis 1: T2_c[m][n] = sum_{k of c} sum_g1 Z1_f1(k)[m][g1] T1_k[g1][n],
//             m = (pencil i1, offset o1), with T1 rounded to BF16 in LDS;
//     level 3 (vector units, FP32) folds the axis-0 factors of q0 into a register window per owner
//             (row pencil, column offsets), as in rowgather.hip.
// Each MFMA is v_mfma_f32_16x16x32_bf16: 16 x 16 outputs, a 32-deep reduction (the <= 30 Gauss
// points of a 2-pencil window along one axis, zero-padded).  The Z tables depend on axes 1 and 2
// only and are built once per workgroup.
//
// Precision: IGA_BF16 rounds the operands to BF16 (8 significant bits); IGA_BF16X3 splits each FP32
// operand x into hi = bf16(x) and lo = bf16(x - hi) and accumulates lo*hi + hi*lo + hi*hi, about 16
// significant bits per product.  Geometry, u and e^u are FP64, accumulation and level 3 FP32.
#include "iga_impl.h"
#include "kern_rg.h"

namespace iga {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMB = 2;     // pencils per block along axes 1 and 2
constexpr int kLD = 40;    // row stride (elements) of the LDS operand tiles: 32 used, padded against bank conflicts
constexpr int kPad = 36;   // zero padding at the end of every cs row (the 32-deep reductions may read past the window)

template <int P>
struct MShape {
  static constexpr int p = P - 1, Q = P, W = 2 * p + 1;
  static constexpr int ME = kMB + p;            // window elements per axis
  static constexpr int G = ME * Q;              // window Gauss points per axis (<= 30 for P <= 5)
  static constexpr int NN = kMB * W;            // (pencil, offset) pairs per axis (<= 18)
  static constexpr int NOWN = NN * NN;          // level-3 owners (row pencil x column offsets)
  static constexpr int NT = NOWN <= 256 ? 256 : ((NOWN + 63) / 64) * 64;
  static constexpr int MT = (G + 15) / 16;      // 16-row tiles over g1 (level 1)
  static constexpr int NT16 = (NN + 15) / 16;   // 16-wide tiles over n (levels 1, 2) and m (level 2)
  static_assert(G <= 32, "one 32-deep reduction step per term");
};

// Terms of eq:jacobian grouped for level 1.  A combination k fixes the axis-0 and axis-1 factor pairs
// (c0 = 2 x0 + y0, f1 = 2 x1 + y1; x_d = 1: parametric derivative along axis d on the row function,
// y_d on the column function); its terms are (coefficient stream, axis-2 factor pair f2 = 2 x2 + y2).
// A group is one or two combinations whose streams are loaded once: ns distinct streams s[], and
// terms (combination slot, index into s[], f2).  Stream numbering of the geometry table mode:
// D'00 D'11 D'22 D'01 D'02 D'12 h0 h1 h2 m'' (rg_coefs in kern_rg.h); on x = xi: kappa W, the
// reaction coefficient.  The terms are those of the row-gather term tables in kern_rg.h.
struct MTerm { int slot, si, f2; };
struct MGroup { int nk, k[2], ns, s[3], nt; MTerm t[4]; };
struct MCombo { int c0, f1; };
__constant__ MCombo kCombosTable[9] = {{3, 0}, {0, 3}, {0, 0}, {2, 1}, {1, 2}, {2, 0}, {1, 0}, {0, 2}, {0, 1}};
__constant__ MGroup kGroupsTable[6] = {
    {1, {0, 0}, 1, {0}, 1, {{0, 0, 0}}},                                       // xi0 on both functions
    {1, {1, 0}, 1, {1}, 1, {{0, 0, 0}}},                                       // xi1 on both
    {1, {2, 0}, 3, {2, 8, 9}, 4, {{0, 0, 3}, {0, 1, 1}, {0, 1, 2}, {0, 2, 0}}},  // xi2 on both, h2, m''
    {2, {3, 4}, 1, {3}, 2, {{0, 0, 0}, {1, 0, 0}}},                            // xi0 x xi1 (both orders)
    {2, {5, 6}, 2, {4, 6}, 4, {{0, 0, 1}, {0, 1, 0}, {1, 0, 2}, {1, 1, 0}}},   // xi0 x xi2, h0
    {2, {7, 8}, 2, {5, 7}, 4, {{0, 0, 1}, {0, 1, 0}, {1, 0, 2}, {1, 1, 0}}}};  // xi1 x xi2, h1
__constant__ MCombo kCombosDiag[3] = {{3, 0}, {0, 3}, {0, 0}};
__constant__ MGroup kGroupsDiag[2] = {
    {2, {0, 1}, 1, {0}, 2, {{0, 0, 0}, {1, 0, 0}}},                            // xi0, xi1 on both
    {1, {2, 0}, 2, {0, 1}, 2, {{0, 0, 3}, {0, 1, 0}}}};                        // xi2 on both, reaction

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }

// ------------------------------------------------------------------------------------------
// k_cs3: coefficient streams at every Gauss point.  A workgroup owns an element row along axis 2
// (fixed e0, e1) and walks it two elements at a time; u by sum factorisation over each element.
// ------------------------------------------------------------------------------------------
template <int P, bool TABLE>
__global__ void __launch_bounds__(256) k_cs3(DevProblem pb, const double *__restrict__ U, float *__restrict__ cs,
                                             int64_t ld) {
  constexpr int p = P - 1, Q = P, QD = Q * Q * Q, NS = TABLE ? 10 : 2;
  constexpr int EPB = 2;                               // elements per pass
  __shared__ double sU[EPB][P][P][P];                  // [el][a2][a1][a0]
  __shared__ double V0[EPB][P][P][Q], V1[EPB][P][Q][Q];
  __shared__ double b0[Q][P], b1[Q][P], w0[Q], w1[Q];
  const int t = threadIdx.x;
  const int e0 = blockIdx.x % pb.ne[0], e1 = blockIdx.x / pb.ne[0];
  const int n0 = pb.n[0], n1 = pb.n[1];
  const int64_t G1tot = (int64_t)pb.ne[1] * Q;
  if (t < Q * P) {
    (&b0[0][0])[t] = pb.ax[0].B[(size_t)e0 * Q * P + t];
    (&b1[0][0])[t] = pb.ax[1].B[(size_t)e1 * Q * P + t];
  }
  if (t < Q) {
    w0[t] = pb.ax[0].wq[(size_t)e0 * Q + t];
    w1[t] = pb.ax[1].wq[(size_t)e1 * Q + t];
  }
  for (int e2s = 0; e2s < pb.ne[2]; e2s += EPB) {
    const int nel = min(EPB, pb.ne[2] - e2s);
    __syncthreads();
    for (int i = t; i < nel * P * P * P; i += 256) {
      const int a0 = i % P, a1 = (i / P) % P, a2 = (i / (P * P)) % P, el = i / (P * P * P);
      const int64_t A = (e0 + a0) + (int64_t)n0 * ((e1 + a1) + (int64_t)n1 * (e2s + el + a2));
      double v = U[A];
      if (TABLE && pb.rational) v *= pb.wts[A];
      sU[el][a2][a1][a0] = v;
    }
    __syncthreads();
    for (int i = t; i < nel * P * P * Q; i += 256) {
      const int q0 = i % Q, a1 = (i / Q) % P, a2 = (i / (Q * P)) % P, el = i / (Q * P * P);
      double s = 0;
#pragma unroll
      for (int a0 = 0; a0 < P; ++a0) s += b0[q0][a0] * sU[el][a2][a1][a0];
      V0[el][a2][a1][q0] = s;
    }
    __syncthreads();
    for (int i = t; i < nel * P * Q * Q; i += 256) {
      const int q0 = i % Q, q1 = (i / Q) % Q, a2 = (i / (Q * Q)) % P, el = i / (Q * Q * P);
      double s = 0;
#pragma unroll
      for (int a1 = 0; a1 < P; ++a1) s += b1[q1][a1] * V0[el][a2][a1][q0];
      V1[el][a2][q1][q0] = s;
    }
    __syncthreads();
    for (int i = t; i < EPB * QD; i += 256) {
      // (q2, element) fastest: consecutive threads write consecutive points of a row
      const int q2 = i % Q, el = (i / Q) % EPB, q1 = (i / (Q * EPB)) % Q, q0 = i / (Q * EPB * Q);
      if (el >= nel) continue;
      const int e2 = e2s + el;
      double ut = 0;
#pragma unroll
      for (int a2 = 0; a2 < P; ++a2) ut += pb.ax[2].B[((size_t)e2 * Q + q2) * P + a2] * V1[el][a2][q1][q0];
      const int64_t e = e0 + (int64_t)pb.ne[0] * (e1 + (int64_t)pb.ne[1] * e2);
      const double Wq = w0[q0] * w1[q1] * pb.ax[2].wq[(size_t)e2 * Q + q2];
      const double kap = (!TABLE && pb.kappa_mode == IGA_KAPPA_ELEMENT) ? pb.kel[e] : 1.0;
      double cv[10];
      rgk::rg_coefs<3, TABLE>(pb, e, q0 + Q * (q1 + Q * q2), QD, Wq, kap, ut, cv);
      float *row = cs + (((int64_t)(e0 * Q + q0) * NS) * G1tot + (int64_t)e1 * Q + q1) * ld + (int64_t)e2 * Q + q2;
#pragma unroll
      for (int s = 0; s < NS; ++s) row[(int64_t)s * G1tot * ld] = (float)cv[s];
    }
  }
}

// ------------------------------------------------------------------------------------------
// k_rgmma3: levels 1-3 and the CSR rows of one 2 x 2 pencil block
// ------------------------------------------------------------------------------------------
template <int P, bool TABLE, bool SPLIT>
__global__ void __launch_bounds__(MShape<P>::NT)
k_rgmma3(DevProblem pb, const float *__restrict__ cs, int64_t ld, float *__restrict__ vals, int nb1, int seg_len,
         int nseg, int nlogical) {
  using S = MShape<P>;
  constexpr int p = S::p, Q = S::Q, W = S::W, ME = S::ME, G = S::G, NN = S::NN, NT = S::NT, T16 = S::NT16;
  constexpr int NS = TABLE ? 10 : 2;
  constexpr int NK = TABLE ? 9 : 3;
  constexpr int NG = TABLE ? 6 : 2;
  constexpr int NWAVE = NT / 64;
  constexpr int NL = SPLIT ? 2 : 1;                       // hi, (lo)

  __shared__ double tB1[2][ME][Q][P], tB2[2][ME][Q][P];   // [value|derivative][element][q][a]
  __shared__ float fX0[2][Q][P];
  __shared__ __attribute__((aligned(16))) __bf16 z2[NL][4][NN][kLD];    // level-1 B operand [f2][n][g2]
  __shared__ __attribute__((aligned(16))) __bf16 z1[NL][4][NN][kLD];    // level-2 A operand [f1][m][g1]
  // level-2 B operand t1 [k][n][g1]; where level 1 rewrites all 32 rows of t1 every step (G > 16) the
  // completed-row staging buffer of the emission shares its memory (used only between steps)
  constexpr int T1B = NL * NK * NN * kLD * 2, RBB = kMB * kMB * W * W * W * 4;
  constexpr bool ALIAS = S::MT * 16 >= 32 && RBB <= T1B;
  __shared__ __attribute__((aligned(16))) unsigned char t1raw[ALIAS ? T1B : T1B + RBB];
  auto t1 = reinterpret_cast<__bf16(*)[NK][NN][kLD]>(t1raw);
  auto rowbuf = reinterpret_cast<float(*)[W * W * W]>(t1raw + (ALIAS ? 0 : T1B));
  __shared__ float T2[4][NN][NN + 1];                     // level-2 results [c0][m][n]
  // the coefficient window of one step (level-1 A operand), FP32 [s, g1][columns of g2].  Odd Q: 36
  // columns, of which the 32 the reduction reads start d = 0 or 2 columns in (the window start
  // rounded down to 16 bytes); rows of 144 bytes put 16 consecutive rows in distinct LDS banks.
  // Q a multiple of 4: the window start is 16-byte aligned, rows hold the 32 columns as eight 16-byte
  // chunks stored in the order chunk ^ (g1 % 8), against bank conflicts.
  constexpr int NCH = (Q % 4 == 0) ? 8 : 9;               // 16-byte chunks per window row
  constexpr int WCH = NS * G * NCH;                       // 16-byte chunks of the window
  constexpr int WCHA = ((WCH + 63) / 64) * 64;            // whole global->LDS loads (64 chunks each)
  __shared__ __attribute__((aligned(16))) float wbuf[WCHA * 4];
  __shared__ int64_t rowBase[kMB * kMB];
  __shared__ int rowLen[kMB * kMB];

  const MCombo *combos = TABLE ? kCombosTable : kCombosDiag;
  const MGroup *groups = TABLE ? kGroupsTable : kGroupsDiag;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, lr = lane & 15, kk = 8 * (lane >> 4);
  // XCD-aware numbering: workgroups b, b + 8, b + 16, ... share an XCD (and its L2); give them
  // neighbouring pencil blocks of one segment, whose coefficient windows overlap
  const int nper = (nlogical + 7) / 8;
  const int logical = (int)(blockIdx.x % 8) * nper + (int)(blockIdx.x / 8);
  if (logical >= nlogical) return;
  const int npb = nb1 * ((pb.n[2] + kMB - 1) / kMB);
  const int seg = logical / npb, pbi = logical % npb;
  const int I1 = (pbi % nb1) * kMB, I2 = (pbi / nb1) * kMB;
  // rows [row_lo, row_hi) of the pencils along axis 0; their element columns start p before row_lo
  // (warm-up columns, whose rows belong to the previous segment and are not emitted)
  const int row_lo = seg * seg_len, row_hi = seg == nseg - 1 ? pb.n[0] : row_lo + seg_len;
  const int e_lo = max(0, row_lo - (P - 1)), e_hi = min(pb.ne[0], row_hi);
  const int E1lo = max(0, I1 - p), E1hi = min(pb.ne[1] - 1, I1 + kMB - 1);
  const int E2lo = max(0, I2 - p), E2hi = min(pb.ne[2] - 1, I2 + kMB - 1);
  const int G1 = (E1hi - E1lo + 1) * Q, G2 = (E2hi - E2lo + 1) * Q;
  const int n0 = pb.n[0], n1 = pb.n[1], n2 = pb.n[2];
  const int64_t G1tot = (int64_t)pb.ne[1] * Q;

  // ---- per-block tables ----
  for (int i = t; i < ME * Q * P; i += NT) {
    const int el = i / (Q * P), r = i % (Q * P);
    const size_t o1 = (size_t)min(E1lo + el, pb.ne[1] - 1) * Q * P + r;
    const size_t o2 = (size_t)min(E2lo + el, pb.ne[2] - 1) * Q * P + r;
    (&tB1[0][0][0][0])[i] = pb.ax[1].B[o1];
    (&tB1[1][0][0][0])[i] = pb.ax[1].dB[o1];
    (&tB2[0][0][0][0])[i] = pb.ax[2].B[o2];
    (&tB2[1][0][0][0])[i] = pb.ax[2].dB[o2];
  }
  // rows of t1 that level 1 never writes (g1 >= 16 MT) enter the 32-deep level-2 reduction: zero
  for (int i = t; i < NL * NK * NN * kLD; i += NT) (&t1[0][0][0][0])[i] = (__bf16)0.f;
  // window entries that no load writes stay finite
  for (int i = t; i < WCHA * 4; i += NT) wbuf[i] = 0.f;
  __syncthreads();
  // Z2_f[n][g2] and Z1_f[m][g1]: products of the 1D factors, zero outside the support overlap and
  // in the padding of the 32-deep reductions
  for (int i = t; i < 2 * 4 * NN * 32; i += NT) {
    const int g = i % 32, n = (i / 32) % NN, f = (i / (32 * NN)) % 4, ax = i / (32 * NN * 4);
    const int il = n / W, o = n % W - p, el = g / Q, q = g % Q;
    const int I = ax ? I2 : I1, Elo = ax ? E2lo : E1lo, Ehi = ax ? E2hi : E1hi, nax = ax ? n2 : n1;
    const int ia = I + il, ja = ia + o, ea = Elo + el;
    double v = 0.0;
    if (g < (ax ? G2 : G1) && ia < nax && ja >= 0 && ja < nax && ea >= max(ia, ja) - p && ea <= min(ia, ja) &&
        ea <= Ehi) {
      const double(*tb)[ME][Q][P] = ax ? tB2 : tB1;
      v = tb[f >> 1][el][q][ia - ea] * tb[f & 1][el][q][ja - ea];
    }
    const float vf = (float)v;
    const __bf16 h = to_bf16(vf);
    __bf16(*z)[4][NN][kLD] = ax ? z2 : z1;
    z[0][f][n][g] = h;
    if constexpr (SPLIT) z[1][f][n][g] = to_bf16(vf - (float)h);
  }

  // ---- level-3 ownership: row pencil (i1l, i2l) and column offsets (o1, o2) ----
  const bool owner = t < S::NOWN;
  const int mo = owner ? t / NN : 0, no = owner ? t % NN : 0;
  const int i1 = I1 + mo / W, i2 = I2 + no / W, j1 = i1 + mo % W - p, j2 = i2 + no % W - p;
  const bool live = owner && i1 < n1 && i2 < n2 && j1 >= 0 && j1 < n1 && j2 >= 0 && j2 < n2;
  float acc[P][W];
#pragma unroll
  for (int a = 0; a < P; ++a)
#pragma unroll
    for (int k = 0; k < W; ++k) acc[a][k] = 0.f;

  // The coefficient window of a step (e0, q0): cs rows E1lo Q + [0, G) (rows past the window's end
  // repeat its last row), columns E2lo Q + [0, 32) (the padding columns meet zero rows of Z2), moved
  // by 16-byte global->LDS loads (lane i to LDS base + 16 i, no registers) issued once level 1 has
  // read the previous window.  The window start E2lo Q is even (E2lo = I2 - p with I2 even, and Q odd
  // only when p is even), so it lies d = 0 or 2 floats past a 16-byte boundary; cs rows are 16-byte
  // multiples (ld % 4 == 0, set on the host).  32-bit offsets inside one step's plane (checked on the
  // host).
  const int ldi = (int)ld, rowoff = E1lo * Q, coloff = E2lo * Q, wd = coloff & 3, cbase = coloff - wd;
  auto dma_step = [&](int step) {
    const float *plane = cs + (int64_t)step * NS * G1tot * ld;
    for (int k = wave; k < WCHA / 64; k += NWAVE) {
      const int f = 64 * k + lane, fr = f / NCH, slot = f % NCH;
      const float *src = plane;                        // chunks past the window (whole loads): any valid value
      if (f < WCH) {
        const int s = fr / G, row = fr % G;
        const int ch = NCH == 8 ? (slot ^ (row & 7)) : slot;   // the logical chunk stored in this slot
        src = plane + (s * (int)G1tot + rowoff + min(row, G1 - 1)) * ldi + cbase + 4 * ch;
      }
      __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)&wbuf[256 * k],
                                       16, 0, 0);
    }
  };
  dma_step(e_lo * Q);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int nsteps = e_hi * Q;

  for (int e0 = e_lo; e0 < e_hi; ++e0) {
    for (int i = t; i < Q * P; i += NT) {
      const size_t o = (size_t)e0 * Q * P + i;
      (&fX0[0][0][0])[i] = (float)pb.ax[0].B[o];
      (&fX0[1][0][0])[i] = (float)pb.ax[0].dB[o];
    }
    __syncthreads();
    for (int q0 = 0; q0 < Q; ++q0) {
      const int step = e0 * Q + q0;
      // ---- level 1: jobs (group, 16-row tile of g1) ----
      for (int job = wave; job < NG * S::MT; job += NWAVE) {
        const MGroup &Gr = groups[job / S::MT];
        const int tm = job % S::MT;
        const int row = min(tm * 16 + lr, G - 1);            // rows past the window: any staged row
        // A operands of the group's streams (register arrays indexed at compile time only)
        bf16x8 ah[3], al[3];
#pragma unroll
        for (int si = 0; si < 3; ++si) {
          if (si >= Gr.ns) break;
          float xs[8];
          if constexpr (NCH == 8) {
            const float *wr = &wbuf[(Gr.s[si] * G + row) * 32];
            const int c0 = kk >> 2, sw = row & 7;
            const float4 x0 = *(const float4 *)&wr[4 * (c0 ^ sw)], x1 = *(const float4 *)&wr[4 * ((c0 + 1) ^ sw)];
            xs[0] = x0.x; xs[1] = x0.y; xs[2] = x0.z; xs[3] = x0.w;
            xs[4] = x1.x; xs[5] = x1.y; xs[6] = x1.z; xs[7] = x1.w;
          } else {
            const float *wr = &wbuf[(Gr.s[si] * G + row) * 36 + wd + kk];      // 8-byte aligned (wd even)
#pragma unroll
            for (int j = 0; j < 8; j += 2) {
              const float2 x = *(const float2 *)&wr[j];
              xs[j] = x.x;
              xs[j + 1] = x.y;
            }
          }
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            ah[si][j] = to_bf16(xs[j]);
            if constexpr (SPLIT) al[si][j] = to_bf16(xs[j] - (float)ah[si][j]);
          }
        }
        f32x4 d0[T16], d1[T16];
#pragma unroll
        for (int tn = 0; tn < T16; ++tn) d0[tn] = d1[tn] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int it = 0; it < 4; ++it) {
          if (it >= Gr.nt) break;
          const MTerm T = Gr.t[it];
          const bf16x8 a = T.si == 0 ? ah[0] : T.si == 1 ? ah[1] : ah[2];
          bf16x8 b = a;
          if constexpr (SPLIT) b = T.si == 0 ? al[0] : T.si == 1 ? al[1] : al[2];
#pragma unroll
          for (int tn = 0; tn < T16; ++tn) {
            const int col = min(tn * 16 + lr, NN - 1);
            const bf16x8 bh = *(const bf16x8 *)&z2[0][T.f2][col][kk];
            f32x4 dd = T.slot ? d1[tn] : d0[tn];
            if constexpr (SPLIT) {
              const bf16x8 bl = *(const bf16x8 *)&z2[1][T.f2][col][kk];
              dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b, bh, dd, 0, 0, 0);
              dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, dd, 0, 0, 0);
            }
            dd = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bh, dd, 0, 0, 0);
            if (T.slot) d1[tn] = dd;
            else d0[tn] = dd;
          }
        }
        // D[g1 = tm*16 + 4 (lane / 16) + i][n = tn*16 + lane % 16] -> t1[k][n][g1]
#pragma unroll
        for (int sl = 0; sl < 2; ++sl) {
          if (sl >= Gr.nk) break;
          const int k = Gr.k[sl];
#pragma unroll
          for (int tn = 0; tn < T16; ++tn) {
            const int n = tn * 16 + lr;
            if (n >= NN) continue;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int g1 = tm * 16 + 4 * (lane >> 4) + i;
              const float x = sl ? d1[tn][i] : d0[tn][i];
              const __bf16 h = to_bf16(x);
              t1[0][k][n][g1] = h;
              if constexpr (SPLIT) t1[1][k][n][g1] = to_bf16(x - (float)h);
            }
          }
        }
      }
      __syncthreads();
      if (step + 1 < nsteps) dma_step(step + 1);        // level 1 has read the window; in flight during levels 2, 3
      // ---- level 2: jobs (c0, 16-row tile of m, 16-column tile of n) ----
      for (int job = wave; job < 4 * T16 * T16; job += NWAVE) {
        const int c = job / (T16 * T16), tm = (job / T16) % T16, tn = job % T16;
        const int row = min(tm * 16 + lr, NN - 1), col = min(tn * 16 + lr, NN - 1);
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < NK; ++k) {
          if (combos[k].c0 != c) continue;
          const int f1 = combos[k].f1;
          const bf16x8 ah = *(const bf16x8 *)&z1[0][f1][row][kk];
          const bf16x8 bh = *(const bf16x8 *)&t1[0][k][col][kk];
          if constexpr (SPLIT) {
            const bf16x8 al = *(const bf16x8 *)&z1[1][f1][row][kk];
            const bf16x8 bl = *(const bf16x8 *)&t1[1][k][col][kk];
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, d, 0, 0, 0);
            d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, d, 0, 0, 0);
          }
          d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, d, 0, 0, 0);
        }
        const int n = tn * 16 + lr;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int m = tm * 16 + 4 * (lane >> 4) + i;
          if (m < NN && n < NN) T2[c][m][n] = d[i];
        }
      }
      __syncthreads();
      // ---- level 3 (FP32): axis-0 factors of this Gauss point into the register window ----
      if (live) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (!TABLE && (c == 1 || c == 2)) continue;      // x = xi: no mixed axis-0 terms
          const float v = T2[c][mo][no];
          const int x0 = c >> 1, y0 = c & 1;
#pragma unroll
          for (int a0 = 0; a0 < P; ++a0) {
            const float xa = fX0[x0][q0][a0] * v;
#pragma unroll
            for (int b0 = 0; b0 < P; ++b0) acc[a0][b0 - a0 + p] += xa * fX0[y0][q0][b0];
          }
        }
      }
      __builtin_amdgcn_s_waitcnt(0);                    // this wave's window loads have landed
      __syncthreads();                                  // ... and every wave's
    }
    // ---- emit the completed row(s) of this column: each owner stages its W values of a row in CSR
    // order (the row's columns are the tensor product of the per-axis ranges, axis 0 fastest), then
    // the block writes its rows as contiguous runs ----
    const int last = (e0 == pb.ne[0] - 1) ? p : 0;
    for (int a0 = 0; a0 <= last; ++a0) {
      const int i0 = e0 + a0;
      if (i0 < row_lo || i0 >= row_hi) continue;          // uniform: a warm-up column's row
      if (t < kMB * kMB) {
        const int ri1 = I1 + (t & 1), ri2 = I2 + (t >> 1);
        rowLen[t] = 0;
        if (ri1 < n1 && ri2 < n2) {
          rowBase[t] = pb.row_ptr[i0 + (int64_t)n0 * (ri1 + (int64_t)n1 * ri2)];
          rowLen[t] = pb.ax[0].stw[i0] * pb.ax[1].stw[ri1] * pb.ax[2].stw[ri2];
        }
      }
      if (live) {
        const bool rowDir = is_dirichlet_idx(pb, i0, i1, i2);
        const int64_t A = i0 + (int64_t)n0 * (i1 + (int64_t)n1 * i2);
        const double wA = (TABLE && pb.rational) ? pb.wts[A] : 1.0;
        const int l0 = pb.ax[0].stl[i0], w0 = pb.ax[0].stw[i0], w1 = pb.ax[1].stw[i1];
        const int seg = ((j2 - pb.ax[2].stl[i2]) * w1 + (j1 - pb.ax[1].stl[i1])) * w0 - l0;
        float *dst = &rowbuf[(mo / W) + kMB * (no / W)][0];
#pragma unroll
        for (int k = 0; k < W; ++k) {
          const int j0 = i0 + k - p;
          if (j0 < 0 || j0 >= n0) continue;
          double v;
          if (rowDir) v = (j0 == i0 && j1 == i1 && j2 == i2) ? 1.0 : 0.0;
          else if (is_dirichlet_idx(pb, j0, j1, j2)) v = 0.0;
          else {
            float av = 0.f;
#pragma unroll
            for (int a = 0; a < P; ++a)
              if (a == a0) av = acc[a][k];                // register window row a0 (no dynamic indexing)
            v = (double)av;
            if (TABLE && pb.rational) v *= wA * pb.wts[j0 + (int64_t)n0 * (j1 + (int64_t)n1 * j2)];
          }
          dst[seg + j0] = (float)v;
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kMB * kMB; ++r)
        for (int i = t; i < rowLen[r]; i += NT) __builtin_nontemporal_store(rowbuf[r][i], &vals[rowBase[r] + i]);
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < P - 1; ++a)
#pragma unroll
      for (int k = 0; k < W; ++k) acc[a][k] = acc[a + 1][k];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[P - 1][k] = 0.f;
  }
}

// coefficient-stream buffer: rows of ne2 Q + kPad floats (the padding zeroed once, at allocation)
iga_status ensure_cs(Handle &h, int64_t *ld) {
  const int Q = h.pb.Q, NS = h.pb.table ? 10 : 2;
  *ld = (((int64_t)h.pb.ne[2] * Q + kPad + 3) / 4) * 4;     // 16-byte rows (the window loads)
  const size_t bytes = (size_t)h.pb.ne[0] * Q * NS * (size_t)h.pb.ne[1] * Q * (size_t)(*ld) * sizeof(float);
  if (h.mma_cs && h.mma_cs_bytes == bytes) return IGA_OK;
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) return fail(IGA_ENOMEM, std::string("hipMalloc (coefficient streams): ") + hipGetErrorString(e));
  h.owned.push_back(q);
  IGA_HIP_CHECK(hipMemsetAsync(q, 0, bytes, h.stream));
  h.mma_cs = (float *)q;
  h.mma_cs_bytes = bytes;
  return IGA_OK;
}

template <int P, bool TABLE, bool SPLIT>
iga_status run_mma(Handle &h, const double *U, float *vals) {
  int64_t ld = 0;
  iga_status st = ensure_cs(h, &ld);
  if (st) return st;
  if ((double)(TABLE ? 10 : 2) * h.pb.ne[1] * h.pb.Q * (double)ld >= 2147483647.0)
    return fail(IGA_EUNSUPPORTED, "BF16 matrix-core Jacobian: a coefficient plane exceeds 32-bit offsets");
  kt_begin(h, "k_cs3");
  hipLaunchKernelGGL((k_cs3<P, TABLE>), dim3((unsigned)(h.pb.ne[0] * h.pb.ne[1])), dim3(256), 0, h.stream, h.pb, U,
                     h.mma_cs, ld);
  kt_end(h);
  IGA_HIP_CHECK(hipGetLastError());
  const int nb1 = (h.pb.n[1] + kMB - 1) / kMB, nb2 = (h.pb.n[2] + kMB - 1) / kMB, npb = nb1 * nb2;
  // segments along axis 0 (IGA_OPT_ROW_SEGMENTS, else planned): minimise (rounds of resident blocks) x
  // (element columns per block), a segment's p warm-up columns weighted twice (they also restart the
  // window stream).  Measured on the quarter cylinder 48^3, Jacobian in ms for 1 / 2 / 3 / 4 segments:
  // p = 4 BF16 4.25 / 4.81 / 4.61 / 5.01, split 5.04 / 5.73 / 5.48 / 5.96; p = 3 BF16 1.46 / 1.59 / 1.64 /
  // 1.69, split 2.38 / 2.26 / 2.21 / 2.32; p = 2 BF16 0.755 / 0.768 / 0.661 / 0.697, split 0.855 / 0.887 /
  // 0.878 / 0.873 (the rule picks 1, 1, 1, 3, 3, 1).
  const int ne0 = h.pb.ne[0], p = h.pb.P - 1;
  int nseg = h.row_segments;
  if (nseg <= 0) {
    int per_cu = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_rgmma3<P, TABLE, SPLIT>, MShape<P>::NT, 0) !=
            hipSuccess || per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, h.device) != hipSuccess || ncu < 1)
      ncu = 256;
    const long slots = (long)per_cu * ncu;
    double best = 1e300;
    nseg = 1;
    for (int s = 1; s <= 16 && s <= ne0; ++s) {
      const int len = (ne0 + s - 1) / s, ns = (ne0 + len - 1) / len;
      const double cost = (double)((npb * (long)ns + slots - 1) / slots) * (len + (ns > 1 ? 2 * p : 0));
      if (cost < best) { best = cost; nseg = s; }
    }
  }
  if (nseg > ne0) nseg = ne0;
  const int seg_len = (ne0 + nseg - 1) / nseg;
  nseg = (ne0 + seg_len - 1) / seg_len;
  const int nlogical = npb * nseg, grid = ((nlogical + 7) / 8) * 8;
  kt_begin(h, SPLIT ? "k_rgmma3 (split BF16)" : "k_rgmma3 (BF16)");
  hipLaunchKernelGGL((k_rgmma3<P, TABLE, SPLIT>), dim3((unsigned)grid), dim3(MShape<P>::NT), 0, h.stream, h.pb,
                     (const float *)h.mma_cs, ld, vals, nb1, seg_len, nseg, nlogical);
  kt_end(h);
  IGA_HIP_CHECK(hipGetLastError());
  return IGA_OK;
}

template <int P>
iga_status pick_mma(Handle &h, const double *U, float *vals, bool split) {
  if (h.pb.table) return split ? run_mma<P, true, true>(h, U, vals) : run_mma<P, true, false>(h, U, vals);
  return split ? run_mma<P, false, true>(h, U, vals) : run_mma<P, false, false>(h, U, vals);
}

}  // namespace

bool mma_supported(const DevProblem &pb) {
  return pb.dim == 3 && pb.simple_knots && !pb.periodic && pb.P >= 3 && pb.P <= 5;
}

iga_status launch_jac_mma(Handle &h, const double *U, float *vals, bool split) {
  if (!mma_supported(h.pb))
    return fail(IGA_EUNSUPPORTED, "BF16 matrix-core Jacobian: 3D, open axes, simple interior knots, degree 2..4");
  switch (h.pb.P) {
    case 3: return pick_mma<3>(h, U, vals, split);
    case 4: return pick_mma<4>(h, U, vals, split);
    case 5: return pick_mma<5>(h, U, vals, split);
  }
  return fail(IGA_EUNSUPPORTED, "BF16 matrix-core Jacobian degree");
}

}  // namespace iga
