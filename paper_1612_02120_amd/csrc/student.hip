// Student network: conv5x5 1->8 ReLU, conv3x3 8->8 ReLU, conv1x1 8->1 sigmoid
// (receptive radius 6). A thinner net that runs everywhere as the fast pass;
// tiles where it disagrees with the plain net on sampled windows fall back to
// the plain net (multi-pass: extra effort only where errors are likely,
// arXiv 1612.02120, Sections 1 and 3).
//
// Parameters (801) in the cnn_create layout: W1[8][1][5][5], b1[8],
// W2[8][8][3][3], b2[8], Wh[8], bh. The library keeps FP32 master weights,
// Adam moments, and "working" weights used by the kernels: W1 / 255 (the input
// is the raw uint8 value) and, in BF16 mode, W1 / 255 and W2 rounded to bf16.
// In BF16 mode conv2's input (h1) and the backward operands dh1, dh2 are also
// rounded to bf16; every product of two bf16 values is exact in FP32 and sums
// accumulate in FP32. The head runs in FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/emcnn.h"
#include "common.h"
#include "device_util.h"
#include "runtime.h"

namespace emcnn {

constexpr int S_C = 8;  // student channels
constexpr int S_NP = 801;
constexpr int OFF_W1 = 0, OFF_B1 = 200, OFF_W2 = 208, OFF_B2 = 784, OFF_WH = 792, OFF_BH = 800;

__device__ __forceinline__ float s_relu(float v) { return v > 0.0f ? v : 0.0f; }
__device__ __forceinline__ float s_bf16(float v) { return (float)(__bf16)v; }
__device__ __forceinline__ float s_sigmoid(float t) {
  if (t >= 0.0f) return 1.0f / (1.0f + expf(-t));
  float e = expf(t);
  return e / (1.0f + e);
}

// ------------------------------------------------------------------ fused inference

// out(z, y, x) = student probability at student-output position (y + crop, x + crop)
// of slice z; student output (y, x) is centred on input (y + 3, x + 3).
template <int TY, int TX>
__global__ __launch_bounds__((TY * TX)) void student_fused(const uint8_t* __restrict__ in, int64_t in_rs, int64_t in_zs,
                                                           float* __restrict__ out, int64_t out_rs, int64_t out_zs,
                                                           int Ho, int Wo, int crop, const float* __restrict__ ww,
                                                           int bf16) {
  constexpr int IR = TY + 6, IC = TX + 6, HR = TY + 2, HC = TX + 2;
  __shared__ float xin[IR * IC];
  __shared__ float h1[S_C][HR * HC];
  const int tid = threadIdx.x;
  const int y0 = blockIdx.y * TY, x0 = blockIdx.x * TX, z = blockIdx.z;
  const uint8_t* src = in + (int64_t)z * in_zs;
  // input rows needed: student coords y0+crop .. +TY+5 (clamped to the last valid input row)
  const int hin_lim = Ho + 2 * crop + 6, win_lim = Wo + 2 * crop + 6;  // input dims implied by the output
  for (int t = tid; t < IR * IC; t += TY * TX) {
    int r = t / IC, c = t % IC;
    int y = min(y0 + crop + r, hin_lim - 1), x = min(x0 + crop + c, win_lim - 1);
    xin[t] = (float)src[(int64_t)y * in_rs + x];
  }
  __syncthreads();
  for (int t = tid; t < HR * HC; t += TY * TX) {
    const int r = t / HC, c = t % HC;
    float a[S_C];
#pragma unroll
    for (int co = 0; co < S_C; ++co) a[co] = ww[OFF_B1 + co];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const float xv = xin[(r + i) * IC + c + j];
#pragma unroll
        for (int co = 0; co < S_C; ++co) a[co] = fmaf(ww[OFF_W1 + co * 25 + i * 5 + j], xv, a[co]);
      }
#pragma unroll
    for (int co = 0; co < S_C; ++co) {
      float v = s_relu(a[co]);
      h1[co][t] = bf16 ? s_bf16(v) : v;
    }
  }
  __syncthreads();
  const int ty = tid / TX, tx = tid % TX;
  float a2[S_C];
#pragma unroll
  for (int co = 0; co < S_C; ++co) a2[co] = ww[OFF_B2 + co];
#pragma unroll
  for (int ci = 0; ci < S_C; ++ci)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float hv = h1[ci][(ty + i) * HC + tx + j];
#pragma unroll
        for (int co = 0; co < S_C; ++co) a2[co] = fmaf(ww[OFF_W2 + (co * 8 + ci) * 9 + i * 3 + j], hv, a2[co]);
      }
  float zl = ww[OFF_BH];
#pragma unroll
  for (int co = 0; co < S_C; ++co) zl = fmaf(ww[OFF_WH + co], s_relu(a2[co]), zl);
  const int y = y0 + ty, x = x0 + tx;
  if (y < Ho && x < Wo) out[(int64_t)z * out_zs + (int64_t)y * out_rs + x] = s_sigmoid(zl);
}

// BF16 mode on MFMA. Both convs run as D = W X on 16x16x32 bf16 MFMAs: the
// working weights and h1 are bf16 values and uint8 inputs are exact in bf16,
// so every product is exact and sums are FP32 (in the MFMA's order). The 8
// output channels fill half of the MFMA's 16 rows: lane (g, n) receives
// channels 4g..4g+3 of pixel n, lanes g >= 2 the zero-weight rows. One
// workgroup of 4 waves computes a TY x TX output tile:
//   input: the uint8 tile converted once to bf16 in LDS (the high half of
//          the float of a byte, whose low half is zero);
//   conv1: h1 for (TY+2) x (16 ceil((TX+2)/16)) positions, one MFMA per 16
//          pixels (K = 25 taps padded to 32), bias, ReLU, bf16 -> LDS
//          (16 bytes per position: 8 channels); wave w takes the h1 rows
//          w, w + 4, ..., so its LDS offsets are a per-lane base plus
//          compile-time immediates;
//   conv2: K = 9 taps x 8 channels in 3 MFMAs per 16 outputs (taps 4s + g,
//          padded to 12), one 16-byte LDS read per lane per MFMA;
//   head:  each lane's 4-channel partial dot; the two real lane groups' sums
//          are gathered for four m-blocks at a time, so that lane group j
//          holds m-block j's 16 probabilities and one sigmoid and one store
//          per lane serve four m-blocks.
template <int TY, int TX>
__global__ __launch_bounds__(256) void student_mfma(const uint8_t* in, int64_t in_rs, int64_t in_zs, float* out,
                                                    int64_t out_rs, int64_t out_zs, int Ho, int Wo, int crop,
                                                    const float* ww) {
  constexpr int HR = TY + 2;               // h1 rows
  constexpr int HMC = (TX + 2 + 15) / 16;  // h1 m-blocks per row
  constexpr int HC = HMC * 16;             // h1 row pitch (positions)
  constexpr int IR = HR + 4, IC = HC + 4;  // input tile (covers the padded h1 columns)
  constexpr int OMC = TX / 16;             // output m-blocks per row
  static_assert(TX % 16 == 0, "output m-blocks of 16 pixels");
  static_assert(OMC == 4 && TY % 4 == 0, "wave w owns output m-block column w; rows in groups of four");
  __shared__ __attribute__((aligned(16))) unsigned short xin[IR * IC];  // bf16 bits
  __shared__ __attribute__((aligned(16))) unsigned char h1[HR * HC * 16];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4, n16 = lane & 15;
  const int y0 = blockIdx.y * TY, x0 = blockIdx.x * TX, z = blockIdx.z;
  const gbyte* src = gin(in) + (int64_t)z * in_zs;
  const int hin_lim = Ho + 2 * crop + 6, win_lim = Wo + 2 * crop + 6;  // input dims implied by the output
  {
    // rows wave + 4k, columns lane + 64 m: all byte loads issued before any is used
    constexpr int NK = (IR + 3) / 4, NM = (IC + 63) / 64;
    unsigned int b[NK][NM];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const gbyte* row = src + (int64_t)min(y0 + crop + wave + 4 * k, hin_lim - 1) * in_rs;
#pragma unroll
      for (int m = 0; m < NM; ++m) b[k][m] = row[min(x0 + crop + lane + 64 * m, win_lim - 1)];
    }
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll
      for (int m = 0; m < NM; ++m)
        if (wave + 4 * k < IR && lane + 64 * m < IC)
          xin[(wave + 4 * k) * IC + lane + 64 * m] =
              (unsigned short)(__builtin_bit_cast(unsigned int, (float)b[k][m]) >> 16);
  }
  // weight fragments: lane (g, c) holds output channel c's K elements 8g..8g+7
  // (every load is unconditional, from a clamped index, and the padding is
  // selected afterwards, so that all of them are in flight together)
  const bool realc = n16 < S_C;
  const int c8 = realc ? n16 : 0;
  float w1v[8], w2v[3][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) w1v[e] = ldf(ww, OFF_W1 + c8 * 25 + min(8 * g + e, 24));
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3)
#pragma unroll
    for (int e = 0; e < 8; ++e) w2v[s3][e] = ldf(ww, OFF_W2 + (c8 * 8 + e) * 9 + min(4 * s3 + g, 8));
  const bool realg = g < 2;  // this lane's rows are real channels 4g..4g+3
  float b1[4], b2[4], wh[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int co = realg ? 4 * g + k : 0;
    b1[k] = ldf(ww, OFF_B1 + co);
    b2[k] = ldf(ww, OFF_B2 + co);
    wh[k] = ldf(ww, OFF_WH + co);
    wh[k] = realg ? wh[k] : 0.f;
  }
  const float bh = ldf(ww, OFF_BH);
  bf16x8 w1f, w2f[3];
#pragma unroll
  for (int e = 0; e < 8; ++e) w1f[e] = (__bf16)(realc && 8 * g + e < 25 ? w1v[e] : 0.f);
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3)
#pragma unroll
    for (int e = 0; e < 8; ++e) w2f[s3][e] = (__bf16)(realc && 4 * s3 + g < 9 ? w2v[s3][e] : 0.f);
  // per-lane bases of the tap reads in the bf16 tile, at h1 row `wave`
  // (taps past 25 read element 0 of that row: zero weights)
  const unsigned short* xb[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int t = 8 * g + e;
    xb[e] = xin + wave * IC + n16 + (t < 25 ? (t / 5) * IC + t % 5 : 0);
  }
  unsigned char* const h1w = h1 + ((wave * HC + n16) * 16 + g * 8);
  __syncthreads();
  // ---- conv1: h1 rows wave + 4k
#pragma unroll
  for (int k = 0; k < (HR + 3) / 4; ++k) {
    if (wave + 4 * k < HR) {
#pragma unroll
      for (int mc = 0; mc < HMC; ++mc) {
        const int off = 4 * k * IC + mc * 16;  // compile-time
        u4v pk;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          pk[e] = (unsigned)xb[2 * e][off] | ((unsigned)xb[2 * e + 1][off] << 16);
        const f4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w1f, __builtin_bit_cast(bf16x8, pk),
                                                             f4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        if (realg) {
          const __bf16 h0 = (__bf16)s_relu(d[0] + b1[0]), h1v = (__bf16)s_relu(d[1] + b1[1]);
          const __bf16 h2 = (__bf16)s_relu(d[2] + b1[2]), h3 = (__bf16)s_relu(d[3] + b1[3]);
          const u2v wv = {(unsigned)__builtin_bit_cast(unsigned short, h0) |
                              ((unsigned)__builtin_bit_cast(unsigned short, h1v) << 16),
                          (unsigned)__builtin_bit_cast(unsigned short, h2) |
                              ((unsigned)__builtin_bit_cast(unsigned short, h3) << 16)};
          st<u2v>(h1w + (4 * k * HC + mc * 16) * 16, wv);
        }
      }
    }
  }
  __syncthreads();
  // ---- conv2 + head: output rows 0..TY-1 of m-block column `wave`
  int hoff[3];
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3) {
    const int t = 4 * s3 + g < 9 ? 4 * s3 + g : 0;  // padded taps: zero weights
    hoff[s3] = ((t / 3) * HC + t % 3) * 16;
  }
  const unsigned char* const b0w = h1 + (wave * 16 + n16) * 16;
  const int x = x0 + wave * 16 + n16;
#pragma unroll
  for (int grp = 0; grp < TY / 4; ++grp) {
    float mine = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned char* b0 = b0w + (4 * grp + j) * HC * 16;
      f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s3 = 0; s3 < 3; ++s3)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w2f[s3], ld<bf16x8>(b0 + hoff[s3]), acc, 0, 0, 0);
      float part = 0.f;
#pragma unroll
      for (int k = 0; k < 4; ++k) part = fmaf(wh[k], s_relu(acc[k] + b2[k]), part);
      // channels 0..3 (lane group 0) + 4..7 (lane group 1) of pixel n16
      const float sum = __shfl(part, n16) + __shfl(part, n16 + 16);
      mine = g == j ? sum : mine;
    }
    const int y = y0 + 4 * grp + g;
    if (y < Ho && x < Wo) st<float>(gout(out) + ((int64_t)z * out_zs + (int64_t)y * out_rs + x) * 4,
                                   s_sigmoid(mine + bh));
  }
}

// ------------------------------------------------------------------ training kernels

// h1[b][y][x][c] over (P-4)^2 positions (post-ReLU; bf16-valued in BF16 mode)
__global__ void st_conv1(const uint8_t* __restrict__ patches, int B, int P, const float* __restrict__ ww,
                         float* __restrict__ h1, int bf16) {
  const int P1 = P - 4;
  const int64_t n = (int64_t)B * P1 * P1;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(p / ((int64_t)P1 * P1));
    const int rem = (int)(p % ((int64_t)P1 * P1));
    const int y = rem / P1, x = rem % P1;
    const uint8_t* s = patches + (int64_t)b * P * P + (int64_t)y * P + x;
    float a[S_C];
#pragma unroll
    for (int co = 0; co < S_C; ++co) a[co] = ww[OFF_B1 + co];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
      for (int j = 0; j < 5; ++j) {
        const float xv = (float)s[i * P + j];
#pragma unroll
        for (int co = 0; co < S_C; ++co) a[co] = fmaf(ww[OFF_W1 + co * 25 + i * 5 + j], xv, a[co]);
      }
#pragma unroll
    for (int co = 0; co < S_C; ++co) {
      float v = s_relu(a[co]);
      h1[p * S_C + co] = bf16 ? s_bf16(v) : v;
    }
  }
}

// conv2 + head + BCE: h2 (FP32), dz = (sigmoid(z) - t)/N, dh2 = dz wh [h2 > 0]
// (bf16-valued in BF16 mode), and one FP64 partial of sum(softplus(z) - t z)
// per block (fixed-order tree inside the block).
__global__ __launch_bounds__(256) void st_conv2_loss(const float* __restrict__ h1, int B, int P,
                                                      const float* __restrict__ ww, const float* __restrict__ teacher,
                                                      float* __restrict__ h2, float* __restrict__ dz,
                                                      float* __restrict__ dh2, double* __restrict__ loss_part,
                                                      double invN, int bf16) {
  __shared__ double red[256];
  const int P1 = P - 4, P2 = P - 6;
  const int64_t n = (int64_t)B * P2 * P2;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double term = 0.0;
  if (p < n) {
    const int b = (int)(p / ((int64_t)P2 * P2));
    const int rem = (int)(p % ((int64_t)P2 * P2));
    const int y = rem / P2, x = rem % P2;
    float a[S_C];
#pragma unroll
    for (int co = 0; co < S_C; ++co) a[co] = ww[OFF_B2 + co];
    const float* hb = h1 + ((int64_t)b * P1 * P1) * S_C;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const float* hp = hb + ((int64_t)(y + i) * P1 + x + j) * S_C;
#pragma unroll
        for (int ci = 0; ci < S_C; ++ci) {
          const float hv = hp[ci];
#pragma unroll
          for (int co = 0; co < S_C; ++co) a[co] = fmaf(ww[OFF_W2 + (co * 8 + ci) * 9 + i * 3 + j], hv, a[co]);
        }
      }
    float zl = ww[OFF_BH];
#pragma unroll
    for (int co = 0; co < S_C; ++co) {
      a[co] = s_relu(a[co]);
      h2[p * S_C + co] = a[co];
      zl = fmaf(ww[OFF_WH + co], a[co], zl);
    }
    const float t = teacher[p];
    const float g = (s_sigmoid(zl) - t) * (float)invN;
    dz[p] = g;
#pragma unroll
    for (int co = 0; co < S_C; ++co) {
      float d = a[co] > 0.0f ? g * ww[OFF_WH + co] : 0.0f;
      dh2[p * S_C + co] = bf16 ? s_bf16(d) : d;
    }
    const double zd = (double)zl;
    term = fmax(zd, 0.0) + log1p(exp(-fabs(zd))) - (double)t * zd;
  }
  red[threadIdx.x] = term;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// dh1 = sum_{co,i,j} W2[co][ci][i][j] dh2[co][y-i][x-j], masked by h1 > 0
__global__ void st_dh1(const float* __restrict__ dh2, const float* __restrict__ h1, int B, int P,
                       const float* __restrict__ ww, float* __restrict__ dh1, int bf16) {
  const int P1 = P - 4, P2 = P - 6;
  const int64_t n = (int64_t)B * P1 * P1;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(p / ((int64_t)P1 * P1));
    const int rem = (int)(p % ((int64_t)P1 * P1));
    const int y = rem / P1, x = rem % P1;
    float a[S_C];
#pragma unroll
    for (int ci = 0; ci < S_C; ++ci) a[ci] = 0.f;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int yy = y - i, xx = x - j;
        if (yy < 0 || xx < 0 || yy >= P2 || xx >= P2) continue;
        const float* d = dh2 + (((int64_t)b * P2 + yy) * P2 + xx) * S_C;
#pragma unroll
        for (int co = 0; co < S_C; ++co) {
          const float dv = d[co];
#pragma unroll
          for (int ci = 0; ci < S_C; ++ci) a[ci] = fmaf(ww[OFF_W2 + (co * 8 + ci) * 9 + i * 3 + j], dv, a[ci]);
        }
      }
#pragma unroll
    for (int ci = 0; ci < S_C; ++ci) {
      float v = h1[p * S_C + ci] > 0.0f ? a[ci] : 0.0f;
      dh1[p * S_C + ci] = bf16 ? s_bf16(v) : v;
    }
  }
}

// Partial weight gradients over a chunk of positions: one thread per
// parameter of the layer, positions in ascending order, FP32 accumulation.
// layer 0: dY = dh1 (P-4)^2 x 8, X = uint8 patch / 255 (5x5, 1 channel)
// layer 1: dY = dh2 (P-6)^2 x 8, X = h1 (3x3, 8 channels)
// layer 2: dY = dz  (P-6)^2 x 1, X = h2 (1x1, 8 channels)
template <int LAYER>
__global__ __launch_bounds__(1024) void st_wgrad(const float* __restrict__ dY, const void* __restrict__ X, int B, int P,
                                                 int chunk, float* __restrict__ part) {
  constexpr int K = LAYER == 0 ? 5 : LAYER == 1 ? 3 : 1;
  constexpr int CI = LAYER == 0 ? 1 : 8;
  constexpr int CO = LAYER == 2 ? 1 : 8;
  constexpr int NW = CO * CI * K * K;
  constexpr int NE = NW + CO;
  constexpr int U = 32;  // positions whose loads are issued together
  const int Ho = LAYER == 0 ? P - 4 : P - 6;
  const int Hi = Ho + K - 1;
  const int64_t n = (int64_t)B * Ho * Ho;
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  const int64_t p1 = min(n, p0 + chunk);
  for (int e = threadIdx.x; e < NE; e += blockDim.x) {
    // element e: weight (co, ci, i, j), or the bias of co (then ci = i = j = 0
    // and the input is not read)
    const bool wt = e < NW;
    const int co = wt ? e / (CI * K * K) : e - NW, r = wt ? e % (CI * K * K) : 0;
    const int ci = r / (K * K), i = (r % (K * K)) / K, j = r % K;
    // position p0 as (b, y, x), advanced one position at a time below (no
    // division per position); the sum runs over p = p0 .. p1 - 1 in order
    int b = (int)(p0 / ((int64_t)Ho * Ho));
    const int rem = (int)(p0 % ((int64_t)Ho * Ho));
    int y = rem / Ho, x = rem % Ho;
    float acc = 0.f;
    for (int64_t pb = p0; pb < p1; pb += U) {
      float dv[U], xv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool live = pb + u < p1;
        const int64_t pp = live ? pb + u : p0;
        dv[u] = dY[pp * CO + co];
        const int64_t xi = ((int64_t)b * Hi + y + i) * Hi + x + j;
        if constexpr (LAYER == 0) xv[u] = (float)reinterpret_cast<const uint8_t*>(X)[live ? xi : 0] * (1.0f / 255.0f);
        else xv[u] = reinterpret_cast<const float*>(X)[(live ? xi : 0) * CI + ci];
        if (++x == Ho) {
          x = 0;
          if (++y == Ho) {
            y = 0;
            ++b;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (pb + u < p1) acc = wt ? fmaf(dv[u], xv[u], acc) : acc + dv[u];
      }
    }
    part[(int64_t)blockIdx.x * NE + e] = acc;
  }
}

struct ReduceArgs {
  const float* part[3];
  int nchunk[3];
  const double* loss_part;
  int nloss;
  double invN;
  float* master;
  float* m;
  float* v;
  float* ww;
  float* grad_out;
  double* loss_out;
  double* gnorm_out;
  int do_update;
  int bf16;
  float lr, b1, b2, eps;
  float c1, c2;  // 1 - b1^t, 1 - b2^t
};

__device__ __forceinline__ void refresh_working(float* ww, const float* master, int e, int bf16) {
  float w = master[e];
  if (e < OFF_B1) w = w * (1.0f / 255.0f);  // the kernels read raw uint8 input
  if (bf16 && (e < OFF_B1 || (e >= OFF_W2 && e < OFF_B2))) w = s_bf16(w);
  ww[e] = w;
}

// One block of 1024 threads: fixed-order reduction of the chunk partials into
// the gradient, FP64 sums of the loss and of g^2, and the Adam update.
__global__ __launch_bounds__(1024) void st_reduce_adam(ReduceArgs a) {
  __shared__ double red[1024];
  const int e = threadIdx.x;
  float g = 0.f;
  if (e < S_NP) {
    int layer, local, ne;
    if (e < OFF_W2) {
      layer = 0;
      local = e;
      ne = OFF_W2;
    } else if (e < OFF_WH) {
      layer = 1;
      local = e - OFF_W2;
      ne = OFF_WH - OFF_W2;
    } else {
      layer = 2;
      local = e - OFF_WH;
      ne = S_NP - OFF_WH;
    }
    for (int c = 0; c < a.nchunk[layer]; ++c) g += a.part[layer][(int64_t)c * ne + local];
    if (a.grad_out) a.grad_out[e] = g;
  }
  red[e] = (double)g * (double)g;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (e < s) red[e] += red[e + s];
    __syncthreads();
  }
  const double g2 = red[0];
  __syncthreads();
  // loss: fixed-order sum of the per-block FP64 partials
  double l = 0.0;
  for (int i = e; i < a.nloss; i += 1024) l += a.loss_part[i];
  red[e] = l;
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (e < s) red[e] += red[e + s];
    __syncthreads();
  }
  if (e == 0) {
    if (a.loss_out) *a.loss_out = red[0] * a.invN;
    if (a.gnorm_out) *a.gnorm_out = sqrt(g2);
  }
  if (e < S_NP && a.do_update) {
    const float m = a.b1 * a.m[e] + (1.0f - a.b1) * g;
    const float v = a.b2 * a.v[e] + (1.0f - a.b2) * g * g;
    a.m[e] = m;
    a.v[e] = v;
    const float mh = m / a.c1, vh = v / a.c2;
    a.master[e] = a.master[e] - a.lr * mh / (sqrtf(vh) + a.eps);
    refresh_working(a.ww, a.master, e, a.bf16);
  }
}

__global__ void st_refresh(float* ww, const float* master, int bf16) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < S_NP) refresh_working(ww, master, e, bf16);
}

// ------------------------------------------------------------------ fallback decisions

// One block per fallback tile: counts sampled voxels whose 0.5-threshold
// decision differs between the student map (already in `prob`) and the
// teacher's sample windows; flags the tile when flips > tau * count.
__global__ __launch_bounds__(256) void st_flag_tiles(const float* __restrict__ prob, int64_t rs, int64_t zs,
                                                      const float* __restrict__ samples, const int32_t* __restrict__ win,
                                                      int n_samples, float tau, int32_t* __restrict__ flags) {
  __shared__ int cnt[256], tot[256];
  const int t = blockIdx.x;
  int c = 0, n = 0;
  for (int s = 0; s < n_samples; ++s) {
    const int32_t* w = win + ((int64_t)t * n_samples + s) * 5;  // z, y, x, h, w
    const int wh = w[3], wwid = w[4];
    const float* sp = samples + ((int64_t)t * n_samples + s) * 256;
    for (int q = threadIdx.x; q < wh * wwid; q += blockDim.x) {
      const int yy = q / wwid, xx = q % wwid;
      const float st = prob[(int64_t)w[0] * zs + (int64_t)(w[1] + yy) * rs + w[2] + xx];
      const float te = sp[yy * 16 + xx];
      c += ((st >= 0.5f) != (te >= 0.5f)) ? 1 : 0;
      n += 1;
    }
  }
  cnt[threadIdx.x] = c;
  tot[threadIdx.x] = n;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      cnt[threadIdx.x] += cnt[threadIdx.x + s];
      tot[threadIdx.x] += tot[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) flags[t] = ((float)cnt[0] > tau * (float)tot[0]) ? 1 : 0;
}

__global__ __launch_bounds__(256) void st_count_flags(const int32_t* __restrict__ flags, int n, int32_t* stats) {
  __shared__ int red[256];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 256) c += flags[i];
  red[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = red[0];
    stats[1] = n;
  }
}

// ------------------------------------------------------------------ training batches

// One training batch gathered from device volumes and their teacher maps:
// block (., b) copies patch b (P x P bytes) and its centred targets
// ((P-6) x (P-6) floats). Sources are passed by value (at most 64).
struct GatherSrc {
  const uint8_t* vol;  // first byte of the patch
  const float* map;    // first target value
  int64_t vol_rs;      // bytes per volume row
  int64_t map_rs;      // floats per map row
};
struct GatherArgs {
  GatherSrc src[64];
  int batch, P;
};

__global__ __launch_bounds__(256) void st_gather(GatherArgs a, uint8_t* __restrict__ patches,
                                                  float* __restrict__ targets) {
  const int b = blockIdx.y;
  const GatherSrc g = a.src[b];
  const int P = a.P, Pt = a.P - 6;
  const gbyte* vs = gin(g.vol);
  const gbyte* ms = gin(g.map);
  gbyte* po = gout(patches) + (int64_t)b * P * P;
  gbyte* to = gout(targets) + (int64_t)b * Pt * Pt * 4;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < P * P; i += gridDim.x * 256) {
    const int r = i / P, c = i % P;
    st<uint8_t>(po + i, ld<uint8_t>(vs + (int64_t)r * g.vol_rs + c));
  }
  for (int i = blockIdx.x * 256 + threadIdx.x; i < Pt * Pt; i += gridDim.x * 256) {
    const int r = i / Pt, c = i % Pt;
    st<float>(to + (int64_t)i * 4, ld<float>(ms + ((int64_t)r * g.map_rs + c) * 4));
  }
}

// ------------------------------------------------------------------ host object

struct Student {
  int prec = 1;
  int device = 0;
  float* master = nullptr;  // [801] device
  float* m = nullptr;
  float* v = nullptr;
  float* ww = nullptr;
  int64_t step = 0;
  // training workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // fallback workspace
  void* fb = nullptr;
  size_t fb_bytes = 0;
  // sample-window table: pinned host memory, uploaded asynchronously; rewritten
  // only after the event recorded behind the previous upload has completed
  int32_t* win_host = nullptr;
  size_t win_host_n = 0;
  hipEvent_t win_done = nullptr;
  bool win_pending = false;
};

static int student_ws(Student* s, size_t need) {
  if (need <= s->ws_bytes) return CNN_OK;
  hipDeviceSynchronize();
  if (s->ws) hipFree(s->ws);
  s->ws = nullptr;
  s->ws_bytes = 0;
  if (hipMalloc(&s->ws, need) != hipSuccess) return fail(CNN_ENOMEM, "student workspace");
  s->ws_bytes = need;
  return CNN_OK;
}

static int grad_impl(Student* s, const uint8_t* patches, const float* teacher, int B, int P, float* grad_out,
                     double* loss_out, double* gnorm_out, const cnn_adam* hp, hipStream_t st) {
  const int P1 = P - 4, P2 = P - 6;
  const int64_t n1 = (int64_t)B * P1 * P1, n2 = (int64_t)B * P2 * P2;
  const int chunk = 2048;
  const int nc0 = (int)((n1 + chunk - 1) / chunk), nc1 = (int)((n2 + chunk - 1) / chunk), nc2 = nc1;
  const int nloss = (int)((n2 + 255) / 256);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t sz_h1 = al(n1 * S_C * 4), sz_h2 = al(n2 * S_C * 4), sz_dz = al(n2 * 4);
  const size_t sz_p0 = al((size_t)nc0 * 208 * 4), sz_p1 = al((size_t)nc1 * 584 * 4), sz_p2 = al((size_t)nc2 * 9 * 4);
  const size_t sz_l = al((size_t)nloss * 8);
  const size_t need = sz_h1 * 2 + sz_h2 * 2 + sz_dz + sz_p0 + sz_p1 + sz_p2 + sz_l + 256;
  int rc = student_ws(s, need);
  if (rc) return rc;
  unsigned char* w = reinterpret_cast<unsigned char*>(s->ws);
  float* h1 = reinterpret_cast<float*>(w);
  w += sz_h1;
  float* dh1 = reinterpret_cast<float*>(w);
  w += sz_h1;
  float* h2 = reinterpret_cast<float*>(w);
  w += sz_h2;
  float* dh2 = reinterpret_cast<float*>(w);
  w += sz_h2;
  float* dz = reinterpret_cast<float*>(w);
  w += sz_dz;
  float* p0 = reinterpret_cast<float*>(w);
  w += sz_p0;
  float* p1 = reinterpret_cast<float*>(w);
  w += sz_p1;
  float* p2 = reinterpret_cast<float*>(w);
  w += sz_p2;
  double* lp = reinterpret_cast<double*>(w);
  const int bf = s->prec == CNN_PREC_BF16;
  const double invN = 1.0 / (double)n2;
  auto blocks = [](int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 65535); };
  hipLaunchKernelGGL(st_conv1, dim3(blocks(n1)), dim3(256), 0, st, patches, B, P, s->ww, h1, bf);
  hipLaunchKernelGGL(st_conv2_loss, dim3(nloss), dim3(256), 0, st, h1, B, P, s->ww, teacher, h2, dz, dh2, lp, invN, bf);
  hipLaunchKernelGGL(st_dh1, dim3(blocks(n1)), dim3(256), 0, st, dh2, h1, B, P, s->ww, dh1, bf);
  // one thread per gradient element of a chunk (8 x 25 + 8, 8 x 72 + 8, 8 + 1)
  hipLaunchKernelGGL(st_wgrad<0>, dim3(nc0), dim3(256), 0, st, dh1, (const void*)patches, B, P, chunk, p0);
  hipLaunchKernelGGL(st_wgrad<1>, dim3(nc1), dim3(640), 0, st, dh2, (const void*)h1, B, P, chunk, p1);
  hipLaunchKernelGGL(st_wgrad<2>, dim3(nc2), dim3(64), 0, st, dz, (const void*)h2, B, P, chunk, p2);
  ReduceArgs a;
  std::memset(&a, 0, sizeof(a));
  a.part[0] = p0;
  a.part[1] = p1;
  a.part[2] = p2;
  a.nchunk[0] = nc0;
  a.nchunk[1] = nc1;
  a.nchunk[2] = nc2;
  a.loss_part = lp;
  a.nloss = nloss;
  a.invN = invN;
  a.master = s->master;
  a.m = s->m;
  a.v = s->v;
  a.ww = s->ww;
  a.grad_out = grad_out;
  a.loss_out = loss_out;
  a.gnorm_out = gnorm_out;
  a.bf16 = bf;
  if (hp) {
    s->step += 1;
    a.do_update = 1;
    a.lr = hp->lr;
    a.b1 = hp->beta1;
    a.b2 = hp->beta2;
    a.eps = hp->eps;
    a.c1 = (float)(1.0 - std::pow((double)hp->beta1, (double)s->step));
    a.c2 = (float)(1.0 - std::pow((double)hp->beta2, (double)s->step));
  }
  hipLaunchKernelGGL(st_reduce_adam, dim3(1), dim3(1024), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "student kernels");
  return CNN_OK;
}

}  // namespace emcnn

using namespace emcnn;

extern "C" int student_create(const double* w_init, int64_t n, int32_t precision, cnn_student** out) {
  clear_error();
  if (!w_init || !out) return fail(CNN_EINVAL, "student_create: null argument");
  if (n != S_NP) return fail(CNN_EINVAL, "student_create: expected 801 parameters");
  if (precision != CNN_PREC_FP32 && precision != CNN_PREC_BF16)
    return fail(CNN_EUNSUPPORTED, "student_create: precision must be FP32 or BF16");
  *out = nullptr;
  Student* s = new Student();
  s->prec = precision;
  hipGetDevice(&s->device);
  std::vector<float> w(S_NP);
  for (int i = 0; i < S_NP; ++i) w[i] = (float)w_init[i];
  hipError_t e;
  if ((e = hipMalloc(&s->master, 4 * S_NP * sizeof(float))) != hipSuccess) {
    delete s;
    return fail(CNN_ENOMEM, "student_create: hipMalloc");
  }
  s->m = s->master + S_NP;
  s->v = s->m + S_NP;
  s->ww = s->v + S_NP;
  e = hipMemcpy(s->master, w.data(), S_NP * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(s->m, 0, 2 * S_NP * sizeof(float));
  if (e == hipSuccess) {
    hipLaunchKernelGGL(st_refresh, dim3(4), dim3(256), 0, 0, s->ww, s->master, s->prec == CNN_PREC_BF16 ? 1 : 0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    hipFree(s->master);
    delete s;
    return hip_fail(e, "student_create");
  }
  *out = reinterpret_cast<cnn_student*>(s);
  return CNN_OK;
}

extern "C" int student_destroy(cnn_student* h) {
  clear_error();
  if (!h) return CNN_OK;
  Student* s = reinterpret_cast<Student*>(h);
  hipDeviceSynchronize();
  if (s->master) hipFree(s->master);
  if (s->ws) hipFree(s->ws);
  if (s->fb) hipFree(s->fb);
  if (s->win_host) hipHostFree(s->win_host);
  if (s->win_done) hipEventDestroy(s->win_done);
  delete s;
  return CNN_OK;
}

extern "C" int student_get_state(cnn_student* h, double* w_out, double* m_out, double* v_out, int64_t* step_out) {
  clear_error();
  if (!h) return fail(CNN_EINVAL, "student_get_state: null student");
  Student* s = reinterpret_cast<Student*>(h);
  std::vector<float> buf(3 * S_NP);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "student_get_state");
  if ((e = hipMemcpy(buf.data(), s->master, 3 * S_NP * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess)
    return hip_fail(e, "student_get_state: copy");
  for (int i = 0; i < S_NP; ++i) {
    if (w_out) w_out[i] = buf[i];
    if (m_out) m_out[i] = buf[S_NP + i];
    if (v_out) v_out[i] = buf[2 * S_NP + i];
  }
  if (step_out) *step_out = s->step;
  return CNN_OK;
}

extern "C" int student_set_state(cnn_student* h, const double* w, const double* m, const double* v, int64_t step) {
  clear_error();
  if (!h || !w || !m || !v || step < 0) return fail(CNN_EINVAL, "student_set_state: bad argument");
  Student* s = reinterpret_cast<Student*>(h);
  std::vector<float> buf(3 * S_NP);
  for (int i = 0; i < S_NP; ++i) {
    buf[i] = (float)w[i];
    buf[S_NP + i] = (float)m[i];
    buf[2 * S_NP + i] = (float)v[i];
  }
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(s->master, buf.data(), 3 * S_NP * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(st_refresh, dim3(4), dim3(256), 0, 0, s->ww, s->master, s->prec == CNN_PREC_BF16 ? 1 : 0);
    e = hipGetLastError();
  }
  if (e == hipSuccess) s->step = step;
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "student_set_state");
  return CNN_OK;
}

static int check_batch(int32_t batch, int32_t patch) {
  if (batch < 1 || patch < 7 || patch > 4096 || (int64_t)batch * patch * patch > (1ll << 31))
    return fail(CNN_EINVAL, "student: batch >= 1 and 7 <= patch <= 4096 required");
  return CNN_OK;
}

extern "C" int student_grad(cnn_student* h, const uint8_t* patches, const float* teacher, int32_t batch, int32_t patch,
                            float* grad_out, double* loss_out, void* stream) {
  clear_error();
  if (!h || !patches || !teacher || !grad_out) return fail(CNN_EINVAL, "student_grad: null argument");
  int rc = check_batch(batch, patch);
  if (rc) return rc;
  return grad_impl(reinterpret_cast<Student*>(h), patches, teacher, batch, patch, grad_out, loss_out, nullptr, nullptr,
                   reinterpret_cast<hipStream_t>(stream));
}

extern "C" int student_train_step(cnn_student* h, const uint8_t* patches, const float* teacher, int32_t batch,
                                  int32_t patch, const cnn_adam* hp, double* loss_out, double* gnorm_out,
                                  void* stream) {
  clear_error();
  if (!h || !patches || !teacher || !hp) return fail(CNN_EINVAL, "student_train_step: null argument");
  if (!(hp->lr > 0) || !(hp->beta1 >= 0 && hp->beta1 < 1) || !(hp->beta2 >= 0 && hp->beta2 < 1) || !(hp->eps > 0))
    return fail(CNN_EINVAL, "student_train_step: bad Adam hyper-parameters");
  int rc = check_batch(batch, patch);
  if (rc) return rc;
  return grad_impl(reinterpret_cast<Student*>(h), patches, teacher, batch, patch, nullptr, loss_out, gnorm_out, hp,
                   reinterpret_cast<hipStream_t>(stream));
}

static int student_launch(Student* s, const uint8_t* vol, int64_t Z, int64_t H, int64_t W, float* out, int64_t out_rs,
                          int64_t out_zs, int Ho, int Wo, int crop, hipStream_t st) {
  hipError_t e;
  if (s->prec == CNN_PREC_BF16) {
    constexpr int TY = 16, TX = 64;
    dim3 grid((Wo + TX - 1) / TX, (Ho + TY - 1) / TY, (unsigned)Z);
    hipLaunchKernelGGL((student_mfma<TY, TX>), grid, dim3(256), 0, st, vol, W, H * W, out, out_rs, out_zs, Ho, Wo, crop,
                       s->ww);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "student_mfma");
    return CNN_OK;
  }
  constexpr int TY = 16, TX = 16;
  dim3 grid((Wo + TX - 1) / TX, (Ho + TY - 1) / TY, (unsigned)Z);
  hipLaunchKernelGGL((student_fused<TY, TX>), grid, dim3(TY * TX), 0, st, vol, W, H * W, out, out_rs, out_zs, Ho, Wo,
                     crop, s->ww, 0);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "student_fused");
  return CNN_OK;
}

extern "C" int student_infer(cnn_student* h, const uint8_t* vol, const int64_t dims[3], float* prob, void* stream) {
  clear_error();
  if (!h || !vol || !dims || !prob) return fail(CNN_EINVAL, "student_infer: null argument");
  const int64_t Z = dims[0], H = dims[1], W = dims[2];
  if (Z < 1 || Z > 65535 || H < 7 || W < 7 || H >= (1 << 30) || W >= (1 << 30))
    return fail(CNN_EINVAL, "student_infer: bad dims");
  Student* s = reinterpret_cast<Student*>(h);
  return student_launch(s, vol, Z, H, W, prob, W - 6, (H - 6) * (W - 6), (int)(H - 6), (int)(W - 6), 0,
                        reinterpret_cast<hipStream_t>(stream));
}

static uint64_t mix64(uint64_t x) {
  // splitmix64 finaliser
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

extern "C" int student_infer_with_fallback(cnn_student* h, cnn_net* th, const uint8_t* vol, const int64_t dims[3],
                                           float* prob, float tau, int32_t tile, int32_t n_samples, uint64_t seed,
                                           int32_t* stats, int32_t* flags_out, void* stream) {
  clear_error();
  if (!h || !th || !vol || !dims || !prob) return fail(CNN_EINVAL, "student_infer_with_fallback: null argument");
  Student* s = reinterpret_cast<Student*>(h);
  Net* net = reinterpret_cast<Net*>(th);
  const int64_t Z = dims[0], H = dims[1], W = dims[2];
  const int R = net->R;
  if (R < 6 || (R - 6) % 2 || net->out_stride != 1 || net->in_channels != 1)
    return fail(CNN_EUNSUPPORTED, "fallback: teacher radius must be even and >= 6, output at full resolution");
  if (Z < 1 || Z > 65535 || H < R + 1 || W < R + 1 || H >= (1 << 30) || W >= (1 << 30))
    return fail(CNN_EINVAL, "fallback: bad dims");
  if (tile < 16 || n_samples < 1 || n_samples > 64 || tau != tau)
    return fail(CNN_EINVAL, "fallback: tile >= 16, 1 <= n_samples <= 64, tau not NaN required");
  int rc = check_device(net);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int Ho = (int)(H - R), Wo = (int)(W - R);
  const int crop = (R - 6) / 2;
  const int ty = (Ho + tile - 1) / tile, tx = (Wo + tile - 1) / tile;
  const int64_t ntile = Z * ty * tx;
  if (ntile > (1 << 24)) return fail(CNN_EINVAL, "fallback: too many tiles");
  // workspace: teacher samples, window table, flags (grown before anything is enqueued)
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t nwin = (size_t)ntile * n_samples * 5;
  const size_t sz_samp = al((size_t)ntile * n_samples * 256 * 4), sz_win = al(nwin * 4), sz_flag = al((size_t)ntile * 4);
  const size_t need = sz_samp + sz_win + sz_flag;
  hipError_t e;
  if (need > s->fb_bytes) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "fallback: workspace grow");
    if (s->fb) hipFree(s->fb);
    s->fb = nullptr;
    s->fb_bytes = 0;
    if (hipMalloc(&s->fb, need) != hipSuccess) return fail(CNN_ENOMEM, "fallback workspace");
    s->fb_bytes = need;
  }
  // the pinned window table is rewritten only after the previous call's upload has run
  if (s->win_pending) {
    if ((e = hipEventSynchronize(s->win_done)) != hipSuccess) return hip_fail(e, "fallback: previous window upload");
    s->win_pending = false;
  }
  if (s->win_host_n < nwin) {
    if (s->win_host) hipHostFree(s->win_host);
    s->win_host = nullptr;
    s->win_host_n = 0;
    if (hipHostMalloc((void**)&s->win_host, nwin * 4) != hipSuccess) return fail(CNN_ENOMEM, "fallback: pinned window table");
    s->win_host_n = nwin;
  }
  if (!s->win_done && (e = hipEventCreateWithFlags(&s->win_done, hipEventDisableTiming)) != hipSuccess)
    return hip_fail(e, "fallback: hipEventCreate");
  float* samples = reinterpret_cast<float*>(s->fb);
  int32_t* win_dev = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(s->fb) + sz_samp);
  int32_t* flags = reinterpret_cast<int32_t*>(reinterpret_cast<unsigned char*>(s->fb) + sz_samp + sz_win);
  // 1) seeded sample windows per tile (positions do not depend on the data)
  std::vector<Region> sample_regs, rerun_regs;
  for (int64_t z = 0; z < Z; ++z)
    for (int a = 0; a < ty; ++a)
      for (int b = 0; b < tx; ++b) {
        const int64_t t = (z * ty + a) * tx + b;
        const int y0 = a * tile, x0 = b * tile;
        const int th_ = std::min(tile, Ho - y0), tw_ = std::min(tile, Wo - x0);
        const int wh = std::min(16, th_), wwid = std::min(16, tw_);
        for (int k = 0; k < n_samples; ++k) {
          const uint64_t r = mix64(seed ^ mix64((uint64_t)t * 64 + k));
          const int oy = (int)(r % (uint64_t)(th_ - wh + 1));
          const int ox = (int)((r >> 32) % (uint64_t)(tw_ - wwid + 1));
          int32_t* w = s->win_host + ((size_t)t * n_samples + k) * 5;
          w[0] = (int32_t)z;
          w[1] = y0 + oy;
          w[2] = x0 + ox;
          w[3] = wh;
          w[4] = wwid;
          Region g;
          g.in = vol + z * H * W + (int64_t)(y0 + oy) * W + (x0 + ox);
          g.in_rs = W;
          g.in_zs = H * W;
          g.z = 1;
          g.h = wh + R;
          g.w = wwid + R;
          g.out = samples + ((size_t)t * n_samples + k) * 256;
          g.out_rs = 16;
          g.out_zs = 256;
          g.gate = nullptr;
          sample_regs.push_back(g);
        }
        Region q;
        q.in = vol + z * H * W + (int64_t)y0 * W + x0;
        q.in_rs = W;
        q.in_zs = H * W;
        q.z = 1;
        q.h = th_ + R;
        q.w = tw_ + R;
        q.out = prob + z * (int64_t)Ho * Wo + (int64_t)y0 * Wo + x0;
        q.out_rs = Wo;
        q.out_zs = (int64_t)Ho * Wo;
        q.gate = flags + t;
        rerun_regs.push_back(q);
      }
  const size_t nj1 = count_region_jobs(net, sample_regs), nj2 = count_region_jobs(net, rerun_regs);
  rc = arena_reserve(net, nj1 + nj2);
  if (rc) return rc;
  std::vector<Launch> l1, l2;
  size_t used1 = 0, used2 = 0, ws1 = 0, ws2 = 0;
  // both passes are planned before either is submitted: size the shared
  // workspace for the larger one first, so that planning the second cannot
  // reallocate the workspace the first one's jobs point into
  rc = plan_regions(net, sample_regs, 0, l1, used1, ws1, true);
  if (rc) return rc;
  rc = plan_regions(net, rerun_regs, 0, l2, used2, ws2, true);
  if (rc) return rc;
  rc = ensure_ws(net, std::max(ws1, ws2));
  if (rc) return rc;
  const void* ws_before = net->ws;
  rc = plan_regions(net, sample_regs, 0, l1, used1, ws1);
  if (rc) return rc;
  rc = plan_regions(net, rerun_regs, used1, l2, used2, ws2);
  if (rc) return rc;
  if (net->ws != ws_before) return fail(CNN_EHIP, "fallback: internal: workspace moved during planning");
  // 2) student everywhere, in the teacher's output frame
  rc = student_launch(s, vol, Z, H, W, prob, Wo, (int64_t)Ho * Wo, Ho, Wo, crop, st);
  if (rc) return rc;
  if ((e = hipMemcpyAsync(win_dev, s->win_host, nwin * 4, hipMemcpyHostToDevice, st)) != hipSuccess)
    return hip_fail(e, "fallback: window upload");
  if ((e = hipEventRecord(s->win_done, st)) != hipSuccess) return hip_fail(e, "fallback: hipEventRecord");
  s->win_pending = true;
  // 3) teacher on the sample windows, then the per-tile decisions on the device
  rc = submit(net, l1, 0, used1 + used2, st, false);
  if (rc) return rc;
  hipLaunchKernelGGL(st_flag_tiles, dim3((unsigned)ntile), dim3(256), 0, st, prob, (int64_t)Wo, (int64_t)Ho * Wo,
                     samples, win_dev, n_samples, tau, flags);
  if (stats) hipLaunchKernelGGL(st_count_flags, dim3(1), dim3(256), 0, st, flags, (int)ntile, stats);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "fallback: flag kernels");
  if (flags_out && (e = hipMemcpyAsync(flags_out, flags, (size_t)ntile * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return hip_fail(e, "fallback: flag copy");
  // 4) teacher re-run of flagged tiles (unflagged tiles are skipped by the gate);
  // the job table of both passes went up with the first submission
  for (const Launch& la : l2) {
    rc = launch_layer(net, net->layers[la.layer], la.js, la.grid, st);
    if (rc) return rc;
  }
  if ((e = hipEventRecord(net->arena[net->cur].done, st)) != hipSuccess) return hip_fail(e, "fallback: hipEventRecord");
  return CNN_OK;
}

extern "C" int student_gather(const cnn_patch_src* src, int32_t batch, int32_t patch, int32_t teacher_R,
                              uint8_t* patches_out, float* teacher_out, void* stream) {
  clear_error();
  if (!src || !patches_out || !teacher_out) return fail(CNN_EINVAL, "student_gather: null argument");
  if (batch < 1 || batch > 64 || patch < 7 || patch > 4096)
    return fail(CNN_EINVAL, "student_gather: 1 <= batch <= 64 and 7 <= patch <= 4096 required");
  if (teacher_R < 6 || (teacher_R - 6) % 2) return fail(CNN_EINVAL, "student_gather: teacher radius even and >= 6");
  const int m = (teacher_R - 6) / 2;  // centring offset between the two output frames
  GatherArgs a;
  std::memset(&a, 0, sizeof(a));
  a.batch = batch;
  a.P = patch;
  for (int b = 0; b < batch; ++b) {
    const cnn_patch_src& q = src[b];
    if (!q.volume || !q.teacher) return fail(CNN_EINVAL, "student_gather: source " + std::to_string(b) + " is null");
    if (q.H < teacher_R + 1 || q.W < teacher_R + 1 || q.Z < 1 || q.z < 0 || q.z >= q.Z || q.y < m || q.x < m ||
        (int64_t)q.y + patch + m > q.H || (int64_t)q.x + patch + m > q.W)
      return fail(CNN_EINVAL, "student_gather: source " + std::to_string(b) +
                                  " is outside its volume (origin must lie in [m, side - patch - m], m = (R-6)/2)");
    const int64_t Hm = q.H - teacher_R, Wm = q.W - teacher_R;
    a.src[b].vol = q.volume + ((int64_t)q.z * q.H + q.y) * q.W + q.x;
    a.src[b].map = q.teacher + ((int64_t)q.z * Hm + (q.y - m)) * Wm + (q.x - m);
    a.src[b].vol_rs = q.W;
    a.src[b].map_rs = Wm;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int gx = std::max(1, std::min(64, (patch * patch + 4095) / 4096));
  hipLaunchKernelGGL(st_gather, dim3(gx, batch), dim3(256), 0, st, a, patches_out, teacher_out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "student_gather");
  return CNN_OK;
}
