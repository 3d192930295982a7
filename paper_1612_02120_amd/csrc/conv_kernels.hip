// Dense convolution kernels for gfx950 (CDNA4).
//
// The network (arXiv 1612.02120, Section 2.2) alternates valid convolutions
// with 2x2 max pooling; the dense per-pixel output is obtained by evaluating
// every pooling as a stride-1 max filter, so every layer is a stride-1 valid
// convolution over the whole slice and no pixel is computed twice.
//
// Kernels here:
//   conv_first  - the 1-channel first layer on MFMA, reading the caller's
//                 uint8 volume (1/255 is folded into its weights on the host).
//   conv_mfma   - every later FP32 conv as an implicit GEMM on MFMA: M = output
//                 pixels (16 consecutive pixels of a row per m-block), N = output
//                 channels (16 per n-block), K = (tap, input channel).
//                 The input tile plus halo is staged in LDS, the preceding 2x2
//                 stride-1 max filter is applied while staging, and bias, ReLU and
//                 the output cast (or the 1x1 head and sigmoid) are fused into the
//                 epilogue. conv_mfma_rr is the same layer with a row-reuse K order.
//   conv_ws     - the BF16 / FP8 convs: the same implicit GEMM, warp-specialised
//                 (producer waves stage the next tile while consumer waves run
//                 MFMA) over channel-blocked activations; in its spaced mode the
//                 BF16 body convs of nets with stride-2 pools.
//   conv_phase  - the convs of nets with stride-2 pools (FastMemb): taps spaced
//   head_*        d apart, tiled per phase sub-lattice (the paper's fragments,
//                 which the maps between layers store as separate blocks);
//                 max-out or two-class softmax epilogues. The two-class layer
//                 also as a GEMM over its taps (head_taps, and over groups of
//                 four phases head_taps4 / head_strip) and on the VALU
//                 (head_phase).
//
// All are persistent: a grid of a multiple of 8 workgroups walks the work
// items (z, tile_y, tile_x) of one or many jobs. Workgroups are dispatched to
// the 8 XCDs round-robin, so workgroup b works on the b%8-th eighth of the item
// range: neighbouring tiles, which share halo rows, meet in the same L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "device_util.h"

namespace emcnn {


template <int P>
struct PT;
template <>
struct PT<F32> {
  static constexpr int CHB = 4, U = 1, BYTES = 4, CB = 16;
};
template <>
struct PT<BF16> {
  static constexpr int CHB = 8, U = 1, BYTES = 2, CB = 24;
};
template <>
struct PT<FP8> {
  static constexpr int CHB = 16, U = 2, BYTES = 1, CB = 48;
};

// Pixel stride of an LDS operand tile, in dwords: the smallest w' >= w with
// w' = 8 (mod 16). gfx950 serves a 16-byte LDS read per half-wave (32 lanes,
// 512 B) from 128 dword banks (measured with SQ_LDS_BANK_CONFLICT). An A
// fragment read has 16 consecutive pixels x 2 chunk groups (+16 B) per half
// wave; with the stride = 8 (mod 16) the 16 pixel starts are exactly the
// multiples of 8 dwords mod 128, the second chunk group fills the gaps, and the
// 128 dwords hit 128 distinct banks.
__host__ __device__ constexpr int pad_words(int w) {
  return (w % 16 == 8) ? w : w + ((24 - (w % 16)) % 16);
}

// CBO: channels staged per LDS pass (0: the precision's default block).
// NMEM > 1: the operand tiles of NMEM phases stacked row-wise (conv_phase over
// phase groups), NMEM times the m-blocks.
template <int P, int CIN, int COUT, int KS, int TY, int TX, int MW, bool HEAD = false, int CBO = 0, int NMEM = 1>
struct Cfg {
  using T = PT<P>;
  static constexpr int CB = CBO ? CBO : (T::CB < CIN) ? T::CB : CIN;
  static_assert(CIN % CB == 0, "channel block must divide CIN");
  static constexpr int NCB = CIN / CB;
  static constexpr int NCHB = CB / T::CHB;  // 16-byte chunks per pixel per block
  static_assert(NCHB * T::CHB == CB, "block must be whole chunks");
  static constexpr int NCHK = KS * KS * NCHB;  // chunks of K per block
  static constexpr int SLOTS = 4 * T::U;       // chunks consumed per group-step
  static constexpr int NGS = (NCHK + SLOTS - 1) / SLOTS;
  static constexpr int NB = COUT / 16;
  static_assert(NB * 16 == COUT, "COUT must be a multiple of 16");
  static constexpr int LR = TY + KS - 1, LC = TX + KS - 1;
  static constexpr int PSB = pad_words(CB * T::BYTES / 4) * 4;
  static constexpr int LDS_IN = NMEM * LR * LC * PSB;
  static constexpr int LDS_TILE = LDS_IN;
  static constexpr int MBLK = NMEM * TY * TX / 16;
  static_assert(TX % 16 == 0, "TX must be a multiple of 16");
  static_assert(MBLK % MW == 0, "m-blocks must split evenly over waves");
  static constexpr int WAVES = MBLK / MW;
  static constexpr int THREADS = WAVES * 64;
};

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ float relu(float v) { return v > 0.0f ? v : 0.0f; }  // +0 for v <= 0

__device__ __forceinline__ float sigmoid_f(float t) {
  if (t >= 0.0f) return 1.0f / (1.0f + expf(-t));
  float e = expf(t);
  return e / (1.0f + e);
}

__device__ __forceinline__ unsigned char to_e4m3(float v) {
  // v >= 0 here (post-ReLU); saturate at the largest finite e4m3fn value.
  v = fminf(v, 448.0f);
  int packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0, false);
  return (unsigned char)(packed & 0xff);
}

// Two floats to bf16 (round to nearest even), lo in the low half: one packed
// conversion (converted one at a time, the compiler adds a shift and an or)
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){lo, hi}, bf16x2v));
}

__device__ __forceinline__ uint32_t pack_e4m3x2(float lo, float hi) {
  // non-negative inputs; saturate at the largest finite e4m3fn value
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(fminf(lo, 448.0f), fminf(hi, 448.0f), 0, false) & 0xffffu;
}

// Signed bf16 activations (nets without ReLU) are stored as order-preserving
// keys: key = b ^ (b < 0 ? 0xffff : 0x8000) per 16-bit half, so that unsigned
// order is float order and a max filter is one packed unsigned max per dword
// (chunk_max<BF16>). bf16_key / bf16_unkey convert two halves at a time.
typedef short s16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_key(uint32_t x) {
  const uint32_t neg = __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, x) >> (short)15);  // 0xffff if < 0
  return x ^ (neg | 0x80008000u);
}
__device__ __forceinline__ uint32_t bf16_unkey(uint32_t k) {
  const uint32_t pos = __builtin_bit_cast(uint32_t, __builtin_bit_cast(s16x2, k) >> (short)15);  // 0xffff if b >= 0
  return k ^ (~pos | 0x80008000u);
}

// Pixel index, inside a slice, of map pixel (y, x) when the map is stored
// fragment-major modulo D = 2^lg (lg = 0: row-major, row stride rs): fragment
// (y mod D, x mod D) is a row-major block of zs / D^2 pixels holding rows y / D
// and columns x / D.
__device__ __forceinline__ int64_t frag_pix(int y, int x, int lg, int64_t rs, int64_t zs) {
  const int m = (1 << lg) - 1;
  return (int64_t)(((y & m) << lg) + (x & m)) * (zs >> (2 * lg)) + (int64_t)(y >> lg) * rs + (x >> lg);
}

// Operand addressing of one phase tile of a spaced conv (taps d apart, 2x2 max
// filter pd = d / 2 apart before it) whose input map is stored fragment-major
// modulo d. Operand pixel (r, c) of phase (py, px) is the filter at input
// (py + d (y0 + r), px + d (x0 + c)): row y0 + r, column x0 + c of fragment
// (py, px). Its partners at +pd lie at the same row and column of fragments
// (py + pd) mod d and (px + pd) mod d, one row / column further where that
// wraps, so each is a fixed offset from the first element for the whole tile.
// Rows and columns are clamped to the last valid filter origin; clamped ones
// only feed outputs that are not stored.
struct FragTile {
  const gbyte* base;  // fragment (py, px), row 0, column 0
  int64_t rowb;       // bytes per fragment row
  int64_t o01, o10, o11;  // byte offsets of the partners at (0, +pd), (+pd, 0), (+pd, +pd)
  int rmax, cmax;     // last valid filter row / column (fragment coordinates)
  __device__ __forceinline__ const gbyte* at(int r, int c, int elb) const {
    return base + (int64_t)min(r, rmax) * rowb + (int64_t)min(c, cmax) * elb;
  }
};

__device__ __forceinline__ FragTile frag_tile(const gbyte* slice, int elb, const LayerJob& J, int py, int px) {
  // pd = 0: no max filter before this conv (its partners are the pixel itself)
  const int d = max(J.geom & 0xff, 1), pd = (J.geom >> 8) & 0xff;
  const int lg = __builtin_ctz(d);
  const int64_t plane = (J.in_zs >> (2 * lg)) * elb;  // bytes per fragment
  FragTile f;
  f.rowb = J.in_rs * elb;
  f.base = slice + (int64_t)(py * d + px) * plane;
  const int fy = (py + pd) & (d - 1), cy = (py + pd) >> lg;
  const int fx = (px + pd) & (d - 1), cx = (px + pd) >> lg;
  f.o01 = (int64_t)(fx - px) * plane + (int64_t)cx * elb;
  f.o10 = (int64_t)(fy - py) * d * plane + (int64_t)cy * f.rowb;
  f.o11 = f.o01 + f.o10;
  f.rmax = (J.hin - 1 - pd - py) >> lg;  // y + pd <= hin - 1
  f.cmax = (J.win - 1 - pd - px) >> lg;
  return f;
}

// Store element idx of an activation array (LDS or global) in the layer's format.
template <int P, class B>
__device__ __forceinline__ void store_act(B* base, int64_t idx, float v, float inv) {
  if constexpr (P == F32) st<float>(base + idx * 4, v);
  else if constexpr (P == BF16) st<__bf16>(base + idx * 2, (__bf16)v);
  else st<unsigned char>(base + idx, to_e4m3(v * inv));
}

// Elementwise max of two 16-byte chunks of non-negative activations. For
// non-negative bf16 and e4m3fn values the bit patterns are ordered like the
// values, so an unsigned integer max is the float max.
template <int P>
__device__ __forceinline__ i4v chunk_max(i4v a, i4v b);
template <>
__device__ __forceinline__ i4v chunk_max<F32>(i4v a, i4v b) {
  f4 x = __builtin_bit_cast(f4, a), y = __builtin_bit_cast(f4, b);
  f4 r;
  r[0] = fmaxf(x[0], y[0]);
  r[1] = fmaxf(x[1], y[1]);
  r[2] = fmaxf(x[2], y[2]);
  r[3] = fmaxf(x[3], y[3]);
  return __builtin_bit_cast(i4v, r);
}
template <>
__device__ __forceinline__ i4v chunk_max<BF16>(i4v a, i4v b) {
  u16x8 x = __builtin_bit_cast(u16x8, a), y = __builtin_bit_cast(u16x8, b);
  return __builtin_bit_cast(i4v, __builtin_elementwise_max(x, y));
}
// e4m3fn codes of non-negative values are 0x00..0x7e (bit 7 clear), so a
// per-byte a - b + 128 never borrows across bytes and its bit 7 is (a >= b).
__device__ __forceinline__ uint32_t max_u7x4(uint32_t a, uint32_t b) {
  const uint32_t hm = ((a | 0x80808080u) - b) & 0x80808080u;  // 0x80 per byte where a >= b
  const uint32_t m = hm | (hm - (hm >> 7));                   // 0xff per byte where a >= b
  return (a & m) | (b & ~m);
}
// The 2x2 max filter of a 3x3 neighbourhood of FP8 chunks (q row-major) into
// its four outputs (o[2d + e] = max over rows d, d+1 and columns e, e+1), per
// byte. A packed u16 max orders each half by its high byte first, so on the
// raw words it gives the odd bytes' max; the even bytes take a packed u16 max
// of the words masked to them. 9 masks, 20 packed maxes and 4 bit-field
// inserts per dword, against 10 SWAR maxes of 7 operations each.
typedef unsigned short u16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pkmax_u16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t,
                            __builtin_elementwise_max(__builtin_bit_cast(u16x2v, a), __builtin_bit_cast(u16x2v, b)));
}
__device__ __forceinline__ void max_filter_fp8(const i4v (&q)[9], i4v (&o)[4]) {
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t hi[9], lo[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      hi[j] = (uint32_t)q[j][w];
      lo[j] = hi[j] & 0x00ff00ffu;
    }
    uint32_t hh[3][2], hl[3][2];  // horizontal maxes of each row
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        hh[r][e] = pkmax_u16(hi[3 * r + e], hi[3 * r + e + 1]);
        hl[r][e] = pkmax_u16(lo[3 * r + e], lo[3 * r + e + 1]);
      }
#pragma unroll
    for (int d = 0; d < 2; ++d)
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const uint32_t mh = pkmax_u16(hh[d][e], hh[d + 1][e]), ml = pkmax_u16(hl[d][e], hl[d + 1][e]);
        o[2 * d + e][w] = (int)((mh & 0xff00ff00u) | ml);
      }
  }
}

template <>
__device__ __forceinline__ i4v chunk_max<FP8>(i4v a, i4v b) {
  i4v r;
  r[0] = (int)max_u7x4((uint32_t)a[0], (uint32_t)b[0]);
  r[1] = (int)max_u7x4((uint32_t)a[1], (uint32_t)b[1]);
  r[2] = (int)max_u7x4((uint32_t)a[2], (uint32_t)b[2]);
  r[3] = (int)max_u7x4((uint32_t)a[3], (uint32_t)b[3]);
  return r;
}

template <int P>
struct Frag;
template <>
struct Frag<F32> {
  f4 v;
};
template <>
struct Frag<BF16> {
  bf16x8 v;
};
template <>
struct Frag<FP8> {
  i8v v;
};

template <int P>
__device__ __forceinline__ void mma(f4& acc, const Frag<P>& a, const Frag<P>& b);
template <>
__device__ __forceinline__ void mma<F32>(f4& acc, const Frag<F32>& a, const Frag<F32>& b) {
  // one 16-byte chunk = 4 channels = 4 MFMA k-steps of 4 (one channel per lane group)
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[0], b.v[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[1], b.v[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[2], b.v[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[3], b.v[3], acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<BF16>(f4& acc, const Frag<BF16>& a, const Frag<BF16>& b) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v, b.v, acc, 0, 0, 0);
}
template <>
__device__ __forceinline__ void mma<FP8>(f4& acc, const Frag<FP8>& a, const Frag<FP8>& b) {
  // format 0 = e4m3 for both operands; unit block scales (E8M0 127 = 2^0)
  acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a.v, b.v, acc, 0, 0, 0, 127, 0, 127);
}

// Load an MFMA operand fragment (16 bytes per lane, FP8: two 16-byte chunks)
// from LDS or global memory.
template <int P, class B>
__device__ __forceinline__ void load_frag(Frag<P>& f, const B* p0, const B* p1) {
  if constexpr (P == F32) {
    f.v = ld<f4>(p0);
  } else if constexpr (P == BF16) {
    f.v = ld<bf16x8>(p0);
  } else {
    const i4v lo = ld<i4v>(p0), hi = ld<i4v>(p1);
    f.v = i8v{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  }
}

// Lane exchange inside groups of 4 lanes (DPP quad permutation).
template <int CTRL>
__device__ __forceinline__ int quad_perm(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
constexpr int kQuadXor1 = 0xB1;  // lanes [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // lanes [2, 3, 0, 1]
constexpr int kRowMirror = 0x140;      // lane i <- lane 15 - i of its 16-lane row
constexpr int kRowHalfMirror = 0x141;  // lane i <- lane 7 - i of its 8-lane half row

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, quad_perm<CTRL>(__builtin_bit_cast(int, v)));
}

// Sums of four per-lane values v[0..3] over the 16 lanes of each row, with
// DPP exchanges only (no LDS): two pairing steps that each keep half of the
// values (across the row mirror, then the half-row mirror), then a quad
// reduction. On return every lane n16 of a row holds the row sum of
// v[n16 >> 2].
__device__ __forceinline__ float row_sum4_transposed(const float v[4], int n16) {
  const bool lo = n16 < 8, q0 = ((n16 >> 2) & 1) == 0;
  const float a = (lo ? v[0] : v[2]) + dpp_f<kRowMirror>(lo ? v[2] : v[0]);
  const float b = (lo ? v[1] : v[3]) + dpp_f<kRowMirror>(lo ? v[3] : v[1]);
  float r = (q0 ? a : b) + dpp_f<kRowHalfMirror>(q0 ? b : a);
  r += dpp_f<kQuadXor1>(r);
  r += dpp_f<kQuadXor2>(r);
  return r;
}


// 1x1 head + sigmoid straight from MFMA accumulators, for NU m-blocks of 16
// pixels. val(u, nb, k) is lane (g, n16)'s accumulator for pixel 4g + k of
// m-block u and channel nb * 16 + n16; pos(u, y, x) gives m-block u's output
// row and first column. The channel sums go through row_sum4_transposed, after
// which the four lanes of a quad hold four different m-blocks, so one sigmoid
// and one store per lane serve four m-blocks.
template <int NU, int NB, class Val, class Pos>
__device__ __forceinline__ void head_epilogue(Val val, Pos pos, const float (&bias)[NB], const float (&osc)[NB],
                                              const float (&hw)[NB], float head_b, int g, int n16, gbyte* out,
                                              int64_t zoff, int64_t rs, int hout, int wout) {
  const int jq = n16 & 3;
#pragma unroll
  for (int grp = 0; grp < (NU + 3) / 4; ++grp) {
    float mine = 0.f;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int u = grp * 4 + jj;
      if (u < NU) {
        float part[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          float pv = 0.f;
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) pv = fmaf(relu(fmaf(val(u, nb, k), osc[nb], bias[nb])), hw[nb], pv);
          part[k] = pv;
        }
        const float r = row_sum4_transposed(part, n16);
        mine = jq == jj ? r : mine;
      }
    }
    const int u = grp * 4 + jq;
    int y, xb;
    pos(u, y, xb);
    const int x = xb + 4 * g + (n16 >> 2);
    if (u < NU && y < hout && x < wout) st<float>(out + (zoff + (int64_t)y * rs + x) * 4, sigmoid_f(mine + head_b));
  }
}

// Persistent work distribution: workgroup b serves XCD b % 8 (hardware
// round-robin) and walks the matching eighth of the item range.
struct ItemRange {
  int64_t begin, end, step;
};

__device__ __forceinline__ ItemRange item_range(int64_t total) {
  const int64_t G = gridDim.x;
  const int64_t b = blockIdx.x;
  if ((G & 7) != 0) return {b, total, G};
  const int64_t per = (total + 7) >> 3;
  const int64_t begin = (b & 7) * per;
  int64_t end = begin + per;
  if (end > total) end = total;
  return {begin + (b >> 3), end, G >> 3};
}

__device__ __forceinline__ const EMCNN_GLOBAL LayerJob* gtab(const LayerJob* t) {
  return (const EMCNN_GLOBAL LayerJob*)t;
}

__device__ __forceinline__ int find_job(const LayerJob* table, int n, int64_t item) {
  const EMCNN_GLOBAL LayerJob* t = gtab(table);
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (t[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Job of a work item: advance the cursor through the table (items ascend).
__device__ __forceinline__ LayerJob job_at(const JobSet& js, int& cur, int64_t item) {
  if (!js.table) return js.single;
  const EMCNN_GLOBAL LayerJob* t = gtab(js.table);
  while (cur + 1 < js.njobs && t[cur + 1].item0 <= item) ++cur;
  static_assert(sizeof(LayerJob) % 16 == 0, "job copied in 16-byte chunks");
  LayerJob J;
  const gbyte* src = reinterpret_cast<const gbyte*>(t + cur);
#pragma unroll
  for (int k = 0; k < (int)sizeof(LayerJob) / 16; ++k) reinterpret_cast<i4v*>(&J)[k] = ld<i4v>(src + 16 * k);
  return J;
}

__device__ __forceinline__ bool gated_off(const LayerJob& J) {
  return J.gate && *(const EMCNN_GLOBAL int32_t*)J.gate == 0;
}

// Stage a LR x LC operand tile (NCHB 16-byte chunks per pixel, pixel stride
// PSB bytes in LDS) whose pixel (r, c) is the stored input at (y0 + r, x0 + c)
// (coordinates clamped to the logical hp x wp input; clamped values only feed
// outputs that are never stored). With POOL the operand pixel is the 2x2
// stride-1 max of the stored (pre-filter) input; each thread then covers a 2x2
// block of operand pixels of one chunk and loads the 3x3 stored neighbourhood
// once (9 loads for 4 pixels instead of 16). The loop stays rolled (registers
// and occupancy of the FP32 kernels).
template <int P, int LR, int LC, int NCHB, int PSB, int THREADS, bool POOL>
__device__ __forceinline__ void stage_tile(unsigned char* lds, const gbyte* in, int64_t rowb, int elb,
                                           int y0, int x0, int hp, int wp, int tid) {
  if constexpr (!POOL) {
    constexpr int NST = LR * LC * NCHB;
    constexpr int NIT = (NST + THREADS - 1) / THREADS;
#pragma unroll 1
    for (int k = 0; k < NIT; ++k) {
      const int t = tid + k * THREADS;
      if (t >= NST) break;
      const int cg = t % NCHB, pix = t / NCHB;
      const int r = pix / LC, c = pix % LC;
      const int y = min(y0 + r, hp - 1), x = min(x0 + c, wp - 1);
      st<i4v>(lds + pix * PSB + cg * 16, ld<i4v>(in + (int64_t)y * rowb + (int64_t)x * elb + cg * 16));
    }
  } else {
    static_assert(LR % 2 == 0 && LC % 2 == 0, "2x2 staging blocks need even tile sides");
    constexpr int BR = LR / 2, BC = LC / 2;
    constexpr int NST = BR * BC * NCHB;
    constexpr int NIT = (NST + THREADS - 1) / THREADS;
#pragma unroll 1
    for (int k = 0; k < NIT; ++k) {
      const int t = tid + k * THREADS;
      if (t >= NST) break;
      const int cg = t % NCHB, blk = t / NCHB;
      const int r = 2 * (blk / BC), c = 2 * (blk % BC);
      // Operand pixel (r + d, c + e) is the max of stored rows Y_d, Y_d + 1 and
      // columns X_e, X_e + 1 with Y_d = min(y0 + r + d, hp - 1) (likewise X_e).
      // Load stored rows Y_0, Y_0 + 1, Y_1 + 1 (and the same for columns): pixel
      // row 0 uses the first two; pixel row 1 uses the last two, which are Y_1
      // and Y_1 + 1 whenever row r + 1 is a valid operand row (a clamped row only
      // feeds outputs that are never stored). All indices stay <= hp (< hin).
      int ys[3], xs[3];
      ys[0] = min(y0 + r, hp - 1);
      ys[1] = ys[0] + 1;
      ys[2] = min(y0 + r + 1, hp - 1) + 1;
      xs[0] = min(x0 + c, wp - 1);
      xs[1] = xs[0] + 1;
      xs[2] = min(x0 + c + 1, wp - 1) + 1;
      i4v q[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          q[a][b] = ld<i4v>(in + (int64_t)ys[a] * rowb + (int64_t)xs[b] * elb + cg * 16);
#pragma unroll
      for (int d = 0; d < 2; ++d)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          i4v v = chunk_max<P>(chunk_max<P>(q[d][e], q[d][e + 1]), chunk_max<P>(q[d + 1][e], q[d + 1][e + 1]));
          *reinterpret_cast<i4v*>(lds + ((r + d) * LC + c + e) * PSB + cg * 16) = v;
        }
    }
  }
}

// ---------------------------------------------------------------- first layer

// conv1 (one input channel, KS x KS, KS*KS <= 32 taps) on MFMA. M = 16
// consecutive output pixels of a tile row per m-block, N = 16 output channels,
// K = taps. BF16 / FP8 nets: one 16x16x32 bf16 MFMA per (m-block, n-block),
// lane group g holding taps 8g..8g+7 (taps >= KS*KS are zero); the uint8 input
// is exact in bf16. FP32 nets: 16x16x4 f32 MFMAs, lane group g holding tap
// 4s+g of step s. Weights are pre-packed per lane (wpack, see the host).
// The uint8 input tile is read in 16-byte row chunks where the rows are
// 16-byte aligned, and converted once, as it is staged, to the MFMA operand
// type (float or bf16) in LDS.
// The epilogue applies bias and ReLU and casts to the stored activation
// format. BF16 / FP8 output is channel-blocked: a lane's four channels of one
// plane are 8 / 4 contiguous bytes, and the 64 lanes of an n-block together
// write the plane's 16 pixels, one contiguous run, straight from registers.
// FP32 output (NHWC) and max-out output pass the m-block through a per-wave
// LDS scratch so that each lane stores 16 contiguous bytes.
template <int PO, int COUT, int KS, int TY, int TX, int ST = 1>
struct FirstCfg {
  // ST: output stride (2: the conv is evaluated only at every second input
  // row and column, as a 2x subsample right after it keeps them)
  static constexpr int LR = ST * (TY - 1) + KS, LC = ST * (TX - 1) + KS;
  static constexpr int ESZ = PO == F32 ? 4 : PO == BF16 ? 2 : 1;
  static constexpr bool BLOCKED = PO != F32;  // BF16 / FP8 activations are channel-blocked
  static constexpr int NB = COUT / 16;
  static constexpr int MBLK = TY * TX / 16;
  static constexpr int WAVES = 4;
  static constexpr int MW = MBLK / WAVES;
  static constexpr int THREADS = 64 * WAVES;
  static constexpr int NSTEP = PO == F32 ? (KS * KS + 3) / 4 : 1;
  // the input tile in LDS: float (FP32 nets) or bf16 elements, rows LCP apart
  static constexpr int AEL = PO == F32 ? 4 : 2;
  static constexpr int NCK = (LC + 15) / 16;  // 16-byte uint8 chunks per tile row
  static constexpr int LCP = NCK * 16;
  static constexpr int LDS = LR * LCP * AEL;
  static_assert(KS * KS <= 32, "first layer supports up to 32 taps");
  static_assert(MBLK % WAVES == 0 && TX % 16 == 0, "tile must split into m-blocks per wave");
  static_assert(MW % (TX / 16) == 0, "each wave owns whole tile rows");
};

// MAXOUT: bias then max over the channel pairs (2c, 2c + 1), COUT / 2 stored
// channels (NHWC, FP32 or BF16), instead of bias then ReLU.
// XS (BF16 / FP8 output): the m-block's channel-blocked output passes through a
// per-wave LDS scratch so that each lane stores 16 contiguous bytes (one wide
// store per lane and plane instead of 4- / 8-byte stores from every lane).
template <int PO, int COUT, int KS, int TY, int TX, bool MAXOUT = false, int ST = 1, int XS = 0>
__global__ __launch_bounds__((FirstCfg<PO, COUT, KS, TY, TX, ST>::THREADS)) void conv_first(JobSet js,
                                                                                           FirstParams prm) {
  using C = FirstCfg<PO, COUT, KS, TY, TX, ST>;
  static_assert(!MAXOUT || PO == F32 || PO == BF16, "max-out first layers are FP32 or BF16");
  using AT = typename std::conditional<PO == F32, float, unsigned short>::type;  // float or bf16 bits
  __shared__ __attribute__((aligned(16))) AT tile[C::LR * C::LCP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  constexpr int MCOLS = TX / 16;
  // per-lane weight fragments and bias
  Frag<PO == F32 ? F32 : BF16> wf[C::NSTEP][C::NB];
  {
    const gbyte* wp = gin(prm.w);
#pragma unroll
    for (int s = 0; s < C::NSTEP; ++s)
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb) {
        if constexpr (PO == F32) {
          wf[s][nb].v = f4{ld<float>(wp + ((s * C::NB + nb) * 64 + lane) * 4), 0.f, 0.f, 0.f};
        } else {
          wf[s][nb].v = ld<bf16x8>(wp + ((size_t)(s * C::NB + nb) * 64 + lane) * 16);
        }
      }
  }
  // D = W X: lane (g, n16) accumulates channels nb * 16 + 4g .. 4g + 3 of
  // pixel n16 of an m-block: 4 consecutive stored channels, which the
  // epilogue gathers through the wave's LDS scratch into 16-byte stores
  float bias[C::NB][4];
#pragma unroll
  for (int nb = 0; nb < C::NB; ++nb)
#pragma unroll
    for (int k = 0; k < 4; ++k) bias[nb][k] = ldf(prm.bias, nb * 16 + 4 * g + k);
  // the lane's tap offsets in the uint8 tile (tap 4s + g of step s for FP32,
  // taps 8g .. 8g + 7 otherwise); taps past KS * KS read the pixel itself:
  // their packed weights are zero, so every tap read is unconditional
  constexpr int NT = PO == F32 ? C::NSTEP : 8;
  int toff[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int k = PO == F32 ? 4 * t + g : 8 * g + t;
    toff[t] = k < KS * KS ? (k / KS) * C::LCP + k % KS : 0;
  }

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int by = (int)(t2 % J.tiles_y);
    const int zz = (int)(t2 / J.tiles_y);
    const int y0 = by * TY, x0 = bx * TX;
    const gbyte* in = gin(J.in) + (int64_t)zz * J.in_zs;
    __syncthreads();
    {
      // chunk (r, k): tile row r, columns 16k .. 16k + 15 (clamped to the
      // image). Whole chunks inside the image of a 16-byte aligned row are one
      // vector load; the others (right edge, unaligned rows) go byte by byte.
      const bool al16 = ((reinterpret_cast<uintptr_t>(in) | (uintptr_t)J.in_rs) & 15) == 0;
      for (int t = tid; t < C::LR * C::NCK; t += C::THREADS) {
        const int r = t / C::NCK, k = t % C::NCK;
        const int y = min(ST * y0 + r, J.hin - 1), xs = ST * x0 + 16 * k;
        const gbyte* row = in + (int64_t)y * J.in_rs;
        unsigned char b[16];
        if (al16 && xs + 15 < J.win) {
          const i4v v = ld<i4v>(row + xs);
#pragma unroll
          for (int e = 0; e < 16; ++e) b[e] = (unsigned char)(v[e >> 2] >> (8 * (e & 3)));
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) b[e] = row[min(xs + e, J.win - 1)];
        }
        AT* dst = tile + r * C::LCP + 16 * k;
        if constexpr (PO == F32) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            *reinterpret_cast<f4*>(dst + 4 * q) =
                f4{(float)b[4 * q], (float)b[4 * q + 1], (float)b[4 * q + 2], (float)b[4 * q + 3]};
        } else {
          // the bf16 of a uint8 is the high half of its float (the low half is zero)
          uint32_t hb[8];
#pragma unroll
          for (int q = 0; q < 8; ++q)
            hb[q] = __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, (float)b[2 * q + 1]),
                                          __builtin_bit_cast(uint32_t, (float)b[2 * q]), 0x07060302u);
          *reinterpret_cast<i4v*>(dst) = i4v{(int)hb[0], (int)hb[1], (int)hb[2], (int)hb[3]};
          *reinterpret_cast<i4v*>(dst + 8) = i4v{(int)hb[4], (int)hb[5], (int)hb[6], (int)hb[7]};
        }
      }
    }
    __syncthreads();
    constexpr int CST = MAXOUT ? COUT / 2 : COUT;  // stored channels
    gbyte* oslice = gout(J.out) + (int64_t)zz * J.out_zs * CST * C::ESZ;
    // channel-blocked output: this lane's bytes of its pixel in the wave's
    // first m-block, and the strides of a tile row and of a plane
    const int wrow = wave * (C::MW / MCOLS);  // the wave's first tile row
    gbyte* const obase = oslice + ((int64_t)(y0 + wrow) * J.out_rs + x0 + n16) * 16 * C::ESZ + 4 * g * C::ESZ;
    const int64_t orow_b = (int64_t)J.out_rs * 16 * C::ESZ, oplane_b = (int64_t)J.out_zs * 16 * C::ESZ;
    int64_t obase_px[MAXOUT ? (COUT / 2) * C::ESZ / 64 : 1];  // max-out stores: see the epilogue
#pragma unroll
    for (int u = 0; u < C::MW; ++u) {
      const int mrow = wrow + u / MCOLS, mcol = u % MCOLS;
      const AT* a0 = tile + ST * (mrow * C::LCP + mcol * 16 + n16);
      f4 acc[C::NB];
#pragma unroll
      // the accumulators start at the bias: the MFMA adds the taps to it
      for (int nb = 0; nb < C::NB; ++nb) acc[nb] = f4{bias[nb][0], bias[nb][1], bias[nb][2], bias[nb][3]};
      if constexpr (PO == F32) {
#pragma unroll
        for (int s = 0; s < C::NSTEP; ++s) {
          const float a = a0[toff[s]];
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb)
            acc[nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wf[s][nb].v[0], a, acc[nb], 0, 0, 0);
        }
      } else {
        bf16x8 a;
#pragma unroll
        for (int t = 0; t < 8; ++t) a[t] = __builtin_bit_cast(__bf16, a0[toff[t]]);
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb)
          acc[nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[0][nb].v, a, acc[nb], 0, 0, 0);
      }
      const int y = y0 + mrow, x = x0 + mcol * 16 + n16;
      if constexpr (MAXOUT) {
        // channels nb*16 + 4g + {0,1} and {2,3} pair up inside the lane: stored
        // channels nb*8 + 2g and nb*8 + 2g + 1 of pixel n16. The m-block's 16
        // stored pixels pass through this wave's LDS scratch, so that each lane
        // stores 16 contiguous bytes. Max-out maps feed a spaced conv and are
        // stored fragment-major.
        static_assert(C::NB == 4, "64 channels, 32 stored per pixel");
        constexpr int PIXB = CST * C::ESZ;  // bytes per stored pixel: 128 (FP32) or 64 (BF16)
        __shared__ __attribute__((aligned(16))) unsigned char scr_all[C::WAVES * 16 * PIXB];
        unsigned char* scr = scr_all + wave * 16 * PIXB;
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          // a compare and a select (fmaxf would first quiet each MFMA result)
          const float m0 = acc[nb][0] > acc[nb][1] ? acc[nb][0] : acc[nb][1];
          const float m1 = acc[nb][2] > acc[nb][3] ? acc[nb][2] : acc[nb][3];
          unsigned char* dst = scr + n16 * PIXB + (nb * 8 + 2 * g) * C::ESZ;
          if constexpr (PO == F32)
            *reinterpret_cast<f2*>(dst) = f2{m0, m1};
          else
            *reinterpret_cast<uint32_t*>(dst) = bf16_key(pack_bf16x2(m0, m1));
        }
        __builtin_amdgcn_wave_barrier();
        const int lgo = (J.geom >> 16) & 0xf;
#pragma unroll
        for (int h = 0; h < PIXB / 64; ++h) {
          // 16-byte chunk c of the block: pixel c / (PIXB / 16), chunk c % (PIXB / 16)
          const int c = h * 64 + lane;
          const i4v o = *reinterpret_cast<const i4v*>(scr + c * 16);
          const int pp = c / (PIXB / 16), xx = x0 + mcol * 16 + pp;
          // pixel index of the row's first m-block, then 16 / 2^lgo further per m-block
          // (the fragment modulus divides 16)
          if (mcol == 0) obase_px[h] = frag_pix(y, x0 + pp, lgo, J.out_rs, J.out_zs);
          if (y < J.hout && xx < J.wout) {
            gbyte* dst = oslice + (obase_px[h] + ((mcol * 16) >> lgo)) * PIXB + (c % (PIXB / 16)) * 16;
            // FP32 maps stream (the hint measured 1-2 % faster there; slower for the BF16 map)
            if constexpr (PO == F32) st_nt<i4v>(dst, o); else st<i4v>(dst, o);
          }
        }
        __builtin_amdgcn_wave_barrier();
        continue;
      }
      if constexpr (C::BLOCKED && XS) {
        // bias + ReLU (and the e4m3 clamp) as below, then plane after plane
        // (16 pixels x 16 channels each) through this wave's LDS scratch
        constexpr int PLB = 16 * 16 * C::ESZ;  // one plane of the m-block
        constexpr int BLK = C::NB * PLB;
        __shared__ __attribute__((aligned(16))) unsigned char xscr[C::WAVES * BLK];
        unsigned char* scr = xscr + wave * BLK;
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          unsigned char* d = scr + nb * PLB + (n16 * 16 + 4 * g) * C::ESZ;
          if constexpr (PO == BF16) {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = relu(acc[nb][k]);
            *reinterpret_cast<u2v*>(d) = u2v{pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3])};
          } else {
            const float inv = prm.out_inv_scale;
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k)
              v[k] = __builtin_amdgcn_fmed3f(acc[nb][k] * inv, 0.0f, 448.0f);
            int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], __builtin_bit_cast(int, v[0]), false);
            w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
            *reinterpret_cast<uint32_t*>(d) = (uint32_t)w & 0x7f7f7f7fu;
          }
        }
        __builtin_amdgcn_wave_barrier();
        const int xb = x0 + mcol * 16;  // the m-block's first pixel
#pragma unroll
        for (int h = 0; h < (BLK / 16 + 63) / 64; ++h) {
          const int c = h * 64 + lane;  // 16-byte chunk of the m-block
          if (c < BLK / 16) {
            const int pl = c / (PLB / 16), cc = c % (PLB / 16);
            const int pp = cc / C::ESZ;  // ESZ chunks per plane pixel
            const i4v o = *reinterpret_cast<const i4v*>(scr + c * 16);
            if (y < J.hout && xb + pp < J.wout)
              st<i4v>(oslice + ((int64_t)pl * J.out_zs + (int64_t)y * J.out_rs + xb) * 16 * C::ESZ + cc * 16, o);
          }
        }
        __builtin_amdgcn_wave_barrier();
      } else if constexpr (C::BLOCKED) {
        // bias + ReLU, stored from registers: lane (g, n16) writes channels
        // 4g .. 4g + 3 of plane nb at pixel n16, bytes 4g * ESZ .. of the
        // pixel's 16 * ESZ, so each n-block's 64 lanes cover the plane's 16
        // pixels as one contiguous run.
        if (y < J.hout && x < J.wout) {
          gbyte* dst = obase + (u / MCOLS) * orow_b + mcol * 16 * 16 * C::ESZ;
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            gbyte* d = dst + nb * oplane_b;
            if constexpr (PO == BF16) {
              float v[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) v[k] = relu(acc[nb][k]);
              st<u2v>(d, u2v{pack_bf16x2(v[0], v[1]), pack_bf16x2(v[2], v[3])});
            } else {
              // relu(t) * s clamped to [0, 448] is the median of (t * s, 0, 448)
              // for s > 0; a negative t can give -0 there, whose code has the
              // sign bit set: clearing bit 7 of each code maps it to +0 and
              // leaves every other (non-negative) code as it is
              const float inv = prm.out_inv_scale;
              float v[4];
#pragma unroll
              for (int k = 0; k < 4; ++k)
                v[k] = __builtin_amdgcn_fmed3f(acc[nb][k] * inv, 0.0f, 448.0f);
              // (the first conversion's high half is any value: the second overwrites it)
              int w = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], __builtin_bit_cast(int, v[0]), false);
              w = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], w, true);
              st<uint32_t>(d, (uint32_t)w & 0x7f7f7f7fu);
            }
          }
        }
      } else {
        // bias + ReLU. The m-block's output (16 pixels x COUT channels, NHWC)
        // passes through this wave's LDS scratch, so that each lane stores 16
        // contiguous bytes.
        static_assert(PO == F32, "BF16 / FP8 output is stored from registers");
        constexpr int BLK = 16 * COUT * 4;  // bytes of the m-block
        __shared__ __attribute__((aligned(16))) unsigned char scr_all[C::WAVES * BLK];
        unsigned char* scr = scr_all + wave * BLK;
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          float v[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) v[k] = relu(acc[nb][k]);
          *reinterpret_cast<f4*>(scr + (n16 * COUT + nb * 16 + 4 * g) * 4) = f4{v[0], v[1], v[2], v[3]};
        }
        __builtin_amdgcn_wave_barrier();
        const int xb = x0 + mcol * 16;  // the m-block's first pixel
        const int64_t pix0 = (int64_t)y * J.out_rs + xb;
#pragma unroll
        for (int h = 0; h < (BLK / 16 + 63) / 64; ++h) {
          const int c = h * 64 + lane;  // 16-byte chunk of the block
          if (c < BLK / 16) {
            const i4v o = *reinterpret_cast<const i4v*>(scr + c * 16);
            const int pp = c / (COUT / 4);  // COUT / 4 chunks per pixel
            gbyte* dst = oslice + (pix0 + pp) * COUT * 4 + (c % (COUT / 4)) * 16;
            if (y < J.hout && xb + pp < J.wout) st_nt<i4v>(dst, o);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA conv

// Packed weights: for channel block cb, group-step s, n-block nb, lane l,
// U chunks of 16 bytes. Lane l (n = l % 16, lane group g = l / 16) holds for
// chunk slot c = 4 U s + 4 uu + g the CHB input channels of tap (i, j), chunk
// cg, where c -> (i, j, cg) row-major over (KS, KS, NCHB). The A side decodes
// the same slot the same way, so the MFMA contracts matching K indices
// whatever order the instruction uses inside a lane's operand bytes.
template <int P, int CIN, int COUT, int KS, bool POOL, bool HEAD, int TY, int TX, int MW>
__global__ __launch_bounds__((Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>::THREADS)) void conv_mfma(JobSet js, ConvParams prm) {
  using C = Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>;
  using T = PT<P>;
  static_assert(P == F32, "conv_mfma is the FP32 (NHWC) kernel; BF16 / FP8 use conv_ws");
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  constexpr int MCOLS = TX / 16;
  constexpr int ELB = CIN * T::BYTES;  // bytes per stored input pixel

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int by = (int)(t2 % J.tiles_y);
    const int zz = (int)(t2 / J.tiles_y);
    const int y0 = by * TY, x0 = bx * TX;
    const int hp = J.hin - (POOL ? 1 : 0), wp = J.win - (POOL ? 1 : 0);  // logical input dims
    const gbyte* in = gin(J.in) + (int64_t)zz * J.in_zs * ELB;
    const int64_t rowb = J.in_rs * ELB;

    f4 acc[MW][C::NB];
#pragma unroll
    for (int u = 0; u < MW; ++u)
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb) acc[u][nb] = f4{0.f, 0.f, 0.f, 0.f};

    for (int cb = 0; cb < C::NCB; ++cb) {
      __syncthreads();
      // ---- stage the (TY+KS-1) x (TX+KS-1) input tile of this channel block,
      //      applying the preceding 2x2 stride-1 max filter while loading
      stage_tile<P, C::LR, C::LC, C::NCHB, C::PSB, C::THREADS, POOL>(
          lds, in + (cb * C::CB) * T::BYTES, rowb, ELB, y0, x0, hp, wp, tid);
      __syncthreads();
      // ---- implicit GEMM over this block's (tap, chunk) slots
      const gbyte* wb = gin(prm.wpack) +
                                (size_t)cb * C::NGS * C::NB * 64 * T::U * 16;
#pragma unroll 2
      for (int s = 0; s < C::NGS; ++s) {
        Frag<P> bfr[C::NB];
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const gbyte* p = wb + ((size_t)(s * C::NB + nb) * 64 + lane) * (T::U * 16);
          load_frag<P>(bfr[nb], p, p + 16);
        }
        int off[T::U];
#pragma unroll
        for (int uu = 0; uu < T::U; ++uu) {
          int c = s * (4 * T::U) + 4 * uu + g;
          c = c < C::NCHK ? c : C::NCHK - 1;  // padded slot: any finite data, weights are 0
          const int i = c / (KS * C::NCHB);
          const int rem = c % (KS * C::NCHB);
          const int j = rem / C::NCHB, cg = rem % C::NCHB;
          off[uu] = (i * C::LC + j) * C::PSB + cg * 16;
        }
#pragma unroll
        for (int u = 0; u < MW; ++u) {
          const int mb = wave * MW + u;
          const int mrow = mb / MCOLS, mcol = mb % MCOLS;
          const unsigned char* a0 = lds + (mrow * C::LC + mcol * 16 + n16) * C::PSB;
          Frag<P> afr;
          load_frag<P>(afr, a0 + off[0], a0 + off[T::U - 1]);
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) mma<P>(acc[u][nb], afr, bfr[nb]);
        }
      }
    }

    // ---- epilogue: lane holds D[m = 4 g + k][n = n16] of each (m-block, n-block)
    float bias[C::NB], osc[C::NB], hw[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) {
      bias[nb] = ldf(prm.bias, nb * 16 + n16);
      osc[nb] = prm.oscale ? ldf(prm.oscale, nb * 16 + n16) : 1.0f;
      if constexpr (HEAD) hw[nb] = ldf(prm.head_w, nb * 16 + n16);
    }
    if constexpr (HEAD) {
      head_epilogue<MW, C::NB>(
          [&](int u, int nb, int k) __attribute__((always_inline)) { return acc[u][nb][k]; },
          [&](int u, int& y, int& xb) __attribute__((always_inline)) {
            const int mb = wave * MW + u;
            y = y0 + mb / MCOLS;
            xb = x0 + (mb % MCOLS) * 16;
          },
          bias, osc, hw, prm.head_b, g, n16, gout(J.out), (int64_t)zz * J.out_zs, J.out_rs, J.hout, J.wout);
    } else {
#pragma unroll
      for (int u = 0; u < MW; ++u) {
        const int mb = wave * MW + u;
        const int y = y0 + mb / MCOLS;
        const int xb = x0 + (mb % MCOLS) * 16 + 4 * g;
        if (y < J.hout) {
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int x = xb + k;
            if (x < J.wout) {
              const int64_t pix = (int64_t)zz * J.out_zs + (int64_t)y * J.out_rs + x;
#pragma unroll
              for (int nb = 0; nb < C::NB; ++nb) {
                const float v = relu(fmaf(acc[u][nb][k], osc[nb], bias[nb]));
                store_act<P>(gout(J.out), pix * COUT + nb * 16 + n16, v, prm.out_inv_scale);
              }
            }
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------- MFMA conv, row reuse

// Same layer as conv_mfma, with the K loop ordered by filter row so that A
// fragments are reused across output rows. A wave owns MR output rows x MC
// m-blocks of 16 pixels. For each group-step of one filter row's (j, chunk)
// slots, the B fragments of all KS filter rows stay in registers, and the A
// fragment of input row q (wave-relative) is loaded from LDS once and feeds
// every filter row i with output row q - i in [0, MR): (MR + KS - 1) LDS loads
// per MR * KS MFMA groups instead of one load per group.
// Packed weights: [cb][i][rs][nb][lane][U chunks of 16 B]; lane (n, g) holds
// for slot c = (4 rs + g) U + uu of filter row i the chunk (j, cg) =
// (c / NCHB, c % NCHB) of tap (i, j); slots past KS * NCHB are zero.
template <int P, int CIN, int COUT, int KS, int MR, int MC, int WX, int WY, bool HEAD, int CBO = 0>
struct CfgRR {
  using T = PT<P>;
  static constexpr int CB = CBO ? CBO : ((T::CB < CIN) ? T::CB : CIN);
  static_assert(CIN % CB == 0, "channel block must divide CIN");
  static constexpr int NCB = CIN / CB;
  static constexpr int NCHB = CB / T::CHB;
  static_assert(NCHB * T::CHB == CB, "block must be whole chunks");
  static constexpr int NCHR = KS * NCHB;  // chunks per filter row
  static constexpr int SLOTS = 4 * T::U;
  static constexpr int NGR = (NCHR + SLOTS - 1) / SLOTS;  // group-steps per filter row
  static constexpr int NB = COUT / 16;
  static constexpr int TY = WY * MR, TX = WX * MC * 16;
  static constexpr int LR = TY + KS - 1, LC = TX + KS - 1;
  static constexpr int PSB = pad_words(CB * T::BYTES / 4) * 4;
  static constexpr int LDS_IN = LR * LC * PSB;
  static constexpr int LDS = LDS_IN;
  static constexpr int THREADS = WX * WY * 64;
  static_assert(LDS <= 160 * 1024, "LDS budget of a gfx950 workgroup");
};

template <int P, int CIN, int COUT, int KS, bool POOL, bool HEAD, int MR, int MC, int WX, int WY, int CBO>
__global__ __launch_bounds__((CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::THREADS)) void conv_mfma_rr(
    JobSet js, ConvParams prm) {
  using C = CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>;
  using T = PT<P>;
  static_assert(P == F32, "conv_mfma_rr is the FP32 (NHWC) kernel; BF16 / FP8 use conv_ws");
  constexpr int TY = C::TY, TX = C::TX;
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  const int wy = wave / WX, wx = wave % WX;
  constexpr int ELB = CIN * T::BYTES;

  // per-lane slot offsets inside a filter row (column and chunk), fixed per lane
  int coff[C::NGR][T::U];
#pragma unroll
  for (int rs = 0; rs < C::NGR; ++rs)
#pragma unroll
    for (int uu = 0; uu < T::U; ++uu) {
      int c = (4 * rs + g) * T::U + uu;
      c = c < C::NCHR ? c : C::NCHR - 1;  // padded slot: finite data, zero weights
      coff[rs][uu] = (c / C::NCHB) * C::PSB + (c % C::NCHB) * 16;
    }

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int by = (int)(t2 % J.tiles_y);
    const int zz = (int)(t2 / J.tiles_y);
    const int y0 = by * TY, x0 = bx * TX;
    const int hp = J.hin - (POOL ? 1 : 0), wp = J.win - (POOL ? 1 : 0);
    const gbyte* in = gin(J.in) + (int64_t)zz * J.in_zs * ELB;
    const int64_t rowb = J.in_rs * ELB;

    f4 acc[MR][MC][C::NB];
#pragma unroll
    for (int r = 0; r < MR; ++r)
#pragma unroll
      for (int m = 0; m < MC; ++m)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) acc[r][m][nb] = f4{0.f, 0.f, 0.f, 0.f};

    for (int cb = 0; cb < C::NCB; ++cb) {
      __syncthreads();
      stage_tile<P, C::LR, C::LC, C::NCHB, C::PSB, C::THREADS, POOL>(
          lds, in + (cb * C::CB) * T::BYTES, rowb, ELB, y0, x0, hp, wp, tid);
      __syncthreads();
      const gbyte* wb = gin(prm.wpack) +
                                (size_t)cb * KS * C::NGR * C::NB * 64 * T::U * 16;
      const unsigned char* abase = lds + ((wy * MR) * C::LC + wx * MC * 16 + n16) * C::PSB;
      for (int rs = 0; rs < C::NGR; ++rs) {
        Frag<P> bfr[KS][C::NB];
#pragma unroll
        for (int i = 0; i < KS; ++i)
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            const gbyte* p = wb + ((size_t)((i * C::NGR + rs) * C::NB + nb) * 64 + lane) * (T::U * 16);
            load_frag<P>(bfr[i][nb], p, p + 16);
          }
        int o0 = coff[0][0], o1 = coff[0][T::U - 1];
#pragma unroll
        for (int q = 0; q < C::NGR; ++q)
          if (q == rs) {
            o0 = coff[q][0];
            o1 = coff[q][T::U - 1];
          }
#pragma unroll
        for (int q = 0; q < MR + KS - 1; ++q) {
#pragma unroll
          for (int m = 0; m < MC; ++m) {
            const unsigned char* a0 = abase + (q * C::LC + m * 16) * C::PSB;
            Frag<P> afr;
            load_frag<P>(afr, a0 + o0, a0 + o1);
#pragma unroll
            for (int i = 0; i < KS; ++i) {
              const int r = q - i;
              if (r >= 0 && r < MR) {
#pragma unroll
                for (int nb = 0; nb < C::NB; ++nb) mma<P>(acc[r][m][nb], afr, bfr[i][nb]);
              }
            }
          }
        }
      }
    }

    float bias[C::NB], osc[C::NB], hw[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) {
      bias[nb] = ldf(prm.bias, nb * 16 + n16);
      osc[nb] = prm.oscale ? ldf(prm.oscale, nb * 16 + n16) : 1.0f;
      if constexpr (HEAD) hw[nb] = ldf(prm.head_w, nb * 16 + n16);
    }
    if constexpr (HEAD) {
      head_epilogue<MR * MC, C::NB>(
          [&](int u, int nb, int k) __attribute__((always_inline)) { return acc[u / MC][u % MC][nb][k]; },
          [&](int u, int& y, int& xb) __attribute__((always_inline)) {
            y = y0 + wy * MR + u / MC;
            xb = x0 + (wx * MC + u % MC) * 16;
          },
          bias, osc, hw, prm.head_b, g, n16, gout(J.out), (int64_t)zz * J.out_zs, J.out_rs, J.hout, J.wout);
    } else {
#pragma unroll
      for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int m = 0; m < MC; ++m) {
          const int y = y0 + wy * MR + r, xb = x0 + (wx * MC + m) * 16 + 4 * g;
          if (y < J.hout) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const int x = xb + k;
              if (x < J.wout) {
                const int64_t pix = (int64_t)zz * J.out_zs + (int64_t)y * J.out_rs + x;
#pragma unroll
                for (int nb = 0; nb < C::NB; ++nb) {
                  const float v = relu(fmaf(acc[r][m][nb][k], osc[nb], bias[nb]));
                  store_act<P>(gout(J.out), pix * COUT + nb * 16 + n16, v, prm.out_inv_scale);
                }
              }
            }
          }
        }
    }
  }
}

// ---------------------------------------------------------------- spaced MFMA conv (stride-2 pool nets)

// One conv of a net whose pools have stride 2 (FastMemb, Section 2.2), in its
// dense form: taps spaced d apart, fed by a 2x2 max filter with spacing pd
// (the geom field of the job). The paper splits every stride-k operation into
// k^2 fragments computed independently; here the fragments are the d^2 phase
// sub-lattices of the output (positions py + d r, px + d c), each tiled like a
// plain conv: an operand pixel of the LDS tile is the input at spacing d, so
// the implicit GEMM (K = (tap, 16-byte chunk), 16x16x4 FP32 MFMA) and its
// packed weights are those of conv_mfma. The maps between layers are stored
// as the fragments themselves: a map read by a conv of spacing d holds each of
// its d^2 phase sub-lattices as a row-major block (fragment-major, see
// LayerJob::geom), so an operand row is a contiguous run of one fragment.
// Staging applies the max filter: 4 loads per operand chunk, the partners pd
// apart being the same run of three other fragments (frag_tile).
// EPI 1: bias, then max-out over channel pairs, COUT / 2 channels stored
// (NHWC pixels, fragment-major modulo the next conv's spacing 2d). EPI 2:
// bias, then the two-class softmax of channels 0 and 1 (the other output
// channels are zero padding), storing the class-1 probability (row-major).
// Elementwise max of two 16-byte chunks of signed activations: FP32 compares
// floats; BF16 chunks hold keys (bf16_key) and compare as unsigned halves.
template <int P>
__device__ __forceinline__ i4v chunk_max_signed(i4v a, i4v b) {
  static_assert(P == F32 || P == BF16, "signed max: FP32 or keyed BF16 activations");
  return chunk_max<P>(a, b);
}

// Stage the LR x LC operand tile of one phase sub-lattice (channel chunks
// 0 .. NCHB-1 of the block at byte offset cofs of each pixel): operand pixel
// (r, c) is the 2x2 max filter addressed by f (frag_tile). P: the stored
// activation type.
template <int P, int LR, int LC, int NCHB, int PSB, int THREADS>
__device__ __forceinline__ void stage_phase_tile(unsigned char* lds, const FragTile& f, int cofs, int elb, int y0,
                                                 int x0, int tid) {
  constexpr int NST = LR * LC * NCHB;
  constexpr int NIT = (NST + THREADS - 1) / THREADS;
#pragma unroll 2
  for (int k = 0; k < NIT; ++k) {
    const int t = tid + k * THREADS;
    if (t < NST) {
      const int cg = t % NCHB, pix = t / NCHB;
      const int r = pix / LC, c = pix % LC;
      const gbyte* q = f.at(y0 + r, x0 + c, elb) + cofs + cg * 16;
      const i4v a = ld<i4v>(q), b = ld<i4v>(q + f.o01);
      const i4v e = ld<i4v>(q + f.o10), g = ld<i4v>(q + f.o11);
      i4v m = chunk_max_signed<P>(chunk_max_signed<P>(a, b), chunk_max_signed<P>(e, g));
      if constexpr (P == BF16) {
#pragma unroll
        for (int w = 0; w < 4; ++w) m[w] = (int)bf16_unkey((uint32_t)m[w]);  // keys -> bf16 operands
      }
      st<i4v>(lds + pix * PSB + cg * 16, m);
    }
  }
}

// Stage the operand tiles of the four phases of a group (channel chunks 0 ..
// NCHB-1 of the block at byte offset cofs of each pixel; fragments and clamps
// as in head_taps4): member m = 2a + b's tile at rows m LR .. m LR + LR - 1,
// its operand pixel (R, C) the max of four of the nine distinct (fragment,
// shift) chunks of position (R, C). P: the stored activation type.
template <int P, int LR, int LC, int NCHB, int PSB, int THREADS>
__device__ __forceinline__ void stage_group_tile(unsigned char* lds, const gbyte* f00, int64_t o01, int64_t o10,
                                                 int64_t rowb, int elb, int rvA, int rvB, int cvA, int cvB, int y0,
                                                 int x0, int tid) {
  constexpr int NST = LR * LC * NCHB;
  constexpr int NIT = (NST + THREADS - 1) / THREADS;
#pragma unroll 2
  for (int k = 0; k < NIT; ++k) {
    const int t = tid + k * THREADS;
    if (t < NST) {
      const int cg = t % NCHB, pix = t / NCHB;
      const int R = y0 + pix / LC, Cc = x0 + pix % LC;
      const int64_t rA = (int64_t)min(R, rvA) * rowb, rB = (int64_t)min(R, rvB) * rowb;
      const int64_t rA1 = (int64_t)min(R + 1, rvA) * rowb;
      const int64_t cA = (int64_t)min(Cc, cvA) * elb, cB = (int64_t)min(Cc, cvB) * elb;
      const int64_t cA1 = (int64_t)min(Cc + 1, cvA) * elb;
      const gbyte* b = f00 + cg * 16;
      const i4v v0 = ld<i4v>(b + rA + cA), v1 = ld<i4v>(b + o01 + rA + cB);
      const i4v v2 = ld<i4v>(b + o10 + rB + cA), v3 = ld<i4v>(b + o10 + o01 + rB + cB);
      const i4v v4 = ld<i4v>(b + rA + cA1), v5 = ld<i4v>(b + o10 + rB + cA1);
      const i4v v6 = ld<i4v>(b + rA1 + cA), v7 = ld<i4v>(b + o01 + rA1 + cB);
      const i4v v8 = ld<i4v>(b + rA1 + cA1);
      i4v op[4];
      op[0] = chunk_max_signed<P>(chunk_max_signed<P>(v0, v1), chunk_max_signed<P>(v2, v3));  // (0, 0)
      op[1] = chunk_max_signed<P>(chunk_max_signed<P>(v1, v4), chunk_max_signed<P>(v3, v5));  // (0, 1)
      op[2] = chunk_max_signed<P>(chunk_max_signed<P>(v2, v3), chunk_max_signed<P>(v6, v7));  // (1, 0)
      op[3] = chunk_max_signed<P>(chunk_max_signed<P>(v3, v5), chunk_max_signed<P>(v7, v8));  // (1, 1)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if constexpr (P == BF16) {
#pragma unroll
          for (int w = 0; w < 4; ++w) op[m][w] = (int)bf16_unkey((uint32_t)op[m][w]);
        }
        st<i4v>(lds + (m * LR * LC + pix) * PSB + cg * 16, op[m]);
      }
    }
  }
}

// GRP = 1: the items are groups of four phases whose max filters share
// fragments (the max filter has half the conv's spacing), each a TY x TX tile
// of every member, staged together (stage_group_tile); m-block mb belongs to
// member mb / (TY TX / 16).
template <int P, int CIN, int COUT, int KS, int TY, int TX, int MW, int EPI, int CB, int GRP = 0>
__global__ __launch_bounds__((Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CB, GRP ? 4 : 1>::THREADS)) void conv_phase(
    JobSet js, ConvParams prm) {
  using C = Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CB, GRP ? 4 : 1>;
  static_assert(!GRP || (EPI == 1 && P == F32), "phase groups: the FP32 max-out convs");
  constexpr int MPM = TY * TX / 16;  // m-blocks of one member's tile
  using T = PT<P>;
  static_assert(P == F32 || P == BF16, "FP32 or BF16 activations (NHWC)");
  static_assert(EPI == 1 || EPI == 2, "max-out or softmax epilogue");
  static_assert(EPI != 2 || C::NB == 1, "the MFMA softmax layer has one 16-channel n-block");
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS_TILE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  constexpr int MCOLS = TX / 16;
  constexpr int ELB = CIN * T::BYTES;  // bytes per stored input pixel

  float bias[C::NB];
#pragma unroll
  for (int nb = 0; nb < C::NB; ++nb) bias[nb] = ldf(prm.bias, nb * 16 + n16);

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    const int d = max(J.geom & 0xff, 1), h = d >> 1;
    // item order: tile column, then phase (GRP: phase group), then tile row,
    // then slice. The d^2 phases of one tile row are neighbours in the item
    // range, so the workgroups of an XCD stage them together: their max
    // filters read each other's pixels, which then meet in that XCD's L2.
    const int nph = GRP ? h * h : d * d;
    const int tpy = J.tiles_y / nph;  // tile rows per phase (group)
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int ph = (int)(t2 % nph);
    const int64_t t3 = t2 / nph;
    const int by = (int)(t3 % tpy);
    const int zz = (int)(t3 / tpy);
    // GRP: (py, px) is the group's first phase (gy, gx); member (a, b) adds (a h, b h)
    const int py = GRP ? ph / h : ph / d, px = GRP ? ph % h : ph % d;
    const int y0 = by * TY, x0 = bx * TX;  // sub-lattice coordinates of the tile
    // operand pixel (r, c) is the max filter at input (py + d (y0 + r), px + d (x0 + c))
    const FragTile ft = frag_tile(gin(J.in) + (int64_t)zz * J.in_zs * ELB, ELB, J, py, px);
    const int lgo = (J.geom >> 16) & 0xf;  // output map: fragment-major modulo 2^lgo

    f4 acc[MW][C::NB];
#pragma unroll
    for (int u = 0; u < MW; ++u)
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb) acc[u][nb] = f4{0.f, 0.f, 0.f, 0.f};

    for (int cb = 0; cb < C::NCB; ++cb) {
      __syncthreads();
      if constexpr (GRP) {
        const int lg = __builtin_ctz(d);
        const int64_t plane = (J.in_zs >> (2 * lg)) * ELB;  // bytes per fragment
        const gbyte* f00 = gin(J.in) + (int64_t)zz * J.in_zs * ELB + (int64_t)(py * d + px) * plane +
                           cb * C::CB * T::BYTES;
        stage_group_tile<P, C::LR, C::LC, C::NCHB, C::PSB, C::THREADS>(
            lds, f00, h * plane, (int64_t)h * d * plane, J.in_rs * ELB, ELB, (J.hin - 1 - py) >> lg,
            (J.hin - 1 - py - h) >> lg, (J.win - 1 - px) >> lg, (J.win - 1 - px - h) >> lg, y0, x0, tid);
      } else {
        stage_phase_tile<P, C::LR, C::LC, C::NCHB, C::PSB, C::THREADS>(lds, ft, cb * C::CB * T::BYTES, ELB, y0, x0,
                                                                        tid);
      }
      __syncthreads();
      // ---- implicit GEMM over this block's (tap, chunk) slots (as conv_mfma)
      const gbyte* wb = gin(prm.wpack) + (size_t)cb * C::NGS * C::NB * 64 * 16;
#pragma unroll 2
      for (int s = 0; s < C::NGS; ++s) {
        Frag<P> bfr[C::NB];
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const gbyte* p = wb + ((size_t)(s * C::NB + nb) * 64 + lane) * 16;
          load_frag<P>(bfr[nb], p, p);
        }
        int c = s * 4 + g;
        c = c < C::NCHK ? c : C::NCHK - 1;  // padded slot: any finite data, weights are 0
        const int i = c / (KS * C::NCHB);
        const int rem = c % (KS * C::NCHB);
        const int j = rem / C::NCHB, cg = rem % C::NCHB;
        const int off = (i * C::LC + j) * C::PSB + cg * 16;
#pragma unroll
        for (int u = 0; u < MW; ++u) {
          const int mb = wave * MW + u;
          const int mm = mb / MPM, lmb = mb % MPM;  // member, m-block in its tile
          const int mrow = lmb / MCOLS, mcol = lmb % MCOLS;
          const unsigned char* a0 = lds + ((mm * C::LR + mrow) * C::LC + mcol * 16 + n16) * C::PSB;
          Frag<P> afr;
          load_frag<P>(afr, a0 + off, a0 + off);
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) mma<P>(acc[u][nb], afr, bfr[nb]);
        }
      }
    }

    // ---- epilogue: lane holds D[m = 4 g + k][n = n16] of each (m-block, n-block)
    if constexpr (EPI == 1 && P == BF16) {
#pragma unroll
      for (int u = 0; u < MW; ++u) {
        const int mb = wave * MW + u;
        const int mrow = mb / MCOLS, mcol = mb % MCOLS;
        const int y = py + d * (y0 + mrow);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int x = px + d * (x0 + mcol * 16 + 4 * g + k);
          const bool ok = y < J.hout && x < J.wout;
          const int64_t pix = (int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs);
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            const float v = acc[u][nb][k] + bias[nb];
            const float m = fmaxf(v, dpp_f<kQuadXor1>(v));  // channel pair (n16 & ~1, n16 | 1)
            // lanes n16 = 4q hold stored channel nb*8 + 2q, lanes 4q + 2 channel nb*8 + 2q + 1
            const float m2 = dpp_f<kQuadXor2>(m);
            if (ok && (n16 & 3) == 0)
              st<uint32_t>(gout(J.out) + (pix * (COUT / 2) + nb * 8 + n16 / 2) * 2, bf16_key(pack_bf16x2(m, m2)));
          }
        }
      }
    } else {
      // The finished operand tile serves as each wave's scratch: FP32 max-out
      // rows leave as 16 contiguous bytes per lane; the class-1 probabilities
      // of a wave's m-blocks leave in one store with every lane active.
      __syncthreads();  // every wave is done reading the operand tile
      if constexpr (EPI == 1) {
        constexpr int PIXB = (COUT / 2) * 4;  // one stored FP32 pixel
        static_assert(C::WAVES * 16 * PIXB <= C::LDS_TILE, "scratch fits in the operand tile");
        unsigned char* scr = lds + wave * 16 * PIXB;
        const int e = n16 & 1, pc = n16 >> 1;  // lanes 2pc, 2pc + 1 hold pair pc's max
#pragma unroll
        for (int u = 0; u < MW; ++u) {
          const int mb = wave * MW + u;
          const int mm = mb / MPM, lmb = mb % MPM;
          const int mrow = lmb / MCOLS, mcol = lmb % MCOLS;
          const int mpy = py + (mm >> 1) * h, mpx = px + (mm & 1) * h;  // the member's phase
          const int y = mpy + d * (y0 + mrow);
          // lane parity e keeps pixels 4g + e and 4g + 2 + e
          float keep[2][C::NB];
#pragma unroll
          for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb) {
              const float v = acc[u][nb][k] + bias[nb];
              const float m = fmaxf(v, dpp_f<kQuadXor1>(v));  // channel pair (n16 & ~1, n16 | 1)
              keep[k >> 1][nb] = (k & 1) ? (e ? m : keep[k >> 1][nb]) : m;
            }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int nb = 0; nb < C::NB; ++nb)
              *reinterpret_cast<float*>(scr + (4 * g + 2 * h + e) * PIXB + (nb * 8 + pc) * 4) = keep[h][nb];
          __builtin_amdgcn_wave_barrier();
          // 16 pixels x PIXB / 16 chunks = PIXB chunks of 16 bytes (40 or 56
          // stored channels leave a partly filled last round)
#pragma unroll
          for (int h = 0; h < (PIXB + 63) / 64; ++h) {
            const int c = h * 64 + lane;  // 16-byte chunk: pixel c / (PIXB / 16)
            if (PIXB % 64 != 0 && c >= PIXB) break;
            const i4v o = *reinterpret_cast<const i4v*>(scr + c * 16);
            const int x = mpx + d * (x0 + mcol * 16 + c / (PIXB / 16));
            if (y < J.hout && x < J.wout)
              st_nt<i4v>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * PIXB +
                             (c % (PIXB / 16)) * 16,
                         o);
          }
          __builtin_amdgcn_wave_barrier();
        }
      } else {
        float* scr = reinterpret_cast<float*>(lds) + wave * MW * 16;
        static_assert(C::WAVES * MW * 16 * 4 <= C::LDS_TILE, "scratch fits in the operand tile");
#pragma unroll
        for (int u = 0; u < MW; ++u)
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const float z = acc[u][0][k] + bias[0];
            const float z0 = dpp_f<kQuadXor1>(z);  // lane 1 receives class 0's logit
            if (n16 == 1) scr[u * 16 + 4 * g + k] = sigmoid_f(z - z0);
          }
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < MW * 16; i += 64) {
          const int mb = wave * MW + i / 16;
          const int mrow = mb / MCOLS, mcol = mb % MCOLS;
          const int y = py + d * (y0 + mrow), x = px + d * (x0 + mcol * 16 + i % 16);
          if (y < J.hout && x < J.wout)
            st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * 4, scr[i]);
        }
      }
    }
  }
}

// The two-class softmax layer of a stride-2 pool net on the VALU. Its two
// output channels would fill 2 of an MFMA's 16 columns; on the VALU the
// class-1 probability needs only the logit difference, KS^2 x CIN FP32
// multiply-adds per pixel with the weight difference W[1] - W[0]. The operand
// tile is conv_phase's (all CIN channels in one stage); one output pixel per
// thread, reading operand pixels along a row, which is conflict-free with the
// 8 (mod 16) dword pixel stride. The weight differences are laid out
// [i][cg][j][4 channels] and read with wave-uniform (scalar) loads.
template <int CIN, int KS, int TY, int TX>
struct CfgHead {
  static constexpr int LR = TY + KS - 1, LC = TX + KS - 1;
  static constexpr int NCHB = CIN / 4;  // 16-byte chunks per operand pixel
  static constexpr int PSB = pad_words(CIN) * 4;
  static constexpr int LDS = LR * LC * PSB;
  static constexpr int THREADS = TY * TX;
  static_assert(THREADS <= 1024 && THREADS % 64 == 0, "one output pixel per thread");
};

// BF16 input (P == BF16): the operand tile is staged widened to FP32, so the
// layer computes in FP32 in every form.
template <int LR, int LC, int NCHB_IN, int PSB, int THREADS>
__device__ __forceinline__ void stage_phase_tile_widen(unsigned char* lds, const FragTile& ft, int elb, int y0, int x0,
                                                       int tid) {
  constexpr int NST = LR * LC * NCHB_IN;
  constexpr int NIT = (NST + THREADS - 1) / THREADS;
#pragma unroll 2
  for (int k = 0; k < NIT; ++k) {
    const int t = tid + k * THREADS;
    if (t < NST) {
      const int cg = t % NCHB_IN, pix = t / NCHB_IN;
      const int r = pix / LC, c = pix % LC;
      const gbyte* q = ft.at(y0 + r, x0 + c, elb) + cg * 16;
      const i4v a = ld<i4v>(q), b = ld<i4v>(q + ft.o01);
      const i4v e = ld<i4v>(q + ft.o10), f = ld<i4v>(q + ft.o11);
      i4v m = chunk_max_signed<BF16>(chunk_max_signed<BF16>(a, b), chunk_max_signed<BF16>(e, f));
#pragma unroll
      for (int w = 0; w < 4; ++w) m[w] = (int)bf16_unkey((uint32_t)m[w]);
      // 8 bf16 channels -> 8 floats (exact)
      f4 lo, hi;
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        lo[2 * w] = __builtin_bit_cast(float, (uint32_t)m[w] << 16);
        lo[2 * w + 1] = __builtin_bit_cast(float, (uint32_t)m[w] & 0xffff0000u);
        hi[2 * w] = __builtin_bit_cast(float, (uint32_t)m[w + 2] << 16);
        hi[2 * w + 1] = __builtin_bit_cast(float, (uint32_t)m[w + 2] & 0xffff0000u);
      }
      st<f4>(lds + pix * PSB + cg * 32, lo);
      st<f4>(lds + pix * PSB + cg * 32 + 16, hi);
    }
  }
}

template <int P, int CIN, int KS, int TY, int TX>
__global__ __launch_bounds__((CfgHead<CIN, KS, TY, TX>::THREADS)) void head_phase(JobSet js, ConvParams prm) {
  using C = CfgHead<CIN, KS, TY, TX>;
  static_assert(P == F32 || P == BF16, "FP32 or BF16 input activations (NHWC)");
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS];
  const int tid = threadIdx.x;
  const int r = tid / TX, c = tid % TX;  // the thread's output pixel inside the tile
  constexpr int ELB = CIN * PT<P>::BYTES;
  // constant address space: the compiler reads uniform addresses with scalar loads
  const __attribute__((address_space(4))) float* wk = (const __attribute__((address_space(4))) float*)prm.wpack;
  const float b0 = ldf(prm.bias, 0), b1 = ldf(prm.bias, 1);

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    // item order and phase decomposition as conv_phase
    const int d = max(J.geom & 0xff, 1);
    const int tpy = J.tiles_y / (d * d);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int ph = (int)(t2 % (d * d));
    const int64_t t3 = t2 / (d * d);
    const int by = (int)(t3 % tpy);
    const int zz = (int)(t3 / tpy);
    const int py = ph / d, px = ph % d;
    const int y0 = by * TY, x0 = bx * TX;
    const FragTile ft = frag_tile(gin(J.in) + (int64_t)zz * J.in_zs * ELB, ELB, J, py, px);
    // the class-1 probability of a two-class softmax is the sigmoid of the
    // logit difference: one dot product with the weight difference
    __syncthreads();
    if constexpr (P == F32)
      stage_phase_tile<F32, C::LR, C::LC, C::NCHB, C::PSB, C::THREADS>(lds, ft, 0, ELB, y0, x0, tid);
    else
      stage_phase_tile_widen<C::LR, C::LC, CIN / 8, C::PSB, C::THREADS>(lds, ft, ELB, y0, x0, tid);
    __syncthreads();
    float z = 0.f;
#pragma unroll
    for (int i = 0; i < KS; ++i)
#pragma unroll
      for (int cg = 0; cg < C::NCHB; ++cg)
#pragma unroll
        for (int j = 0; j < KS; ++j) {
          const f4 x = *reinterpret_cast<const f4*>(lds + ((r + i) * C::LC + c + j) * C::PSB + cg * 16);
          const __attribute__((address_space(4))) float* w = wk + ((i * C::NCHB + cg) * KS + j) * 4;
#pragma unroll
          for (int e = 0; e < 4; ++e) z = fmaf(x[e], w[e], z);
        }
    const int y = py + d * (y0 + r), x = px + d * (x0 + c);
    if (y < J.hout && x < J.wout)
      st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, (J.geom >> 16) & 0xf, J.out_rs, J.out_zs)) * 4,
                sigmoid_f(z + (b1 - b0)));
  }
}

// The two-class softmax layer of a stride-2 pool net as one small GEMM per
// operand pixel. With Wd = W[1] - W[0], the logit difference at output (r, c)
// of a phase tile is the sum over taps (i, j) of D[(r + i, c + j)][(i, j)],
// where D[p][t] = sum over channels of X[p][ch] Wd[t][ch]: one 16-column
// n-block over the KS^2 = 16 taps. Each operand pixel (the 2x2 max filter)
// thus goes through the MFMA once, against once per tap with 14 of 16
// columns zero in the padded implicit GEMM. D leaves the accumulators for LDS
// as planes E[t][pixel]; each thread then sums its output pixel's 16 taps from
// 16 planes and stores the class-1 probability, the sigmoid of the sum plus
// b1 - b0.
//
// Operand tile: LR = TY + KS - 1 rows of LCP = 16 NBC columns (whole
// m-blocks), TX = LCP - KS + 1 outputs a row. Lane (n16, g) of an m-block
// loads 16-byte chunk 4t + g of pixel n16 for MFMA step t; the packed B
// fragment of step t holds, in lane (n16, g), tap n16's differences for the
// same chunk's channels. Plane stride PS = 8 (mod 16) dwords: the sixteen
// planes one 16-byte accumulator store spans land on distinct banks.
template <int P, int CIN, int KS, int TY, int NBC, int NW>
struct CfgTaps {
  static constexpr int LR = TY + KS - 1, LCP = 16 * NBC, TX = LCP - KS + 1;
  static constexpr int MB = LR * NBC;                      // m-blocks of the operand tile
  static constexpr int NK = CIN * PT<P>::BYTES / 64;       // MFMA steps (16-byte chunks per lane group)
  static constexpr int PS = pad_words(LR * LCP);
  static constexpr int LDS = 16 * PS * 4;
  static constexpr int THREADS = NW * 64;
  static constexpr int UB = 4;                             // m-blocks a wave loads at once
  static_assert(KS * KS == 16, "the taps fill one 16-column n-block");
  static_assert(NK * 64 == CIN * PT<P>::BYTES, "whole 16-byte chunks per lane group");
  static_assert(LDS <= 160 * 1024, "LDS budget of a gfx950 workgroup");
};

template <int P, int CIN, int KS, int TY, int NBC, int NW>
__global__ __launch_bounds__(NW * 64) void head_taps(JobSet js, ConvParams prm) {
  using C = CfgTaps<P, CIN, KS, TY, NBC, NW>;
  static_assert(P == F32 || P == BF16, "FP32 or keyed BF16 input activations (NHWC)");
  __shared__ __attribute__((aligned(16))) float E[16 * C::PS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  constexpr int ELB = CIN * PT<P>::BYTES;
  Frag<P> wf[C::NK];
#pragma unroll
  for (int t = 0; t < C::NK; ++t) {
    const gbyte* p = gin(prm.wpack) + ((size_t)t * 64 + lane) * 16;
    load_frag<P>(wf[t], p, p);
  }
  const float bd = ldf(prm.bias, 1) - ldf(prm.bias, 0);

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    // item order and phase decomposition as conv_phase
    const int d = max(J.geom & 0xff, 1);
    const int tpy = J.tiles_y / (d * d);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int ph = (int)(t2 % (d * d));
    const int64_t t3 = t2 / (d * d);
    const int by = (int)(t3 % tpy);
    const int zz = (int)(t3 / tpy);
    const int py = ph / d, px = ph % d;
    const int y0 = by * TY, x0 = bx * C::TX;
    const FragTile ft = frag_tile(gin(J.in) + (int64_t)zz * J.in_zs * ELB, ELB, J, py, px);
    __syncthreads();  // every thread is done reading the previous item's planes
    // ---- D = X Wd, m-blocks round-robin over the waves, UB loaded at once
    for (int mb0 = wave; mb0 < C::MB; mb0 += NW * C::UB) {
      i4v q[C::UB][C::NK][4];
#pragma unroll
      for (int u = 0; u < C::UB; ++u) {
        const int mb = mb0 + u * NW;
        if (mb < C::MB) {
          const int rr = mb / NBC, cc = (mb % NBC) * 16 + n16;
          const gbyte* p = ft.at(y0 + rr, x0 + cc, ELB) + g * 16;
#pragma unroll
          for (int t = 0; t < C::NK; ++t) {
            q[u][t][0] = ld<i4v>(p + t * 64);
            q[u][t][1] = ld<i4v>(p + t * 64 + ft.o01);
            q[u][t][2] = ld<i4v>(p + t * 64 + ft.o10);
            q[u][t][3] = ld<i4v>(p + t * 64 + ft.o11);
          }
        }
      }
#pragma unroll
      for (int u = 0; u < C::UB; ++u) {
        const int mb = mb0 + u * NW;
        if (mb < C::MB) {
          f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int t = 0; t < C::NK; ++t) {
            i4v m = chunk_max_signed<P>(chunk_max_signed<P>(q[u][t][0], q[u][t][1]),
                                        chunk_max_signed<P>(q[u][t][2], q[u][t][3]));
            if constexpr (P == BF16) {
#pragma unroll
              for (int w = 0; w < 4; ++w) m[w] = (int)bf16_unkey((uint32_t)m[w]);
            }
            Frag<P> a;
            if constexpr (P == BF16) a.v = __builtin_bit_cast(bf16x8, m);
            else a.v = __builtin_bit_cast(f4, m);
            mma<P>(acc, a, wf[t]);
          }
          const int rr = mb / NBC;
          // lane (n16, g) holds taps n16 of pixels 4g .. 4g + 3 of the m-block
          *reinterpret_cast<f4*>(&E[n16 * C::PS + rr * C::LCP + (mb % NBC) * 16 + 4 * g]) = acc;
        }
      }
    }
    __syncthreads();
    // ---- tap sums, one output pixel per thread and pass
    const int lgo = (J.geom >> 16) & 0xf;
    for (int o = tid; o < TY * C::TX; o += C::THREADS) {
      const int r = o / C::TX, c = o % C::TX;
      float z = 0.f;
#pragma unroll
      for (int i = 0; i < KS; ++i)
#pragma unroll
        for (int j = 0; j < KS; ++j) z += E[(i * KS + j) * C::PS + (r + i) * C::LCP + c + j];
      const int y = py + d * (y0 + r), x = px + d * (x0 + c);
      if (y < J.hout && x < J.wout)
        st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * 4,
                  sigmoid_f(z + bd));
    }
  }
}

// head_taps over phase groups. The 2x2 max filter before a conv at spacing d
// has spacing h = d / 2, so the filters of the four phases (gy + a h, gx + b h),
// a, b in {0, 1}, read the same four fragments F[a][b] (fragment of phase
// (gy + a h, gx + b h)): operand pixel (R, C) of member (a, b) is the max of
// F[a ^ a'][b ^ b'][R + (a & a')][C + (b & b')] over a', b'. One work item is
// a group's tile: each lane loads the nine distinct (fragment, shift) chunks
// of its pixel once (against sixteen for four separate phase tiles, and the
// shifted ones mostly hit lines the same wave just brought into the L1), forms
// all four members' operand pixels and runs four MFMAs. The members' D stay in
// registers; their tap sums then pass through the LDS planes one member at a
// time. Needs a max filter at h = d / 2 >= 1 (the host offers it only then).
template <int P, int CIN, int KS, int TY, int NBC, int NW>
struct CfgTaps4 : CfgTaps<P, CIN, KS, TY, NBC, NW> {
  using B = CfgTaps<P, CIN, KS, TY, NBC, NW>;
  static_assert(B::MB % NW == 0, "m-blocks split evenly over the waves");
  static constexpr int MBW = B::MB / NW;  // m-blocks of a wave
  static constexpr bool PF = P == BF16;   // prefetch the next m-block's chunks
};

template <int P, int CIN, int KS, int TY, int NBC, int NW>
__global__ __launch_bounds__(NW * 64) void head_taps4(JobSet js, ConvParams prm) {
  using C = CfgTaps4<P, CIN, KS, TY, NBC, NW>;
  static_assert(P == F32 || P == BF16, "FP32 or keyed BF16 input activations (NHWC)");
  __shared__ __attribute__((aligned(16))) float E[16 * C::PS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, n16 = lane & 15;
  constexpr int ELB = CIN * PT<P>::BYTES;
  Frag<P> wf[C::NK];
#pragma unroll
  for (int t = 0; t < C::NK; ++t) {
    const gbyte* p = gin(prm.wpack) + ((size_t)t * 64 + lane) * 16;
    load_frag<P>(wf[t], p, p);
  }
  const float bd = ldf(prm.bias, 1) - ldf(prm.bias, 0);

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    // item order: tile column, then phase group, then tile row, then slice
    const int d = J.geom & 0xff, h = d >> 1, lg = __builtin_ctz(d);
    const int tpy = J.tiles_y / (h * h);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int grp = (int)(t2 % (h * h));
    const int64_t t3 = t2 / (h * h);
    const int by = (int)(t3 % tpy);
    const int zz = (int)(t3 / tpy);
    const int gy = grp / h, gx = grp % h;
    const int y0 = by * TY, x0 = bx * C::TX;
    const int64_t plane = (J.in_zs >> (2 * lg)) * ELB;  // bytes per fragment
    const int64_t rowb = J.in_rs * ELB;
    const gbyte* f00 = gin(J.in) + (int64_t)zz * J.in_zs * ELB + (int64_t)(gy * d + gx) * plane;
    const int64_t o01 = h * plane, o10 = (int64_t)h * d * plane;  // fragments (gy, gx + h), (gy + h, gx)
    // last valid row / column of the fragments with fy = gy (A) or gy + h (B), fx = gx or gx + h
    const int rvA = (J.hin - 1 - gy) >> lg, rvB = (J.hin - 1 - gy - h) >> lg;
    const int cvA = (J.win - 1 - gx) >> lg, cvB = (J.win - 1 - gx - h) >> lg;

    // the nine chunks of m-block k (of this wave) per MFMA step
    auto load_mb = [&](int k, i4v (&q)[C::NK][9]) __attribute__((always_inline)) {
      const int mb = wave + k * NW;
      const int R = y0 + mb / NBC, Cc = x0 + (mb % NBC) * 16 + n16;
      const int rA = min(R, rvA), rB = min(R, rvB), rA1 = min(R + 1, rvA);
      const int cA = min(Cc, cvA), cB = min(Cc, cvB), cA1 = min(Cc + 1, cvA);
#pragma unroll
      for (int t = 0; t < C::NK; ++t) {
        const gbyte* b = f00 + g * 16 + t * 64;
        q[t][0] = ld<i4v>(b + rA * rowb + cA * ELB);              // F00[R][C]
        q[t][1] = ld<i4v>(b + o01 + rA * rowb + cB * ELB);        // F01[R][C]
        q[t][2] = ld<i4v>(b + o10 + rB * rowb + cA * ELB);        // F10[R][C]
        q[t][3] = ld<i4v>(b + o10 + o01 + rB * rowb + cB * ELB);  // F11[R][C]
        q[t][4] = ld<i4v>(b + rA * rowb + cA1 * ELB);             // F00[R][C+1]
        q[t][5] = ld<i4v>(b + o10 + rB * rowb + cA1 * ELB);       // F10[R][C+1]
        q[t][6] = ld<i4v>(b + rA1 * rowb + cA * ELB);             // F00[R+1][C]
        q[t][7] = ld<i4v>(b + o01 + rA1 * rowb + cB * ELB);       // F01[R+1][C]
        q[t][8] = ld<i4v>(b + rA1 * rowb + cA1 * ELB);            // F00[R+1][C+1]
      }
    };
    f4 dacc[C::MBW][4];
    auto mma_mb = [&](int k, const i4v (&q)[C::NK][9]) __attribute__((always_inline)) {
#pragma unroll
      for (int m = 0; m < 4; ++m) dacc[k][m] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < C::NK; ++t) {
        const i4v* v = q[t];
        i4v op[4];
        op[0] = chunk_max_signed<P>(chunk_max_signed<P>(v[0], v[1]), chunk_max_signed<P>(v[2], v[3]));  // (0, 0)
        op[1] = chunk_max_signed<P>(chunk_max_signed<P>(v[1], v[4]), chunk_max_signed<P>(v[3], v[5]));  // (0, 1)
        op[2] = chunk_max_signed<P>(chunk_max_signed<P>(v[2], v[3]), chunk_max_signed<P>(v[6], v[7]));  // (1, 0)
        op[3] = chunk_max_signed<P>(chunk_max_signed<P>(v[3], v[5]), chunk_max_signed<P>(v[7], v[8]));  // (1, 1)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if constexpr (P == BF16) {
#pragma unroll
            for (int w = 0; w < 4; ++w) op[m][w] = (int)bf16_unkey((uint32_t)op[m][w]);
          }
          Frag<P> a;
          if constexpr (P == BF16) a.v = __builtin_bit_cast(bf16x8, op[m]);
          else a.v = __builtin_bit_cast(f4, op[m]);
          mma<P>(dacc[k][m], a, wf[t]);
        }
      }
    };
    // BF16: the loads of m-block k + 1 are issued before the work of m-block
    // k; FP32 (twice the chunks) one m-block at a time
    if constexpr (C::PF) {
      i4v qa[C::NK][9], qb[C::NK][9];
      load_mb(0, qa);
#pragma unroll
      for (int k = 0; k < C::MBW; k += 2) {
        if (k + 1 < C::MBW) load_mb(k + 1, qb);
        __builtin_amdgcn_sched_barrier(0);
        mma_mb(k, qa);
        if (k + 1 < C::MBW) {
          if (k + 2 < C::MBW) load_mb(k + 2, qa);
          __builtin_amdgcn_sched_barrier(0);
          mma_mb(k + 1, qb);
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < C::MBW; ++k) {
        i4v q[C::NK][9];
        load_mb(k, q);
        mma_mb(k, q);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
    const int lgo = (J.geom >> 16) & 0xf;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      __syncthreads();  // the previous member's (or item's) tap sums are done
#pragma unroll
      for (int k = 0; k < C::MBW; ++k) {
        const int mb = wave + k * NW;
        // lane (n16, g) holds taps n16 of pixels 4g .. 4g + 3 of the m-block
        *reinterpret_cast<f4*>(&E[n16 * C::PS + (mb / NBC) * C::LCP + (mb % NBC) * 16 + 4 * g]) = dacc[k][m];
      }
      __syncthreads();
      const int py = gy + (m >> 1) * h, px = gx + (m & 1) * h;
      for (int o = tid; o < TY * C::TX; o += C::THREADS) {
        const int r = o / C::TX, c = o % C::TX;
        float z = 0.f;
#pragma unroll
        for (int i = 0; i < KS; ++i)
#pragma unroll
          for (int j = 0; j < KS; ++j) z += E[(i * KS + j) * C::PS + (r + i) * C::LCP + c + j];
        const int y = py + d * (y0 + r), x = px + d * (x0 + c);
        if (y < J.hout && x < J.wout)
          st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * 4,
                    sigmoid_f(z + bd));
      }
    }
  }
}

// head_taps4 without LDS: one wave walks a vertical strip of a phase group,
// TY output rows x 13 columns of each of the four members. At operand row R
// it computes, for pixels C .. C + 15 (lane n16: pixel C + n16), each member's
// D^T = Wd^T X^T in the transposed MFMA form: lane (g, n16) holds taps
// (i = g, j = 0 .. 3) of pixel n16. Three DPP row shifts sum j into lane
// n16's output column (pixels n16 + j; columns 13 .. 15 lack their right
// neighbours and are not stored), leaving row i = g's share of output row
// R - g. Output row r accumulates in lane group r mod 4, so one ds_bpermute
// routes each share to its row; after row R, output row R - 3 is complete
// and its lane group stores it. The chunks of the first two fragments at row
// R + 1 (loaded for the members one phase row down) are carried to the next
// row, so a row costs six new chunk loads per MFMA step.
template <int P, int CIN, int KS, int TY>
__global__ __launch_bounds__(64) void head_strip(JobSet js, ConvParams prm) {
  static_assert(P == F32 || P == BF16, "FP32 or keyed BF16 input activations (NHWC)");
  static_assert(KS == 4, "sixteen taps: one MFMA tile, four per lane");
  constexpr int NK = CIN * PT<P>::BYTES / 64;  // MFMA steps (16-byte chunks per lane group)
  static_assert(NK * 64 == CIN * PT<P>::BYTES, "whole 16-byte chunks per lane group");
  constexpr int TXS = 16 - KS + 1;             // output columns of a strip
  constexpr int NS = TY + KS - 1;              // operand rows of a strip
  constexpr int ELB = CIN * PT<P>::BYTES;
  const int lane = threadIdx.x, g = lane >> 4, n16 = lane & 15;
  Frag<P> wf[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    const gbyte* p = gin(prm.wpack) + ((size_t)t * 64 + lane) * 16;
    load_frag<P>(wf[t], p, p);
  }
  const float bd = ldf(prm.bias, 1) - ldf(prm.bias, 0);

  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    // item order: strip column, then phase group, then strip row, then slice
    const int d = J.geom & 0xff, h = d >> 1, lg = __builtin_ctz(d);
    const int tpy = J.tiles_y / (h * h);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int grp = (int)(t2 % (h * h));
    const int64_t t3 = t2 / (h * h);
    const int by = (int)(t3 % tpy);
    const int zz = (int)(t3 / tpy);
    const int gy = grp / h, gx = grp % h;
    const int y0 = by * TY, x0 = bx * TXS;
    const int64_t plane = (J.in_zs >> (2 * lg)) * ELB;  // bytes per fragment
    const int64_t rowb = J.in_rs * ELB;
    const int64_t o01 = h * plane;  // fragment (gy, gx + h) from (gy, gx); (gy + h, .) at o10
    const gbyte* bA = gin(J.in) + (int64_t)zz * J.in_zs * ELB + (int64_t)(gy * d + gx) * plane + g * 16;
    const gbyte* bB = bA + (int64_t)h * d * plane;
    // last valid row / column of the fragments with fy = gy (A) or gy + h (B), fx = gx or gx + h
    const int rvA = (J.hin - 1 - gy) >> lg, rvB = (J.hin - 1 - gy - h) >> lg;
    const int cvA = (J.win - 1 - gx) >> lg, cvB = (J.win - 1 - gx - h) >> lg;
    const int Cc = x0 + n16;
    const int64_t xA = (int64_t)min(Cc, cvA) * ELB, xB = (int64_t)min(Cc, cvB) * ELB;
    const int64_t xA1 = (int64_t)min(Cc + 1, cvA) * ELB;
    // new chunks of operand row R: F10[R][C], F11[R][C], F10[R][C+1], F00[R+1][C], F01[R+1][C], F00[R+1][C+1]
    auto load_row = [&](int R, i4v (&q)[NK][6]) __attribute__((always_inline)) {
      const int64_t ra1 = (int64_t)min(R + 1, rvA) * rowb, rb = (int64_t)min(R, rvB) * rowb;
#pragma unroll
      for (int t = 0; t < NK; ++t) {
        q[t][0] = ld<i4v>(bB + rb + xA + t * 64);
        q[t][1] = ld<i4v>(bB + o01 + rb + xB + t * 64);
        q[t][2] = ld<i4v>(bB + rb + xA1 + t * 64);
        q[t][3] = ld<i4v>(bA + ra1 + xA + t * 64);
        q[t][4] = ld<i4v>(bA + o01 + ra1 + xB + t * 64);
        q[t][5] = ld<i4v>(bA + ra1 + xA1 + t * 64);
      }
    };
    // carried chunks of row R of fragments F00, F01: F00[R][C], F01[R][C], F00[R][C+1]
    i4v cr[NK][3];
    {
      const int64_t ra = (int64_t)min(y0, rvA) * rowb;
#pragma unroll
      for (int t = 0; t < NK; ++t) {
        cr[t][0] = ld<i4v>(bA + ra + xA + t * 64);
        cr[t][1] = ld<i4v>(bA + o01 + ra + xB + t * 64);
        cr[t][2] = ld<i4v>(bA + ra + xA1 + t * 64);
      }
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};  // output row (strip row) = lane group mod 4, per member
    const int lgo = (J.geom >> 16) & 0xf;
    auto row = [&](int s, const i4v (&q)[NK][6]) __attribute__((always_inline)) {
      f4 dm[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) dm[m] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int t = 0; t < NK; ++t) {
        // v[0..8] as in head_taps4: F00, F01, F10, F11 at (R, C); F00, F10 at C + 1;
        // F00, F01 at R + 1; F00 at (R + 1, C + 1)
        const i4v v0 = cr[t][0], v1 = cr[t][1], v2 = q[t][0], v3 = q[t][1], v4 = cr[t][2], v5 = q[t][2];
        const i4v v6 = q[t][3], v7 = q[t][4], v8 = q[t][5];
        i4v op[4];
        op[0] = chunk_max_signed<P>(chunk_max_signed<P>(v0, v1), chunk_max_signed<P>(v2, v3));  // (0, 0)
        op[1] = chunk_max_signed<P>(chunk_max_signed<P>(v1, v4), chunk_max_signed<P>(v3, v5));  // (0, 1)
        op[2] = chunk_max_signed<P>(chunk_max_signed<P>(v2, v3), chunk_max_signed<P>(v6, v7));  // (1, 0)
        op[3] = chunk_max_signed<P>(chunk_max_signed<P>(v3, v5), chunk_max_signed<P>(v7, v8));  // (1, 1)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if constexpr (P == BF16) {
#pragma unroll
            for (int w = 0; w < 4; ++w) op[m][w] = (int)bf16_unkey((uint32_t)op[m][w]);
          }
          Frag<P> a;
          if constexpr (P == BF16) a.v = __builtin_bit_cast(bf16x8, op[m]);
          else a.v = __builtin_bit_cast(f4, op[m]);
          mma<P>(dm[m], wf[t], a);  // weights as A: lane (g, n16) gets taps 4g .. 4g + 3 of pixel n16
        }
        cr[t][0] = v6;
        cr[t][1] = v7;
        cr[t][2] = v8;
      }
      const int src = ((((s - g) & 3) << 4) + n16) << 2;  // lane holding row s - (row of this group)'s share
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const float sh = dm[m][0] + dpp_f<0x101>(dm[m][1]) + dpp_f<0x102>(dm[m][2]) + dpp_f<0x103>(dm[m][3]);
        acc[m] += __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(src, __builtin_bit_cast(int, sh)));
      }
      if (g == ((s + 1) & 3)) {  // this lane group holds output row s - 3, now complete
        if (s >= KS - 1 && n16 < TXS) {
          const int r = y0 + s - (KS - 1), x_ = x0 + n16;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            const int y = gy + (m >> 1) * h + d * r, x = gx + (m & 1) * h + d * x_;
            if (y < J.hout && x < J.wout)
              st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * 4,
                        sigmoid_f(acc[m] + bd));
          }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) acc[m] = 0.f;
      }
    };
    i4v qa[NK][6], qb[NK][6];
    load_row(y0, qa);
#pragma unroll 1
    for (int s = 0; s < NS; s += 2) {
      if (s + 1 < NS) load_row(y0 + s + 1, qb);
      row(s, qa);
      if (s + 1 < NS) {
        if (s + 2 < NS) load_row(y0 + s + 2, qa);
        row(s + 1, qb);
      }
    }
  }
}

// A 1x1 conv to NCLS classes with a softmax, keeping class 0's probability:
// the output layer of a multi-class net (MaskExtend), on the VALU, one output
// pixel per thread. Input: row-major NHWC FP32 maps of CIN channels, read as
// 16-byte chunks; weights [class][CIN] and biases read with scalar loads.
// The softmax subtracts the largest logit before exponentiating.
template <int CIN, int NCLS, int TX>
__global__ __launch_bounds__(TX) void head_1x1(JobSet js, ConvParams prm) {
  static_assert(CIN % 4 == 0 && NCLS >= 2 && NCLS <= 4, "4-channel chunks, 2 to 4 classes");
  const __attribute__((address_space(4))) float* wk = (const __attribute__((address_space(4))) float*)prm.wpack;
  const __attribute__((address_space(4))) float* bk = (const __attribute__((address_space(4))) float*)prm.bias;
  const ItemRange rg = item_range(js.total_items);
  int cur = 0;
  if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  for (int64_t item = rg.begin; item < rg.end; item += rg.step) {
    const LayerJob J = job_at(js, cur, item);
    if (gated_off(J)) continue;
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int y = (int)(t2 % J.tiles_y);
    const int zz = (int)(t2 / J.tiles_y);
    const int x = bx * TX + (int)threadIdx.x;
    if (x >= J.wout) continue;
    const gbyte* px = gin(J.in) + ((int64_t)zz * J.in_zs + (int64_t)y * J.in_rs + x) * (CIN * 4);
    float z[NCLS];
#pragma unroll
    for (int k = 0; k < NCLS; ++k) z[k] = bk[k];
#pragma unroll
    for (int c = 0; c < CIN / 4; ++c) {
      const f4 v = ld<f4>(px + c * 16);
#pragma unroll
      for (int k = 0; k < NCLS; ++k)
#pragma unroll
        for (int e = 0; e < 4; ++e) z[k] = fmaf(v[e], wk[k * CIN + 4 * c + e], z[k]);
    }
    float m = z[0];
#pragma unroll
    for (int k = 1; k < NCLS; ++k) m = fmaxf(m, z[k]);
    float den = 0.f;
#pragma unroll
    for (int k = 0; k < NCLS; ++k) den += expf(z[k] - m);
    st<float>(gout(J.out) + ((int64_t)zz * J.out_zs + (int64_t)y * J.out_rs + x) * 4, expf(z[0] - m) / den);
  }
}

// ---------------------------------------------------------------- pipelined MFMA conv (BF16 / FP8)

// BF16 and FP8 activations are channel-blocked: element (z, y, x, c) of a
// C-channel tensor lives at z*zs*C + (c/16)*zs*16 + (y*rs + x)*16 + c%16
// (elements; rs, zs in pixels). A 16-channel plane pixel is 32 B (BF16) or
// 16 B (FP8), so a stage of 16 channels reads whole contiguous rows, and the
// epilogue writes each (m-block, n-block) as one 512 B / 256 B run.
//
// conv_ws is warp-specialised. NCW consumer waves run the implicit GEMM of
// conv_mfma with both operands in LDS; NPW producer waves fill the LDS. A
// stage is (tile, channel block): its operand tile (max filter applied) and,
// for BF16 layers whose packed weights do not fit in LDS next to two operand
// buffers, its weight slice. Weights that fit are copied to LDS once per
// workgroup; FP8 consumers of layers whose weights do not fit read them
// through the L1. Stages are double-buffered with one workgroup barrier per stage,
// and the producers issue the global loads of stage k+1 before that barrier,
// so the load latency overlaps a whole stage of MFMA work.

// NMEM > 1 (grouped spaced form): the operand tiles of NMEM phases stacked
// row-wise in one buffer, and the tile's m-blocks NMEM times TY x TX / 16.
template <int P, int CIN, int COUT, int KS, int TY, int TX, int NCW, int NPW, int K1 = 0, int NMEM = 1>
struct CfgWS {
  using T = PT<P>;
  static constexpr int KSZ = KS;
  // channels per stage: 16 (one plane) for BF16; all of CIN for FP8, whose
  // 128-deep MFMA needs the longer K of a stage to stay filled
  static constexpr int CB = P == FP8 ? CIN : 16;
  static_assert(CIN % 16 == 0 && CIN % CB == 0, "channels must be whole planes");
  static constexpr int NCB = CIN / CB;       // stages per tile
  static constexpr int NCHB = CB / T::CHB;   // 16-byte chunks per operand pixel
  static constexpr int NCHK = KS * KS * NCHB;
  static constexpr int SLOTS = 4 * T::U;
  static constexpr int NGS = (NCHK + SLOTS - 1) / SLOTS;
  static constexpr int NB = COUT / 16;
  static_assert(NB * 16 == COUT, "COUT must be a multiple of 16");
  static constexpr int LR = TY + KS - 1, LC = TX + KS - 1;
  // BF16: pixel stride = 8 (mod 16) dwords; with the chunk-slot order below
  // the two lane groups of a half-wave read chunks 16 B apart, which is
  // conflict-free. FP8: the 48 data bytes unpadded (12 dwords), which leaves
  // room for all packed weights of the 5x5 conv next to the two operand
  // buffers; with a 96-B stride they did not fit, and B fragments through the
  // L1 kept the texture addresser ~80 % busy (6 % slower conv2 despite fewer
  // LDS bank conflicts)
  static constexpr int PSB = P == FP8 ? CB * T::BYTES : pad_words(CB * T::BYTES / 4) * 4;
  // Row-quad K order (k_slot) where a pixel's chunks are unpadded and it takes
  // no more group-steps than the flattened order: each lane then reads at a
  // fixed offset from a uniform per-slot address (FP8 5x5: 15 chunks a filter
  // row, 16 slots a row, the same 80 slots as flattened).
  // group-steps per unrolled body of the consumer loop
  static constexpr int KUNROLL = P == FP8 ? 1 : 2;
  static constexpr bool ROWK = PSB == NCHB * 16 && KS * NCHB >= 4 &&
                               KS * rowq_quads(KS, NCHB) * 4 <= NGS * SLOTS;
  static constexpr int BUF = NMEM * LR * LC * PSB;         // one operand buffer
  static constexpr int WB = NGS * NB * 64 * T::U * 16;     // packed weights of one stage
  static constexpr int LDS_MAX = 160 * 1024;
  // BF16 consumers read B fragments from LDS: resident for the workgroup's
  // lifetime when all packed weights fit next to the two operand buffers,
  // else one slice per stage, staged by the producers. FP8 consumers read B
  // from LDS when all weights are resident, else through the L1 (with a
  // register prefetch ring).
  static constexpr bool FITS = 2 * BUF + NCB * WB <= LDS_MAX;
  static constexpr bool BL = P != FP8 || FITS;
  static constexpr bool WRES = BL && FITS;  // all weights resident in LDS
  static constexpr int WOFF = 2 * BUF;
  static constexpr int WLDS = !BL ? 0 : WRES ? NCB * WB : 2 * WB;
  // Fused first layer (K1 > 0): producer wave w builds operand rows
  // [w*RPW, (w+1)*RPW) from RPW + 1 first-layer output rows, computed in
  // m-blocks of 16 pixels at a column stride of 15 (a block yields 15
  // max-filtered columns), from its own uint8 rows in LDS.
  static constexpr int RPW = (LR + NPW - 1) / NPW;
  static constexpr int NMC = (LC + 14) / 15;
  static constexpr int U8R = RPW + K1;
  static constexpr int U8C = (15 * NMC + K1 + 3) / 4 * 4;
  static constexpr int U8W = K1 ? U8R * U8C : 0;  // uint8 bytes per producer wave
  static constexpr int U8PL = (U8W + 63) / 64;    // per lane
  static constexpr int U8OFF = WOFF + WLDS;
  static constexpr int LDS = U8OFF + NPW * U8W;
  static constexpr int MBLK = NMEM * TY * TX / 16;
  static_assert(TX % 16 == 0, "TX must be a multiple of 16");
  static_assert(MBLK % NCW == 0, "m-blocks must split evenly over consumer waves");
  static constexpr int MW = MBLK / NCW;
  static_assert(MW % (TX / 16) == 0, "each consumer wave owns whole tile rows");
  static constexpr int WROWS = MW / (TX / 16);  // tile rows per consumer wave
  static_assert(NMEM == 1 || TY % WROWS == 0, "a consumer wave's rows lie in one member's tile");
  static constexpr int THREADS = (NCW + NPW) * 64;
  static_assert(THREADS <= 1024, "workgroup size limit");
  static_assert(LDS <= LDS_MAX, "LDS budget of a gfx950 workgroup");
  static_assert(K1 == 0 || K1 * K1 <= 32, "fused first layer: one 16x16x32 MFMA per block");
};

// LDS offset, from the lane's pixel, of the chunk that lane group g reads for
// operand chunk uu of group-step s (slot 4U s + 4 uu + g, see k_slot). Row
// quads: a uniform offset plus 16 g bytes; the caller adds the 16 g (the
// lane's base carries it), so the offset is the same for every lane.
template <class C>
__device__ __forceinline__ int slot_off(int s, int uu, int g) {
  const int c = s * (4 * C::T::U) + 4 * uu + (C::ROWK ? 0 : g);
  const KSlot k = k_slot(c, C::KSZ, C::NCHB, C::ROWK);
  return (k.i * C::LC + k.j) * C::PSB + k.cg * 16;
}

// Output fields of a job that a conv_ws epilogue needs after the tile walk
// has moved on to the next item.
struct EpiJob {
  void* out;
  int64_t out_rs, out_zs;
  int32_t hout, wout;
};

// Walk of the work items of one workgroup (see item_range), skipping items
// of gated-off jobs. Every wave of the workgroup walks the same sequence.
struct TileWalk {
  int64_t item, end, step;
  int cur;
  LayerJob J;
  __device__ void init(const JobSet& js, const ItemRange& rg) {
    item = rg.begin - rg.step;
    end = rg.end;
    step = rg.step;
    cur = 0;
    if (js.table && rg.begin < rg.end) cur = find_job(js.table, js.njobs, rg.begin);
  }
  __device__ bool next(const JobSet& js) {
    for (item += step; item < end; item += step) {
      J = job_at(js, cur, item);
      if (gated_off(J)) continue;
      return true;
    }
    return false;
  }
  // tile origin and slice of the current item
  template <int TY, int TX>
  __device__ void coords(int& zz, int& y0, int& x0) const {
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    y0 = (int)(t2 % J.tiles_y) * TY;
    x0 = bx * TX;
    zz = (int)(t2 / J.tiles_y);
  }
  // items over groups of four phases (head_taps4's order: tile column, then
  // group, then tile row, then slice); the group's first phase (gy, gx), gy,
  // gx < d / 2; (y0, x0) in sub-lattice coordinates
  template <int TY, int TX>
  __device__ void group_coords(int& zz, int& gy, int& gx, int& y0, int& x0) const {
    const int h = (J.geom & 0xff) >> 1;
    const int tpy = J.tiles_y / (h * h);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int grp = (int)(t2 % (h * h));
    const int64_t t3 = t2 / (h * h);
    y0 = (int)(t3 % tpy) * TY;
    x0 = bx * TX;
    zz = (int)(t3 / tpy);
    gy = grp / h;
    gx = grp % h;
  }
  // phase-tiled items of a spaced conv (the order of conv_phase: tile column,
  // then phase, then tile row, then slice); (y0, x0) in sub-lattice coordinates
  template <int TY, int TX>
  __device__ void phase_coords(int& zz, int& py, int& px, int& y0, int& x0) const {
    const int d = max(J.geom & 0xff, 1);
    const int tpy = J.tiles_y / (d * d);
    const int64_t local = item - J.item0;
    const int bx = (int)(local % J.tiles_x);
    const int64_t t2 = local / J.tiles_x;
    const int ph = (int)(t2 % (d * d));
    const int64_t t3 = t2 / (d * d);
    y0 = (int)(t3 % tpy) * TY;
    x0 = bx * TX;
    zz = (int)(t3 / tpy);
    py = ph / d;
    px = ph % d;
  }
};

// One stage's operand tile held in producer registers between its global
// loads and its LDS writes. Chunk cg of an operand pixel holds channels
// c0 + cg*CHB .. +CHB-1, read from plane c / 16 at byte offset
// ((c % 16) / CHB) * 16 of the plane pixel. With POOL a thread item is a 2x2
// block of operand pixels of one chunk, loaded as its 3x3 stored
// neighbourhood (see stage_tile for the clamping); without it, one pixel.
template <int P, int LR, int LC, int NCHB, int PSB, int NPT, bool POOL>
struct AStage {
  using T = PT<P>;
  static constexpr int PB = 16 * T::BYTES;
  static constexpr int NST = POOL ? (LR / 2) * (LC / 2) * NCHB : LR * LC * NCHB;
  static constexpr int NIT = (NST + NPT - 1) / NPT;
  static constexpr int NL = POOL ? 9 : 1;
  i4v q[NIT][NL];

  __device__ __forceinline__ void load(const gbyte* slice, int64_t plane_b, int64_t rowb, int c0, int y0,
                                       int x0, int hp, int wp, int ptid) {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, it = t / NCHB;
        const int c = c0 + cg * T::CHB;
        const gbyte* base = slice + (c >> 4) * plane_b + ((c & 15) / T::CHB) * 16;
        if constexpr (POOL) {
          static_assert(LR % 2 == 0 && LC % 2 == 0, "2x2 staging blocks need even tile sides");
          const int r = 2 * (it / (LC / 2)), cc = 2 * (it % (LC / 2));
          int ys[3], xs[3];
          ys[0] = min(y0 + r, hp - 1);
          ys[1] = ys[0] + 1;
          ys[2] = min(y0 + r + 1, hp - 1) + 1;
          xs[0] = min(x0 + cc, wp - 1);
          xs[1] = xs[0] + 1;
          xs[2] = min(x0 + cc + 1, wp - 1) + 1;
#pragma unroll
          for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
              q[k][a * 3 + b] = ld<i4v>(base + (int64_t)ys[a] * rowb + (int64_t)xs[b] * PB);
        } else {
          const int r = it / LC, cc = it % LC;
          const int y = min(y0 + r, hp - 1), x = min(x0 + cc, wp - 1);
          q[k][0] = ld<i4v>(base + (int64_t)y * rowb + (int64_t)x * PB);
        }
      }
    }
  }

  __device__ __forceinline__ void store(unsigned char* lds, int ptid) const {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, it = t / NCHB;
        if constexpr (POOL) {
          const int r = 2 * (it / (LC / 2)), cc = 2 * (it % (LC / 2));
          i4v mo[4];
          if constexpr (P == FP8) {
            max_filter_fp8(q[k], mo);
          } else {
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
              for (int e = 0; e < 2; ++e)
                mo[2 * d + e] = chunk_max<P>(chunk_max<P>(q[k][d * 3 + e], q[k][d * 3 + e + 1]),
                                             chunk_max<P>(q[k][(d + 1) * 3 + e], q[k][(d + 1) * 3 + e + 1]));
          }
#pragma unroll
          for (int d = 0; d < 2; ++d)
#pragma unroll
            for (int e = 0; e < 2; ++e)
              *reinterpret_cast<i4v*>(lds + ((r + d) * LC + cc + e) * PSB + cg * 16) = mo[2 * d + e];
        } else {
          *reinterpret_cast<i4v*>(lds + it * PSB + cg * 16) = q[k][0];
        }
      }
    }
  }
};

// A contiguous block of BYTES bytes (packed weights) held in producer
// registers between its global loads and its LDS writes.
template <int BYTES, int NPT>
struct WStage {
  static constexpr int N = BYTES / 16;
  static_assert(N * 16 == BYTES, "whole 16-byte chunks");
  static constexpr int NIT = (N + NPT - 1) / NPT;
  i4v v[NIT];
  __device__ __forceinline__ void load(const gbyte* src, int ptid) {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < N) v[k] = ld<i4v>(src + (int64_t)t * 16);
    }
  }
  __device__ __forceinline__ void store(unsigned char* dst, int ptid) const {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < N) reinterpret_cast<i4v*>(dst)[t] = v[k];
    }
  }
};


// One stage's operand tile of a spaced conv (stride-2 pool nets) held in
// producer registers: operand pixel (r, c) is the 2x2 max filter addressed by
// f (frag_tile) over an NHWC map of keyed bf16 activations (elb bytes per
// pixel; cofs = byte offset of the stage's first channel). The max is taken on
// keys and the winner is stored to LDS as a bf16 operand.
template <int LR, int LC, int NCHB, int PSB, int NPT>
struct PhStage {
  static constexpr int NST = LR * LC * NCHB;
  static constexpr int NIT = (NST + NPT - 1) / NPT;
  i4v q[NIT][4];

  __device__ __forceinline__ void load(const FragTile& f, int cofs, int elb, int y0, int x0, int ptid) {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, pix = t / NCHB;
        const int r = pix / LC, c = pix % LC;
        const gbyte* p = f.at(y0 + r, x0 + c, elb) + cofs + cg * 16;
        q[k][0] = ld<i4v>(p);
        q[k][1] = ld<i4v>(p + f.o01);
        q[k][2] = ld<i4v>(p + f.o10);
        q[k][3] = ld<i4v>(p + f.o11);
      }
    }
  }

  __device__ __forceinline__ void store(unsigned char* lds, int ptid) const {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, pix = t / NCHB;
        i4v m = chunk_max<BF16>(chunk_max<BF16>(q[k][0], q[k][1]), chunk_max<BF16>(q[k][2], q[k][3]));
#pragma unroll
        for (int w = 0; w < 4; ++w) m[w] = (int)bf16_unkey((uint32_t)m[w]);
        *reinterpret_cast<i4v*>(lds + pix * PSB + cg * 16) = m;
      }
    }
  }
};

// One stage's operand tiles of the four phases of a group (PH = 2) held in
// producer registers: for operand position (R, C) and chunk cg, the nine
// distinct (fragment, shift) chunks that the four members' max filters read
// (see head_taps4). The store forms the members' operand pixels (max on keys,
// then bf16) and writes member m's tile at rows m LR .. m LR + LR - 1.
template <int LR, int LC, int NCHB, int PSB, int NPT>
struct GrpStage {
  static constexpr int NST = LR * LC * NCHB;
  static constexpr int NIT = (NST + NPT - 1) / NPT;
  i4v q[NIT][9];

  // f00: fragment (gy, gx) of the slice plus the stage's channel offset;
  // o01 / o10: offsets of fragments (gy, gx + h) / (gy + h, gx); rv / cv: last
  // valid row / column of the fragments at gy, gy + h / gx, gx + h
  __device__ __forceinline__ void load(const gbyte* f00, int64_t o01, int64_t o10, int64_t rowb, int elb, int rvA,
                                       int rvB, int cvA, int cvB, int y0, int x0, int ptid) {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, pix = t / NCHB;
        const int R = y0 + pix / LC, Cc = x0 + pix % LC;
        const int64_t rA = (int64_t)min(R, rvA) * rowb, rB = (int64_t)min(R, rvB) * rowb;
        const int64_t rA1 = (int64_t)min(R + 1, rvA) * rowb;
        const int64_t cA = (int64_t)min(Cc, cvA) * elb, cB = (int64_t)min(Cc, cvB) * elb;
        const int64_t cA1 = (int64_t)min(Cc + 1, cvA) * elb;
        const gbyte* b = f00 + cg * 16;
        q[k][0] = ld<i4v>(b + rA + cA);              // F00[R][C]
        q[k][1] = ld<i4v>(b + o01 + rA + cB);        // F01[R][C]
        q[k][2] = ld<i4v>(b + o10 + rB + cA);        // F10[R][C]
        q[k][3] = ld<i4v>(b + o10 + o01 + rB + cB);  // F11[R][C]
        q[k][4] = ld<i4v>(b + rA + cA1);             // F00[R][C+1]
        q[k][5] = ld<i4v>(b + o10 + rB + cA1);       // F10[R][C+1]
        q[k][6] = ld<i4v>(b + rA1 + cA);             // F00[R+1][C]
        q[k][7] = ld<i4v>(b + o01 + rA1 + cB);       // F01[R+1][C]
        q[k][8] = ld<i4v>(b + rA1 + cA1);            // F00[R+1][C+1]
      }
    }
  }

  __device__ __forceinline__ void store(unsigned char* lds, int ptid) const {
#pragma unroll
    for (int k = 0; k < NIT; ++k) {
      const int t = ptid + k * NPT;
      if (t < NST) {
        const int cg = t % NCHB, pix = t / NCHB;
        const i4v* v = q[k];
        i4v op[4];
        op[0] = chunk_max<BF16>(chunk_max<BF16>(v[0], v[1]), chunk_max<BF16>(v[2], v[3]));  // (0, 0)
        op[1] = chunk_max<BF16>(chunk_max<BF16>(v[1], v[4]), chunk_max<BF16>(v[3], v[5]));  // (0, 1)
        op[2] = chunk_max<BF16>(chunk_max<BF16>(v[2], v[3]), chunk_max<BF16>(v[6], v[7]));  // (1, 0)
        op[3] = chunk_max<BF16>(chunk_max<BF16>(v[3], v[5]), chunk_max<BF16>(v[7], v[8]));  // (1, 1)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
          for (int w = 0; w < 4; ++w) op[m][w] = (int)bf16_unkey((uint32_t)op[m][w]);
          *reinterpret_cast<i4v*>(lds + (m * LR * LC + pix) * PSB + cg * 16) = op[m];
        }
      }
    }
  }
};

// PH = 1: a spaced conv of a stride-2 pool net (the work of conv_phase with
// max-out, BF16): NHWC keyed input, operand pixels are the spaced 2x2 max
// filter, items are phase tiles, and the epilogue is bias + max-out over
// channel pairs, stored as NHWC keys.
template <int P, int CIN, int COUT, int KS, bool POOL, bool HEAD, int TY, int TX, int NCW, int NPW, int K1, int PH = 0>
__global__ __launch_bounds__((CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1, PH == 2 ? 4 : 1>::THREADS)) void conv_ws(
    JobSet js, ConvParams prm) {
  using C = CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1, PH == 2 ? 4 : 1>;
  static_assert(K1 == 0 || POOL, "the fused first layer feeds a max filter");
  using T = PT<P>;
  static_assert(P != F32, "conv_ws reads and writes the channel-blocked BF16 / FP8 layout");
  static_assert(!PH || (P == BF16 && POOL && !HEAD && K1 == 0 && C::WRES),
                "spaced form: BF16 max-out conv with all weights resident in LDS");
  static_assert(PH != 2 || TX == 16, "grouped form: one m-block column per member tile");
  __shared__ __attribute__((aligned(16))) unsigned char lds[C::LDS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform role
  constexpr int MCOLS = TX / 16;
  constexpr int PB = 16 * T::BYTES;
  const gbyte* wglob = gin(prm.wpack);

  const ItemRange rg = item_range(js.total_items);
  TileWalk w;
  w.init(js, rg);
  if (!w.next(js)) return;  // no work for this workgroup (uniform)

  if constexpr (C::WRES) {
    // all packed weights to LDS once (every wave helps)
    WStage<C::NCB * C::WB, C::THREADS> wl;
    wl.load(wglob, tid);
    wl.store(lds + C::WOFF, tid);
  }

  if constexpr (K1 > 0) if (wave >= NCW) {
    // ---------------- producer waves, fused first layer
    const int pw = wave - NCW;
    const int g = lane >> 4, n16 = lane & 15;
    const int orow0 = pw * C::RPW;  // first operand row of this wave
    unsigned char* u8r = lds + C::U8OFF + pw * C::U8W;
    const gbyte* w1 = gin(prm.w1);
    // per-lane tap offsets in the uint8 rows: lane group g holds taps 8g..8g+7
    // (taps past K1*K1 read byte 0: their packed weights are zero)
    int toff[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int t = 8 * g + e;
      toff[e] = t < K1 * K1 ? (t / K1) * C::U8C + t % K1 : 0;
    }
    int ub[C::U8PL];
    WStage<C::WB, NPW * 64> ws;
    const int ptid = tid - NCW * 64;
    int cb = 0;
    // global loads of the stage's weight slice (BF16 weights that do not stay
    // resident) and, at a tile's first stage, of the uint8 rows orow0 ..
    // orow0 + U8R - 1 of the tile of w.item (clamped)
    auto issue = [&]() __attribute__((always_inline)) {
      if constexpr (C::BL && !C::WRES) ws.load(wglob + (size_t)cb * C::WB, ptid);
      if (cb != 0) return;
      int zz, y0, x0;
      w.coords<TY, TX>(zz, y0, x0);
      const gbyte* in = gin(w.J.in) + (int64_t)zz * w.J.in_zs;
#pragma unroll
      for (int q = 0; q < C::U8PL; ++q) {
        const int idx = q * 64 + lane;
        if (idx < C::U8W) {
          const int r = idx / C::U8C, c = idx % C::U8C;
          const int y = min(y0 + orow0 + r, w.J.hin - 1), x = min(x0 + c, w.J.win - 1);
          ub[q] = in[(int64_t)y * w.J.in_rs + x];
        }
      }
    };
    auto advance = [&]() __attribute__((always_inline)) -> bool {
      if (++cb < C::NCB) return true;
      cb = 0;
      return w.next(js);
    };
    // Operand rows of this wave for stage cb into buffer sel. The first layer
    // runs as D = W X on a 16x16x32 bf16 MFMA: A = weights (lane (g, c) holds
    // channel c's taps 8g..8g+7, the packed layout), B = the taps of 16
    // pixels, so lane (g, n) receives channels 4g..4g+3 of pixel n. The right
    // neighbour of pixel n is then lane n+1 of the same 16-lane row (one DPP
    // shift), and a lane's 4 channels are one 8-byte (BF16) / 4-byte (FP8)
    // operand store. The products are exact (uint8 times bf16), and the
    // outputs are max-filtered as floats and converted once: bf16 rounding
    // and e4m3 quantisation are monotone, so this equals filtering the stored
    // values of the unfused path.
    auto put = [&](int sel) __attribute__((always_inline)) {
      if constexpr (C::BL && !C::WRES) ws.store(lds + C::WOFF + sel * C::WB, ptid);
      if (cb == 0) {
#pragma unroll
        for (int q = 0; q < C::U8PL; ++q) {
          const int idx = q * 64 + lane;
          if (idx < C::U8W) u8r[idx] = (unsigned char)ub[q];
        }
      }
      unsigned char* obuf = lds + sel * C::BUF;
      constexpr int NB1 = C::CB / 16;  // first-layer n-blocks per stage
      bf16x8 wfr[NB1];
      float b4[NB1][4];
#pragma unroll
      for (int nb1 = 0; nb1 < NB1; ++nb1) {
        const int n1 = cb * NB1 + nb1;  // first-layer output channels 16 n1 .. 16 n1 + 15
        wfr[nb1] = ld<bf16x8>(w1 + ((int64_t)n1 * 64 + lane) * 16);
#pragma unroll
        for (int k = 0; k < 4; ++k) b4[nb1][k] = ldf(prm.b1, n1 * 16 + 4 * g + k);
      }
      for (int mc = 0; mc < C::NMC; ++mc) {
        // taps of pixel 15 mc + n for all RPW + 1 first-layer rows of this wave:
        // all byte loads are issued before any is used
        const unsigned char* a0 = u8r + 15 * mc + n16;
        unsigned int raw[C::RPW + 1][8];
#pragma unroll
        for (int rr = 0; rr <= C::RPW; ++rr)
#pragma unroll
          for (int e = 0; e < 8; ++e) raw[rr][e] = a0[rr * C::U8C + toff[e]];
        __builtin_amdgcn_sched_barrier(0);
        // uint8 -> bf16 is exact: the float of an integer below 256 has a zero low half
        bf16x8 xb[C::RPW + 1];
#pragma unroll
        for (int rr = 0; rr <= C::RPW; ++rr) {
          u4v pk;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            pk[e] = __builtin_amdgcn_perm(__builtin_bit_cast(unsigned int, (float)raw[rr][2 * e + 1]),
                                          __builtin_bit_cast(unsigned int, (float)raw[rr][2 * e]), 0x07060302u);
          xb[rr] = __builtin_bit_cast(bf16x8, pk);
        }
        const int col = 15 * mc + n16;
        const bool colok = (n16 != 15) && (col < C::LC);
#pragma unroll
        for (int nb1 = 0; nb1 < NB1; ++nb1) {
          float hprev[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int rr = 0; rr <= C::RPW; ++rr) {
            // started at the bias, as the separate first layer does
            const f4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                wfr[nb1], xb[rr], f4{b4[nb1][0], b4[nb1][1], b4[nb1][2], b4[nb1][3]}, 0, 0, 0);
            float h[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
              const float t = relu(acc[k]);
              // pixel n + 1 (lane n + 1 of the row; lane 15's value is never stored)
              const float r = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, t),
                                                                                    0x101, 0xF, 0xF, false));
              h[k] = fmaxf(t, r);
            }
            if (rr > 0) {
              const int orow = orow0 + rr - 1;
              if (colok && orow < C::LR) {
                unsigned char* dst = obuf + (orow * C::LC + col) * C::PSB + (nb1 * 16 + 4 * g) * T::BYTES;
                const float v0 = fmaxf(hprev[0], h[0]), v1 = fmaxf(hprev[1], h[1]);
                const float v2 = fmaxf(hprev[2], h[2]), v3 = fmaxf(hprev[3], h[3]);
                if constexpr (P == BF16) {
                  st<u2v>(dst, u2v{pack_bf16x2(v0, v1), pack_bf16x2(v2, v3)});
                } else {
                  const float inv = prm.w1_inv_scale;
                  st<uint32_t>(dst, pack_e4m3x2(v0 * inv, v1 * inv) | (pack_e4m3x2(v2 * inv, v3 * inv) << 16));
                }
              }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) hprev[k] = h[k];
          }
        }
      }
    };
    issue();
    put(0);
    bool more = advance();
    if (more) issue();
    __syncthreads();  // stage 0 ready
    int sel = 1;
    while (more) {
      put(sel);
      more = advance();
      if (more) issue();
      __syncthreads();  // this stage ready; the consumers finished the previous one
      sel ^= 1;
    }
    __syncthreads();  // the consumers' last stage
    return;
  }

  if constexpr (PH == 2) if (wave >= NCW) {
    // ---------------- producer waves, spaced max filter over a phase group
    const int ptid = tid - NCW * 64;
    constexpr int ELB = CIN * T::BYTES;  // bytes per stored input pixel (NHWC)
    GrpStage<C::LR, C::LC, C::NCHB, C::PSB, NPW * 64> a;
    int cb = 0;
    auto issue = [&]() __attribute__((always_inline)) {
      int zz, gy, gx, y0, x0;
      w.group_coords<TY, TX>(zz, gy, gx, y0, x0);
      const LayerJob& J = w.J;
      const int d = J.geom & 0xff, h = d >> 1, lg = __builtin_ctz(d);
      const int64_t plane = (J.in_zs >> (2 * lg)) * ELB;  // bytes per fragment
      const gbyte* f00 = gin(J.in) + (int64_t)zz * J.in_zs * ELB + (int64_t)(gy * d + gx) * plane +
                         cb * C::CB * T::BYTES;
      a.load(f00, h * plane, (int64_t)h * d * plane, J.in_rs * ELB, ELB, (J.hin - 1 - gy) >> lg,
             (J.hin - 1 - gy - h) >> lg, (J.win - 1 - gx) >> lg, (J.win - 1 - gx - h) >> lg, y0, x0, ptid);
    };
    auto advance = [&]() __attribute__((always_inline)) -> bool {
      if (++cb < C::NCB) return true;
      cb = 0;
      return w.next(js);
    };
    issue();
    a.store(lds, ptid);
    bool more = advance();
    if (more) issue();
    __syncthreads();  // stage 0 ready
    int sel = 1;
    while (more) {
      a.store(lds + sel * C::BUF, ptid);  // the consumers finished this buffer's previous stage
      more = advance();
      if (more) issue();
      __syncthreads();  // this stage ready; the consumers finished the previous one
      sel ^= 1;
    }
    __syncthreads();  // the consumers' last stage
    return;
  }

  if constexpr (PH == 1) if (wave >= NCW) {
    // ---------------- producer waves, spaced max filter
    const int ptid = tid - NCW * 64;
    constexpr int ELB = CIN * T::BYTES;  // bytes per stored input pixel (NHWC)
    PhStage<C::LR, C::LC, C::NCHB, C::PSB, NPW * 64> a;
    int cb = 0;
    auto issue = [&]() __attribute__((always_inline)) {
      int zz, py, px, y0, x0;
      w.phase_coords<TY, TX>(zz, py, px, y0, x0);
      const FragTile ft = frag_tile(gin(w.J.in) + (int64_t)zz * w.J.in_zs * ELB, ELB, w.J, py, px);
      a.load(ft, cb * C::CB * T::BYTES, ELB, y0, x0, ptid);
    };
    auto advance = [&]() __attribute__((always_inline)) -> bool {
      if (++cb < C::NCB) return true;
      cb = 0;
      return w.next(js);
    };
    issue();
    a.store(lds, ptid);
    bool more = advance();
    if (more) issue();
    __syncthreads();  // stage 0 ready
    int sel = 1;
    while (more) {
      a.store(lds + sel * C::BUF, ptid);  // the consumers finished this buffer's previous stage
      more = advance();
      if (more) issue();
      __syncthreads();  // this stage ready; the consumers finished the previous one
      sel ^= 1;
    }
    __syncthreads();  // the consumers' last stage
    return;
  }

  if constexpr (K1 == 0 && !PH) if (wave >= NCW) {
    // ---------------- producer waves
    const int ptid = tid - NCW * 64;
    AStage<P, C::LR, C::LC, C::NCHB, C::PSB, NPW * 64, POOL> a;
    WStage<C::WB, NPW * 64> ws;
    int cb = 0;
    // global loads of the stage (w.item, cb) into registers
    auto issue = [&]() __attribute__((always_inline)) {
      int zz, y0, x0;
      w.coords<TY, TX>(zz, y0, x0);
      const int hp = w.J.hin - (POOL ? 1 : 0), wp = w.J.win - (POOL ? 1 : 0);
      const gbyte* slice = gin(w.J.in) + (int64_t)zz * w.J.in_zs * CIN * T::BYTES;
      a.load(slice, w.J.in_zs * PB, w.J.in_rs * PB, cb * C::CB, y0, x0, hp, wp, ptid);
      if constexpr (C::BL && !C::WRES) ws.load(wglob + (size_t)cb * C::WB, ptid);
    };
    auto advance = [&]() __attribute__((always_inline)) -> bool {
      if (++cb < C::NCB) return true;
      cb = 0;
      return w.next(js);
    };
    auto put = [&](int sel) __attribute__((always_inline)) {
      a.store(lds + sel * C::BUF, ptid);
      if constexpr (C::BL && !C::WRES) ws.store(lds + C::WOFF + sel * C::WB, ptid);
    };
    issue();
    put(0);
    bool more = advance();
    if (more) issue();
    __syncthreads();  // stage 0 ready
    int sel = 1;
    while (more) {
      put(sel);  // the consumers finished this buffer's previous stage before the last barrier
      more = advance();
      if (more) issue();
      __syncthreads();  // this stage ready; the consumers finished the previous one
      sel ^= 1;
    }
    __syncthreads();  // the consumers' last stage
    return;
  }

  // ---------------- consumer waves: tile rows wave*WROWS .. +WROWS-1. The
  // m-block offsets inside a wave's rows are compile-time constants, so the
  // per-m-block LDS and global addresses are immediates on one lane base.
  const int g = lane >> 4, n16 = lane & 15;
  // the wave's first tile row; grouped form: member wmem's rows, stacked
  // after the LR operand rows of each earlier member in LDS
  const int wrow0 = PH == 2 ? (wave * C::WROWS) % TY : wave * C::WROWS;
  const int wmem = PH == 2 ? (wave * C::WROWS) / TY : 0;
  const int lrow0 = wmem * C::LR + wrow0;
  // TRANS: weights as the MFMA's A operand and pixels as B, so lane (g, n16)
  // accumulates channels 4g .. 4g + 3 of pixel n16 (4 consecutive channels:
  // stored ones, or two max-out pairs); otherwise (the fused head) channel n16
  // of pixels 4g .. 4g + 3
  constexpr bool TRANS = !HEAD;
  // Rolled K loop over the flattened order (FP8 3x3): the lane's LDS offsets
  // of every (step, chunk) slot, computed once and packed as 16-bit values
  // (two steps per register), so a step extracts its two offsets with a
  // select and a shift instead of redoing the divisions of slot_off.
  constexpr bool OTAB = !C::ROWK && C::KUNROLL == 1 && C::NGS <= 4 && C::BL;
  constexpr int OTW = OTAB ? (C::NGS + 1) / 2 : 1;
  uint32_t otab[T::U][OTW];
  if constexpr (OTAB) {
    static_assert(((C::KSZ - 1) * (C::LC + 1) + 1) * C::PSB <= 65535, "16-bit slot offsets");
#pragma unroll
    for (int uu = 0; uu < T::U; ++uu)
#pragma unroll
      for (int q = 0; q < OTW; ++q) {
        const uint32_t lo = (uint32_t)slot_off<C>(2 * q, uu, g);
        const uint32_t hi = 2 * q + 1 < C::NGS ? (uint32_t)slot_off<C>(2 * q + 1, uu, g) : 0u;
        otab[uu][q] = lo | (hi << 16);
      }
  }
  __syncthreads();  // the first stage is ready
  int cb = 0, sel = 0;
  f4 acc[C::MW][C::NB];
  // B fragments through the L1 (FP8): a two-step register ring. The loads of
  // step s + 1 are issued before the MFMAs of step s, and the last step of a
  // stage loads the first step of the next stage, so the L1 latency is hidden
  // behind a whole step (and across the stage barrier).
  constexpr int U16 = T::U * 16;
  Frag<P> bq[2][C::NB];
  auto load_b = [&](Frag<P>* dst, const gbyte* wl, int s) __attribute__((always_inline)) {
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) {
      const gbyte* p = wl + (s * C::NB + nb) * 64 * U16;
      load_frag<P>(dst[nb], p, p + 64 * 16);
    }
  };
  if constexpr (!C::BL) load_b(bq[0], wglob + lane * 16, 0);
  // Epilogue of the plain form straight from the accumulators, for the tile
  // at (zz, y0, x0) of the job whose output fields are in J.
  auto plain_epi = [&](const EpiJob& J, int zz, int y0, int x0) __attribute__((always_inline)) {
    float bias[C::NB], osc[C::NB], hw[C::NB];
#pragma unroll
    for (int nb = 0; nb < C::NB; ++nb) {
      bias[nb] = ldf(prm.bias, nb * 16 + n16);
      osc[nb] = prm.oscale ? ldf(prm.oscale, nb * 16 + n16) : 1.0f;
      hw[nb] = HEAD ? ldf(prm.head_w, nb * 16 + n16) : 0.f;
    }
    const int ty0 = y0 + wrow0;
    if constexpr (HEAD) {
      head_epilogue<C::MW, C::NB>(
          [&](int u, int nb, int k) __attribute__((always_inline)) { return acc[u][nb][k]; },
          [&](int u, int& y, int& xb) __attribute__((always_inline)) {
            y = ty0 + u / MCOLS;
            xb = x0 + (u % MCOLS) * 16;
          },
          bias, osc, hw, prm.head_b, g, n16, gout(J.out), (int64_t)zz * J.out_zs, J.out_rs, J.hout, J.wout);
    } else {
      // TRANS: a lane's 4 channels of an n-block are 4 (FP8) / 8 (BF16)
      // contiguous bytes of its pixel's entry in that 16-channel plane, and
      // an n-block's 64 lanes cover 16 pixels x 16 channels, one contiguous
      // run, stored straight from the accumulators
      static_assert(TRANS, "non-head epilogue of the plain form");
      f4 bs[C::NB], sc[C::NB];
#pragma unroll
      for (int nb = 0; nb < C::NB; ++nb) {
        bs[nb] = ld<f4>(gin(prm.bias) + (nb * 16 + 4 * g) * 4);
        sc[nb] = prm.oscale ? ld<f4>(gin(prm.oscale) + (nb * 16 + 4 * g) * 4) : f4{1.f, 1.f, 1.f, 1.f};
      }
      const float inv = prm.out_inv_scale;
      gbyte* const obase = gout(J.out) + (int64_t)zz * J.out_zs * COUT * T::BYTES + (int64_t)(4 * g) * T::BYTES;
#pragma unroll
      for (int u = 0; u < C::MW; ++u) {
        const int y = ty0 + u / MCOLS;
        const int x = x0 + (u % MCOLS) * 16 + n16;
        if (y < J.hout && x < J.wout) {
          gbyte* const d0 = obase + ((int64_t)y * J.out_rs + x) * PB;
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            gbyte* const d = d0 + (int64_t)nb * J.out_zs * PB;
            float t[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) t[k] = fmaf(acc[u][nb][k], sc[nb][k], bs[nb][k]);
            if constexpr (P == BF16) {
              st<u2v>(d, u2v{pack_bf16x2(relu(t[0]), relu(t[1])), pack_bf16x2(relu(t[2]), relu(t[3]))});
            } else {
              // relu(t) * s clamped to [0, 448] is the median of (t * s, 0, 448)
              // for s > 0; clearing bit 7 of each code maps a -0 to +0
              float v[4];
#pragma unroll
              for (int k = 0; k < 4; ++k) v[k] = __builtin_amdgcn_fmed3f(t[k] * inv, 0.0f, 448.0f);
              int wd = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], __builtin_bit_cast(int, v[0]), false);
              wd = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], wd, true);
              st<uint32_t>(d, (uint32_t)wd & 0x7f7f7f7fu);
            }
          }
        }
      }
    }
  };
  // The second half of the consumer waves (one per SIMD beside one of the
  // first half) defers a tile's epilogue to the start of the next stage: its
  // epilogue then overlaps the other wave's MFMAs instead of both waves of a
  // SIMD running theirs after the same barrier. The epilogue reads only
  // registers and global memory, so the delay needs no extra LDS buffer; the
  // accumulators are cleared after it. Measured on net B over 8 x 2048^2:
  // conv2 FP8 1.70 -> 1.63 ms, BF16 2.84 -> 2.78 ms; with the fused head
  // (conv3) slower (FP8 0.96 -> 1.03 ms, BF16 1.55 -> 1.65 ms), so not there.
  // The spaced form's epilogue measured no gain from the same delay; those
  // kernels and the fused head keep the loop without it.
  constexpr bool DEFER = !PH && !HEAD;
  const bool defer = DEFER && wave >= NCW / 2;
  bool pend = false, more = true;
  EpiJob pj{};
  int pz = 0, py0 = 0, px0 = 0;
  for (;;) {
    if constexpr (DEFER) {
      if (pend) {
        plain_epi(pj, pz, py0, px0);
        pend = false;
      }
      if (!more) break;
    }
    if (cb == 0) {
#pragma unroll
      for (int u = 0; u < C::MW; ++u)
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) acc[u][nb] = f4{0.f, 0.f, 0.f, 0.f};
    }
    const unsigned char* abase = lds + sel * C::BUF + (lrow0 * C::LC + n16) * C::PSB + (C::ROWK ? 16 * g : 0);
    // implicit GEMM over the stage's (tap, chunk) slots; B fragments from
    // LDS (BF16) or global memory (FP8)
    // FP8: not unrolled, so the accumulators stay in place (unrolled twice,
    // the allocator alternates them between two register sets, which spills
    // the 6-m-block shapes); BF16: unrolled twice, measured faster
    auto kloop = [&](auto wl) __attribute__((always_inline)) {
#pragma unroll C::KUNROLL
      for (int s = 0; s < C::NGS; ++s) {
        Frag<P> bfr[C::NB];
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) {
          const auto p = wl + (s * C::NB + nb) * 64 * (T::U * 16);
          load_frag<P>(bfr[nb], p, p + 64 * 16);
        }
        int off[T::U];
#pragma unroll
        for (int uu = 0; uu < T::U; ++uu) {
          if constexpr (OTAB) {
            uint32_t wd = otab[uu][0];
#pragma unroll
            for (int q = 1; q < OTW; ++q) wd = s >= 2 * q ? otab[uu][q] : wd;
            off[uu] = (int)((wd >> ((s & 1) * 16)) & 0xffffu);
          } else {
            off[uu] = slot_off<C>(s, uu, g);
          }
        }
        const unsigned char* a0 = abase + off[0];
        const unsigned char* a1 = abase + off[T::U - 1];
#pragma unroll
        for (int u = 0; u < C::MW; ++u) {
          const int mo = ((u / MCOLS) * C::LC + (u % MCOLS) * 16) * C::PSB;
          Frag<P> afr;
          load_frag<P>(afr, a0 + mo, a1 + mo);
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            if constexpr (TRANS)
              mma<P>(acc[u][nb], bfr[nb], afr);
            else
              mma<P>(acc[u][nb], afr, bfr[nb]);
          }
        }
      }
    };
    if constexpr (C::BL) {
      kloop(static_cast<const unsigned char*>(lds + C::WOFF + (C::WRES ? cb : sel) * C::WB + lane * 16));
    } else {
      // one step of A fragments and MFMAs with the B fragments in `cur`
      auto mstep = [&](int s, const Frag<P>* cur) __attribute__((always_inline)) {
        int off[T::U];
#pragma unroll
        for (int uu = 0; uu < T::U; ++uu) off[uu] = slot_off<C>(s, uu, g);
        const unsigned char* a0 = abase + off[0];
        const unsigned char* a1 = abase + off[T::U - 1];
#pragma unroll
        for (int u = 0; u < C::MW; ++u) {
          const int mo = ((u / MCOLS) * C::LC + (u % MCOLS) * 16) * C::PSB;
          Frag<P> afr;
          load_frag<P>(afr, a0 + mo, a1 + mo);
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            if constexpr (TRANS)
              mma<P>(acc[u][nb], cur[nb], afr);
            else
              mma<P>(acc[u][nb], afr, cur[nb]);
          }
        }
      };
      {
        static_assert(C::NGS % 2 == 0, "the B ring starts every stage at slot 0");
        const gbyte* wl = wglob + (size_t)cb * C::WB + lane * 16;
        const gbyte* wn = wglob + (size_t)(cb + 1 == C::NCB ? 0 : cb + 1) * C::WB + lane * 16;
        // issue the B loads of the following step into `nxt`, then step s
        auto step = [&](int s, const Frag<P>* cur, Frag<P>* nxt, const gbyte* np, int ns)
                        __attribute__((always_inline)) {
          load_b(nxt, np, ns);
          __builtin_amdgcn_sched_barrier(0);  // keep the loads ahead of this step's MFMAs
          mstep(s, cur);
        };
#pragma unroll 1
        for (int s = 0; s < C::NGS; s += 2) {
          step(s, bq[0], bq[1], wl, s + 1);
          const bool last = s + 2 == C::NGS;
          step(s + 1, bq[1], bq[0], last ? wn : wl, last ? 0 : s + 2);
        }
      }
    }

    if constexpr (PH) {
      if (cb == C::NCB - 1) {
        // ---- spaced-form epilogue: lane (g, n16) holds channels nb*16 + 4g + k
        // of pixel n16, two max-out pairs whose maxima are stored channels
        // nb*8 + 2g, +1 (one dword). An m-block's 16 pixels x 32 stored
        // channels (1 KB) pass through this wave's LDS scratch, so that each
        // lane stores 16 contiguous bytes.
        static_assert(C::NB == 4, "64 channels, 32 stored: 64 bytes per pixel");
        __shared__ __attribute__((aligned(16))) unsigned char scr_all[NCW * 1024];
        unsigned char* scr = scr_all + wave * 1024;
        int zz, py, px, y0, x0;
        if constexpr (PH == 2) {
          w.group_coords<TY, TX>(zz, py, px, y0, x0);
          const int h = (w.J.geom & 0xff) >> 1;
          py += (wmem >> 1) * h;  // member (a, b) = (wmem / 2, wmem % 2): phase (gy + a h, gx + b h)
          px += (wmem & 1) * h;
        } else {
          w.phase_coords<TY, TX>(zz, py, px, y0, x0);
        }
        const LayerJob& J = w.J;
        const int d = max(J.geom & 0xff, 1), lgo = (J.geom >> 16) & 0xf;
        f4 bs[C::NB];
#pragma unroll
        for (int nb = 0; nb < C::NB; ++nb) bs[nb] = ld<f4>(gin(prm.bias) + (nb * 16 + 4 * g) * 4);
#pragma unroll
        for (int u = 0; u < C::MW; ++u) {
#pragma unroll
          for (int nb = 0; nb < C::NB; ++nb) {
            float v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = acc[u][nb][k] + bs[nb][k];
            *reinterpret_cast<uint32_t*>(scr + n16 * 64 + nb * 16 + g * 4) =
                bf16_key(pack_bf16x2(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
          }
          __builtin_amdgcn_wave_barrier();
          // lane l: stored channels 8 (l % 4) .. + 7 of pixel l / 4
          const i4v o = *reinterpret_cast<const i4v*>(scr + lane * 16);
          __builtin_amdgcn_wave_barrier();
          const int y = py + d * (y0 + wrow0 + u / MCOLS);
          const int x = px + d * (x0 + (u % MCOLS) * 16 + (lane >> 2));
          if (y < J.hout && x < J.wout)
            st<i4v>(gout(J.out) + ((int64_t)zz * J.out_zs + frag_pix(y, x, lgo, J.out_rs, J.out_zs)) * 64 +
                        (lane & 3) * 16,
                    o);
        }
      }
    } else if (cb == C::NCB - 1) {
      int zz, y0, x0;
      w.coords<TY, TX>(zz, y0, x0);
      const EpiJob ej{w.J.out, w.J.out_rs, w.J.out_zs, w.J.hout, w.J.wout};
      if (DEFER && defer) {
        pj = ej;
        pz = zz;
        py0 = y0;
        px0 = x0;
        pend = true;
      } else {
        plain_epi(ej, zz, y0, x0);
      }
    }

    __syncthreads();  // done with this buffer; the next stage is ready
    sel ^= 1;
    if (++cb == C::NCB) {
      cb = 0;
      if constexpr (DEFER)
        more = w.next(js);
      else if (!w.next(js))
        break;
    }
  }
}

// ---------------------------------------------------------------- registry

#define EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, TY, TX, MW)                                          \
  VariantInfo{P, CIN, COUT, KS, POOL, HEAD, TY, TX, MW,                                               \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>::THREADS,                                       \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>::CB,                                            \
              PT<P>::CHB,                                                                             \
              PT<P>::U,                                                                               \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>::NGS,                                           \
              0, 0, 0,                                                                                \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, HEAD>::LDS_TILE,                                      \
              reinterpret_cast<const void*>(&conv_mfma<P, CIN, COUT, KS, POOL, HEAD, TY, TX, MW>), \
              "conv_mfma<" #P "," #CIN "," #COUT "," #KS "," #POOL "," #HEAD "," #TY "," #TX "," #MW ">"}

#define EMCNN_RR(P, CIN, COUT, KS, POOL, HEAD, MR, MC, WX, WY, CBO)                                   \
  VariantInfo{P, CIN, COUT, KS, POOL, HEAD,                                                           \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::TY,                                 \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::TX,                                 \
              MR * MC,                                                                                \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::THREADS,                            \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::CB,                                 \
              PT<P>::CHB,                                                                             \
              PT<P>::U,                                                                               \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::NGR,                                \
              1, 0, 0,                                                                                \
              CfgRR<P, CIN, COUT, KS, MR, MC, WX, WY, HEAD, CBO>::LDS,                                \
              reinterpret_cast<const void*>(&conv_mfma_rr<P, CIN, COUT, KS, POOL, HEAD, MR, MC, WX, WY, CBO>), \
              "conv_mfma_rr<" #P "," #CIN "," #COUT "," #KS "," #POOL "," #HEAD "," #MR "," #MC "," #WX "," #WY \
              "," #CBO ">"}

#define EMCNN_WSK(P, CIN, COUT, KS, POOL, HEAD, TY, TX, NCW, NPW, K1)                                \
  VariantInfo{P, CIN, COUT, KS, POOL, HEAD, TY, TX,                                                   \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::MW,                                      \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::THREADS,                                 \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::CB,                                      \
              PT<P>::CHB,                                                                             \
              PT<P>::U,                                                                               \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::NGS,                                     \
              0, K1, 0,                                                                               \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::LDS,                                     \
              reinterpret_cast<const void*>(&conv_ws<P, CIN, COUT, KS, POOL, HEAD, TY, TX, NCW, NPW, K1>), \
              "conv_ws<" #P "," #CIN "," #COUT "," #KS "," #POOL "," #HEAD "," #TY "," #TX "," #NCW "," #NPW \
              "," #K1 ">",                                                                            \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, K1>::ROWK}
#define EMCNN_WS_PHASE(P, CIN, COUT, KS, TY, TX, NCW, NPW)                                           \
  VariantInfo{P, CIN, COUT, KS, 1, 0, TY, TX,                                                         \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::MW,                                       \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::THREADS,                                  \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::CB,                                       \
              PT<P>::CHB,                                                                             \
              PT<P>::U,                                                                               \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::NGS,                                      \
              0, 0, 1,                                                                                \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::LDS + NCW * 1024,                         \
              reinterpret_cast<const void*>(&conv_ws<P, CIN, COUT, KS, true, false, TY, TX, NCW, NPW, 0, 1>), \
              "conv_ws_phase<" #P "," #CIN "," #COUT "," #KS "," #TY "," #TX "," #NCW "," #NPW ">",        \
              CfgWS<P, CIN, COUT, KS, TY, TX, NCW, NPW, 0>::ROWK}
#define EMCNN_WS_GROUP(P, CIN, COUT, KS, TY, NCW, NPW)                                               \
  VariantInfo{P, CIN, COUT, KS, 1, 0, TY, 16,                                                         \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::MW,                                    \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::THREADS,                               \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::CB,                                    \
              PT<P>::CHB,                                                                             \
              PT<P>::U,                                                                               \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::NGS,                                   \
              0, 0, 1,                                                                                \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::LDS + NCW * 1024,                      \
              reinterpret_cast<const void*>(&conv_ws<P, CIN, COUT, KS, true, false, TY, 16, NCW, NPW, 0, 2>), \
              "conv_ws_group<" #P "," #CIN "," #COUT "," #KS "," #TY "," #NCW "," #NPW ">",               \
              CfgWS<P, CIN, COUT, KS, TY, 16, NCW, NPW, 0, 4>::ROWK, 1}
#define EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, TY, TX, NCW, NPW) \
  EMCNN_WSK(P, CIN, COUT, KS, POOL, HEAD, TY, TX, NCW, NPW, 0)

#define EMCNN_PHASE(P, CIN, COUT, KS, TY, TX, MW, EPI, CBL)                                               \
  VariantInfo{P, CIN, COUT, KS, 1, 0, TY, TX, MW,                                                   \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CBL>::THREADS,                                \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CBL>::CB,                                     \
              PT<P>::CHB,                                                                           \
              PT<P>::U,                                                                             \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CBL>::NGS,                                    \
              0, 0, EPI,                                                                              \
              Cfg<P, CIN, COUT, KS, TY, TX, MW, false, CBL>::LDS_TILE,                               \
              reinterpret_cast<const void*>(&conv_phase<P, CIN, COUT, KS, TY, TX, MW, EPI, CBL>),         \
              "conv_phase<" #P "," #CIN "," #COUT "," #KS "," #TY "," #TX "," #MW "," #EPI "," #CBL ">"}
#define EMCNN_PHASE_GROUP(P, CIN, COUT, KS, TY, MW, CBL)                                                  \
  VariantInfo{P, CIN, COUT, KS, 1, 0, TY, 16, MW,                                                    \
              Cfg<P, CIN, COUT, KS, TY, 16, MW, false, CBL, 4>::THREADS,                              \
              Cfg<P, CIN, COUT, KS, TY, 16, MW, false, CBL, 4>::CB,                                   \
              PT<P>::CHB,                                                                           \
              PT<P>::U,                                                                             \
              Cfg<P, CIN, COUT, KS, TY, 16, MW, false, CBL, 4>::NGS,                                  \
              0, 0, 1,                                                                              \
              Cfg<P, CIN, COUT, KS, TY, 16, MW, false, CBL, 4>::LDS_TILE,                             \
              reinterpret_cast<const void*>(&conv_phase<P, CIN, COUT, KS, TY, 16, MW, 1, CBL, 1>),         \
              "conv_phase_group<" #P "," #CIN "," #COUT "," #KS "," #TY "," #MW "," #CBL ">", 0, 1}
#define EMCNN_HEAD_PHASE(P, CIN, KS, TY, TX)                                                              \
  VariantInfo{P, CIN, 2, KS, 1, 0, TY, TX, 0, CfgHead<CIN, KS, TY, TX>::THREADS, CIN, PT<F32>::CHB, 1, 0, 0, 0, 3, \
              CfgHead<CIN, KS, TY, TX>::LDS, reinterpret_cast<const void*>(&head_phase<P, CIN, KS, TY, TX>),       \
              "head_phase<" #P "," #CIN "," #KS "," #TY "," #TX ">"}
#define EMCNN_HEAD_TAPS(P, CIN, KS, TY, NBC, NW)                                                          \
  VariantInfo{P, CIN, 2, KS, 1, 0, TY, CfgTaps<P, CIN, KS, TY, NBC, NW>::TX, 0,                            \
              CfgTaps<P, CIN, KS, TY, NBC, NW>::THREADS, CIN, PT<P>::CHB, 1, 0, 0, 0, 5,                     \
              CfgTaps<P, CIN, KS, TY, NBC, NW>::LDS, reinterpret_cast<const void*>(&head_taps<P, CIN, KS, TY, NBC, NW>), \
              "head_taps<" #P "," #CIN "," #KS "," #TY "," #NBC "," #NW ">"}
#define EMCNN_HEAD_TAPS4(P, CIN, KS, TY, NBC, NW)                                                         \
  VariantInfo{P, CIN, 2, KS, 1, 0, TY, CfgTaps<P, CIN, KS, TY, NBC, NW>::TX, 0,                            \
              CfgTaps<P, CIN, KS, TY, NBC, NW>::THREADS, CIN, PT<P>::CHB, 1, 0, 0, 0, 6,                     \
              CfgTaps<P, CIN, KS, TY, NBC, NW>::LDS, reinterpret_cast<const void*>(&head_taps4<P, CIN, KS, TY, NBC, NW>), \
              "head_taps4<" #P "," #CIN "," #KS "," #TY "," #NBC "," #NW ">", 0, 1}
#define EMCNN_HEAD_STRIP(P, CIN, KS, TY)                                                                   \
  VariantInfo{P, CIN, 2, KS, 1, 0, TY, 16 - KS + 1, 0, 64, CIN, PT<P>::CHB, 1, 0, 0, 0, 6, 0,               \
              reinterpret_cast<const void*>(&head_strip<P, CIN, KS, TY>), "head_strip<" #P "," #CIN "," #KS "," #TY ">", \
              0, 1}
#define EMCNN_HEAD1(P, CIN, NCLS, TX)                                                                    \
  VariantInfo{P, CIN, NCLS, 1, 0, 0, 1, TX, 0, TX, CIN, PT<F32>::CHB, 1, 0, 0, 0, 4, 0,                     \
              reinterpret_cast<const void*>(&head_1x1<CIN, NCLS, TX>), "head_1x1<" #CIN "," #NCLS "," #TX ">"}

// Pipelined (BF16 / FP8) tile shapes: TY x TX outputs, consumer x producer
// waves, per layer signature (shapes that fit the LDS and the 168 registers
// of a 12-wave workgroup without spilling).
#define EMCNN_WS_NARROW(P, CIN, COUT, KS, POOL, HEAD) \
  EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, 8, 64, 8, 4), EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, 8, 48, 8, 4)
// Four consumer waves with two tile rows (8 m-blocks) each: 512 threads, so
// 256 registers per lane, and B fragments shared by twice the m-blocks.
#define EMCNN_WS_W4(P, CIN, COUT, KS, POOL, HEAD) \
  EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, 8, 64, 4, 4), EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, 8, 48, 4, 4)
#define EMCNN_WS_SHAPES(P, CIN, COUT, KS, POOL, HEAD) \
  EMCNN_WS(P, CIN, COUT, KS, POOL, HEAD, 16, 48, 8, 4), EMCNN_WS_NARROW(P, CIN, COUT, KS, POOL, HEAD)

// Flattened-K tile shapes. The first is each signature's default: 16 x 64
// outputs with 8 m-blocks per wave (halo overhead 1.33x) measured fastest for
// the body convs of net B in every precision on MI355X.
#define EMCNN_SHAPES(P, CIN, COUT, KS, POOL, HEAD)                                                \
  EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, 16, 64, 8), EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, 8, 64, 4), \
      EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, 8, 32, 4), EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, 4, 64, 4), \
      EMCNN_CONV(P, CIN, COUT, KS, POOL, HEAD, 8, 32, 2)

// Row-reuse tile shapes (MR rows x MC m-blocks per wave, WX x WY waves).
#define EMCNN_RR_SHAPES(P, CIN, COUT, KS, POOL, HEAD, CBO)                                                 \
  EMCNN_RR(P, CIN, COUT, KS, POOL, HEAD, 4, 1, 2, 2, CBO), EMCNN_RR(P, CIN, COUT, KS, POOL, HEAD, 8, 1, 2, 1, CBO), \
      EMCNN_RR(P, CIN, COUT, KS, POOL, HEAD, 4, 2, 2, 2, CBO), EMCNN_RR(P, CIN, COUT, KS, POOL, HEAD, 8, 1, 4, 1, CBO)

// The first entry of each layer signature is the default; the rest are
// candidates for the autotuner (which only accepts those whose output is
// bitwise equal to the default's, i.e. the same K order and channel block)
// and for explicit selection with cnn_set_variant.
static const VariantInfo kConv[] = {
    // net B body: 48 -> 48, 5x5 after a pool; 3x3 after a pool with the head fused
    EMCNN_SHAPES(F32, 48, 48, 5, true, false),
    EMCNN_RR_SHAPES(F32, 48, 48, 5, true, false, 0),
    EMCNN_SHAPES(F32, 48, 48, 3, true, true),
    EMCNN_RR_SHAPES(F32, 48, 48, 3, true, true, 0),
    // conv2: separate first layer (defaults first), then with the first layer computed inside
    EMCNN_WS(BF16, 48, 48, 5, true, false, 24, 32, 8, 4), EMCNN_WS(BF16, 48, 48, 5, true, false, 16, 32, 8, 4),
    EMCNN_WS_NARROW(BF16, 48, 48, 5, true, false),
    EMCNN_WSK(BF16, 48, 48, 5, true, false, 8, 64, 8, 4, 5),
    EMCNN_WSK(BF16, 48, 48, 5, true, false, 8, 48, 8, 4, 5),
    EMCNN_WS_W4(BF16, 48, 48, 5, true, false),
    EMCNN_WS_SHAPES(BF16, 48, 48, 3, true, true),
    EMCNN_WS_W4(BF16, 48, 48, 3, true, true),
    // conv2 BF16 / FP8: 24 x 32 tiles, 6 m-blocks per consumer wave (halo
    // 1.31x, against 1.59x for 8 x 64; B fragments shared by 6 m-blocks)
    EMCNN_WS(FP8, 48, 48, 5, true, false, 24, 32, 8, 4), EMCNN_WS(FP8, 48, 48, 5, true, false, 16, 32, 8, 4),
    EMCNN_WS_NARROW(FP8, 48, 48, 5, true, false),
    EMCNN_WSK(FP8, 48, 48, 5, true, false, 8, 64, 8, 4, 5),
    EMCNN_WSK(FP8, 48, 48, 5, true, false, 8, 48, 8, 4, 5),
    EMCNN_WS_W4(FP8, 48, 48, 5, true, false),
    // FP8 conv3: 16 x 48 tiles (6 m-blocks per consumer wave) carry 1.5x the
    // MFMA work of an 8 x 64 tile per stage barrier, with a smaller halo
    EMCNN_WS(FP8, 48, 48, 3, true, true, 16, 48, 8, 4), EMCNN_WS_NARROW(FP8, 48, 48, 3, true, true),
    EMCNN_WS_W4(FP8, 48, 48, 3, true, true), EMCNN_WS(FP8, 48, 48, 3, true, true, 24, 32, 8, 4),
    // net A body: 16 -> 16, 5x5, no pool, head fused (FP32)
    EMCNN_SHAPES(F32, 16, 16, 5, false, true),
    // same layer shapes without the pool / with the head elsewhere (generic specs)
    EMCNN_CONV(F32, 48, 48, 5, false, false, 8, 64, 4),
    EMCNN_CONV(F32, 48, 48, 3, false, true, 8, 64, 4),
    EMCNN_CONV(F32, 48, 48, 5, false, true, 8, 64, 4),
    EMCNN_WS(BF16, 48, 48, 5, false, false, 8, 64, 8, 4),
    EMCNN_WS(BF16, 48, 48, 3, false, true, 8, 64, 8, 4),
    EMCNN_WS(FP8, 48, 48, 5, false, false, 8, 64, 8, 4),
    EMCNN_WS(FP8, 48, 48, 3, false, true, 8, 64, 8, 4),
    EMCNN_CONV(F32, 16, 16, 5, true, true, 8, 32, 4),
    EMCNN_CONV(F32, 16, 16, 5, false, false, 8, 32, 4),
    // FastMemb body convs (4x4, 32 -> 64, max-out to 32), spaced form: over
    // groups of four phases with 16-channel stages (the default where the max
    // filter has half the conv's spacing; 17.7-17.8 against 18.1-18.2 ms per
    // conv) or 32 (bitwise the same as one phase's 8 x 64 tile), or per phase
    // (all 32 channels per stage use a whole 128-byte pixel line at once)
    EMCNN_PHASE_GROUP(F32, 32, 64, 4, 8, 4, 16), EMCNN_PHASE_GROUP(F32, 32, 64, 4, 8, 4, 32),
    EMCNN_PHASE(F32, 32, 64, 4, 8, 64, 4, 1, 32), EMCNN_PHASE(F32, 32, 64, 4, 8, 64, 8, 1, 32),
    EMCNN_PHASE(F32, 32, 64, 4, 16, 64, 8, 1, 16), EMCNN_PHASE(F32, 32, 64, 4, 8, 64, 4, 1, 16),
    // the softmax layer (the host orders its candidates: phase-group kernels
    // first, head_strip's 61-row strips the default): as a GEMM over the 16
    // taps of the weight difference per phase group (head_strip, head_taps4)
    // or per phase (head_taps), on the VALU (head_phase), or as a conv with
    // 14 zero MFMA columns (conv_phase)
    EMCNN_HEAD_PHASE(F32, 32, 4, 8, 64), EMCNN_HEAD_PHASE(F32, 32, 4, 4, 64),
    EMCNN_HEAD_TAPS(F32, 32, 4, 13, 4, 8), EMCNN_HEAD_TAPS(F32, 32, 4, 8, 4, 4), EMCNN_HEAD_TAPS(F32, 32, 4, 5, 4, 4),
    EMCNN_HEAD_TAPS(F32, 32, 4, 8, 8, 8),
    EMCNN_HEAD_STRIP(F32, 32, 4, 61), EMCNN_HEAD_STRIP(F32, 32, 4, 41), EMCNN_HEAD_STRIP(F32, 32, 4, 31),
    EMCNN_HEAD_TAPS4(F32, 32, 4, 13, 4, 8), EMCNN_HEAD_TAPS4(F32, 32, 4, 5, 4, 4), EMCNN_HEAD_TAPS4(F32, 32, 4, 6, 4, 4),
    EMCNN_PHASE(F32, 32, 16, 4, 8, 64, 4, 2, 32), EMCNN_PHASE(F32, 32, 16, 4, 16, 64, 8, 2, 16),
    // FastMemb BF16: bf16 activations (NHWC, 64 B per pixel) and weights, FP32
    // accumulation; the softmax layer's kernels as for FP32, on bf16 MFMA
    // (head_phase: FP32 on the VALU)
    // body convs: warp-specialised (16-channel stages, weights resident in
    // LDS) over groups of four phases (the default where the max filter has
    // half the conv's spacing: 12 x 16 tiles of each member, 1.93 against
    // 2.38 ms for one phase's 8 x 64 tile) or one phase, conv_phase with the
    // same 16-channel stages (the same MFMA sequence), and conv_phase staging
    // all 32 channels at once
    EMCNN_WS_GROUP(BF16, 32, 64, 4, 12, 8, 4), EMCNN_WS_GROUP(BF16, 32, 64, 4, 8, 8, 4),
    EMCNN_WS_PHASE(BF16, 32, 64, 4, 16, 32, 8, 4), EMCNN_WS_PHASE(BF16, 32, 64, 4, 8, 64, 8, 4),
    EMCNN_WS_PHASE(BF16, 32, 64, 4, 8, 64, 4, 4),
    EMCNN_PHASE(BF16, 32, 64, 4, 8, 64, 4, 1, 16),
    EMCNN_PHASE(BF16, 32, 64, 4, 8, 64, 4, 1, 32), EMCNN_PHASE(BF16, 32, 64, 4, 16, 64, 8, 1, 32),
    EMCNN_PHASE(BF16, 32, 16, 4, 8, 64, 4, 2, 32), EMCNN_HEAD_PHASE(BF16, 32, 4, 8, 64),
    EMCNN_HEAD_TAPS(BF16, 32, 4, 13, 4, 8), EMCNN_HEAD_TAPS(BF16, 32, 4, 8, 4, 4), EMCNN_HEAD_TAPS(BF16, 32, 4, 5, 4, 4),
    EMCNN_HEAD_TAPS(BF16, 32, 4, 8, 8, 8),
    EMCNN_HEAD_STRIP(BF16, 32, 4, 61), EMCNN_HEAD_STRIP(BF16, 32, 4, 41), EMCNN_HEAD_STRIP(BF16, 32, 4, 31),
    EMCNN_HEAD_TAPS4(BF16, 32, 4, 13, 4, 8), EMCNN_HEAD_TAPS4(BF16, 32, 4, 5, 4, 4), EMCNN_HEAD_TAPS4(BF16, 32, 4, 6, 4, 4),
    // MaskExtend (FP32): twelve input maps, max-out convs to 32, 40, 48, 56, 64
    // features (channels staged per LDS pass chosen to fit 160 KB with the
    // 8 (mod 16) dword pixel stride), the 1x1 three-class softmax on the VALU
    // (the three widest layers: 4 x 64 tiles of 2 m-blocks per wave, 7 or 8
    // n-blocks each, 138-162 registers instead of 192-236: 14-25 % faster than
    // 8 x 64 tiles of 4 m-blocks, bitwise the same)
    // (the three widest over phase groups of 4 x 16 tiles: 15.4 against 15.9,
    // 11.95 against 12.0 and 9.43 against 9.48 ms; the narrowest's group
    // candidate measured 1 % slower)
    EMCNN_PHASE(F32, 12, 64, 4, 8, 64, 4, 1, 12), EMCNN_PHASE(F32, 32, 80, 4, 8, 64, 4, 1, 32),
    EMCNN_PHASE_GROUP(F32, 40, 96, 4, 4, 2, 40), EMCNN_PHASE_GROUP(F32, 48, 112, 4, 4, 2, 24),
    EMCNN_PHASE_GROUP(F32, 56, 128, 4, 4, 2, 28), EMCNN_HEAD1(F32, 64, 3, 256),
    EMCNN_PHASE(F32, 32, 80, 4, 4, 64, 2, 1, 32), EMCNN_PHASE(F32, 40, 96, 4, 8, 64, 4, 1, 40),
    EMCNN_PHASE(F32, 48, 112, 4, 8, 64, 4, 1, 24), EMCNN_PHASE(F32, 56, 128, 4, 8, 64, 4, 1, 28),
    EMCNN_PHASE_GROUP(F32, 32, 80, 4, 4, 2, 32), EMCNN_PHASE(F32, 40, 96, 4, 4, 64, 2, 1, 40),
    EMCNN_PHASE(F32, 48, 112, 4, 4, 64, 2, 1, 24), EMCNN_PHASE(F32, 56, 128, 4, 4, 64, 2, 1, 28),
};

#define EMCNN_FIRSTV(PO, COUT, KS, TY, TX, MX, ST, XS, SUFFIX)                                       \
  FirstInfo{PO, COUT, KS, MX, ST, TY, TX, FirstCfg<PO, COUT, KS, TY, TX, ST>::THREADS,                \
            FirstCfg<PO, COUT, KS, TY, TX, ST>::LDS,                                                  \
            reinterpret_cast<const void*>(&conv_first<PO, COUT, KS, TY, TX, MX, ST, XS>),             \
            "conv_first<" #PO "," #COUT "," #KS "," #TY "," #TX "," #MX "," #ST SUFFIX ">"}
#define EMCNN_FIRSTS(PO, COUT, KS, TY, TX, MX, ST) EMCNN_FIRSTV(PO, COUT, KS, TY, TX, MX, ST, 0, "")
// output staged through LDS for 16-byte stores
#define EMCNN_FIRSTX(PO, COUT, KS, TY, TX) EMCNN_FIRSTV(PO, COUT, KS, TY, TX, false, 1, 1, ",xs")
#define EMCNN_FIRSTM(PO, COUT, KS, TY, TX, MX) EMCNN_FIRSTS(PO, COUT, KS, TY, TX, MX, 1)
#define EMCNN_FIRST(PO, COUT, KS, TY, TX) EMCNN_FIRSTM(PO, COUT, KS, TY, TX, false)

static const FirstInfo kFirst[] = {
    // defaults (first match per signature) are the measured fastest shapes:
    // FP8 output staged through LDS for 16-byte stores (0.39 against 0.53 ms
    // stored from registers, on 8 x 2048^2), BF16 stored from registers. Tall
    // tiles pay off where the layer is cheap per staged row: 16 x 128 BF16 and
    // 32 x 128 FP8 against 8 x 64 and 16 x 128 (5 % and 3 % faster); for the
    // max-out layers 16 x 128 FP32 and 32 x 128 BF16 against 4 x 64 (13 % and
    // 26 % faster; a 4-row tile stages 7 rows)
    EMCNN_FIRST(F32, 48, 5, 4, 64),  EMCNN_FIRST(BF16, 48, 5, 16, 128), EMCNN_FIRSTX(FP8, 48, 5, 32, 128),
    EMCNN_FIRST(F32, 16, 5, 4, 64),  EMCNN_FIRST(F32, 48, 5, 8, 32),   EMCNN_FIRST(F32, 48, 5, 8, 64),
    EMCNN_FIRST(BF16, 48, 5, 8, 64), EMCNN_FIRST(BF16, 48, 5, 32, 64), EMCNN_FIRST(BF16, 48, 5, 4, 64),
    EMCNN_FIRST(FP8, 48, 5, 8, 64),  EMCNN_FIRST(FP8, 48, 5, 4, 64),   EMCNN_FIRST(FP8, 48, 5, 16, 64),
    EMCNN_FIRSTX(BF16, 48, 5, 8, 64), EMCNN_FIRSTX(FP8, 48, 5, 16, 64), EMCNN_FIRSTX(FP8, 48, 5, 16, 128),
    EMCNN_FIRSTX(FP8, 48, 5, 16, 256),
    // FastMemb first conv: 4x4, 1 -> 64, max-out to 32
    EMCNN_FIRSTM(F32, 64, 4, 16, 128, true), EMCNN_FIRSTM(F32, 64, 4, 32, 64, true), EMCNN_FIRSTM(F32, 64, 4, 4, 64, true),
    EMCNN_FIRSTM(BF16, 64, 4, 32, 128, true), EMCNN_FIRSTM(BF16, 64, 4, 16, 256, true), EMCNN_FIRSTM(BF16, 64, 4, 4, 64, true),
    // FastMemb_ss first conv: evaluated only where the 2x subsample after it
    // keeps a pixel (16 x 64 FP32 and 8 x 64 BF16: 7 % and 2 % faster than 4 x 64)
    EMCNN_FIRSTS(F32, 64, 4, 16, 64, true, 2), EMCNN_FIRSTS(F32, 64, 4, 8, 64, true, 2), EMCNN_FIRSTS(F32, 64, 4, 4, 64, true, 2),
    EMCNN_FIRSTS(BF16, 64, 4, 8, 64, true, 2), EMCNN_FIRSTS(BF16, 64, 4, 16, 64, true, 2), EMCNN_FIRSTS(BF16, 64, 4, 4, 64, true, 2),
};

int conv_variant_count() { return (int)(sizeof(kConv) / sizeof(kConv[0])); }
const VariantInfo* conv_variant(int i) { return &kConv[i]; }
int first_variant_count() { return (int)(sizeof(kFirst) / sizeof(kFirst[0])); }
const FirstInfo* first_variant(int i) { return &kFirst[i]; }

}  // namespace emcnn
