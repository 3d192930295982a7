// Internal types shared by the library's host runtime and its kernels.
#pragma once

#include <stdint.h>

namespace emcnn {

enum Prec : int { F32 = 0, BF16 = 1, FP8 = 2 };

// One 3-D activation volume processed by one layer launch.
//
// Activations between layers: FP32 nets use NHWC, element (z, y, x, c) of a
// C-channel tensor at ((z * zs) + y * rs + x) * C + c; BF16 / FP8 nets use the
// channel-blocked layout, the same element at z*zs*C + (c/16)*zs*16 +
// (y*rs + x)*16 + c%16 (rs / zs in pixels in both). A slice occupies zs*C
// elements either way. The first layer reads the caller's uint8 volume with
// the same addressing (C = 1); the head layer writes float32 probabilities
// (C = 1).
//
// (hin, win) are the dims of the STORED input. When the layer pools its input
// (a 2x2 stride-1 max filter sits between the previous conv and this one) the
// layer sees a (hin-1) x (win-1) input. (hout, wout) are this layer's conv
// output dims.
struct LayerJob {
  const void* in;
  void* out;
  int64_t in_rs, in_zs;
  int64_t out_rs, out_zs;
  int64_t item0;  // index of this job's first work item across the launch
  const int32_t* gate;  // device flag; the job's items are skipped when *gate == 0 (nullptr: always run)
  int32_t z, hin, win, hout, wout;
  int32_t tiles_x, tiles_y;
  // Spaced layers (nets with stride-2 pools, evaluated densely): bits 0-7 the
  // spacing d of the conv taps, bits 8-15 the spacing of the 2x2 max filter
  // before it (0: no max filter); 0 for the plain kernels. With d > 1 the output splits into d^2
  // phase sub-lattices (positions py + d r, px + d c) that are tiled
  // separately: tiles_y counts d^2 x the tile rows of the largest phase.
  // Bits 16-19: lg, the output map is stored fragment-major modulo D = 2^lg
  // (0: row-major). Such a map keeps each of its D^2 fragments (pixels
  // (fy + D r, fx + D c)) as a separate row-major block: pixel (y, x) of a
  // slice is at ((y % D) D + x % D) (zs / D^2) + (y / D) rs + x / D, with
  // rs = ceil(w / D) and zs = D^2 ceil(h / D) ceil(w / D). The input map of a
  // spaced layer is stored fragment-major modulo its own d.
  int32_t geom;
};

// Work description of one layer launch: either a single job passed by value,
// or a device table of jobs (batched submissions).
struct JobSet {
  const LayerJob* table;  // device; nullptr -> use `single`
  int32_t njobs;
  int32_t pad_;
  int64_t total_items;
  LayerJob single;
};

struct ConvParams {
  const void* wpack;     // packed B fragments (layout decided by the kernel variant)
  const float* bias;     // [cout]
  const float* oscale;   // [cout] epilogue multiplier, nullptr = 1
  const float* head_w;   // [cout] head weights (head variants)
  float head_b;
  float out_inv_scale;   // FP8 output codes: e4m3(v * out_inv_scale)
  // fused variants only: the uint8 first layer computed in the producers
  const void* w1;        // first-layer B fragments, bf16 [n-block][lane][8 taps], 1/255 folded in
  const float* b1;       // [cin] first-layer bias
  float w1_inv_scale;    // FP8: first-layer output codes e4m3(v * w1_inv_scale)
  float pad_;
};

struct FirstParams {
  const float* w;     // [cout][k][k], with 1/255 folded in (bf16 values in BF16/FP8 nets)
  const float* bias;  // [cout]
  float out_inv_scale;
  float pad_;
};

// Compile-time description of a conv-kernel variant (also used on the host to
// pack weights in the layout the variant reads).
struct VariantInfo {
  int prec, cin, cout, ks, pool_in, head;
  int ty, tx, mw;       // output tile rows / cols, m-blocks per wave
  int threads;
  int cb;               // channels staged per LDS pass
  int chb;              // channels per 16-byte chunk
  int u;                // chunks per lane per MFMA
  int ngs;              // group-steps per channel block (row reuse: per filter row)
  int rr;               // 1: row-reuse kernel (weights packed per filter row)
  int fused;            // k > 0: the kernel reads the uint8 input and computes the preceding
                        // 1-channel k x k first layer (and the max filter) itself
  int epi;              // epilogue: 0 bias + ReLU (or the fused 1x1 sigmoid head),
                        // 1 bias + max-out over channel pairs (stores cout / 2 channels),
                        // 2 bias + two-class softmax of channels 0, 1 (stores the class-1 probability),
                        // 3 the two-class softmax layer on the VALU (head_phase),
                        // 4 a 1x1 conv to cout classes with a softmax, storing class 0 (head_1x1),
                        // 5 the two-class softmax layer as a GEMM over its 16 taps (head_taps),
                        // 6 the same over groups of four phases (head_taps4)
  int lds_bytes;        // LDS of the staged operand tiles and weights (descriptive; launches and
                        // occupancy take the kernel's own static LDS, epilogue scratch included)
  const void* fn;       // kernel symbol (host pointer for hipLaunchKernel)
  const char* name;
  int rowq = 0;         // 1: row-quad K order (k_slot); 0: flattened
  int groups = 0;       // 1: a work item is a tile of four phases whose max filters share
                        // fragments (spaced layers whose max filter has half their spacing)
};

// K order of the implicit-GEMM convs over one channel block. K slot c is read
// by lane group c % 4 of the (c / 4)-th quad of slots, and holds 16-byte chunk
// cg of tap (i, j) of the block's pixels.
// * Flattened: chunk c of the block's KS x KS x NCHB chunks, row-major over
//   (i, j, cg); slots past the last chunk carry zero weights.
// * Row quads (conv_ws, whose LDS pixels are unpadded, so a filter row's
//   KS x NCHB chunks of a pixel run are one contiguous run): quad q covers 4
//   consecutive chunks e .. e + 3 of filter row q / QR (QR = quads per row),
//   e = 4 (q % QR) except that a row's last quad ends at its last chunk.
//   Chunks a quad repeats, and quads past the last row (which read row 0's
//   first quad), carry zero weights. Lane group g then reads 16 g bytes past
//   its quad's first chunk, whatever the quad.
struct KSlot {
  int i, j, cg;
  bool live;  // false: the slot's weights are zero
};
__host__ __device__ constexpr int rowq_quads(int ks, int nchb) { return (ks * nchb + 3) / 4; }
__host__ __device__ inline KSlot k_slot(int c, int ks, int nchb, bool rowq) {
  const int nrow = ks * nchb;  // chunks of one filter row
  KSlot k{0, 0, 0, false};
  int i, e;
  if (!rowq) {
    k.live = c < ks * nrow;
    const int cc = k.live ? c : ks * nrow - 1;  // a padded slot reads real (finite) data
    i = cc / nrow;
    e = cc % nrow;
  } else {
    const int qr_n = rowq_quads(ks, nchb), q = c / 4, g = c % 4;
    i = q / qr_n;
    const int qr = q % qr_n;
    int e0 = 4 * qr;
    if (e0 + 4 > nrow) e0 = nrow - 4;  // the row's last quad (nrow >= 4)
    e = e0 + g;
    k.live = i < ks && e >= 4 * qr;
    if (i >= ks) {
      i = 0;
      e = g;
    }
  }
  k.i = i;
  k.j = e / nchb;
  k.cg = e % nchb;
  return k;
}

struct FirstInfo {
  int prec_out, cout, ks;
  int maxout;  // 1: bias + max-out over channel pairs (stores cout / 2 channels); 0: bias + ReLU
  int stride;  // output stride: 2 evaluates the conv at every second input row and column only
  int ty, tx, threads;
  int lds_bytes;  // the uint8 input tile (descriptive; the per-wave epilogue scratch comes on top)
  const void* fn;
  const char* name;
};

// Registries implemented in conv_kernels.hip.
int conv_variant_count();
const VariantInfo* conv_variant(int i);
int first_variant_count();
const FirstInfo* first_variant(int i);

}  // namespace emcnn
