/*
 * emcnn.h - C ABI of an MI355X (gfx950) library for dense membrane-probability
 * inference: a uint8 electron-microscopy stack goes in, one membrane
 * probability per voxel comes out (arXiv 1612.02120, Section 2.1 "Membrane
 * classification": EM images are mapped to per-pixel membrane probability maps
 * by a CNN; Section 2.2 "Accelerating dense computation": all pixel labels are
 * produced in one dense pass, with max-pooling replaced by stride-1 max
 * filtering).
 *
 * Conventions for every entry point:
 *  - Return CNN_OK (0) or a negative CNN_E* code; cnn_last_error() gives a
 *    thread-local message for the last failure on the calling thread.
 *  - Arguments are validated before anything is enqueued: a failed call leaves
 *    the stream untouched. Nothing is printed, nothing aborts, no C++ exception
 *    crosses the ABI.
 *  - Volume, output, patch and teacher pointers are DEVICE pointers owned by the
 *    caller. Weight arrays and tile descriptor arrays are HOST memory, copied
 *    during the call (the caller may free them on return).
 *  - `stream` is a hipStream_t (NULL = legacy default stream). Inference and
 *    training calls only enqueue work and return; faults of enqueued kernels
 *    surface at the caller's next synchronisation of that stream.
 *  - A handle owns device workspace: do not use one handle on two streams
 *    concurrently.
 *  - Dense geometry: a net with receptive radius R (r += (k-1) j over the
 *    layers, a 2x2 pool counting as k = 2, a subsample as k = 1, with j the
 *    input spacing, doubled after every stride-2 layer; field of view R+1)
 *    maps a Z x H x W volume to a Z x (H-R) x (W-R) float32 map, C order;
 *    output (z, y, x) is the net on the field-of-view window at input (z, y, x),
 *    centred on (z, y + R/2, x + R/2). A net with a 2x subsample
 *    (CNN_LAYER_SUBSAMPLE2) outputs every second of those rows and columns:
 *    Z x Ho x Wo with Ho = (H - R - 1) / 2 + 1, output (z, y, x) being the
 *    window at input (z, 2y, 2x) (cnn_output_dims). Slices are independent
 *    (2-D nets).
 *  - Input scaling: the network sees V/255; the library folds 1/255 into the
 *    first convolution.
 */
#ifndef EMCNN_H
#define EMCNN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CNN_OK 0
#define CNN_EINVAL (-1)       /* null pointer, bad size, dims < field of view, bad spec */
#define CNN_ENOMEM (-2)       /* device or pinned-host allocation failed */
#define CNN_EHIP (-3)         /* a HIP runtime call failed (text in cnn_last_error) */
#define CNN_EUNSUPPORTED (-4) /* valid request outside what the kernels implement */

enum cnn_layer_kind {
  CNN_LAYER_CONV = 0,
  CNN_LAYER_MAXPOOL = 1,
  CNN_LAYER_MAXPOOL_S2 = 2,
  CNN_LAYER_SUBSAMPLE2 = 3 /* keep every second row and column (window 1, stride 2) */
};
enum cnn_act {
  CNN_ACT_NONE = 0,
  CNN_ACT_RELU = 1,
  CNN_ACT_SIGMOID = 2,
  CNN_ACT_MAXOUT = 3,  /* max over channel pairs (2c, 2c+1): cout / 2 channels out */
  CNN_ACT_SOFTMAX = 4, /* two classes; the output map is the class-1 (membrane) probability */
  CNN_ACT_SOFTMAX0 = 5 /* softmax over cout classes; the output map is class 0's probability */
};
enum cnn_precision { CNN_PREC_FP32 = 0, CNN_PREC_BF16 = 1, CNN_PREC_FP8 = 2 };

/* One layer of the network (Section 2.2: alternating convolution and max
 * pooling; pooling is evaluated densely as a 2x2 stride-1 max filter).
 *  kind      CNN_LAYER_CONV (valid k x k cross-correlation, bias, activation),
 *            CNN_LAYER_MAXPOOL (2x2 window, stride 1; k must be 2, other fields 0) or
 *            CNN_LAYER_MAXPOOL_S2 (2x2 window, stride 2, as in a sliding-window
 *            classifier such as FastMemb; k must be 2). The library still
 *            produces every pixel's label: it evaluates such a pool as a 2x2 max
 *            filter whose elements are j apart and doubles j for every later
 *            layer (j = 1 at the input; a conv's taps are then j apart), which
 *            equals computing the paper's 4 fragments per pool and interleaving
 *            them.
 *  act_scale FP8 nets only: the per-tensor scale s of this conv's INPUT
 *            activation (codes are e4m3fn(a / s)); ignored for the first conv,
 *            the head and other precisions. */
typedef struct cnn_layer {
  int32_t kind;
  int32_t k;
  int32_t cin;
  int32_t cout;
  int32_t act;
  float act_scale;
} cnn_layer;

typedef struct cnn_layer_spec {
  int32_t n_layers;
  const cnn_layer* layers; /* host array of n_layers entries */
  int32_t precision;       /* enum cnn_precision */
} cnn_layer_spec;

typedef struct cnn_net cnn_net;

/* Build a network on the current HIP device.
 * Two families of nets are supported: the ReLU nets described below, and the
 * FastMemb family (Section 2.2), FP32 or BF16 (bf16 weights and stored
 * activations with FP32 accumulation in every conv, the first conv with
 * bf16(w / 255) weights; the two-class softmax layer takes the weight
 * difference W[1] - W[0], rounded once to the form's type, by default on MFMA
 * with FP32 accumulation, and its VALU candidate reads bf16 activations with
 * FP32 weights):
 * conv(k=4, 1 -> 64, MAXOUT), then
 * one or more pairs { MAXPOOL_S2, conv(k=4, 32 -> 64, MAXOUT) }, then
 * MAXPOOL_S2 and conv(k=4, 32 -> 2, SOFTMAX); no other transfer function.
 * FastMemb itself has two inner pairs: field of view 53 (R = 52). The first
 * conv may be followed by SUBSAMPLE2 and a conv(k=4, 32 -> 64, MAXOUT) without
 * a pool before the pairs (FastMemb_ss, Section 2.2, "A subsampling CNN for
 * 3 nm data": a 3 nm stack gives a 6 nm map); only the kept fragment is
 * computed: the first conv at every second row and column, the rest densely
 * on that half-resolution map. FP32 nets may instead start with
 * conv(k=4, C -> 2F, MAXOUT) on C > 1 real-valued maps (cnn_infer_maps), use
 * any widths conv(k=4, F -> 2F', MAXOUT) that the library has kernels for, and
 * end with a conv(1x1, F -> n, SOFTMAX0) right after the last conv: MaskExtend
 * (Section 3) has C = 12 and widths 32, 40, 48, 56, 64 with three classes.
 * weights: host float64, for each conv in order W[cout][cin][k][k] (C order)
 *   followed by b[cout]; n_weights must equal that total. Copied, then packed
 *   and quantised once here:
 *     FP32: all products in FP32 with FP32 accumulation;
 *     BF16: every conv but the 1x1 head takes bf16 weights and bf16 input
 *           activations (round to nearest even), FP32 accumulation;
 *     FP8:  the first conv as BF16; later convs except the head take e4m3fn
 *           weights with per-output-channel scale max|W[co]|/448 and e4m3fn
 *           input codes with the layer's act_scale, FP32 accumulation,
 *           dequantised in the epilogue as acc * s * sw[co] + b[co].
 *   The head (last layer, 1x1 conv to one channel with sigmoid) is FP32 in
 *   every precision.
 * Supported shape: conv(k=5, 1 -> 16 or 48, ReLU) [pool], then one or more
 *   conv(k in {3,5}, C -> C, ReLU) [pool] with C = 16 (FP32) or 48, then the
 *   head conv(1x1, C -> 1, sigmoid) with no pool before it. Other valid specs
 *   return CNN_EUNSUPPORTED.
 * On success *out owns device memory until cnn_destroy. */
int cnn_create(const double* weights, int64_t n_weights, const cnn_layer_spec* spec,
               cnn_net** out);

/* Release a network and its device memory (synchronises the device first).
 * NULL is accepted. */
int cnn_destroy(cnn_net* net);

/* Receptive radius R and field of view R+1 (either pointer may be NULL). */
int cnn_geometry(const cnn_net* net, int32_t* R, int32_t* fov);

/* Output dims of an H x W slice: H - R and W - R, or for a net with a 2x
 * subsample (H - R - 1) / 2 + 1 and (W - R - 1) / 2 + 1. CNN_EINVAL if H or W
 * is below the field of view. */
int cnn_output_dims(const cnn_net* net, int64_t H, int64_t W, int64_t* Ho, int64_t* Wo);

/* Dense inference of a whole volume (Section 2.2: every pixel label in one
 * pass, no per-patch recomputation).
 * volume_u8: device, Z x H x W uint8, C order (x fastest).
 * dims: host {Z, H, W}; H and W must be >= R+1, Z >= 1, each < 2^30.
 * prob_out: device, Z x Ho x Wo float32 (cnn_output_dims; Z x (H-R) x (W-R)
 * for nets without a subsample), fully overwritten.
 * Grows the handle's workspace with hipMalloc when needed (the only allocation
 * it may make). */
int cnn_infer(cnn_net* net, const uint8_t* volume_u8, const int64_t dims[3], float* prob_out,
              void* stream);

/* Dense inference of a net whose first conv reads C > 1 real-valued input
 * maps (MaskExtend, Section 3: EM sections, object masks and membrane maps
 * stacked as the input of one section), FP32.
 * maps: device, Z x H x W x C float32 (C fastest), taken as they are (no
 * scaling); dims: host {Z, H, W, C} with C the first conv's cin.
 * prob_out: device, Z x (H-R) x (W-R) float32. Otherwise as cnn_infer. */
int cnn_infer_maps(cnn_net* net, const float* maps, const int64_t dims[4], float* prob_out, void* stream);

/* cnn_infer for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and result (bit for bit) as cnn_infer, but no
 * allocation of any kind: the inter-layer maps live in a static device array
 * of CNN_NOALLOC_SCRATCH_BYTES, which every device the library runs on holds
 * until the process ends. The volume runs as slabs of whole slices when one
 * slice fits the array, else as strips of output rows (a multiple of 16) that
 * overlap by R input rows. Rows too wide for a 16-row strip return CNN_EINVAL
 * before anything is enqueued (for net B in FP32, widths above about 16,000
 * columns). All calls on one device share its array and keep no state in it
 * (every map is written before it is read): calls that overlap on one device
 * (two streams, two threads) race and must be serialised by the caller.
 * Per-layer profiling (cnn_profile) does not record these launches. */
#define CNN_NOALLOC_SCRATCH_BYTES ((int64_t)128 << 20)
int cnn_infer_noalloc(cnn_net* net, const uint8_t* volume_u8, const int64_t dims[3], float* prob_out,
                      void* stream);

/* One block of a volume with its halo of input context (Section 2.1, "Block
 * merging": blocks are processed independently).
 * in:  device, z x h x w uint8 (the block plus `halo` pixels on every side).
 * out: device, z x (h - 2 halo) x (w - 2 halo) float32, the block's interior;
 *      out (t, y, x) is the probability centred on in (t, y + halo, x + halo).
 * halo must be >= R/2 and h, w > 2 halo. */
typedef struct cnn_tile {
  const uint8_t* in;
  int64_t z, h, w;
  int32_t halo;
  float* out;
} cnn_tile;

/* Many uneven blocks in one submission: the descriptors are copied to the
 * device and every layer runs as ONE persistent kernel over the work items of
 * all blocks; the submission is captured once as a HIP graph and replayed on
 * later calls with the same structure. tiles: host array of n descriptors.
 * Results equal per-block cnn_infer on each block's input, bit for bit. */
int cnn_infer_batch(cnn_net* net, const cnn_tile* tiles, int32_t n, void* stream);

/* Pick, per layer, the fastest compiled tile shape for H x W slices by timing
 * every candidate on the device (synchronous; repeated launches totalling about
 * 5 ms per candidate). Each candidate's output must be
 * bitwise equal to the default's or it is rejected. cache_path (nullable): a
 * text file of earlier choices, read first and updated. */
int cnn_autotune(cnn_net* net, int64_t H, int64_t W, const char* cache_path, void* stream);

/* Per tile class tile shapes for cnn_infer_batch (Section 2.2: the volume is
 * processed as independent blocks, of varied sizes). Tiles are classed by
 * their smaller output side, with representative sides 64, 128, 256, 512 and
 * 1024 (class edges at their geometric means, 91, 181, 362 and 724). For each
 * class present in `tiles` (the same descriptors cnn_infer_batch takes), every
 * layer's candidates are timed, greedily layer by layer, on submissions of
 * that class's tiles; a candidate is accepted only if every output of the class
 * is bitwise equal to the default variants' output. cnn_infer_batch then plans
 * each class with its own variants (classes with equal choices together);
 * cnn_infer keeps the handle's selected variants, and cnn_set_variant drops the
 * per-class choice. The tiles' output buffers are overwritten (their content
 * afterwards is unspecified). Synchronous; allocates a copy of the largest
 * class's outputs while it runs. */
int cnn_autotune_batch(cnn_net* net, const cnn_tile* tiles, int32_t n, void* stream);

/* Batched submissions are captured as a HIP graph by default; enable = 0
 * launches the same kernels directly instead (a per-call launch sequence). */
int cnn_set_batch_graph(cnn_net* net, int32_t enable);

/* Upper bound in bytes of the handle's inter-layer workspace (default 24 GiB,
 * or EMCNN_WORKSPACE_MB); larger volumes are processed in slabs of slices. */
int cnn_set_workspace_limit(cnn_net* net, int64_t bytes);

/* Per-layer kernel timing: while enabled, every layer launch of this handle
 * is bracketed by HIP events recorded on the launch stream (direct launches
 * only; graph replays are not timed). cnn_profile_read waits for the events,
 * writes the summed milliseconds and launch count per executed layer (first
 * layer, body convs; the head is fused into the last body conv) and clears
 * the record. */
int cnn_profile(cnn_net* net, int32_t enable);
int cnn_profile_read(cnn_net* net, double* ms_per_layer, int32_t* launches_per_layer,
                     int32_t max_layers);

/* Executed layers: 0 = first conv, then one per body conv (the head is fused
 * into the last one). cnn_variant_name writes the name of candidate `index`
 * of `layer` (CNN_EINVAL past the last); cnn_set_variant selects a candidate
 * by name for later calls. Candidates of one layer may differ in accumulation
 * order (and so in the last bits of the result).
 * In BF16 / FP8 nets whose first conv is 1->C 5x5 followed by a max pool and a
 * C->C 5x5 conv, layer 1 also has candidates (names ending in ",5>") that read
 * the uint8 input and compute layer 0 themselves, with a bitwise-equal result
 * and no layer-0 output in HBM; while one is selected, layer 0 is not launched
 * (no launches in cnn_profile_read). The default keeps the separate layer-0
 * launch (measured as fast or faster on MI355X). */
int cnn_variant_name(const cnn_net* net, int32_t layer, int32_t index, char* buf, int32_t buf_len);
int cnn_set_variant(cnn_net* net, int32_t layer, const char* name);

/* Diagnostics (layer-by-layer tests): copy the stored output map of executed
 * layer `layer` (0 = first conv, up to the last body conv before the one that
 * carries the head) of the most recent cnn_infer on this handle into dst
 * (device, dst_bytes), in its stored layout: FP32 maps NHWC [z][y][x][c]
 * float32; BF16 / FP8 maps channel-blocked [z][c/16][y][x][16] bf16 values /
 * e4m3fn codes (x fastest), before the max filter that the next layer applies.
 * shape_out (host int64[4]) receives {Z, C, h, w}, also when dst_bytes is too
 * small (CNN_EINVAL, nothing copied). The last cnn_infer must have
 * run as one slab (the volume fit the workspace) and the map must be row-major
 * (not a stride-2 pool net, not a first layer computed inside layer 1);
 * CNN_EINVAL / CNN_EUNSUPPORTED otherwise. Only enqueues the copy. */
int cnn_read_activation(cnn_net* net, int32_t layer, void* dst, int64_t dst_bytes, int64_t shape_out[4],
                        void* stream);

/* Describe the current tile choice (for logs); writes a NUL-terminated string. */
int cnn_describe(const cnn_net* net, char* buf, int32_t buf_len);

/* ------------------------------------------------------------------------
 * Student network and fallback (Section 1 / 2: a fast pass everywhere and
 * extra effort only where errors are likely). The student is a thinner net,
 * conv5x5 1->8 ReLU, conv3x3 8->8 ReLU, conv1x1 8->1 sigmoid (R = 6), trained
 * on the GPU by distillation from the plain net's probability maps.
 * ---------------------------------------------------------------------- */
typedef struct cnn_student cnn_student;

typedef struct cnn_adam {
  float lr, beta1, beta2, eps;
} cnn_adam;

/* w_init: host float64 parameters in the cnn_create layout (801 values).
 * precision: CNN_PREC_FP32 or CNN_PREC_BF16 (forward and backward operands
 * rounded to bf16, FP32 accumulation, FP32 master weights and Adam state). */
int student_create(const double* w_init, int64_t n_weights, int32_t precision,
                   cnn_student** out);
int student_destroy(cnn_student* s);

/* Copy the FP32 master parameters (as float64) / Adam moments / step count to
 * host. Any pointer may be NULL. Synchronous. */
int student_get_state(cnn_student* s, double* w_out, double* m_out, double* v_out,
                      int64_t* step_out);
/* Restore a saved state (resume). Synchronous. */
int student_set_state(cnn_student* s, const double* w, const double* m, const double* v,
                      int64_t step);

/* Gradient of the mean BCE-with-logits L = mean(softplus(z) - t z) over
 * batch x (P-6) x (P-6) outputs. patches: device batch x P x P uint8;
 * teacher_prob: device batch x (P-6) x (P-6) float32 targets in [0,1].
 * grad_out: device float32[801]; loss_out: device float64 scalar (nullable).
 * The loss and gradient reductions are deterministic (fixed order). */
int student_grad(cnn_student* s, const uint8_t* patches, const float* teacher_prob,
                 int32_t batch, int32_t patch, float* grad_out, double* loss_out, void* stream);

/* One source patch of a training batch: a device volume Z x H x W uint8, its
 * teacher map Z x (H-R) x (W-R) float32 (R: the teacher's radius) and the
 * patch origin (z, y, x) in the volume. */
typedef struct cnn_patch_src {
  const uint8_t* volume;
  const float* teacher;
  int64_t Z, H, W;
  int32_t z, y, x;
} cnn_patch_src;

/* Gather a training batch on the device (distillation from the plain net's
 * maps): patches_out[b] = volume[z, y : y+P, x : x+P] and teacher_out[b] =
 * teacher[z, y-m : y-m+P-6, x-m : x-m+P-6] with m = (R-6)/2, i.e. the
 * teacher probabilities centred on the student's (P-6) x (P-6) outputs.
 * src: host array of `batch` (1..64) sources, read during the call; every
 * origin must satisfy m <= y <= H-P-m and m <= x <= W-P-m.
 * patches_out: device batch x P x P uint8; teacher_out: device
 * batch x (P-6) x (P-6) float32. Only enqueues the copy. */
int student_gather(const cnn_patch_src* src, int32_t batch, int32_t patch, int32_t teacher_R,
                   uint8_t* patches_out, float* teacher_out, void* stream);

/* One training step: forward, loss (FP64 sum), backward, FP64 squared gradient
 * norm, Adam update (Kingma & Ba, bias-corrected) of the FP32 master weights.
 * loss_out, gnorm_out: device float64 scalars (nullable); gnorm is ||g||_2. */
int student_train_step(cnn_student* s, const uint8_t* patches, const float* teacher_prob,
                       int32_t batch, int32_t patch, const cnn_adam* hp, double* loss_out,
                       double* gnorm_out, void* stream);

/* Student inference: volume Z x H x W -> Z x (H-6) x (W-6) float32. */
int student_infer(cnn_student* s, const uint8_t* volume_u8, const int64_t dims[3],
                  float* prob_out, void* stream);

/* Student inference aligned to the teacher's output frame, with per-tile
 * fallback to the teacher (a multi-pass scheme: cheap pass everywhere,
 * expensive pass where sampled disagreement is high).
 * prob_out: device, Z x (H-R) x (W-R) float32 with R the teacher's radius (the
 * student map cropped by (R-6)/2 per side).
 * The output of each slice is split into tiles of tile x tile pixels, numbered
 * t = (z * ty + a) * tx + b for tile row a < ty = ceil((H-R) / tile) and tile
 * column b < tx = ceil((W-R) / tile); a tile at the lower or right edge keeps
 * its th x tw in-bounds pixels. In each tile, n_samples windows of
 * wh x ww = min(16, th) x min(16, tw) outputs are recomputed by the teacher.
 * Window k of tile t starts at tile offset (r mod (th - wh + 1),
 * (r >> 32) mod (tw - ww + 1)) with r = m(seed ^ m(64 t + k)), where m is the
 * splitmix64 output mix (Steele, Lea and Flood 2014) applied to
 * x + 0x9e3779b97f4a7c15 (64-bit wrap-around). Windows may overlap; every
 * sampled voxel counts once per window. A voxel flips when its decisions
 * p >= 0.5 differ between the student and the teacher. A tile whose flip count
 * exceeds tau times its sampled-voxel count (flips > tau * count, in float32)
 * is recomputed by the teacher; tau < 0: every tile, tau >= 1: none.
 * Decisions stay on the device and the call only enqueues work (its pinned
 * window table is reused once the previous call's upload has run).
 * stats_out (device int32[2], nullable): {tiles flagged, tiles total}.
 * flags_out (device int32[Z * ty * tx], nullable): per tile t, 1 if it was
 * recomputed by the teacher, else 0. */
int student_infer_with_fallback(cnn_student* s, cnn_net* teacher, const uint8_t* volume_u8,
                                const int64_t dims[3], float* prob_out, float tau,
                                int32_t tile, int32_t n_samples, uint64_t seed,
                                int32_t* stats_out, int32_t* flags_out, void* stream);

/* ------------------------------------------------------------------------
 * 3-D watershed (Section 2.1: the membrane map is turned into an
 * over-segmentation by a 3-D watershed before agglomeration).
 * ---------------------------------------------------------------------- */

/* Watershed by steepest descent with seeded minima, in 3-D with 6-neighbours:
 * voxels are ordered by (p, index), index = (z H + y) W + x; seeds are the
 * voxels with p < seed_threshold, grouped into 6-connected components labelled
 * 1 + the least index in each; every other voxel descends to the least of
 * itself and its neighbours until it reaches a seed (and takes its
 * component's label) or a local minimum of the order m (label 1 + index(m)).
 * The labelling is unique; it is an over-segmentation whose seeded basins are
 * the cells when the map separates them.
 * prob: device Z x H x W float32, finite; labels_out: device int32, same
 * shape; work: device int32[Z H W + 1] scratch (caller-owned, overwritten;
 * its last word is not used); Z H W < 2^31 - 1. The call only enqueues three
 * kernels on `stream` (descent pointers, one lock-free union-find pass over
 * the seeds, root finding with path halving) and never waits on the host. */
int watershed_3d(const float* prob, const int64_t dims[3], float seed_threshold, int32_t* labels_out,
                 int32_t* work, void* stream);

/* ------------------------------------------------------------------------
 * Diagnostics: the matrix-core instructions the conv kernels use, for tests
 * of their arithmetic and for a measured throughput ceiling.
 * ---------------------------------------------------------------------- */

/* D = sum over c < chain of A_c B_c for ntiles independent 16 x 16 output
 * tiles, with the instruction a conv of `precision` uses per operand chunk
 * (FP32: four 16x16x4 f32 MFMAs; BF16: one 16x16x32 bf16; FP8: one
 * 16x16x128 f8f6f4 with e4m3fn operands and unit block scales), each step
 * accumulating onto the previous result from zero, as over a conv's K steps.
 * a, b: device, ntiles x chain x 64 lanes x 16 bytes (FP8: 32); lane
 * (g, n) = (lane / 16, lane % 16) holds its k-slot g bytes of row n of A and
 * column n of B; byte t of a lane's A bytes meets byte t of the matching B
 * lane, so A_c B_c [m][n] = sum over g, t of A(16 g + m)[t] B(16 g + n)[t].
 * d: device, ntiles x 64 lanes x 4 float32; lane (g, n) receives D[4g + k][n]
 * in element k. 1 <= chain <= 64. Only enqueues. */
int cnn_mfma_probe(int32_t precision, const void* a, const void* b, float* d, int32_t ntiles,
                   int32_t chain, void* stream);

/* MFMA throughput of `precision`'s instruction: `blocks` workgroups of 4 waves,
 * each wave running iters x 8 MFMAs on register operands read from ops (device,
 * at least 256 x 2 x 64 x 32 bytes of the caller's data, e.g. random codes),
 * after a shorter warm-up launch. Writes the algorithmic TFLOP/s over the
 * timed launch (HIP events) and the mean shader clock in MHz that the waves
 * ran at (s_memtime cycles over s_memrealtime's 100 MHz ticks). Synchronous;
 * allocates its own small result buffers. */
int cnn_mfma_bench(int32_t precision, int32_t blocks, int32_t iters, const void* ops, double* tflops,
                   double* mhz, void* stream);

/* Thread-local text of the last error on this thread ("" if none). */
const char* cnn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EMCNN_H */
