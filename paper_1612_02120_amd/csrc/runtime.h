// Host-side objects of the library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"

namespace emcnn {

// One executed conv layer. A 2x2/s1 max filter before it is folded into its
// staging (pool_in); the 1x1 sigmoid head after the last body conv is folded
// into that conv's epilogue (head).
struct ExecLayer {
  int first = 0;  // 1: the uint8 first layer (conv_first kernel)
  int cin = 0, cout = 0, ks = 0;
  int pool_in = 0, head = 0;
  int in_off = 0;  // receptive radius consumed by earlier layers
  // nets with stride-2 pools, in their dense form: the conv taps are dil apart
  // and the 2x2 max filter before the conv (pool_in) takes elements pd apart
  int dil = 1, pd = 1;
  int epi = 0;     // epilogue kind (VariantInfo::epi; first layers: 1 = max-out)
  // the output map is stored fragment-major modulo 2^out_lg (the spacing of
  // the conv that reads it; 0: row-major), see LayerJob::geom
  int out_lg = 0;
  int cstore = 0;  // channels stored per output pixel: cout, or cout / 2 after max-out
  int stride = 1;  // output stride of a first layer (2: only where a 2x subsample keeps pixels)
  int spaced = 0;  // conv of a stride-2 pool net: tiled per phase, max-filter spacing from the job
  int variant = -1;
  std::vector<int> candidates;
  std::vector<void*> wpacks;  // packed weights per candidate (layouts differ between variants)
  void* wpack = nullptr;      // == wpacks[index of variant in candidates]
  float* bias = nullptr;
  float* oscale = nullptr;
  float* head_w = nullptr;
  float head_b = 0.f;
  float out_inv_scale = 1.f;
};

// Stored geometry of a layer's h x w output map in pixels: row stride rs and
// slice size zs. A fragment-major map (out_lg > 0) holds D^2 fragments of
// ceil(h / D) x ceil(w / D) pixels each, D = 2^out_lg.
inline void map_strides(const ExecLayer& L, int64_t h, int64_t w, int64_t& rs, int64_t& zs) {
  const int64_t D = (int64_t)1 << L.out_lg, hq = (h + D - 1) / D, wq = (w + D - 1) / D;
  rs = wq;
  zs = D * D * hq * wq;
}

struct Net {
  int device = 0;
  int prec = 0;
  int R = 0;
  int out_stride = 1;  // 2 for nets with a 2x subsample: output (y, x) is the window at input (2y, 2x)
  int in_channels = 1;  // > 1: the input is real-valued maps, NHWC float32 (cnn_infer_maps)
  int in_elb = 1;       // bytes per input pixel: 1 (uint8) or 4 in_channels
  int num_cus = 256;
  std::string arch;
  std::vector<ExecLayer> layers;
  // workspace for inter-layer activations (grown on demand)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_budget = (size_t)24 << 30;
  // batched submissions: two job-table arenas used in turn, so a submission
  // waits on the host only for the one two calls back (still reading its
  // pinned table) and never for the previous one
  struct Arena {
    void* tab_dev = nullptr;
    size_t tab_dev_bytes = 0;
    void* tab_host = nullptr;  // pinned
    size_t tab_host_bytes = 0;
    hipGraphExec_t graph_exec = nullptr;  // captured submission reading this arena
    std::vector<unsigned char> graph_key;
    hipEvent_t done = nullptr;  // recorded behind the arena's last submission
    bool done_pending = false;
  };
  Arena arena[2];
  int cur = 0;  // arena of the submission being planned
  hipStream_t cap_stream = nullptr;
  // geometry of the last run_volume (for cnn_read_activation): dims, slices per
  // slab and the byte offset of the odd-layer half of the workspace
  int64_t last_Z = 0, last_H = 0, last_W = 0, last_zslab = 0;
  size_t last_half = 0;
  int use_graph = 1;
  // optional per-layer timing: events recorded on the launch stream around
  // every layer kernel while enabled
  int profiling = 0;
  struct Timed {
    int layer;
    hipEvent_t a, b;
  };
  std::vector<Timed> timed;
  std::vector<hipEvent_t> event_pool;
  // per tile class (kTileClasses), the variant of every layer that batched
  // submissions use for that class's tiles; empty: the selected variants
  std::vector<std::vector<int>> class_variants;
};

// Tile classes of the batched form, by the smaller output side of a tile:
// representative sides 64, 128, 256, 512, 1024 (class edges at their
// geometric means).
constexpr int kTileClasses = 5;
inline int tile_class(int64_t side) {
  const int64_t edges[kTileClasses - 1] = {91, 181, 362, 724};
  int c = 0;
  while (c < kTileClasses - 1 && side >= edges[c]) ++c;
  return c;
}
inline int tile_class_side(int c) { return 64 << c; }

// Conv output dims of every executed layer for an input region of h x w.
struct Dims {
  std::vector<int> hin, win, hout, wout;
};

// A 3-D input region of a uint8 volume (strided) and where its dense output
// goes. h, w are the input dims; the output is (h-R) x (w-R) per slice.
struct Region {
  const uint8_t* in;
  int64_t in_rs, in_zs;
  int z, h, w;
  float* out;
  int64_t out_rs, out_zs;
  const int32_t* gate;
};

struct Launch {
  int layer;
  int grid;
  JobSet js;
  // the layer's variant (and its packed weights) when the launch was planned;
  // batches plan tile classes with different variants
  int variant = -1;
  void* wpack = nullptr;
};
// Launch la with the variant it was planned with.
int launch_planned(Net* net, const Launch& la, hipStream_t st);

Dims layer_dims(const Net* net, int h, int w);
inline int stored_channels(const ExecLayer& L) { return L.cstore ? L.cstore : L.cout; }
int ensure_ws(Net* net, size_t need);
int run_volume(Net* net, const uint8_t* vol, int64_t Z, int64_t H, int64_t W, float* prob, hipStream_t st);
int arena_reserve(Net* net, size_t njobs);
size_t count_region_jobs(const Net* net, const std::vector<Region>& regs);
// Plan the regions' launches into the job arena from job_off on; ws_need
// receives the workspace bytes they need, which this call allocates (growing
// frees the previous workspace). dry: compute ws_need only, write nothing.
int plan_regions(Net* net, const std::vector<Region>& regs, size_t job_off, std::vector<Launch>& launches,
                 size_t& njobs_used, size_t& ws_need, bool dry = false);
int submit(Net* net, const std::vector<Launch>& launches, size_t job_off, size_t njobs, hipStream_t st, bool graph);
int launch_layer(Net* net, const ExecLayer& L, const JobSet& js, int grid, hipStream_t st, bool timed = true);
int check_device(const Net* net);

int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
void clear_error();
const char* last_error();

float bf16_rne(float x);
uint8_t e4m3_code(double x);

int layer_threads(const ExecLayer& L);
int layer_ty(const ExecLayer& L);
int layer_tx(const ExecLayer& L);
bool layer_phase_groups(const ExecLayer& L);  // work items are groups of four phases (head_taps4)
const void* layer_fn(const ExecLayer& L);
const char* layer_name(const ExecLayer& L);
int persistent_grid(Net* net, const ExecLayer& L, int64_t total_items);
// Select candidate `variant` of layer L (binds its packed weights).
bool select_variant(ExecLayer& L, int variant);
// True when layer 1 runs a fused variant: it reads the uint8 input and computes
// layer 0 itself, so layer 0 is not launched and has no output buffer.
bool first_fused(const Net* net);

}  // namespace emcnn
