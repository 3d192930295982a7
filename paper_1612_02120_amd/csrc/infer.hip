// Work planning and launches for cnn_infer / cnn_infer_batch and the
// teacher passes of the student fallback.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/emcnn.h"
#include "common.h"
#include "runtime.h"

namespace emcnn {

static int act_bytes_of(int prec) { return prec == F32 ? 4 : prec == BF16 ? 2 : 1; }

Dims layer_dims(const Net* net, int h, int w) {
  Dims d;
  for (const auto& L : net->layers) {
    d.hin.push_back(h);
    d.win.push_back(w);
    const int shrink = (L.pool_in ? L.pd : 0) + (L.ks - 1) * L.dil;
    // a strided first layer is evaluated at every stride-th position only
    h = (h - shrink - 1) / L.stride + 1;
    w = (w - shrink - 1) / L.stride + 1;
    d.hout.push_back(h);
    d.wout.push_back(w);
  }
  return d;
}

// Bytes per slice of each layer's stored output (0 for the head layer, and
// for a first layer that the next layer computes itself).
static std::vector<size_t> layer_bytes(const Net* net, const Dims& d) {
  std::vector<size_t> b;
  const int nl = (int)net->layers.size();
  const bool fused = first_fused(net);
  for (int l = 0; l < nl; ++l) {
    int64_t rs, zs;
    map_strides(net->layers[l], d.hout[l], d.wout[l], rs, zs);
    b.push_back(l == nl - 1 || (l == 0 && fused)
                    ? 0
                    : (size_t)zs * stored_channels(net->layers[l]) * act_bytes_of(net->prec));
  }
  return b;
}

int ensure_ws(Net* net, size_t need) {
  if (need <= net->ws_bytes) return CNN_OK;
  hipError_t e;
  if (net->ws) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "workspace grow: sync");
    hipFree(net->ws);
    net->ws = nullptr;
    net->ws_bytes = 0;
  }
  need = (need + (1 << 20) - 1) & ~(size_t)((1 << 20) - 1);
  if ((e = hipMalloc(&net->ws, need)) != hipSuccess) {
    net->ws = nullptr;
    return fail(CNN_ENOMEM, std::string("workspace hipMalloc(") + std::to_string(need) + "): " + hipGetErrorString(e));
  }
  net->ws_bytes = need;
  return CNN_OK;
}

static LayerJob make_job(const ExecLayer& L, const void* in, void* out, int z, int hin, int win, int64_t in_rs,
                         int64_t in_zs, int hout, int wout, int64_t out_rs, int64_t out_zs, int64_t item0,
                         const int32_t* gate) {
  LayerJob j;
  std::memset(&j, 0, sizeof(j));
  j.in = in;
  j.out = out;
  j.z = z;
  j.hin = hin;
  j.win = win;
  j.in_rs = in_rs;
  j.in_zs = in_zs;
  j.hout = hout;
  j.wout = wout;
  j.out_rs = out_rs;
  j.out_zs = out_zs;
  if (L.spaced && !L.first) {
    // d^2 phase sub-lattices, each tiled on its own (the largest phase has
    // ceil(hout / d) x ceil(wout / d) positions)
    const int d = L.dil, hs = (hout + d - 1) / d, wsub = (wout + d - 1) / d;
    // kernels over phase groups (four phases whose max filters share fragments) tile d^2 / 4 groups
    const int phases = layer_phase_groups(L) ? d * d / 4 : d * d;
    j.tiles_x = (wsub + layer_tx(L) - 1) / layer_tx(L);
    j.tiles_y = phases * ((hs + layer_ty(L) - 1) / layer_ty(L));
    j.geom = d | (L.pd << 8) | (L.out_lg << 16);
  } else {
    j.geom = L.out_lg << 16;
    j.tiles_x = (wout + layer_tx(L) - 1) / layer_tx(L);
    j.tiles_y = (hout + layer_ty(L) - 1) / layer_ty(L);
  }
  j.item0 = item0;
  j.gate = gate;
  return j;
}

static int64_t job_items(const LayerJob& j) { return (int64_t)j.z * j.tiles_y * j.tiles_x; }

static hipEvent_t pool_event(Net* net) {
  if (!net->event_pool.empty()) {
    hipEvent_t e = net->event_pool.back();
    net->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int launch_layer(Net* net, const ExecLayer& L, const JobSet& js, int grid, hipStream_t st, bool timed) {
  const void* fn = layer_fn(L);
  hipError_t e;
  Net::Timed tm{(int)(&L - net->layers.data()), nullptr, nullptr};
  timed = timed && net->profiling;
  if (timed) {
    tm.a = pool_event(net);
    tm.b = pool_event(net);
    if (tm.a) hipEventRecord(tm.a, st);
  }
  if (L.first) {
    FirstParams p;
    p.w = reinterpret_cast<const float*>(L.wpack);
    p.bias = L.bias;
    p.out_inv_scale = L.out_inv_scale;
    p.pad_ = 0.f;
    void* args[] = {(void*)&js, (void*)&p};
    e = hipLaunchKernel(fn, dim3(grid), dim3(layer_threads(L)), args, 0, st);
  } else {
    ConvParams p;
    std::memset(&p, 0, sizeof(p));
    p.wpack = L.wpack;
    p.bias = L.bias;
    p.oscale = L.oscale;
    p.head_w = L.head_w;
    p.head_b = L.head_b;
    p.out_inv_scale = L.out_inv_scale;
    if (conv_variant(L.variant)->fused) {
      const ExecLayer& L0 = net->layers[0];
      p.w1 = L0.wpack;
      p.b1 = L0.bias;
      p.w1_inv_scale = L0.out_inv_scale;
    }
    void* args[] = {(void*)&js, (void*)&p};
    e = hipLaunchKernel(fn, dim3(grid), dim3(layer_threads(L)), args, 0, st);
  }
  if (e != hipSuccess) return hip_fail(e, layer_name(L));
  if (timed && tm.a && tm.b) {
    hipEventRecord(tm.b, st);
    net->timed.push_back(tm);
  }
  return CNN_OK;
}

// Every layer of one region (zc slices of an h x w input window of the
// volume, row stride in_rs and slice stride in_zs; output window at prob with
// strides out_rs / out_zs) as one persistent launch per layer with the job
// passed by value; inter-layer maps alternate between buf0 and buf1.
static int run_region(Net* net, const uint8_t* in, int64_t in_rs, int64_t in_zs, int zc, int h, int w, float* prob,
                      int64_t out_rs, int64_t out_zs, unsigned char* buf0, unsigned char* buf1, hipStream_t st,
                      bool timed) {
  const Dims d = layer_dims(net, h, w);
  const int nl = (int)net->layers.size();
  const bool fused = first_fused(net);
  unsigned char* buf[2] = {buf0, buf1};
  for (int l = fused ? 1 : 0; l < nl; ++l) {
    const ExecLayer& L = net->layers[l];
    // a fused layer 1 reads the uint8 input with layer 0's geometry
    const int li = (l == 1 && fused) ? 0 : l;
    const void* lin = (li == 0) ? (const void*)in : (const void*)buf[(l - 1) % 2];
    void* out = (l == nl - 1) ? (void*)prob : (void*)buf[l % 2];
    int64_t lin_rs = in_rs, lin_zs = in_zs, lout_rs = out_rs, lout_zs = out_zs;
    if (li > 0) map_strides(net->layers[li - 1], d.hin[li], d.win[li], lin_rs, lin_zs);
    if (l < nl - 1) map_strides(L, d.hout[l], d.wout[l], lout_rs, lout_zs);
    LayerJob j = make_job(L, lin, out, zc, d.hin[li], d.win[li], lin_rs, lin_zs, d.hout[l], d.wout[l], lout_rs,
                          lout_zs, 0, nullptr);
    JobSet js;
    std::memset(&js, 0, sizeof(js));
    js.njobs = 1;
    js.total_items = job_items(j);
    js.single = j;
    const int rc = launch_layer(net, L, js, persistent_grid(net, L, js.total_items), st, timed);
    if (rc) return rc;
  }
  return CNN_OK;
}

// Inter-layer bytes (both parity halves) of a zc-slice region of h x w input.
static void region_bytes(const Net* net, int h, int w, size_t& b0, size_t& b1) {
  const std::vector<size_t> lb = layer_bytes(net, layer_dims(net, h, w));
  b0 = b1 = 0;
  for (size_t l = 0; l < lb.size(); ++l) (l % 2 ? b1 : b0) = std::max((l % 2 ? b1 : b0), lb[l]);
}

// A whole volume: slabs of slices sized so the two inter-layer buffers stay
// within the workspace budget; one persistent launch per layer per slab.
int run_volume(Net* net, const uint8_t* vol, int64_t Z, int64_t H, int64_t W, float* prob, hipStream_t st) {
  size_t b0 = 0, b1 = 0;
  region_bytes(net, (int)H, (int)W, b0, b1);
  const size_t per = std::max<size_t>(1, b0 + b1);
  int64_t zs = std::max<int64_t>(1, std::min<int64_t>(Z, (int64_t)(net->ws_budget / per)));
  int rc = ensure_ws(net, zs * (b0 + b1));
  if (rc) return rc;
  unsigned char* buf0 = reinterpret_cast<unsigned char*>(net->ws);
  unsigned char* buf1 = buf0 + zs * b0;
  const Dims d = layer_dims(net, (int)H, (int)W);
  const int64_t Ho = d.hout.back(), Wo = d.wout.back();
  net->last_Z = Z;
  net->last_H = H;
  net->last_W = W;
  net->last_zslab = zs;
  net->last_half = zs * b0;
  for (int64_t z0 = 0; z0 < Z; z0 += zs) {
    const int zc = (int)std::min<int64_t>(zs, Z - z0);
    rc = run_region(net, vol + z0 * H * W * net->in_elb, W, H * W, zc, (int)H, (int)W, prob + z0 * Ho * Wo, Wo,
                    Ho * Wo, buf0, buf1, st, true);
    if (rc) return rc;
  }
  return CNN_OK;
}

// ------------------------------------------------------------------ static scratch

// The inter-layer maps of cnn_infer_noalloc live in this file-scope device
// array; each device holds its own copy, reached through the address that
// hipGetSymbolAddress returns on that device (never the host-side name).
static __device__ __align__(256) unsigned char scratch[CNN_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

static int scratch_ptr(int device, unsigned char** out) {
  if (device < 0 || device >= 64) return fail(CNN_EUNSUPPORTED, "cnn_infer_noalloc: device index >= 64");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "cnn_infer_noalloc: hipGetSymbolAddress(scratch)");
    if (!p) return fail(CNN_EHIP, "cnn_infer_noalloc: null scratch address");
    g_scratch_ptr[device] = p;
  }
  *out = reinterpret_cast<unsigned char*>(g_scratch_ptr[device]);
  return CNN_OK;
}

// Input rows that produce hs output rows (field of view R + 1; a net with a
// 2x subsample advances two input rows per output row).
static int64_t strip_rows(const Net* net, int64_t hs) { return net->out_stride * (hs - 1) + net->R + 1; }

// The volume as regions that fit the static scratch: slabs of whole slices
// when one slice fits, otherwise strips of output rows (a multiple of 16, so
// that every phase lattice of a stride-2 pool net starts at the same parity
// as in the whole slice) with R rows of input overlap. Results are bitwise
// those of run_volume: each output voxel takes the same arithmetic in the same
// order whatever region holds it.
int plan_static(const Net* net, int64_t Z, int64_t H, int64_t W, size_t cap, int64_t& zslab, int64_t& strip) {
  size_t b0 = 0, b1 = 0;
  region_bytes(net, (int)H, (int)W, b0, b1);
  if (b0 + b1 <= cap) {
    zslab = std::max<int64_t>(1, std::min<int64_t>(Z, (int64_t)(cap / std::max<size_t>(1, b0 + b1))));
    strip = layer_dims(net, (int)H, (int)W).hout.back();
    return CNN_OK;
  }
  zslab = 1;
  const int64_t Ho = layer_dims(net, (int)H, (int)W).hout.back();
  int64_t lo = 0;
  for (int64_t hs = 16; hs < Ho; hs *= 2) {  // largest power-of-two multiple of 16 that fits, then refine
    region_bytes(net, (int)strip_rows(net, hs), (int)W, b0, b1);
    if (b0 + b1 > cap) break;
    lo = hs;
  }
  if (lo == 0)
    return fail(CNN_EINVAL, "cnn_infer_noalloc: a 16-row strip of width " + std::to_string(W) +
                                " needs more than the static scratch (" + std::to_string(cap) + " bytes)");
  for (int64_t step = lo / 2; step >= 16; step /= 2) {
    region_bytes(net, (int)strip_rows(net, lo + step), (int)W, b0, b1);
    if (lo + step < Ho && b0 + b1 <= cap) lo += step;
  }
  strip = lo;
  return CNN_OK;
}

// ------------------------------------------------------------------ regions

// Switch to the other job-table arena, wait until the submission that last
// used it no longer reads its pinned table, then make it hold `njobs` jobs
// (host and device copies).
int arena_reserve(Net* net, size_t njobs) {
  hipError_t e;
  net->cur ^= 1;
  Net::Arena& A = net->arena[net->cur];
  if (A.done_pending) {
    if ((e = hipEventSynchronize(A.done)) != hipSuccess) return hip_fail(e, "wait for the arena's last submission");
    A.done_pending = false;
  }
  const size_t bytes = std::max<size_t>(1, njobs) * sizeof(LayerJob);
  if (A.tab_host_bytes < bytes) {
    if (A.tab_host) hipHostFree(A.tab_host);
    A.tab_host = nullptr;
    A.tab_host_bytes = 0;
    if ((e = hipHostMalloc(&A.tab_host, bytes)) != hipSuccess) return fail(CNN_ENOMEM, "pinned job table");
    A.tab_host_bytes = bytes;
  }
  if (A.tab_dev_bytes < bytes) {
    if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "job table grow: sync");
    if (A.tab_dev) hipFree(A.tab_dev);
    A.tab_dev = nullptr;
    A.tab_dev_bytes = 0;
    if ((e = hipMalloc(&A.tab_dev, bytes)) != hipSuccess) return fail(CNN_ENOMEM, "device job table");
    A.tab_dev_bytes = bytes;
    if (A.graph_exec) hipGraphExecDestroy(A.graph_exec);
    A.graph_exec = nullptr;
    A.graph_key.clear();
  }
  if (!A.done) {
    if ((e = hipEventCreateWithFlags(&A.done, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreate");
  }
  return CNN_OK;
}

// Split regions whose slices alone exceed the budget, then group regions so a
// group's inter-layer buffers fit the workspace budget. Writes one job per
// (group, layer, region) into the arena from `job_off` on and appends the
// launches. Returns the workspace bytes needed in ws_need.
int plan_regions(Net* net, const std::vector<Region>& in_regions, size_t job_off, std::vector<Launch>& launches,
                 size_t& njobs_used, size_t& ws_need, bool dry) {
  const int nl = (int)net->layers.size();
  // per-region geometry; regions with too many slices are split by z
  std::vector<Region> regs;
  std::vector<Dims> dims;
  std::vector<std::vector<size_t>> lbs;
  for (const Region& r0 : in_regions) {
    Dims d = layer_dims(net, r0.h, r0.w);
    std::vector<size_t> lb = layer_bytes(net, d);
    size_t per = 0;
    for (size_t x : lb) per += x;
    int64_t zmax = std::max<int64_t>(1, (int64_t)(net->ws_budget / std::max<size_t>(per, 1)));
    for (int z0 = 0; z0 < r0.z; z0 += (int)zmax) {
      Region r = r0;
      r.z = (int)std::min<int64_t>(zmax, r0.z - z0);
      r.in = r0.in + (int64_t)z0 * r0.in_zs;
      r.out = r0.out + (int64_t)z0 * r0.out_zs;
      regs.push_back(r);
      dims.push_back(d);
      lbs.push_back(lb);
    }
  }
  const int n = (int)regs.size();
  std::vector<size_t> b0(n), b1(n);
  for (int t = 0; t < n; ++t) {
    b0[t] = b1[t] = 0;
    for (int l = 0; l < nl; ++l) (l % 2 ? b1[t] : b0[t]) += lbs[t][l] * regs[t].z;
  }
  std::vector<std::pair<int, int>> groups;
  ws_need = 0;
  {
    int g0 = 0;
    size_t s0 = 0, s1 = 0;
    for (int t = 0; t < n; ++t) {
      if (t > g0 && s0 + s1 + b0[t] + b1[t] > net->ws_budget) {
        groups.push_back({g0, t});
        ws_need = std::max(ws_need, s0 + s1);
        g0 = t;
        s0 = s1 = 0;
      }
      s0 += b0[t];
      s1 += b1[t];
    }
    groups.push_back({g0, n});
    ws_need = std::max(ws_need, s0 + s1);
  }
  if (dry) return CNN_OK;  // only the workspace size was asked for
  const size_t need_jobs = job_off + (size_t)n * nl;
  Net::Arena& A = net->arena[net->cur];
  if (need_jobs * sizeof(LayerJob) > A.tab_host_bytes) return fail(CNN_EINVAL, "internal: job arena too small");
  // growing the workspace frees the old one: jobs planned earlier into it (by
  // a caller that plans several region lists before submitting) would be
  // left pointing at freed memory, so such callers size the workspace first
  // with dry runs (see the fallback in student.hip)
  int rc = ensure_ws(net, ws_need);
  if (rc) return rc;
  LayerJob* tab = reinterpret_cast<LayerJob*>(A.tab_host);
  size_t pos = job_off;
  for (auto& G : groups) {
    size_t half0 = 0;
    for (int t = G.first; t < G.second; ++t) half0 += b0[t];
    unsigned char* base0 = reinterpret_cast<unsigned char*>(net->ws);
    unsigned char* base1 = base0 + half0;
    std::vector<unsigned char*> r0(n), r1(n);
    {
      size_t a = 0, b = 0;
      for (int t = G.first; t < G.second; ++t) {
        r0[t] = base0 + a;
        r1[t] = base1 + b;
        a += b0[t];
        b += b1[t];
      }
    }
    const bool fused = first_fused(net);
    for (int l = fused ? 1 : 0; l < nl; ++l) {
      const ExecLayer& L = net->layers[l];
      const size_t first = pos;
      int64_t item0 = 0;
      for (int t = G.first; t < G.second; ++t) {
        const Region& R = regs[t];
        const Dims& d = dims[t];
        // output of layer q lives in half q % 2 after earlier layers of that parity
        auto buf_of = [&](int q) -> unsigned char* {
          size_t off = 0;
          for (int p = q % 2; p < q; p += 2) off += lbs[t][p] * R.z;
          return (q % 2 ? r1[t] : r0[t]) + off;
        };
        const void* in;
        int64_t in_rs, in_zs;
        const int li = (l == 1 && fused) ? 0 : l;  // a fused layer 1 reads the uint8 input
        if (li == 0) {
          in = R.in;
          in_rs = R.in_rs;
          in_zs = R.in_zs;
        } else {
          in = buf_of(l - 1);
          map_strides(net->layers[l - 1], d.hin[l], d.win[l], in_rs, in_zs);
        }
        void* out;
        int64_t out_rs, out_zs;
        if (l == nl - 1) {
          out = R.out;
          out_rs = R.out_rs;
          out_zs = R.out_zs;
        } else {
          out = buf_of(l);
          map_strides(L, d.hout[l], d.wout[l], out_rs, out_zs);
        }
        LayerJob j = make_job(L, in, out, R.z, d.hin[li], d.win[li], in_rs, in_zs, d.hout[l], d.wout[l], out_rs,
                              out_zs, item0, R.gate);
        item0 += job_items(j);
        tab[pos++] = j;
      }
      Launch la;
      la.layer = l;
      la.variant = L.variant;
      la.wpack = L.wpack;
      std::memset(&la.js, 0, sizeof(la.js));
      la.js.table = reinterpret_cast<const LayerJob*>(A.tab_dev) + first;
      la.js.njobs = (int)(pos - first);
      la.js.total_items = item0;
      la.grid = persistent_grid(net, L, (int64_t)1 << 40);  // full persistent grid: structure-stable
      launches.push_back(la);
    }
  }
  njobs_used = pos - job_off;
  return CNN_OK;
}

size_t count_region_jobs(const Net* net, const std::vector<Region>& regs) {
  // upper bound of the jobs plan_regions writes (regions may split by z)
  const int nl = (int)net->layers.size();
  size_t n = 0;
  for (const Region& r : regs) {
    Dims d = layer_dims(net, r.h, r.w);
    std::vector<size_t> lb = layer_bytes(net, d);
    size_t per = 0;
    for (size_t x : lb) per += x;
    int64_t zmax = std::max<int64_t>(1, (int64_t)(net->ws_budget / std::max<size_t>(per, 1)));
    n += (size_t)((r.z + zmax - 1) / zmax) * nl;
  }
  return n;
}

// Upload the arena's first `njobs` jobs and run the launches, either directly on
// `st` or through a captured graph that is replayed while the structure holds.
int submit(Net* net, const std::vector<Launch>& launches, size_t job_off, size_t njobs, hipStream_t st, bool graph) {
  hipError_t e;
  const size_t tab_bytes = std::max<size_t>(1, njobs) * sizeof(LayerJob);
  Net::Arena& A = net->arena[net->cur];
  void* dsrc = reinterpret_cast<LayerJob*>(A.tab_dev) + job_off;
  const void* hsrc = reinterpret_cast<const LayerJob*>(A.tab_host) + job_off;
  if (!graph) {
    if ((e = hipMemcpyAsync(dsrc, hsrc, tab_bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
      return hip_fail(e, "job table upload");
    for (auto& la : launches) {
      int rc = launch_planned(net, la, st);
      if (rc) return rc;
    }
  } else {
    std::vector<unsigned char> key;
    auto put = [&key](const void* p, size_t b) {
      const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
      key.insert(key.end(), c, c + b);
    };
    put(&tab_bytes, sizeof(tab_bytes));
    put(&job_off, sizeof(job_off));
    for (auto& la : launches) {
      put(&la.layer, sizeof(int));
      put(&la.grid, sizeof(int));
      put(&la.js.table, sizeof(void*));
      put(&la.js.njobs, sizeof(int));
      put(&la.js.total_items, sizeof(int64_t));
      put(&la.variant, sizeof(int));
    }
    if (!A.graph_exec || key != A.graph_key) {
      if (A.graph_exec) hipGraphExecDestroy(A.graph_exec);
      A.graph_exec = nullptr;
      A.graph_key.clear();
      if (!net->cap_stream) {
        if ((e = hipStreamCreateWithFlags(&net->cap_stream, hipStreamNonBlocking)) != hipSuccess)
          return hip_fail(e, "hipStreamCreate");
      }
      if ((e = hipStreamBeginCapture(net->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
      int crc = CNN_OK;
      if ((e = hipMemcpyAsync(dsrc, hsrc, tab_bytes, hipMemcpyHostToDevice, net->cap_stream)) != hipSuccess)
        crc = hip_fail(e, "capture: job table upload");
      for (auto& la : launches) {
        if (crc) break;
        crc = launch_planned(net, la, net->cap_stream);
      }
      hipGraph_t g = nullptr;
      e = hipStreamEndCapture(net->cap_stream, &g);
      if (crc) {
        if (g) hipGraphDestroy(g);
        return crc;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&A.graph_exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        A.graph_exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
      }
      A.graph_key = key;
    }
    if ((e = hipGraphLaunch(A.graph_exec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  if ((e = hipEventRecord(A.done, st)) != hipSuccess) return hip_fail(e, "hipEventRecord");
  A.done_pending = true;
  return CNN_OK;
}

int launch_planned(Net* net, const Launch& la, hipStream_t st) {
  ExecLayer& L = net->layers[la.layer];
  const int v0 = L.variant;
  void* w0 = L.wpack;
  if (la.variant >= 0) {
    L.variant = la.variant;
    L.wpack = la.wpack;
  }
  const int rc = launch_layer(net, L, la.js, la.grid, st);
  L.variant = v0;
  L.wpack = w0;
  return rc;
}

int check_device(const Net* net) {
  int dev = -1;
  hipGetDevice(&dev);
  if (dev != net->device)
    return fail(CNN_EINVAL, "handle was created on device " + std::to_string(net->device) + ", current is " +
                                std::to_string(dev));
  return CNN_OK;
}

}  // namespace emcnn

using namespace emcnn;

extern "C" int cnn_infer(cnn_net* h, const uint8_t* vol, const int64_t dims[3], float* prob, void* stream) {
  clear_error();
  if (!h || !vol || !dims || !prob) return fail(CNN_EINVAL, "cnn_infer: null argument");
  Net* net = reinterpret_cast<Net*>(h);
  if (net->in_channels != 1) return fail(CNN_EINVAL, "cnn_infer: this net reads real-valued maps (cnn_infer_maps)");
  const int64_t Z = dims[0], H = dims[1], W = dims[2];
  if (Z < 1 || H < net->R + 1 || W < net->R + 1)
    return fail(CNN_EINVAL, "cnn_infer: dims smaller than the field of view (" + std::to_string(net->R + 1) + ")");
  if (H >= (1ll << 30) || W >= (1ll << 30) || Z >= (1ll << 30))
    return fail(CNN_EINVAL, "cnn_infer: dims must be < 2^30");
  int rc = check_device(net);
  if (rc) return rc;
  return run_volume(net, vol, Z, H, W, prob, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int cnn_infer_maps(cnn_net* h, const float* maps, const int64_t dims[4], float* prob, void* stream) {
  clear_error();
  if (!h || !maps || !dims || !prob) return fail(CNN_EINVAL, "cnn_infer_maps: null argument");
  Net* net = reinterpret_cast<Net*>(h);
  const int64_t Z = dims[0], H = dims[1], W = dims[2], C = dims[3];
  if (net->in_channels == 1 || C != net->in_channels)
    return fail(CNN_EINVAL, "cnn_infer_maps: the net's first conv takes " + std::to_string(net->in_channels) +
                                " input maps (nets on one uint8 channel use cnn_infer)");
  if (Z < 1 || H < net->R + 1 || W < net->R + 1)
    return fail(CNN_EINVAL, "cnn_infer_maps: dims smaller than the field of view (" + std::to_string(net->R + 1) + ")");
  if (H >= (1ll << 30) || W >= (1ll << 30) || Z >= (1ll << 30))
    return fail(CNN_EINVAL, "cnn_infer_maps: dims must be < 2^30");
  int rc = check_device(net);
  if (rc) return rc;
  return run_volume(net, reinterpret_cast<const uint8_t*>(maps), Z, H, W, prob, reinterpret_cast<hipStream_t>(stream));
}

extern "C" int cnn_infer_noalloc(cnn_net* h, const uint8_t* vol, const int64_t dims[3], float* prob, void* stream) {
  clear_error();
  if (!h || !vol || !dims || !prob) return fail(CNN_EINVAL, "cnn_infer_noalloc: null argument");
  Net* net = reinterpret_cast<Net*>(h);
  if (net->in_channels != 1) return fail(CNN_EUNSUPPORTED, "cnn_infer_noalloc: nets on one uint8 channel only");
  const int64_t Z = dims[0], H = dims[1], W = dims[2];
  if (Z < 1 || H < net->R + 1 || W < net->R + 1)
    return fail(CNN_EINVAL, "cnn_infer_noalloc: dims smaller than the field of view (" + std::to_string(net->R + 1) +
                                ")");
  if (H >= (1ll << 30) || W >= (1ll << 30) || Z >= (1ll << 30))
    return fail(CNN_EINVAL, "cnn_infer_noalloc: dims must be < 2^30");
  int rc = check_device(net);
  if (rc) return rc;
  int64_t zslab = 1, strip = 1;
  rc = plan_static(net, Z, H, W, CNN_NOALLOC_SCRATCH_BYTES, zslab, strip);
  if (rc) return rc;
  unsigned char* base = nullptr;
  rc = scratch_ptr(net->device, &base);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const Dims dv = layer_dims(net, (int)H, (int)W);
  const int64_t Ho = dv.hout.back(), Wo = dv.wout.back();
  for (int64_t z0 = 0; z0 < Z; z0 += zslab) {
    const int zc = (int)std::min<int64_t>(zslab, Z - z0);
    for (int64_t y0 = 0; y0 < Ho; y0 += strip) {
      const int64_t hs = std::min<int64_t>(strip, Ho - y0);
      const int64_t rows = hs == Ho ? H : strip_rows(net, hs);
      size_t b0 = 0, b1 = 0;
      region_bytes(net, (int)rows, (int)W, b0, b1);
      rc = run_region(net, vol + z0 * H * W + net->out_stride * y0 * W, W, H * W, zc, (int)rows, (int)W,
                      prob + z0 * Ho * Wo + y0 * Wo, Wo, Ho * Wo, base, base + zc * b0, st, false);
      if (rc) return rc;
    }
  }
  return CNN_OK;
}

extern "C" int cnn_read_activation(cnn_net* h, int32_t layer, void* dst, int64_t dst_bytes, int64_t* shape,
                                   void* stream) {
  clear_error();
  if (!h || !dst || !shape) return fail(CNN_EINVAL, "cnn_read_activation: null argument");
  Net* net = reinterpret_cast<Net*>(h);
  const int nl = (int)net->layers.size();
  if (layer < 0 || layer >= nl - 1) return fail(CNN_EINVAL, "cnn_read_activation: layer must be a stored map");
  if (net->last_Z < 1 || net->last_zslab < net->last_Z)
    return fail(CNN_EINVAL, "cnn_read_activation: the last cnn_infer did not run as a single slab");
  const ExecLayer& L = net->layers[layer];
  if (L.out_lg != 0 || (layer == 0 && first_fused(net)))
    return fail(CNN_EUNSUPPORTED, "cnn_read_activation: the map is not stored row-major");
  const Dims d = layer_dims(net, (int)net->last_H, (int)net->last_W);
  const int64_t C = stored_channels(L), hh = d.hout[layer], ww = d.wout[layer];
  const int64_t bytes = net->last_Z * C * hh * ww * act_bytes_of(net->prec);
  shape[0] = net->last_Z;
  shape[1] = C;
  shape[2] = hh;
  shape[3] = ww;
  if (dst_bytes < bytes) return fail(CNN_EINVAL, "cnn_read_activation: dst holds fewer than " + std::to_string(bytes) + " bytes");
  const unsigned char* src = reinterpret_cast<const unsigned char*>(net->ws) + (layer % 2 ? net->last_half : 0);
  const hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "cnn_read_activation");
  return CNN_OK;
}

extern "C" int cnn_output_dims(const cnn_net* h, int64_t H, int64_t W, int64_t* Ho, int64_t* Wo) {
  clear_error();
  if (!h || !Ho || !Wo) return fail(CNN_EINVAL, "cnn_output_dims: null argument");
  const Net* net = reinterpret_cast<const Net*>(h);
  if (H < net->R + 1 || W < net->R + 1 || H >= (1ll << 30) || W >= (1ll << 30))
    return fail(CNN_EINVAL, "cnn_output_dims: dims must be >= the field of view and < 2^30");
  const Dims d = layer_dims(net, (int)H, (int)W);
  *Ho = d.hout.back();
  *Wo = d.wout.back();
  return CNN_OK;
}

extern "C" int cnn_set_batch_graph(cnn_net* h, int32_t enable) {
  clear_error();
  if (!h) return fail(CNN_EINVAL, "cnn_set_batch_graph: null net");
  reinterpret_cast<Net*>(h)->use_graph = enable ? 1 : 0;
  return CNN_OK;
}

extern "C" int cnn_set_workspace_limit(cnn_net* h, int64_t bytes) {
  clear_error();
  if (!h || bytes < (1 << 20)) return fail(CNN_EINVAL, "cnn_set_workspace_limit: null net or limit < 1 MiB");
  reinterpret_cast<Net*>(h)->ws_budget = (size_t)bytes;
  return CNN_OK;
}

namespace emcnn {

// Regions of a batch's tiles, the halo surplus beyond R/2 dropped (a tile's
// interior is then exactly the valid output); validates every tile.
static int batch_regions(const Net* net, const cnn_tile* tiles, int32_t n, const char* who, std::vector<Region>& regs) {
  if (net->R % 2 || net->out_stride != 1 || net->in_channels != 1)
    return fail(CNN_EUNSUPPORTED,
                std::string(who) + ": blocks need an odd field of view, a full-resolution output and uint8 input");
  const int R2 = net->R / 2;
  regs.assign(n, Region());
  for (int t = 0; t < n; ++t) {
    const cnn_tile& T = tiles[t];
    if (!T.in || !T.out) return fail(CNN_EINVAL, std::string(who) + ": tile " + std::to_string(t) + " has a null pointer");
    if (T.z < 1 || T.halo < R2 || T.h <= 2 * (int64_t)T.halo || T.w <= 2 * (int64_t)T.halo || T.h >= (1 << 30) ||
        T.w >= (1 << 30) || T.z >= (1 << 30))
      return fail(CNN_EINVAL, std::string(who) + ": tile " + std::to_string(t) + " has bad dims or halo < R/2");
    const int e = T.halo - R2;
    Region& r = regs[t];
    r.in = T.in + (int64_t)e * T.w + e;
    r.in_rs = T.w;
    r.in_zs = T.h * T.w;
    r.z = (int)T.z;
    r.h = (int)(T.h - 2 * e);
    r.w = (int)(T.w - 2 * e);
    r.out = T.out;
    r.out_rs = T.w - 2 * T.halo;
    r.out_zs = (T.h - 2 * T.halo) * (T.w - 2 * T.halo);
    r.gate = nullptr;
  }
  return CNN_OK;
}

// Tile class of a region (its smaller output side).
static int region_class(const Net* net, const Region& r) { return tile_class(std::min(r.h, r.w) - net->R); }

}  // namespace emcnn

extern "C" int cnn_infer_batch(cnn_net* h, const cnn_tile* tiles, int32_t n, void* stream) {
  clear_error();
  if (!h || !tiles || n < 1) return fail(CNN_EINVAL, "cnn_infer_batch: null argument or n < 1");
  Net* net = reinterpret_cast<Net*>(h);
  int rc = check_device(net);
  if (rc) return rc;
  std::vector<Region> regs;
  rc = batch_regions(net, tiles, n, "cnn_infer_batch", regs);
  if (rc) return rc;
  rc = arena_reserve(net, count_region_jobs(net, regs));
  if (rc) return rc;
  std::vector<Launch> launches;
  size_t used = 0, ws_need = 0;
  if (net->class_variants.empty()) {
    rc = plan_regions(net, regs, 0, launches, used, ws_need);
    if (rc) return rc;
  } else {
    // each tile class with its own variants, planned one class after another;
    // classes that chose the same variants share one plan (one launch per
    // layer over all their tiles)
    const int nl = (int)net->layers.size();
    std::vector<std::vector<Region>> byc(kTileClasses);
    for (const Region& r : regs) {
      int c = region_class(net, r);
      for (int k = 0; k < c; ++k)
        if (net->class_variants[k] == net->class_variants[c]) {
          c = k;  // the first class with the same choice
          break;
        }
      byc[c].push_back(r);
    }
    std::vector<int> defaults(nl);
    for (int l = 0; l < nl; ++l) defaults[l] = net->layers[l].variant;
    auto use = [&](const std::vector<int>& v) {
      for (int l = 0; l < nl; ++l) select_variant(net->layers[l], v[l]);
    };
    // the workspace for every class first: growing it while planning a later
    // class would free it under the jobs of an earlier one
    size_t ws_max = 0;
    for (int c = 0; c < kTileClasses && !rc; ++c) {
      if (byc[c].empty()) continue;
      use(net->class_variants[c]);
      std::vector<Launch> none;
      size_t u = 0, wn = 0;
      rc = plan_regions(net, byc[c], 0, none, u, wn, true);
      ws_max = std::max(ws_max, wn);
    }
    use(defaults);
    if (!rc) rc = ensure_ws(net, ws_max);
    if (rc) return rc;
    const void* ws_before = net->ws;
    for (int c = 0; c < kTileClasses && !rc; ++c) {
      if (byc[c].empty()) continue;
      use(net->class_variants[c]);
      size_t u = 0;
      rc = plan_regions(net, byc[c], used, launches, u, ws_need);
      used += u;
    }
    use(defaults);
    if (rc) return rc;
    if (net->ws != ws_before) return fail(CNN_EHIP, "cnn_infer_batch: internal: workspace moved during planning");
  }
  return submit(net, launches, 0, used, reinterpret_cast<hipStream_t>(stream), net->use_graph != 0);
}

// ------------------------------------------------------------------ autotuner

namespace emcnn {

static std::string layer_sig(const Net* net, const ExecLayer& L) {
  return net->arch + "|p" + std::to_string(net->prec) + "|f" + std::to_string(L.first) + "|" + std::to_string(L.cin) +
         "x" + std::to_string(L.cout) + "k" + std::to_string(L.ks) + "p" + std::to_string(L.pool_in) + "h" +
         std::to_string(L.head);
}

static int candidate_name_index(const ExecLayer& L, const std::string& name) {
  for (int c : L.candidates) {
    const char* n = L.first ? first_variant(c)->name : conv_variant(c)->name;
    if (name == n) return c;
  }
  return -1;
}

// One launch of layer l over a single H x W slice region (a fused layer 1
// reads the uint8 input, passed as `in`, with layer 0's geometry).
static int run_one_layer(Net* net, int l, const void* in, void* out, const Dims& d, hipStream_t st) {
  const ExecLayer& L = net->layers[l];
  const int li = (l == 1 && first_fused(net)) ? 0 : l;
  const int nl = (int)net->layers.size();
  int64_t in_rs = d.win[li], in_zs = (int64_t)d.hin[li] * d.win[li], out_rs = d.wout[l],
          out_zs = (int64_t)d.hout[l] * d.wout[l];
  if (li > 0) map_strides(net->layers[li - 1], d.hin[li], d.win[li], in_rs, in_zs);
  if (l < nl - 1) map_strides(L, d.hout[l], d.wout[l], out_rs, out_zs);
  LayerJob j = make_job(L, in, out, 1, d.hin[li], d.win[li], in_rs, in_zs, d.hout[l], d.wout[l], out_rs, out_zs, 0,
                        nullptr);
  JobSet js;
  std::memset(&js, 0, sizeof(js));
  js.njobs = 1;
  js.total_items = job_items(j);
  js.single = j;
  return launch_layer(net, L, js, persistent_grid(net, L, js.total_items), st);
}

}  // namespace emcnn

extern "C" int cnn_autotune(cnn_net* h, int64_t H, int64_t W, const char* cache_path, void* stream) {
  clear_error();
  if (!h) return fail(CNN_EINVAL, "cnn_autotune: null net");
  Net* net = reinterpret_cast<Net*>(h);
  if (H < net->R + 1 || W < net->R + 1 || H > 16384 || W > 16384)
    return fail(CNN_EINVAL, "cnn_autotune: need R+1 <= H, W <= 16384");
  if (net->in_channels != 1) return fail(CNN_EUNSUPPORTED, "cnn_autotune: nets on one uint8 channel only");
  int rc = check_device(net);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nl = (int)net->layers.size();
  const std::string shape = std::to_string(H) + "x" + std::to_string(W);
  // cached choices
  std::vector<std::string> lines;
  std::vector<int> chosen(nl, -1);
  if (cache_path) {
    std::ifstream f(cache_path);
    std::string line;
    while (std::getline(f, line)) {
      lines.push_back(line);
      for (int l = 0; l < nl; ++l) {
        const std::string pre = layer_sig(net, net->layers[l]) + "|" + shape + "|";
        if (line.rfind(pre, 0) == 0) chosen[l] = candidate_name_index(net->layers[l], line.substr(pre.size()));
      }
    }
  }
  bool all = true;
  for (int l = 0; l < nl; ++l)
    if (net->layers[l].candidates.size() > 1 && chosen[l] < 0) all = false;
  if (all) {
    for (int l = 0; l < nl; ++l)
      if (chosen[l] >= 0) select_variant(net->layers[l], chosen[l]);
    return CNN_OK;
  }
  // synthetic slice (fixed LCG pattern) and per-layer buffers
  const Dims d = layer_dims(net, (int)H, (int)W);
  std::vector<uint8_t> host_in((size_t)H * W);
  uint32_t s = 12345u;
  for (auto& b : host_in) {
    s = s * 1664525u + 1013904223u;
    b = (uint8_t)(s >> 24);
  }
  const int eb = net->prec == F32 ? 4 : net->prec == BF16 ? 2 : 1;
  std::vector<size_t> ob(nl);
  for (int l = 0; l < nl; ++l) {
    int64_t rs, zs;
    map_strides(net->layers[l], d.hout[l], d.wout[l], rs, zs);
    ob[l] = (l == nl - 1) ? (size_t)d.hout[l] * d.wout[l] * 4 : (size_t)zs * stored_channels(net->layers[l]) * eb;
  }
  std::vector<void*> bufs(nl + 2, nullptr);
  hipError_t e;
  size_t maxb = 0;
  for (size_t b : ob) maxb = std::max(maxb, b);
  bool okm = hipMalloc(&bufs[0], host_in.size()) == hipSuccess && hipMalloc(&bufs[nl + 1], maxb) == hipSuccess;
  for (int l = 0; l < nl && okm; ++l) okm = hipMalloc(&bufs[l + 1], ob[l]) == hipSuccess;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (void* p : bufs)
      if (p) hipFree(p);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (!okm) {
    cleanup();
    return fail(CNN_ENOMEM, "cnn_autotune: buffers");
  }
  hipEventCreate(&e0);
  hipEventCreate(&e1);
  if ((e = hipMemcpy(bufs[0], host_in.data(), host_in.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    cleanup();
    return hip_fail(e, "cnn_autotune: input upload");
  }
  // reference pass with the default variants (layer 0's output is still made
  // when layer 1 computes it itself: it is the reference for tuning layer 0)
  const bool fused = first_fused(net);
  auto layer_in = [&](int l) { return (l == 1 && fused) ? bufs[0] : bufs[l]; };
  for (int l = 0; l < nl && !rc; ++l) rc = run_one_layer(net, l, layer_in(l), bufs[l + 1], d, st);
  if (!rc && (e = hipStreamSynchronize(st)) != hipSuccess) rc = hip_fail(e, "cnn_autotune: reference pass");
  if (rc) {
    cleanup();
    return rc;
  }
  for (int l = 0; l < nl && !rc; ++l) {
    ExecLayer& L = net->layers[l];
    if (chosen[l] >= 0) {
      select_variant(L, chosen[l]);
      continue;
    }
    if (L.candidates.size() < 2 || (l == 0 && fused)) continue;  // a fused layer 0 is never launched
    std::vector<unsigned char> ref(ob[l]), got(ob[l]);
    if ((e = hipMemcpy(ref.data(), bufs[l + 1], ob[l], hipMemcpyDeviceToHost)) != hipSuccess) {
      rc = hip_fail(e, "cnn_autotune: reference copy");
      break;
    }
    const int def = L.variant;
    int best = def;
    float best_ms = 1e30f;
    for (int c : L.candidates) {
      // only candidates with the default's accumulation order (K layout and channel block)
      if (!L.first && (conv_variant(c)->rr != conv_variant(def)->rr || conv_variant(c)->cb != conv_variant(def)->cb ||
                       conv_variant(c)->fused != conv_variant(def)->fused))
        continue;
      select_variant(L, c);
      rc = run_one_layer(net, l, layer_in(l), bufs[nl + 1], d, st);  // warm-up, also the checked output
      if (rc) break;
      // one timed launch sizes the repetitions: about 5 ms of work per candidate
      hipEventRecord(e0, st);
      rc = run_one_layer(net, l, layer_in(l), bufs[nl + 1], d, st);
      hipEventRecord(e1, st);
      if (rc) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_fail(e, "cnn_autotune: timing");
        break;
      }
      float ms1 = 0.f;
      hipEventElapsedTime(&ms1, e0, e1);
      const int reps = (int)std::min(200.0f, std::max(5.0f, 5.0f / std::max(ms1, 1e-3f)));
      hipEventRecord(e0, st);
      for (int r = 0; r < reps && !rc; ++r) rc = run_one_layer(net, l, layer_in(l), bufs[nl + 1], d, st);
      hipEventRecord(e1, st);
      if (rc) break;
      if ((e = hipEventSynchronize(e1)) != hipSuccess) {
        rc = hip_fail(e, "cnn_autotune: timing");
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms /= reps;
      if ((e = hipMemcpy(got.data(), bufs[nl + 1], ob[l], hipMemcpyDeviceToHost)) != hipSuccess) {
        rc = hip_fail(e, "cnn_autotune: candidate copy");
        break;
      }
      const bool same = std::memcmp(got.data(), ref.data(), ob[l]) == 0;
      if (same && ms < best_ms) {
        best_ms = ms;
        best = c;
      }
    }
    select_variant(L, rc ? def : best);
    chosen[l] = L.variant;
  }
  cleanup();
  if (rc) return rc;
  if (cache_path) {
    std::ofstream f(cache_path, std::ios::trunc);
    for (const std::string& line : lines) {
      bool replaced = false;
      for (int l = 0; l < nl; ++l)
        if (line.rfind(layer_sig(net, net->layers[l]) + "|" + shape + "|", 0) == 0) replaced = true;
      if (!replaced) f << line << "\n";
    }
    for (int l = 0; l < nl; ++l)
      if (net->layers[l].candidates.size() > 1)
        f << layer_sig(net, net->layers[l]) << "|" << shape << "|" << layer_name(net->layers[l]) << "\n";
  }
  return CNN_OK;
}

namespace emcnn {

// Number of 32-bit words that differ between a and b (n words), added to *cnt.
__global__ __launch_bounds__(256) void count_mismatch(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b,
                                                      int64_t n, unsigned int* cnt) {
  unsigned int c = 0;
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) c += a[i] != b[i];
  if (c) atomicAdd(cnt, c);
}

}  // namespace emcnn

extern "C" int cnn_autotune_batch(cnn_net* h, const cnn_tile* tiles, int32_t n, void* stream) {
  clear_error();
  if (!h || !tiles || n < 1) return fail(CNN_EINVAL, "cnn_autotune_batch: null argument or n < 1");
  Net* net = reinterpret_cast<Net*>(h);
  int rc = check_device(net);
  if (rc) return rc;
  std::vector<Region> regs;
  rc = batch_regions(net, tiles, n, "cnn_autotune_batch", regs);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int nl = (int)net->layers.size();
  std::vector<int> defaults(nl);
  for (int l = 0; l < nl; ++l) defaults[l] = net->layers[l].variant;
  auto use = [&](const std::vector<int>& v) {
    for (int l = 0; l < nl; ++l) select_variant(net->layers[l], v[l]);
  };
  std::vector<std::vector<int>> byc(kTileClasses);
  for (int t = 0; t < n; ++t) byc[region_class(net, regs[t])].push_back(t);
  std::vector<std::vector<int>> cv(kTileClasses, defaults);
  net->class_variants.clear();
  hipEvent_t e0 = nullptr, e1 = nullptr;
  void* ref = nullptr;
  unsigned int* cnt = nullptr;
  auto cleanup = [&]() {
    use(defaults);
    if (ref) hipFree(ref);
    if (cnt) hipFree(cnt);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  hipError_t e;
  if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess ||
      (e = hipMalloc(&cnt, sizeof(unsigned int))) != hipSuccess) {
    cleanup();
    return hip_fail(e, "cnn_autotune_batch: setup");
  }
  for (int c = 0; c < kTileClasses && !rc; ++c) {
    if (byc[c].empty()) continue;
    std::vector<Region> rc_regs;
    std::vector<size_t> off;  // each tile's output, in 32-bit words, inside the reference copy
    size_t words = 0;
    for (int t : byc[c]) {
      rc_regs.push_back(regs[t]);
      off.push_back(words);
      words += (size_t)tiles[t].z * (tiles[t].h - 2 * tiles[t].halo) * (tiles[t].w - 2 * tiles[t].halo);
    }
    if (ref) hipFree(ref);
    ref = nullptr;
    if ((e = hipMalloc(&ref, words * 4)) != hipSuccess) {
      rc = fail(CNN_ENOMEM, "cnn_autotune_batch: reference outputs");
      break;
    }
    // one submission of this class's tiles with variants v (direct launches)
    auto pass = [&](const std::vector<int>& v) -> int {
      use(v);
      int r = arena_reserve(net, count_region_jobs(net, rc_regs));
      std::vector<Launch> launches;
      size_t used = 0, wn = 0;
      if (!r) r = plan_regions(net, rc_regs, 0, launches, used, wn);
      if (!r) r = submit(net, launches, 0, used, st, false);
      return r;
    };
    // timed passes: one untimed, then enough for ~10 ms
    auto timed = [&](const std::vector<int>& v, float& ms) -> int {
      int r = pass(v);
      if (!r && (e = hipEventRecord(e0, st)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      if (!r) r = pass(v);
      if (!r && (e = hipEventRecord(e1, st)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      if (!r && (e = hipEventSynchronize(e1)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      float ms1 = 0.f;
      if (!r) hipEventElapsedTime(&ms1, e0, e1);
      const int reps = (int)std::min(20.0f, std::max(2.0f, 10.0f / std::max(ms1, 1e-3f)));
      if (!r && (e = hipEventRecord(e0, st)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      for (int k = 0; k < reps && !r; ++k) r = pass(v);
      if (!r && (e = hipEventRecord(e1, st)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      if (!r && (e = hipEventSynchronize(e1)) != hipSuccess) r = hip_fail(e, "cnn_autotune_batch: timing");
      if (!r) {
        hipEventElapsedTime(&ms, e0, e1);
        ms /= reps;
      }
      return r;
    };
    // the reference: the class's outputs with the default variants
    float best_ms = 0.f;
    rc = timed(defaults, best_ms);
    for (size_t k = 0; k < byc[c].size() && !rc; ++k) {
      const cnn_tile& T = tiles[byc[c][k]];
      const size_t bytes = (size_t)T.z * (T.h - 2 * T.halo) * (T.w - 2 * T.halo) * 4;
      if ((e = hipMemcpyAsync(reinterpret_cast<uint32_t*>(ref) + off[k], T.out, bytes, hipMemcpyDeviceToDevice, st)) !=
          hipSuccess)
        rc = hip_fail(e, "cnn_autotune_batch: reference copy");
    }
    if (rc) break;
    std::vector<int> best = defaults;
    for (int l = 0; l < nl && !rc; ++l) {
      const ExecLayer& L = net->layers[l];
      for (int cand : L.candidates) {
        if (cand == best[l]) continue;
        // only candidates with the default's accumulation order
        if (!L.first && (conv_variant(cand)->rr != conv_variant(defaults[l])->rr ||
                         conv_variant(cand)->cb != conv_variant(defaults[l])->cb ||
                         conv_variant(cand)->fused != conv_variant(defaults[l])->fused))
          continue;
        std::vector<int> trial = best;
        trial[l] = cand;
        float ms = 0.f;
        rc = timed(trial, ms);
        if (rc) break;
        // bitwise check of every tile's output against the reference
        if ((e = hipMemsetAsync(cnt, 0, sizeof(unsigned int), st)) != hipSuccess) {
          rc = hip_fail(e, "cnn_autotune_batch: check");
          break;
        }
        for (size_t k = 0; k < byc[c].size(); ++k) {
          const cnn_tile& T = tiles[byc[c][k]];
          const int64_t w = (int64_t)T.z * (T.h - 2 * T.halo) * (T.w - 2 * T.halo);
          const int grid = (int)std::min<int64_t>((w + 255) / 256, 4096);
          hipLaunchKernelGGL(count_mismatch, dim3(grid), dim3(256), 0, st,
                             reinterpret_cast<const uint32_t*>(T.out), reinterpret_cast<const uint32_t*>(ref) + off[k],
                             w, cnt);
        }
        unsigned int bad = 1;
        if ((e = hipMemcpyAsync(&bad, cnt, sizeof(bad), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
          rc = hip_fail(e, "cnn_autotune_batch: check");
          break;
        }
        if (bad == 0 && ms < best_ms) {
          best_ms = ms;
          best = trial;
        }
      }
    }
    cv[c] = best;
  }
  cleanup();
  if (rc) return rc;
  net->class_variants = cv;
  return CNN_OK;
}

extern "C" int cnn_profile(cnn_net* h, int32_t enable) {
  clear_error();
  if (!h) return fail(CNN_EINVAL, "cnn_profile: null net");
  Net* net = reinterpret_cast<Net*>(h);
  net->profiling = enable ? 1 : 0;
  return CNN_OK;
}

extern "C" int cnn_profile_read(cnn_net* h, double* ms, int32_t* launches, int32_t max_layers) {
  clear_error();
  if (!h || !ms || !launches || max_layers < 1) return fail(CNN_EINVAL, "cnn_profile_read: bad argument");
  Net* net = reinterpret_cast<Net*>(h);
  const int nl = (int)net->layers.size();
  for (int l = 0; l < max_layers; ++l) {
    ms[l] = 0.0;
    launches[l] = 0;
  }
  int rc = CNN_OK;
  for (auto& t : net->timed) {
    float v = 0.f;
    hipError_t e = hipEventSynchronize(t.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&v, t.a, t.b);
    if (e != hipSuccess && rc == CNN_OK) rc = hip_fail(e, "cnn_profile_read");
    if (t.layer >= 0 && t.layer < std::min(nl, (int)max_layers)) {
      ms[t.layer] += v;
      launches[t.layer] += 1;
    }
    net->event_pool.push_back(t.a);
    net->event_pool.push_back(t.b);
  }
  net->timed.clear();
  return rc;
}

extern "C" int cnn_set_variant(cnn_net* h, int32_t layer, const char* name) {
  clear_error();
  if (!h || !name) return fail(CNN_EINVAL, "cnn_set_variant: null argument");
  Net* net = reinterpret_cast<Net*>(h);
  if (layer < 0 || layer >= (int)net->layers.size()) return fail(CNN_EINVAL, "cnn_set_variant: bad layer index");
  ExecLayer& L = net->layers[layer];
  const int c = candidate_name_index(L, name);
  if (c < 0 || !select_variant(L, c)) return fail(CNN_EINVAL, std::string("cnn_set_variant: no candidate ") + name);
  net->class_variants.clear();  // an explicit choice applies to batches too
  return CNN_OK;
}

extern "C" int cnn_variant_name(const cnn_net* h, int32_t layer, int32_t index, char* buf, int32_t len) {
  clear_error();
  if (!h || !buf || len < 1) return fail(CNN_EINVAL, "cnn_variant_name: bad argument");
  const Net* net = reinterpret_cast<const Net*>(h);
  if (layer < 0 || layer >= (int)net->layers.size()) return fail(CNN_EINVAL, "cnn_variant_name: bad layer index");
  const ExecLayer& L = net->layers[layer];
  if (index < 0 || index >= (int)L.candidates.size()) return fail(CNN_EINVAL, "cnn_variant_name: index out of range");
  const int c = L.candidates[index];
  std::snprintf(buf, len, "%s", L.first ? first_variant(c)->name : conv_variant(c)->name);
  return CNN_OK;
}
