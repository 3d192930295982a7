// 3-D watershed of a membrane probability map (Section 2.1: the stage after
// membrane classification turns the map into an over-segmentation with a 3-D
// watershed). Watershed by steepest descent with seeded minima:
//   order   u < v iff p[u] < p[v], or p[u] == p[v] and index(u) < index(v)
//   seeds   S = { v : p[v] < t }, its 6-connected components labelled
//           1 + the least index in each
//   descent next(v) = v on S, else the least of v and its 6-neighbours
//   label   of v: the seed component's label where the descent from v ends
//           in S, else 1 + the index of the local minimum it ends at.
// The result is unique (a total order, no flooding order to choose), so the
// kernels reproduce it exactly whatever the scheduling. One forest a[] holds
// both parts: a non-seed points along its descent, a seed into its
// component's tree. Roots are fixed points: component minima and non-seed
// local minima.
//   ws_init   one pass: a seed points to the first seed of its run along x
//             (the run's least index; a ballot scan per row), any other
//             voxel to next(v). The x-links of the seed graph are then made.
//   ws_union  one pass over the seeds: runs adjacent along y or z are united
//             by a lock-free union-find (the structure of ECL-CC): find both
//             roots, hook the larger root under the smaller with a
//             compare-and-swap that only succeeds while it is still a root,
//             and retry from the new roots when another thread hooked it
//             first. Two runs that touch are united once, at the first column
//             where they do (the pair one column left, when both are seeds,
//             joins the same two runs). A seed's parent index only
//             decreases, so every component ends rooted at its least index.
//   ws_label  every voxel finds its root (a component minimum or a local
//             minimum), halving the path as it goes, and takes root + 1.
// Path halving points a node at its grandparent, an ancestor in the same
// tree, so concurrent finds stay valid; it never writes a root.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/emcnn.h"
#include "device_util.h"
#include "runtime.h"

namespace emcnn {

struct Vol3 {
  int Z, H, W;
  int64_t N;
};

__device__ __forceinline__ float wp(const float* p, int64_t v) { return ld<float>(gin(p) + v * 4); }
__device__ __forceinline__ int32_t wa(const int32_t* a, int64_t v) {
  return __atomic_load_n(a + v, __ATOMIC_RELAXED);
}

// Work split: one row (z, y) of W voxels per block iteration, x over the
// threads in chunks of 256 columns; indices fit in 32 bits (Z H W < 2^31 - 1).
__global__ __launch_bounds__(256) void ws_init(const float* __restrict__ p, Vol3 g, float t, int32_t* __restrict__ a) {
  __shared__ int wbreak[4];  // per wave: its last non-seed column in the chunk, or -1
  const int HW = g.H * g.W;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int row = blockIdx.x; row < g.Z * g.H; row += gridDim.x) {
    const int z = row / g.H, y = row - z * g.H, base = row * g.W;
    int carry = -1;  // the last non-seed column before the chunk
    for (int x0 = 0; x0 < g.W; x0 += 256) {  // uniform over the block: every thread takes every chunk
      const int x = x0 + threadIdx.x;
      const int v = base + x;
      const bool in = x < g.W;
      const float pv = in ? wp(p, v) : 0.f;
      const bool seed = in && pv < t;
      // lb: the last non-seed column at or before x (columns past the row count as non-seeds)
      const uint64_t brk = __ballot(!seed);
      const uint64_t upto = brk & ((2ull << lane) - 1);  // lanes 0 .. lane (all 64 bits for lane 63)
      const int wx = x0 + wv * 64 + 63;                   // the wave's last column
      int lb = upto ? wx - __builtin_clzll(upto) : -1;
      if (lane == 0) wbreak[wv] = brk ? wx - __builtin_clzll(brk) : -1;
      __syncthreads();
      if (lb < 0) {
        lb = carry;
        for (int k = 0; k < wv; ++k) lb = max(lb, wbreak[k]);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) carry = max(carry, wbreak[k]);
      __syncthreads();  // wbreak is rewritten for the next chunk
      if (!in) continue;
      if (seed) {
        a[v] = base + lb + 1;  // the run's first seed
        continue;
      }
      int best = v;
      float pb = pv;
      // candidates in ascending index order: a later candidate wins only if strictly lower
      const int cand[6] = {z > 0 ? v - HW : -1, y > 0 ? v - g.W : -1, x > 0 ? v - 1 : -1,
                           x < g.W - 1 ? v + 1 : -1, y < g.H - 1 ? v + g.W : -1, z < g.Z - 1 ? v + HW : -1};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const int u = cand[k];
        if (u < 0) continue;
        const float pu = wp(p, u);
        if (pu < pb || (pu == pb && u < best)) {
          pb = pu;
          best = u;
        }
      }
      a[v] = best;
    }
  }
}

// Root of r with path halving (any node may be passed; roots are fixed points).
__device__ __forceinline__ int32_t ws_find(int32_t* a, int32_t r) {
  int32_t par = wa(a, r);
  while (par != r) {
    const int32_t gp = wa(a, par);
    if (gp == par) return par;
    __atomic_store_n(a + r, gp, __ATOMIC_RELAXED);  // r is not a root: an ancestor is a valid parent
    r = gp;
    par = wa(a, r);
  }
  return r;
}

__device__ __forceinline__ void ws_unite(int32_t* a, int32_t u, int32_t v) {
  int32_t ru = ws_find(a, u), rv = ws_find(a, v);
  while (ru != rv) {
    const int32_t hi = ru > rv ? ru : rv, lo = ru < rv ? ru : rv;
    const int32_t old = atomicCAS(a + hi, hi, lo);
    if (old == hi) return;  // hooked while hi was still a root
    // hi was hooked meanwhile: continue from the current roots
    ru = ws_find(a, hi);
    rv = ws_find(a, lo);
  }
}

__global__ __launch_bounds__(256) void ws_union(const float* __restrict__ p, Vol3 g, float t, int32_t* a) {
  const int HW = g.H * g.W;
  for (int row = blockIdx.x; row < g.Z * g.H; row += gridDim.x) {
    const int z = row / g.H, y = row - z * g.H, base = row * g.W;
    for (int x = threadIdx.x; x < g.W; x += 256) {
      const int v = base + x;
      if (!(wp(p, v) < t)) continue;
      const bool left = x > 0 && wp(p, v - 1) < t;  // v is not its run's first seed
      const int fwd[2] = {y < g.H - 1 ? v + g.W : -1, z < g.Z - 1 ? v + HW : -1};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int u = fwd[k];
        if (u < 0 || !(wp(p, u) < t)) continue;
        if (left && wp(p, u - 1) < t) continue;  // the pair one column left joins the same two runs
        ws_unite(a, v, u);
      }
    }
  }
}

__global__ __launch_bounds__(256) void ws_label(Vol3 g, int32_t* a, int32_t* __restrict__ out) {
  const int n = (int)g.N;
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) out[v] = ws_find(a, v) + 1;
}

}  // namespace emcnn

using namespace emcnn;

extern "C" int watershed_3d(const float* prob, const int64_t dims[3], float seed_threshold, int32_t* labels_out,
                            int32_t* work, void* stream) {
  clear_error();
  if (!prob || !dims || !labels_out || !work) return fail(CNN_EINVAL, "watershed_3d: null argument");
  const int64_t Z = dims[0], H = dims[1], W = dims[2];
  if (Z < 1 || H < 1 || W < 1 || Z > (1 << 30) || H > (1 << 30) || W > (1 << 30) || Z * H * W >= 2147483647ll)
    return fail(CNN_EINVAL, "watershed_3d: dims must be >= 1 with Z H W < 2^31 - 1");
  if (seed_threshold != seed_threshold) return fail(CNN_EINVAL, "watershed_3d: NaN threshold");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  Vol3 g{(int)Z, (int)H, (int)W, Z * H * W};
  const int grid = (int)std::min<int64_t>((g.N + 255) / 256, 2048 * 8);
  const int rows = (int)std::min<int64_t>(Z * H, 2048 * 8);  // row-per-block kernels
  hipError_t e;
  hipLaunchKernelGGL(ws_init, dim3(rows), dim3(256), 0, st, prob, g, seed_threshold, work);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: init");
  hipLaunchKernelGGL(ws_union, dim3(rows), dim3(256), 0, st, prob, g, seed_threshold, work);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: union");
  hipLaunchKernelGGL(ws_label, dim3(grid), dim3(256), 0, st, g, work, labels_out);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: label");
  return CNN_OK;
}
