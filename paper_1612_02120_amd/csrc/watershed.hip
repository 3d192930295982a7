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
// kernels reproduce it exactly whatever the scheduling:
//   ws_init      one pass: a[v] = v on S, else next(v)
//   ws_hook      seed components by hooking: for each pair of 6-adjacent
//                seeds in different trees, the larger root is pointed at the
//                smaller one (atomicMin); a[] only ever decreases and a[v] <= v,
//                so the forest stays valid under any interleaving, and the
//                least index of a component is its final root
//   ws_compress  path compression, a[v] = root, between hooking rounds
//   ws_label     every voxel follows a[] to a seed (then takes its root) or to
//                a non-seed fixed point (a local minimum of the order)
// Rounds repeat until a hooking round changes nothing; each round reads a
// one-word flag back to the host.
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

__global__ __launch_bounds__(256) void ws_init(const float* __restrict__ p, Vol3 g, float t, int32_t* __restrict__ a) {
  const int64_t HW = (int64_t)g.H * g.W;
  for (int64_t v = blockIdx.x * 256ll + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * 256) {
    const float pv = wp(p, v);
    if (pv < t) {
      a[v] = (int32_t)v;
      continue;
    }
    const int x = (int)(v % g.W), y = (int)((v / g.W) % g.H), z = (int)(v / HW);
    int64_t best = v;
    float pb = pv;
    // candidates in ascending index order: a later candidate wins only if strictly lower
    const int64_t cand[6] = {z > 0 ? v - HW : -1, y > 0 ? v - g.W : -1, x > 0 ? v - 1 : -1,
                             x < g.W - 1 ? v + 1 : -1, y < g.H - 1 ? v + g.W : -1, z < g.Z - 1 ? v + HW : -1};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int64_t u = cand[k];
      if (u < 0) continue;
      const float pu = wp(p, u);
      if (pu < pb || (pu == pb && u < best)) {
        pb = pu;
        best = u;
      }
    }
    a[v] = (int32_t)best;
  }
}

__device__ __forceinline__ int32_t ws_find(const int32_t* a, int32_t r) {
  int32_t q = wa(a, r);
  while (q != r) {
    r = q;
    q = wa(a, r);
  }
  return r;
}

__global__ __launch_bounds__(256) void ws_hook(const float* __restrict__ p, Vol3 g, float t, int32_t* a,
                                               int32_t* flag) {
  const int64_t HW = (int64_t)g.H * g.W;
  int changed = 0;
  for (int64_t v = blockIdx.x * 256ll + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * 256) {
    if (!(wp(p, v) < t)) continue;
    const int x = (int)(v % g.W), y = (int)((v / g.W) % g.H), z = (int)(v / HW);
    const int64_t fwd[3] = {x < g.W - 1 ? v + 1 : -1, y < g.H - 1 ? v + g.W : -1, z < g.Z - 1 ? v + HW : -1};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int64_t u = fwd[k];
      if (u < 0 || !(wp(p, u) < t)) continue;
      const int32_t rv = ws_find(a, (int32_t)v), ru = ws_find(a, (int32_t)u);
      if (rv != ru) {
        atomicMin(a + (rv > ru ? rv : ru), rv < ru ? rv : ru);
        changed = 1;
      }
    }
  }
  if (__any(changed) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void ws_compress(const float* __restrict__ p, Vol3 g, float t, int32_t* a) {
  for (int64_t v = blockIdx.x * 256ll + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * 256)
    if (wp(p, v) < t) a[v] = ws_find(a, (int32_t)v);
}

__global__ __launch_bounds__(64) void ws_clear(int32_t* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

__global__ __launch_bounds__(256) void ws_label(const float* __restrict__ p, Vol3 g, float t,
                                                const int32_t* __restrict__ a, int32_t* __restrict__ out) {
  for (int64_t v = blockIdx.x * 256ll + threadIdx.x; v < g.N; v += (int64_t)gridDim.x * 256) {
    int32_t u = (int32_t)v;
    // descend until a seed or a fixed point; on a seed a[] is its root
    while (!(wp(p, u) < t)) {
      const int32_t n = a[u];
      if (n == u) break;
      u = n;
    }
    out[v] = (wp(p, u) < t ? a[u] : u) + 1;
  }
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
  int32_t* flag = work + g.N;
  const int grid = (int)std::min<int64_t>((g.N + 255) / 256, 2048 * 8);
  hipError_t e;
  hipLaunchKernelGGL(ws_init, dim3(grid), dim3(256), 0, st, prob, g, seed_threshold, work);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: init");
  for (int round = 0;; ++round) {
    if (round >= 4096) return fail(CNN_EHIP, "watershed_3d: seed components did not converge");
    hipLaunchKernelGGL(ws_clear, dim3(1), dim3(64), 0, st, flag);
    hipLaunchKernelGGL(ws_hook, dim3(grid), dim3(256), 0, st, prob, g, seed_threshold, work, flag);
    hipLaunchKernelGGL(ws_compress, dim3(grid), dim3(256), 0, st, prob, g, seed_threshold, work);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: hook");
    int32_t h = 0;
    if ((e = hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, st)) != hipSuccess)
      return hip_fail(e, "watershed_3d: flag");
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "watershed_3d: sync");
    if (!h) break;
  }
  hipLaunchKernelGGL(ws_label, dim3(grid), dim3(256), 0, st, prob, g, seed_threshold, work, labels_out);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "watershed_3d: label");
  return CNN_OK;
}
