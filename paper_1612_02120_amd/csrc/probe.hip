// MFMA diagnostics: the matrix instructions the conv kernels use, run on given
// operands (cnn_mfma_probe) and in a throughput loop with the shader clock
// read inside the kernel (cnn_mfma_bench).
//
// Operand layout, as in the conv kernels (D = A B with M = N = 16): lane
// (g, n) = (lane / 16, lane % 16) of a wave holds, for k-slot g, its 16 bytes
// (FP8: 32 bytes) of row n of A and of column n of B; byte t of a lane's A
// chunk meets byte t of the matching B chunk, so
//   D[m][n] = sum_g sum_t A(lane g*16 + m)[t] * B(lane g*16 + n)[t],
// and lane (g, n) receives D[4g + k][n] in accumulator k. FP32 chunks are four
// 16x16x4 MFMAs (one float per lane each), BF16 one 16x16x32, FP8 (e4m3fn,
// unit block scales) one 16x16x128.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/emcnn.h"
#include "common.h"
#include "device_util.h"
#include "runtime.h"

namespace emcnn {

template <int P>
__device__ __forceinline__ f4 probe_mma(f4 acc, const gbyte* a, const gbyte* b) {
  if constexpr (P == F32) {
    const f4 x = ld<f4>(a), y = ld<f4>(b);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[0], y[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[1], y[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[2], y[2], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x[3], y[3], acc, 0, 0, 0);
  } else if constexpr (P == BF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld<bf16x8>(a), ld<bf16x8>(b), acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(ld<i8v>(a), ld<i8v>(b), acc, 0, 0, 0, 127, 0, 127);
  }
  return acc;
}

// One wave per output tile: D accumulated over `chain` consecutive operand
// tiles (each instruction takes the previous one's result as its
// accumulator, as over the K steps of a conv), from zero.
template <int P>
__global__ __launch_bounds__(64) void mfma_probe(const void* a, const void* b, float* d, int ntiles, int chain) {
  constexpr int CH = P == FP8 ? 32 : 16;  // operand bytes per lane
  const int t = blockIdx.x, lane = threadIdx.x;
  if (t >= ntiles) return;
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
  for (int c = 0; c < chain; ++c) {
    const int64_t off = (((int64_t)t * chain + c) * 64 + lane) * CH;
    acc = probe_mma<P>(acc, gin(a) + off, gin(b) + off);
  }
  st<f4>(gout(d) + ((int64_t)t * 64 + lane) * 16, acc);
}

// Throughput loop: every wave keeps NACC independent accumulators and runs
// `iters` rounds of NACC MFMAs on register operands (taken from `ops`, so the
// data is the caller's); the shader clock (s_memtime) and the constant 100 MHz
// clock (s_memrealtime) are read before and after the loop by lane 0 of each
// wave. The accumulators are folded into one value per lane and stored, so no
// MFMA is dead code.
template <int P>
__global__ __launch_bounds__(256) void mfma_bench(const void* ops, int iters, float* sink, int64_t* clocks) {
  constexpr int NACC = 8;
  constexpr int CH = P == FP8 ? 32 : 16;
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const gbyte* src = gin(ops) + (int64_t)(wave & 255) * 64 * 2 * CH;
  f4 acc[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i) acc[i] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t t0 = (int64_t)__builtin_readcyclecounter();
  const int64_t r0 = (int64_t)__builtin_amdgcn_s_memrealtime();
  if constexpr (P == F32) {
    const float x = ld<float>(src + lane * 4), y = ld<float>(src + 64 * CH + lane * 4);
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, acc[i], 0, 0, 0);
  } else if constexpr (P == BF16) {
    const bf16x8 x = ld<bf16x8>(src + lane * CH), y = ld<bf16x8>(src + 64 * CH + lane * CH);
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < NACC; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[i], 0, 0, 0);
  } else {
    const i8v x = ld<i8v>(src + lane * CH), y = ld<i8v>(src + 64 * CH + lane * CH);
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int i = 0; i < NACC; ++i)
        acc[i] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(x, y, acc[i], 0, 0, 0, 127, 0, 127);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NACC; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  const int64_t t1 = (int64_t)__builtin_readcyclecounter();
  const int64_t r1 = (int64_t)__builtin_amdgcn_s_memrealtime();
  st<float>(gout(sink) + ((int64_t)wave * 64 + lane) * 4, s);
  if (lane == 0) {
    st<int64_t>(gout(clocks) + (int64_t)wave * 16, t1 - t0);
    st<int64_t>(gout(clocks) + (int64_t)wave * 16 + 8, r1 - r0);
  }
}

}  // namespace emcnn

using namespace emcnn;

extern "C" int cnn_mfma_probe(int32_t precision, const void* a, const void* b, float* d, int32_t ntiles,
                              int32_t chain, void* stream) {
  clear_error();
  if (!a || !b || !d || ntiles < 1 || ntiles > (1 << 20) || chain < 1 || chain > 64)
    return fail(CNN_EINVAL, "cnn_mfma_probe: bad argument");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (precision == CNN_PREC_FP32)
    hipLaunchKernelGGL(mfma_probe<F32>, dim3(ntiles), dim3(64), 0, st, a, b, d, ntiles, chain);
  else if (precision == CNN_PREC_BF16)
    hipLaunchKernelGGL(mfma_probe<BF16>, dim3(ntiles), dim3(64), 0, st, a, b, d, ntiles, chain);
  else if (precision == CNN_PREC_FP8)
    hipLaunchKernelGGL(mfma_probe<FP8>, dim3(ntiles), dim3(64), 0, st, a, b, d, ntiles, chain);
  else
    return fail(CNN_EINVAL, "cnn_mfma_probe: unknown precision");
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "cnn_mfma_probe");
  return CNN_OK;
}

extern "C" int cnn_mfma_bench(int32_t precision, int32_t blocks, int32_t iters, const void* ops, double* tflops,
                              double* mhz, void* stream) {
  clear_error();
  if (!ops || !tflops || !mhz || blocks < 1 || blocks > 65536 || iters < 1 || iters > (1 << 24))
    return fail(CNN_EINVAL, "cnn_mfma_bench: bad argument");
  if (precision != CNN_PREC_FP32 && precision != CNN_PREC_BF16 && precision != CNN_PREC_FP8)
    return fail(CNN_EINVAL, "cnn_mfma_bench: unknown precision");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t waves = (int64_t)blocks * 4;
  float* sink = nullptr;
  int64_t* clocks = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&sink, waves * 64 * 4);
  if (e == hipSuccess) e = hipMalloc(&clocks, waves * 16);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    if (sink) hipFree(sink);
    if (clocks) hipFree(clocks);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
  };
  if (e != hipSuccess) {
    cleanup();
    return hip_fail(e, "cnn_mfma_bench: setup");
  }
  auto launch = [&](int it) {
    if (precision == CNN_PREC_FP32)
      hipLaunchKernelGGL(mfma_bench<F32>, dim3(blocks), dim3(256), 0, st, ops, it, sink, clocks);
    else if (precision == CNN_PREC_BF16)
      hipLaunchKernelGGL(mfma_bench<BF16>, dim3(blocks), dim3(256), 0, st, ops, it, sink, clocks);
    else
      hipLaunchKernelGGL(mfma_bench<FP8>, dim3(blocks), dim3(256), 0, st, ops, it, sink, clocks);
  };
  launch(std::max(1, iters / 16));  // warm-up (clock ramp)
  e = hipEventRecord(e0, st);
  launch(iters);
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  std::vector<int64_t> ck(waves * 2);
  if (e == hipSuccess) e = hipMemcpy(ck.data(), clocks, waves * 16, hipMemcpyDeviceToHost);
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "cnn_mfma_bench");
  const double flop_per_mfma = precision == CNN_PREC_FP32 ? 2.0 * 16 * 16 * 4
                               : precision == CNN_PREC_BF16 ? 2.0 * 16 * 16 * 32
                                                             : 2.0 * 16 * 16 * 128;
  *tflops = (double)waves * iters * 8 * flop_per_mfma / (ms * 1e-3) / 1e12;
  // shader clock: cycles over constant-clock ticks (100 MHz), averaged over waves
  double cyc = 0, rt = 0;
  for (int64_t w = 0; w < waves; ++w) {
    cyc += (double)ck[2 * w];
    rt += (double)ck[2 * w + 1];
  }
  *mhz = rt > 0 ? cyc / rt * 100.0 : 0.0;
  return CNN_OK;
}
