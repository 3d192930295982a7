// Device-side helpers shared by the library's kernels: operand vector types
// and global-memory access through the global address space.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emcnn {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef int i8v __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef unsigned char u8x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Global-memory access. Pointers read from job tables and parameter structs
// are generic to the compiler, which then emits FLAT instructions; a FLAT load
// also counts against the LDS wait counter, so every wait for an LDS read
// would wait for it as well. Accesses through these global-address-space
// pointers compile to global_load / global_store (vector memory counter only).
#define EMCNN_GLOBAL __attribute__((address_space(1)))
typedef EMCNN_GLOBAL unsigned char gbyte;
__device__ __forceinline__ const gbyte* gin(const void* p) { return (const gbyte*)p; }
__device__ __forceinline__ gbyte* gout(void* p) { return (gbyte*)p; }
template <class V>
__device__ __forceinline__ V ld(const unsigned char* p) {
  return *reinterpret_cast<const V*>(p);
}
template <class V>
__device__ __forceinline__ V ld(const gbyte* p) {
  return *reinterpret_cast<const EMCNN_GLOBAL V*>(p);
}
template <class V>
__device__ __forceinline__ void st(unsigned char* p, V v) {
  *reinterpret_cast<V*>(p) = v;
}
template <class V>
__device__ __forceinline__ void st(gbyte* p, V v) {
  *reinterpret_cast<EMCNN_GLOBAL V*>(p) = v;
}
// Store with the nontemporal (streaming) hint, for FP32 maps that a layer
// writes once and the next layer reads only after this one has ended: at
// hundreds of MB to GB per layer they do not stay in the caches anyway.
template <class V>
__device__ __forceinline__ void st_nt(gbyte* p, V v) {
  __builtin_nontemporal_store(v, reinterpret_cast<EMCNN_GLOBAL V*>(p));
}
__device__ __forceinline__ float ldf(const float* p, int i) { return ld<float>(gin(p) + (int64_t)i * 4); }

}  // namespace emcnn
