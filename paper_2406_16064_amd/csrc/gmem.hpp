// Explicit memory spaces for the hot-path kernels (gfx950).
//
// Pointers that the kernels read out of structs in device memory are generic
// to the compiler, which then emits flat instructions: each one counts against
// both the vector-memory and the LDS wait counters, so an LDS access right
// after a global load waits for that load too.  These helpers put the access
// in the global space (vector global loads and stores, complex values in one
// 8- or 16-byte access) and read uniform structs through the constant space
// (scalar loads into SGPRs, once per workgroup).
#pragma once

#include "mm_internal.hpp"

#define MMX_GLOBAL __attribute__((address_space(1)))
#define MMX_CONST __attribute__((address_space(4)))

namespace mmx {

typedef float mmx_f2 __attribute__((ext_vector_type(2)));
typedef double mmx_d2 __attribute__((ext_vector_type(2)));

// loads and stores through global-space pointers
__device__ __forceinline__ float gld_(const MMX_GLOBAL float* p) { return *p; }
__device__ __forceinline__ double gld_(const MMX_GLOBAL double* p) { return *p; }
__device__ __forceinline__ Cx<float> gld_(const MMX_GLOBAL Cx<float>* p) {
  const mmx_f2 v = *(const MMX_GLOBAL mmx_f2*)p;
  return Cx<float>{v.x, v.y};
}
__device__ __forceinline__ Cx<double> gld_(const MMX_GLOBAL Cx<double>* p) {
  const mmx_d2 v = *(const MMX_GLOBAL mmx_d2*)p;
  return Cx<double>{v.x, v.y};
}
__device__ __forceinline__ void gst_(MMX_GLOBAL float* p, float v) { *p = v; }
__device__ __forceinline__ void gst_(MMX_GLOBAL double* p, double v) { *p = v; }
__device__ __forceinline__ void gst_(MMX_GLOBAL Cx<float>* p, Cx<float> v) { *(MMX_GLOBAL mmx_f2*)p = mmx_f2{v.x, v.y}; }
__device__ __forceinline__ void gst_(MMX_GLOBAL Cx<double>* p, Cx<double> v) {
  *(MMX_GLOBAL mmx_d2*)p = mmx_d2{v.x, v.y};
}

template <typename T>
__device__ __forceinline__ T gld(const T* p) { return gld_((const MMX_GLOBAL T*)p); }
template <typename T>
__device__ __forceinline__ void gst(T* p, T v) { gst_((MMX_GLOBAL T*)p, v); }

// base (same in every lane) + a 32-bit byte offset: the address arithmetic
// happens in the global space, so the scalar-base form of the instruction
// applies (one 32-bit offset register per lane instead of a 64-bit address).
template <typename T>
__device__ __forceinline__ T gldo(const T* base, uint32_t boff) {
  const MMX_GLOBAL char* b = (const MMX_GLOBAL char*)base;
  return gld_((const MMX_GLOBAL T*)(b + boff));
}
template <typename T>
__device__ __forceinline__ void gsto(T* base, uint32_t boff, T v) {
  MMX_GLOBAL char* b = (MMX_GLOBAL char*)base;
  gst_((MMX_GLOBAL T*)(b + boff), v);
}

// Read-only uniform struct (same address in every lane, not written while the
// kernel runs): scalar loads through the constant space.
template <class S>
__device__ __forceinline__ S ldu(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "ldu needs a whole number of dwords");
  constexpr int n = (int)(sizeof(S) / 4);
  uint32_t w[n];
  const MMX_CONST uint32_t* src = (const MMX_CONST uint32_t*)p;
#pragma unroll
  for (int i = 0; i < n; ++i) w[i] = src[i];
  S out;
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

}  // namespace mmx
