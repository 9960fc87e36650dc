// Device-memory access helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lac {

// Accesses through a pointer known to address global memory.  Through a
// generic pointer they compile to flat instructions, which may reach LDS as
// well: the compiler then cannot tell their completion order from that of
// other memory operations, and every later wait for a load in flight becomes
// a wait for all of them (a prefetched load is waited for as soon as it is
// issued).  The kernels' per-pixel and per-word accesses go through these.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T ldg(const T* p, int64_t i) {
  return gp(p)[i];
}
template <typename T>
__device__ __forceinline__ void stg(T* p, int64_t i, T v) {
  gp(p)[i] = v;
}
// The same through a wave-uniform base and a non-negative 32-bit per-lane
// index: the base stays in scalar registers and the address is base plus a
// 32-bit vector offset, with no 64-bit address arithmetic per lane.
template <typename T>
__device__ __forceinline__ T ldg_u(const T* base, uint32_t i) {
  return gp(base)[i];
}
template <typename T>
__device__ __forceinline__ void stg_u(T* base, uint32_t i, T v) {
  gp(base)[i] = v;
}
// Device-scope relaxed atomics on global memory (those of atomicOr and its
// kin, without the generic pointer).
template <typename T>
__device__ __forceinline__ T atom_or(T* p, T v) {
  return __hip_atomic_fetch_or(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atom_and(T* p, T v) {
  return __hip_atomic_fetch_and(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T atom_add(T* p, T v) {
  return __hip_atomic_fetch_add(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace lac
