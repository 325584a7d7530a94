// Host emulation of the few HIP/AMDGCN features the pass code uses, written
// from the instruction definitions, for CPU-side logic checks only.
#pragma once
#include <cstdint>
#include <cstring>
#include <cstdio>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(x)
struct emu_dim3 { unsigned x = 0, y = 0, z = 0; };
extern emu_dim3 threadIdx, blockDim, blockIdx, gridDim;
struct uint2 { uint32_t x, y; };
inline uint2 make_uint2(uint32_t a, uint32_t b) { return {a, b}; }
inline uint32_t __builtin_amdgcn_perm(uint32_t s0, uint32_t s1, uint32_t sel) {
  uint64_t d = ((uint64_t)s0 << 32) | s1; uint32_t r = 0;
  for (int i = 0; i < 4; ++i) {
    uint32_t b = (sel >> (8 * i)) & 0xFF, v;
    if (b >= 13) v = 0xFF; else if (b == 12) v = 0;
    else if (b == 11) v = (d >> 63) & 1 ? 0xFF : 0; else if (b == 10) v = (d >> 47) & 1 ? 0xFF : 0;
    else if (b == 9) v = (d >> 31) & 1 ? 0xFF : 0; else if (b == 8) v = (d >> 15) & 1 ? 0xFF : 0;
    else v = (d >> (8 * b)) & 0xFF;
    r |= v << (8 * i);
  }
  return r;
}
inline uint32_t __builtin_amdgcn_udot4(uint32_t a, uint32_t b, uint32_t c, bool) {
  uint32_t s = c; for (int i = 0; i < 4; ++i) s += ((a >> (8*i)) & 0xFF) * ((b >> (8*i)) & 0xFF); return s;
}
inline uint32_t __builtin_amdgcn_udot8(uint32_t a, uint32_t b, uint32_t c, bool) {
  uint32_t s = c; for (int i = 0; i < 8; ++i) s += ((a >> (4*i)) & 0xF) * ((b >> (4*i)) & 0xF); return s;
}
struct uint4 { uint32_t x, y, z, w; };
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return {a, b, c, d}; }
inline uint32_t __builtin_amdgcn_alignbyte(uint32_t hi, uint32_t lo, uint32_t sh) {
  return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (8 * (sh & 3)));
}
inline uint32_t __popc(uint32_t x) { return __builtin_popcount(x); }
inline void __syncthreads() {}
inline int __builtin_amdgcn_readfirstlane(int v) { return v; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
template <class T> T atomicAdd(T* p, T v) { T o = *p; *p += v; return o; }
#define __HIP_MEMORY_SCOPE_AGENT 3
inline void __builtin_amdgcn_s_sleep(int) {}
inline void __builtin_amdgcn_s_setprio(int) {}
template <class T> inline void __hip_atomic_store(T* p, T v, int, int) { *p = v; }
template <class T> inline T __hip_atomic_load(T* p, int, int) { return *p; }
// Cross-lane operations have no meaning when threads run one at a time; the
// tests emulate the per-lane phases and redo the cross-lane sums themselves.
inline int __builtin_amdgcn_update_dpp(int, int v, int, int, int, bool) { return 0; }
inline int __builtin_amdgcn_readlane(int v, int) { return v; }
