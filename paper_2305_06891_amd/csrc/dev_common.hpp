// Device helpers shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hm {

using bf16_t = uint16_t;  // bfloat16 storage (upper half of an IEEE binary32)

__host__ __device__ inline float bf16_to_f32(bf16_t h) {
  union { uint32_t u; float f; } c;
  c.u = (uint32_t)h << 16;
  return c.f;
}

// Round-to-nearest-even conversion; NaN stays NaN.
__host__ __device__ inline bf16_t f32_to_bf16(float f) {
  union { uint32_t u; float f; } c;
  c.f = f;
  if ((c.u & 0x7f800000u) == 0x7f800000u && (c.u & 0x007fffffu)) return (bf16_t)((c.u >> 16) | 0x40);
  uint32_t lsb = (c.u >> 16) & 1u;
  c.u += 0x7fffu + lsb;
  return (bf16_t)(c.u >> 16);
}

// Dithered rounding of factor entries to BF16: an entry goes to its BF16
// neighbour away from zero with probability equal to its distance from the
// neighbour toward zero (in units of their spacing), so the rounding error
// has mean zero and no correlation between entries.  Round-to-nearest-even
// instead gives near-equal entries (the factors of blocks seen from nearly
// the same direction) errors of one sign, which add up coherently in a
// product.  The draw is a 16-bit value from the SplitMix64 output function
// (Steele, Lea and Flood, OOPSLA 2014) applied twice to a key of the entry:
// factor side (1 for U, 2 for V), the entry's permuted row (U) or column (V)
// in its cavity, the block's first column (U) or row (V), and the rank
// index.  The key does not depend on the batch, so a cavity's factors are
// the same assembled alone or with others.
__host__ __device__ inline uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint32_t dither_draw16(uint32_t side, uint32_t idx, uint32_t other, uint32_t l) {
  constexpr uint64_t gamma = 0x9e3779b97f4a7c15ull;
  const uint64_t z = splitmix64_mix((((uint64_t)side << 32) | idx) + gamma);
  return (uint32_t)(splitmix64_mix(z + ((((uint64_t)other << 32) | l) + gamma)) >> 48);
}
// FP32 -> BF16, dithered by the 16-bit draw r (non-finite values round to
// nearest even)
__host__ __device__ inline bf16_t f32_to_bf16_dither(float f, uint32_t r) {
  union { uint32_t u; float f; } c;
  c.f = f;
  if ((c.u & 0x7f800000u) == 0x7f800000u) return f32_to_bf16(f);
  const uint32_t low = c.u & 0xffffu;
  return (bf16_t)((c.u >> 16) + (r < low ? 1u : 0u));
}

template <class T> struct Cvt;
template <> struct Cvt<double> {
  __device__ static double to_f64(double v) { return v; }
  __device__ static double from_f64(double v) { return v; }
};
template <> struct Cvt<float> {
  __device__ static double to_f64(float v) { return v; }
  __device__ static float from_f64(double v) { return (float)v; }
};
template <> struct Cvt<bf16_t> {
  __device__ static double to_f64(bf16_t v) { return bf16_to_f32(v); }
  // FP64 -> FP32 -> BF16 (double rounding is harmless at BF16 precision for
  // the magnitudes stored here; the FP32 step is exact for the result bits)
  __device__ static bf16_t from_f64(double v) { return f32_to_bf16((float)v); }
};

// Load an element of storage type MT as the arithmetic type VT.
template <class VT, class MT> __device__ inline VT ld_as(const MT* p) { return (VT)(*p); }
template <> __device__ inline float ld_as<float, bf16_t>(const bf16_t* p) { return bf16_to_f32(*p); }
template <> __device__ inline double ld_as<double, bf16_t>(const bf16_t* p) { return (double)bf16_to_f32(*p); }

// Global-memory views of pointers whose address space the compiler cannot
// see (pointers read from descriptors): accesses through them compile to
// global loads and stores rather than flat ones, which would also hold up
// every wait on LDS results.
// (The host pass only parses device code; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using gptr = __attribute__((address_space(1))) T*;
#else
template <class T> using gptr = T*;
#endif
template <class T> __device__ __forceinline__ gptr<const T> gbl(const T* p) { return (gptr<const T>)p; }
template <class T> __device__ __forceinline__ gptr<T> gbl_w(T* p) { return (gptr<T>)p; }
// Data read once per kernel and larger than the caches (factor panels):
// non-temporal loads, which stream past the caches instead of displacing
// the vectors that are reused.
template <class T> __device__ __forceinline__ T ld_stream(const T* p) { return __builtin_nontemporal_load(gbl(p)); }

// A descriptor that every lane of the wave reads at the same address,
// loaded through the constant address space (scalar loads into SGPRs; the
// descriptors do not change while a kernel runs) and kept wave-uniform, so
// that branches on its fields stay scalar and do not wait on unrelated loads.
#if defined(__HIP_DEVICE_COMPILE__)
template <class T> using cptr = __attribute__((address_space(4))) T*;
#else
template <class T> using cptr = T*;
#endif
template <class T> __device__ __forceinline__ T uniform_load(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "descriptor size must be a multiple of 4");
  T v = *(cptr<const T>)p;
  int* w = reinterpret_cast<int*>(&v);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) w[k] = __builtin_amdgcn_readfirstlane(w[k]);
  return v;
}
__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <class T> __device__ inline T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace hm
