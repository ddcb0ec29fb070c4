// Device-side helpers shared by the ragsnn kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

constexpr int WAVE = 64;

// Random stream tags: key word 1 = tag | proj << 8.
enum Tag : uint32_t {
  TAG_CONN = 1, TAG_WINIT = 2, TAG_SIGN = 3, TAG_DR_ROW = 4, TAG_DR_TGT = 5,
  TAG_TP_ROW = 6, TAG_TP_TGT = 7, TAG_TP_ELIM = 8, TAG_TP_FORM = 9, TAG_INPUT = 10,
  TAG_STIM = 11, TAG_TP_INPUT = 12, TAG_CUSTOM = 13
};
constexpr int MAX_TRIES = 64;   // draws before the bounded fallback scan
constexpr int MAX_ROUNDS = 64;  // redistribution rounds before deterministic fallback
constexpr double FIX_SCALE = 68719476736.0;       // 2^36: fixed-point input accumulation
constexpr double FIX_INV = 1.0 / 68719476736.0;

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based generator.
struct U64x4 { uint64_t x0, x1, x2, x3; };

__device__ __forceinline__ U64x4 philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1,
                                        uint64_t c2, uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t draw_u32(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0,
                                             uint64_t c1, uint64_t c2, uint64_t c3) {
  U64x4 o = philox(seed, (uint64_t)tag | ((uint64_t)proj << 8), c0, c1, c2, c3);
  return (uint32_t)(o.x0 >> 32);
}

// integer uniformly below n (multiply-shift)
__device__ __forceinline__ uint32_t below(uint32_t u, uint32_t n) {
  return (uint32_t)(((uint64_t)u * (uint64_t)n) >> 32);
}

// standard normal by Box-Muller on output words 0 and 1, in double
__device__ __forceinline__ double draw_normal(uint64_t seed, uint32_t tag, uint32_t proj, uint64_t c0,
                                              uint64_t c1, uint64_t c2, uint64_t c3) {
  U64x4 o = philox(seed, (uint64_t)tag | ((uint64_t)proj << 8), c0, c1, c2, c3);
  const double two_m53 = 1.0 / 9007199254740992.0;
  double u1 = (double)((o.x0 >> 11) + 1) * two_m53;
  double u2 = (double)(o.x1 >> 11) * two_m53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

// ---- wave-level reductions (deterministic order, same result in every lane) ----
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// A read through a pointer known to address global memory: a global load
// counts only in the vector-memory counter, so waits for LDS reads after it
// do not wait for it (a flat load counts in both).
template <class T>
__device__ __forceinline__ T ld_global(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

// Sum over the 64 lanes: DPP adds within each row of 16 lanes (quad swaps,
// half-row and row mirrors), then the four row sums combined in a fixed order.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_f32<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f32<0x141>(v);  // row_half_mirror
  v += dpp_f32<0x140>(v);  // row_mirror
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
  return (r0 + r1) + (r2 + r3);
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, WAVE));
  return v;
}
__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Index of the calling wave in its workgroup, as a wave-uniform value.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x / WAVE)); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ bool get_bit(const uint32_t* bits, int words, int row, int j) {
  return (bits[(int64_t)row * words + (j >> 5)] >> (j & 31)) & 1u;
}

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// Allow a kernel up to `want` bytes of dynamic LDS, clamped to what the current
// device offers per workgroup; leaves no pending runtime error behind.
inline void allow_dynamic_lds(const void* kernel, int want) {
  int dev = 0, cap = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cap, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess) {
    int v = want < cap ? want : cap;
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, v - 1024);
  }
  (void)hipGetLastError();
}

}  // namespace rs
