// Device kernels of the colour-coding dynamic programme for gfx950
// (wave64).  Every kernel is bound by memory traffic (HBM, L2 or LDS), none
// is a dense contraction, so none uses MFMA.
//
// Table layout: a count table of a sub-template with `cols` colour-set
// columns holds b colourings side by side: element (i, j*cols + c) of a
// row-major n x ld array (ld padded to 128 bytes).  Colourings are stored
// colouring-major, one byte per vertex.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace sg2v {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int WAVES_PER_BLOCK = BLOCK / WAVE;

// Block coordinates of a kernel body: the hardware's (HwBlk), or a virtual
// block of a recorded launch run by the persistent scheduler (VBlk).
struct HwBlk {
  __device__ unsigned x() const { return blockIdx.x; }
  __device__ unsigned y() const { return blockIdx.y; }
  __device__ unsigned gx() const { return gridDim.x; }
  __device__ unsigned gy() const { return gridDim.y; }
};
struct VBlk {
  unsigned bx, by, ngx, ngy;
  __device__ unsigned x() const { return bx; }
  __device__ unsigned y() const { return by; }
  __device__ unsigned gx() const { return ngx; }
  __device__ unsigned gy() const { return ngy; }
};

template <typename T>
constexpr bool is_u64 = std::is_same<T, uint64_t>::value;

// ---------------------------------------------------------------------------
// element arithmetic: float/double add and fused multiply-add; uint64 adds and
// multiplies modulo 2^64 with an overflow flag.

template <typename T>
struct Arith {
  __device__ static inline T add(T a, T b, bool &) { return a + b; }
  __device__ static inline T mul(T a, T b, bool &) { return a * b; }
  __device__ static inline T fma(T a, T b, T c, bool &) { return a * b + c; }
};

template <>
struct Arith<uint64_t> {
  __device__ static inline uint64_t add(uint64_t a, uint64_t b, bool &ovf) {
    uint64_t r = a + b;
    ovf |= r < a;
    return r;
  }
  __device__ static inline uint64_t mul(uint64_t a, uint64_t b, bool &ovf) {
    ovf |= __umul64hi(a, b) != 0;
    return a * b;
  }
  __device__ static inline uint64_t fma(uint64_t a, uint64_t b, uint64_t c, bool &ovf) {
    return add(mul(a, b, ovf), c, ovf);
  }
};

// 16-byte vector of T
template <typename T>
struct alignas(16) V16 {
  static constexpr int N = 16 / sizeof(T);
  T x[N];
};

// wave shuffles for 4- and 8-byte values (ds_bpermute)
__device__ inline int shfl_i32(int v, int src) {
  return __builtin_amdgcn_ds_bpermute(src << 2, v);
}
template <typename T>
__device__ inline T shfl(T v, int src) {
  if constexpr (sizeof(T) == 4) {
    int x = shfl_i32(__builtin_bit_cast(int, v), src);
    return __builtin_bit_cast(T, x);
  } else {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    int lo = shfl_i32((int)(uint32_t)u, src);
    int hi = shfl_i32((int)(uint32_t)(u >> 32), src);
    return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
  }
}
template <typename T>
__device__ inline T shfl_xor(T v, int mask) {
  int lane = threadIdx.x & (WAVE - 1);
  return shfl(v, lane ^ mask);
}

// float exponent helpers for the FP32 per-column scaling
__device__ inline int ilog2_bits(uint32_t bits) {  // floor(log2 x) for x > 0 (subnormal: -127)
  return (int)((bits >> 23) & 0xFF) - 127;
}
__device__ inline float exp2_int(int d) {  // exact 2^d as float, 0 below the subnormal range
  if (d > 127) d = 127;
  if (d >= -126) return __builtin_bit_cast(float, (uint32_t)(d + 127) << 23);
  if (d >= -149) return __builtin_bit_cast(float, 1u << (d + 149));
  return 0.0f;
}

}  // namespace sg2v
