// knn_common.cuh -- device helpers shared by the HIP kernels (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "knn_internal.h"

namespace knn {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kSentinel = 0x7FFFFFF0;  // "no row yet" index; +4 still fits int32

// 2^k as a float for k in [-149, 127] (exact)
__device__ __forceinline__ float exp2i(int k) {
  return k >= -126 ? __uint_as_float((unsigned)(k + 127) << 23) : __uint_as_float(1u << (k + 149));
}

// element d of row `row` of a row-major FP32 or BF16 array, widened exactly to FP32
__device__ __forceinline__ float load_elem(const void* src, int dt, int64_t i) {
  if (dt == DT_F32) return reinterpret_cast<const float*>(src)[i];
  unsigned short b = reinterpret_cast<const unsigned short*>(src)[i];
  return __uint_as_float((unsigned)b << 16);
}

// FP32 -> BF16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return u >> 16;
}

// FP32 -> OCP E4M3 code, round to nearest even, saturating at +-448 (finite inputs).
// Every step before the rounding is an exact scaling by a power of two.
__device__ __forceinline__ unsigned fp8_e4m3_rne(float y) {
  unsigned sign = (__float_as_uint(y) >> 31) << 7;
  float a = fabsf(y);
  if (a >= 448.f) return sign | 0x7Eu;
  unsigned code;
  if (a < 0.015625f) {  // below the smallest normal 2^-6: spacing 2^-9
    code = (unsigned)__builtin_rintf(a * 512.f);  // 8 rolls into the first normal code
  } else {
    int E = (int)((__float_as_uint(a) >> 23) & 255u) - 127;  // -6..8
    float q = (a * exp2i(-E) - 1.f) * 8.f;                    // mantissa steps, exact
    code = (unsigned)(E + 7) * 8u + (unsigned)__builtin_rintf(q);
  }
  if (code > 0x7Eu) code = 0x7Eu;
  return sign | code;
}

__device__ __forceinline__ float fp8_e4m3_value(unsigned c) {
  unsigned E = (c >> 3) & 15u, m = c & 7u;
  float v = E == 0 ? (float)m * 0.001953125f : (float)(8u + m) * exp2i((int)E - 10);
  return (c & 0x80u) ? -v : v;
}

// smallest e with amax <= 448 * 2^e, clamped to [-127, 127]; 0 for amax == 0
__device__ __forceinline__ int fp8_row_exponent(float amax) {
  if (!(amax > 0.f)) return 0;
  int ef = (int)((__float_as_uint(amax) >> 23) & 255u);
  int e = ef - 127 - 8;
  if (e < -127) return -127;
  if (amax * exp2i(-e) > 448.f) e += 1;
  return e > 127 ? 127 : e;
}

// order-preserving map float -> uint32 (larger float -> larger key)
__device__ __forceinline__ unsigned float_key(float v) {
  unsigned u = __float_as_uint(v);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float key_float(unsigned k) {
  unsigned u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)v, m), hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), m);
  return ((unsigned long long)hi << 32) | lo;
}

// Sort 64*R keys held by one wave (element e = 64*r + lane) in descending order:
// a bitonic network whose exchanges within a lane's registers are plain compares
// and whose exchanges across lanes are shuffles.
template <int R>
__device__ __forceinline__ void wave_sort_desc(unsigned long long (&k)[R], int lane) {
  constexpr int N = 64 * R;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (r & rs) continue;  // handle each in-lane pair once, from its lower element
          const int e = 64 * r + lane;
          const bool desc = (e & size) == 0;
          const unsigned long long a = k[r], b = k[r | rs];
          const bool sw = desc ? (a < b) : (a > b);
          k[r] = sw ? b : a;
          k[r | rs] = sw ? a : b;
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int e = 64 * r + lane;
          const bool desc = (e & size) == 0, lower = (e & stride) == 0;
          const unsigned long long o = shfl_xor_u64(k[r], stride);
          const bool take_max = desc == lower;
          k[r] = take_max ? (o > k[r] ? o : k[r]) : (o < k[r] ? o : k[r]);
        }
      }
    }
  }
}

// first row of bin b under the contiguous balanced partition
__device__ __forceinline__ int64_t bin_start(int64_t b, int64_t N, int64_t L) {
  return (int64_t)(((unsigned long long)b * (unsigned long long)N) / (unsigned long long)L);
}

}  // namespace knn
