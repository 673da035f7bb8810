// Shared device helpers and host plumbing of libfamst (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>
#include <stddef.h>

#include "../../include/famst.h"

namespace famst {

// ---------------------------------------------------------------- types
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef __attribute__((__vector_size__(4 * sizeof(int)))) int i32x4;
typedef __attribute__((__vector_size__(8 * sizeof(int)))) int i32x8;
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int WAVE = 64;
constexpr float F_INF = __builtin_inff();

// ------------------------------------------------------------ host status
struct Status {
  int code = FAMST_OK;
};

#define FAMST_HIP(call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return FAMST_EHIP;              \
  } while (0)

#define FAMST_TRY(call)                                   \
  do {                                                    \
    int s_ = (call);                                      \
    if (s_ < 0) return s_;                                \
  } while (0)

// Carves a caller-provided workspace.  Run once with base == nullptr to
// compute the size, then with the real base.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~size_t(255); }
};

// ------------------------------------------------------------- profiling
void prof_begin(const char* name, hipStream_t s);
void prof_end(hipStream_t s);

template <class K, class... Args>
inline int launch(const char* name, K kernel, dim3 grid, dim3 block, size_t lds,
                  hipStream_t s, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return FAMST_OK;
  // a dispatch holds fewer than 2^32 work-items
  if ((uint64_t)grid.x * grid.y * grid.z * block.x * block.y * block.z >= (uint64_t(1) << 32))
    return FAMST_ENOTIMPL;
  prof_begin(name, s);
  hipLaunchKernelGGL(kernel, grid, block, lds, s, args...);
  hipError_t e = hipGetLastError();
  prof_end(s);
  return e == hipSuccess ? FAMST_OK : FAMST_EHIP;
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Grid of a kernel that loops over its work units with a stride of the grid:
// enough blocks to fill the chip many times over, far below the dispatch limit.
constexpr int64_t kMaxStrideBlocks = int64_t(1) << 20;
inline unsigned stride_grid(int64_t units) { return (unsigned)std::min<int64_t>(units, kMaxStrideBlocks); }

// ------------------------------------------------------- device helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned long long ballot(bool p) {
  return __ballot(p);
}

__device__ __forceinline__ float readlane_f(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ int readlane_i(int v, int l) {
  return __builtin_amdgcn_readlane(v, l);
}

// Relative error bound of the float32 direct-difference squared distance
// computed by sq32_group below: each of 16 lanes sums at most
// 4 ceil(d/64) products with fused multiply-adds, then 4 pairwise
// additions, and the differences are rounded once.  Doubled for safety
// margin.
__host__ __device__ inline float tau32(int d) {
  int m = 4 * ((d + 63) / 64);
  return 2.0f * (float)(m + 4 + 2) * 5.9604645e-8f;  // 2^-24
}

// Canonical float32 squared distance by direct difference.  The dimensions
// form chunks of four (chunk c = dimensions 4c .. 4c+3); partial sum r
// (r = 0..15) runs over chunks r, r+16, r+32, ... in ascending dimension
// order with fmaf, and the 16 partials are combined pairwise as
// ((p0+p8)+(p4+p12)) + ((p2+p10)+(p6+p14)) + ... , i.e. an xor butterfly
// over 8, 4, 2, 1.  Every kernel that needs a float32 distance produces
// exactly these bits, whatever its lane mapping (IEEE addition is
// commutative), and sq32(a, b) == sq32(b, a) because (a-b)^2 == (b-a)^2.
//
// This version is evaluated by a group of 16 consecutive lanes; lane r owns
// partial r and all lanes of the group return the same bits.
__device__ __forceinline__ float sq32_group(const float* __restrict__ a,
                                            const float* __restrict__ b, int d, int r) {
  float acc = 0.f;
  const bool vec = (((uintptr_t)a | (uintptr_t)b) & 15) == 0;
  for (int t0 = 4 * r; t0 < d; t0 += 64) {
    if (vec && t0 + 4 <= d) {
      const f32x4 xa = *reinterpret_cast<const f32x4*>(a + t0);
      const f32x4 xb = *reinterpret_cast<const f32x4*>(b + t0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float df = xa[i] - xb[i];
        acc = __builtin_fmaf(df, df, acc);
      }
    } else {
      for (int t = t0; t < t0 + 4 && t < d; ++t) {
        const float df = a[t] - b[t];
        acc = __builtin_fmaf(df, df, acc);
      }
    }
  }
  acc += __shfl_xor(acc, 8, 16);
  acc += __shfl_xor(acc, 4, 16);
  acc += __shfl_xor(acc, 2, 16);
  acc += __shfl_xor(acc, 1, 16);
  return acc;
}

// float64 squared distance of the same pair (used only to order two
// float32 values that are within rounding of each other).
__device__ __forceinline__ double sq64_group(const float* __restrict__ a,
                                             const float* __restrict__ b, int d, int r) {
  double acc = 0.0;
  for (int t0 = 4 * r; t0 < d; t0 += 64)
    for (int t = t0; t < t0 + 4 && t < d; ++t) {
      double df = (double)a[t] - (double)b[t];
      acc = __builtin_fma(df, df, acc);
    }
  acc += __shfl_xor(acc, 8, 16);
  acc += __shfl_xor(acc, 4, 16);
  acc += __shfl_xor(acc, 2, 16);
  acc += __shfl_xor(acc, 1, 16);
  return acc;
}

// (s, id) lexicographic order.
__device__ __forceinline__ bool key_less(float s1, int i1, float s2, int i2) {
  return s1 < s2 || (s1 == s2 && i1 < i2);
}
__device__ __forceinline__ bool key_less64(double s1, int i1, double s2, int i2) {
  return s1 < s2 || (s1 == s2 && i1 < i2);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the
// two-multiplier S-box with a Weyl-sequence key schedule.
struct U4 { uint32_t x, y, z, w; };
__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    U4 o;
    o.x = hi1 ^ c.y ^ k0;
    o.y = lo1;
    o.z = hi0 ^ c.w ^ k1;
    o.w = lo0;
    c = o;
    k0 += W0;
    k1 += W1;
  }
  return c;
}

// (r * size) >> 32
__device__ __forceinline__ uint32_t range_map(uint32_t r, uint32_t size) {
  return __umulhi(r, size);
}

// IEEE float32 -> bfloat16 bits, round to nearest even (finite inputs).
__host__ __device__ inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__host__ __device__ inline float bf16_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, (uint32_t)b << 16);
}

// Binary search: index b with offs[b] <= v < offs[b+1] (offs ascending).
__device__ __forceinline__ int find_cloud(const int64_t* offs, int B, int64_t v) {
  int lo = 0, hi = B - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace famst
