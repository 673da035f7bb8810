// Gradient of the spanning-tree weight W = sum over tree edges of
// |x_i - x_j| (the weight in Eq. (1)) with respect to the coordinates, the
// tree held fixed: every edge adds its unit direction (x_i - x_j)/|x_i - x_j|
// to row i and the opposite to row j.  Rows gather their incident edges in
// ascending edge order, so the sums are deterministic.
#include <mutex>

#include "famst_common.hpp"
#include "prims.hpp"

namespace famst {

__global__ void incid_keys_kernel(const int32_t* __restrict__ tu, const int32_t* __restrict__ tv,
                                  int64_t m, int64_t n, uint64_t* __restrict__ keys,
                                  int64_t* __restrict__ deg, int* __restrict__ bad) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  int64_t a = tu[e], b = tv[e];
  if (a < 0 || a >= n || b < 0 || b >= n) {
    atomicOr(bad, 1);
    a = 0;
    b = 0;
  }
  keys[2 * e] = ((uint64_t)a << 32) | (uint64_t)e;
  keys[2 * e + 1] = ((uint64_t)b << 32) | (uint64_t)e;
  atomicAdd(reinterpret_cast<unsigned long long*>(&deg[a]), 1ull);
  atomicAdd(reinterpret_cast<unsigned long long*>(&deg[b]), 1ull);
}

// one 16-lane group per row
__global__ __launch_bounds__(256) void tree_grad_kernel(const float* __restrict__ X, int d, int64_t n,
                                                        const int64_t* __restrict__ offs, int B,
                                                        const int32_t* __restrict__ tu,
                                                        const int32_t* __restrict__ tv,
                                                        const uint64_t* __restrict__ skeys,
                                                        const int64_t* __restrict__ ptr,
                                                        const float* __restrict__ gW,
                                                        float* __restrict__ grad) {
  const int64_t v = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int r16 = threadIdx.x & 15;
  if (v >= n) return;
  const float* xv = X + v * d;
  const float g = gW[find_cloud(offs, B, v)];
  const int64_t p0 = ptr[v], p1 = ptr[v + 1];
  float* out = grad + v * d;
  for (int t0 = 0; t0 < d; t0 += 16 * 8) {
    float acc[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] = 0.f;
    for (int64_t p = p0; p < p1; ++p) {
      uint32_t e = (uint32_t)skeys[p];
      int o = (tu[e] == v) ? tv[e] : tu[e];
      const float* xo = X + (int64_t)o * d;
      float s = sq32_group(xv, xo, d, r16);
      if (s == 0.f) continue;
      float w = __builtin_sqrtf(s);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        int t = t0 + q * 16 + r16;
        if (t < d) acc[q] += (xv[t] - xo[t]) / w;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      int t = t0 + q * 16 + r16;
      if (t < d) out[t] = g * acc[q];
    }
  }
}

// The same sums for d <= 64 NC (NC = 1, 2, 4, 8, 16), d a multiple of 4, 16-byte aligned
// rows: lane r holds dimension chunks r, r + 16, r + 32, ... of its row (the mapping of
// sq32_group, so s has the same bits) in registers, each neighbour row is
// read once as whole chunks, and every element adds the same terms in the
// same edge order as tree_grad_kernel.
template <int NC>
__global__ __launch_bounds__(256) void tree_grad_vec_kernel(const float* __restrict__ X, int d, int64_t n,
                                                            const int64_t* __restrict__ offs, int B,
                                                            const int32_t* __restrict__ tu,
                                                            const int32_t* __restrict__ tv,
                                                            const uint64_t* __restrict__ skeys,
                                                            const int64_t* __restrict__ ptr,
                                                            const float* __restrict__ gW,
                                                            float* __restrict__ grad) {
  const int64_t v = (int64_t)blockIdx.x * 16 + (threadIdx.x >> 4);
  const int r16 = threadIdx.x & 15;
  if (v >= n) return;   // uniform in the 16-lane group
  const float g = gW[find_cloud(offs, B, v)];
  const int64_t p0 = ptr[v], p1 = ptr[v + 1];
  f32x4 a[NC], acc[NC];
  bool ok[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int t0 = 4 * r16 + 64 * c;
    ok[c] = t0 < d;
    a[c] = ok[c] ? *reinterpret_cast<const f32x4*>(X + v * d + t0) : f32x4{0.f, 0.f, 0.f, 0.f};
    acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (int64_t p = p0; p < p1; ++p) {
    const uint32_t e = (uint32_t)skeys[p];
    const int o = (tu[e] == v) ? tv[e] : tu[e];
    f32x4 b[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c)
      b[c] = ok[c] ? *reinterpret_cast<const f32x4*>(X + (int64_t)o * d + 4 * r16 + 64 * c)
                   : f32x4{0.f, 0.f, 0.f, 0.f};
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (ok[c]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float df = a[c][i] - b[c][i];
          s = __builtin_fmaf(df, df, s);
        }
      }
    s += __shfl_xor(s, 8, 16);
    s += __shfl_xor(s, 4, 16);
    s += __shfl_xor(s, 2, 16);
    s += __shfl_xor(s, 1, 16);
    if (s == 0.f) continue;   // uniform in the group
    const float w = __builtin_sqrtf(s);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[c][i] += (a[c][i] - b[c][i]) / w;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (ok[c]) {
      f32x4 r;
#pragma unroll
      for (int i = 0; i < 4; ++i) r[i] = g * acc[c][i];
      *reinterpret_cast<f32x4*>(grad + v * d + 4 * r16 + 64 * c) = r;
    }
}

}  // namespace famst

using namespace famst;

extern "C" int famst_mst_backward(const float* X, int64_t n, int32_t d, const int64_t* offs_h,
                                  int32_t B, const int32_t* tu, const int32_t* tv, const float* gW,
                                  float* grad_X, void* ws, size_t* ws_bytes, void* stream) {
  if (!ws_bytes) return FAMST_EINVAL;
  if (n < 2 || d < 1 || B < 1) return FAMST_EINVAL;
  if (n >= (int64_t(1) << 31)) return FAMST_EINVAL;
  int64_t one[2] = {0, n};
  const int64_t* offs = offs_h ? offs_h : one;
  if (!offs_h && B != 1) return FAMST_EINVAL;
  if (offs[0] != 0 || offs[B] != n) return FAMST_EINVAL;
  for (int b = 0; b < B; ++b)
    if (offs[b + 1] - offs[b] < 2) return FAMST_EINVAL;
  const int64_t m = n - B;
  Carve cv(ws);
  uint64_t* keys = cv.take<uint64_t>(2 * m);
  uint64_t* skeys = cv.take<uint64_t>(2 * m);
  int64_t* deg = cv.take<int64_t>(n + 1);
  int64_t* ptr = cv.take<int64_t>(n + 1);
  int64_t* offs_d = cv.take<int64_t>(B + 1);
  int* bad = cv.take<int>(1);
  size_t tmpb = std::max(sort_keys_u64_bytes(2 * m), scan_i64_bytes(n + 1));
  void* tmp = cv.take<char>(tmpb);
  if (!ws) {
    *ws_bytes = cv.bytes();
    return FAMST_OK;
  }
  if (*ws_bytes < cv.bytes() || (reinterpret_cast<uintptr_t>(ws) & 255)) return FAMST_EWORKSPACE;
  if (!X || !tu || !tv || !gW || !grad_X) return FAMST_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  FAMST_HIP(hipMemcpyAsync(offs_d, offs, sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice, s));
  FAMST_TRY(fill_i32(bad, 0, 1, s));
  FAMST_TRY(fill_i64(deg, 0, n + 1, s));
  FAMST_TRY(launch("incid_keys", incid_keys_kernel, dim3(cdiv(m, 256)), dim3(256), 0, s, tu, tv, m, n,
                   keys, deg, bad));
  // (vertex << 32 | edge) keys: the vertex needs bits_for(n) bits
  FAMST_TRY(sort_keys_u64(tmp, tmpb, keys, skeys, 2 * m, 32 + bits_for(n), s));
  FAMST_TRY(exclusive_scan_i64(tmp, tmpb, deg, ptr, n + 1, s));
  int hbad = 0;
  FAMST_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FAMST_HIP(hipStreamSynchronize(s));
  if (hbad) return FAMST_EINVAL;
  const bool vec = d % 4 == 0 && d <= 1024 && ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(grad_X)) & 15) == 0;
  if (vec) {
    auto kern = d <= 64 ? tree_grad_vec_kernel<1>
              : d <= 128 ? tree_grad_vec_kernel<2>
              : d <= 256 ? tree_grad_vec_kernel<4>
              : d <= 512 ? tree_grad_vec_kernel<8> : tree_grad_vec_kernel<16>;
    return launch("mst_backward", kern, dim3(cdiv(n, 16)), dim3(256), 0, s, X, d, n, offs_d, B, tu, tv, skeys,
                  ptr, gW, grad_X);
  }
  return launch("mst_backward", tree_grad_kernel, dim3(cdiv(n, 16)), dim3(256), 0, s, X, d, n, offs_d, B, tu,
                tv, skeys, ptr, gW, grad_X);
}

// ------------------------------------------------ allocation-free variant
// The workspace of famst_mst_backward lives in a file-scope device array.
// In host code `scratch` names a host-side stand-in, not device memory: its
// device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only that address reaches the kernels.
namespace famst {
static __device__ __align__(256) char scratch[FAMST_NOALLOC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static void* g_scratch_dev[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_address(void** out) {
  int dev = -1;
  FAMST_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return FAMST_ENOTIMPL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FAMST_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return FAMST_OK;
}
}  // namespace famst

extern "C" int famst_mst_backward_noalloc(const float* X, int64_t n, int32_t d, const int64_t* offs_h,
                                          int32_t B, const int32_t* tu, const int32_t* tv, const float* gW,
                                          float* grad_X, size_t* scratch_needed, void* stream) {
  size_t need = 0;
  FAMST_TRY(famst_mst_backward(X, n, d, offs_h, B, tu, tv, gW, grad_X, nullptr, &need, stream));
  if (scratch_needed) *scratch_needed = need;
  if (need > FAMST_NOALLOC_SCRATCH_BYTES) return FAMST_ECAPACITY;
  if (!X || !tu || !tv || !gW || !grad_X) return FAMST_EINVAL;
  void* ws = nullptr;
  FAMST_TRY(scratch_address(&ws));
  return famst_mst_backward(X, n, d, offs_h, B, tu, tv, gW, grad_X, ws, &need, stream);
}
