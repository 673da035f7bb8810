#include "prims.hpp"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace famst {

size_t sort_keys_u64_bytes(size_t n) {
  size_t b = 0;
  rocprim::radix_sort_keys(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr, n, 0, 64);
  return b;
}
size_t sort_pairs_u64_u32_bytes(size_t n) {
  size_t b = 0;
  rocprim::radix_sort_pairs(nullptr, b, (uint64_t*)nullptr, (uint64_t*)nullptr,
                            (uint32_t*)nullptr, (uint32_t*)nullptr, n, 0, 64);
  return b;
}
size_t sort_pairs_u32_i32_bytes(size_t n) {
  size_t b = 0;
  rocprim::radix_sort_pairs(nullptr, b, (uint32_t*)nullptr, (uint32_t*)nullptr,
                            (int32_t*)nullptr, (int32_t*)nullptr, n, 0, 32);
  return b;
}
size_t scan_i64_bytes(size_t n) {
  size_t b = 0;
  rocprim::exclusive_scan(nullptr, b, (int64_t*)nullptr, (int64_t*)nullptr, int64_t(0), n,
                          rocprim::plus<int64_t>());
  return b;
}

int sort_keys_u64(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, size_t n,
                  int end_bit, hipStream_t s) {
  if (n == 0) return FAMST_OK;
  prof_begin("sort", s);
  hipError_t e = rocprim::radix_sort_keys(tmp, tmp_bytes, in, out, n, 0, end_bit, s);
  prof_end(s);
  return e == hipSuccess ? FAMST_OK : FAMST_EHIP;
}
int sort_pairs_u64_u32(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout,
                       const uint32_t* vin, uint32_t* vout, size_t n, int end_bit, hipStream_t s) {
  if (n == 0) return FAMST_OK;
  prof_begin("sort", s);
  hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, end_bit, s);
  prof_end(s);
  return e == hipSuccess ? FAMST_OK : FAMST_EHIP;
}
int sort_pairs_u32_i32(void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout,
                       const int32_t* vin, int32_t* vout, size_t n, int end_bit, hipStream_t s) {
  if (n == 0) return FAMST_OK;
  prof_begin("sort", s);
  hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, n, 0, end_bit, s);
  prof_end(s);
  return e == hipSuccess ? FAMST_OK : FAMST_EHIP;
}
int exclusive_scan_i64(void* tmp, size_t tmp_bytes, const int64_t* in, int64_t* out, size_t n,
                       hipStream_t s) {
  if (n == 0) return FAMST_OK;
  prof_begin("scan", s);
  hipError_t e = rocprim::exclusive_scan(tmp, tmp_bytes, in, out, int64_t(0), n,
                                         rocprim::plus<int64_t>(), s);
  prof_end(s);
  return e == hipSuccess ? FAMST_OK : FAMST_EHIP;
}

template <class T>
__global__ void fill_kernel(T* p, T v, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void iota_kernel(int32_t* p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int32_t)i;
}

int fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s) {
  return launch("fill", fill_kernel<int32_t>, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
}
int fill_i64(int64_t* p, int64_t v, size_t n, hipStream_t s) {
  return launch("fill", fill_kernel<int64_t>, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
}
int fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
  return launch("fill", fill_kernel<uint64_t>, dim3(cdiv(n, 256)), dim3(256), 0, s, p, v, n);
}
int iota_i32(int32_t* p, size_t n, hipStream_t s) {
  return launch("iota", iota_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, p, n);
}

}  // namespace famst
