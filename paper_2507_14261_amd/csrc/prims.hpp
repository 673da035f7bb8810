// Device-wide sort and scan primitives (rocPRIM radix sort / scan) and a
// few elementwise kernels shared by the phases.
#pragma once
#include "famst_common.hpp"

namespace famst {

// Temporary-storage sizes (bytes) for the primitives below.
size_t sort_keys_u64_bytes(size_t n);
size_t sort_pairs_u64_u32_bytes(size_t n);
size_t sort_pairs_u32_i32_bytes(size_t n);
size_t scan_i64_bytes(size_t n);

// Stable LSD radix sorts on bits [0, end_bit).
int sort_keys_u64(void* tmp, size_t tmp_bytes, const uint64_t* in, uint64_t* out, size_t n,
                  int end_bit, hipStream_t s);
int sort_pairs_u64_u32(void* tmp, size_t tmp_bytes, const uint64_t* kin, uint64_t* kout,
                       const uint32_t* vin, uint32_t* vout, size_t n, int end_bit, hipStream_t s);
int sort_pairs_u32_i32(void* tmp, size_t tmp_bytes, const uint32_t* kin, uint32_t* kout,
                       const int32_t* vin, int32_t* vout, size_t n, int end_bit, hipStream_t s);
// out[i] = sum_{j<i} in[j], i in [0, n)
int exclusive_scan_i64(void* tmp, size_t tmp_bytes, const int64_t* in, int64_t* out, size_t n,
                       hipStream_t s);

int fill_i32(int32_t* p, int32_t v, size_t n, hipStream_t s);
int fill_i64(int64_t* p, int64_t v, size_t n, hipStream_t s);
int fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
int iota_i32(int32_t* p, size_t n, hipStream_t s);

inline int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

}  // namespace famst
