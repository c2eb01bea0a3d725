// Sorting and scan primitives used while a plan is built (rocPRIM device
// algorithms: stable LSD radix sort and a prefix scan of integers, both
// deterministic).
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "internal.h"

namespace fmm {

size_t sort_pairs_u64_i32_temp(int n) {
  size_t bytes = 0;
  FMM_HIP(rocprim::radix_sort_pairs(nullptr, bytes, (const uint64_t*)nullptr,
                                    (uint64_t*)nullptr, (const int32_t*)nullptr,
                                    (int32_t*)nullptr, (unsigned)n));
  return bytes;
}

void sort_pairs_u64_i32(void* temp, size_t temp_bytes, const uint64_t* kin,
                        uint64_t* kout, const int32_t* vin, int32_t* vout,
                        int n, hipStream_t st) {
  FMM_HIP(rocprim::radix_sort_pairs(temp, temp_bytes, kin, kout, vin, vout,
                                    (unsigned)n, 0, 64, st));
}

size_t sort_keys_u64_temp(int64_t n) {
  size_t bytes = 0;
  FMM_HIP(rocprim::radix_sort_keys(nullptr, bytes, (const uint64_t*)nullptr,
                                   (uint64_t*)nullptr, (size_t)n));
  return bytes;
}

void sort_keys_u64(void* temp, size_t temp_bytes, const uint64_t* kin,
                   uint64_t* kout, int64_t n, int end_bit, hipStream_t st) {
  FMM_HIP(rocprim::radix_sort_keys(temp, temp_bytes, kin, kout, (size_t)n, 0,
                                   (unsigned)end_bit, st));
}

size_t scan_i32_temp(int64_t n) {
  size_t bytes = 0;
  FMM_HIP(rocprim::exclusive_scan(nullptr, bytes, (const int32_t*)nullptr,
                                  (int32_t*)nullptr, 0, (size_t)n,
                                  rocprim::plus<int32_t>()));
  return bytes;
}

void exclusive_scan_i32(void* temp, size_t temp_bytes, const int32_t* in,
                        int32_t* out, int64_t n, hipStream_t st) {
  FMM_HIP(rocprim::exclusive_scan(temp, temp_bytes, in, out, 0, (size_t)n,
                                  rocprim::plus<int32_t>(), st));
}

}  // namespace fmm
