// rocPRIM instantiations behind sort.h.
#include "sort.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

namespace splotch_sort {

size_t pairs64_temp(size_t n) {
    size_t b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                    (const uint32_t*)nullptr, (uint32_t*)nullptr, n, 0u, 64u);
    return b;
}

hipError_t pairs64(void* temp, size_t temp_bytes, const uint64_t* keys_in, uint64_t* keys_out,
                   const uint32_t* vals_in, uint32_t* vals_out, size_t n, int end_bit,
                   hipStream_t st) {
    return rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, n,
                                     0u, (unsigned)end_bit, st);
}

size_t pairs32_temp(size_t n) {
    size_t b = 0;
    (void)rocprim::radix_sort_pairs(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                    (const uint32_t*)nullptr, (uint32_t*)nullptr, n, 0u, 32u);
    return b;
}

hipError_t pairs32(void* temp, size_t temp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                   const uint32_t* vals_in, uint32_t* vals_out, size_t n, int end_bit,
                   hipStream_t st) {
    return rocprim::radix_sort_pairs(temp, temp_bytes, keys_in, keys_out, vals_in, vals_out, n,
                                     0u, (unsigned)end_bit, st);
}

size_t exclusive_sum64_temp(size_t n) {
    size_t b = 0;
    (void)rocprim::exclusive_scan(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                  (uint64_t)0, n, rocprim::plus<uint64_t>());
    return b;
}

hipError_t exclusive_sum64(void* temp, size_t temp_bytes, const uint64_t* in, uint64_t* out,
                           size_t n, hipStream_t st) {
    return rocprim::exclusive_scan(temp, temp_bytes, in, out, (uint64_t)0, n,
                                   rocprim::plus<uint64_t>(), st);
}

}  // namespace splotch_sort
