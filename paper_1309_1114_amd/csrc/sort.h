// Device-wide sort and scan primitives of the ordered (E != A) render,
// implemented with rocPRIM in sort.hip (a translation unit of its own, so
// the heavy templates compile once and in parallel with the rest).
// Internal to the library: none of these are exported.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace splotch_sort {

// Stable ascending radix sort of (key, value) pairs on key bits
// [0, end_bit).  temp_bytes for a size is returned by the *_temp query.
size_t pairs64_temp(size_t n);
hipError_t pairs64(void* temp, size_t temp_bytes, const uint64_t* keys_in, uint64_t* keys_out,
                   const uint32_t* vals_in, uint32_t* vals_out, size_t n, int end_bit,
                   hipStream_t st);
size_t pairs32_temp(size_t n);
hipError_t pairs32(void* temp, size_t temp_bytes, const uint32_t* keys_in, uint32_t* keys_out,
                   const uint32_t* vals_in, uint32_t* vals_out, size_t n, int end_bit,
                   hipStream_t st);

// Exclusive prefix sum out[i] = in[0] + ... + in[i-1] over n values.
size_t exclusive_sum64_temp(size_t n);
hipError_t exclusive_sum64(void* temp, size_t temp_bytes, const uint64_t* in, uint64_t* out,
                           size_t n, hipStream_t st);

}  // namespace splotch_sort
