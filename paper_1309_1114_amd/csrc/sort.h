// Device-wide sort and scan primitives of the ordered (E != A) render, the
// "sort by key" step of Section "CUDA Implementation" written for gfx950:
// a stable least-significant-digit radix sort (8-bit digits; per-workgroup
// digit counts, one exclusive scan, a stable scatter whose ranks come from
// wave ballots) and a three-phase exclusive scan.  Element counts may live
// in device memory, so a pass whose size is only known on the device needs
// no host round trip.  Internal to the library: none of these are exported.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace splotch_sort {

// Workgroups of a radix pass over at most n_max elements, and the temporary
// bytes of every call below for that size.
int radix_blocks(size_t n_max);
size_t temp_bytes(size_t n_max);

// Stable ascending sort of (key, value) pairs by key bits [0, end_bit)
// (end_bit <= 32), ping-ponging between (k0, v0) and (k1, v1).  The count
// is n (n_dev == nullptr) or *n_dev (a device word, at most n).  Returns
// the buffer index (0 or 1) that holds the result: the pass count
// ceil(end_bit / 8) taken modulo 2.
int pairs32(void* temp, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, size_t n,
            const uint64_t* n_dev, int end_bit, hipStream_t st);

// Stable sort of the values 0 .. n-1 by (key64[value], value), for keys
// below 2^63, with UINT64_MAX marking values to put last: the keys are mapped
// on the device to 32 bits (key - min, shifted right past the low bits every
// key shares, and further until the range fits) and sorted by those (four
// passes).  When the mapping drops precision, the dropped bits travel with
// the pairs through the passes and each run of equal 32-bit keys is then
// put in (dropped bits, value) order.  k32_0/k32_1/v0/v1/lo0/lo1 are scratch
// of n entries; the sorted values end in v0.
void sort_by_key64(void* temp, const uint64_t* key64, uint32_t* k32_0, uint32_t* k32_1,
                   uint32_t* v0, uint32_t* v1, uint32_t* lo0, uint32_t* lo1, size_t n,
                   hipStream_t st);

// Exclusive prefix sum out[i] = in[0] + ... + in[i-1] over n values.
void exclusive_sum64(void* temp, const uint64_t* in, uint64_t* out, size_t n, hipStream_t st);

}  // namespace splotch_sort
