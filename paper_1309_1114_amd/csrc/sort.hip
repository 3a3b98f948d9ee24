// Sort and scan primitives of the ordered render (declared in sort.h).
//
// Radix pass over 8 bits of a 32-bit key, stable:
//   k_rs_hist     each workgroup counts the digits of its contiguous slice
//                 (digit-major table: count[digit][workgroup]);
//   (scan)        an exclusive scan of that table gives every workgroup the
//                 first output slot of each digit;
//   k_rs_scatter  each workgroup walks its slice in order, 256 elements at a
//                 time; a wave finds the lanes that share its digit with
//                 eight ballots (rank = earlier peers), the waves of the
//                 workgroup add their per-digit counts in wave order, and a
//                 running count per digit carries over to the next 256.
// Equal digits therefore keep their input order: LSD passes compose to a
// stable sort.
#include "sort.h"

#include <algorithm>

namespace splotch_sort {
namespace {

constexpr int kRT = 256;                 // threads of a radix workgroup
constexpr int kDigits = 256;
constexpr int kMaxRadixBlocks = 2048;
constexpr int kScanThreads = 1024;
constexpr int kScanBlocks = 1024;        // workgroups of the scan's first and last phase

// Temporary layout: [digit table][scan partials][key-range words]
constexpr size_t kHistBytes = (size_t)kDigits * kMaxRadixBlocks * 8;
constexpr size_t kPartBytes = (size_t)(kScanBlocks + 1) * 8;
constexpr size_t kCtrlBytes = 256;

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ size_t eff_n(size_t n, const uint64_t* n_dev) {
    return n_dev ? (size_t)min((uint64_t)n, *n_dev) : n;
}

// Slice [beg, end) of workgroup b of g over n elements (the same in every
// kernel of a pass).
__device__ __forceinline__ void slice(size_t n, int g, int b, size_t& beg, size_t& end) {
    const size_t per = (n + (size_t)g - 1) / (size_t)g;
    beg = min(n, (size_t)b * per);
    end = min(n, beg + per);
}

// Lanes of the wave whose digit equals this lane's (valid lanes only).
__device__ __forceinline__ uint64_t digit_peers(bool valid, uint32_t d) {
    uint64_t peers = wave_ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const bool set = ((d >> bit) & 1u) != 0u;
        const uint64_t m = wave_ballot(valid && set);
        peers &= set ? m : ~m;
    }
    return peers;
}

__global__ __launch_bounds__(kRT) void k_rs_hist(const uint32_t* __restrict__ keys, size_t n_cap,
                                                 const uint64_t* __restrict__ n_dev, int shift,
                                                 uint64_t* __restrict__ hist) {
    __shared__ uint32_t h[kDigits];
    const int tid = threadIdx.x, lane = tid & 63;
    h[tid] = 0u;
    __syncthreads();
    size_t beg, end;
    slice(eff_n(n_cap, n_dev), gridDim.x, blockIdx.x, beg, end);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (size_t base = beg; base < end; base += kRT) {
        const size_t i = base + tid;
        const bool valid = i < end;
        const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
        const uint64_t peers = digit_peers(valid, d);
        if (valid && (peers & lt) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(size_t)tid * gridDim.x + blockIdx.x] = h[tid];
}

__global__ __launch_bounds__(kRT) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                    uint32_t* __restrict__ kout,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ vout, size_t n_cap,
                                                    const uint64_t* __restrict__ n_dev, int shift,
                                                    const uint64_t* __restrict__ offs) {
    __shared__ uint32_t run[kDigits];            // next output slot of each digit
    __shared__ uint32_t wcnt[kRT / 64][kDigits];  // this round's count per wave and digit
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = (uint32_t)offs[(size_t)tid * gridDim.x + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kRT / 64; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    size_t beg, end;
    slice(eff_n(n_cap, n_dev), gridDim.x, blockIdx.x, beg, end);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (size_t base = beg; base < end; base += kRT) {
        const size_t i = base + tid;
        const bool valid = i < end;
        const uint32_t k = valid ? kin[i] : 0u;
        const uint32_t v = valid ? vin[i] : 0u;
        const uint32_t d = (k >> shift) & 255u;
        const uint64_t peers = digit_peers(valid, d);
        if (valid && (peers & lt) == 0ull) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t dst = run[d] + (uint32_t)__popcll(peers & lt);
            for (int w = 0; w < wave; ++w) dst += wcnt[w][d];
            kout[dst] = k;
            vout[dst] = v;
        }
        __syncthreads();
        uint32_t add = 0u;
#pragma unroll
        for (int w = 0; w < kRT / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0u;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of 64-bit values: slice sums, a scan of the sums, then each
// slice scanned from its offset.

__device__ __forceinline__ uint64_t wave_incl_sum64(uint64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t u = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// Inclusive scan over the workgroup (kScanThreads); *total gets the sum.
__device__ __forceinline__ uint64_t block_incl_sum64(uint64_t v, uint64_t* red, uint64_t* total) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    v = wave_incl_sum64(v, lane);
    if (lane == 63) red[wave] = v;
    __syncthreads();
    if (wave == 0) {
        uint64_t s = lane < kScanThreads / 64 ? red[lane] : 0ull;
        s = wave_incl_sum64(s, lane);
        if (lane < kScanThreads / 64) red[lane] = s;
    }
    __syncthreads();
    const uint64_t out = v + (wave > 0 ? red[wave - 1] : 0ull);
    *total = red[kScanThreads / 64 - 1];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partial(const uint64_t* __restrict__ in,
                                                               size_t n,
                                                               uint64_t* __restrict__ part) {
    __shared__ uint64_t red[kScanThreads / 64];
    size_t beg, end;
    slice(n, gridDim.x, blockIdx.x, beg, end);
    uint64_t s = 0;
    for (size_t i = beg + threadIdx.x; i < end; i += kScanThreads) s += in[i];
    uint64_t total;
    (void)block_incl_sum64(s, red, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// One workgroup: exclusive scan of the g slice sums in place.
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint64_t* __restrict__ part, int g) {
    __shared__ uint64_t red[kScanThreads / 64];
    const int t = threadIdx.x;
    const uint64_t v = t < g ? part[t] : 0ull;
    uint64_t total;
    const uint64_t incl = block_incl_sum64(v, red, &total);
    if (t < g) part[t] = incl - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint64_t* in,
                                                            uint64_t* out, size_t n,
                                                            const uint64_t* __restrict__ part) {
    __shared__ uint64_t red[kScanThreads / 64];
    size_t beg, end;
    slice(n, gridDim.x, blockIdx.x, beg, end);
    uint64_t carry = part[blockIdx.x];
    for (size_t base = beg; base < end; base += kScanThreads) {
        const size_t i = base + threadIdx.x;
        const uint64_t v = i < end ? in[i] : 0ull;
        uint64_t total;
        const uint64_t incl = block_incl_sum64(v, red, &total);
        if (i < end) out[i] = carry + incl - v;
        carry += total;
    }
}

// ---------------------------------------------------------------------------
// 64-bit keys: range, 32-bit keys, and the order of runs of equal 32-bit keys

__global__ void k_key_range_init(uint64_t* ctrl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl[0] = ~0ull;
        ctrl[1] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_key_range(const uint64_t* __restrict__ key, size_t n,
                                                   uint64_t* ctrl) {
    uint64_t mn = ~0ull, mx = 0ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        if (k == ~0ull) continue;
        mn = min(mn, k);
        mx = max(mx, k);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mn = min(mn, (uint64_t)__shfl_xor(mn, d, 64));
        mx = max(mx, (uint64_t)__shfl_xor(mx, d, 64));
    }
    if ((threadIdx.x & 63) == 0 && mn <= mx) {
        atomicMin(reinterpret_cast<unsigned long long*>(ctrl), (unsigned long long)mn);
        atomicMax(reinterpret_cast<unsigned long long*>(ctrl + 1), (unsigned long long)mx);
    }
}

// k32 = (key - min) >> s with the smallest s that keeps every drawn key
// below 0xffffffff; keys marked UINT64_MAX map to 0xffffffff.  Monotone, so
// sorting by k32 orders by key except among equal k32.
__global__ __launch_bounds__(256) void k_key32(const uint64_t* __restrict__ key, size_t n,
                                               const uint64_t* __restrict__ ctrl,
                                               uint32_t* __restrict__ k32, uint32_t* __restrict__ v) {
    const uint64_t mn = ctrl[0], mx = ctrl[1];
    const uint64_t range = mx >= mn ? mx - mn : 0ull;
    int s = 0;
    while ((range >> s) >= 0xffffffffull) ++s;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        k32[i] = k == ~0ull ? 0xffffffffu : (uint32_t)((k - mn) >> s);
        v[i] = (uint32_t)i;
    }
}

// Each run of equal k32 (found from its first element) is put in (key,
// value) order by one thread (insertion sort; runs arrive in value order,
// so runs of equal keys cost one comparison per element).
__global__ __launch_bounds__(256) void k_fix_runs(const uint32_t* __restrict__ k32,
                                                  uint32_t* __restrict__ v,
                                                  const uint64_t* __restrict__ key, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t ki = k32[i];
        if (ki == 0xffffffffu || (i > 0 && k32[i - 1] == ki)) continue;
        size_t j = i + 1;
        while (j < n && k32[j] == ki) ++j;
        for (size_t a = i + 1; a < j; ++a) {
            const uint32_t x = v[a];
            const uint64_t kx = key[x];
            size_t b = a;
            while (b > i) {
                const uint32_t y = v[b - 1];
                const uint64_t ky = key[y];
                if (ky < kx || (ky == kx && y < x)) break;
                v[b] = y;
                --b;
            }
            v[b] = x;
        }
    }
}

int grid_for(size_t n, int per_block, int cap) {
    return (int)std::max<size_t>(1, std::min<size_t>((size_t)cap, (n + per_block - 1) / per_block));
}

}  // namespace

int radix_blocks(size_t n_max) { return grid_for(n_max, 16 * kRT, kMaxRadixBlocks); }

size_t temp_bytes(size_t /*n_max*/) { return kHistBytes + kPartBytes + kCtrlBytes; }

void exclusive_sum64(void* temp, const uint64_t* in, uint64_t* out, size_t n, hipStream_t st) {
    if (n == 0) return;
    uint64_t* part = reinterpret_cast<uint64_t*>(static_cast<unsigned char*>(temp) + kHistBytes);
    const int g = grid_for(n, 4 * kScanThreads, kScanBlocks);
    k_scan_partial<<<g, kScanThreads, 0, st>>>(in, n, part);
    k_scan_top<<<1, kScanThreads, 0, st>>>(part, g);
    k_scan_down<<<g, kScanThreads, 0, st>>>(in, out, n, part);
}

int pairs32(void* temp, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, size_t n,
            const uint64_t* n_dev, int end_bit, hipStream_t st) {
    const int passes = (end_bit + 7) / 8;
    if (n == 0) return passes & 1;
    uint64_t* hist = static_cast<uint64_t*>(temp);
    const int g = radix_blocks(n);
    uint32_t *kin = k0, *kout = k1, *vin = v0, *vout = v1;
    for (int p = 0; p < passes; ++p) {
        k_rs_hist<<<g, kRT, 0, st>>>(kin, n, n_dev, 8 * p, hist);
        exclusive_sum64(temp, hist, hist, (size_t)kDigits * g, st);
        k_rs_scatter<<<g, kRT, 0, st>>>(kin, kout, vin, vout, n, n_dev, 8 * p, hist);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
    return passes & 1;
}

void sort_by_key64(void* temp, const uint64_t* key64, uint32_t* k32_0, uint32_t* k32_1,
                   uint32_t* v0, uint32_t* v1, size_t n, hipStream_t st) {
    if (n == 0) return;
    uint64_t* ctrl = reinterpret_cast<uint64_t*>(static_cast<unsigned char*>(temp) + kHistBytes +
                                                 kPartBytes);
    const int g = grid_for(n, 4096, 4096);
    k_key_range_init<<<1, 64, 0, st>>>(ctrl);
    k_key_range<<<g, 256, 0, st>>>(key64, n, ctrl);
    k_key32<<<g, 256, 0, st>>>(key64, n, ctrl, k32_0, v0);
    (void)pairs32(temp, k32_0, k32_1, v0, v1, n, nullptr, 32, st);   // four passes: ends in 0
    k_fix_runs<<<g, 256, 0, st>>>(k32_0, v0, key64, n);
}

}  // namespace splotch_sort
