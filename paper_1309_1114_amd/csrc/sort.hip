// Sort and scan primitives of the ordered render (declared in sort.h).
//
// Radix pass over 8 bits of a 32-bit key, stable:
//   k_rs_hist     each workgroup counts the digits of its contiguous slice
//                 (digit-major table: count[digit][workgroup]);
//   (scan)        an exclusive scan of that table gives every workgroup the
//                 first output slot of each digit;
//   k_rs_scatter  each workgroup walks its slice in order, in tiles of 4096
//                 elements: a wave finds the lanes that share its digit with
//                 eight ballots (rank = earlier peers), the waves of the
//                 workgroup add their per-digit counts in wave order, round
//                 after round; the tile is laid out by digit in LDS and
//                 written so that each digit's elements go to consecutive
//                 slots, after the earlier tiles' (a running count per digit).
// Equal digits therefore keep their input order: LSD passes compose to a
// stable sort.
#include "sort.h"

#include <algorithm>

namespace splotch_sort {
namespace {

constexpr int kRT = 256;                 // threads of a radix workgroup
constexpr int kRounds = 16;              // elements per thread of a scatter tile
constexpr int kHistBatch = 8;            // keys per thread in flight while counting
constexpr int kTile = kRT * kRounds;
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
    // kHistBatch keys per thread are loaded before any is counted, so each
    // wave keeps several loads in flight
    for (size_t base = beg; base < end; base += (size_t)kHistBatch * kRT) {
        uint32_t d[kHistBatch];
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const size_t i = base + (size_t)u * kRT + tid;
            d[u] = i < end ? (keys[i] >> shift) & 255u : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const bool valid = base + (size_t)u * kRT + tid < end;
            const uint64_t peers = digit_peers(valid, d[u]);
            if (valid && (peers & lt) == 0ull) atomicAdd(&h[d[u]], (uint32_t)__popcll(peers));
        }
    }
    __syncthreads();
    hist[(size_t)tid * gridDim.x + blockIdx.x] = h[tid];
}

// Each workgroup walks its slice in tiles of kTile elements (element
// tile_base + r * kRT + tid in round r).  Ranks within the tile come round by
// round (earlier rounds, then earlier waves, then earlier lanes with the same
// digit), so they follow input order; the tile is then laid out in LDS by
// digit and written out in that order, each digit's elements to
// consecutive output slots.
__global__ __launch_bounds__(kRT) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                    uint32_t* __restrict__ kout,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ vout, size_t n_cap,
                                                    const uint64_t* __restrict__ n_dev, int shift,
                                                    const uint64_t* __restrict__ offs) {
    __shared__ uint32_t sk[kTile], sv[kTile];     // the tile, by digit
    __shared__ uint32_t run[kDigits];            // next output slot of each digit
    __shared__ uint32_t tc[kDigits];             // tile count so far, then tile start
    __shared__ uint32_t wcnt[kRT / 64][kDigits];  // this round's count per wave and digit
    __shared__ uint32_t red[kRT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = (uint32_t)offs[(size_t)tid * gridDim.x + blockIdx.x];
    tc[tid] = 0u;
#pragma unroll
    for (int w = 0; w < kRT / 64; ++w) wcnt[w][tid] = 0u;
    __syncthreads();
    size_t beg, end;
    slice(eff_n(n_cap, n_dev), gridDim.x, blockIdx.x, beg, end);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (size_t tb = beg; tb < end; tb += kTile) {
        const int tn = (int)min((size_t)kTile, end - tb);
        uint32_t key[kRounds], val[kRounds], rank[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int j = r * kRT + tid;
            const bool valid = j < tn;
            key[r] = valid ? kin[tb + j] : 0u;
            val[r] = valid ? vin[tb + j] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const bool valid = r * kRT + tid < tn;
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint64_t peers = digit_peers(valid, d);
            if (valid && (peers & lt) == 0ull) wcnt[wave][d] = (uint32_t)__popcll(peers);
            __syncthreads();
            uint32_t rk = tc[d] + (uint32_t)__popcll(peers & lt);
            for (int w = 0; w < wave; ++w) rk += wcnt[w][d];
            rank[r] = rk;
            __syncthreads();
            uint32_t add = 0u;
#pragma unroll
            for (int w = 0; w < kRT / 64; ++w) {
                add += wcnt[w][tid];
                wcnt[w][tid] = 0u;
            }
            tc[tid] += add;
            __syncthreads();
        }
        // exclusive scan of the tile counts: tc becomes each digit's start
        const uint32_t cnt = tc[tid];
        uint32_t incl = cnt;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t u = __shfl_up(incl, (unsigned)d, 64);
            if (lane >= d) incl += u;
        }
        if (lane == 63) red[wave] = incl;
        __syncthreads();
        uint32_t before = 0u;
        for (int w = 0; w < wave; ++w) before += red[w];
        tc[tid] = before + incl - cnt;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            if (r * kRT + tid < tn) {
                const uint32_t d = (key[r] >> shift) & 255u;
                const uint32_t pos = tc[d] + rank[r];
                sk[pos] = key[r];
                sv[pos] = val[r];
            }
        }
        __syncthreads();
        for (int j = tid; j < tn; j += kRT) {
            const uint32_t k = sk[j];
            const uint32_t d = (k >> shift) & 255u;
            const uint32_t dst = run[d] + ((uint32_t)j - tc[d]);
            kout[dst] = k;
            vout[dst] = sv[j];
        }
        __syncthreads();
        // next tile: advance each digit's output slot, clear the counts
        run[tid] += cnt;
        tc[tid] = 0u;
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

// ctrl: [0] min, [1] max, [2] AND, [3] OR of the drawn keys.
__global__ void k_key_range_init(uint64_t* ctrl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl[0] = ~0ull;
        ctrl[1] = 0ull;
        ctrl[2] = ~0ull;
        ctrl[3] = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_key_range(const uint64_t* __restrict__ key, size_t n,
                                                   uint64_t* ctrl) {
    uint64_t mn = ~0ull, mx = 0ull, an = ~0ull, orr = 0ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        if (k == ~0ull) continue;
        mn = min(mn, k);
        mx = max(mx, k);
        an &= k;
        orr |= k;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        mn = min(mn, (uint64_t)__shfl_xor(mn, d, 64));
        mx = max(mx, (uint64_t)__shfl_xor(mx, d, 64));
        an &= (uint64_t)__shfl_xor(an, d, 64);
        orr |= (uint64_t)__shfl_xor(orr, d, 64);
    }
    if ((threadIdx.x & 63) == 0 && mn <= mx) {
        atomicMin(reinterpret_cast<unsigned long long*>(ctrl), (unsigned long long)mn);
        atomicMax(reinterpret_cast<unsigned long long*>(ctrl + 1), (unsigned long long)mx);
        atomicAnd(reinterpret_cast<unsigned long long*>(ctrl + 2), (unsigned long long)an);
        atomicOr(reinterpret_cast<unsigned long long*>(ctrl + 3), (unsigned long long)orr);
    }
}

// Right shift of (key - min) that keeps every drawn key below 0xffffffff:
// the low bits every drawn key shares can go (they are equal in all of
// them, so key - min is zero there); beyond that, precision is dropped and
// the runs of equal 32-bit keys need the full keys (exact is set to 0).
__device__ __forceinline__ int key_shift(const uint64_t* ctrl, bool& exact) {
    const uint64_t mn = ctrl[0], mx = ctrl[1];
    const uint64_t range = mx >= mn ? mx - mn : 0ull;
    const uint64_t diff = ctrl[2] ^ ctrl[3];      // bits that differ between drawn keys
    const int tz = diff ? __builtin_ctzll(diff) : 63;
    int s = 0;
    while ((range >> s) >= 0xffffffffull) ++s;
    exact = s <= tz;
    return exact ? min(tz, 63) : s;
}

// k32 = (key - min) >> s with the smallest s that keeps every drawn key
// below 0xffffffff; keys marked UINT64_MAX map to 0xffffffff.  Monotone, so
// sorting by k32 orders by key except among equal k32.
__global__ __launch_bounds__(256) void k_key32(const uint64_t* __restrict__ key, size_t n,
                                               const uint64_t* __restrict__ ctrl,
                                               uint32_t* __restrict__ k32, uint32_t* __restrict__ v) {
    const uint64_t mn = ctrl[0];
    bool exact;
    const int s = key_shift(ctrl, exact);
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        k32[i] = k == ~0ull ? 0xffffffffu : (uint32_t)((k - mn) >> s);
        v[i] = (uint32_t)i;
    }
}

// Each run of equal k32 is put in (key, value) order by the thread of its
// first element (insertion sort; runs arrive in value order, so a run of
// equal keys costs one comparison per element).  The neighbours' k32 come
// from the adjacent lanes, so the common case (no equal neighbour) is one
// coalesced load per element.
__global__ __launch_bounds__(256) void k_fix_runs(const uint32_t* __restrict__ k32,
                                                  uint32_t* __restrict__ v,
                                                  const uint64_t* __restrict__ key, size_t n,
                                                  const uint64_t* __restrict__ ctrl) {
    bool exact;
    (void)key_shift(ctrl, exact);
    if (exact) return;     // equal 32-bit keys are equal keys: index order holds
    const int lane = threadIdx.x & 63;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t base = (size_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const size_t i = base + threadIdx.x;
        const uint32_t ki = i < n ? k32[i] : 0xffffffffu;
        uint32_t prev = __shfl_up(ki, 1u, 64);
        uint32_t next = __shfl_down(ki, 1u, 64);
        if (lane == 0) prev = i > 0 && i <= n ? k32[i - 1] : ~ki;
        if (lane == 63) next = i + 1 < n ? k32[i + 1] : ~ki;
        if (i >= n || ki == 0xffffffffu || prev == ki || next != ki) continue;
        size_t j = i + 2;
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
    k_fix_runs<<<g, 256, 0, st>>>(k32_0, v0, key64, n, ctrl);
}

}  // namespace splotch_sort
