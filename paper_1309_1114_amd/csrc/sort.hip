// Sort and scan primitives of the ordered render (declared in sort.h).
//
// Radix pass over 8 bits of a 32-bit key, stable:
//   k_rs_hist     each workgroup counts the digits of its contiguous slice
//                 (digit-major table: count[digit][workgroup]);
//   (scan)        an exclusive scan of that table gives every workgroup the
//                 first output slot of each digit;
//   k_rs_scatter  each workgroup walks its slice in order, in tiles of 4096
//                 elements, each wave over its own run of 512 of them: a
//                 wave ranks an element among the tile's equal digits from
//                 eight ballots (its earlier lanes with that digit) and a
//                 wave-private count per digit; the waves' counts and a scan
//                 over digits place the tile by digit in LDS, which is then
//                 written so that each digit's elements go to consecutive
//                 slots, after the earlier tiles' (a running count per digit).
// Equal digits therefore keep their input order: LSD passes compose to a
// stable sort.
#include "sort.h"

#include <algorithm>

namespace splotch_sort {
namespace {

constexpr int kRT = 256;                 // threads of a counting workgroup
constexpr int kST = 512;                 // threads of a scatter workgroup
constexpr int kRounds = 8;               // elements per thread of a scatter tile
constexpr int kHistBatch = 8;            // keys per thread in flight while counting
constexpr int kTile = kST * kRounds;
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
    const __attribute__((address_space(1))) uint32_t* gkeys =
        (const __attribute__((address_space(1))) uint32_t*)keys;
    // kHistBatch keys per thread are loaded before any is counted, so each
    // wave keeps several loads in flight.  One LDS add per key; a wave whose
    // keys all share one digit (runs of equal keys) adds its count once
    // instead of 64 times to one word.
    for (size_t base = beg; base < end; base += (size_t)kHistBatch * kRT) {
        uint32_t d[kHistBatch];
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const size_t i = base + (size_t)u * kRT + tid;
            d[u] = i < end ? (gkeys[i] >> shift) & 255u : 0u;
        }
#pragma unroll
        for (int u = 0; u < kHistBatch; ++u) {
            const bool valid = base + (size_t)u * kRT + tid < end;
            const uint64_t vb = wave_ballot(valid);
            const uint32_t d0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)d[u]);
            if (wave_ballot(valid && d[u] == d0) == vb) {
                if (lane == 0 && vb) atomicAdd(&h[d0], (uint32_t)__popcll(vb));
            } else if (valid) {
                atomicAdd(&h[d[u]], 1u);
            }
        }
    }
    __syncthreads();
    hist[(size_t)tid * gridDim.x + blockIdx.x] = h[tid];
}

// Each workgroup walks its slice in tiles of kTile elements; wave w takes
// the tile's w-th run of 64 * kRounds consecutive elements, 64 per round.
// A wave ranks its elements by itself: per digit, the count of its earlier
// rounds (a wave-private LDS counter) plus the earlier lanes of the round
// with the same digit.  Once every wave is done, each digit's tile start
// (a scan over digits) and its count in earlier waves complete the rank, so
// ranks follow input order.  The tile is laid out in LDS by digit and
// written so that each digit's elements go to consecutive output slots,
// after the earlier tiles' (a running count per digit).  With LO, a third
// array (the low key bits a 64-bit sort dropped) moves with the pairs while
// carry[0] is nonzero.
template <bool LO>
__global__ __launch_bounds__(kST) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                    uint32_t* __restrict__ kout,
                                                    const uint32_t* __restrict__ vin,
                                                    uint32_t* __restrict__ vout,
                                                    const uint32_t* __restrict__ lin,
                                                    uint32_t* __restrict__ lout, size_t n_cap,
                                                    const uint64_t* __restrict__ n_dev, int shift,
                                                    const uint64_t* __restrict__ offs,
                                                    const uint32_t* __restrict__ carry) {
    constexpr int kW = kST / 64;                 // waves
    __shared__ uint32_t sk[kTile], sv[kTile];     // the tile, by digit
    __shared__ uint32_t sl[LO ? kTile : 1];
    __shared__ uint32_t run[kDigits];            // next output slot of each digit
    __shared__ uint32_t ts[kDigits];             // tile start of each digit
    __shared__ uint32_t wc[kW][kDigits];         // per wave and digit: count, then offset
    __shared__ uint32_t red[kDigits / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const bool dt = tid < kDigits;               // a thread of the per-digit steps
    const bool move_lo = LO && carry[0] != 0u;
    if (dt) run[tid] = (uint32_t)offs[(size_t)tid * gridDim.x + blockIdx.x];
    size_t beg, end;
    slice(eff_n(n_cap, n_dev), gridDim.x, blockIdx.x, beg, end);
    const uint64_t lt = (1ull << lane) - 1ull;
    const int w0 = wave * 64 * kRounds;          // the wave's run inside the tile
    for (size_t tb = beg; tb < end; tb += kTile) {
        const int tn = (int)min((size_t)kTile, end - tb);
        for (int i = tid; i < kW * kDigits; i += kST) (&wc[0][0])[i] = 0u;
        __syncthreads();
        uint32_t key[kRounds], val[kRounds], lo[LO ? kRounds : 1], rank[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const int j = w0 + r * 64 + lane;
            const bool valid = j < tn;
            key[r] = valid ? kin[tb + j] : 0u;
            val[r] = valid ? vin[tb + j] : 0u;
            if constexpr (LO) lo[r] = valid && move_lo ? lin[tb + j] : 0u;
        }
        uint32_t* cnt = wc[wave];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            const bool valid = w0 + r * 64 + lane < tn;
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint64_t peers = digit_peers(valid, d);
            const uint32_t before = valid ? cnt[d] : 0u;
            rank[r] = before + (uint32_t)__popcll(peers & lt);
            __builtin_amdgcn_wave_barrier();
            if (valid && (peers & lt) == 0ull) cnt[d] = before + (uint32_t)__popcll(peers);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // digit tid: counts of the waves -> offsets of each wave, tile count
        uint32_t c = 0u;
        if (dt) {
#pragma unroll
            for (int w = 0; w < kW; ++w) {
                const uint32_t x = wc[w][tid];
                wc[w][tid] = c;
                c += x;
            }
        }
        // exclusive scan of the tile counts over digits: each digit's start
        uint32_t incl = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t u = __shfl_up(incl, (unsigned)d, 64);
            if (lane >= d) incl += u;
        }
        if (dt && lane == 63) red[wave] = incl;
        __syncthreads();
        if (dt) {
            uint32_t before = 0u;
            for (int w = 0; w < wave; ++w) before += red[w];
            ts[tid] = before + incl - c;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            if (w0 + r * 64 + lane < tn) {
                const uint32_t d = (key[r] >> shift) & 255u;
                const uint32_t pos = ts[d] + cnt[d] + rank[r];
                sk[pos] = key[r];
                sv[pos] = val[r];
                if constexpr (LO) sl[pos] = lo[r];
            }
        }
        __syncthreads();
        for (int j = tid; j < tn; j += kST) {
            const uint32_t k = sk[j];
            const uint32_t d = (k >> shift) & 255u;
            const uint32_t dst = run[d] + ((uint32_t)j - ts[d]);
            kout[dst] = k;
            vout[dst] = sv[j];
            if constexpr (LO)
                if (move_lo) lout[dst] = sl[j];
        }
        __syncthreads();
        // next tile: advance each digit's output slot
        if (dt) run[tid] += c;
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

// ctrl: [0] min, [1] max, [2] AND, [3] OR of the drawn keys; [4] set when
// the 32-bit keys drop precision; [5] runs listed for ordering.
__global__ void k_key_range_init(uint64_t* ctrl) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctrl[0] = ~0ull;
        ctrl[1] = 0ull;
        ctrl[2] = ~0ull;
        ctrl[3] = 0ull;
        ctrl[5] = 0ull;
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
    // the workgroup's four waves combine in LDS: one set of atomics per
    // workgroup (per wave, the four words would see thousands of atomics)
    __shared__ uint64_t red[4][4];
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = mn;
        red[wave][1] = mx;
        red[wave][2] = an;
        red[wave][3] = orr;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) {
            mn = min(mn, red[w][0]);
            mx = max(mx, red[w][1]);
            an &= red[w][2];
            orr |= red[w][3];
        }
        if (mn <= mx) {
            atomicMin(reinterpret_cast<unsigned long long*>(ctrl), (unsigned long long)mn);
            atomicMax(reinterpret_cast<unsigned long long*>(ctrl + 1), (unsigned long long)mx);
            atomicAnd(reinterpret_cast<unsigned long long*>(ctrl + 2), (unsigned long long)an);
            atomicOr(reinterpret_cast<unsigned long long*>(ctrl + 3), (unsigned long long)orr);
        }
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
// sorting by k32 orders by key except among equal k32.  When that drops
// precision, lo gets the dropped bits ((key - min) mod 2^s; s <= 32 for keys
// below 2^63) and ctrl word 4 is set, so that the passes carry them along.
__global__ __launch_bounds__(256) void k_key32(const uint64_t* __restrict__ key, size_t n,
                                               uint64_t* __restrict__ ctrl,
                                               uint32_t* __restrict__ k32, uint32_t* __restrict__ v,
                                               uint32_t* __restrict__ lo) {
    const uint64_t mn = ctrl[0];
    bool exact;
    const int s = key_shift(ctrl, exact);
    if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[4] = exact ? 0ull : 1ull;
    const uint64_t mask = s >= 64 ? ~0ull : (1ull << s) - 1ull;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint64_t k = key[i];
        k32[i] = k == ~0ull ? 0xffffffffu : (uint32_t)((k - mn) >> s);
        v[i] = (uint32_t)i;
        if (!exact) lo[i] = k == ~0ull ? 0u : (uint32_t)((k - mn) & mask);
    }
}

// Runs of equal k32 arrive in value order with their lo bits alongside; a
// run is in (key, value) order unless some element's lo is below its
// predecessor's.  k_fix_mark finds those descents in one coalesced pass and
// lists the head of every run that has one (the thread of the run's first
// descent walks back to the head); k_fix_list then puts each listed run in
// (lo, value) order over its contiguous entries.  Runs of equal
// keys (the common case for depths computed from float positions) cost one
// comparison per element.  ctrl word 5 counts the listed runs.
__global__ __launch_bounds__(256) void k_fix_mark(const uint32_t* __restrict__ k32,
                                                  const uint32_t* __restrict__ lo, size_t n,
                                                  uint64_t* __restrict__ ctrl,
                                                  uint32_t* __restrict__ heads) {
    if (ctrl[4] == 0ull) return;   // exact mapping: equal k32 are equal keys
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t ki = k32[i];
        if (ki == 0xffffffffu || k32[i - 1] != ki || lo[i - 1] <= lo[i]) continue;
        // a descent: walk back to the run's head; an earlier descent on the
        // way means another thread lists this run (and ends the walk, so a
        // run costs each element one step however many descents it holds)
        size_t h = i - 1;
        bool first = true;
        while (h > 0 && k32[h - 1] == ki) {
            if (lo[h - 1] > lo[h]) {
                first = false;
                break;
            }
            --h;
        }
        if (first) {
            const unsigned long long slot =
                atomicAdd(reinterpret_cast<unsigned long long*>(ctrl + 5), 1ull);
            heads[slot] = (uint32_t)h;
        }
    }
}

// Insertion sort of (lo, v) over [a, b) by lo (equal lo keep their order).
__device__ __forceinline__ void insertion_by_lo(uint32_t* lo, uint32_t* v, size_t a, size_t b) {
    for (size_t c = a + 1; c < b; ++c) {
        const uint32_t lc = lo[c], vc = v[c];
        size_t d = c;
        while (d > a && lo[d - 1] > lc) {
            lo[d] = lo[d - 1];
            v[d] = v[d - 1];
            --d;
        }
        lo[d] = lc;
        v[d] = vc;
    }
}

// Each listed run [i, j) is put in (lo, v) order by one thread: insertion
// for short runs; for long ones (only inputs with many distinct depths
// closer than the 32-bit keys resolve) a bottom-up merge sort through tlo /
// tv (free scratch with the same indices), so the work stays O(m log m).
__global__ __launch_bounds__(256) void k_fix_list(const uint32_t* __restrict__ k32,
                                                  uint32_t* __restrict__ lo,
                                                  uint32_t* __restrict__ v,
                                                  uint32_t* __restrict__ tlo,
                                                  uint32_t* __restrict__ tv, size_t n,
                                                  const uint64_t* __restrict__ ctrl,
                                                  const uint32_t* __restrict__ heads) {
    constexpr size_t kShort = 16;
    const uint64_t m = ctrl[5];
    for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < m;
         q += (uint64_t)gridDim.x * blockDim.x) {
        const size_t i = heads[q];
        const uint32_t ki = k32[i];
        size_t j = i + 1;
        while (j < n && k32[j] == ki) ++j;
        for (size_t a = i; a < j; a += kShort) insertion_by_lo(lo, v, a, min(a + kShort, j));
        uint32_t *sl = lo, *sv = v, *dl = tlo, *dv = tv;
        for (size_t width = kShort; width < j - i; width *= 2) {
            for (size_t a = i; a < j; a += 2 * width) {
                const size_t mid = min(a + width, j), end = min(a + 2 * width, j);
                size_t x = a, y = mid, o = a;
                while (x < mid && y < end) {
                    if (sl[y] < sl[x]) {         // ties take the left run: stable
                        dl[o] = sl[y];
                        dv[o++] = sv[y++];
                    } else {
                        dl[o] = sl[x];
                        dv[o++] = sv[x++];
                    }
                }
                while (x < mid) {
                    dl[o] = sl[x];
                    dv[o++] = sv[x++];
                }
                while (y < end) {
                    dl[o] = sl[y];
                    dv[o++] = sv[y++];
                }
            }
            uint32_t* t = sl; sl = dl; dl = t;
            t = sv; sv = dv; dv = t;
        }
        if (sl != lo)
            for (size_t a = i; a < j; ++a) {
                lo[a] = sl[a];
                v[a] = sv[a];
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

// ceil(end_bit / 8) stable passes over (key, value[, lo]) pairs; returns
// the index (0 or 1) of the buffers that hold the result.
template <bool LO>
int radix_passes(void* temp, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1,
                 uint32_t* l0, uint32_t* l1, const uint32_t* carry, size_t n,
                 const uint64_t* n_dev, int end_bit, hipStream_t st) {
    const int passes = (end_bit + 7) / 8;
    if (n == 0) return passes & 1;
    uint64_t* hist = static_cast<uint64_t*>(temp);
    const int g = radix_blocks(n);
    uint32_t *kin = k0, *kout = k1, *vin = v0, *vout = v1, *lin = l0, *lout = l1;
    for (int p = 0; p < passes; ++p) {
        k_rs_hist<<<g, kRT, 0, st>>>(kin, n, n_dev, 8 * p, hist);
        exclusive_sum64(temp, hist, hist, (size_t)kDigits * g, st);
        k_rs_scatter<LO><<<g, kST, 0, st>>>(kin, kout, vin, vout, lin, lout, n, n_dev, 8 * p,
                                            hist, carry);
        std::swap(kin, kout);
        std::swap(vin, vout);
        std::swap(lin, lout);
    }
    return passes & 1;
}

int pairs32(void* temp, uint32_t* k0, uint32_t* k1, uint32_t* v0, uint32_t* v1, size_t n,
            const uint64_t* n_dev, int end_bit, hipStream_t st) {
    return radix_passes<false>(temp, k0, k1, v0, v1, nullptr, nullptr, nullptr, n, n_dev,
                               end_bit, st);
}

void sort_by_key64(void* temp, const uint64_t* key64, uint32_t* k32_0, uint32_t* k32_1,
                   uint32_t* v0, uint32_t* v1, uint32_t* lo0, uint32_t* lo1, size_t n,
                   hipStream_t st) {
    if (n == 0) return;
    uint64_t* ctrl = reinterpret_cast<uint64_t*>(static_cast<unsigned char*>(temp) + kHistBytes +
                                                 kPartBytes);
    const int g = grid_for(n, 4096, 4096);
    k_key_range_init<<<1, 64, 0, st>>>(ctrl);
    k_key_range<<<g, 256, 0, st>>>(key64, n, ctrl);
    k_key32<<<g, 256, 0, st>>>(key64, n, ctrl, k32_0, v0, lo0);
    // four passes: the result ends in buffers 0
    (void)radix_passes<true>(temp, k32_0, k32_1, v0, v1, lo0, lo1,
                             reinterpret_cast<const uint32_t*>(ctrl + 4), n, nullptr, 32, st);
    // k32_1 (free now) lists the runs to put in order; lo1 and v1 are the
    // merge scratch of long runs
    k_fix_mark<<<g, 256, 0, st>>>(k32_0, lo0, n, ctrl, k32_1);
    k_fix_list<<<g, 256, 0, st>>>(k32_0, lo0, v0, lo1, v1, n, ctrl, k32_1);
}

}  // namespace splotch_sort
