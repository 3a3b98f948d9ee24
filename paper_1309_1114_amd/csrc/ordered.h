// Kernels of the ordered render (emission and absorption set independently,
// Eq. 1 in its general form, Section "Splotch Overview").  With E != A the
// image depends on the order of the particles along each ray, so:
//
//   k_ord_project     per particle: the screen record (position, Gaussian,
//                     E and A per channel, tile box), the FP64 camera depth
//                     as a sortable key, and its tile box by index;
//   (sort)            particles by (depth, index): a stable radix sort of
//                     the depth bits with the indices as values;
//   k_ord_rank_counts tile boxes and entry counts in depth order, then an
//                     exclusive scan of the counts;
//   k_ord_pass_bounds the slice of the depth-ordered entry list a pass takes
//                     (fixed-size slices: a particle's entries may continue
//                     in the next pass) and the ranks that meet it;
//   k_ord_emit        (tile, particle) entries of the pass, in depth order;
//   (sort)            entries by tile, stable: each tile keeps depth order;
//   k_ord_items       each tile's entry list cut into work items of at most
//                     kOrdChunk entries (clustered data puts 15 times the
//                     mean on the densest tiles; one workgroup per tile would
//                     leave the chip waiting on them);
//   k_ord_composite   one workgroup per item, one thread per pixel (each wave
//                     an 8x8 quadrant, skipping records that cannot reach
//                     it), crosses the item's records front to back carrying
//                     the pixel's intensity I and transmittance T per
//                     channel: into the
//                     pixel state for a tile of one item, into a partial
//                     (I, T) from (0, 1) otherwise;
//   k_ord_merge       folds a tile's partials in depth order, I += T I_k,
//                     T *= T_k (compositing is associative).
//
// Front to back, a particle with column weight w adds T E w g(A w) to I and
// multiplies T by exp(-A w), g(t) = (1 - exp(-t))/t: the same sum as the
// far-to-near recursion I -> I exp(-A w) + E w g(A w).  Every pixel is owned
// by one thread, so the result is deterministic without atomics.  The terms
// are evaluated in FP32; the carried state I and T is FP64 (full rate on
// this chip), so thousands of factors exp(-A w) = 1 + expm1(-A w) compound
// without the per-factor float rounding.
#pragma once
#include "device.h"

namespace splotch_dev {

constexpr int kOrdT = 16;                    // tile side of the ordered render
constexpr int kOrdThreads = kOrdT * kOrdT;   // one thread per tile pixel
constexpr int kOrdQ = 8;                     // each wave owns one kOrdQ x kOrdQ quadrant
static_assert(kOrdQ * kOrdQ == 64 && kOrdT == 2 * kOrdQ, "four wave64 quadrants per tile");
constexpr int kOrdGrid = 2048;               // workgroups of the grid-stride kernels
constexpr uint32_t kOrdChunk = 8192;         // entries per composite work item

// Screen record of one particle, 48 bytes.  Tile box: tx = tx0 | tx1 << 16,
// ty = ty0 | ty1 << 16 (empty box tx0 > tx1 for particles that draw nothing).
struct __align__(16) OrdRec {
    float X, Y, k2, R2;
    float e[3];    // emission E per channel (peak column scale)
    float a[3];    // absorption A per channel
    uint32_t tx, ty;
};

struct OrdJob {
    Frame F;
    PartPtrs pp;
    int64_t n;
    const float* cmap;
    OrdRec* recs;        // [n] by particle index
    uint64_t* keys;      // [n] depth keys (UINT64_MAX: draws nothing)
    uint32_t* idx;       // [n] particle indices (sort values)
    uint64_t* box_p;     // [n] tile box tx | ty << 32 by particle index
    uint64_t* box_r;     // [n] the same boxes in depth-rank order
    uint64_t* cnt_r;     // [n+1] entries per depth rank (last 0)
    uint64_t* prefix;    // [n+1] exclusive prefix of cnt_r
    float* rgb;          // I (output, written by k_ord_finish)
    double* I;           // [3][H][W] intensity
    double* T;           // [3][H][W] transmittance
    float* S;            // [3][H][W] absorption depth sum A w
    float* logacc;       // optional output: S
    int32_t* ccount;     // optional output: centre counts
    unsigned long long* stats;
    uint32_t* tile_lo;   // [tiles+1] first entry of each tile (pass)
    uint64_t* item_n;    // [tiles+1] work items per tile (last 0)
    uint64_t* item_off;  // [tiles+1] exclusive prefix of item_n
    double* partI;       // [items][3][256] partial intensity of multi-item tiles
    double* partT;       // [items][3][256] partial transmittance
    float* partS;        // [items][3][256] partial absorption depth
};

__global__ void k_ord_init(OrdJob J) {
    const size_t plane = (size_t)J.F.W * J.F.H;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * plane; i += stride) {
        J.I[i] = 0.0;
        J.T[i] = 1.0;
        J.S[i] = 0.0f;
        if (J.ccount && i < plane) J.ccount[i] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < kStatWords) J.stats[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(256) void k_ord_project(OrdJob J) {
    const Frame& F = J.F;
    uint32_t active = 0;
    uint64_t entries = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < J.n; p += stride) {
        const RawPart q = load_part(J.pp, p, F.colmode);
        Rec r;
        int x0, x1, y0, y1;
        float amp, col[3], keep = 1.0f;
        double cz = 0.0;
        OrdRec o;
        uint64_t key = ~0ull;
        uint32_t ne = 0;
        o.tx = 1u;   // empty box
        o.ty = 1u;
        if (project_particle(F, J.cmap, q.x, q.y, q.z, q.h, q.inten, q.col, q.sp, r, x0, x1, y0,
                             y1, amp, col, &cz, &keep)) {
            float aamp = pick4(q.sp, F.a0, F.a1, F.a2, F.a3) * q.inten;
            if (F.col_norm) aamp *= kSqrtPi * q.h;
            aamp *= keep;
            o.X = r.X;
            o.Y = r.Y;
            o.k2 = r.k2;
            o.R2 = r.R2;
            o.e[0] = r.r;
            o.e[1] = r.g;
            o.e[2] = r.b;
            o.a[0] = aamp * col[0];
            o.a[1] = aamp * col[1];
            o.a[2] = aamp * col[2];
            // tiles of the pixels the in-disk test can pass (none: the
            // particle draws nothing and gets no entry)
            const float R = sqrtf(r.R2);
            float fx0, fx1, fy0, fy1;
            disk_span(r.X, R, 0.0f, (float)(F.W - 1), fx0, fx1);
            disk_span(r.Y, R, 0.0f, (float)(F.H - 1), fy0, fy1);
            if (fx0 <= fx1 && fy0 <= fy1) {
                const uint32_t tx0 = (uint32_t)fx0 / kOrdT, tx1 = (uint32_t)fx1 / kOrdT;
                const uint32_t ty0 = (uint32_t)fy0 / kOrdT, ty1 = (uint32_t)fy1 / kOrdT;
                o.tx = tx0 | (tx1 << 16);
                o.ty = ty0 | (ty1 << 16);
                ne = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
                key = (uint64_t)__double_as_longlong(cz);   // cz > 0: bits order as values
            }
            ++active;
            entries += ne;
            if (J.ccount && r.X >= 0.0f && r.X < (float)F.W && r.Y >= 0.0f && r.Y < (float)F.H)
                atomicAdd(J.ccount + (size_t)(int)r.Y * F.W + (int)r.X, 1);
        }
        J.recs[p] = o;
        J.keys[p] = key;
        J.box_p[p] = (uint64_t)o.tx | ((uint64_t)o.ty << 32);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        active += __shfl_xor(active, d, 64);
        entries += __shfl_xor(entries, d, 64);
    }
    if ((threadIdx.x & 63) == 0 && (active | entries)) {
        atomicAdd(J.stats + ST_ACTIVE, (unsigned long long)active);
        atomicAdd(J.stats + ST_ENTRIES, (unsigned long long)entries);
    }
}

// Tile entries of a box tx | ty << 32 (each tx0 | tx1 << 16, ty likewise;
// tx0 > tx1 for a particle that draws nothing).
__device__ __forceinline__ uint32_t box_entries(uint64_t b) {
    const uint32_t tx = (uint32_t)b, ty = (uint32_t)(b >> 32);
    const uint32_t tx0 = tx & 0xffffu, tx1 = tx >> 16, ty0 = ty & 0xffffu, ty1 = ty >> 16;
    return tx0 > tx1 || ty0 > ty1 ? 0u : (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
}

// In depth-rank order: box_r[r] = the box of the particle at rank r (one
// gather, so that k_ord_emit reads the boxes in order) and cnt_r[r] = its
// entries; cnt_r[n] = 0.
__global__ void k_ord_rank_counts(OrdJob J, const uint32_t* __restrict__ sorted_idx) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= J.n; r += stride) {
        if (r == J.n) {
            J.cnt_r[r] = 0ull;
            continue;
        }
        const uint64_t b = J.box_p[sorted_idx[r]];
        J.box_r[r] = b;
        J.cnt_r[r] = (uint64_t)box_entries(b);
    }
}

// Pass k of the ordered render takes the global entries [k cap, (k+1) cap)
// of the depth-ordered entry list (a particle's entries may continue in the
// next pass: every tile still receives its entries in depth order).  One
// thread: the pass's entry count m and the depth ranks [r0, r1) whose
// entries meet it; bounds[0..3] = E0, m, r0, r1.
__global__ void k_ord_pass_bounds(const uint64_t* __restrict__ prefix, int64_t n, uint64_t k,
                                  uint64_t cap, uint64_t* __restrict__ bounds) {
    const uint64_t total = prefix[n];
    const uint64_t e0 = min(total, k * cap), e1 = min(total, e0 + cap);
    // r0: the last rank with prefix[r] <= e0; r1: the first rank with
    // prefix[r] >= e1 (prefix is non-decreasing)
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (prefix[mid] <= e0) lo = mid; else hi = mid - 1;
    }
    const int64_t r0 = lo;
    lo = r0;
    hi = n;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (prefix[mid] >= e1) hi = mid; else lo = mid + 1;
    }
    bounds[0] = e0;
    bounds[1] = e1 - e0;
    bounds[2] = (uint64_t)r0;
    bounds[3] = (uint64_t)lo;
}

// Entries (tile, particle) of the pass described by bounds (see
// k_ord_pass_bounds): the ranks' entries inside the pass's slice, at their
// offsets in it, so the array is in depth order.  A particle's entries run
// over its tile box row by row.
__global__ void k_ord_emit(OrdJob J, const uint32_t* __restrict__ sorted_idx,
                           const uint64_t* __restrict__ bounds, uint32_t* __restrict__ ekey,
                           uint32_t* __restrict__ eval) {
    const uint64_t e0 = bounds[0], e1 = e0 + bounds[1];
    const int64_t r0 = (int64_t)bounds[2], r1 = (int64_t)bounds[3];
    const int tiles_x = (J.F.W + kOrdT - 1) / kOrdT;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = r0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < r1; r += stride) {
        const uint64_t p0 = J.prefix[r], p1 = J.prefix[r + 1];
        const uint64_t a = max(p0, e0), b = min(p1, e1);
        if (a >= b) continue;
        const uint32_t p = sorted_idx[r];
        const uint64_t bx = J.box_r[r];
        const uint32_t tx = (uint32_t)bx, ty = (uint32_t)(bx >> 32);
        const uint32_t tx0 = tx & 0xffffu, tx1 = tx >> 16, ty0 = ty & 0xffffu;
        const uint32_t bw = tx1 - tx0 + 1;
        for (uint64_t e = a; e < b; ++e) {
            const uint32_t i = (uint32_t)(e - p0);        // entry of the particle's box
            ekey[e - e0] = (ty0 + i / bw) * (uint32_t)tiles_x + tx0 + i % bw;
            eval[e - e0] = p;
        }
    }
}

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t m,
                                                    uint32_t v) {
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (a[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Per tile t: tile_lo[t] = first entry of tile t in the sorted pass
// (tile_lo[tiles] = m) and item_n[t] = ceil(entries / kOrdChunk);
// item_n[tiles] = 0 (the scan then leaves the item total there).
__global__ void k_ord_items(OrdJob J, const uint32_t* __restrict__ ekey,
                            const uint64_t* __restrict__ bounds, uint32_t n_tiles) {
    const uint32_t m = (uint32_t)bounds[1];
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t <= n_tiles;
         t += gridDim.x * blockDim.x) {
        if (t == n_tiles) {
            J.tile_lo[t] = m;
            J.item_n[t] = 0;
            continue;
        }
        const uint32_t lo = lower_bound_u32(ekey, m, t), hi = lower_bound_u32(ekey, m, t + 1);
        J.tile_lo[t] = lo;
        J.item_n[t] = (hi - lo + kOrdChunk - 1) / kOrdChunk;
    }
}

// Tile of work item b: the last t with item_off[t] <= b (item_off is the
// exclusive prefix of the item counts, n_tiles + 1 entries).
__device__ __forceinline__ uint32_t item_tile(const uint64_t* __restrict__ off, uint32_t n_tiles,
                                              uint64_t b) {
    uint32_t lo = 0, hi = n_tiles;   // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Pixel of thread tid in a tile: wave w owns the quadrant (w & 1, w >> 1),
// lanes run along its rows.
__device__ __forceinline__ void ord_pixel(uint32_t tile, int tiles_x, int tid, int& px, int& py) {
    const int w = tid >> 6, l = tid & 63;
    px = (int)(tile % (uint32_t)tiles_x) * kOrdT + (w & 1) * kOrdQ + (l & (kOrdQ - 1));
    py = (int)(tile / (uint32_t)tiles_x) * kOrdT + (w >> 1) * kOrdQ + (l >> 3);
}

// Bit w set if the disk of o may reach a pixel centre of quadrant w of the
// tile whose first pixel is (x0, y0), inside a W x H image.  A superset: the
// nearest point of the quadrant's centre box, with a margin above the
// rounding of the per-pixel test, which still decides.
__device__ __forceinline__ uint32_t ord_quadrants(const OrdRec& o, int x0, int y0, int W, int H) {
    uint32_t m = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const float bx0 = (float)(x0 + (w & 1) * kOrdQ) + 0.5f;
        const float by0 = (float)(y0 + (w >> 1) * kOrdQ) + 0.5f;
        const float bx1 = fminf(bx0 + (float)(kOrdQ - 1), (float)W - 0.5f);
        const float by1 = fminf(by0 + (float)(kOrdQ - 1), (float)H - 0.5f);
        const float dx = fmaxf(fmaxf(bx0 - o.X, o.X - bx1), 0.0f);
        const float dy = fmaxf(fmaxf(by0 - o.Y, o.Y - by1), 0.0f);
        if (bx0 <= bx1 && by0 <= by1 && dx * dx + dy * dy <= fmaf(o.R2, 1.0001f, 1e-4f))
            m |= 1u << w;
    }
    return m;
}

// h(t) = (1 - exp(-t))/t and g = 1 - exp(-t) = t h for t = a w.  Below
// |t| = 2^-7 the series of h to t^2 (remainder under |t|^3/24 = 2e-8), to
// t^4 below 1/8 (under t^5/720 = 4e-8), else through expm1.  Since w <= 1,
// max |a| over the channels bounds |t|, so a record (and a staged set of
// records) picks one evaluation for all its samples.
constexpr float kOrdShortSeries = 0.0078125f;

// One front-to-back step of a pixel's state: I += T E w h, T *= exp(-t)
// (= 1 - g), and the optional absorption depth S += t.
template <bool kDepth>
__device__ __forceinline__ void ord_add(double& I, double& T, float& S, float ewh, float g,
                                        float t) {
    I = fma(T, (double)ewh, I);
    T = fma(T, -(double)g, T);
    if (kDepth) S += t;
}

// Grid: an upper bound of the pass's work items, one workgroup of
// kOrdThreads each (those past the total exit).  ekey/eval: the pass's
// entries sorted by tile (depth order within a tile).  kDepth: also sum the
// absorption depth S (only the optional log_accum output reads it).
template <bool kDepth>
__global__ __launch_bounds__(kOrdThreads) void k_ord_composite(OrdJob J,
                                                               const uint32_t* __restrict__ eval,
                                                               uint32_t n_tiles) {
    __shared__ OrdRec st[kOrdThreads];
    __shared__ uint8_t quad[kOrdThreads];   // ord_quadrants of st[]
    const uint64_t b = blockIdx.x;
    if (b >= J.item_off[n_tiles]) return;
    const uint32_t tile = item_tile(J.item_off, n_tiles, b);
    const uint64_t k = b - J.item_off[tile];
    const bool single = J.item_n[tile] == 1;
    const uint32_t lo = J.tile_lo[tile] + (uint32_t)k * kOrdChunk;
    const uint32_t hi = min(J.tile_lo[tile + 1], lo + kOrdChunk);
    const Frame& F = J.F;
    const int tiles_x = (F.W + kOrdT - 1) / kOrdT;
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    int px, py;
    ord_pixel(tile, tiles_x, (int)threadIdx.x, px, py);
    const int x0 = (int)(tile % (uint32_t)tiles_x) * kOrdT, y0 = (int)(tile / (uint32_t)tiles_x) * kOrdT;
    const bool inside = px < F.W && py < F.H;
    const size_t plane = (size_t)F.W * F.H;
    const size_t pix = inside ? (size_t)py * F.W + px : 0;
    double I[3], T[3];
    float S[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        I[c] = single && inside ? J.I[c * plane + pix] : 0.0;
        T[c] = single && inside ? J.T[c * plane + pix] : 1.0;
        S[c] = single && inside ? J.S[c * plane + pix] : 0.0f;
    }
    // pixel centre, as in the tile splat
    const float cx = (float)px + 0.5f, cy = (float)py + 0.5f;
    // Each wave walks, in list order, only the staged records that may reach
    // its quadrant (a scalar mask per 64 records); the others cannot change
    // its pixels, so every pixel sees the same sequence of terms.
    for (uint32_t c0 = lo; c0 < hi; c0 += kOrdThreads) {
        const uint32_t e = c0 + threadIdx.x;
        uint32_t m = 0;
        if (e < hi) {
            const OrdRec r = J.recs[eval[e]];
            st[threadIdx.x] = r;
            m = ord_quadrants(r, x0, y0, F.W, F.H);
            // bit 7: some channel's |a| reaches 2^-7, so the record needs
            // more than the short series (see below)
            const float amax = fmaxf(fmaxf(fabsf(r.a[0]), fabsf(r.a[1])), fabsf(r.a[2]));
            if (!(amax < kOrdShortSeries)) m |= 0x80u;
        }
        quad[threadIdx.x] = (uint8_t)m;
        __syncthreads();
        for (int g64 = 0; g64 < kOrdThreads / 64; ++g64) {
            const uint32_t qm = quad[64 * g64 + lane];
            const bool mine = ((qm >> wave) & 1u) != 0u;
            uint64_t bal = __builtin_amdgcn_ballot_w64(mine);
            const bool longer = __builtin_amdgcn_ballot_w64(mine && (qm & 0x80u) != 0u) != 0ull;
            if (!longer) {
                // every record of the set takes the series of h to t^2
                while (bal) {
                    const float4* q = reinterpret_cast<const float4*>(
                        &st[64 * g64 + (int)__builtin_ctzll(bal)]);
                    bal &= bal - 1;
                    const float4 r0 = q[0];
                    const float dx = cx - r0.x, dy = cy - r0.y;
                    const float d2 = fmaf(dx, dx, dy * dy);
                    if (!inside || !(d2 <= r0.w)) continue;   // NaN-safe
                    const float4 r1 = q[1], r2 = q[2];
                    const float e3[3] = {r1.x, r1.y, r1.z};
                    const float a3[3] = {r1.w, r2.x, r2.y};
                    const float w = __builtin_amdgcn_exp2f(d2 * r0.z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float t = a3[c] * w;
                        const float h = fmaf(fmaf(t, 1.0f / 6.0f, -0.5f), t, 1.0f);
                        ord_add<kDepth>(I[c], T[c], S[c], e3[c] * w * h, t * h, t);
                    }
                }
                continue;
            }
            while (bal) {
                const float4* q =
                    reinterpret_cast<const float4*>(&st[64 * g64 + (int)__builtin_ctzll(bal)]);
                bal &= bal - 1;
                const float4 r0 = q[0];                 // X, Y, k2, R2
                const float dx = cx - r0.x, dy = cy - r0.y;
                const float d2 = fmaf(dx, dx, dy * dy);
                if (!inside || !(d2 <= r0.w)) continue;   // NaN-safe
                const float4 r1 = q[1], r2 = q[2];      // e[0..2], a[0] | a[1], a[2], tx, ty
                const float e3[3] = {r1.x, r1.y, r1.z};
                const float a3[3] = {r1.w, r2.x, r2.y};
                const float w = __builtin_amdgcn_exp2f(d2 * r0.z);
                // |t| <= max |a| (w <= 1), one value for the record, which
                // picks the evaluation of h for its three channels
                const float amax = __int_as_float(__builtin_amdgcn_readfirstlane(
                    __float_as_int(fmaxf(fmaxf(fabsf(a3[0]), fabsf(a3[1])), fabsf(a3[2])))));
                if (amax < kOrdShortSeries) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float t = a3[c] * w;
                        const float h = fmaf(fmaf(t, 1.0f / 6.0f, -0.5f), t, 1.0f);
                        ord_add<kDepth>(I[c], T[c], S[c], e3[c] * w * h, t * h, t);
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        const float t = a3[c] * w;
                        float h, g;
                        if (fabsf(t) < 0.125f) {
                            h = fmaf(fmaf(fmaf(fmaf(t, 1.0f / 120.0f, -1.0f / 24.0f), t,
                                               1.0f / 6.0f), t, -0.5f), t, 1.0f);
                            g = t * h;
                        } else {
                            g = -expm1f(-t);
                            h = g / t;
                        }
                        ord_add<kDepth>(I[c], T[c], S[c], e3[c] * w * h, g, t);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!inside) return;
    if (single) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            J.I[c * plane + pix] = I[c];
            J.T[c * plane + pix] = T[c];
            J.S[c * plane + pix] = S[c];
        }
    } else {
        const size_t base = (size_t)b * 3 * kOrdThreads + threadIdx.x;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            J.partI[base + c * kOrdThreads] = I[c];
            J.partT[base + c * kOrdThreads] = T[c];
            J.partS[base + c * kOrdThreads] = S[c];
        }
    }
}

// One workgroup per tile: fold the partials of a multi-item tile into the
// pixel state in depth order.
__global__ __launch_bounds__(kOrdThreads) void k_ord_merge(OrdJob J, uint32_t n_tiles) {
    const uint32_t tile = blockIdx.x;
    const uint64_t i0 = J.item_off[tile], i1 = i0 + J.item_n[tile];
    if (i1 - i0 < 2) return;
    const int tiles_x = (J.F.W + kOrdT - 1) / kOrdT;
    int px, py;
    ord_pixel(tile, tiles_x, (int)threadIdx.x, px, py);
    if (px >= J.F.W || py >= J.F.H) return;
    const size_t plane = (size_t)J.F.W * J.F.H;
    const size_t pix = (size_t)py * J.F.W + px;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double I = J.I[c * plane + pix], T = J.T[c * plane + pix];
        float S = J.S[c * plane + pix];
        for (uint64_t b = i0; b < i1; ++b) {
            const size_t q = (size_t)b * 3 * kOrdThreads + c * kOrdThreads + threadIdx.x;
            I = fma(T, J.partI[q], I);
            T *= J.partT[q];
            S += J.partS[q];
        }
        J.I[c * plane + pix] = I;
        J.T[c * plane + pix] = T;
        J.S[c * plane + pix] = S;
    }
}

// The image (rounded once to float) and the optional absorption depth, in
// the image layout.
__global__ void k_ord_finish(OrdJob J) {
    const size_t plane = (size_t)J.F.W * J.F.H;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += stride)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            J.rgb[3 * i + c] = (float)J.I[c * plane + i];
            if (J.logacc) J.logacc[3 * i + c] = J.S[c * plane + i];
        }
}

}  // namespace splotch_dev
