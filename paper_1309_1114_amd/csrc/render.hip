// Splotch rendering path for MI355X (gfx950): the C ABI of include/splotch.h.
//
// One render runs these kernels on the caller's stream, with no host sync:
//
//   k_clear     zero the optical-depth planes and the context counters
//   k_count     one thread per particle: roto-translation, projection and
//               palette colour (processing stage of Section "Splotch
//               Overview"; Eq. 7 for the screen radius), classification by
//               footprint, and a per-workgroup LDS histogram of tile keys
//   k_segsum / k_binscan / k_offsets
//               exclusive scan of the (key, workgroup) histogram: a
//               one-digit counting sort by tile key, the sort step of
//               Section "CUDA Implementation"
//   k_scatter   re-derives each record and writes it at its sorted slot
//   k_items     cuts each tile's list into work items of bounded length
//   k_large     cooperative pass for particles whose footprint covers many
//               tiles: workgroups own pixel blocks and gather, no atomics
//               inside the block (replaces the paper's CPU path for large
//               particles, Section "Large Particles")
//   k_splat     persistent workgroups pull tile items and splat the clipped
//               Gaussians (Eq. 2) into an LDS tile, then add it to the plane
//   k_resolve   I = 1 - exp(-L) per pixel and colour (Eq. 1 with E = A)
//
// Every kernel that draws a (particle, pixel) sample calls the same
// sample_weight() so the int64 fixed-point image is bit-identical whatever
// class, tile or work item a sample is drawn in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "splotch.h"

struct StageEvents {
    int stage;
    hipEvent_t start, stop;
};

struct splotch_ctx {
    int device = 0;
    int cu_count = 256;
    std::string err;
    unsigned long long* dstats = nullptr;  // device counters, kStatWords words
    splotch_stats last{};
    int last_accum = 0;
    bool timing = false;
    int timed_renders = 0;
    std::vector<StageEvents> events;       // pending stage timings
};

namespace {

constexpr int kCountThreads = 512;
constexpr int kSplatThreads = 256;
constexpr int kLargeThreads = 256;
constexpr int kSeg = 32;                 // workgroups per scan segment
constexpr int kMaxBins = 16400;          // LDS histogram capacity (tiles + 1)
constexpr int kLargeGroup = 128;         // pixel side of a large-pass group
constexpr int kLargeBlock = 32;          // pixel side of a large-pass block
constexpr int kStatWords = 8;
constexpr size_t kAlign = 256;
constexpr int64_t kMinChunk = 65536;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kSqrtPi = 1.77245385090551602730f;

enum { ST_ACTIVE = 0, ST_ENTRIES = 1, ST_LARGE = 2, ST_ITEMS = 3, ST_OVERFLOW = 4, ST_BADSLOT = 5 };

// Per-render constants (kernel argument).
struct Frame {
    float rx, ry, rz, ux, uy, uz, fx, fy, fz;  // camera basis
    float ex, ey, ez;                          // eye
    float focal, halfW, halfH, z_near, chi;
    float b0, b1, b2, b3;                      // brightness per species
    float s0, s1, s2, s3;                      // fixed sigma (px) per species, 0 = from h
    float smin, sinv;
    int slog, col_norm;
    int W, H;
    int T, tiles_x, tiles_y, n_tiles;
    int halo, max_clip;
    int ncmap;
    float qscale;                              // 2^frac_bits
    float inv_qscale;                          // 2^-frac_bits
    unsigned int* oflag;                       // int64 mode: set on overflow
};

// Screen record of one particle, 32 bytes.  meta bit 0: drawn in the
// bordered tile around its centre (otherwise clipped to its entry's tile).
struct __align__(16) Rec {
    float X, Y, k2, R2;
    float r, g, b;
    uint32_t meta;
};

__device__ __forceinline__ float pick4(int k, float a, float b, float c, float d) {
    return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
}

// Processing stage: camera transform, projection, screen sigma, palette
// colour and the conservative pixel box of the footprint (clipped to the
// image).  Returns false for particles that draw nothing.
__device__ __forceinline__ bool project_particle(const Frame& F, const float* __restrict__ cmap,
                                                 float x, float y, float z, float h, float inten,
                                                 float s, int sp, Rec& rec, int& x0, int& x1,
                                                 int& y0, int& y1) {
    const float dx = x - F.ex, dy = y - F.ey, dz = z - F.ez;
    const float cz = fmaf(F.fz, dz, fmaf(F.fy, dy, F.fx * dx));
    if (!(cz > F.z_near)) return false;
    const float cx = fmaf(F.rz, dz, fmaf(F.ry, dy, F.rx * dx));
    const float cy = fmaf(F.uz, dz, fmaf(F.uy, dy, F.ux * dx));
    const float icz = 1.0f / cz;
    const float X = fmaf(F.focal, cx * icz, F.halfW);
    const float Y = fmaf(-F.focal, cy * icz, F.halfH);
    const float fixs = pick4(sp, F.s0, F.s1, F.s2, F.s3);
    const float sig = fixs > 0.0f ? fixs : (F.focal * h) * icz;
    if (!(sig > 0.0f) || !(sig < 1.0e18f) || !(fabsf(X) < 1.0e30f) || !(fabsf(Y) < 1.0e30f))
        return false;
    const float R = F.chi * sig;
    float fx0 = floorf(X - R - 0.5f), fx1 = ceilf(X + R - 0.5f);
    float fy0 = floorf(Y - R - 0.5f), fy1 = ceilf(Y + R - 0.5f);
    fx0 = fmaxf(fx0, 0.0f);
    fy0 = fmaxf(fy0, 0.0f);
    fx1 = fminf(fx1, (float)(F.W - 1));
    fy1 = fminf(fy1, (float)(F.H - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
    x0 = (int)fx0;
    x1 = (int)fx1;
    y0 = (int)fy0;
    y1 = (int)fy1;
    // palette colour of the normalised scalar
    const float g = F.slog ? log10f(s) : s;
    float sn = (g - F.smin) * F.sinv;
    sn = sn > 0.0f ? fminf(sn, 1.0f) : 0.0f;
    const float u = sn * (float)(F.ncmap - 1);
    const int m = min((int)floorf(u), F.ncmap - 2);
    const float t = u - (float)m;
    const float omt = 1.0f - t;
    const float* c0 = cmap + 3 * m;
    float amp = pick4(sp, F.b0, F.b1, F.b2, F.b3) * inten;
    if (F.col_norm) amp *= kSqrtPi * h;
    rec.X = X;
    rec.Y = Y;
    rec.k2 = -kLog2e / (sig * sig);
    rec.R2 = R * R;
    rec.r = amp * fmaf(t, c0[3], omt * c0[0]);
    rec.g = amp * fmaf(t, c0[4], omt * c0[1]);
    rec.b = amp * fmaf(t, c0[5], omt * c0[2]);
    rec.meta = 0u;
    return true;
}

// Footprint classes.  kind 0: one entry in the bordered tile around the
// centre; kind 1: one entry per touched tile (drawn clipped to that tile);
// kind 2: one entry in the large list (key n_tiles).
struct Cls {
    int kind, bin, tx0, tx1, ty0, ty1;
};

__device__ __forceinline__ int classify(const Frame& F, float X, float Y, int x0, int x1, int y0,
                                        int y1, Cls& c) {
    const int T = F.T;
    if (X >= 0.0f && X < (float)F.W && Y >= 0.0f && Y < (float)F.H) {
        const int tx = (int)X / T, ty = (int)Y / T;
        const int ex0 = tx * T - F.halo, ex1 = tx * T + T - 1 + F.halo;
        const int ey0 = ty * T - F.halo, ey1 = ty * T + T - 1 + F.halo;
        if (x0 >= ex0 && x1 <= ex1 && y0 >= ey0 && y1 <= ey1) {
            c.kind = 0;
            c.bin = ty * F.tiles_x + tx;
            return 1;
        }
    }
    c.tx0 = x0 / T;
    c.tx1 = x1 / T;
    c.ty0 = y0 / T;
    c.ty1 = y1 / T;
    const int nt = (c.tx1 - c.tx0 + 1) * (c.ty1 - c.ty0 + 1);
    if (nt <= F.max_clip) {
        c.kind = 1;
        return nt;
    }
    c.kind = 2;
    c.bin = F.n_tiles;
    return 1;
}

// The weight exp(-d^2/sigma^2) of pixel (gx, gy) for record r, or false if
// the pixel centre is outside the clip circle d^2 <= R^2 (Eq. 2 clipped at
// chi*sigma).  Shared by every drawing kernel.
__device__ __forceinline__ bool sample_weight(float X, float Y, float k2, float R2, int gx, int gy,
                                              float& w) {
    const float dx = ((float)gx + 0.5f) - X;
    const float dy = ((float)gy + 0.5f) - Y;
    const float d2 = fmaf(dx, dx, dy * dy);
    if (!(d2 <= R2)) return false;
    w = __builtin_amdgcn_exp2f(d2 * k2);
    return true;
}

// Row form of sample_weight: dy2 = dy*dy precomputed for the row (the
// same operations in the same order).
__device__ __forceinline__ bool sample_weight_row(float X, float k2, float R2, float dy2, int gx,
                                                  float& w) {
    const float dx = ((float)gx + 0.5f) - X;
    const float d2 = fmaf(dx, dx, dy2);
    if (!(d2 <= R2)) return false;
    w = __builtin_amdgcn_exp2f(d2 * k2);
    return true;
}

template <typename Acc>
struct AccOps;

template <>
struct AccOps<float> {
    __device__ static __forceinline__ float term(float tau, const Frame&) { return tau; }
    __device__ static __forceinline__ void lds_add(float* p, float v) { atomicAdd(p, v); }
    __device__ static __forceinline__ void global_add(float* p, float v) { unsafeAtomicAdd(p, v); }
};

template <>
struct AccOps<long long> {
    // round(tau * 2^F); terms at or above 2^62 (or NaN) set the overflow
    // flag and count as zero
    __device__ static __forceinline__ long long term(float tau, const Frame& F) {
        const float v = tau * F.qscale;
        if (!(fabsf(v) < 4.0e18f)) {
            atomicOr(F.oflag, 1u);
            return 0;
        }
        return __float2ll_rn(v);
    }
    __device__ static __forceinline__ void lds_add(long long* p, long long v) {
        atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    }
    __device__ static __forceinline__ void global_add(long long* p, long long v) {
        atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    }
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// ---------------------------------------------------------------------------
// k_clear: zero n16 uint4 words of the plane and the counters.
// ---------------------------------------------------------------------------
__global__ void k_clear(uint4* __restrict__ p, size_t n16, unsigned long long* __restrict__ stats) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (stats && blockIdx.x == 0 && threadIdx.x < kStatWords) stats[threadIdx.x] = 0ull;
}

__global__ void k_zero_i32(int32_t* __restrict__ p, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0;
}

struct PartPtrs {
    const float *x, *y, *z, *h, *inten, *scalar;
    const uint8_t* species;
};

// ---------------------------------------------------------------------------
// k_count: per-workgroup histogram of keys over a contiguous particle range.
// hist is [P][NB] (workgroup-major).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kCountThreads) void k_count(Frame F, PartPtrs pp,
                                                         const float* __restrict__ cmap,
                                                         int64_t n, int64_t per_block,
                                                         uint32_t* __restrict__ hist, int NB,
                                                         unsigned long long* __restrict__ stats,
                                                         int32_t* __restrict__ center_count) {
    extern __shared__ uint32_t sh_hist[];
    for (int b = threadIdx.x; b < NB; b += blockDim.x) sh_hist[b] = 0u;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * per_block;
    const int64_t end = min(n, beg + per_block);
    uint32_t active = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const int sp = pp.species ? min((int)pp.species[i], 3) : 0;
        Rec r;
        int x0, x1, y0, y1;
        if (!project_particle(F, cmap, pp.x[i], pp.y[i], pp.z[i], pp.h[i], pp.inten[i],
                              pp.scalar[i], sp, r, x0, x1, y0, y1))
            continue;
        ++active;
        if (center_count && r.X >= 0.0f && r.X < (float)F.W && r.Y >= 0.0f && r.Y < (float)F.H)
            atomicAdd(center_count + (size_t)((int)r.Y) * F.W + (int)r.X, 1);
        Cls c;
        classify(F, r.X, r.Y, x0, x1, y0, y1, c);
        if (c.kind != 1) {
            atomicAdd(&sh_hist[c.bin], 1u);
        } else {
            for (int ty = c.ty0; ty <= c.ty1; ++ty)
                for (int tx = c.tx0; tx <= c.tx1; ++tx) atomicAdd(&sh_hist[ty * F.tiles_x + tx], 1u);
        }
    }
    // one counter update per wave
    uint32_t wsum = active;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) wsum += __shfl_xor(wsum, d, 64);
    if ((threadIdx.x & 63) == 0 && wsum) atomicAdd(stats + ST_ACTIVE, (unsigned long long)wsum);
    __syncthreads();
    uint32_t* out = hist + (size_t)blockIdx.x * NB;
    for (int b = threadIdx.x; b < NB; b += blockDim.x) out[b] = sh_hist[b];
}

// segsum[s][b] = sum over workgroups w of segment s of hist[w][b]
__global__ void k_segsum(const uint32_t* __restrict__ hist, uint32_t* __restrict__ segsum, int NB) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (b >= NB) return;
    uint32_t acc = 0;
    const uint32_t* p = hist + (size_t)s * kSeg * NB + b;
#pragma unroll 8
    for (int w = 0; w < kSeg; ++w) acc += p[(size_t)w * NB];
    segsum[(size_t)s * NB + b] = acc;
}

// Single workgroup: bin totals -> exclusive bin starts (bin_start[0..NB]),
// and segsum rewritten in place to each segment's starting offset.
__global__ __launch_bounds__(1024) void k_binscan(uint32_t* __restrict__ segsum,
                                                  uint32_t* __restrict__ bin_start, int NB,
                                                  int nseg) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (NB + 1023) / 1024;
    const int b0 = min(NB, t * per), b1 = min(NB, b0 + per);
    uint32_t local = 0;
    for (int b = b0; b < b1; ++b)
        for (int s = 0; s < nseg; ++s) local += segsum[(size_t)s * NB + b];
    part[t] = local;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - local;  // exclusive prefix
    for (int b = b0; b < b1; ++b) {
        bin_start[b] = run;
        for (int s = 0; s < nseg; ++s) {
            const uint32_t v = segsum[(size_t)s * NB + b];
            segsum[(size_t)s * NB + b] = run;
            run += v;
        }
    }
    if (t == 1023) bin_start[NB] = part[1023];
}

// hist[w][b] := offset of workgroup w's first record with key b.
__global__ void k_offsets(uint32_t* __restrict__ hist, const uint32_t* __restrict__ segoff, int NB) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (b >= NB) return;
    uint32_t run = segoff[(size_t)s * NB + b];
    uint32_t* p = hist + (size_t)s * kSeg * NB + b;
    for (int w = 0; w < kSeg; ++w) {
        const uint32_t v = p[(size_t)w * NB];
        p[(size_t)w * NB] = run;
        run += v;
    }
}

// k_scatter: same particle ranges as k_count; writes each record at its slot.
__global__ __launch_bounds__(kCountThreads) void k_scatter(Frame F, PartPtrs pp,
                                                           const float* __restrict__ cmap,
                                                           int64_t n, int64_t per_block,
                                                           const uint32_t* __restrict__ hist,
                                                           int NB, Rec* __restrict__ recs,
                                                           uint32_t cap,
                                                           unsigned long long* __restrict__ stats) {
    extern __shared__ uint32_t sh_cur[];
    const uint32_t* base = hist + (size_t)blockIdx.x * NB;
    for (int b = threadIdx.x; b < NB; b += blockDim.x) sh_cur[b] = base[b];
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * per_block;
    const int64_t end = min(n, beg + per_block);
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x) {
        const int sp = pp.species ? min((int)pp.species[i], 3) : 0;
        Rec r;
        int x0, x1, y0, y1;
        if (!project_particle(F, cmap, pp.x[i], pp.y[i], pp.z[i], pp.h[i], pp.inten[i],
                              pp.scalar[i], sp, r, x0, x1, y0, y1))
            continue;
        Cls c;
        classify(F, r.X, r.Y, x0, x1, y0, y1, c);
        const float4 lo = make_float4(r.X, r.Y, r.k2, r.R2);
        // k_count made the same decisions, so every slot lies inside its
        // key's range; the capacity test only guards against a mismatch
        if (c.kind != 1) {
            const uint32_t pos = atomicAdd(&sh_cur[c.bin], 1u);
            const float4 hi = make_float4(r.r, r.g, r.b, __uint_as_float(c.kind == 0 ? 1u : 0u));
            if (pos < cap) {
                float4* dst = reinterpret_cast<float4*>(recs + pos);
                dst[0] = lo;
                dst[1] = hi;
            } else {
                atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
            }
        } else {
            const float4 hi = make_float4(r.r, r.g, r.b, __uint_as_float(0u));
            for (int ty = c.ty0; ty <= c.ty1; ++ty)
                for (int tx = c.tx0; tx <= c.tx1; ++tx) {
                    const uint32_t pos = atomicAdd(&sh_cur[ty * F.tiles_x + tx], 1u);
                    if (pos < cap) {
                        float4* dst = reinterpret_cast<float4*>(recs + pos);
                        dst[0] = lo;
                        dst[1] = hi;
                    } else {
                        atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
                    }
                }
        }
    }
}

// k_items: split every tile's record range into items of at most `chunk`
// records.  items[k] = (tile, begin, end, 0).  Also resets the work counter.
__global__ __launch_bounds__(1024) void k_items(const uint32_t* __restrict__ bin_start, int n_tiles,
                                                int chunk, int4* __restrict__ items,
                                                uint32_t max_items, uint32_t cap,
                                                uint32_t* __restrict__ ctrl,
                                                unsigned long long* __restrict__ stats) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    const int t0 = min(n_tiles, t * per), t1 = min(n_tiles, t0 + per);
    uint32_t local = 0;
    for (int k = t0; k < t1; ++k) {
        const uint32_t cnt = bin_start[k + 1] - bin_start[k];
        local += (cnt + chunk - 1) / chunk;
    }
    part[t] = local;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t out = part[t] - local;
    const bool sane = bin_start[n_tiles + 1] <= cap && part[1023] <= max_items;
    if (sane) {
        for (int k = t0; k < t1; ++k) {
            const uint32_t b = bin_start[k], e = bin_start[k + 1];
            for (uint32_t s = b; s < e; s += chunk) {
                items[out++] = make_int4(k, (int)s, (int)min(e, s + (uint32_t)chunk), 0);
            }
        }
    }
    if (t == 1023) {
        // an inconsistent count (never expected) draws nothing rather than
        // reading past the record buffer
        const uint32_t n_items = sane ? part[1023] : 0u;
        if (!sane) atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
        ctrl[0] = n_items;
        ctrl[1] = 0u;  // work counter of k_splat
        const uint32_t n_entries = bin_start[n_tiles + 1];
        const uint32_t n_large = bin_start[n_tiles + 1] - bin_start[n_tiles];
        atomicAdd(stats + ST_ENTRIES, (unsigned long long)n_entries);
        atomicAdd(stats + ST_LARGE, (unsigned long long)n_large);
        atomicAdd(stats + ST_ITEMS, (unsigned long long)n_items);
    }
}

// ---------------------------------------------------------------------------
// k_large: cooperative pass over the large list.  Work item = (128x128 pixel
// group, chunk of 256 list entries).  The workgroup keeps the entries of its
// chunk that touch the group, then each thread gathers 4 pixels of every
// 32x32 block of the group over that short list, and adds its sums to the
// plane once per pixel.
// ---------------------------------------------------------------------------
template <typename Acc>
__global__ __launch_bounds__(kLargeThreads) void k_large(Frame F, const Rec* __restrict__ recs,
                                                         const uint32_t* __restrict__ bin_start,
                                                         uint32_t cap, Acc* __restrict__ Lg) {
    __shared__ float4 sA[kLargeThreads];
    __shared__ float4 sB[kLargeThreads];
    __shared__ int4 sR[kLargeThreads];
    __shared__ int s_cnt;
    const uint32_t le = min(bin_start[F.n_tiles + 1], cap);
    const uint32_t lb = min(bin_start[F.n_tiles], le);
    const uint32_t nl = le - lb;
    if (nl == 0) return;
    const int ngx = (F.W + kLargeGroup - 1) / kLargeGroup;
    const int ngy = (F.H + kLargeGroup - 1) / kLargeGroup;
    const uint64_t ngroups = (uint64_t)ngx * ngy;
    const uint64_t nchunks = (nl + kLargeThreads - 1) / kLargeThreads;
    const uint64_t nitems = ngroups * nchunks;
    const size_t plane = (size_t)F.W * F.H;
    const int tid = threadIdx.x;
    const int lx = tid & (kLargeBlock - 1);
    const int ly0 = tid >> 5;  // 0..7; rows ly0 + 8k
    for (uint64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int g = (int)(it % ngroups);
        const uint32_t ch = (uint32_t)(it / ngroups);
        const int gx0 = (g % ngx) * kLargeGroup, gy0 = (g / ngx) * kLargeGroup;
        const int gx1 = min(gx0 + kLargeGroup, F.W) - 1, gy1 = min(gy0 + kLargeGroup, F.H) - 1;
        if (tid == 0) s_cnt = 0;
        __syncthreads();
        const uint32_t e = lb + ch * kLargeThreads + tid;
        if (e < le) {
            const float4* rp = reinterpret_cast<const float4*>(recs + e);
            const float4 a = rp[0], b = rp[1];
            const float R = sqrtf(a.w);
            const float fx0 = fmaxf(floorf(a.x - R - 0.5f), (float)gx0);
            const float fx1 = fminf(ceilf(a.x + R - 0.5f), (float)gx1);
            const float fy0 = fmaxf(floorf(a.y - R - 0.5f), (float)gy0);
            const float fy1 = fminf(ceilf(a.y + R - 0.5f), (float)gy1);
            if (fx0 <= fx1 && fy0 <= fy1) {
                const int slot = atomicAdd(&s_cnt, 1);
                sA[slot] = a;
                sB[slot] = b;
                sR[slot] = make_int4((int)fx0, (int)fx1, (int)fy0, (int)fy1);
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        for (int by = gy0; by <= gy1; by += kLargeBlock) {
            for (int bx = gx0; bx <= gx1; bx += kLargeBlock) {
                const int bx1 = min(bx + kLargeBlock - 1, gx1), by1 = min(by + kLargeBlock - 1, gy1);
                Acc acc[4][3];
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[k][0] = acc[k][1] = acc[k][2] = (Acc)0;
                const int gx = bx + lx;
                for (int j = 0; j < cnt; ++j) {
                    const int4 rr = sR[j];
                    if (rr.x > bx1 || rr.y < bx || rr.z > by1 || rr.w < by) continue;  // uniform
                    const float4 a = sA[j];
                    const float4 b = sB[j];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int gy = by + ly0 + 8 * k;
                        float w;
                        if (gx <= bx1 && gy <= by1 && sample_weight(a.x, a.y, a.z, a.w, gx, gy, w)) {
                            acc[k][0] += AccOps<Acc>::term(b.x * w, F);
                            acc[k][1] += AccOps<Acc>::term(b.y * w, F);
                            acc[k][2] += AccOps<Acc>::term(b.z * w, F);
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int gy = by + ly0 + 8 * k;
                    if (gx <= bx1 && gy <= by1) {
                        const size_t p = (size_t)gy * F.W + gx;
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            if (acc[k][c] != (Acc)0) AccOps<Acc>::global_add(Lg + c * plane + p, acc[k][c]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// k_splat: persistent workgroups pull items (tile, record range).  The LDS
// accumulator covers the tile plus `halo` pixels on each side (records with
// meta bit 0 are drawn over their whole footprint there; others are clipped
// to the tile).  Each wave expands 64 records into a flat list of Q-pixel
// row segments: a wave prefix sum gives every record its first segment, a
// ballot of the record starts inside each 64-segment window gives every
// lane its owner record, and the lane draws its Q pixels with LDS atomics.
// ---------------------------------------------------------------------------
template <typename Acc, int Q>
__global__ __launch_bounds__(kSplatThreads) void k_splat(Frame F, const Rec* __restrict__ recs,
                                                         const int4* __restrict__ items,
                                                         uint32_t* __restrict__ ctrl,
                                                         Acc* __restrict__ Lg) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int E = F.T + 2 * F.halo;
    const int ES = E | 1;           // odd row stride spreads rows over banks
    const int PS = E * ES;          // plane stride
    Acc* acc = reinterpret_cast<Acc*>(smem);
    const size_t acc_bytes = ((size_t)3 * PS * sizeof(Acc) + 15) & ~(size_t)15;
    float4* stA = reinterpret_cast<float4*>(smem + acc_bytes);
    float4* stB = stA + kSplatThreads;
    uint2* stC = reinterpret_cast<uint2*>(stB + kSplatThreads);
    int* own = reinterpret_cast<int*>(stC + kSplatThreads);
    __shared__ int s_item;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    float4* wA = stA + wv * 64;
    float4* wB = stB + wv * 64;
    uint2* wC = stC + wv * 64;
    int* wO = own + wv * 64;
    const uint32_t n_items = ctrl[0];
    const size_t plane = (size_t)F.W * F.H;
    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(ctrl + 1, 1u);
        __syncthreads();
        const int it = s_item;
        if ((uint32_t)it >= n_items) break;
        const int4 item = items[it];
        const int tx = item.x % F.tiles_x, ty = item.x / F.tiles_x;
        const int ox = tx * F.T - F.halo, oy = ty * F.T - F.halo;  // accumulator origin
        // core (clipped entries) and bordered region (centre entries), in image
        const int cx0 = tx * F.T, cx1 = min(tx * F.T + F.T, F.W) - 1;
        const int cy0 = ty * F.T, cy1 = min(ty * F.T + F.T, F.H) - 1;
        const int hx0 = max(ox, 0), hx1 = min(ox + E, F.W) - 1;
        const int hy0 = max(oy, 0), hy1 = min(oy + E, F.H) - 1;
        for (int i = tid; i < 3 * PS; i += kSplatThreads) acc[i] = (Acc)0;
        __syncthreads();
        for (int base = item.y + wv * 64; base < item.z; base += kSplatThreads) {
            const int e = base + lane;
            float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
            uint32_t packed = 0, nq = 0;
            if (e < item.z) {
                const float4* rp = reinterpret_cast<const float4*>(recs + e);
                const float4 a = rp[0], b = rp[1];
                const bool centre = (__float_as_uint(b.w) & 1u) != 0u;
                const float R = sqrtf(a.w);
                const float fx0 = fmaxf(floorf(a.x - R - 0.5f), (float)(centre ? hx0 : cx0));
                const float fx1 = fminf(ceilf(a.x + R - 0.5f), (float)(centre ? hx1 : cx1));
                const float fy0 = fmaxf(floorf(a.y - R - 0.5f), (float)(centre ? hy0 : cy0));
                const float fy1 = fminf(ceilf(a.y + R - 0.5f), (float)(centre ? hy1 : cy1));
                if (fx0 <= fx1 && fy0 <= fy1) {
                    const int x0 = (int)fx0 - ox, x1 = (int)fx1 - ox;
                    const int y0 = (int)fy0 - oy, y1 = (int)fy1 - oy;
                    const uint32_t qpr = (uint32_t)(x1 - x0 + Q) / Q;
                    nq = qpr * (uint32_t)(y1 - y0 + 1);
                    packed = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)x1 << 16) | (qpr << 24);
                    A = a;
                    B = make_float4(b.x, b.y, b.z, 1.0f / (float)qpr);
                }
            }
            const uint32_t incl = wave_incl_scan(nq, lane);
            const uint32_t excl = incl - nq;
            const uint32_t total = __shfl(incl, 63, 64);
            wA[lane] = A;
            wB[lane] = B;
            wC[lane] = make_uint2(excl, packed);
            wave_lds_sync();
            int carry = 0;
            for (uint32_t wb = 0; wb < total; wb += 64) {
                // owner of segment wb + lane: the last record whose first
                // segment is at or before it.  Each record starting inside
                // the window marks its start position; a prefix max over the
                // positions (record indices grow with position) finds it.
                wO[lane] = -1;
                if (nq > 0 && excl >= wb && excl < wb + 64) wO[excl - wb] = lane;
                wave_lds_sync();
                int v = wO[lane];
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int t = __shfl_up(v, d, 64);
                    if (lane >= d) v = max(v, t);
                }
                const int o = (v >= 0 ? v : carry) & 63;
                carry = __shfl(o, 63, 64);
                const uint32_t s = wb + (uint32_t)lane;
                if (s < total) {
                    const float4 a = wA[o];
                    const float4 b = wB[o];
                    const uint2 c = wC[o];
                    const uint32_t q = s - c.x;
                    const int qpr = (int)(c.y >> 24);
                    const int row = (int)(((float)q + 0.5f) * b.w);
                    const int qc = (int)q - row * qpr;
                    const int ly = (int)((c.y >> 8) & 255u) + row;
                    const int lx0 = (int)(c.y & 255u) + qc * Q;
                    const int lx1 = (int)((c.y >> 16) & 255u);
                    const float dy = ((float)(ly + oy) + 0.5f) - a.y;
                    const float dy2 = dy * dy;
                    Acc* rowp = acc + ly * ES;
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        const int lx = lx0 + k;
                        float w;
                        if (lx <= lx1 && sample_weight_row(a.x, a.z, a.w, dy2, lx + ox, w)) {
                            AccOps<Acc>::lds_add(rowp + lx, AccOps<Acc>::term(b.x * w, F));
                            AccOps<Acc>::lds_add(rowp + PS + lx, AccOps<Acc>::term(b.y * w, F));
                            AccOps<Acc>::lds_add(rowp + 2 * PS + lx, AccOps<Acc>::term(b.z * w, F));
                        }
                    }
                }
                wave_lds_sync();
            }
        }
        __syncthreads();
        // add the local accumulator to the plane (pixels inside the image)
        for (int i = tid; i < E * E; i += kSplatThreads) {
            const int ly = i / E, lx = i - ly * E;
            const int gx = ox + lx, gy = oy + ly;
            if (gx < 0 || gy < 0 || gx >= F.W || gy >= F.H) continue;
            const size_t p = (size_t)gy * F.W + gx;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Acc v = acc[c * PS + ly * ES + lx];
                if (v != (Acc)0) AccOps<Acc>::global_add(Lg + c * plane + p, v);
            }
        }
        __syncthreads();
    }
}

// k_resolve: I = 1 - exp(-L) = -expm1(-L); optional L output.
template <typename Acc>
__global__ void k_resolve(const Acc* __restrict__ Lg, int W, int H, float inv_qscale,
                          float* __restrict__ rgb, float* __restrict__ logacc,
                          unsigned long long* __restrict__ stats) {
    const size_t plane = (size_t)W * H;
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= plane) return;
    bool bad = false;
    float L[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Acc v = Lg[c * plane + p];
        if constexpr (sizeof(Acc) == 8) {
            bad |= v < 0;
            L[c] = __ll2float_rn((long long)v) * inv_qscale;
        } else {
            L[c] = (float)v;
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) rgb[3 * p + c] = -expm1f(-L[c]);
    if (logacc) {
#pragma unroll
        for (int c = 0; c < 3; ++c) logacc[3 * p + c] = L[c];
    }
    if (bad) atomicOr(reinterpret_cast<unsigned int*>(stats + ST_OVERFLOW), 1u);
}

// ---------------------------------------------------------------------------
// Host side: validation, schedule, workspace layout, launches.
// ---------------------------------------------------------------------------
struct Knobs {
    int T, halo, max_clip, chunk;
};

struct Plan {
    Knobs k;
    int W, H, tiles_x, tiles_y, n_tiles, NB;
    int P, nseg;
    int accsize;
    int64_t n, chunk_n;
    size_t cap, max_items;
    size_t off_L, off_hist, off_seg, off_bin, off_items, off_ctrl, off_recs, total;
    size_t splat_lds;
};

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

splotch_status fail(splotch_ctx* ctx, splotch_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

size_t splat_lds_bytes(int T, int halo, int accsize) {
    const int E = T + 2 * halo;
    const int ES = E | 1;
    const size_t acc = ((size_t)3 * E * ES * accsize + 15) & ~(size_t)15;
    return acc + (size_t)kSplatThreads * (16 + 16 + 8) + (size_t)kSplatThreads * 4;
}

constexpr size_t kSplatLdsBudget = 96 * 1024;

// Choose the schedule knobs (explicit values are validated, zeros tuned).
splotch_status choose_knobs(splotch_ctx* ctx, const splotch_camera* cam, const splotch_params* p,
                            Knobs& k) {
    const int accsize = p->accum == SPLOTCH_ACCUM_INT64 ? 8 : 4;
    const int W = cam->width, H = cam->height;
    auto tiles = [&](int T) { return (int64_t)((W + T - 1) / T) * ((H + T - 1) / T); };
    if (p->tile != 0) {
        if (p->tile != 8 && p->tile != 16 && p->tile != 32 && p->tile != 64)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.tile must be 0, 8, 16, 32 or 64");
        k.T = p->tile;
    } else {
        k.T = 32;
        if (tiles(32) + 1 > kMaxBins) k.T = 64;
    }
    if (tiles(k.T) + 1 > kMaxBins)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "image has too many tiles for this tile size");
    if (p->halo >= 0) {
        if (p->halo > k.T) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.halo must be <= tile");
        k.halo = p->halo;
    } else {
        k.halo = std::min(8, k.T / 2);
    }
    while (k.halo > 0 && splat_lds_bytes(k.T, k.halo, accsize) > kSplatLdsBudget) k.halo /= 2;
    if (splat_lds_bytes(k.T, k.halo, accsize) > kSplatLdsBudget || k.T + 2 * k.halo > 255)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "tile/halo do not fit in LDS");
    if (p->max_clip_tiles != 0) {
        if (p->max_clip_tiles < 1 || p->max_clip_tiles > 64)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.max_clip_tiles must be 1..64");
        k.max_clip = p->max_clip_tiles;
    } else {
        k.max_clip = 4;
    }
    if (p->chunk != 0) {
        if (p->chunk < 32 || p->chunk > (1 << 20))
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.chunk must be 32..2^20");
        k.chunk = p->chunk;
    } else {
        k.chunk = 1024;
    }
    return SPLOTCH_OK;
}

void layout(Plan& pl, int64_t chunk_n) {
    pl.chunk_n = chunk_n;
    const int64_t per_particle = std::max(1, pl.k.max_clip);
    pl.cap = (size_t)std::max<int64_t>(chunk_n, 1) * per_particle;
    int P = (int)std::min<int64_t>(512, (std::max<int64_t>(chunk_n, 1) + 4095) / 4096);
    P = ((std::max(P, 1) + kSeg - 1) / kSeg) * kSeg;
    pl.P = P;
    pl.nseg = P / kSeg;
    pl.max_items = (size_t)pl.n_tiles + pl.cap / pl.k.chunk + 2;
    size_t off = 0;
    pl.off_L = off;
    off = align_up(off + (size_t)3 * pl.W * pl.H * pl.accsize);
    pl.off_hist = off;
    off = align_up(off + (size_t)pl.P * pl.NB * 4);
    pl.off_seg = off;
    off = align_up(off + (size_t)pl.nseg * pl.NB * 4);
    pl.off_bin = off;
    off = align_up(off + (size_t)(pl.NB + 1) * 4);
    pl.off_items = off;
    off = align_up(off + pl.max_items * 16);
    pl.off_ctrl = off;
    off = align_up(off + 64);
    pl.off_recs = off;
    off = align_up(off + pl.cap * sizeof(Rec));
    pl.total = off;
}

splotch_status validate(splotch_ctx* ctx, const splotch_particles* parts, const splotch_camera* cam,
                        const splotch_params* p, bool need_data) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!parts || !cam || !p) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "NULL argument");
    if (parts->n < 0) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "particles.n < 0");
    if (parts->n > (int64_t)1 << 40) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "particles.n too large");
    if (need_data && parts->n > 0 &&
        (!parts->x || !parts->y || !parts->z || !parts->h || !parts->intensity || !parts->scalar))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "NULL particle array");
    if (cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "camera width/height outside 1..32768");
    if (!(cam->fov_deg > 0.0f && cam->fov_deg < 180.0f))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "camera fov_deg outside (0,180)");
    if (!(cam->z_near > 0.0f) || !std::isfinite(cam->z_near))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "camera z_near must be > 0");
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(cam->eye[i]) || !std::isfinite(cam->target[i]) || !std::isfinite(cam->up[i]))
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "camera vectors must be finite");
    if (!(p->chi > 0.0f) || !std::isfinite(p->chi))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.chi must be > 0");
    if (p->accum != SPLOTCH_ACCUM_FP32 && p->accum != SPLOTCH_ACCUM_INT64)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.accum must be FP32 or INT64");
    if (p->accum == SPLOTCH_ACCUM_INT64 && (p->frac_bits < 8 || p->frac_bits > 56))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.frac_bits must be 8..56");
    if (!(p->scalar_max != p->scalar_min) || !std::isfinite(p->scalar_min) ||
        !std::isfinite(p->scalar_max))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.scalar_min/max must differ");
    for (int k = 0; k < SPLOTCH_MAX_SPECIES; ++k)
        if (!std::isfinite(p->brightness[k]) || !std::isfinite(p->fixed_sigma_frac[k]) ||
            p->fixed_sigma_frac[k] < 0.0f)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params brightness/fixed_sigma_frac invalid");
    return SPLOTCH_OK;
}

// Camera basis in double precision, rounded to float for the kernels.
bool make_frame(const splotch_camera* cam, const splotch_params* p, Frame& F) {
    double e[3], t[3], u[3];
    for (int i = 0; i < 3; ++i) {
        e[i] = cam->eye[i];
        t[i] = cam->target[i];
        u[i] = cam->up[i];
    }
    double f[3] = {t[0] - e[0], t[1] - e[1], t[2] - e[2]};
    const double nf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(nf > 0.0)) return false;
    for (double& v : f) v /= nf;
    double r[3] = {f[1] * u[2] - f[2] * u[1], f[2] * u[0] - f[0] * u[2], f[0] * u[1] - f[1] * u[0]};
    const double nr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(nr > 1e-12)) return false;
    for (double& v : r) v /= nr;
    const double up[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
    const double focal = 0.5 * cam->width / std::tan(0.5 * (double)cam->fov_deg * M_PI / 180.0);
    F.rx = (float)r[0]; F.ry = (float)r[1]; F.rz = (float)r[2];
    F.ux = (float)up[0]; F.uy = (float)up[1]; F.uz = (float)up[2];
    F.fx = (float)f[0]; F.fy = (float)f[1]; F.fz = (float)f[2];
    F.ex = cam->eye[0]; F.ey = cam->eye[1]; F.ez = cam->eye[2];
    F.focal = (float)focal;
    F.halfW = 0.5f * (float)cam->width;
    F.halfH = 0.5f * (float)cam->height;
    F.z_near = cam->z_near;
    F.chi = p->chi;
    F.b0 = p->brightness[0]; F.b1 = p->brightness[1]; F.b2 = p->brightness[2]; F.b3 = p->brightness[3];
    F.s0 = (float)((double)p->fixed_sigma_frac[0] * cam->width);
    F.s1 = (float)((double)p->fixed_sigma_frac[1] * cam->width);
    F.s2 = (float)((double)p->fixed_sigma_frac[2] * cam->width);
    F.s3 = (float)((double)p->fixed_sigma_frac[3] * cam->width);
    F.smin = p->scalar_min;
    F.sinv = (float)(1.0 / ((double)p->scalar_max - (double)p->scalar_min));
    F.slog = p->scalar_log10 ? 1 : 0;
    F.col_norm = p->col_norm ? 1 : 0;
    F.W = cam->width;
    F.H = cam->height;
    F.qscale = std::ldexp(1.0f, p->frac_bits);
    F.inv_qscale = std::ldexp(1.0f, -p->frac_bits);
    return true;
}

splotch_status make_plan(splotch_ctx* ctx, const splotch_particles* parts,
                         const splotch_camera* cam, const splotch_params* p, Plan& pl) {
    Knobs k{};
    splotch_status s = choose_knobs(ctx, cam, p, k);
    if (s != SPLOTCH_OK) return s;
    pl.k = k;
    pl.W = cam->width;
    pl.H = cam->height;
    pl.tiles_x = (pl.W + k.T - 1) / k.T;
    pl.tiles_y = (pl.H + k.T - 1) / k.T;
    pl.n_tiles = pl.tiles_x * pl.tiles_y;
    pl.NB = pl.n_tiles + 1;
    pl.accsize = p->accum == SPLOTCH_ACCUM_INT64 ? 8 : 4;
    pl.n = parts->n;
    pl.splat_lds = splat_lds_bytes(k.T, k.halo, pl.accsize);
    // records are indexed with 32-bit offsets
    const int64_t max_chunk = ((int64_t)1 << 31) / std::max(1, k.max_clip);
    layout(pl, std::min<int64_t>(std::max<int64_t>(parts->n, 1), max_chunk));
    return SPLOTCH_OK;
}

// Brackets a stage's launches with events on the stream when timing is on.
struct StageTimer {
    splotch_ctx* ctx;
    hipStream_t st;
    StageEvents cur{};
    bool on;
    StageTimer(splotch_ctx* c, hipStream_t s, int stage) : ctx(c), st(s), on(c->timing) {
        if (!on) return;
        cur.stage = stage;
        if (hipEventCreate(&cur.start) != hipSuccess || hipEventCreate(&cur.stop) != hipSuccess) {
            on = false;
            return;
        }
        (void)hipEventRecord(cur.start, st);
    }
    ~StageTimer() {
        if (!on) return;
        (void)hipEventRecord(cur.stop, st);
        ctx->events.push_back(cur);
    }
};

template <typename Acc>
splotch_status launch_all(splotch_ctx* ctx, const Plan& pl, const Frame& F0,
                          const splotch_particles* parts, const splotch_colormap* cmap,
                          const splotch_image* img, unsigned char* ws, hipStream_t st) {
    Frame F = F0;
    F.oflag = reinterpret_cast<unsigned int*>(ctx->dstats + ST_OVERFLOW);
    F.T = pl.k.T;
    F.tiles_x = pl.tiles_x;
    F.tiles_y = pl.tiles_y;
    F.n_tiles = pl.n_tiles;
    F.halo = pl.k.halo;
    F.max_clip = pl.k.max_clip;
    F.ncmap = cmap->n;
    Acc* Lg = reinterpret_cast<Acc*>(ws + pl.off_L);
    uint32_t* hist = reinterpret_cast<uint32_t*>(ws + pl.off_hist);
    uint32_t* seg = reinterpret_cast<uint32_t*>(ws + pl.off_seg);
    uint32_t* bin = reinterpret_cast<uint32_t*>(ws + pl.off_bin);
    int4* items = reinterpret_cast<int4*>(ws + pl.off_items);
    uint32_t* ctrl = reinterpret_cast<uint32_t*>(ws + pl.off_ctrl);
    Rec* recs = reinterpret_cast<Rec*>(ws + pl.off_recs);
    const size_t plane_bytes = (size_t)3 * pl.W * pl.H * sizeof(Acc);
    const size_t n16 = (plane_bytes + 15) / 16;  // region is padded to 256 bytes
    const int clear_blocks = (int)std::min<size_t>(4096, (n16 + 255) / 256 + 1);
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_CLEAR);
        k_clear<<<clear_blocks, 256, 0, st>>>(reinterpret_cast<uint4*>(Lg), n16, ctx->dstats);
        if (img->center_count) {
            const size_t np = (size_t)pl.W * pl.H;
            k_zero_i32<<<(unsigned)std::min<size_t>(4096, (np + 255) / 256), 256, 0, st>>>(
                img->center_count, np);
        }
    }
    PartPtrs pp{parts->x, parts->y, parts->z, parts->h, parts->intensity, parts->scalar,
                parts->species};
    const size_t hist_lds = (size_t)pl.NB * 4;
    int passes = 0;
    for (int64_t p0 = 0; p0 < pl.n; p0 += pl.chunk_n) {
        const int64_t cn = std::min(pl.chunk_n, pl.n - p0);
        PartPtrs q = pp;
        q.x += p0; q.y += p0; q.z += p0; q.h += p0; q.inten += p0; q.scalar += p0;
        if (q.species) q.species += p0;
        const int64_t per_block = (cn + pl.P - 1) / pl.P;
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_COUNT);
            k_count<<<pl.P, kCountThreads, hist_lds, st>>>(F, q, cmap->rgb, cn, per_block, hist,
                                                           pl.NB, ctx->dstats, img->center_count);
        }
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_SCAN);
            const dim3 sg((pl.NB + 255) / 256, pl.nseg);
            k_segsum<<<sg, 256, 0, st>>>(hist, seg, pl.NB);
            k_binscan<<<1, 1024, 0, st>>>(seg, bin, pl.NB, pl.nseg);
            k_offsets<<<sg, 256, 0, st>>>(hist, seg, pl.NB);
        }
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_SCATTER);
            k_scatter<<<pl.P, kCountThreads, hist_lds, st>>>(F, q, cmap->rgb, cn, per_block, hist,
                                                             pl.NB, recs, (uint32_t)pl.cap,
                                                             ctx->dstats);
        }
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_ITEMS);
            k_items<<<1, 1024, 0, st>>>(bin, pl.n_tiles, pl.k.chunk, items, (uint32_t)pl.max_items,
                                        (uint32_t)pl.cap, ctrl, ctx->dstats);
        }
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_LARGE);
            k_large<Acc><<<ctx->cu_count * 4, kLargeThreads, 0, st>>>(F, recs, bin,
                                                                       (uint32_t)pl.cap, Lg);
        }
        {
            StageTimer tm(ctx, st, SPLOTCH_STAGE_SPLAT);
            k_splat<Acc, 4><<<ctx->cu_count * 4, kSplatThreads, pl.splat_lds, st>>>(F, recs, items,
                                                                                    ctrl, Lg);
        }
        ++passes;
    }
    const size_t npix = (size_t)pl.W * pl.H;
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_RESOLVE);
        k_resolve<Acc><<<(unsigned)((npix + 255) / 256), 256, 0, st>>>(
            Lg, pl.W, pl.H, F.inv_qscale, img->rgb, img->log_accum, ctx->dstats);
    }
    if (ctx->timing) ctx->timed_renders++;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    ctx->last = splotch_stats{};
    ctx->last.n_input = pl.n;
    ctx->last.passes = passes;
    ctx->last.tile = pl.k.T;
    ctx->last.halo = pl.k.halo;
    ctx->last.max_clip_tiles = pl.k.max_clip;
    ctx->last.chunk = pl.k.chunk;
    return SPLOTCH_OK;
}

bool g_attrs_set[64] = {false};

void set_kernel_attrs(int device) {
    if (device < 0 || device >= 64 || g_attrs_set[device]) return;
    const int big = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_count),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scatter),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<float, 4>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<long long, 4>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipGetLastError();
    g_attrs_set[device] = true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* splotch_status_string(splotch_status s) {
    switch (s) {
        case SPLOTCH_OK: return "SPLOTCH_OK";
        case SPLOTCH_ERR_INVALID_ARG: return "SPLOTCH_ERR_INVALID_ARG";
        case SPLOTCH_ERR_WORKSPACE: return "SPLOTCH_ERR_WORKSPACE";
        case SPLOTCH_ERR_HIP: return "SPLOTCH_ERR_HIP";
        case SPLOTCH_ERR_OVERFLOW: return "SPLOTCH_ERR_OVERFLOW";
        case SPLOTCH_ERR_UNSUPPORTED: return "SPLOTCH_ERR_UNSUPPORTED";
        default: return "SPLOTCH_ERR_UNKNOWN";
    }
}

int32_t splotch_abi_version(void) { return SPLOTCH_ABI_VERSION; }

splotch_status splotch_default_params(splotch_params* p) {
    if (!p) return SPLOTCH_ERR_INVALID_ARG;
    std::memset(p, 0, sizeof(*p));
    p->chi = 3.0f;
    for (int k = 0; k < SPLOTCH_MAX_SPECIES; ++k) p->brightness[k] = 1.0f;
    p->scalar_min = 0.0f;
    p->scalar_max = 1.0f;
    p->accum = SPLOTCH_ACCUM_FP32;
    p->frac_bits = 40;
    p->tile = 0;
    p->halo = -1;
    p->max_clip_tiles = 0;
    p->chunk = 0;
    return SPLOTCH_OK;
}

splotch_status splotch_ctx_create(splotch_ctx** out, int32_t device) {
    if (!out) return SPLOTCH_ERR_INVALID_ARG;
    *out = nullptr;
    if (device < 0) return SPLOTCH_ERR_INVALID_ARG;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device >= count) {
        (void)hipGetLastError();
        return SPLOTCH_ERR_HIP;
    }
    if (hipSetDevice(device) != hipSuccess) return SPLOTCH_ERR_HIP;
    splotch_ctx* ctx = new splotch_ctx();
    ctx->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->cu_count = prop.multiProcessorCount;
    if (hipMalloc(reinterpret_cast<void**>(&ctx->dstats), kStatWords * sizeof(unsigned long long)) !=
        hipSuccess) {
        delete ctx;
        return SPLOTCH_ERR_HIP;
    }
    (void)hipMemset(ctx->dstats, 0, kStatWords * sizeof(unsigned long long));
    set_kernel_attrs(device);
    *out = ctx;
    return SPLOTCH_OK;
}

splotch_status splotch_ctx_destroy(splotch_ctx* ctx) {
    if (!ctx) return SPLOTCH_OK;
    for (StageEvents& e : ctx->events) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    if (ctx->dstats) {
        (void)hipSetDevice(ctx->device);
        (void)hipFree(ctx->dstats);
    }
    delete ctx;
    return SPLOTCH_OK;
}

const char* splotch_last_error(const splotch_ctx* ctx) {
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

splotch_status splotch_render_workspace_size(splotch_ctx* ctx, const splotch_particles* parts,
                                             const splotch_camera* cam,
                                             const splotch_params* params, size_t* bytes) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!bytes) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "bytes is NULL");
    splotch_status s = validate(ctx, parts, cam, params, false);
    if (s != SPLOTCH_OK) return s;
    Plan pl{};
    s = make_plan(ctx, parts, cam, params, pl);
    if (s != SPLOTCH_OK) return s;
    *bytes = pl.total;
    return SPLOTCH_OK;
}

splotch_status splotch_render(splotch_ctx* ctx, const splotch_particles* parts,
                              const splotch_camera* cam, const splotch_colormap* cmap,
                              const splotch_params* params, const splotch_image* img,
                              void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    splotch_status s = validate(ctx, parts, cam, params, true);
    if (s != SPLOTCH_OK) return s;
    if (!cmap || cmap->n < 2 || !cmap->rgb)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "colormap needs n >= 2 entries");
    if (!img || !img->rgb) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "image.rgb is NULL");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    Frame F{};
    if (!make_frame(cam, params, F))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "degenerate camera (eye == target or up parallel)");
    Plan pl{};
    s = make_plan(ctx, parts, cam, params, pl);
    if (s != SPLOTCH_OK) return s;
    if (workspace_bytes < pl.total) {
        // fit the largest particle chunk into the given workspace
        int64_t lo = kMinChunk, hi = pl.chunk_n;
        Plan probe = pl;
        layout(probe, lo);
        if (probe.total > workspace_bytes)
            return fail(ctx, SPLOTCH_ERR_WORKSPACE, "workspace smaller than the minimum for this image");
        while (hi - lo > 1024) {
            const int64_t mid = lo + (hi - lo) / 2;
            layout(probe, mid);
            if (probe.total <= workspace_bytes) lo = mid; else hi = mid;
        }
        layout(pl, lo);
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    ctx->last_accum = params->accum;
    if (params->accum == SPLOTCH_ACCUM_INT64)
        return launch_all<long long>(ctx, pl, F, parts, cmap, img, ws, st);
    return launch_all<float>(ctx, pl, F, parts, cmap, img, ws, st);
}

splotch_status splotch_set_timing(splotch_ctx* ctx, int32_t enable) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->timing = enable != 0;
    return SPLOTCH_OK;
}

splotch_status splotch_get_stage_times(splotch_ctx* ctx, void* hip_stream, float* ms,
                                       int32_t* renders) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!ms) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "ms is NULL");
    for (int i = 0; i < SPLOTCH_NUM_STAGES; ++i) ms[i] = 0.0f;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    if (hipStreamSynchronize(reinterpret_cast<hipStream_t>(hip_stream)) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "stream synchronize failed");
    splotch_status rc = SPLOTCH_OK;
    for (StageEvents& e : ctx->events) {
        float t = 0.0f;
        if (hipEventSynchronize(e.stop) == hipSuccess &&
            hipEventElapsedTime(&t, e.start, e.stop) == hipSuccess) {
            if (e.stage >= 0 && e.stage < SPLOTCH_NUM_STAGES) ms[e.stage] += t;
        } else {
            rc = fail(ctx, SPLOTCH_ERR_HIP, "event timing failed");
        }
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    ctx->events.clear();
    if (renders) *renders = ctx->timed_renders;
    ctx->timed_renders = 0;
    return rc;
}

splotch_status splotch_get_stats(splotch_ctx* ctx, void* hip_stream, splotch_stats* out) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!out) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "stats is NULL");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    unsigned long long h[kStatWords];
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipMemcpyAsync(h, ctx->dstats, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "reading counters failed");
    *out = ctx->last;
    out->n_active = (int64_t)h[ST_ACTIVE];
    out->n_entries = (int64_t)h[ST_ENTRIES];
    out->n_large = (int64_t)h[ST_LARGE];
    out->n_items = (int64_t)h[ST_ITEMS];
    out->overflow = h[ST_OVERFLOW] ? 1 : 0;
    if (h[ST_BADSLOT])
        return fail(ctx, SPLOTCH_ERR_HIP, "internal error: record counts of the two passes differ");
    if (out->overflow && ctx->last_accum == SPLOTCH_ACCUM_INT64)
        return fail(ctx, SPLOTCH_ERR_OVERFLOW, "int64 accumulator overflowed");
    return SPLOTCH_OK;
}

}  // extern "C"
