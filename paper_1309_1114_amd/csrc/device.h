// Device-side types and helpers shared by the render kernels (gfx950).
//
// Everything that decides whether a (particle, pixel) sample exists and what
// it is worth lives here, once, so that every kernel that draws a sample
// computes it with the same operations in the same order.  With that, the
// int64 fixed-point image is bit-identical whatever kernel, tile or work
// item a sample is drawn in.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace splotch_dev {

// Device memory through the global address space.  Pointers read from the
// job table are generic to the compiler, which then emits flat loads and
// stores; those also count against the LDS wait counter, so a wave waiting
// for an LDS result would wait for its outstanding stores to device memory
// as well.  These casts give global instructions instead.
#define SPLOTCH_GLOBAL __attribute__((address_space(1)))
#define SPLOTCH_LDS __attribute__((address_space(3)))
template <class T>
__device__ __forceinline__ SPLOTCH_GLOBAL T* gmem(T* p) {
    return (SPLOTCH_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const SPLOTCH_GLOBAL T* gmem(const T* p) {
    return (const SPLOTCH_GLOBAL T*)p;
}

// 16-byte loads and stores of device memory (through a builtin vector type:
// the float4 class has no assignment for address-space-qualified objects).
typedef float gvec4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 gload4(const float4* p) {
    const gvec4 v = *(const SPLOTCH_GLOBAL gvec4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void gstore4(float4* p, float4 v) {
    *(SPLOTCH_GLOBAL gvec4*)p = gvec4{v.x, v.y, v.z, v.w};
}

// Relaxed device-scope atomic adds on device memory (global instructions;
// the float add is the hardware one).
__device__ __forceinline__ float gatomic_add(float* p, float v) {
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long gatomic_add(unsigned long long* p,
                                                          unsigned long long v) {
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int gatomic_add(int* p, int v) {
    return __hip_atomic_fetch_add(gmem(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int kCountThreads = 512;
constexpr int kSplatThreads = 512;
#ifndef SPLOTCH_SPLAT_Q
#define SPLOTCH_SPLAT_Q 8
#endif
constexpr int kSplatQ = SPLOTCH_SPLAT_Q;  // pixels per row segment of the tile splat
// Records per tile work item, at most: the item's tile is summed in 64-bit
// LDS words from terms below 2^50 in magnitude (one per record and pixel),
// so 8191 of them stay below 2^63.
constexpr int kMaxChunk = 8191;
// LDS staging of the tile splat per thread (record 16 + 16 + 8, owner mark
// 4) plus the work-queue slot
constexpr int kSplatStageBytes = 16 + 16 + 8 + 4;
constexpr int kSplatStageExtra = 16;
constexpr int kLoadBatch = 4;       // particles a thread loads at once (count, scatter)
constexpr int kLdsPalette = 1024;  // largest palette the scatter pass stages in LDS
constexpr int kLdsBytesPerCU = 160 * 1024;  // LDS of one gfx950 CU
constexpr int kMaxCountBlocks = 768;  // count/scatter workgroups per job: 3 per CU of 512
constexpr int kLargeThreads = 256;
constexpr int kSeg = 32;            // workgroups per scan segment
constexpr int kMaxBins = 16400;     // LDS key-histogram capacity (tiles + 1)
constexpr int kLargeGroup = 128;    // smallest pixel side of a large-pass group
constexpr int kMaxLargeGroups = 4096; // groups per frame (the side doubles until they fit)
constexpr int kLgBlocks = 256;      // workgroups per job binning the large list
constexpr int kLgTargetItems = 4096; // large-pass items aimed at per job (entries per item 16..256)
constexpr int kLargeBlock = 32;     // pixel side of a large-pass block
constexpr int kStatWords = 16;
constexpr int kCtrlWords = 16;
constexpr float kLog2e = 1.44269504088896340736f;
constexpr float kSqrtPi = 1.77245385090551602730f;

enum { ST_ACTIVE = 0, ST_ENTRIES = 1, ST_LARGE = 2, ST_ITEMS = 3, ST_OVERFLOW = 4, ST_BADSLOT = 5,
       ST_RHIST = 6,      // 5 words: active particles by screen radius chi*sigma (px):
                          // <= 2, (2, 4], (4, 8], (8, 16], > 16
       ST_RSUM = 11,      // sum of the radii of active particles (a double)
       ST_SAMPLES = 12 }; // (particle, pixel) samples drawn, when counted
// control words of a batch (device)
enum { CT_NITEMS = 0, CT_WORK = 1, CT_NLARGE_ITEMS = 2 };

// Per-job constants: camera, parameters and tile geometry.
struct Frame {
    double rx, ry, rz, ux, uy, uz, fx, fy, fz; // camera basis (right, up, forward)
    double ex, ey, ez;                         // eye
    double focal;                              // pixels per unit of tan(angle)
    float halfW, halfH, z_near, chi;
    float b0, b1, b2, b3;                      // brightness per species
    float a0, a1, a2, a3;                      // absorption per species (ordered transfer)
    float s0, s1, s2, s3;                      // fixed sigma (px) per species, 0 = from h
    float smin, sinv;                          // scalar normalisation
    int slog, col_norm;
    int colmode, pad0;                         // 1: colour from the vector (vx, vy, vz)
    float pf2;                                 // prefilter sigma squared (px^2), 0 = none
    int pad1;
    int W, H;
    int T, tiles_x, tiles_y, n_tiles;
    int Tshift;                                // log2(T): tile sides are powers of two
    int halo, max_clip;
    int ncmap;
    float qscale;                              // 2^frac_bits
    float inv_qscale;                          // 2^-frac_bits
    float tau_lim;                             // 2^50 / qscale: largest |tau| of a fixed-point record
    unsigned int* oflag;                       // int64 mode: overflow flag
};

// Screen record of one particle, 32 bytes.  meta bit 0: drawn over its whole
// footprint in the bordered tile around its centre; otherwise clipped to the
// tile of its entry.
struct __align__(16) Rec {
    float X, Y, k2, R2;
    float r, g, b;
    uint32_t meta;
};

struct PartPtrs {
    const float *x, *y, *z, *h, *inten, *scalar;
    const uint8_t* species;
    const float *vx, *vy, *vz;                 // vector colour mode only
};

// One job of a batch as the kernels see it (device memory, written by the
// host before the launches; large_item0 is filled in by k_items).
struct JobDev {
    Frame F;
    PartPtrs pp;
    int64_t n;            // particles of this pass
    int64_t per_block;    // particles per count/scatter workgroup
    const float* cmap;
    void* L;              // optical-depth planes [3][H][W] (float or int64)
    uint32_t* hist;       // [P][NB] key counts, then slot offsets
    uint32_t* seg;        // [nseg][NB] segment sums, then segment offsets
    uint32_t* bin;        // [NB+1] key starts
    Rec* recs;            // record slots
    float* rgb;           // outputs
    float* logacc;
    int32_t* ccount;
    uint32_t cap;         // record capacity
    uint32_t max_items;   // tile work items this job may produce
    int NB, P, nseg;
    uint32_t item0;       // first slot of this job in the item array
    uint32_t large_item0; // first large-pass item of this job (set on device)
    uint32_t n_large_items;
    int chunk;            // records per tile work item
    int lg_fallback;      // set on device: 1 if the group index lists overflowed
    // large-pass binning: the large list is indexed per pixel group
    uint32_t* lg_cnt;     // [NG] counts, then write cursors
    uint32_t* lg_start;   // [NG+1] first index of each group's list
    uint32_t* lg_chunk;   // [NG+1] first large-pass item of each group
    uint32_t* lg_idx;     // [cap_idx] record offsets into the large list
    uint32_t cap_idx;
    int NG, ngx, lg_side; // groups, groups per row, group side in pixels
    int lg_per_item;      // set on device: index entries per large-pass item
    int pad2;
    // optional region mask: only tiles and pixels of marked regions are drawn
    const uint8_t* rmask; // [ceil(H / 2^rshift)][rgx] bytes, nullptr: every pixel
    int rshift, rgx;      // log2 of the region side, regions per row
    uint8_t* tlive;       // [n_tiles] with a mask: bit 0 core, bit 1 bordered tile marked
};

// Whether the region holding pixel (px, py) is marked (true without a mask).
__device__ __forceinline__ bool region_on(const JobDev& J, int px, int py) {
    return !J.rmask || J.rmask[(size_t)(py >> J.rshift) * J.rgx + (px >> J.rshift)] != 0;
}

// Whether any marked region meets the pixel rectangle [x0, x1] x [y0, y1].
__device__ __forceinline__ bool rect_on(const JobDev& J, int x0, int x1, int y0, int y1) {
    if (!J.rmask) return true;
    for (int ry = y0 >> J.rshift; ry <= (y1 >> J.rshift); ++ry)
        for (int rx = x0 >> J.rshift; rx <= (x1 >> J.rshift); ++rx)
            if (J.rmask[(size_t)ry * J.rgx + rx]) return true;
    return false;
}

// Whether tile t, widened by `border` pixels on each side, meets a marked
// region (always true without a mask).  Records drawn clipped to a tile need
// its core (border 0); records drawn over their whole footprint in the
// bordered tile around their centre reach `halo` pixels further.
__device__ __forceinline__ bool tile_on(const JobDev& J, int t, int border) {
    if (!J.rmask) return true;
    const int T = J.F.T, tx = t % J.F.tiles_x, ty = t / J.F.tiles_x;
    return rect_on(J, max(tx * T - border, 0), min(tx * T + T + border, J.F.W) - 1,
                   max(ty * T - border, 0), min(ty * T + T + border, J.F.H) - 1);
}

// The same from the tile flags (staged in LDS by the counting and scattering
// passes): `bordered` asks for the tile widened by the halo.  live ==
// nullptr: no mask.
__device__ __forceinline__ bool tile_live(const SPLOTCH_LDS uint8_t* live, int t, bool bordered) {
    return !live || ((live[t] >> (bordered ? 1 : 0)) & 1u) != 0u;
}

// Raw inputs of one particle (SoA loads).  col: the scalar in the palette
// mode (col[1], col[2] unused), the vector (vx, vy, vz) in the vector mode.
struct RawPart {
    float x, y, z, h, inten;
    float col[3];
    int sp;
};

__device__ __forceinline__ RawPart load_part(const PartPtrs& pp, int64_t i, int colmode) {
    RawPart q;
    q.x = gmem(pp.x)[i];
    q.y = gmem(pp.y)[i];
    q.z = gmem(pp.z)[i];
    q.h = gmem(pp.h)[i];
    q.inten = gmem(pp.inten)[i];
    if (colmode) {
        q.col[0] = gmem(pp.vx)[i];
        q.col[1] = gmem(pp.vy)[i];
        q.col[2] = gmem(pp.vz)[i];
    } else {
        q.col[0] = gmem(pp.scalar)[i];
        q.col[1] = q.col[2] = 0.0f;
    }
    q.sp = pp.species ? min((int)gmem(pp.species)[i], 3) : 0;
    return q;
}

// Min/max normalisation of a colour input, clamped to [0, 1] (NaN -> 0).
__device__ __forceinline__ float norm01(const Frame& F, float g) {
    const float sn = (g - F.smin) * F.sinv;
    return sn > 0.0f ? fminf(sn, 1.0f) : 0.0f;
}

__device__ __forceinline__ float pick4(int k, float a, float b, float c, float d) {
    return k == 0 ? a : (k == 1 ? b : (k == 2 ? c : d));
}

// Processing stage of one particle: camera transform (roto-translation),
// perspective projection of the position and of the smoothing length,
// colour (palette look-up of the scalar, or the normalised vector), and the
// conservative pixel box of its footprint, clipped to the image.  Returns
// false for particles that draw nothing.
template <class PalPtr>
__device__ __forceinline__ bool project_particle(const Frame& F, PalPtr cmap,
                                                 float x, float y, float z, float h, float inten,
                                                 const float* col, int sp, Rec& rec, int& x0,
                                                 int& x1, int& y0, int& y1, float& amp_out,
                                                 float* colour_out = nullptr,
                                                 double* depth_out = nullptr,
                                                 float* keep_out = nullptr) {
    // transform and projection in double, each result rounded once to
    // float: the screen position then carries half an ulp of error (3e-5 px
    // at 1000 px), which matters where thousands of narrow Gaussians overlap
    const double dx = (double)x - F.ex, dy = (double)y - F.ey, dz = (double)z - F.ez;
    const double cz = fma(F.fz, dz, fma(F.fy, dy, F.fx * dx));
    if (!(cz > (double)F.z_near)) return false;
    const double cx = fma(F.rz, dz, fma(F.ry, dy, F.rx * dx));
    const double cy = fma(F.uz, dz, fma(F.uy, dy, F.ux * dx));
    // 1/cz: hardware reciprocal refined by one Newton step (relative error
    // far below the float rounding that follows)
    const double r0 = __builtin_amdgcn_rcp(cz);
    const double icz = fma(r0, fma(-cz, r0, 1.0), r0);
    const double s_over_z = F.focal * icz;
    const float X = (float)fma(s_over_z, cx, (double)F.halfW);
    const float Y = (float)fma(-s_over_z, cy, (double)F.halfH);
    const float fixs = pick4(sp, F.s0, F.s1, F.s2, F.s3);
    float sig = fixs > 0.0f ? fixs : (float)(s_over_z * (double)h);
    if (!(sig > 0.0f) || !(sig < 1.0e18f) || !(fabsf(X) < 1.0e30f) || !(fabsf(Y) < 1.0e30f))
        return false;
    // screen-plane prefilter: the Gaussian convolved with the normalised
    // Gaussian of sigma s is the Gaussian of sigma' = sqrt(sigma^2 + s^2)
    // whose peak is scaled by sigma^2 / sigma'^2 (same integral)
    float keep = 1.0f;
    if (F.pf2 > 0.0f) {
        const float s2 = sig * sig;
        const float t2 = s2 + F.pf2;
        keep = s2 / t2;
        sig = sqrtf(t2);
    }
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
    float amp = pick4(sp, F.b0, F.b1, F.b2, F.b3) * inten;
    if (F.col_norm) amp *= kSqrtPi * h;
    amp *= keep;
    amp_out = amp;
    if (keep_out) *keep_out = keep;
    rec.X = X;
    rec.Y = Y;
    rec.k2 = -kLog2e / fmaxf(sig * sig, 1.0e-30f);   // finite: w = 1 at d = 0
    rec.R2 = R * R;
    float cr, cg, cb;
    if (F.colmode) {
        // colour by vector: each channel its own normalised component
        cr = norm01(F, col[0]);
        cg = norm01(F, col[1]);
        cb = norm01(F, col[2]);
    } else {
        // palette colour of the normalised scalar (linear between entries)
        const float sn = norm01(F, F.slog ? log10f(col[0]) : col[0]);
        const float u = sn * (float)(F.ncmap - 1);
        const int m = min((int)floorf(u), F.ncmap - 2);
        const float t = u - (float)m;
        const float omt = 1.0f - t;
        const auto c0 = cmap + 3 * m;
        cr = fmaf(t, c0[3], omt * c0[0]);
        cg = fmaf(t, c0[4], omt * c0[1]);
        cb = fmaf(t, c0[5], omt * c0[2]);
    }
    rec.r = amp * cr;
    rec.g = amp * cg;
    rec.b = amp * cb;
    rec.meta = 0u;
    if (colour_out) {
        colour_out[0] = cr;
        colour_out[1] = cg;
        colour_out[2] = cb;
    }
    if (depth_out) *depth_out = cz;
    return true;
}

// Footprint classes.  kind 0: one entry in the bordered tile around the
// centre; kind 1: one entry per touched tile (drawn clipped to that tile);
// kind 2: one entry in the large list (key n_tiles).
struct Cls {
    int kind, bin, tx0, tx1, ty0, ty1;
};

// Pixels i in [f0, f1] (as floats) whose centre i + 1/2 can pass the
// in-disk test of sample_weight along one axis, clipped to [lo, hi]: the
// pixels with |i + 1/2 - X| <= R, R = sqrtf(R2), widened by a margin.  A
// pixel that passes the test has |i + 1/2 - X| <= R (1 + 2^-21) (one
// rounding each in dx, d2 and R); the margin covers that and the three
// roundings here, each below 2^-24 (|X| + R + 1).  The range is empty
// (f0 > f1) when no pixel can pass.
__device__ __forceinline__ void disk_span(float X, float R, float lo, float hi, float& f0,
                                          float& f1) {
    const float m = fmaf(1.0e-6f, fabsf(X) + R, 1.0e-3f);
    f0 = fmaxf(ceilf(X - R - 0.5f - m), lo);
    f1 = fminf(floorf(X + R - 0.5f + m), hi);
}

__device__ __forceinline__ void classify(const Frame& F, float X, float Y, int x0, int x1, int y0,
                                         int y1, Cls& c) {
    const int T = F.T;
    if (X >= 0.0f && X < (float)F.W && Y >= 0.0f && Y < (float)F.H) {
        // X, Y >= 0 here and the box corners are clipped to the image, so
        // the divisions by the power-of-two tile side are shifts
        const int tx = (int)X >> F.Tshift, ty = (int)Y >> F.Tshift;
        const int ex0 = tx * T - F.halo, ex1 = tx * T + T - 1 + F.halo;
        const int ey0 = ty * T - F.halo, ey1 = ty * T + T - 1 + F.halo;
        if (x0 >= ex0 && x1 <= ex1 && y0 >= ey0 && y1 <= ey1) {
            c.kind = 0;
            c.bin = ty * F.tiles_x + tx;
            return;
        }
    }
    c.tx0 = x0 >> F.Tshift;
    c.tx1 = x1 >> F.Tshift;
    c.ty0 = y0 >> F.Tshift;
    c.ty1 = y1 >> F.Tshift;
    const int nt = (c.tx1 - c.tx0 + 1) * (c.ty1 - c.ty0 + 1);
    if (nt <= F.max_clip) {
        c.kind = 1;
        return;
    }
    c.kind = 2;
    c.bin = F.n_tiles;
}

// Records that may reach |tau| >= tau_lim (|tau| * 2^F >= 2^50) go to the
// large list whatever their footprint: the large pass converts terms with
// the general rounding and range test, the tile splat with the short exact
// one that needs |term| < 2^51.  Same samples, same values.  The test uses
// the bound |amplitude| * max |colour| (max |palette entry|, or 1 for the
// clamped vector colour; no look-up, so the counting pass does not read
// the colour input); NaN fails it.
__device__ __forceinline__ void bright_class(const Frame& F, float amp, float cmax, Cls& c) {
    if (fabsf(amp) * cmax < F.tau_lim) return;
    c.kind = 2;
    c.bin = F.n_tiles;
}

// Largest |palette entry| (NaN counts as infinite), reduced by the whole
// workgroup into *out; every thread must call it.
__device__ __forceinline__ void palette_absmax(const float* __restrict__ cmap, int ncmap,
                                               float* red, float* out) {
    float m = 0.0f;
    for (int i = threadIdx.x; i < 3 * ncmap; i += blockDim.x) {
        const float v = fabsf(cmap[i]);
        m = (v == v) ? fmaxf(m, v) : __builtin_inff();
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t = fmaxf(t, red[k]);
        *out = t;
    }
    __syncthreads();
}

// Bound on |colour| of the job's colour mode, in *out (workgroup-wide,
// every thread must call it): the palette's largest |entry|, or 1 for the
// clamped vector colour.
__device__ __forceinline__ void colour_absmax(const Frame& F, const float* __restrict__ cmap,
                                              float* red, float* out) {
    if (F.colmode) {
        if (threadIdx.x == 0) *out = 1.0f;
        __syncthreads();
    } else {
        palette_absmax(cmap, F.ncmap, red, out);
    }
}

// The weight exp(-d^2/sigma^2) of pixel (gx, gy) for a record, or false if
// the pixel centre is outside the clip circle d^2 <= R^2 (Eq. 2 clipped at
// chi*sigma).
__device__ __forceinline__ bool sample_weight(float X, float Y, float k2, float R2, int gx, int gy,
                                              float& w) {
    const float dx = ((float)gx + 0.5f) - X;
    const float dy = ((float)gy + 0.5f) - Y;
    const float d2 = fmaf(dx, dx, dy * dy);
    if (!(d2 <= R2)) return false;
    w = __builtin_amdgcn_exp2f(d2 * k2);
    return true;
}

template <typename Acc>
struct AccOps;

template <>
struct AccOps<float> {
    // FP32 planes: tau * w in float (tq carries no scale in this form)
    __device__ static __forceinline__ float term(float tau, float w, const Frame&) {
        return tau * w;
    }
    __device__ static __forceinline__ void lds_add(float* p, float v) { atomicAdd(p, v); }
    __device__ static __forceinline__ void global_add(float* p, float v) { (void)gatomic_add(p, v); }
};

// Fixed-point term of one sample: rint(tq * w) with tq = tau * 2^F (a
// float; the power-of-two scale is exact) and w the Gaussian weight.  The
// product of two floats is exact in double, so the term is the exact
// product rounded once to the nearest integer (ties to even).
//
// Short form for |tq * w| < 2^51: fma(tq, w, 1.5 * 2^52) rounds the exact
// product to an integer held in the low mantissa bits; the magic number's
// low word is zero, so one 32-bit subtraction from the high word recovers
// the two's complement integer.
__device__ __forceinline__ long long term_short(double tq, double w) {
    const double d = fma(tq, w, 6755399441055744.0);
    const unsigned long long b = (unsigned long long)__double_as_longlong(d);
    const uint32_t lo = (uint32_t)b;
    const uint32_t hi = (uint32_t)(b >> 32) - 0x43380000u;
    return (long long)(((unsigned long long)hi << 32) | lo);
}

template <>
struct AccOps<long long> {
    // General form, any magnitude: a term at or above 2^62 (or NaN) sets the
    // overflow flag and counts as zero.  The tile splat, which only sees
    // records with |tq| < 2^50 (bright_class), uses term_short.
    __device__ static __forceinline__ long long term(float tq, float w, const Frame& F) {
        const double p = (double)tq * (double)w;
        if (!(fabs(p) < 4.0e18)) {
            atomicOr(F.oflag, 1u);
            return 0;
        }
        return __double2ll_rn(p);
    }
    __device__ static __forceinline__ void lds_add(long long* p, long long v) {
        atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    }
    __device__ static __forceinline__ void global_add(long long* p, long long v) {
        (void)gatomic_add(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    }
};

// Checked int64 additions.  Every addition into an int64 pixel sum goes
// through one of these, so a sum that leaves the int64 range sets the
// overflow flag the moment it does (whatever the signs of the terms); the
// tile splat's LDS partials need no check, since a work item adds at most
// kMaxChunk terms below 2^50 per pixel.
__device__ __forceinline__ long long add_checked(long long a, long long b, unsigned int* oflag) {
    long long s;
    if (__builtin_add_overflow(a, b, &s)) atomicOr(oflag, 1u);
    return s;
}

__device__ __forceinline__ void global_add_checked(long long* p, long long v, unsigned int* oflag) {
    const unsigned long long old =
        gatomic_add(reinterpret_cast<unsigned long long*>(p), (unsigned long long)v);
    const unsigned long long s = old + (unsigned long long)v;
    // signed overflow: both operands have the sign the sum does not
    if ((long long)((old ^ s) & ((unsigned long long)v ^ s)) < 0) atomicOr(oflag, 1u);
}

// A 64-bit LDS word addressed through the local address space, and an
// integer add into it (no return value).
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ __forceinline__ void lds_add_u64(lds_u64* p, long long v) {
    __hip_atomic_fetch_add(p, (unsigned long long)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Wave64 inclusive scans with DPP: a Hillis-Steele scan inside each row of
// 16 lanes (row_shr 1, 2, 4, 8; with bound_ctrl a lane without a source
// reads 0, the identity, so no identity register has to be refreshed), then
// the last lane of row 0 and 2 is broadcast into rows 1 and 3 (row_bcast:15)
// and the last lane of row 1 into rows 2 and 3 (row_bcast:31); rows left
// out by the row mask keep the old operand, 0.  No LDS round trip.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t u) {
    int v = (int)u;
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
    return (uint32_t)v;
}

// Inclusive prefix maximum over the wave of non-negative values (identity
// 0), same pattern.
__device__ __forceinline__ int wave_incl_max0(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
    return v;
}

}  // namespace splotch_dev
