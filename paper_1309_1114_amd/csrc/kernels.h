// Render kernels.  Every kernel reads its jobs from a device table, so one
// launch sequence serves a single render (one job) and a batch of jobs of
// uneven sizes and resolutions.  No kernel waits on the host.
//
//   k_clear     zero each job's optical-depth planes (and centre counts)
//   k_count     one thread per particle: processing stage (transform,
//               projection, palette), footprint class, per-workgroup LDS
//               histogram of tile keys (optionally the radius statistics);
//               the centre counts are taken where the records are drawn
//               (k_splat, k_large), in LDS
//   k_segsum / k_binscan / k_offsets
//               exclusive scan of the (key, workgroup) counts: a one-digit
//               counting sort by tile key (the sort step of Section "CUDA
//               Implementation")
//   k_scatter   re-derives each record and writes it at its sorted slot
//   k_items     cuts the tile lists of all jobs into one list of work items
//   k_lgcount / k_lgscan / k_lgscatter
//               index the large-footprint list by pixel group
//   k_large     per-group pixel-block gather over the large records (no
//               per-sample atomics; replaces the paper's CPU path for large
//               particles, Section "Large Particles")
//   k_splat     persistent workgroups pull tile items of any job and splat
//               the clipped Gaussians (Eq. 2) into an LDS tile
//   k_resolve   I = 1 - exp(-L) per pixel and colour (Eq. 1 with E = A)
#pragma once

#include "device.h"

namespace splotch_dev {

// ---------------------------------------------------------------------------
template <typename Acc>
__global__ void k_clear(const JobDev* __restrict__ jobs, unsigned long long* __restrict__ stats,
                        int clear_stats) {
    const JobDev& J = jobs[blockIdx.y];
    const size_t plane_bytes = (size_t)3 * J.F.W * J.F.H * sizeof(Acc);
    const size_t n16 = (plane_bytes + 15) / 16;  // the region is padded to 256 bytes
    uint4* p = reinterpret_cast<uint4*>(J.L);
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
    if (J.ccount) {
        const size_t np = (size_t)J.F.W * J.F.H;
        for (size_t i = t0; i < np; i += stride) J.ccount[i] = 0;
    }
    if (clear_stats && stats && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < kStatWords)
        stats[threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// k_tile_live: grid (ceil(NB_max / 256), n_jobs).  With a region mask, the
// flags of every tile: bit 0 its core meets a marked region, bit 1 the tile
// widened by the halo does.
__global__ void k_tile_live(const JobDev* __restrict__ jobs) {
    const JobDev& J = jobs[blockIdx.y];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!J.rmask || t >= J.F.n_tiles) return;
    J.tlive[t] = (uint8_t)((tile_on(J, t, 0) ? 1 : 0) | (tile_on(J, t, J.F.halo) ? 2 : 0));
}

// Stages a job's tile flags in LDS after the NB key words (all threads
// call it); nullptr without a mask.
__device__ __forceinline__ const SPLOTCH_LDS uint8_t* stage_live(const JobDev& J, uint32_t* sh) {
    if (!J.rmask) return nullptr;
    SPLOTCH_LDS uint8_t* live = (SPLOTCH_LDS uint8_t*)(sh + J.NB);
    for (int t = threadIdx.x; t < J.F.n_tiles; t += blockDim.x) live[t] = gmem(J.tlive)[t];
    return live;
}

// ---------------------------------------------------------------------------
// k_count: grid (P_max, n_jobs).  Workgroup w of job j counts the keys of
// particles [w*per_block, (w+1)*per_block) into hist[w][key].
template <bool RSTATS>
__global__ __launch_bounds__(kCountThreads) void k_count(const JobDev* __restrict__ jobs,
                                                         unsigned long long* __restrict__ stats) {
    extern __shared__ uint32_t sh_hist[];
    const JobDev& J = jobs[blockIdx.y];
    const int P = J.P;
    if ((int)blockIdx.x >= P) return;
    const Frame F = J.F;
    const PartPtrs pp = J.pp;
    const float* __restrict__ cmap = J.cmap;
    const int NB = J.NB;
    __shared__ float s_red[kCountThreads / 64];
    __shared__ float s_cmax;
    for (int b = threadIdx.x; b < NB; b += blockDim.x) sh_hist[b] = 0u;
    const SPLOTCH_LDS uint8_t* live = stage_live(J, sh_hist);
    colour_absmax(F, cmap, s_red, &s_cmax);     // (synchronises the workgroup)
    const float cmax = s_cmax;
    const int64_t beg = (int64_t)blockIdx.x * J.per_block;
    const int64_t end = min(J.n, beg + J.per_block);
    uint32_t active = 0;
    uint32_t rh[5] = {0u, 0u, 0u, 0u, 0u};   // radius histogram of active particles
    double rsum = 0.0;
    // kLoadBatch particles per thread are loaded before any is processed,
    // so each wave keeps several loads of the particle stream in flight
    for (int64_t i0 = beg + threadIdx.x; i0 < end; i0 += kLoadBatch * blockDim.x) {
        RawPart q[kLoadBatch];
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            const int64_t i = i0 + (int64_t)u * blockDim.x;
            if (i < end) q[u] = load_part(pp, i, F.colmode);
        }
#pragma unroll
        for (int u = 0; u < kLoadBatch; ++u) {
            if (i0 + (int64_t)u * blockDim.x >= end) break;
            Rec r;
            int x0, x1, y0, y1;
            float amp;
            if (!project_particle(F, cmap, q[u].x, q[u].y, q[u].z, q[u].h, q[u].inten,
                                  q[u].col, q[u].sp, r, x0, x1, y0, y1, amp))
                continue;
            ++active;
            if constexpr (RSTATS) {
                const float rad = sqrtf(r.R2);
                rsum += (double)rad;
                const int bin = rad <= 2.0f ? 0 : rad <= 4.0f ? 1 : rad <= 8.0f ? 2
                                : rad <= 16.0f ? 3 : 4;
#pragma unroll
                for (int k = 0; k < 5; ++k) rh[k] += bin == k ? 1u : 0u;
            }
            Cls c;
            classify(F, r.X, r.Y, x0, x1, y0, y1, c);
            bright_class(F, amp, cmax, c);
            // with a region mask, entries of tiles outside the marked
            // regions are not made (k_scatter takes the same decisions)
            if (c.kind != 1) {
                if (c.kind == 2 || tile_live(live, c.bin, true)) atomicAdd(&sh_hist[c.bin], 1u);
            } else {
                for (int ty = c.ty0; ty <= c.ty1; ++ty)
                    for (int tx = c.tx0; tx <= c.tx1; ++tx)
                        if (tile_live(live, ty * F.tiles_x + tx, false))
                            atomicAdd(&sh_hist[ty * F.tiles_x + tx], 1u);
            }
        }
    }
    uint32_t wsum = active;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        wsum += __shfl_xor(wsum, d, 64);
        if constexpr (RSTATS) {
            rsum += __shfl_xor(rsum, d, 64);
#pragma unroll
            for (int k = 0; k < 5; ++k) rh[k] += __shfl_xor(rh[k], d, 64);
        }
    }
    if ((threadIdx.x & 63) == 0 && wsum) {
        atomicAdd(stats + ST_ACTIVE, (unsigned long long)wsum);
        if constexpr (RSTATS) {
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (rh[k]) atomicAdd(stats + ST_RHIST + k, (unsigned long long)rh[k]);
            atomicAdd(reinterpret_cast<double*>(stats + ST_RSUM), rsum);
        }
    }
    __syncthreads();
    SPLOTCH_GLOBAL uint32_t* out = gmem(J.hist + (size_t)blockIdx.x * NB);
    for (int b = threadIdx.x; b < NB; b += blockDim.x) out[b] = sh_hist[b];
}

// grid (ceil(NB_max/256), nseg_max, n_jobs): seg[s][b] = sum over the
// segment's workgroups of hist[w][b]
__global__ void k_segsum(const JobDev* __restrict__ jobs) {
    const JobDev& J = jobs[blockIdx.z];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    const int NB = J.NB;
    if (b >= NB || s >= J.nseg) return;
    uint32_t acc = 0;
    const uint32_t* p = J.hist + (size_t)s * kSeg * NB + b;
#pragma unroll 8
    for (int w = 0; w < kSeg; ++w) acc += p[(size_t)w * NB];
    J.seg[(size_t)s * NB + b] = acc;
}

// grid (n_jobs) x 1024: key totals -> exclusive key starts bin[0..NB], and
// seg rewritten in place to each segment's first slot per key.
__global__ __launch_bounds__(1024) void k_binscan(const JobDev* __restrict__ jobs) {
    __shared__ uint32_t part[1024];
    const JobDev& J = jobs[blockIdx.x];
    const int NB = J.NB, nseg = J.nseg;
    uint32_t* seg = J.seg;
    uint32_t* bin = J.bin;
    const int t = threadIdx.x;
    const int per = (NB + 1023) / 1024;
    const int b0 = min(NB, t * per), b1 = min(NB, b0 + per);
    uint32_t local = 0;
    for (int b = b0; b < b1; ++b)
        for (int s = 0; s < nseg; ++s) local += seg[(size_t)s * NB + b];
    part[t] = local;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - local;
    for (int b = b0; b < b1; ++b) {
        bin[b] = run;
        for (int s = 0; s < nseg; ++s) {
            const uint32_t v = seg[(size_t)s * NB + b];
            seg[(size_t)s * NB + b] = run;
            run += v;
        }
    }
    if (t == 1023) bin[NB] = part[1023];
}

// grid as k_segsum: hist[w][b] := first slot of workgroup w's records of key b
__global__ void k_offsets(const JobDev* __restrict__ jobs) {
    const JobDev& J = jobs[blockIdx.z];
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    const int NB = J.NB;
    if (b >= NB || s >= J.nseg) return;
    uint32_t run = J.seg[(size_t)s * NB + b];
    uint32_t* p = J.hist + (size_t)s * kSeg * NB + b;
    for (int w = 0; w < kSeg; ++w) {
        const uint32_t v = p[(size_t)w * NB];
        p[(size_t)w * NB] = run;
        run += v;
    }
}

// k_scatter: the same particle ranges and decisions as k_count; writes each
// record at its slot.
__global__ __launch_bounds__(kCountThreads) void k_scatter(const JobDev* __restrict__ jobs,
                                                           unsigned long long* __restrict__ stats) {
    extern __shared__ uint32_t sh_cur[];
    const JobDev& J = jobs[blockIdx.y];
    if ((int)blockIdx.x >= J.P) return;
    const Frame F = J.F;
    const PartPtrs pp = J.pp;
    const float* __restrict__ cmap = J.cmap;
    const int NB = J.NB;
    const uint32_t cap = J.cap;
    Rec* __restrict__ recs = J.recs;
    const SPLOTCH_GLOBAL uint32_t* base = gmem(J.hist + (size_t)blockIdx.x * NB);
    __shared__ float s_red[kCountThreads / 64];
    __shared__ float s_cmax;
    // palettes of up to kLdsPalette entries are read from LDS: the look-up
    // sits in each particle's dependent chain (load, colour, slot, store)
    __shared__ float s_pal[3 * kLdsPalette];
    for (int b = threadIdx.x; b < NB; b += blockDim.x) sh_cur[b] = base[b];
    const SPLOTCH_LDS uint8_t* live = stage_live(J, sh_cur);
    colour_absmax(F, cmap, s_red, &s_cmax);     // (synchronises the workgroup)
    const float cmax = s_cmax;
    const bool lds_pal = !F.colmode && F.ncmap <= kLdsPalette;
    if (lds_pal) {
        for (int i = threadIdx.x; i < 3 * F.ncmap; i += blockDim.x) s_pal[i] = cmap[i];
        __syncthreads();
    }
    const int64_t beg = (int64_t)blockIdx.x * J.per_block;
    const int64_t end = min(J.n, beg + J.per_block);
    // the particle loop, instantiated once per palette address space (the
    // LDS copy or device memory), so that no access in it is a flat one
    auto particles = [&](auto pal) {
    for (int64_t i0 = beg + threadIdx.x; i0 < end; i0 += kLoadBatch * blockDim.x) {
      RawPart q[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        const int64_t i = i0 + (int64_t)u * blockDim.x;
        if (i < end) q[u] = load_part(pp, i, F.colmode);
      }
      // all particles of the batch are projected and classified first, so
      // their slot atomics and record stores are issued back to back
      Rec r[kLoadBatch];
      Cls c[kLoadBatch];
      bool ok[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        int x0, x1, y0, y1;
        float amp;
        ok[u] = i0 + (int64_t)u * blockDim.x < end &&
                project_particle(F, pal, q[u].x, q[u].y, q[u].z, q[u].h, q[u].inten, q[u].col,
                                 q[u].sp, r[u], x0, x1, y0, y1, amp);
        if (ok[u]) {
            classify(F, r[u].X, r[u].Y, x0, x1, y0, y1, c[u]);
            bright_class(F, amp, cmax, c[u]);
        }
      }
      // one record (own bordered tile, or the large list): one slot each.
      // k_count made the same decisions, so every slot lies inside its
      // key's range; the capacity test only guards against a mismatch
      uint32_t pos[kLoadBatch];
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        if (ok[u] && c[u].kind == 0 && !tile_live(live, c[u].bin, true)) ok[u] = false;
        pos[u] = ok[u] && c[u].kind != 1 ? atomicAdd(&sh_cur[c[u].bin], 1u) : 0u;
      }
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        if (!ok[u] || c[u].kind == 1) continue;
        if (pos[u] < cap) {
            float4* dst = reinterpret_cast<float4*>(recs + pos[u]);
            gstore4(dst, make_float4(r[u].X, r[u].Y, r[u].k2, r[u].R2));
            gstore4(dst + 1, make_float4(r[u].r, r[u].g, r[u].b,
                                         __uint_as_float(c[u].kind == 0 ? 1u : 0u)));
        } else {
            atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
        }
      }
      // one record per touched tile, clipped there
#pragma unroll
      for (int u = 0; u < kLoadBatch; ++u) {
        if (!ok[u] || c[u].kind != 1) continue;
        const float4 lo = make_float4(r[u].X, r[u].Y, r[u].k2, r[u].R2);
        const float4 hi = make_float4(r[u].r, r[u].g, r[u].b, __uint_as_float(0u));
        for (int ty = c[u].ty0; ty <= c[u].ty1; ++ty)
            for (int tx = c[u].tx0; tx <= c[u].tx1; ++tx) {
                if (!tile_live(live, ty * F.tiles_x + tx, false)) continue;
                const uint32_t p = atomicAdd(&sh_cur[ty * F.tiles_x + tx], 1u);
                if (p < cap) {
                    float4* dst = reinterpret_cast<float4*>(recs + p);
                    gstore4(dst, lo);
                    gstore4(dst + 1, hi);
                } else {
                    atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
                }
            }
      }
    }
    };
    if (lds_pal)
        particles((const SPLOTCH_LDS float*)s_pal);
    else
        particles(gmem(cmap));
}

// ---------------------------------------------------------------------------
// k_items: one workgroup.  For every job in turn, split each tile's record
// range into items of at most `chunk` records: items[k] = (job, tile, begin,
// end), dense over all jobs.  Also sizes each job's large-footprint pass.
__global__ __launch_bounds__(1024) void k_items(JobDev* __restrict__ jobs, int n_jobs,
                                                int4* __restrict__ items, uint32_t max_items_total,
                                                uint32_t* __restrict__ ctrl,
                                                unsigned long long* __restrict__ stats) {
    __shared__ uint32_t part[1024];
    __shared__ uint32_t s_base;
    const int t = threadIdx.x;
    if (t == 0) s_base = 0u;
    __syncthreads();
    for (int j = 0; j < n_jobs; ++j) {
        JobDev& J = jobs[j];
        const int n_tiles = J.F.n_tiles;
        const uint32_t* bin = J.bin;
        const uint32_t chunk = (uint32_t)J.chunk;
        const int per = (n_tiles + 1023) / 1024;
        const int t0 = min(n_tiles, t * per), t1 = min(n_tiles, t0 + per);
        uint32_t local = 0;
        for (int k = t0; k < t1; ++k) {
            const uint32_t cnt = bin[k + 1] - bin[k];
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
        const uint32_t job_items = part[1023];
        const uint32_t base = s_base;
        // counts beyond the record capacity or the item space are never
        // expected; such a job draws nothing rather than read past a buffer
        const bool sane = bin[n_tiles + 1] <= J.cap && job_items <= J.max_items &&
                          base + job_items <= max_items_total;
        if (sane) {
            uint32_t out = base + part[t] - local;
            for (int k = t0; k < t1; ++k) {
                const uint32_t b = bin[k], e = bin[k + 1];
                for (uint32_t s = b; s < e; s += chunk)
                    items[out++] = make_int4(j, k, (int)s, (int)min(e, s + chunk));
            }
        }
        for (int g = t; g < J.NG; g += 1024) J.lg_cnt[g] = 0u;
        __syncthreads();
        if (t == 0) {
            const uint32_t n_large = sane ? bin[n_tiles + 1] - bin[n_tiles] : 0u;
            s_base = base + (sane ? job_items : 0u);
            if (!sane) atomicOr(reinterpret_cast<unsigned int*>(stats + ST_BADSLOT), 1u);
            atomicAdd(stats + ST_ENTRIES, (unsigned long long)(sane ? bin[n_tiles + 1] : 0u));
            atomicAdd(stats + ST_LARGE, (unsigned long long)n_large);
            atomicAdd(stats + ST_ITEMS, (unsigned long long)(sane ? job_items : 0u));
        }
        __syncthreads();
    }
    if (t == 0) {
        ctrl[CT_NITEMS] = s_base;
        ctrl[CT_WORK] = 0u;
    }
}

// Adds each thread's sample count to the statistics word (one atomic per
// wave).  The statistics mode that calls it is off in timed renders.
__device__ __forceinline__ void count_samples(uint32_t nsamp,
                                              unsigned long long* __restrict__ stats) {
    unsigned long long v = nsamp;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if ((threadIdx.x & 63) == 0 && v) atomicAdd(stats + ST_SAMPLES, v);
}

// ---------------------------------------------------------------------------
// Large-pass binning.  Every record of a job's large list gets one index
// entry per pixel group (lg_side x lg_side pixels) its footprint box
// touches, so the large pass gathers, for each group, only the records that
// reach it.  Count (per-workgroup LDS histograms added to lg_cnt), scan
// (one workgroup for all jobs: list starts, item starts, job item offsets),
// scatter (each workgroup reserves its runs, then writes them).

// Pixel groups touched by the footprint box of a record, clipped to the
// image; false if the box misses the image.
__device__ __forceinline__ bool record_groups(const JobDev& J, float4 a, int& gx0, int& gx1,
                                              int& gy0, int& gy1) {
    const float R = sqrtf(a.w);
    const float fx0 = fmaxf(floorf(a.x - R - 0.5f), 0.0f);
    const float fx1 = fminf(ceilf(a.x + R - 0.5f), (float)(J.F.W - 1));
    const float fy0 = fmaxf(floorf(a.y - R - 0.5f), 0.0f);
    const float fy1 = fminf(ceilf(a.y + R - 0.5f), (float)(J.F.H - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
    gx0 = (int)fx0 / J.lg_side;
    gx1 = (int)fx1 / J.lg_side;
    gy0 = (int)fy0 / J.lg_side;
    gy1 = (int)fy1 / J.lg_side;
    return true;
}

__device__ __forceinline__ void large_range(const JobDev& J, uint32_t& lb, uint32_t& le) {
    le = min(J.bin[J.F.n_tiles + 1], J.cap);
    lb = min(J.bin[J.F.n_tiles], le);
}

// Histogram of this workgroup's slice of the large list into h[NG].
__device__ __forceinline__ void large_histogram(const JobDev& J, uint32_t lb, uint32_t le,
                                                uint32_t* h) {
    const uint32_t n = le - lb;
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t e0 = lb + blockIdx.x * per, e1 = min(le, e0 + per);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const float4 a = reinterpret_cast<const float4*>(J.recs + e)[0];
        int gx0, gx1, gy0, gy1;
        if (!record_groups(J, a, gx0, gx1, gy0, gy1)) continue;
        for (int gy = gy0; gy <= gy1; ++gy)
            for (int gx = gx0; gx <= gx1; ++gx) atomicAdd(&h[gy * J.ngx + gx], 1u);
    }
}

// grid (kLgBlocks, n_jobs) x 256
__global__ __launch_bounds__(256) void k_lgcount(const JobDev* __restrict__ jobs) {
    __shared__ uint32_t h[kMaxLargeGroups];
    const JobDev& J = jobs[blockIdx.y];
    uint32_t lb, le;
    large_range(J, lb, le);
    if (lb == le) return;
    for (int g = threadIdx.x; g < J.NG; g += blockDim.x) h[g] = 0u;
    __syncthreads();
    large_histogram(J, lb, le, h);
    __syncthreads();
    for (int g = threadIdx.x; g < J.NG; g += blockDim.x)
        if (h[g]) atomicAdd(J.lg_cnt + g, h[g]);
}

// one workgroup x 1024: per job, exclusive scans of the group counts (list
// starts) and of their item counts (one item per E entries, E a power of two
// in 16..256 chosen so that the job has about kLgTargetItems items); job item
// offsets over all jobs; cursors for the scatter.  A job whose entries
// exceed cap_idx falls back to scanning its whole list per group.
__global__ __launch_bounds__(1024) void k_lgscan(JobDev* __restrict__ jobs, int n_jobs,
                                                 uint32_t* __restrict__ ctrl) {
    __shared__ uint32_t pc[1024], pk[1024];
    __shared__ uint32_t s_lbase, s_total;
    const int t = threadIdx.x;
    if (t == 0) s_lbase = 0u;
    __syncthreads();
    for (int j = 0; j < n_jobs; ++j) {
        JobDev& J = jobs[j];
        const int NG = J.NG;
        const int per = (NG + 1023) / 1024;
        const int g0 = min(NG, t * per), g1 = min(NG, g0 + per);
        uint32_t c = 0;
        for (int g = g0; g < g1; ++g) c += J.lg_cnt[g];
        if (t == 0) s_total = 0u;
        __syncthreads();
        if (c) atomicAdd(&s_total, c);
        __syncthreads();
        uint32_t E = 16;
        while (E < (uint32_t)kLargeThreads && (uint64_t)E * kLgTargetItems < s_total) E *= 2;
        uint32_t k = 0;
        for (int g = g0; g < g1; ++g) k += (J.lg_cnt[g] + E - 1) / E;
        pc[t] = c;
        pk[t] = k;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const uint32_t vc = t >= d ? pc[t - d] : 0u, vk = t >= d ? pk[t - d] : 0u;
            __syncthreads();
            pc[t] += vc;
            pk[t] += vk;
            __syncthreads();
        }
        uint32_t rc = pc[t] - c, rk = pk[t] - k;
        for (int g = g0; g < g1; ++g) {
            const uint32_t v = J.lg_cnt[g];
            J.lg_start[g] = rc;
            J.lg_chunk[g] = rk;
            J.lg_cnt[g] = rc;          // cursor for k_lgscatter
            rc += v;
            rk += (v + E - 1) / E;
        }
        __syncthreads();
        if (t == 0) {
            const uint32_t total = pc[1023], items = pk[1023];
            J.lg_start[NG] = total;
            J.lg_chunk[NG] = items;
            uint32_t lb, le;
            large_range(J, lb, le);
            const int fb = total > J.cap_idx ? 1 : 0;
            const int ngy = (J.F.H + J.lg_side - 1) / J.lg_side;
            const uint32_t nli = lb == le ? 0u
                                 : fb ? (uint32_t)(J.ngx * ngy) *
                                            ((le - lb + kLargeThreads - 1) / kLargeThreads)
                                      : items;
            J.lg_fallback = fb;
            J.lg_per_item = (int)E;
            J.large_item0 = s_lbase;
            J.n_large_items = nli;
            s_lbase += nli;
        }
        __syncthreads();
    }
    if (t == 0) ctrl[CT_NLARGE_ITEMS] = s_lbase;
}

// grid (kLgBlocks, n_jobs) x 256: the same slices as k_lgcount; each
// workgroup reserves one run per group, then writes its entries there.
__global__ __launch_bounds__(256) void k_lgscatter(const JobDev* __restrict__ jobs) {
    __shared__ uint32_t h[kMaxLargeGroups];
    const JobDev& J = jobs[blockIdx.y];
    uint32_t lb, le;
    large_range(J, lb, le);
    if (lb == le || J.lg_fallback) return;
    for (int g = threadIdx.x; g < J.NG; g += blockDim.x) h[g] = 0u;
    __syncthreads();
    large_histogram(J, lb, le, h);
    __syncthreads();
    for (int g = threadIdx.x; g < J.NG; g += blockDim.x)
        if (h[g]) h[g] = atomicAdd(J.lg_cnt + g, h[g]);
    __syncthreads();
    const uint32_t n = le - lb;
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    const uint32_t e0 = lb + blockIdx.x * per, e1 = min(le, e0 + per);
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        const float4 a = reinterpret_cast<const float4*>(J.recs + e)[0];
        int gx0, gx1, gy0, gy1;
        if (!record_groups(J, a, gx0, gx1, gy0, gy1)) continue;
        for (int gy = gy0; gy <= gy1; ++gy)
            for (int gx = gx0; gx <= gx1; ++gx) {
                const int g = gy * J.ngx + gx;
                const uint32_t slot = atomicAdd(&h[g], 1u);
                // the counts match k_lgcount's, so the slot lies in the
                // group's list; the tests only guard the buffer
                if (slot < J.lg_start[g + 1] && slot < J.cap_idx) J.lg_idx[slot] = e - lb;
            }
    }
}

// ---------------------------------------------------------------------------
// k_large: persistent grid-stride loop over the large-pass items of all jobs.
// Item = (pixel group, up to 256 entries of the group's index list): the
// workgroup loads those records; each thread then gathers 4 pixels of every
// 32x32 block of the group over that short list and adds its sums to the
// plane once per pixel.  A job whose index lists overflowed uses items
// (group, chunk of 256 consecutive large records) and keeps the records of
// the chunk that touch the group.
template <typename Acc, bool CNT>
__global__ __launch_bounds__(kLargeThreads) void k_large(const JobDev* __restrict__ jobs, int n_jobs,
                                                         const uint32_t* __restrict__ ctrl,
                                                         unsigned long long* __restrict__ stats) {
    __shared__ float4 sA[kLargeThreads];
    __shared__ float4 sB[kLargeThreads];
    __shared__ int4 sR[kLargeThreads];
    __shared__ int s_cnt;
    __shared__ int s_nonfinite;   // some staged record has a non-finite coefficient
    const uint32_t nitems = ctrl[CT_NLARGE_ITEMS];
    const int tid = threadIdx.x;
    const int lx = tid & (kLargeBlock - 1);
    const int ly0 = tid >> 5;  // rows ly0 + 8k, k = 0..3
    uint32_t nsamp = 0;        // samples drawn by this thread (CNT only)
    for (uint32_t it = blockIdx.x; it < nitems; it += gridDim.x) {
        int j = 0;
        while (j + 1 < n_jobs && it >= jobs[j + 1].large_item0) ++j;
        const JobDev& J = jobs[j];
        const Frame F = J.F;
        const uint32_t local = it - J.large_item0;
        uint32_t lb, le;
        large_range(J, lb, le);
        const int G = J.lg_side, ngx = J.ngx;
        int g;
        uint32_t e = 0xffffffffu;          // this thread's record, if any
        if (J.lg_fallback) {
            g = (int)(local % (uint32_t)J.NG);
            const uint32_t ch = local / (uint32_t)J.NG;
            const uint32_t c = lb + ch * kLargeThreads + tid;
            if (c < le) e = c;
        } else {
            // the group whose items contain `local`: lg_chunk[g] <= local
            // < lg_chunk[g + 1] (binary search, the same in every thread)
            int lo = 0, hi = J.NG;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (J.lg_chunk[mid] <= local) lo = mid; else hi = mid;
            }
            g = lo;
            const uint32_t E = (uint32_t)J.lg_per_item;
            const uint32_t i = J.lg_start[g] + (local - J.lg_chunk[g]) * E + tid;
            if ((uint32_t)tid < E && i < J.lg_start[g + 1] && i < J.cap_idx) {
                const uint32_t c = lb + J.lg_idx[i];
                if (c < le) e = c;
            }
        }
        const int gx0 = (g % ngx) * G, gy0 = (g / ngx) * G;
        const int gx1 = min(gx0 + G, F.W) - 1, gy1 = min(gy0 + G, F.H) - 1;
        if (!rect_on(J, gx0, gx1, gy0, gy1)) e = 0xffffffffu;   // nothing drawn here
        Acc* __restrict__ Lg = reinterpret_cast<Acc*>(J.L);
        const size_t plane = (size_t)F.W * F.H;
        if (tid == 0) {
            s_cnt = 0;
            s_nonfinite = 0;
        }
        __syncthreads();
        if (e != 0xffffffffu) {
            const float4* rp = reinterpret_cast<const float4*>(J.recs + e);
            const float4 a = gload4(rp), b = gload4(rp + 1);
            // centre count: the group holding the centre pixel counts the
            // record (every group of its footprint box sees it once)
            if (J.ccount && a.x >= 0.0f && a.x < (float)F.W && a.y >= 0.0f && a.y < (float)F.H) {
                const int px = (int)a.x, py = (int)a.y;
                if (px >= gx0 && px <= gx1 && py >= gy0 && py <= gy1)
                    atomicAdd(J.ccount + (size_t)py * F.W + px, 1);
            }
            const float R = sqrtf(a.w);
            float fx0, fx1, fy0, fy1;
            disk_span(a.x, R, (float)gx0, (float)gx1, fx0, fx1);
            disk_span(a.y, R, (float)gy0, (float)gy1, fy0, fy1);
            if (fx0 <= fx1 && fy0 <= fy1) {
                const int slot = atomicAdd(&s_cnt, 1);
                sA[slot] = a;
                float4 tq = b;          // int64 planes: tau * 2^F (exact scale)
                if constexpr (sizeof(Acc) == 8) {
                    tq.x *= F.qscale;
                    tq.y *= F.qscale;
                    tq.z *= F.qscale;
                }
                sB[slot] = tq;
                sR[slot] = make_int4((int)fx0, (int)fx1, (int)fy0, (int)fy1);
                if (!(fabsf(b.x) <= 3.4e38f && fabsf(b.y) <= 3.4e38f && fabsf(b.z) <= 3.4e38f))
                    s_nonfinite = 1;
            }
        }
        __syncthreads();
        const int cnt = s_cnt;
        // FP32 planes with finite coefficients: the pixel loop without a
        // branch per pixel (a weight of 0 outside the disk; the same samples
        // and values).  A non-finite coefficient times that 0 would reach
        // pixels outside its disk, so its item takes the loop below.
        const bool branch_free = sizeof(Acc) == 4 && !CNT && s_nonfinite == 0;
        for (int by = gy0; by <= gy1; by += kLargeBlock) {
            for (int bx = gx0; bx <= gx1; bx += kLargeBlock) {
                const int bx1 = min(bx + kLargeBlock - 1, gx1), by1 = min(by + kLargeBlock - 1, gy1);
                Acc acc[4][3];
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[k][0] = acc[k][1] = acc[k][2] = (Acc)0;
                const int gx = bx + lx;
                if constexpr (sizeof(Acc) == 4 && !CNT) {
                    if (branch_free) {
                        // (sums of pixels past the block's edge are never
                        // written, so those need no test)
                        const float cxp = (float)gx + 0.5f;
                        float cyp[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) cyp[k] = (float)(by + ly0 + 8 * k) + 0.5f;
                        for (int q = 0; q < cnt; ++q) {
                            const int4 rr = sR[q];
                            if (rr.x > bx1 || rr.y < bx || rr.z > by1 || rr.w < by) continue;
                            const float4 a = sA[q];
                            const float4 b = sB[q];
                            const float dx = cxp - a.x;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                // sample_weight's operations, selected
                                const float dy = cyp[k] - a.y;
                                const float d2 = fmaf(dx, dx, dy * dy);
                                const float wk = __builtin_amdgcn_exp2f(d2 * a.z);
                                const float w = d2 <= a.w ? wk : 0.0f;
                                acc[k][0] = fmaf(b.x, w, acc[k][0]);
                                acc[k][1] = fmaf(b.y, w, acc[k][1]);
                                acc[k][2] = fmaf(b.z, w, acc[k][2]);
                            }
                        }
                    }
                }
                for (int q = 0; q < (branch_free ? 0 : cnt); ++q) {
                    const int4 rr = sR[q];
                    if (rr.x > bx1 || rr.y < bx || rr.z > by1 || rr.w < by) continue;  // uniform
                    const float4 a = sA[q];
                    const float4 b = sB[q];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int gy = by + ly0 + 8 * k;
                        float w;
                        if (gx <= bx1 && gy <= by1 && sample_weight(a.x, a.y, a.z, a.w, gx, gy, w)) {
                            if constexpr (CNT) ++nsamp;
                            if constexpr (sizeof(Acc) == 4) {
                                // FP32 planes: one fused multiply-add per channel
                                acc[k][0] = fmaf(b.x, w, acc[k][0]);
                                acc[k][1] = fmaf(b.y, w, acc[k][1]);
                                acc[k][2] = fmaf(b.z, w, acc[k][2]);
                            } else {
                                acc[k][0] = add_checked(acc[k][0], AccOps<Acc>::term(b.x, w, F), F.oflag);
                                acc[k][1] = add_checked(acc[k][1], AccOps<Acc>::term(b.y, w, F), F.oflag);
                                acc[k][2] = add_checked(acc[k][2], AccOps<Acc>::term(b.z, w, F), F.oflag);
                            }
                        }
                    }
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int gy = by + ly0 + 8 * k;
                    if (gx <= bx1 && gy <= by1) {
                        const size_t p = (size_t)gy * F.W + gx;
#pragma unroll
                        for (int c = 0; c < 3; ++c) {
                            if (acc[k][c] == (Acc)0) continue;
                            if constexpr (sizeof(Acc) == 8)
                                global_add_checked(Lg + c * plane + p, acc[k][c], F.oflag);
                            else
                                AccOps<Acc>::global_add(Lg + c * plane + p, acc[k][c]);
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if constexpr (CNT) count_samples(nsamp, stats);
}

// ---------------------------------------------------------------------------
// k_splat: persistent workgroups pull items (job, tile, record range).  The
// LDS accumulator covers the tile plus `halo` pixels on each side (records
// with meta bit 0 are drawn over their whole footprint there; others are
// clipped to the tile), over the pixels its in-disk test can pass
// (disk_span).  Each wave orders its 64 records by segment width and
// expands them into a flat list of segments of up to Q columns by two rows
// (a lane shares the column arithmetic and the loop test between the rows;
// the segments of a row split its width evenly): a wave prefix sum gives
// every record its first segment; inside each 64-segment window every
// record marks its start position and a prefix max over positions gives
// each lane its record.
//
// The tile accumulates in 64-bit fixed point (q = rint(tau * 2^F)) with
// integer LDS atomics in both modes: on gfx950 an LDS float atomic add
// costs about 3 clocks per lane against a fixed 6 clocks per wave
// instruction for a 64-bit integer add.  At the end the tile is added to
// the plane: as int64 in the int64 mode, converted to float in the FP32
// mode.  With a centre-count plane, each record whose centre pixel lies in
// the item's tile counts itself in an LDS array of 16-bit counts (an item
// holds at most kMaxChunk records), added to the plane with the tile.
template <typename Acc, int Q, bool CNT>
__global__ __launch_bounds__(kSplatThreads) void k_splat(const JobDev* __restrict__ jobs,
                                                         const int4* __restrict__ items,
                                                         uint32_t* __restrict__ ctrl,
                                                         int stage_bytes_off, int cnt_off,
                                                         unsigned long long* __restrict__ stats) {
    extern __shared__ __align__(16) unsigned char smem[];
    long long* acc = reinterpret_cast<long long*>(smem);
    float4* stA = reinterpret_cast<float4*>(smem + stage_bytes_off);
    float4* stB = stA + kSplatThreads;
    uint2* stC = reinterpret_cast<uint2*>(stB + kSplatThreads);
    int* own = reinterpret_cast<int*>(stC + kSplatThreads);
    // the work-queue slot lives in the dynamic block too, so the accumulator
    // starts at LDS address 0 and pixel offsets fold into the ds_add offsets
    int& s_item = own[kSplatThreads];
    uint32_t* cnt = reinterpret_cast<uint32_t*>(smem + cnt_off);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    float4* wA = stA + wv * 64;
    float4* wB = stB + wv * 64;
    uint2* wC = stC + wv * 64;
    int* wO = own + wv * 64;
    const uint32_t n_items = ctrl[CT_NITEMS];
    uint32_t nsamp = 0;        // samples drawn by this thread (CNT only)
    for (;;) {
        if (tid == 0) s_item = (int)atomicAdd(ctrl + CT_WORK, 1u);
        __syncthreads();
        const int it = s_item;
        if ((uint32_t)it >= n_items) break;
        const int4 item = items[it];
        const JobDev& J = jobs[item.x];
        const Frame F = J.F;
        const Rec* __restrict__ recs = J.recs;
        Acc* __restrict__ Lg = reinterpret_cast<Acc*>(J.L);
        int32_t* __restrict__ ccount = J.ccount;
        const size_t plane = (size_t)F.W * F.H;
        const int E = F.T + 2 * F.halo;
        const int ES = E | 1;           // odd row stride spreads rows over banks
        const int PS = E * ES;          // pixels of the accumulator (RGB interleaved)
        const int tx = item.y % F.tiles_x, ty = item.y / F.tiles_x;
        const int ox = tx * F.T - F.halo, oy = ty * F.T - F.halo;  // accumulator origin
        // core (clipped entries) and bordered region (centre entries), in image
        const int cx0 = tx * F.T, cx1 = min(tx * F.T + F.T, F.W) - 1;
        const int cy0 = ty * F.T, cy1 = min(ty * F.T + F.T, F.H) - 1;
        const int hx0 = max(ox, 0), hx1 = min(ox + E, F.W) - 1;
        const int hy0 = max(oy, 0), hy1 = min(oy + E, F.H) - 1;
        for (int i = tid; i < 3 * PS; i += kSplatThreads) acc[i] = 0;
        if (ccount)
            for (int i = tid; i < (F.T * F.T) / 2; i += kSplatThreads) cnt[i] = 0u;
        __syncthreads();
        for (int base = item.z + wv * 64; base < item.w; base += kSplatThreads) {
            const int e = base + lane;
            float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
            uint32_t packed = 0, nq = 0, seg_w = 0;
            if (e < item.w) {
                const float4* rp = reinterpret_cast<const float4*>(recs + e);
                const float4 a = gload4(rp), b = gload4(rp + 1);
                const bool centre = (__float_as_uint(b.w) & 1u) != 0u;
                // the particle's centre pixel, counted by the one entry whose
                // tile holds it (the same float test as the other passes)
                if (ccount && a.x >= 0.0f && a.y >= 0.0f) {
                    const int px = (int)a.x, py = (int)a.y;
                    if (px >= cx0 && px <= cx1 && py >= cy0 && py <= cy1) {
                        const int c = (py - cy0) * F.T + (px - cx0);
                        atomicAdd(&cnt[c >> 1], (c & 1) ? 0x10000u : 1u);
                    }
                }
                // the pixels the in-disk test can pass, inside the region
                const float R = sqrtf(a.w);
                float fx0, fx1, fy0, fy1;
                disk_span(a.x, R, (float)(centre ? hx0 : cx0), (float)(centre ? hx1 : cx1), fx0, fx1);
                disk_span(a.y, R, (float)(centre ? hy0 : cy0), (float)(centre ? hy1 : cy1), fy0, fy1);
                if (fx0 <= fx1 && fy0 <= fy1) {
                    const int x0 = (int)fx0 - ox, x1 = (int)fx1 - ox;
                    const int y0 = (int)fy0 - oy, y1 = (int)fy1 - oy;
                    // segments: up to Q columns of a pair of rows; a row's
                    // qpr segments share its width evenly (9 columns: 5 + 4,
                    // not 8 + 1), so the column loop of a wave ends sooner
                    const uint32_t w = (uint32_t)(x1 - x0 + 1);
                    const uint32_t qpr = (w + Q - 1) / Q;
                    seg_w = (w + qpr - 1) / qpr;
                    nq = qpr * ((uint32_t)(y1 - y0 + 2) / 2);
                    packed = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)x1 << 16) |
                             ((uint32_t)y1 << 24);
                    A = a;
                    // tau * 2^F (a power-of-two scale is exact)
                    B = make_float4(b.x * F.qscale, b.y * F.qscale, b.z * F.qscale,
                                    1.0f / (float)qpr);
                }
            }
            // The wave's records in order of segment width (a stable
            // counting sort over one ballot per width): the segments of a
            // 64-segment window then share one column loop length.
            uint32_t pos = 0;
#pragma unroll
            for (uint32_t v = 0; v <= (uint32_t)Q; ++v) {
                const uint64_t bv = __builtin_amdgcn_ballot_w64(seg_w == v);
                if (v < seg_w)
                    pos += (uint32_t)__popcll(bv);
                else if (v == seg_w)
                    pos += __builtin_amdgcn_mbcnt_hi((uint32_t)(bv >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bv, 0u));
            }
            wA[pos] = A;
            wB[pos] = B;
            wC[pos] = make_uint2(seg_w << 24, packed);
            wO[pos] = (int)nq;
            wave_lds_sync();
            nq = (uint32_t)wO[lane];               // from here on, lane = sorted position
            const uint32_t incl = wave_incl_scan(nq);
            const uint32_t excl = incl - nq;
            const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
            wC[lane].x |= excl;                    // excl < 2^24
            wave_lds_sync();
            int carry = 0;
            for (uint32_t wb = 0; wb < total; wb += 64) {
                // owner of segment wb + lane: the last record whose first
                // segment is at or before it (record indices grow with
                // position, so a prefix max over the marked starts finds it;
                // a mark holds the record's lane + 1, 0 is no mark)
                wO[lane] = 0;
                if (nq > 0 && excl >= wb && excl < wb + 64) wO[excl - wb] = lane + 1;
                wave_lds_sync();
                const int v = wave_incl_max0(wO[lane]);
                const int o = (v > 0 ? v - 1 : carry) & 63;
                carry = __builtin_amdgcn_readlane(o, 63);
                const uint32_t s = wb + (uint32_t)lane;
                if (s < total) {
                    const float4 a = wA[o];
                    const float4 b = wB[o];
                    const uint2 c = wC[o];
                    const uint32_t q = s - (c.x & 0xffffffu);
                    const int sw = (int)(c.x >> 24);                   // segment width
                    const int x0 = (int)(c.y & 255u), y0 = (int)((c.y >> 8) & 255u);
                    const int x1 = (int)((c.y >> 16) & 255u), y1 = (int)(c.y >> 24);
                    const int qpr = (x1 - x0 + Q) / Q;
                    const int pr = (int)(((float)q + 0.5f) * b.w);   // row pair
                    const int qc = (int)q - pr * qpr;
                    const int ly = y0 + 2 * pr;
                    const int lx0 = x0 + qc * sw;
                    const int nlen = min(x1 - lx0, sw - 1);            // last k
                    // rows ly and ly + 1 (the second only inside the box)
                    const float dyA = ((float)(ly + oy) + 0.5f) - a.y;
                    const float dyB = ((float)(ly + 1 + oy) + 0.5f) - a.y;
                    const float dy2A = dyA * dyA, dy2B = dyB * dyB;
                    const float R2B = ly < y1 ? a.w : -1.0f;
                    const double tqx = b.x, tqy = b.y, tqz = b.z;
                    // pixel centre of the segment's first pixel; adding k to
                    // it is exact, so dx is bit-identical to sample_weight's
                    const float cx0 = (float)(lx0 + ox) + 0.5f;
                    // the rows' LDS addresses are pinned in registers so that
                    // every pixel uses them with an immediate offset
                    lds_u64* pixA = (lds_u64*)(acc + 3 * (ly * ES + lx0));
                    lds_u64* pixB = pixA + 3 * ES;
                    asm volatile("" : "+v"(pixA));
                    asm volatile("" : "+v"(pixB));
#pragma unroll
                    for (int k = 0; k < Q; ++k) {
                        if (k > nlen) break;
                        const float dx = (cx0 + (float)k) - a.x;
                        const float d2A = fmaf(dx, dx, dy2A);
                        const float d2B = fmaf(dx, dx, dy2B);
                        if (d2A <= a.w) {
                            if constexpr (CNT) ++nsamp;
                            const double w = __builtin_amdgcn_exp2f(d2A * a.z);
                            lds_add_u64(pixA + 3 * k, term_short(tqx, w));
                            lds_add_u64(pixA + 3 * k + 1, term_short(tqy, w));
                            lds_add_u64(pixA + 3 * k + 2, term_short(tqz, w));
                        }
                        if (d2B <= R2B) {
                            if constexpr (CNT) ++nsamp;
                            const double w = __builtin_amdgcn_exp2f(d2B * a.z);
                            lds_add_u64(pixB + 3 * k, term_short(tqx, w));
                            lds_add_u64(pixB + 3 * k + 1, term_short(tqy, w));
                            lds_add_u64(pixB + 3 * k + 2, term_short(tqz, w));
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
                const long long v = acc[3 * (ly * ES + lx) + c];
                if (v == 0) continue;
                if constexpr (sizeof(Acc) == 8)
                    global_add_checked(Lg + c * plane + p, (Acc)v, F.oflag);
                else
                    AccOps<Acc>::global_add(Lg + c * plane + p, __ll2float_rn(v) * F.inv_qscale);
            }
        }
        if (ccount) {
            for (int i = tid; i < F.T * F.T; i += kSplatThreads) {
                const int gx = cx0 + (i % F.T), gy = cy0 + (i / F.T);
                if (gx > cx1 || gy > cy1) continue;
                const uint32_t c = (cnt[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
                if (c) (void)gatomic_add(ccount + (size_t)gy * F.W + gx, (int)c);
            }
        }
        __syncthreads();
    }
    if constexpr (CNT) count_samples(nsamp, stats);
}

// ---------------------------------------------------------------------------
// k_resolve: grid (blocks, n_jobs).  I = 1 - exp(-L) = -expm1(-L); optional
// L output.  (An int64 sum that left the int64 range was flagged by the
// checked addition that made it leave.)
template <typename Acc>
__global__ void k_resolve(const JobDev* __restrict__ jobs) {
    const JobDev& J = jobs[blockIdx.y];
    const int W = J.F.W, H = J.F.H;
    const size_t plane = (size_t)W * H;
    const SPLOTCH_GLOBAL Acc* __restrict__ Lg = gmem(reinterpret_cast<const Acc*>(J.L));
    SPLOTCH_GLOBAL float* __restrict__ rgb = gmem(J.rgb);
    SPLOTCH_GLOBAL float* __restrict__ logacc = J.logacc ? gmem(J.logacc) : nullptr;
    const float inv_q = J.F.inv_qscale;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x; p < plane; p += stride) {
        if (J.rmask && !region_on(J, (int)(p % (size_t)W), (int)(p / (size_t)W))) continue;
        float L[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const Acc v = Lg[c * plane + p];
            if constexpr (sizeof(Acc) == 8) {
                L[c] = __ll2float_rn((long long)v) * inv_q;
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
    }
}

}  // namespace splotch_dev
