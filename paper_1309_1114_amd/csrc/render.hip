// Host side of the MI355X particle renderer: the C ABI of include/splotch.h.
//
// A render (or a batch of renders) is planned on the host -- schedule knobs,
// workspace layout, job table -- and then runs as one fixed sequence of
// kernel launches on the caller's stream (kernels.h), without any host
// synchronisation.  A batch is captured once into a HIP graph per job-shape
// signature and replayed afterwards; only the job table is re-uploaded.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "splotch.h"
#include "kernels.h"
#include "ordered.h"
#include "sort.h"

using namespace splotch_dev;

namespace {

struct StageEvents {
    int stage;
    hipEvent_t start, stop;
};

struct Knobs {
    int T = 0, halo = 0, max_clip = 0, chunk = 0;
};

struct GraphEntry {
    std::string sig;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct splotch_ctx {
    int device = 0;
    int cu_count = 256;
    std::string arch;
    std::string err;
    unsigned long long* dstats = nullptr;  // device counters, kStatWords words
    splotch_stats last{};
    int last_accum = 0;
    bool last_sample_count = false;        // the last render counted its samples
    bool timing = false;
    int timed_renders = 0;
    std::vector<StageEvents> events;       // pending stage timings
    std::map<std::string, Knobs> tuned;    // autotuner results by job bucket
    std::vector<GraphEntry> graphs;        // captured batches
    hipStream_t capture_stream = nullptr;  // private stream the batches are captured on
    hipStream_t copy_stream = nullptr;     // host-to-device copies of streamed renders
    bool radius_stats = false;             // collect the radius statistics
    bool sample_count = false;             // count the samples drawn
};

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kMinChunk = 65536;
constexpr size_t kSplatLdsBudget = 160 * 1024;
constexpr int kMaxJobs = 64;
constexpr int kMaxGraphs = 16;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

// ---------------------------------------------------------------------------
// Fixed scratch of splotch_render_noalloc: a file-scope device array (each
// device that loads the library holds its own copy until the process ends).
// Host code never uses the array's name as an address: the device address
// is looked up once per device (scratch_setup, from splotch_ctx_create with
// that device current) and kept in g_scratch.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = SPLOTCH_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Looks up this device's copy of the scratch array (the device must be
// current).  Returns false if the runtime does not give its address.
bool scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return true;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return false;
    }
    g_scratch[device] = ptr;
    return true;
}

void* scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}

splotch_status fail(splotch_ctx* ctx, splotch_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

// The tile accumulator is 64-bit fixed point in both modes.
size_t splat_acc_bytes(int T, int halo, int /*accsize*/) {
    const int E = T + 2 * halo;
    const int ES = E | 1;
    return ((size_t)3 * E * ES * 8 + 15) & ~(size_t)15;
}

// Centre counts of a tile: 16-bit, two per 32-bit word.
size_t splat_cnt_bytes(int T) { return ((size_t)T * T * 2 + 15) & ~(size_t)15; }

// LDS of the tile splat: accumulator, staging, work-queue slot, counts.
size_t splat_lds_bytes(int T, int halo, int accsize) {
    return splat_acc_bytes(T, halo, accsize) + (size_t)kSplatThreads * kSplatStageBytes +
           kSplatStageExtra + splat_cnt_bytes(T);
}

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
// The arrays a colour mode reads are all set.
bool particle_arrays_set(const splotch_particles* parts, int colour_mode) {
    if (!parts->x || !parts->y || !parts->z || !parts->h || !parts->intensity) return false;
    if (colour_mode == SPLOTCH_COLOUR_VECTOR) return parts->vx && parts->vy && parts->vz;
    return parts->scalar != nullptr;
}

splotch_status validate(splotch_ctx* ctx, const splotch_particles* parts, const splotch_camera* cam,
                        const splotch_params* p, bool need_data) {
    if (!parts || !cam || !p) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "NULL argument");
    if (parts->n < 0) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "particles.n < 0");
    if (parts->n > ((int64_t)1 << 40))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "particles.n too large");
    if (p->colour_mode != SPLOTCH_COLOUR_PALETTE && p->colour_mode != SPLOTCH_COLOUR_VECTOR)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.colour_mode must be PALETTE or VECTOR");
    if (p->colour_mode == SPLOTCH_COLOUR_VECTOR && p->scalar_log10)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "the vector colour mode needs scalar_log10 = 0");
    if (need_data && parts->n > 0 && !particle_arrays_set(parts, p->colour_mode))
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
    if (p->transfer != SPLOTCH_TRANSFER_EQUAL && p->transfer != SPLOTCH_TRANSFER_ORDERED)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.transfer must be EQUAL or ORDERED");
    for (int k = 0; k < SPLOTCH_MAX_SPECIES; ++k)
        if (!std::isfinite(p->absorption[k]) || p->absorption[k] < 0.0f)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.absorption must be finite and >= 0");
    if (!(p->prefilter >= 0.0f && p->prefilter <= 1.0e4f))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.prefilter must be in [0, 1e4] pixels");
    return SPLOTCH_OK;
}

splotch_status validate_outputs(splotch_ctx* ctx, const splotch_colormap* cmap,
                                const splotch_image* img, int colour_mode) {
    if (colour_mode == SPLOTCH_COLOUR_PALETTE && (!cmap || cmap->n < 2 || !cmap->rgb))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "colormap needs n >= 2 entries");
    if (!img || !img->rgb) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "image.rgb is NULL");
    if (img->region_mask) {
        const int rs = img->region_size;
        if (rs < 8 || rs > 1024 || (rs & (rs - 1)) != 0)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG,
                        "image.region_size must be a power of two in 8..1024");
        if (img->center_count)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG,
                        "a region mask does not go with the centre-count output");
    }
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
    const double up[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2],
                          r[0] * f[1] - r[1] * f[0]};
    const double focal = 0.5 * cam->width / std::tan(0.5 * (double)cam->fov_deg * M_PI / 180.0);
    F = Frame{};
    F.rx = r[0]; F.ry = r[1]; F.rz = r[2];
    F.ux = up[0]; F.uy = up[1]; F.uz = up[2];
    F.fx = f[0]; F.fy = f[1]; F.fz = f[2];
    F.ex = cam->eye[0]; F.ey = cam->eye[1]; F.ez = cam->eye[2];
    F.focal = focal;
    F.halfW = 0.5f * (float)cam->width;
    F.halfH = 0.5f * (float)cam->height;
    F.z_near = cam->z_near;
    F.chi = p->chi;
    F.b0 = p->brightness[0]; F.b1 = p->brightness[1]; F.b2 = p->brightness[2]; F.b3 = p->brightness[3];
    F.a0 = p->absorption[0]; F.a1 = p->absorption[1]; F.a2 = p->absorption[2]; F.a3 = p->absorption[3];
    F.s0 = (float)((double)p->fixed_sigma_frac[0] * cam->width);
    F.s1 = (float)((double)p->fixed_sigma_frac[1] * cam->width);
    F.s2 = (float)((double)p->fixed_sigma_frac[2] * cam->width);
    F.s3 = (float)((double)p->fixed_sigma_frac[3] * cam->width);
    F.smin = p->scalar_min;
    F.sinv = (float)(1.0 / ((double)p->scalar_max - (double)p->scalar_min));
    F.slog = p->scalar_log10 ? 1 : 0;
    F.col_norm = p->col_norm ? 1 : 0;
    F.colmode = p->colour_mode == SPLOTCH_COLOUR_VECTOR ? 1 : 0;
    F.pf2 = p->prefilter * p->prefilter;
    F.W = cam->width;
    F.H = cam->height;
    // fixed-point scale of the tile partial sums (both modes) and of the
    // int64 planes; the FP32 mode uses 40 fractional bits for its partials
    const int fb = p->accum == SPLOTCH_ACCUM_INT64 ? p->frac_bits : 40;
    F.qscale = std::ldexp(1.0f, fb);
    F.inv_qscale = std::ldexp(1.0f, -fb);
    F.tau_lim = std::ldexp(1.0f, 50 - fb);
    return true;
}

// ---------------------------------------------------------------------------
// Schedule knobs and the tuned-value cache
// ---------------------------------------------------------------------------
std::string bucket_key(const splotch_particles* parts, const splotch_camera* cam,
                       const splotch_params* p) {
    const int ln = parts->n > 0 ? (int)std::floor(std::log2((double)parts->n)) : 0;
    const int lp = (int)std::floor(std::log2((double)cam->width * cam->height));
    char buf[96];
    std::snprintf(buf, sizeof buf, "a%d_n%d_p%d", p->accum, ln, lp);
    return buf;
}

int64_t tiles_for(int W, int H, int T) { return (int64_t)((W + T - 1) / T) * ((H + T - 1) / T); }

splotch_status choose_knobs(splotch_ctx* ctx, const splotch_particles* parts,
                            const splotch_camera* cam, const splotch_params* p, Knobs& k) {
    const int accsize = p->accum == SPLOTCH_ACCUM_INT64 ? 8 : 4;
    const int W = cam->width, H = cam->height;
    Knobs tuned;
    bool have_tuned = false;
    if (ctx) {
        auto it = ctx->tuned.find(bucket_key(parts, cam, p));
        if (it != ctx->tuned.end()) {
            tuned = it->second;
            have_tuned = tiles_for(W, H, tuned.T) + 1 <= kMaxBins;
        }
    }
    if (p->tile != 0) {
        if (p->tile != 8 && p->tile != 16 && p->tile != 32 && p->tile != 64)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.tile must be 0, 8, 16, 32 or 64");
        k.T = p->tile;
    } else if (have_tuned) {
        k.T = tuned.T;
    } else {
        k.T = 32;
        if (tiles_for(W, H, 32) + 1 > kMaxBins) k.T = 64;
    }
    if (tiles_for(W, H, k.T) + 1 > kMaxBins)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "image has too many tiles for this tile size");
    if (p->halo >= 0) {
        if (p->halo > k.T) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.halo must be <= tile");
        k.halo = p->halo;
        if (splat_lds_bytes(k.T, k.halo, accsize) > kSplatLdsBudget || k.T + 2 * k.halo > 255)
            return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "tile and halo do not fit in LDS");
    } else {
        // untuned: a border of 8 pixels (T/2 for small tiles), halved while
        // the accumulator does not fit (a sweep on C2 at 1080p: halo 8 and
        // clip 8 at T = 32 were best, 13.0 against 13.6 ms for halo 4, clip 4)
        k.halo = (have_tuned && p->tile == 0) ? std::min(tuned.halo, k.T) : std::min(8, k.T / 2);
        while (k.halo > 0 && splat_lds_bytes(k.T, k.halo, accsize) > kSplatLdsBudget) k.halo /= 2;
        if (splat_lds_bytes(k.T, k.halo, accsize) > kSplatLdsBudget)
            return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "tile does not fit in LDS");
    }
    if (p->max_clip_tiles != 0) {
        if (p->max_clip_tiles < 1 || p->max_clip_tiles > 64)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.max_clip_tiles must be 1..64");
        k.max_clip = p->max_clip_tiles;
    } else {
        // untuned: 8 tiles, 16 from 2^23 pixels up (footprints in tiles grow
        // with the resolution; C2 at 4096^2: 39 ms at 16 against 48 ms at 8,
        // where the large pass took 15 ms)
        k.max_clip = have_tuned ? tuned.max_clip
                                : ((int64_t)W * H >= ((int64_t)1 << 23) ? 16 : 8);
    }
    if (p->chunk != 0) {
        if (p->chunk < 32 || p->chunk > kMaxChunk)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "params.chunk must be 32..8191");
        k.chunk = p->chunk;
    } else {
        // untuned: records per tile work item grow with the particle count
        // (each item adds its whole tile accumulator to the image, so fewer,
        // longer items for big sets; at least 1024): the largest power of
        // two <= n / 16384 within [1024, 4096] (C2, 1e8 particles: 4096)
        int ch = 1024;
        while (ch < 4096 && (int64_t)ch * 2 * 16384 <= parts->n) ch *= 2;
        k.chunk = have_tuned ? tuned.chunk : ch;
    }
    return SPLOTCH_OK;
}

// ---------------------------------------------------------------------------
// Per-job plan and workspace layout
// ---------------------------------------------------------------------------
struct JobPlan {
    Knobs k;
    int W = 0, H = 0, tiles_x = 0, tiles_y = 0, n_tiles = 0, NB = 0, P = 0, nseg = 0, accsize = 4;
    int64_t n = 0, chunk_n = 0;
    size_t cap = 0, max_items = 0, acc_bytes = 0, splat_lds = 0;
    size_t sz_L = 0, sz_hist = 0, sz_seg = 0, sz_bin = 0, sz_recs = 0;
    int NG = 0, ngx = 0, lg_side = 0;   // large-pass pixel groups
    size_t cap_idx = 0, sz_lg = 0;      // large-pass index entries and arrays
    size_t sz_live = 0;                 // tile flags of a region mask
    size_t total() const { return sz_L + sz_hist + sz_seg + sz_bin + sz_recs + sz_lg + sz_live; }
};

// Pixel groups of the large pass: side 128, doubled until at most
// kMaxLargeGroups cover the image.
void large_groups(JobPlan& pl) {
    int side = kLargeGroup;
    for (;;) {
        const int64_t gx = (pl.W + side - 1) / side, gy = (pl.H + side - 1) / side;
        if (gx * gy <= kMaxLargeGroups) {
            pl.lg_side = side;
            pl.ngx = (int)gx;
            pl.NG = (int)(gx * gy);
            return;
        }
        side *= 2;
    }
}

void size_job(JobPlan& pl, int64_t chunk_n) {
    pl.chunk_n = chunk_n;
    const int64_t per_particle = std::max(1, pl.k.max_clip);
    pl.cap = (size_t)std::max<int64_t>(chunk_n, 1) * per_particle;
    // workgroups of the counting and scatter passes: at most as many as
    // fit on the chip at once for the counting pass (its LDS key histogram
    // limits it to 1..3 per CU), so that no second partial round runs
    const int64_t hist_bytes = (int64_t)pl.NB * 4 + 256;
    const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(3, kLdsBytesPerCU / hist_bytes));
    const int max_blocks = std::min(kMaxCountBlocks, per_cu * (kMaxCountBlocks / 3));
    int P = (int)std::min<int64_t>(max_blocks, (std::max<int64_t>(chunk_n, 1) + 4095) / 4096);
    P = ((std::max(P, 1) + kSeg - 1) / kSeg) * kSeg;
    pl.P = P;
    pl.nseg = P / kSeg;
    pl.max_items = (size_t)pl.n_tiles + pl.cap / pl.k.chunk + 2;
    pl.sz_L = align_up((size_t)3 * pl.W * pl.H * pl.accsize);
    pl.sz_hist = align_up((size_t)pl.P * pl.NB * 4);
    pl.sz_seg = align_up((size_t)pl.nseg * pl.NB * 4);
    pl.sz_bin = align_up((size_t)(pl.NB + 1) * 4);
    pl.sz_recs = align_up(pl.cap * sizeof(Rec));
    // one index entry per record slot: a large record touching several
    // groups uses several, the many small ones none; overflow falls back
    large_groups(pl);
    pl.cap_idx = pl.cap;
    pl.sz_live = align_up((size_t)pl.n_tiles);
    pl.sz_lg = align_up((size_t)pl.NG * 4) + 2 * align_up((size_t)(pl.NG + 1) * 4) +
               align_up(pl.cap_idx * 4);
}

splotch_status plan_job(splotch_ctx* ctx, const splotch_particles* parts, const splotch_camera* cam,
                        const splotch_params* p, JobPlan& pl) {
    Knobs k;
    splotch_status s = choose_knobs(ctx, parts, cam, p, k);
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
    pl.acc_bytes = splat_acc_bytes(k.T, k.halo, pl.accsize);
    pl.splat_lds = splat_lds_bytes(k.T, k.halo, pl.accsize);
    // records are addressed with 32-bit offsets
    const int64_t max_chunk = ((int64_t)1 << 31) / std::max(1, k.max_clip);
    size_job(pl, std::min<int64_t>(std::max<int64_t>(parts->n, 1), max_chunk));
    return SPLOTCH_OK;
}

// Batch layout: [JobDev x n | ctrl | items | per-job regions ...]
struct BatchLayout {
    size_t off_jobs = 0, off_ctrl = 0, off_items = 0, total = 0;
    size_t items_cap = 0;
    std::vector<size_t> off_job;   // start of each job's regions
};

BatchLayout layout_batch(const std::vector<JobPlan>& plans) {
    BatchLayout b;
    size_t off = 0;
    b.off_jobs = off;
    off = align_up(off + plans.size() * sizeof(JobDev));
    b.off_ctrl = off;
    off = align_up(off + kCtrlWords * sizeof(uint32_t));
    b.items_cap = 0;
    for (const JobPlan& p : plans) b.items_cap += p.max_items;
    b.off_items = off;
    off = align_up(off + b.items_cap * sizeof(int4));
    for (const JobPlan& p : plans) {
        b.off_job.push_back(off);
        off += p.total();
    }
    b.total = off;
    return b;
}

// Particle range of one pass of a job.
void set_pass(JobDev& J, const JobPlan& pl, const splotch_particles* parts, int64_t p0, int64_t cn) {
    J.pp = PartPtrs{parts->x, parts->y, parts->z, parts->h, parts->intensity, parts->scalar,
                    parts->species, parts->vx, parts->vy, parts->vz};
    if (cn > 0) {
        J.pp.x += p0; J.pp.y += p0; J.pp.z += p0; J.pp.h += p0;
        J.pp.inten += p0;
        if (J.pp.scalar) J.pp.scalar += p0;
        if (J.pp.species) J.pp.species += p0;
        if (J.pp.vx) { J.pp.vx += p0; J.pp.vy += p0; J.pp.vz += p0; }
    }
    J.n = cn;
    J.per_block = std::max<int64_t>(1, (cn + pl.P - 1) / pl.P);
}

// Device view of one job: pointers into the workspace, whole particle set.
JobDev make_jobdev(const JobPlan& pl, const Frame& F0, const splotch_particles* parts,
                   const splotch_colormap* cmap, const splotch_image* img, unsigned char* ws,
                   size_t off, unsigned int* oflag, uint32_t item0) {
    JobDev J{};
    J.F = F0;
    J.F.T = pl.k.T;
    J.F.Tshift = 0;
    while ((1 << J.F.Tshift) < pl.k.T) ++J.F.Tshift;
    J.F.tiles_x = pl.tiles_x;
    J.F.tiles_y = pl.tiles_y;
    J.F.n_tiles = pl.n_tiles;
    J.F.halo = pl.k.halo;
    J.F.max_clip = pl.k.max_clip;
    // the vector colour mode reads no palette
    J.F.ncmap = F0.colmode ? 2 : cmap->n;
    J.F.oflag = oflag;
    set_pass(J, pl, parts, 0, parts->n);
    J.cmap = F0.colmode ? nullptr : cmap->rgb;
    unsigned char* p = ws + off;
    J.L = p;
    p += pl.sz_L;
    J.hist = reinterpret_cast<uint32_t*>(p);
    p += pl.sz_hist;
    J.seg = reinterpret_cast<uint32_t*>(p);
    p += pl.sz_seg;
    J.bin = reinterpret_cast<uint32_t*>(p);
    p += pl.sz_bin;
    J.recs = reinterpret_cast<Rec*>(p);
    p += pl.sz_recs;
    J.lg_cnt = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)pl.NG * 4);
    J.lg_start = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)(pl.NG + 1) * 4);
    J.lg_chunk = reinterpret_cast<uint32_t*>(p);
    p += align_up((size_t)(pl.NG + 1) * 4);
    J.lg_idx = reinterpret_cast<uint32_t*>(p);
    p += align_up(pl.cap_idx * 4);
    J.tlive = p;
    J.cap_idx = (uint32_t)pl.cap_idx;
    J.NG = pl.NG;
    J.ngx = pl.ngx;
    J.lg_side = pl.lg_side;
    J.rgb = img->rgb;
    J.logacc = img->log_accum;
    J.ccount = img->center_count;
    J.rmask = img->region_mask;
    J.rshift = 0;
    J.rgx = 0;
    if (img->region_mask) {
        while ((1 << J.rshift) < img->region_size) ++J.rshift;
        J.rgx = (pl.W + img->region_size - 1) / img->region_size;
    }
    J.cap = (uint32_t)pl.cap;
    J.max_items = (uint32_t)pl.max_items;
    J.NB = pl.NB;
    J.P = pl.P;
    J.nseg = pl.nseg;
    J.item0 = item0;
    J.chunk = pl.k.chunk;
    return J;
}

// Brackets a stage's launches with events on the stream when timing is on.
// Names of the render stages in roctx ranges (rocprofv3 --marker-trace).
const char* const kStageNames[SPLOTCH_NUM_STAGES] = {
    "splotch clear", "splotch count", "splotch scan", "splotch scatter",
    "splotch items", "splotch large", "splotch splat", "splotch resolve"};

// One render stage: a roctx range around its launches (host side, always),
// and, with stage timing on, events around its GPU work.
struct StageTimer {
    splotch_ctx* ctx;
    hipStream_t st;
    StageEvents cur{};
    bool on;
    StageTimer(splotch_ctx* c, hipStream_t s, int stage, bool enabled)
        : ctx(c), st(s), on(enabled && c->timing) {
        roctxRangePushA(kStageNames[stage]);
        if (!on) return;
        cur.stage = stage;
        if (hipEventCreate(&cur.start) != hipSuccess || hipEventCreate(&cur.stop) != hipSuccess) {
            on = false;
            return;
        }
        (void)hipEventRecord(cur.start, st);
    }
    ~StageTimer() {
        roctxRangePop();
        if (!on) return;
        (void)hipEventRecord(cur.stop, st);
        ctx->events.push_back(cur);
    }
};

struct LaunchShape {
    int n_jobs = 0;
    int P_max = 0, NB_max = 0, nseg_max = 0;
    int max_pix_blocks = 0, clear_blocks = 0;
    size_t hist_lds = 0, splat_lds = 0, stage_off = 0;
    size_t cnt_off = 0;                 // splat LDS: the centre counts
    bool masked = false;                // some job draws only marked regions
    uint32_t items_cap = 0;
};

LaunchShape launch_shape(const std::vector<JobPlan>& plans, const BatchLayout& bl,
                         bool masked = false) {
    LaunchShape s;
    s.n_jobs = (int)plans.size();
    s.masked = masked;
    size_t max_pix = 0, cnt = 0;
    for (const JobPlan& p : plans) {
        s.P_max = std::max(s.P_max, p.P);
        s.NB_max = std::max(s.NB_max, p.NB);
        s.nseg_max = std::max(s.nseg_max, p.nseg);
        s.stage_off = std::max(s.stage_off, p.acc_bytes);
        cnt = std::max(cnt, splat_cnt_bytes(p.k.T));
        max_pix = std::max(max_pix, (size_t)p.W * p.H);
    }
    // counting and scattering passes: the key histogram (cursors), then the
    // tile flags of a region mask
    // the tile flags of a region mask follow the key words only when some
    // job has a mask
    s.hist_lds = (size_t)s.NB_max * 4 + (masked ? (((size_t)s.NB_max + 3) & ~(size_t)3) : 0);
    s.cnt_off = s.stage_off + (size_t)kSplatThreads * kSplatStageBytes + kSplatStageExtra;
    s.splat_lds = s.cnt_off + cnt;
    s.max_pix_blocks = (int)std::min<size_t>(4096, (max_pix + 255) / 256);
    s.clear_blocks = (int)std::min<size_t>(2048, (max_pix * 3 * 8 / 16 + 255) / 256 + 1);
    s.items_cap = (uint32_t)bl.items_cap;
    return s;
}

// The per-pass kernels (count .. splat).  `timed` adds stage events.
template <typename Acc>
void launch_pass(splotch_ctx* ctx, const LaunchShape& s, JobDev* djobs, int4* items,
                 uint32_t* ctrl, hipStream_t st, bool timed) {
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_COUNT, timed);
        if (s.masked)
            k_tile_live<<<dim3((s.NB_max + 255) / 256, s.n_jobs), 256, 0, st>>>(djobs);
        if (ctx->radius_stats)
            k_count<true><<<dim3(s.P_max, s.n_jobs), kCountThreads, s.hist_lds, st>>>(djobs,
                                                                                    ctx->dstats);
        else
            k_count<false><<<dim3(s.P_max, s.n_jobs), kCountThreads, s.hist_lds, st>>>(djobs,
                                                                                     ctx->dstats);
    }
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_SCAN, timed);
        const dim3 sg((s.NB_max + 255) / 256, s.nseg_max, s.n_jobs);
        k_segsum<<<sg, 256, 0, st>>>(djobs);
        k_binscan<<<s.n_jobs, 1024, 0, st>>>(djobs);
        k_offsets<<<sg, 256, 0, st>>>(djobs);
    }
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_SCATTER, timed);
        k_scatter<<<dim3(s.P_max, s.n_jobs), kCountThreads, s.hist_lds, st>>>(djobs, ctx->dstats);
    }
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_ITEMS, timed);
        k_items<<<1, 1024, 0, st>>>(djobs, s.n_jobs, items, s.items_cap, ctrl, ctx->dstats);
    }
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_LARGE, timed);
        k_lgcount<<<dim3(kLgBlocks, s.n_jobs), 256, 0, st>>>(djobs);
        k_lgscan<<<1, 1024, 0, st>>>(djobs, s.n_jobs, ctrl);
        k_lgscatter<<<dim3(kLgBlocks, s.n_jobs), 256, 0, st>>>(djobs);
        if (ctx->sample_count)
            k_large<Acc, true><<<ctx->cu_count * 4, kLargeThreads, 0, st>>>(djobs, s.n_jobs, ctrl,
                                                                            ctx->dstats);
        else
            k_large<Acc, false><<<ctx->cu_count * 4, kLargeThreads, 0, st>>>(djobs, s.n_jobs, ctrl,
                                                                             ctx->dstats);
    }
    {
        StageTimer tm(ctx, st, SPLOTCH_STAGE_SPLAT, timed);
        if (ctx->sample_count)
            k_splat<Acc, kSplatQ, true><<<ctx->cu_count * 4, kSplatThreads, s.splat_lds, st>>>(
                djobs, items, ctrl, (int)s.stage_off, (int)s.cnt_off, ctx->dstats);
        else
            k_splat<Acc, kSplatQ, false><<<ctx->cu_count * 4, kSplatThreads, s.splat_lds, st>>>(
                djobs, items, ctrl, (int)s.stage_off, (int)s.cnt_off, ctx->dstats);
    }
}

template <typename Acc>
void launch_clear(splotch_ctx* ctx, const LaunchShape& s, JobDev* djobs, hipStream_t st, bool timed,
                  bool clear_stats = true) {
    StageTimer tm(ctx, st, SPLOTCH_STAGE_CLEAR, timed);
    k_clear<Acc><<<dim3(s.clear_blocks, s.n_jobs), 256, 0, st>>>(djobs, ctx->dstats,
                                                                 clear_stats ? 1 : 0);
}

template <typename Acc>
void launch_resolve(splotch_ctx* ctx, const LaunchShape& s, JobDev* djobs, hipStream_t st,
                    bool timed) {
    StageTimer tm(ctx, st, SPLOTCH_STAGE_RESOLVE, timed);
    k_resolve<Acc><<<dim3(s.max_pix_blocks, s.n_jobs), 256, 0, st>>>(djobs);
}

// Writes one job's table entry from a kernel argument (the allocation-free
// render's upload: no host staging, nothing but a launch on the stream).
static_assert(sizeof(JobDev) <= 2048, "a job table entry travels as one kernel argument");
__global__ void k_put_job(JobDev* __restrict__ dst, JobDev job) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = job;
}

splotch_status upload_jobs(splotch_ctx* ctx, JobDev* djobs, const std::vector<JobDev>& jobs,
                           hipStream_t st, bool by_kernel = false) {
    if (by_kernel) {
        for (size_t j = 0; j < jobs.size(); ++j) k_put_job<<<1, 64, 0, st>>>(djobs + j, jobs[j]);
        if (hipGetLastError() != hipSuccess)
            return fail(ctx, SPLOTCH_ERR_HIP, "job table upload failed");
        return SPLOTCH_OK;
    }
    // pageable source: the runtime stages it before returning, so the host
    // vector may be reused immediately
    if (hipMemcpyAsync(djobs, jobs.data(), jobs.size() * sizeof(JobDev), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "job table upload failed");
    return SPLOTCH_OK;
}

void record_last(splotch_ctx* ctx, const std::vector<JobPlan>& plans, int passes, int accum) {
    ctx->last = splotch_stats{};
    int64_t n = 0;
    for (const JobPlan& p : plans) n += p.n;
    ctx->last.n_input = n;
    ctx->last.passes = passes;
    ctx->last.tile = plans[0].k.T;
    ctx->last.halo = plans[0].k.halo;
    ctx->last.max_clip_tiles = plans[0].k.max_clip;
    ctx->last.chunk = plans[0].k.chunk;
    ctx->last_accum = accum;
    ctx->last_sample_count = ctx->sample_count;
}

// Eager single render, possibly in several particle chunks (L is additive).
// noalloc: the job table is written by a kernel and no stage events are
// created (the allocation-free entry point).
template <typename Acc>
splotch_status render_eager(splotch_ctx* ctx, const JobPlan& pl, const Frame& F,
                            const splotch_particles* parts, const splotch_colormap* cmap,
                            const splotch_image* img, unsigned char* ws, hipStream_t st,
                            bool noalloc = false, bool clear_stats = true,
                            int* passes_out = nullptr) {
    const std::vector<JobPlan> plans{pl};
    const BatchLayout bl = layout_batch(plans);
    const LaunchShape s = launch_shape(plans, bl, img->region_mask != nullptr);
    JobDev* djobs = reinterpret_cast<JobDev*>(ws + bl.off_jobs);
    uint32_t* ctrl = reinterpret_cast<uint32_t*>(ws + bl.off_ctrl);
    int4* items = reinterpret_cast<int4*>(ws + bl.off_items);
    std::vector<JobDev> jobs{make_jobdev(pl, F, parts, cmap, img, ws, bl.off_job[0],
                                         reinterpret_cast<unsigned int*>(ctx->dstats + ST_OVERFLOW),
                                         0u)};
    const bool timed = !noalloc;
    splotch_status rc = upload_jobs(ctx, djobs, jobs, st, noalloc);
    if (rc != SPLOTCH_OK) return rc;
    launch_clear<Acc>(ctx, s, djobs, st, timed, clear_stats);
    int passes = 0;
    for (int64_t p0 = 0; p0 < pl.n; p0 += pl.chunk_n) {
        const int64_t cn = std::min(pl.chunk_n, pl.n - p0);
        set_pass(jobs[0], pl, parts, p0, cn);
        rc = upload_jobs(ctx, djobs, jobs, st, noalloc);
        if (rc != SPLOTCH_OK) return rc;
        launch_pass<Acc>(ctx, s, djobs, items, ctrl, st, timed);
        ++passes;
    }
    launch_resolve<Acc>(ctx, s, djobs, st, timed);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    if (ctx->timing && timed) ctx->timed_renders++;
    if (passes_out) *passes_out = passes;
    else record_last(ctx, plans, passes, sizeof(Acc) == 8 ? SPLOTCH_ACCUM_INT64 : SPLOTCH_ACCUM_FP32);
    return SPLOTCH_OK;
}

// Everything a captured launch sequence depends on besides the job table:
// launch shapes, workspace address and size, and the kernel variants chosen
// on the host (accumulation type, radius statistics).
std::string batch_signature(const LaunchShape& s, const BatchLayout& bl, const void* ws,
                            int accum, bool radius_stats, bool sample_count) {
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "j%d_m%d_a%d_r%d_n%d_P%d_B%d_S%d_x%d_c%d_L%zu_O%zu_C%zu_I%u_T%zu_w%p",
                  s.n_jobs, s.masked ? 1 : 0, accum, radius_stats ? 1 : 0, sample_count ? 1 : 0,
                  s.P_max,
                  s.NB_max, s.nseg_max, s.max_pix_blocks, s.clear_blocks, s.splat_lds, s.stage_off,
                  s.cnt_off, s.items_cap, bl.total, ws);
    return buf;
}

// Batched render: one graph per signature, replayed after a fresh upload of
// the job table (the table carries every pointer and size the kernels use).
template <typename Acc>
splotch_status render_batch(splotch_ctx* ctx, const std::vector<JobPlan>& plans,
                            const std::vector<JobDev>& jobs, const BatchLayout& bl,
                            unsigned char* ws, hipStream_t st, bool clear_stats = true,
                            bool record = true) {
    bool masked = false;
    for (const JobDev& J : jobs) masked = masked || J.rmask != nullptr;
    const LaunchShape s = launch_shape(plans, bl, masked);
    JobDev* djobs = reinterpret_cast<JobDev*>(ws + bl.off_jobs);
    uint32_t* ctrl = reinterpret_cast<uint32_t*>(ws + bl.off_ctrl);
    int4* items = reinterpret_cast<int4*>(ws + bl.off_items);
    splotch_status rc = upload_jobs(ctx, djobs, jobs, st);
    if (rc != SPLOTCH_OK) return rc;
    const std::string sig = batch_signature(s, bl, ws, sizeof(Acc) == 8 ? 1 : 0, ctx->radius_stats,
                                            ctx->sample_count) +
                            (clear_stats ? "_z1" : "_z0");
    GraphEntry* ge = nullptr;
    for (GraphEntry& g : ctx->graphs)
        if (g.sig == sig) ge = &g;
    if (!ge) {
        if ((int)ctx->graphs.size() >= kMaxGraphs) {
            (void)hipGraphExecDestroy(ctx->graphs.front().exec);
            (void)hipGraphDestroy(ctx->graphs.front().graph);
            ctx->graphs.erase(ctx->graphs.begin());
        }
        GraphEntry g;
        g.sig = sig;
        // capture on the context's own stream (a default stream cannot be
        // captured); the graph is then launched on the caller's stream
        hipStream_t cs = ctx->capture_stream;
        if (!cs || hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, SPLOTCH_ERR_HIP, "graph capture could not start");
        }
        launch_clear<Acc>(ctx, s, djobs, cs, false, clear_stats);
        launch_pass<Acc>(ctx, s, djobs, items, ctrl, cs, false);
        launch_resolve<Acc>(ctx, s, djobs, cs, false);
        hipError_t e = hipStreamEndCapture(cs, &g.graph);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, SPLOTCH_ERR_HIP, "graph capture failed");
        }
        e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g.graph);
            return fail(ctx, SPLOTCH_ERR_HIP, "graph instantiation failed");
        }
        ctx->graphs.push_back(g);
        ge = &ctx->graphs.back();
    }
    if (hipGraphLaunch(ge->exec, st) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "graph launch failed");
    if (record)
        record_last(ctx, plans, 1, sizeof(Acc) == 8 ? SPLOTCH_ACCUM_INT64 : SPLOTCH_ACCUM_FP32);
    return SPLOTCH_OK;
}

bool g_attrs_set[64] = {false};

void set_kernel_attrs(int device) {
    if (device < 0 || device >= 64 || g_attrs_set[device]) return;
    const int big = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_count<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_count<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_scatter),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<float, kSplatQ, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<long long, kSplatQ, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<float, kSplatQ, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_splat<long long, kSplatQ, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, big);
    (void)hipGetLastError();
    g_attrs_set[device] = true;
}

// Validation and planning of a single render; shrinks the particle chunk
// when the workspace is smaller than a one-pass render needs.
splotch_status prepare_single(splotch_ctx* ctx, const splotch_particles* parts,
                              const splotch_camera* cam, const splotch_colormap* cmap,
                              const splotch_params* params, const splotch_image* img,
                              void* workspace, size_t workspace_bytes, JobPlan& pl, Frame& F) {
    splotch_status s = validate(ctx, parts, cam, params, true);
    if (s != SPLOTCH_OK) return s;
    s = validate_outputs(ctx, cmap, img, params->colour_mode);
    if (s != SPLOTCH_OK) return s;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    if (!make_frame(cam, params, F))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "degenerate camera (eye == target or up parallel)");
    s = plan_job(ctx, parts, cam, params, pl);
    if (s != SPLOTCH_OK) return s;
    std::vector<JobPlan> plans{pl};
    if (layout_batch(plans).total > workspace_bytes) {
        JobPlan probe = pl;
        size_job(probe, kMinChunk);
        plans[0] = probe;
        if (layout_batch(plans).total > workspace_bytes)
            return fail(ctx, SPLOTCH_ERR_WORKSPACE, "workspace smaller than the minimum for this image");
        int64_t lo = kMinChunk, hi = pl.chunk_n;
        while (hi - lo > 1024) {
            const int64_t mid = lo + (hi - lo) / 2;
            size_job(probe, mid);
            plans[0] = probe;
            if (layout_batch(plans).total <= workspace_bytes) lo = mid; else hi = mid;
        }
        size_job(pl, lo);
    }
    return SPLOTCH_OK;
}

splotch_status plan_batch(splotch_ctx* ctx, const splotch_job* jobs, int32_t n_jobs,
                          std::vector<JobPlan>& plans, std::vector<Frame>& frames, bool need_data) {
    if (!jobs || n_jobs < 1 || n_jobs > kMaxJobs)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "n_jobs must be 1..64 with a job array");
    plans.assign(n_jobs, JobPlan{});
    frames.assign(n_jobs, Frame{});
    for (int j = 0; j < n_jobs; ++j) {
        const splotch_job& J = jobs[j];
        splotch_status s = validate(ctx, &J.particles, &J.camera, &J.params, need_data);
        if (s != SPLOTCH_OK) return s;
        if (J.params.transfer != SPLOTCH_TRANSFER_EQUAL)
            return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "batched renders use the E = A transfer");
        if (need_data) {
            s = validate_outputs(ctx, &J.colormap, &J.image, J.params.colour_mode);
            if (s != SPLOTCH_OK) return s;
        }
        if (J.params.accum != jobs[0].params.accum)
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "all jobs of a batch need the same accum mode");
        if (!make_frame(&J.camera, &J.params, frames[j]))
            return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "degenerate camera in a job");
        s = plan_job(ctx, &J.particles, &J.camera, &J.params, plans[j]);
        if (s != SPLOTCH_OK) return s;
        if (plans[j].chunk_n < J.particles.n)
            return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "a batch job exceeds the 32-bit record space");
    }
    return SPLOTCH_OK;
}

// Streamed render: particles stay in host memory; chunks are copied into
// two device staging buffers on the context's copy stream while the render
// stream draws the previous chunk (L is additive, so the passes just add).
struct StreamLayout {
    BatchLayout bl;
    size_t stage_bytes = 0;        // one staging buffer
    size_t off_stage[2] = {0, 0};
    size_t off_tables = 0;         // four job tables: buffer 0/1, full/last chunk
    size_t total = 0;
};

// float arrays staged per chunk: x, y, z, h, intensity and the colour
// input (the scalar, or the three vector components)
int staged_floats(bool vec) { return vec ? 8 : 6; }

StreamLayout layout_stream(const JobPlan& pl, int64_t chunk, bool species, bool vec) {
    StreamLayout L;
    L.bl = layout_batch({pl});
    L.stage_bytes = staged_floats(vec) * align_up((size_t)chunk * 4) +
                    (species ? align_up((size_t)chunk) : 0);
    size_t off = L.bl.total;
    L.off_stage[0] = off;
    off += L.stage_bytes;
    L.off_stage[1] = off;
    off += L.stage_bytes;
    L.off_tables = off;
    off += 4 * align_up(sizeof(JobDev));
    L.total = off;
    return L;
}

splotch_particles stage_particles(unsigned char* base, int64_t chunk, bool species, bool vec) {
    splotch_particles sp{};
    const size_t a = align_up((size_t)chunk * 4);
    const int nf = staged_floats(vec);
    float* f[8];
    for (int k = 0; k < nf; ++k) f[k] = reinterpret_cast<float*>(base + k * a);
    sp.x = f[0]; sp.y = f[1]; sp.z = f[2]; sp.h = f[3]; sp.intensity = f[4];
    if (vec) {
        sp.vx = f[5]; sp.vy = f[6]; sp.vz = f[7];
    } else {
        sp.scalar = f[5];
    }
    sp.species = species ? base + nf * a : nullptr;
    sp.n = chunk;
    return sp;
}

splotch_status plan_stream(splotch_ctx* ctx, const splotch_particles* hp, const splotch_camera* cam,
                           const splotch_params* params, int64_t chunk, JobPlan& pl,
                           int64_t& ch) {
    splotch_status s = validate(ctx, hp, cam, params, false);
    if (s != SPLOTCH_OK) return s;
    if (params->transfer != SPLOTCH_TRANSFER_EQUAL)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "streamed renders use the E = A transfer");
    if (chunk < 1) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "chunk must be >= 1");
    ch = std::min<int64_t>(chunk, std::max<int64_t>(hp->n, 1));
    splotch_particles one = *hp;
    one.n = ch;
    s = plan_job(ctx, &one, cam, params, pl);
    if (s != SPLOTCH_OK) return s;
    if (pl.chunk_n < ch)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "chunk exceeds the 32-bit record space");
    return SPLOTCH_OK;
}

template <typename Acc>
splotch_status render_streamed(splotch_ctx* ctx, const JobPlan& pl, const Frame& F,
                               const splotch_particles* hp, int64_t ch,
                               const splotch_colormap* cmap, const splotch_image* img,
                               unsigned char* ws, const StreamLayout& L, hipStream_t st) {
    const bool species = hp->species != nullptr;
    const bool vec = F.colmode != 0;
    const std::vector<JobPlan> plans{pl};
    const LaunchShape s = launch_shape(plans, L.bl, img->region_mask != nullptr);
    uint32_t* ctrl = reinterpret_cast<uint32_t*>(ws + L.bl.off_ctrl);
    int4* items = reinterpret_cast<int4*>(ws + L.bl.off_items);
    const int64_t n = hp->n;
    const int64_t last = n > 0 ? n - (n - 1) / ch * ch : 0;
    // tables[2b + t]: staging buffer b, t = 0 full chunk, t = 1 last chunk
    JobDev* tables[4];
    std::vector<JobDev> host(4);
    for (int b = 0; b < 2; ++b) {
        const splotch_particles sp = stage_particles(ws + L.off_stage[b], ch, species, vec);
        for (int t = 0; t < 2; ++t) {
            JobDev J = make_jobdev(pl, F, &sp, cmap, img, ws, L.bl.off_job[0],
                                   reinterpret_cast<unsigned int*>(ctx->dstats + ST_OVERFLOW), 0u);
            set_pass(J, pl, &sp, 0, t == 0 ? ch : last);
            host[2 * b + t] = J;
            tables[2 * b + t] = reinterpret_cast<JobDev*>(ws + L.off_tables +
                                                          (2 * b + t) * align_up(sizeof(JobDev)));
        }
    }
    for (int k = 0; k < 4; ++k) {
        std::vector<JobDev> one{host[k]};
        splotch_status rc = upload_jobs(ctx, tables[k], one, st);
        if (rc != SPLOTCH_OK) return rc;
    }
    if (!ctx->copy_stream &&
        hipStreamCreateWithFlags(&ctx->copy_stream, hipStreamNonBlocking) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "copy stream creation failed");
    hipEvent_t copied[2], done[2], start;
    for (int b = 0; b < 2; ++b) {
        if (hipEventCreateWithFlags(&copied[b], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&done[b], hipEventDisableTiming) != hipSuccess)
            return fail(ctx, SPLOTCH_ERR_HIP, "event creation failed");
    }
    if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, "event creation failed");
    // the staging buffers may still be read by earlier work on the caller's stream
    (void)hipEventRecord(start, st);
    (void)hipStreamWaitEvent(ctx->copy_stream, start, 0);
    launch_clear<Acc>(ctx, s, tables[0], st, true);
    const int64_t nchunks = n > 0 ? (n + ch - 1) / ch : 0;
    bool ok = true;
    for (int64_t c = 0; c < nchunks && ok; ++c) {
        const int b = (int)(c & 1);
        const int64_t p0 = c * ch, cn = std::min(ch, n - p0);
        if (c >= 2) ok &= hipStreamWaitEvent(ctx->copy_stream, done[b], 0) == hipSuccess;
        const splotch_particles sp = stage_particles(ws + L.off_stage[b], ch, species, vec);
        const float* src[8] = {hp->x, hp->y, hp->z, hp->h, hp->intensity,
                               vec ? hp->vx : hp->scalar, hp->vy, hp->vz};
        const float* dst[8] = {sp.x, sp.y, sp.z, sp.h, sp.intensity,
                               vec ? sp.vx : sp.scalar, sp.vy, sp.vz};
        for (int k = 0; k < staged_floats(vec) && ok; ++k)
            ok &= hipMemcpyAsync(const_cast<float*>(dst[k]), src[k] + p0, (size_t)cn * 4,
                                 hipMemcpyHostToDevice, ctx->copy_stream) == hipSuccess;
        if (species && ok)
            ok &= hipMemcpyAsync(const_cast<uint8_t*>(sp.species), hp->species + p0, (size_t)cn,
                                 hipMemcpyHostToDevice, ctx->copy_stream) == hipSuccess;
        ok &= hipEventRecord(copied[b], ctx->copy_stream) == hipSuccess;
        ok &= hipStreamWaitEvent(st, copied[b], 0) == hipSuccess;
        launch_pass<Acc>(ctx, s, tables[2 * b + (cn == ch ? 0 : 1)], items, ctrl, st, true);
        ok &= hipEventRecord(done[b], st) == hipSuccess;
    }
    launch_resolve<Acc>(ctx, s, tables[0], st, true);
    for (int b = 0; b < 2; ++b) {
        (void)hipEventDestroy(copied[b]);
        (void)hipEventDestroy(done[b]);
    }
    (void)hipEventDestroy(start);
    const hipError_t e = hipGetLastError();
    if (!ok || e != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, std::string("streamed render failed: ") +
                                              hipGetErrorString(e));
    if (ctx->timing) ctx->timed_renders++;
    JobPlan rec = pl;
    rec.n = n;
    record_last(ctx, {rec}, (int)nchunks, sizeof(Acc) == 8 ? SPLOTCH_ACCUM_INT64 : SPLOTCH_ACCUM_FP32);
    return SPLOTCH_OK;
}


// ---------------------------------------------------------------------------
// Ordered render (E != A): depth sort, per-tile entry lists in depth order,
// front-to-back compositing per pixel.  The particles are cut into passes
// of consecutive depth ranks whose tile entries fit the entry buffers; the
// pixel state (I, T, absorption depth) carries over from pass to pass.
// ---------------------------------------------------------------------------
struct OrdLayout {
    int64_t n = 0;
    uint64_t cap = 0;            // tile entries per pass
    int tiles_x = 0, tiles_y = 0, tile_bits = 1;
    size_t recs = 0, keys0 = 0, keys1 = 0, idx0 = 0, idx1 = 0, box_p = 0, cnt_r = 0, prefix = 0;
    size_t ek0 = 0, ek1 = 0, ev0 = 0, ev1 = 0, I = 0, T = 0, S = 0, ctrl = 0, temp = 0;
    size_t tile_lo = 0, item_n = 0, item_off = 0, partI = 0, partT = 0, partS = 0;
    uint64_t max_items = 0;     // composite work items of a full pass
    size_t temp_bytes = 0, total = 0;
};

constexpr uint64_t kOrdMinCap = 4096;   // smallest entry capacity of a pass

// cap = 0: the default capacity, 3n + tiles entries within [2^20, 2^30]
// (a clustered 1e8-particle frame at 1080p has about 2.3 entries per
// particle at 16-pixel tiles).
OrdLayout layout_ordered(int64_t n, int W, int H, uint64_t cap = 0) {
    OrdLayout L;
    L.n = n;
    L.tiles_x = (W + kOrdT - 1) / kOrdT;
    L.tiles_y = (H + kOrdT - 1) / kOrdT;
    const int64_t nt = (int64_t)L.tiles_x * L.tiles_y;
    while (((int64_t)1 << L.tile_bits) < nt) ++L.tile_bits;
    L.cap = cap ? cap
                : (uint64_t)std::min<int64_t>(std::max<int64_t>(3 * n + nt, (int64_t)1 << 20),
                                              (int64_t)1 << 30);
    const size_t plane = (size_t)W * H;
    size_t off = 0;
    auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return o; };
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    L.recs = take(nn * sizeof(OrdRec));
    L.keys0 = take(nn * 8);
    L.keys1 = take(nn * 8);
    L.idx0 = take(nn * 4);
    L.idx1 = take(nn * 4);
    L.box_p = take(nn * 8);
    L.cnt_r = take((nn + 1) * 8);
    L.prefix = take((nn + 1) * 8);
    L.ek0 = take(L.cap * 4);
    L.ek1 = take(L.cap * 4);
    L.ev0 = take(L.cap * 4);
    L.ev1 = take(L.cap * 4);
    L.I = take(3 * plane * 8);
    L.T = take(3 * plane * 8);
    L.S = take(3 * plane * 4);
    L.tile_lo = take(((size_t)nt + 1) * 4);
    L.item_n = take(((size_t)nt + 1) * 8);
    L.item_off = take(((size_t)nt + 1) * 8);
    L.max_items = L.cap / kOrdChunk + 1 + (uint64_t)nt;
    const size_t part = (size_t)L.max_items * 3 * kOrdThreads;
    L.partI = take(part * 8);
    L.partT = take(part * 8);
    L.partS = take(part * 4);
    L.ctrl = take(256);
    L.temp_bytes = splotch_sort::temp_bytes(std::max<size_t>(nn + 1, L.cap));
    L.temp = take(L.temp_bytes);
    L.total = off;
    return L;
}

constexpr int64_t kOrdMaxN = (int64_t)1 << 31;   // particle indices are 32-bit

splotch_status check_ordered(splotch_ctx* ctx, const splotch_particles* parts,
                             const splotch_params* params) {
    if (params->accum != SPLOTCH_ACCUM_FP32)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED,
                    "the ordered transfer composites in FP32 (deterministic without int64)");
    if (parts->n > kOrdMaxN)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "the ordered transfer takes at most 2^31 particles");
    return SPLOTCH_OK;
}

splotch_status render_ordered(splotch_ctx* ctx, const splotch_particles* parts,
                              const splotch_camera* cam, const splotch_colormap* cmap,
                              const splotch_params* params, const splotch_image* img,
                              void* workspace, size_t workspace_bytes, hipStream_t st) {
    splotch_status s = validate(ctx, parts, cam, params, true);
    if (s != SPLOTCH_OK) return s;
    s = validate_outputs(ctx, cmap, img, params->colour_mode);
    if (s != SPLOTCH_OK) return s;
    s = check_ordered(ctx, parts, params);
    if (s != SPLOTCH_OK) return s;
    if (img->region_mask)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "the ordered transfer draws whole images");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    Frame F;
    if (!make_frame(cam, params, F)) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "degenerate camera");
    F.ncmap = F.colmode ? 2 : cmap->n;
    const int64_t n = parts->n;
    // a smaller workspace holds fewer tile entries per pass: more passes,
    // the same image
    OrdLayout L = layout_ordered(n, cam->width, cam->height);
    while (workspace_bytes < L.total && L.cap > kOrdMinCap)
        L = layout_ordered(n, cam->width, cam->height, std::max(kOrdMinCap, L.cap / 2));
    if (workspace_bytes < L.total)
        return fail(ctx, SPLOTCH_ERR_WORKSPACE, "workspace smaller than the ordered render needs");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    auto at = [&](size_t off) { return ws + off; };
    OrdJob J{};
    J.F = F;
    J.pp = PartPtrs{parts->x, parts->y, parts->z, parts->h, parts->intensity, parts->scalar,
                    parts->species, parts->vx, parts->vy, parts->vz};
    J.n = n;
    J.cmap = F.colmode ? nullptr : cmap->rgb;
    J.recs = reinterpret_cast<OrdRec*>(at(L.recs));
    J.keys = reinterpret_cast<uint64_t*>(at(L.keys0));
    J.idx = reinterpret_cast<uint32_t*>(at(L.idx0));
    J.box_p = reinterpret_cast<uint64_t*>(at(L.box_p));
    J.cnt_r = reinterpret_cast<uint64_t*>(at(L.cnt_r));
    J.prefix = reinterpret_cast<uint64_t*>(at(L.prefix));
    J.rgb = img->rgb;
    J.I = reinterpret_cast<double*>(at(L.I));
    J.T = reinterpret_cast<double*>(at(L.T));
    J.S = reinterpret_cast<float*>(at(L.S));
    J.logacc = img->log_accum;
    J.ccount = img->center_count;
    J.stats = ctx->dstats;
    J.tile_lo = reinterpret_cast<uint32_t*>(at(L.tile_lo));
    J.item_n = reinterpret_cast<uint64_t*>(at(L.item_n));
    J.item_off = reinterpret_cast<uint64_t*>(at(L.item_off));
    J.partI = reinterpret_cast<double*>(at(L.partI));
    J.partT = reinterpret_cast<double*>(at(L.partT));
    J.partS = reinterpret_cast<float*>(at(L.partS));
    uint64_t* keys1 = reinterpret_cast<uint64_t*>(at(L.keys1));
    J.box_r = keys1;   // the sorted depth keys are not read after the sort
    uint32_t* idx1 = reinterpret_cast<uint32_t*>(at(L.idx1));
    uint32_t* ek0 = reinterpret_cast<uint32_t*>(at(L.ek0));
    uint32_t* ek1 = reinterpret_cast<uint32_t*>(at(L.ek1));
    uint32_t* ev0 = reinterpret_cast<uint32_t*>(at(L.ev0));
    uint32_t* ev1 = reinterpret_cast<uint32_t*>(at(L.ev1));
    uint64_t* dctrl = reinterpret_cast<uint64_t*>(at(L.ctrl));
    void* temp = at(L.temp);
    const size_t plane = (size_t)cam->width * cam->height;
    const int init_blocks = (int)std::min<size_t>(4096, (3 * plane + 255) / 256);
    const int n_tiles = L.tiles_x * L.tiles_y;
    int passes = 0;
    bool ok = true;
    k_ord_init<<<init_blocks, 256, 0, st>>>(J);
    if (n > 0) {
        k_ord_project<<<kOrdGrid, 256, 0, st>>>(J);
        // particles by (depth, index); the 32-bit sort keys live in the
        // buffer that later holds the boxes in rank order, the dropped key
        // bits in the rank counts (both written after the sort)
        uint32_t* k32 = reinterpret_cast<uint32_t*>(keys1);
        uint32_t* lo = reinterpret_cast<uint32_t*>(J.cnt_r);
        splotch_sort::sort_by_key64(temp, J.keys, k32, k32 + n, J.idx, idx1, lo, lo + n,
                                    (size_t)n, st);
        k_ord_rank_counts<<<kOrdGrid, 256, 0, st>>>(J, J.idx);
        splotch_sort::exclusive_sum64(temp, J.cnt_r, J.prefix, (size_t)n + 1, st);
        // the entry total decides the number of passes: the one value the
        // call reads back (each pass then finds its slice on the device)
        uint64_t total = 0;
        if (hipMemcpyAsync(&total, J.prefix + n, sizeof total, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            ok = false;
        const uint64_t npass = ok ? (total + L.cap - 1) / L.cap : 0;
        // an upper bound of a pass's work items: sum of ceil(e_t / chunk) <=
        // cap / chunk + tiles
        const uint64_t grid = L.cap / kOrdChunk + 1 + (uint64_t)n_tiles;
        const int item_blocks = (int)std::min<int64_t>(kOrdGrid, (n_tiles + 1 + 255) / 256);
        for (uint64_t k = 0; k < npass; ++k) {
            k_ord_pass_bounds<<<1, 1, 0, st>>>(J.prefix, n, k, L.cap, dctrl);
            k_ord_emit<<<kOrdGrid, 256, 0, st>>>(J, J.idx, dctrl, ek0, ev0);
            // entries by tile, stable: each tile keeps depth order
            const int sb = splotch_sort::pairs32(temp, ek0, ek1, ev0, ev1, (size_t)L.cap,
                                                 dctrl + 1, L.tile_bits, st);
            const uint32_t* ekey = sb ? ek1 : ek0;
            const uint32_t* eval = sb ? ev1 : ev0;
            k_ord_items<<<item_blocks, 256, 0, st>>>(J, ekey, dctrl, (uint32_t)n_tiles);
            splotch_sort::exclusive_sum64(temp, J.item_n, J.item_off, (size_t)n_tiles + 1, st);
            if (J.logacc)
                k_ord_composite<true><<<(unsigned)grid, kOrdThreads, 0, st>>>(J, eval, (uint32_t)n_tiles);
            else
                k_ord_composite<false><<<(unsigned)grid, kOrdThreads, 0, st>>>(J, eval, (uint32_t)n_tiles);
            k_ord_merge<<<n_tiles, kOrdThreads, 0, st>>>(J, (uint32_t)n_tiles);
            ++passes;
        }
    }
    k_ord_finish<<<init_blocks, 256, 0, st>>>(J);
    const hipError_t e = hipGetLastError();
    if (!ok || e != hipSuccess)
        return fail(ctx, SPLOTCH_ERR_HIP, std::string("ordered render failed: ") +
                                              hipGetErrorString(e));
    ctx->last = splotch_stats{};
    ctx->last.n_input = n;
    ctx->last.passes = passes;
    ctx->last.tile = kOrdT;
    ctx->last_accum = SPLOTCH_ACCUM_FP32;
    ctx->last_sample_count = false;
    return SPLOTCH_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// the C ABI is the library's only exported interface (built with
// -fvisibility=hidden)
#pragma GCC visibility push(default)
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
    p->colour_mode = SPLOTCH_COLOUR_PALETTE;
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
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        if (prop.multiProcessorCount > 0) ctx->cu_count = prop.multiProcessorCount;
        ctx->arch = prop.gcnArchName;
    }
    if (hipMalloc(reinterpret_cast<void**>(&ctx->dstats), kStatWords * sizeof(unsigned long long)) !=
        hipSuccess) {
        delete ctx;
        return SPLOTCH_ERR_HIP;
    }
    (void)hipMemset(ctx->dstats, 0, kStatWords * sizeof(unsigned long long));
    if (hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(ctx->dstats);
        delete ctx;
        return SPLOTCH_ERR_HIP;
    }
    set_kernel_attrs(device);
    // the allocation-free render's scratch address on this device (a failure
    // only disables that entry point, which then reports it)
    (void)scratch_setup(device);
    *out = ctx;
    return SPLOTCH_OK;
}

splotch_status splotch_ctx_destroy(splotch_ctx* ctx) {
    if (!ctx) return SPLOTCH_OK;
    (void)hipSetDevice(ctx->device);
    for (StageEvents& e : ctx->events) {
        (void)hipEventDestroy(e.start);
        (void)hipEventDestroy(e.stop);
    }
    for (GraphEntry& g : ctx->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    if (ctx->copy_stream) (void)hipStreamDestroy(ctx->copy_stream);
    if (ctx->dstats) (void)hipFree(ctx->dstats);
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
    if (params->transfer == SPLOTCH_TRANSFER_ORDERED) {
        s = check_ordered(ctx, parts, params);
        if (s != SPLOTCH_OK) return s;
        *bytes = layout_ordered(parts->n, cam->width, cam->height).total;
        return SPLOTCH_OK;
    }
    JobPlan pl;
    s = plan_job(ctx, parts, cam, params, pl);
    if (s != SPLOTCH_OK) return s;
    *bytes = layout_batch(std::vector<JobPlan>{pl}).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render(splotch_ctx* ctx, const splotch_particles* parts,
                              const splotch_camera* cam, const splotch_colormap* cmap,
                              const splotch_params* params, const splotch_image* img,
                              void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    if (params && params->transfer == SPLOTCH_TRANSFER_ORDERED)
        return render_ordered(ctx, parts, cam, cmap, params, img, workspace, workspace_bytes,
                              reinterpret_cast<hipStream_t>(hip_stream));
    JobPlan pl;
    Frame F;
    splotch_status s = prepare_single(ctx, parts, cam, cmap, params, img, workspace,
                                      workspace_bytes, pl, F);
    if (s != SPLOTCH_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    if (params->accum == SPLOTCH_ACCUM_INT64)
        return render_eager<long long>(ctx, pl, F, parts, cmap, img, ws, st);
    return render_eager<float>(ctx, pl, F, parts, cmap, img, ws, st);
}

splotch_status splotch_render_noalloc(splotch_ctx* ctx, const splotch_particles* parts,
                                      const splotch_camera* cam, const splotch_colormap* cmap,
                                      const splotch_params* params, const splotch_image* img,
                                      void* hip_stream) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    if (params && params->transfer == SPLOTCH_TRANSFER_ORDERED)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED,
                    "splotch_render_noalloc draws the emission = absorption transfer only");
    unsigned char* ws = reinterpret_cast<unsigned char*>(scratch_ptr(ctx->device));
    if (!ws)
        return fail(ctx, SPLOTCH_ERR_HIP, "the fixed scratch of this device has no address");
    JobPlan pl;
    Frame F;
    splotch_status s = prepare_single(ctx, parts, cam, cmap, params, img, ws, kScratchBytes, pl, F);
    if (s == SPLOTCH_ERR_WORKSPACE)
        return fail(ctx, s, "this image needs more than the 512 MiB fixed scratch");
    if (s != SPLOTCH_OK) return s;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (params->accum == SPLOTCH_ACCUM_INT64)
        return render_eager<long long>(ctx, pl, F, parts, cmap, img, ws, st, true);
    return render_eager<float>(ctx, pl, F, parts, cmap, img, ws, st, true);
}

splotch_status splotch_render_stream_workspace_size(splotch_ctx* ctx,
                                                   const splotch_particles* host_particles,
                                                   const splotch_camera* cam,
                                                   const splotch_params* params, int64_t chunk,
                                                   size_t* bytes) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!bytes) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "bytes is NULL");
    JobPlan pl;
    int64_t ch = 0;
    splotch_status s = plan_stream(ctx, host_particles, cam, params, chunk, pl, ch);
    if (s != SPLOTCH_OK) return s;
    *bytes = layout_stream(pl, ch, host_particles->species != nullptr,
                                     params->colour_mode == SPLOTCH_COLOUR_VECTOR).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render_streamed(splotch_ctx* ctx, const splotch_particles* host_particles,
                                       const splotch_camera* cam, const splotch_colormap* cmap,
                                       const splotch_params* params, const splotch_image* img,
                                       int64_t chunk, void* workspace, size_t workspace_bytes,
                                       void* hip_stream) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    JobPlan pl;
    int64_t ch = 0;
    splotch_status s = plan_stream(ctx, host_particles, cam, params, chunk, pl, ch);
    if (s != SPLOTCH_OK) return s;
    s = validate_outputs(ctx, cmap, img, params->colour_mode);
    if (s != SPLOTCH_OK) return s;
    if (host_particles->n > 0 && !particle_arrays_set(host_particles, params->colour_mode))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "particle arrays must be non-NULL");
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    const StreamLayout L = layout_stream(pl, ch, host_particles->species != nullptr,
                                     params->colour_mode == SPLOTCH_COLOUR_VECTOR);
    if (L.total > workspace_bytes)
        return fail(ctx, SPLOTCH_ERR_WORKSPACE, "workspace smaller than the streamed render needs");
    Frame F;
    if (!make_frame(cam, params, F))
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "degenerate camera (eye == target or up parallel)");
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    if (params->accum == SPLOTCH_ACCUM_INT64)
        return render_streamed<long long>(ctx, pl, F, host_particles, ch, cmap, img, ws, L, st);
    return render_streamed<float>(ctx, pl, F, host_particles, ch, cmap, img, ws, L, st);
}

splotch_status splotch_batch_workspace_size(splotch_ctx* ctx, const splotch_job* jobs,
                                            int32_t n_jobs, size_t* bytes) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!bytes) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "bytes is NULL");
    std::vector<JobPlan> plans;
    std::vector<Frame> frames;
    splotch_status s = plan_batch(ctx, jobs, n_jobs, plans, frames, false);
    if (s != SPLOTCH_OK) return s;
    *bytes = layout_batch(plans).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render_batched(splotch_ctx* ctx, const splotch_job* jobs, int32_t n_jobs,
                                      void* workspace, size_t workspace_bytes, void* hip_stream) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    std::vector<JobPlan> plans;
    std::vector<Frame> frames;
    splotch_status s = plan_batch(ctx, jobs, n_jobs, plans, frames, true);
    if (s != SPLOTCH_OK) return s;
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & (kAlign - 1)) != 0)
        return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    // Jobs are drawn in consecutive groups that fit the workspace (the whole
    // batch when it fits); a job that does not fit alone is drawn in particle
    // chunks, as a single render with that workspace is.  Each job's image is
    // the same whatever the grouping.  Every group is planned before any
    // launch.
    struct Group { int j0, j1; bool chunked; JobPlan pl; };
    std::vector<Group> groups;
    for (int i = 0; i < n_jobs;) {
        int j = i + 1;
        auto fits = [&](int a, int b) {
            return layout_batch(std::vector<JobPlan>(plans.begin() + a, plans.begin() + b)).total <=
                   workspace_bytes;
        };
        if (fits(i, j)) {
            while (j < n_jobs && fits(i, j + 1)) ++j;
            groups.push_back({i, j, false, JobPlan{}});
        } else {
            JobPlan pl = plans[i];
            size_job(pl, kMinChunk);
            if (layout_batch(std::vector<JobPlan>{pl}).total > workspace_bytes)
                return fail(ctx, SPLOTCH_ERR_WORKSPACE,
                            "workspace smaller than the minimum for a job of the batch");
            int64_t lo = kMinChunk, hi = plans[i].chunk_n;
            while (hi - lo > 1024) {
                const int64_t mid = lo + (hi - lo) / 2;
                size_job(pl, mid);
                if (layout_batch(std::vector<JobPlan>{pl}).total <= workspace_bytes) lo = mid;
                else hi = mid;
            }
            size_job(pl, lo);
            groups.push_back({i, j, true, pl});
        }
        i = j;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* ws = reinterpret_cast<unsigned char*>(workspace);
    const bool i64 = jobs[0].params.accum == SPLOTCH_ACCUM_INT64;
    int passes = 0;
    for (size_t g = 0; g < groups.size(); ++g) {
        const Group& G = groups[g];
        const bool first = g == 0;
        splotch_status rc;
        if (G.chunked) {
            const int j = G.j0;
            int np = 0;
            rc = i64 ? render_eager<long long>(ctx, G.pl, frames[j], &jobs[j].particles,
                                               &jobs[j].colormap, &jobs[j].image, ws, st, false,
                                               first, &np)
                     : render_eager<float>(ctx, G.pl, frames[j], &jobs[j].particles,
                                           &jobs[j].colormap, &jobs[j].image, ws, st, false,
                                           first, &np);
            passes += np;
        } else {
            const std::vector<JobPlan> sub(plans.begin() + G.j0, plans.begin() + G.j1);
            const BatchLayout bl = layout_batch(sub);
            std::vector<JobDev> dev(sub.size());
            uint32_t item0 = 0;
            for (int j = G.j0; j < G.j1; ++j) {
                dev[j - G.j0] = make_jobdev(plans[j], frames[j], &jobs[j].particles,
                                            &jobs[j].colormap, &jobs[j].image, ws,
                                            bl.off_job[j - G.j0],
                                            reinterpret_cast<unsigned int*>(ctx->dstats + ST_OVERFLOW),
                                            item0);
                item0 += (uint32_t)plans[j].max_items;
            }
            rc = i64 ? render_batch<long long>(ctx, sub, dev, bl, ws, st, first, false)
                     : render_batch<float>(ctx, sub, dev, bl, ws, st, first, false);
            passes += 1;
        }
        if (rc != SPLOTCH_OK) return rc;
    }
    record_last(ctx, plans, passes, i64 ? SPLOTCH_ACCUM_INT64 : SPLOTCH_ACCUM_FP32);
    return SPLOTCH_OK;
}

splotch_status splotch_set_radius_stats(splotch_ctx* ctx, int32_t enable) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->radius_stats = enable != 0;
    return SPLOTCH_OK;
}

splotch_status splotch_set_sample_count(splotch_ctx* ctx, int32_t enable) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->sample_count = enable != 0;
    return SPLOTCH_OK;
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
    for (int k = 0; k < 5; ++k) out->radius_hist[k] = (int64_t)h[ST_RHIST + k];
    double rsum;
    std::memcpy(&rsum, &h[ST_RSUM], sizeof rsum);
    out->radius_mean = h[ST_ACTIVE] ? rsum / (double)h[ST_ACTIVE] : 0.0;
    out->n_samples = ctx->last_sample_count ? (int64_t)h[ST_SAMPLES] : -1;
    if (h[ST_BADSLOT])
        return fail(ctx, SPLOTCH_ERR_HIP, "internal error: record counts of the two passes differ");
    if (out->overflow)
        return fail(ctx, SPLOTCH_ERR_OVERFLOW, "fixed-point accumulator overflowed");
    return SPLOTCH_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times candidate schedules of one job on the caller's stream and
// remembers the fastest for the job's size bucket.
// ---------------------------------------------------------------------------
splotch_status splotch_autotune(splotch_ctx* ctx, const splotch_job* job, void* workspace,
                                size_t workspace_bytes, void* hip_stream, splotch_params* best,
                                float* best_ms) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    ctx->err.clear();
    if (!job || !best) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "NULL argument");
    if (job->params.transfer != SPLOTCH_TRANSFER_EQUAL)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "the ordered transfer has no tuned knobs");
    const std::string key = bucket_key(&job->particles, &job->camera, &job->params);
    hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "hipSetDevice failed");
    const bool saved_timing = ctx->timing;
    ctx->timing = false;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(ctx, SPLOTCH_ERR_HIP, "event creation failed");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SPLOTCH_ERR_HIP, "event creation failed");
    }
    float best_t = 1e30f;
    splotch_params bp = job->params;
    bool any = false;
    const int tiles[] = {16, 32, 64};
    const int halos[] = {0, 4, 8};
    const int clips[] = {8, 16};
    const int chunks[] = {1024, 4096, kMaxChunk};
    ctx->tuned.erase(key);
    for (int T : tiles)
        for (int hl : halos)
            for (int mc : clips)
                for (int ch : chunks) {
                    if (hl > T / 2) continue;
                    splotch_params p = job->params;
                    p.tile = T;
                    p.halo = hl;
                    p.max_clip_tiles = mc;
                    p.chunk = ch;
                    JobPlan pl;
                    Frame F;
                    // candidates that need more than one pass, or do not fit, are skipped
                    if (prepare_single(ctx, &job->particles, &job->camera, &job->colormap, &p,
                                       &job->image, workspace, workspace_bytes, pl, F) != SPLOTCH_OK)
                        continue;
                    if (pl.chunk_n < job->particles.n) continue;
                    float tsum = 0.0f;
                    bool ok = true;
                    for (int rep = 0; rep < 3 && ok; ++rep) {
                        if (rep > 0) (void)hipEventRecord(e0, st);
                        ok = splotch_render(ctx, &job->particles, &job->camera, &job->colormap, &p,
                                            &job->image, workspace, workspace_bytes, hip_stream) ==
                             SPLOTCH_OK;
                        if (rep > 0 && ok) {
                            (void)hipEventRecord(e1, st);
                            float t = 0.0f;
                            if (hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&t, e0, e1) != hipSuccess)
                                ok = false;
                            tsum += t;
                        }
                    }
                    if (!ok) continue;
                    any = true;
                    if (tsum / 2.0f < best_t) {
                        best_t = tsum / 2.0f;
                        bp = p;
                    }
                }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->timing = saved_timing;
    if (!any) return fail(ctx, SPLOTCH_ERR_WORKSPACE, "no candidate schedule fits the workspace");
    Knobs k;
    k.T = bp.tile;
    k.halo = bp.halo;
    k.max_clip = bp.max_clip_tiles;
    k.chunk = bp.chunk;
    ctx->tuned[key] = k;
    *best = bp;
    if (best_ms) *best_ms = best_t;
    return SPLOTCH_OK;
}

splotch_status splotch_tune_save(splotch_ctx* ctx, const char* path) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!path) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "path is NULL");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "cannot open tune cache for writing");
    std::fprintf(f, "{\"device\": \"%s\", \"buckets\": {", ctx->arch.c_str());
    bool first = true;
    for (const auto& kv : ctx->tuned) {
        std::fprintf(f, "%s\n  \"%s\": {\"tile\": %d, \"halo\": %d, \"max_clip_tiles\": %d, \"chunk\": %d}",
                     first ? "" : ",", kv.first.c_str(), kv.second.T, kv.second.halo,
                     kv.second.max_clip, kv.second.chunk);
        first = false;
    }
    std::fprintf(f, "\n}}\n");
    std::fclose(f);
    return SPLOTCH_OK;
}

splotch_status splotch_tune_load(splotch_ctx* ctx, const char* path) {
    if (!ctx) return SPLOTCH_ERR_INVALID_ARG;
    if (!path) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "path is NULL");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(ctx, SPLOTCH_ERR_INVALID_ARG, "cannot open tune cache");
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    const std::string dev_tag = "\"device\": \"" + ctx->arch + "\"";
    if (text.find(dev_tag) == std::string::npos)
        return fail(ctx, SPLOTCH_ERR_UNSUPPORTED, "tune cache was made on another device");
    size_t pos = text.find("\"buckets\"");
    int loaded = 0;
    while (pos != std::string::npos && (pos = text.find("\"a", pos + 1)) != std::string::npos) {
        const size_t end = text.find('"', pos + 1);
        if (end == std::string::npos) break;
        const std::string key = text.substr(pos + 1, end - pos - 1);
        Knobs k;
        if (std::sscanf(text.c_str() + end,
                        "\": {\"tile\": %d, \"halo\": %d, \"max_clip_tiles\": %d, \"chunk\": %d}",
                        &k.T, &k.halo, &k.max_clip, &k.chunk) == 4 &&
            (k.T == 8 || k.T == 16 || k.T == 32 || k.T == 64) && k.halo >= 0 && k.halo <= k.T &&
            k.max_clip >= 1 && k.max_clip <= 64 && k.chunk >= 32 && k.chunk <= kMaxChunk) {
            ctx->tuned[key] = k;
            ++loaded;
        }
        pos = end;
    }
    return loaded > 0 ? SPLOTCH_OK : fail(ctx, SPLOTCH_ERR_INVALID_ARG, "no entries in tune cache");
}

}  // extern "C"
#pragma GCC visibility pop
