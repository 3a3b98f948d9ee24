/*
 * splotch.h -- C ABI of the MI355X particle renderer.
 *
 * The library renders particles the way Splotch does (Rivi et al.,
 * "GPU Accelerated Particle Visualization with Splotch"): each particle is
 * roto-translated and projected by the camera together with its smoothing
 * length (Section "Splotch Overview", processing stage; Eq. 7), coloured
 * through a palette (same section, last paragraph), and its Gaussian
 * (Eq. 2), clipped at chi*sigma, is added along every pixel ray.  With
 * emission equal to absorption the radiative-transfer equation (Eq. 1) is
 * independent of the particle order, so the library accumulates the optical
 * depth L per pixel and colour and resolves I = 1 - exp(-L) at the end.
 * With independent emission and absorption (splotch_params.transfer) the
 * particles are composited per pixel in depth order instead.
 *
 * Conventions shared by every entry point:
 *  - All buffer pointers are DEVICE pointers (hipMalloc or torch CUDA
 *    memory on the context's device) unless a comment says otherwise.
 *  - The caller owns every buffer and keeps it alive until the work queued
 *    on the given stream has finished.  The library never frees or retains
 *    caller pointers after a call returns.
 *  - Entry points that take a stream queue work on it and return without
 *    synchronising (except splotch_get_stats, and splotch_render with the
 *    ordered transfer, which synchronises once to read its entry count).  `hip_stream` is a hipStream_t
 *    passed as void*; NULL means the default stream.
 *  - Errors are returned, never thrown.  Argument checks happen before any
 *    work is queued; on failure nothing is launched and outputs are left
 *    untouched.  splotch_last_error() then describes the failure.
 *  - One context per host thread (and per stream).
 */
#ifndef SPLOTCH_H
#define SPLOTCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SPLOTCH_ABI_VERSION 7
#define SPLOTCH_MAX_SPECIES 4

typedef int32_t splotch_status;
#define SPLOTCH_OK 0
#define SPLOTCH_ERR_INVALID_ARG (-1)
#define SPLOTCH_ERR_WORKSPACE (-2)
#define SPLOTCH_ERR_HIP (-3)
#define SPLOTCH_ERR_OVERFLOW (-4)
#define SPLOTCH_ERR_UNSUPPORTED (-5)

#define SPLOTCH_ACCUM_FP32 0
#define SPLOTCH_ACCUM_INT64 1

/* Colour modes (splotch_params.colour_mode). */
#define SPLOTCH_COLOUR_PALETTE 0
#define SPLOTCH_COLOUR_VECTOR 1

/* Radiative transfer (splotch_params.transfer). */
#define SPLOTCH_TRANSFER_EQUAL 0
#define SPLOTCH_TRANSFER_ORDERED 1

typedef struct splotch_ctx splotch_ctx;

/*
 * Particles, structure of arrays, n entries each (float32 device arrays).
 * x, y, z: world position.  h: smoothing length (the sigma of Eq. 2, world
 * units).  intensity: per-particle factor of the optical depth.  scalar:
 * the property mapped through the palette (e.g. density or temperature);
 * not read (may be NULL) in the vector colour mode.
 * species: optional uint8 array (NULL means every particle is species 0);
 * values above SPLOTCH_MAX_SPECIES-1 are read as SPLOTCH_MAX_SPECIES-1.
 * vx, vy, vz: the three components of a vector quantity (e.g. velocity)
 * that give the red, green and blue colour in the vector colour mode
 * (Section "Splotch Overview", colour by vector); NULL in the palette mode.
 */
typedef struct {
    int64_t n;
    const float* x;
    const float* y;
    const float* z;
    const float* h;
    const float* intensity;
    const float* scalar;
    const uint8_t* species;
    const float* vx;
    const float* vy;
    const float* vz;
} splotch_particles;

/*
 * Pinhole camera (host struct).  forward = (target-eye)/|target-eye|,
 * right = forward x up (normalised), up' = right x forward.  fov_deg is
 * the HORIZONTAL field of view, 0 < fov_deg < 180; the focal length in
 * pixels is (width/2)/tan(fov/2) on both axes.  Particles with depth
 * (forward . (x - eye)) <= z_near are not drawn; z_near > 0.
 * Pixel (i, j) is column i, row j counted from the TOP; its centre is at
 * screen position (i + 1/2, j + 1/2).
 */
typedef struct {
    float eye[3];
    float target[3];
    float up[3];
    float fov_deg;
    float z_near;
    int32_t width;
    int32_t height;
} splotch_camera;

/* Palette: n >= 2 entries of RGB float32 (device array of 3*n floats).
 * A normalised scalar s in [0,1] maps to u = s (n-1), m = min(floor u, n-2),
 * colour = (1 - (u-m)) rgb[m] + (u-m) rgb[m+1]. */
typedef struct {
    int32_t n;
    const float* rgb;
} splotch_colormap;

/*
 * Render parameters (host struct).  Fill with splotch_default_params().
 *
 * chi               clip radius in units of sigma (Eq. 2), > 0.  Default 3.
 *                   The clip is a step: a pixel centre within float
 *                   rounding of a disk's rim (|d^2 - R^2| about 1e-6 R^2)
 *                   may be taken on one side by the float arithmetic and
 *                   on the other by exact arithmetic, and that one sample
 *                   weighs tau0 exp(-chi^2).  The FP32 image therefore
 *                   agrees with exact arithmetic to 1e-5 where
 *                   tau0 exp(-chi^2) stays below that (chi = 3: 1.2e-4
 *                   tau0); at small chi and random positions, isolated
 *                   rim pixels can differ by up to tau0 exp(-chi^2).
 * brightness[k]     optical-depth scale of species k (the E = A coefficient
 *                   is brightness * palette colour).
 * fixed_sigma_frac  > 0: species k is drawn with a fixed screen sigma of
 *                   fixed_sigma_frac[k] * width pixels instead of f h / depth.
 * scalar_min/max    normalisation bounds of the scalar (min/max
 *                   normalisation, Section "CUDA Implementation" footnote);
 *                   scalar_log10 != 0 normalises log10(scalar) instead.
 * col_norm          0: peak optical depth = brightness * intensity * colour.
 *                   1: additionally times sqrt(pi) * h (the column of a 3-D
 *                   Gaussian of unit central density).
 * accum             SPLOTCH_ACCUM_FP32 (default) or SPLOTCH_ACCUM_INT64:
 *                   every term is quantised to round(tau * 2^frac_bits) and
 *                   summed in int64, which makes the image bit-exact for any
 *                   schedule, tile size and class threshold.  Every addition
 *                   into a pixel sum is checked: a term of magnitude 2^62 or
 *                   more, or a sum that leaves the int64 range at any point
 *                   (terms of either sign), sets the overflow flag.
 * frac_bits         fractional bits of the int64 mode, 8..56.  Default 40.
 * tile, halo, max_clip_tiles, chunk
 *                   schedule knobs; they never change the image (int64 mode:
 *                   bit-for-bit).  0 (or -1 for halo) picks tuned values.
 *                   tile: screen tile side in pixels (8, 16, 32 or 64).
 *                   halo: extra border (pixels, 0..tile) of a tile's local
 *                   accumulator; a particle whose footprint fits in the
 *                   bordered tile around its centre is drawn there once.
 *                   max_clip_tiles: a larger footprint touching at most this
 *                   many tiles is drawn tile by tile; beyond that it goes to
 *                   the cooperative large-particle pass.  1..64.
 *                   chunk: records per work item of the tile pass,
 *                   32..8191 (an item sums at most one term below 2^50 per
 *                   record and pixel in 64-bit words, so its sums cannot
 *                   overflow).
 * colour_mode       SPLOTCH_COLOUR_PALETTE (default): colour = palette of
 *                   the normalised scalar.  SPLOTCH_COLOUR_VECTOR: colour
 *                   channel c = clamp((v_c - scalar_min)/(scalar_max -
 *                   scalar_min), 0, 1) of the particle's vector (vx, vy,
 *                   vz); the palette is not read (the colormap argument may
 *                   be NULL) and scalar_log10 must be 0.
 * transfer          SPLOTCH_TRANSFER_EQUAL (default): emission equal to
 *                   absorption (Eq. 1 is order-free; I = 1 - exp(-L)).
 *                   SPLOTCH_TRANSFER_ORDERED: independent coefficients,
 *                   E = brightness[k] * intensity * colour and
 *                   A = absorption[k] * intensity * colour (each times
 *                   sqrt(pi) h with col_norm).  Every particle is a slab at
 *                   its camera depth; along each pixel ray the slabs are
 *                   crossed from the far end toward the eye, I -> I exp(-A w)
 *                   + E w (1 - exp(-A w))/(A w), w = exp(-d^2/sigma^2); equal
 *                   depths are ordered by particle index.  FP32 only (the
 *                   result is deterministic), at most 2^31 particles,
 *                   splotch_render only (batched, streamed and autotune
 *                   calls return SPLOTCH_ERR_UNSUPPORTED).  log_accum, when
 *                   given, receives the absorption depth sum A w.  The
 *                   depth-ordered list of (tile, particle) entries is drawn
 *                   in passes of consecutive entries that fit the workspace
 *                   (a workspace below the queried size shortens the
 *                   passes, down to 4096 entries; a particle's entries may
 *                   run over several passes; the image is bit-identical
 *                   from run to run and equal to rounding across pass
 *                   counts).  The call reads back one value, the entry
 *                   count, so it synchronises its stream once; every
 *                   check happens before any launch.
 * absorption[k]     absorption scale of species k (>= 0; read by the ordered
 *                   transfer only).
 * prefilter         >= 0, pixels.  0 (default): the pixel rays sample the
 *                   particles' Gaussians as they are.  s > 0: the optical
 *                   depth is first convolved with the normalised Gaussian
 *                   exp(-d^2/s^2)/(pi s^2) of the screen plane, so that each
 *                   pixel centre samples a smoothed image (an anti-aliased
 *                   render at a coarse resolution).  A Gaussian convolved
 *                   with a Gaussian is a Gaussian: every particle is drawn
 *                   with sigma' = sqrt(sigma^2 + s^2) and its coefficients
 *                   (E, A, or E = A) scaled by sigma^2 / sigma'^2, which
 *                   keeps its integrated optical depth; the clip is at
 *                   chi * sigma'.
 */
typedef struct {
    float chi;
    float brightness[SPLOTCH_MAX_SPECIES];
    float fixed_sigma_frac[SPLOTCH_MAX_SPECIES];
    float scalar_min;
    float scalar_max;
    int32_t scalar_log10;
    int32_t col_norm;
    int32_t accum;
    int32_t frac_bits;
    int32_t tile;
    int32_t halo;
    int32_t max_clip_tiles;
    int32_t chunk;
    int32_t colour_mode;
    int32_t transfer;
    float absorption[SPLOTCH_MAX_SPECIES];
    float prefilter;
} splotch_params;

/*
 * Outputs (device arrays, row-major, row 0 at the top, RGB interleaved).
 * rgb:          height*width*3 float32, I = 1 - exp(-L), required.
 * log_accum:    optional height*width*3 float32, the optical depth L.
 * center_count: optional height*width int32, number of particles in front of
 *               the camera whose projected centre falls inside the pixel.
 * region_mask:  optional, one byte per square region of region_size pixels
 *               (a power of two, 8..1024), row-major over
 *               ceil(width/region_size) x ceil(height/region_size) regions.
 *               When given, only the pixels of regions whose byte is
 *               nonzero are drawn and written (rgb and log_accum there equal
 *               the unmasked render's; bit for bit in int64 mode); every
 *               other pixel of the outputs is left as it was, and tiles
 *               outside the marked regions are skipped.  Not with
 *               center_count or the ordered transfer.  NULL: every pixel.
 * Every provided output is fully overwritten (only the marked regions with a
 * region_mask).
 */
typedef struct {
    float* rgb;
    float* log_accum;
    int32_t* center_count;
    const uint8_t* region_mask;
    int32_t region_size;
} splotch_image;

/* Counters of the last render on a context (see splotch_get_stats). */
typedef struct {
    int64_t n_input;      /* particles given */
    int64_t n_active;     /* in front of the camera with a footprint box that
                             meets the image */
    int64_t n_entries;    /* (tile, particle) work entries, all classes */
    int64_t n_large;      /* particles sent to the cooperative large pass */
    int64_t n_items;      /* tile work items executed */
    int32_t overflow;     /* int64 mode: 1 if a pixel overflowed */
    int32_t passes;       /* particle chunks (1 unless the workspace was small) */
    int32_t tile, halo, max_clip_tiles, chunk;   /* the schedule used */
    /* Only when enabled with splotch_set_radius_stats (zero otherwise):
     * active particles by screen radius r = chi * sigma in pixels (the
     * radius of Eq. 7): r <= 2, 2 < r <= 4, 4 < r <= 8, 8 < r <= 16, r > 16
     * (the bins of the paper's zoom tests, Section "Speed-up"), and their
     * mean radius R0 = <r>. */
    int64_t radius_hist[5];
    double radius_mean;
    /* Only when enabled with splotch_set_sample_count (-1 otherwise): the
     * number of (particle, pixel centre) samples with d^2 <= R^2 drawn by
     * the render, i.e. the beta R0^2 work term of Eq. 6, as the kernels
     * decided them. */
    int64_t n_samples;
} splotch_stats;

/* Human-readable name of a status code (static string). */
const char* splotch_status_string(splotch_status status);

/* SPLOTCH_ABI_VERSION of the loaded library. */
int32_t splotch_abi_version(void);

/* Fill *params with the defaults: chi 3, brightness 1, no fixed sigma,
 * scalar range [0,1] linear, col_norm 0, FP32, frac_bits 40, tuned knobs.
 * Returns SPLOTCH_ERR_INVALID_ARG if params is NULL. */
splotch_status splotch_default_params(splotch_params* params);

/* Create a context on HIP device `device` (>= 0).  The context holds a few
 * hundred bytes of device memory for counters and never allocates large
 * buffers.  *out is set to NULL on failure. */
splotch_status splotch_ctx_create(splotch_ctx** out, int32_t device);

/* Destroy a context (NULL is accepted).  Work queued with it must be done. */
splotch_status splotch_ctx_destroy(splotch_ctx* ctx);

/* Message of the last failed call on ctx (static storage of the context;
 * empty string if none).  Returns a static message when ctx is NULL. */
const char* splotch_last_error(const splotch_ctx* ctx);

/*
 * Workspace needed by splotch_render for these particles, camera and
 * parameters, in bytes (*bytes).  Rendering with exactly this size runs in
 * one pass.  A smaller workspace (at least the size reported for n = 65536)
 * is accepted: the particles are then rendered in several chunks, which
 * gives the same image (bit-identical in int64 mode; same up to summation
 * order in FP32).  Particle and colour arrays are not read.
 */
splotch_status splotch_render_workspace_size(splotch_ctx* ctx,
                                             const splotch_particles* particles,
                                             const splotch_camera* camera,
                                             const splotch_params* params,
                                             size_t* bytes);

/*
 * Render one image (Eqs. 1, 2, 7 with E = A) asynchronously on hip_stream.
 * workspace: device buffer of workspace_bytes bytes, 256-byte aligned; its
 * contents on entry do not matter and are garbage afterwards.  n = 0 gives
 * a black image.  Returns SPLOTCH_ERR_WORKSPACE if the workspace is below
 * the minimum, SPLOTCH_ERR_INVALID_ARG for bad arguments (NULL required
 * pointers, n < 0, width or height outside 1..32768, fov outside (0,180),
 * chi <= 0, colormap with n < 2, z_near <= 0, frac_bits outside 8..56,
 * unsupported tile or knob values), SPLOTCH_ERR_HIP if a launch fails.
 */
splotch_status splotch_render(splotch_ctx* ctx, const splotch_particles* particles,
                              const splotch_camera* camera,
                              const splotch_colormap* colormap,
                              const splotch_params* params, const splotch_image* image,
                              void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * Allocation-free variant of splotch_render, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the same render (E = A
 * transfer only), with the workspace taken from a fixed scratch array of
 * SPLOTCH_NOALLOC_SCRATCH_BYTES that the library holds on each device
 * from its first splotch_ctx_create there until the process ends.  The
 * call allocates nothing; the caller still passes the particles, palette
 * and image.  Particle sets whose one-pass workspace exceeds the scratch
 * are rendered in several chunks (same image, bit-identical in int64
 * mode; same up to summation order in FP32).  Stage timing
 * (splotch_set_timing) does not apply to these renders.
 *
 * Every call on one device shares that device's scratch: calls whose work
 * overlaps on the device (different streams or contexts without ordering
 * between them) race and give undefined images.  Calls ordered on one
 * stream are safe; nothing in the scratch is assumed clear on entry.
 *
 * Returns SPLOTCH_ERR_WORKSPACE (before any launch, outputs untouched) if
 * the image alone needs more than the scratch (the optical-depth planes
 * take 12 bytes per pixel in FP32 mode and 24 in int64 mode, plus the
 * binning arrays of at least 65536 particles), SPLOTCH_ERR_UNSUPPORTED for
 * the ordered transfer, SPLOTCH_ERR_HIP if the scratch has no address on
 * this device or a launch fails, and otherwise the errors of
 * splotch_render.
 */
#define SPLOTCH_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)
splotch_status splotch_render_noalloc(splotch_ctx* ctx, const splotch_particles* particles,
                                      const splotch_camera* camera,
                                      const splotch_colormap* colormap,
                                      const splotch_params* params,
                                      const splotch_image* image, void* hip_stream);

/*
 * Streamed render for particle sets held in HOST memory (the chunked data
 * flow of the paper's Section "Splotch Overview" model, Eqs. 3-4, with the
 * host-to-device offload overlapped with rendering).  host_particles holds
 * host pointers (page-locked memory, e.g. hipHostMalloc, lets the copies
 * overlap the rendering; pageable memory works but copies synchronously).
 * The particles are copied in chunks of `chunk` particles into two device
 * staging buffers on a copy stream owned by the context, while hip_stream
 * renders the previous chunk; all chunks add into one image (bit-identical
 * to splotch_render in int64 mode).  camera, colormap, params and image are
 * as for splotch_render (device colormap and image).  workspace: device
 * buffer of at least splotch_render_stream_workspace_size bytes (render
 * workspace for one chunk, two staging buffers, job tables), 256-byte
 * aligned.  The host arrays must stay valid and unchanged until hip_stream
 * has completed the render.  Errors as splotch_render; SPLOTCH_ERR_INVALID_ARG
 * for chunk < 1.
 */
splotch_status splotch_render_stream_workspace_size(splotch_ctx* ctx,
                                                   const splotch_particles* host_particles,
                                                   const splotch_camera* camera,
                                                   const splotch_params* params, int64_t chunk,
                                                   size_t* bytes);
splotch_status splotch_render_streamed(splotch_ctx* ctx, const splotch_particles* host_particles,
                                       const splotch_camera* camera,
                                       const splotch_colormap* colormap,
                                       const splotch_params* params, const splotch_image* image,
                                       int64_t chunk, void* workspace, size_t workspace_bytes,
                                       void* hip_stream);

/*
 * Synchronise hip_stream and read the counters of the last render on ctx
 * into *stats (host struct).  Returns SPLOTCH_ERR_OVERFLOW if that render
 * used int64 accumulation and a pixel overflowed (the stats are still
 * filled), SPLOTCH_OK otherwise.
 */
splotch_status splotch_get_stats(splotch_ctx* ctx, void* hip_stream, splotch_stats* stats);

/* Collect the radius statistics of splotch_stats in later renders on ctx
 * (enable != 0) or not (the default; collecting costs a little time in the
 * counting pass).  SPLOTCH_ERR_INVALID_ARG for a NULL context. */
splotch_status splotch_set_radius_stats(splotch_ctx* ctx, int32_t enable);

/* Count the samples drawn (splotch_stats.n_samples) in later E = A renders
 * on ctx (enable != 0) or not (the default; counting costs a little time in
 * the tile and large passes).  SPLOTCH_ERR_INVALID_ARG for a NULL context. */
splotch_status splotch_set_sample_count(splotch_ctx* ctx, int32_t enable);

/*
 * One job of a batch: a complete render description (the same meaning as
 * the arguments of splotch_render).  Host struct; its pointers are device
 * pointers.
 */
typedef struct {
    splotch_particles particles;
    splotch_camera camera;
    splotch_colormap colormap;
    splotch_params params;
    splotch_image image;
} splotch_job;

/* Workspace for splotch_render_batched on these jobs (*bytes).  Particle
 * and colour arrays are not read.  1 <= n_jobs <= 64. */
splotch_status splotch_batch_workspace_size(splotch_ctx* ctx, const splotch_job* jobs,
                                            int32_t n_jobs, size_t* bytes);

/*
 * Render n_jobs independent images (different particle sets, cameras,
 * resolutions and parameters; all jobs must share one accum mode) with one
 * fixed launch sequence on hip_stream.  Tile work of all jobs goes through a
 * single queue consumed by persistent workgroups, so uneven job sizes are
 * balanced on the device.  The launch sequence is captured into a HIP graph
 * the first time a batch of this shape (job count, per-job launch sizes,
 * workspace address and size) is seen, and replayed afterwards with the new
 * job descriptions, which are uploaded on the stream before the graph.
 * Every image equals the one splotch_render gives for the same job (int64
 * mode: bit for bit).  A workspace below splotch_batch_workspace_size draws
 * the jobs in consecutive groups that fit it, one launch sequence (and
 * graph) per group, and a job that does not fit alone in particle chunks as
 * splotch_render does; the images are the same.  SPLOTCH_ERR_WORKSPACE if
 * some job does not fit even with its smallest chunk.  Other errors as
 * splotch_render; a failing job rejects the whole batch before any launch.
 */
splotch_status splotch_render_batched(splotch_ctx* ctx, const splotch_job* jobs, int32_t n_jobs,
                                      void* workspace, size_t workspace_bytes, void* hip_stream);

/*
 * Autotuner.  Renders `job` with candidate schedules (tile 16/32/64, halo
 * 0/4/8, max_clip_tiles 8/16, chunk 1024/4096; candidates that do not fit the
 * workspace in one pass are skipped), timing each with HIP events on
 * hip_stream (this call synchronises).  The fastest is written to *best
 * (a copy of job->params with the knobs set) and its mean time in ms to
 * *best_ms (may be NULL), and remembered on ctx for the job's size bucket
 * (accum mode, floor(log2 n), floor(log2 width*height)): later renders and
 * batches on ctx whose knobs are left at 0/-1 use it.  The job's image
 * buffers are overwritten.
 */
splotch_status splotch_autotune(splotch_ctx* ctx, const splotch_job* job, void* workspace,
                                size_t workspace_bytes, void* hip_stream, splotch_params* best,
                                float* best_ms);

/* Write the tuned schedules of ctx to a JSON file at `path` (host string),
 * tagged with the device architecture. */
splotch_status splotch_tune_save(splotch_ctx* ctx, const char* path);

/* Load tuned schedules written by splotch_tune_save on the same device
 * architecture (SPLOTCH_ERR_UNSUPPORTED for another device). */
splotch_status splotch_tune_load(splotch_ctx* ctx, const char* path);

/* Stages of a render, in launch order (indices of splotch_get_stage_times). */
#define SPLOTCH_STAGE_CLEAR 0    /* zero the optical-depth planes */
#define SPLOTCH_STAGE_COUNT 1    /* transform, classify, per-workgroup key counts */
#define SPLOTCH_STAGE_SCAN 2     /* exclusive scan of the key counts */
#define SPLOTCH_STAGE_SCATTER 3  /* transform again, write records in key order */
#define SPLOTCH_STAGE_ITEMS 4    /* cut tile lists into work items */
#define SPLOTCH_STAGE_LARGE 5    /* cooperative pass over large footprints */
#define SPLOTCH_STAGE_SPLAT 6    /* per-tile LDS splat */
#define SPLOTCH_STAGE_RESOLVE 7  /* I = 1 - exp(-L) */
#define SPLOTCH_NUM_STAGES 8

/* Turn per-stage timing on (enable != 0) or off for later renders on ctx.
 * When on, every stage of a render is bracketed by HIP events recorded on
 * the render's stream (a little launch overhead is added).  Independently
 * of this, the launches of each stage sit in a roctx range named
 * "splotch <stage>" (clear, count, scan, scatter, items, large, splat,
 * resolve), which a profiler's marker trace records. */
splotch_status splotch_set_timing(splotch_ctx* ctx, int32_t enable);

/* Synchronise hip_stream, then write to ms[0..SPLOTCH_NUM_STAGES-1] the GPU
 * time in milliseconds of each stage summed over the timed renders since
 * the last call, and their number to *renders (may be NULL).  Resets the
 * accumulation.  ms is a host array. */
splotch_status splotch_get_stage_times(splotch_ctx* ctx, void* hip_stream, float* ms,
                                       int32_t* renders);

#ifdef __cplusplus
}
#endif

#endif /* SPLOTCH_H */
