/*
 * fourier_llf.h -- C ABI of libfourier_llf.so, a gfx950 (MI355X) implementation
 * of the Fourier local Laplacian filter ("Gaussian Fourier Pyramid for Local
 * Laplacian Filter", Sumiya, Otsuka, Maeda, Fukushima, IEEE SPL).
 *
 * What one call computes, per channel of an image I with values in [0, R]
 * (problem statement of Sec. II-A and Sec. II-C):
 *   - the period T of Eq. (12) (unless given), omega_k = 2 pi k / T and
 *     alpha~_k = 2 sigma_r^2 alpha_k omega_k of Eq. (9) and Eq. (11), k = 1..K;
 *   - the Gaussian pyramid G_l[I] and the 2K Gaussian Fourier pyramids
 *     G_l[cos(omega_k I)], G_l[sin(omega_k I)] (Eq. (1), Eq. (14) "where" clause);
 *   - the output Laplacian pyramid L_l[O] by the product-sum of Eq. (14);
 *   - the collapse O of Eq. (4).
 * The remap is the detail remap r(i,g) = i + m (i-g) exp(-(i-g)^2 / 2 sigma_r^2)
 * expanded as in Eq. (11): m > 0 enhances detail, m < 0 smooths it, m = 0 returns I.
 * The 5-tap binomial [1 4 6 4 1]/16 filter is used for REDUCE and (with gain 4)
 * for EXPAND; borders are reflect-101; level l+1 has ceil(W_l/2) x ceil(H_l/2)
 * pixels; the output is not clipped.
 *
 * Conventions for every entry point:
 *   - Pointers named "device" are HIP device pointers owned by the caller; the
 *     library never allocates device memory.  Scratch comes from the caller's
 *     workspace (size from fourier_llf_workspace_size).
 *   - All parameters are validated before anything is enqueued; on a non-OK
 *     status nothing was launched and fourier_llf_last_error() says why.
 *   - fourier_llf_run is asynchronous on the caller's stream; results are valid
 *     once that stream has been synchronised.  A context is not thread-safe; use
 *     one context per host thread / stream.
 */
#ifndef FOURIER_LLF_H
#define FOURIER_LLF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLLF_MAX_K 32      /* largest number of Fourier terms K */
#define FLLF_MAX_LEVELS 16 /* largest |L| (levels, counting the residual level) */

typedef enum {
  FLLF_OK = 0,
  FLLF_EINVAL = -1,       /* a parameter is out of range or a pointer is NULL */
  FLLF_ENOMEM = -2,       /* the workspace passed is smaller than required */
  FLLF_EDEVICE = -3,      /* a HIP runtime call failed (also reports earlier async faults) */
  FLLF_EUNSUPPORTED = -4  /* valid request the library does not implement */
} fllf_status;

/* Storage of the 2K cosine/sine Gaussian Fourier pyramid levels in the
 * workspace.  Filtering and accumulation are always float32; G_l[I], the output
 * Laplacian levels and the collapse stay float32 for every storage mode. */
typedef enum {
  FLLF_STORE_F32 = 0,
  FLLF_STORE_F16 = 1,
  FLLF_STORE_BF16 = 2
} fllf_storage;

typedef struct fllf_ctx fllf_ctx; /* opaque, host-side state only */

/* fllf_job.flags: run the fast LLF comparator (Sec. II-C) instead of Fourier LLF:
 * the remap r(i, g) = i + m (i - g) exp(-(i - g)^2 / 2 sigma_r^2) is sampled at K
 * intensities tau j, j = 0 .. K-1, tau = R / (K - 1) (K even, 2..32), the
 * Laplacian pyramids of the K remapped images are built (K + 1 pyramids with
 * G_l[I]), and at every level-l pixel p the output coefficient interpolates
 * them linearly at g = G_l[I]_p (clamped to [0, R]); the top level is
 * G_lmax[I].  Same kernels (REDUCE, EXPAND, collapse) with the sampled remaps in
 * place of the Fourier pairs.  Single-job runs only (n = 1; not batched, not
 * served, no maps, period_T = 0). */
#define FLLF_FLAG_FAST_LLF 1

/* One image to filter (Sec. II-A problem statement: image, levels, sigma_r, m, K).
 * Zero-initialise the struct: every field added after m_map means "dense" or
 * "absent" when 0. */
typedef struct {
  const float *in;   /* device; planar channels x height x width float32 (pitches below) */
  float *out;        /* device; channels x height x width float32 (pitches below); must not
                        overlap in, another job's images or the workspace */
  int32_t width;     /* >= 1 */
  int32_t height;    /* >= 1 */
  int32_t channels;  /* >= 1; each channel is filtered independently */
  int32_t levels;    /* |L| >= 1, counts the residual level;
                        at most fourier_llf_max_levels(height, width) and FLLF_MAX_LEVELS */
  int32_t K;         /* number of Fourier terms, 1..FLLF_MAX_K (fast LLF: samples, see flags) */
  int32_t flags;     /* 0, or FLLF_FLAG_FAST_LLF */
  double sigma_r;    /* range scale of the remap (Eq. (6)), > 0, same units as the pixels */
  double m;          /* detail boost of Eq. (6): > 0 enhance, < 0 smooth, 0 identity */
  double range_R;    /* intensity range R of Eq. (12) (1.0 for [0,1] images), > 0 */
  double period_T;   /* 0 -> fit by Eq. (12); otherwise the period to use, must be > range_R */
  const float *m_map;/* optional device map height x width of per-pixel boosts m_p
                        (pixel-by-pixel form, Sec. III-B); NULL -> the scalar m.
                        Shared by all channels.  At level l the boost of a level-l
                        pixel is the Gaussian pyramid value G_l[m_map] there.
                        Dense rows (row pitch = width). */
  /* Strided images (Sec. II-A takes an image as it is stored): element pitches,
   * 0 = dense.  A crop or other view of a larger tensor is filtered in place
   * of a copy. */
  int64_t row_pitch;       /* elements between rows of in; 0 -> width; else >= width */
  int64_t plane_pitch;     /* elements between channels of in; 0 -> row_pitch * height */
  int64_t out_row_pitch;   /* elements between rows of out; 0 -> width; else >= width */
  int64_t out_plane_pitch; /* elements between channels of out; 0 -> out_row_pitch * height;
                              the channels of out must not overlap: either stacked
                              (>= (height-1)*out_row_pitch + width) or row-interleaved
                              (>= width, with out_row_pitch >= (channels-1)*out_plane_pitch + width) */
  const float *sigma_map;  /* optional device map height x width (dense rows) of per-pixel
                              range scales sigma_p (pixel-by-pixel alpha~_{k,p}, Sec. III-B);
                              NULL -> the scalar sigma_r.  Shared by all channels; at level l
                              the range scale of a level-l pixel is G_l[sigma_map] there.
                              With a map, sigma_r is the smallest value the map holds and
                              sigma_max the largest (both > 0): one period T serves every
                              pixel, fitted by Eq. (12) with each of its two terms taken at
                              the scale where it is largest (period_T overrides). */
  double sigma_max;        /* with sigma_map: the largest range scale in the map (>= sigma_r);
                              ignored without a map */
} fllf_job;

/* Create a context bound to HIP device `device` that stores the Fourier
 * pyramids (the 2K Gaussian Fourier pyramids of Eq. (14)) as `storage`.
 * Fails with FLLF_EDEVICE when the device is absent. */
fllf_status fourier_llf_create(fllf_ctx **out, int device, fllf_storage storage);

/* Bytes of device workspace fourier_llf_run needs for these n jobs (n >= 1):
 * levels 1.. of the 2K+1 pyramids of Eq. (14) (Sec. III-A counts them) and the
 * output Laplacian levels.  Equals the resident footprint of the jobs beyond
 * their in/out images. */
fllf_status fourier_llf_workspace_size(const fllf_ctx *ctx, const fllf_job *jobs, int n,
                                       size_t *bytes);

/* Filter n jobs -- the fit of Eq. (9)-(12), the pyramids of Eq. (1) and
 * Eq. (14), the product-sum of Eq. (14) and the collapse of Eq. (4), per the
 * problem statement of Sec. II-A -- (n >= 1, sizes/K/sigma_r may differ) on `hip_stream` (a
 * hipStream_t; NULL = the legacy default stream).  `workspace` is a device buffer
 * of at least the size returned by fourier_llf_workspace_size, 256-byte aligned,
 * owned by the caller and not used by anything else until the stream syncs.
 *
 * n >= 2 is the batched form: each pass of the filter (REDUCE to level l + 1,
 * then the product-sum and collapse at level l) runs for all jobs that have it
 * as one launch per kernel class (K loop, boost map, top level), the launches
 * finding their jobs in a table at the start of the workspace.  The table is
 * copied from pinned host memory held by the context, on the stream.  Each
 * job's output equals that of a single-job run bit for bit. */
fllf_status fourier_llf_run(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                            size_t ws_bytes, void *hip_stream);

/* ---- a run that allocates nothing ----------------------------------------- */

/* Bytes of the library's own static workspace (256 MiB per device). */
#define FLLF_STATIC_WORKSPACE_BYTES ((size_t)256 << 20)

/* (For callers that cannot allocate: the filter of fourier_llf_run.)
 * For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): filters one
 * job exactly as fourier_llf_run(ctx, job, 1, ...) does (same kernels, same
 * result bit for bit) with the workspace taken from an array of
 * FLLF_STATIC_WORKSPACE_BYTES that the library holds on each device from the
 * first call on that device until the process ends.  The call itself performs
 * no device, pinned or heap allocation (context timing hooks are not applied).
 * Fails with FLLF_ENOMEM, launching nothing, when the job's workspace
 * (fourier_llf_workspace_size) exceeds the limit.  Every call on a device
 * shares that device's array: calls whose work may overlap on one device (two
 * streams, or two host threads) race and must be serialised by the caller,
 * e.g. on one stream.  The array needs no clearing: each call writes every
 * workspace element before it reads it.  Asynchronous on hip_stream. */
fllf_status fourier_llf_run_static(fllf_ctx *ctx, const fllf_job *job, void *hip_stream);

/* ---- re-parameterisation from resident pyramids --------------------------- */

/* After fourier_llf_run(ctx, prev, 1, workspace, ...) the workspace holds the
 * Gaussian pyramid of the input and the 2K Fourier pyramids of prev.  With the
 * period T kept (Sec. III: the pyramids depend on the remap only through
 * omega_k = 2 pi k / T), a new boost m or range scale sigma_r changes only the
 * coefficients of the per-level product-sum (Eq. (11), (14)).  This call
 * filters `next` -- the same input, size, channels, levels, K and R as prev,
 * new m and/or sigma_r, period_T = 0 (keep prev's T) or equal to it, any
 * output buffer -- from the resident pyramids: the product-sum and collapse
 * passes only, each term reweighted by alpha~_k(next) / alpha~_k(prev).
 * Exact up to float32 rounding (the weights multiply stored values); K must
 * be 4, 8 or 16 and neither job may have a boost map (FLLF_EUNSUPPORTED
 * otherwise, also when a term the new parameters need underflowed to zero in
 * the resident pyramids).  The workspace must be the one prev ran in, unused
 * since; its pyramids stay valid, so further calls may follow.  Asynchronous
 * on hip_stream. */
fllf_status fourier_llf_reparam(fllf_ctx *ctx, const fllf_job *prev, const fllf_job *next, void *workspace,
                                size_t ws_bytes, void *hip_stream);

/* ---- launch shape: tuning and autotuning --------------------------------- */

/* Launch-shape parameters of a context (index: meaning):
 *   FLLF_TUNE_DOWN0, FLLF_TUNE_DOWN, FLLF_TUNE_UP0, FLLF_TUNE_UP: the number of
 *     waves a pass aims for when it splits its rows into segments (more waves =
 *     shorter segments = more halo rows re-read): the REDUCE pass from level 0;
 *     from levels >= 1; the up passes that evaluate the product-sum of Eq. (14)
 *     (to level 0 and to levels below 2^20 samples; re-parameterised passes
 *     use a built-in target); and the one-plane collapse to the larger levels
 *     >= 1;
 *   FLLF_TUNE_GRID_CAP: 0 = a batched launch has one wave per work item; c > 0
 *     = at most c times the blocks resident on the device at once, each wave
 *     looping over work items (persistent launch);
 *   FLLF_TUNE_NT_STORES: the pass kinds whose stores are non-temporal (not kept
 *     in the caches for reuse), a bit set: 1 = REDUCE from level 0, 2 = REDUCE
 *     from the levels >= 1 that take the fused form, 4 = the other REDUCE passes
 *     from levels >= 1, 8 = the up pass to level 0, 16 = the up passes and
 *     collapses to levels >= 1 (0..31). */
enum {
  FLLF_TUNE_DOWN0 = 0,
  FLLF_TUNE_DOWN = 1,
  FLLF_TUNE_UP0 = 2,
  FLLF_TUNE_UP = 3,
  FLLF_TUNE_GRID_CAP = 4,
  FLLF_TUNE_NT_STORES = 5,
  FLLF_TUNE_PARAMS = 6
};

/* Launch shape only (no passage of the paper: results do not depend on it).
 * Set the context's parameters; params[i] <= 0 for i < FLLF_TUNE_GRID_CAP,
 * params[FLLF_TUNE_NT_STORES] < 0, or params == NULL, restores the built-in
 * value.  Results do not depend on them. */
fllf_status fourier_llf_set_tuning(fllf_ctx *ctx, const int32_t *params);
/* Read the context's parameters into params[0 .. FLLF_TUNE_PARAMS-1]. */
fllf_status fourier_llf_get_tuning(const fllf_ctx *ctx, int32_t *params);

/* (Launch shape only; no passage of the paper.)
 * Autotuner: times fourier_llf_run of these jobs (same arguments as run) for
 * candidate values of each parameter in turn (coordinate descent; each
 * candidate 1 warm-up and `reps` timed runs, reps >= 1), keeps the fastest in
 * the context and writes them to chosen[0 .. FLLF_TUNE_PARAMS-1] (may be NULL).
 * Synchronous: returns after the stream has drained.  The workspace contents
 * and the jobs' outputs are overwritten. */
fllf_status fourier_llf_autotune(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                 size_t ws_bytes, void *hip_stream, int reps, int32_t *chosen);

/* Autotuner with a persistent cache: the launch shape of a job set depends only
 * on the device, the storage and each job's size, channels, levels, K, flags
 * and maps (not on sigma_r or m).  If the text file `cache_path` holds an entry
 * for that key, its parameters are set in the context without timing anything;
 * otherwise this runs fourier_llf_autotune and appends the result as one line
 * "<key> <p0> .. <p5>" (a missing file is created; unreadable lines are
 * skipped).  Otherwise as fourier_llf_autotune. */
fllf_status fourier_llf_autotune_cached(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                        size_t ws_bytes, void *hip_stream, int reps, const char *cache_path,
                                        int32_t *chosen);

/* ---- captured schedules (HIP graphs) ------------------------------------- */

typedef struct fllf_graph fllf_graph; /* opaque */

/* (Scheduling of the filter of fourier_llf_run; no passage of the paper.)
 * Capture the launches fourier_llf_run would make for these jobs into an
 * instantiated HIP graph.  The batch table is written to the workspace now
 * (synchronously); the graph binds the jobs' in/out/m_map pointers and the
 * workspace, which must stay valid and must not be used for anything else
 * while the graph is in use.  Uses the context's tuning at capture time. */
fllf_status fourier_llf_graph_create(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                     size_t ws_bytes, fllf_graph **out);
/* Enqueue one replay of the captured schedule on `hip_stream`. */
fllf_status fourier_llf_graph_launch(fllf_graph *graph, void *hip_stream);
/* Release the graph.  NULL-safe.  The caller must have synchronised its streams. */
void fourier_llf_graph_destroy(fllf_graph *graph);

/* Release the context.  NULL-safe.  The caller must have synchronised its streams.
 * (Resource management; no passage of the paper.) */
void fourier_llf_destroy(fllf_ctx *ctx);

/* (Error reporting; no passage of the paper.)
 * Human-readable reason for the last non-OK status returned on this thread
 * (ctx may be NULL).  The string stays valid until the next call on this thread. */
const char *fourier_llf_last_error(const fllf_ctx *ctx);

/* ---- serving: continuous batching over a device arena --------------------- */

/* (Scheduling of the filter of fourier_llf_run; no passage of the paper.)
 * A server runs many independent jobs that arrive over time.  Each job is the
 * same filter as fourier_llf_run (same result bit for bit); what differs is
 * the schedule.  Every fourier_llf_server_step
 *   1. admits queued jobs in arrival order while their workspace fits in the
 *      arena (first fit; admission stops at the first job that does not fit,
 *      so no job is overtaken) and while fewer than max_active are in flight;
 *   2. enqueues the next pass of every admitted job -- REDUCE to level l + 1 or
 *      product-sum and collapse at level l -- as batched launches, passes of
 *      the same kernel class sharing one launch whatever their job or level
 *      (iteration-level batching: jobs join and leave between passes).
 * A job's workspace returns to the arena once its last pass has completed on
 * the device (seen by step or poll).  Everything runs on the stream given to
 * step.  The arena is a caller-owned device buffer; it bounds the device
 * memory the server uses beyond the jobs' own input and output images.  A
 * server is not thread-safe. */
typedef struct fllf_server fllf_server; /* opaque */

typedef struct {
  int32_t queued;       /* submitted, not yet admitted */
  int32_t active;       /* admitted, with passes left to enqueue */
  int32_t finishing;    /* all passes enqueued, completion not yet seen */
  int32_t max_active;
  int64_t steps;        /* steps that enqueued work */
  int64_t launches;     /* kernel launches and copies enqueued */
  int64_t completed;    /* jobs reported by fourier_llf_server_poll */
  int64_t passes;       /* job passes enqueued (a pass of one job in one step) */
  int32_t max_step_jobs;/* most jobs advanced by a single step */
  int32_t reserved;
  uint64_t arena_bytes; /* bytes available to job workspaces */
  uint64_t arena_used;  /* bytes held by admitted jobs now */
  uint64_t arena_peak;  /* largest arena_used so far */
} fllf_server_stats;

/* Create a server over `arena` (device, 256-byte aligned, arena_bytes long,
 * owned by the caller and used by nothing else while the server lives) for a
 * context.  At most max_active (1..4096) jobs are in flight at once; a few
 * tables of launch arguments are carved from the front of the arena. */
fllf_status fourier_llf_server_create(fllf_ctx *ctx, void *arena, size_t arena_bytes, int max_active,
                                      fllf_server **out);

/* Queue one job (validated now).  `tag` identifies it in fourier_llf_server_poll.
 * `ready_event` (a hipEvent_t, may be NULL) marks the job's input as written,
 * e.g. the end of its upload on another stream: its first pass waits for it on
 * the device.  FLLF_ENOMEM if its workspace exceeds what the arena can ever
 * hold.  in/out must stay valid until the job is reported done. */
fllf_status fourier_llf_server_submit(fllf_server *srv, const fllf_job *job, uint64_t tag,
                                      void *ready_event);

/* Admit and enqueue one pass of every admitted job on `hip_stream` (see above).
 * Sets *pending (may be NULL) to the number of jobs not yet reported done.
 * Does not wait for the device, except when the ring of launch tables is full
 * (the table of the step four steps back must have been consumed). */
fllf_status fourier_llf_server_step(fllf_server *srv, void *hip_stream, int *pending);

/* Non-blocking: write the tags of up to max jobs whose output is ready (in
 * completion order) to tags[] and their number to *n; releases their workspace. */
fllf_status fourier_llf_server_poll(fllf_server *srv, uint64_t *tags, int max, int *n);

fllf_status fourier_llf_server_stats(const fllf_server *srv, fllf_server_stats *out);

/* Release the server.  NULL-safe; waits for the work it enqueued. */
void fourier_llf_server_destroy(fllf_server *srv);

/* ---- boost map from local variance --------------------------------------- */

/* Boost map of the variance-driven pixel-by-pixel enhancement (Sec. IV: the
 * enhancement of a pixel follows the variance of the pixels in a local window,
 * small where the variance is low):
 *   out[y][x] = m_max v / (v + v_half),
 * v the population variance of `in` over the (2 radius + 1)^2 window around
 * (x, y) with reflect-101 borders.  in: device, height x width float32 with
 * row pitch row_pitch (0 = width; e.g. one channel of a job's input); out:
 * device, dense height x width float32, usable as fllf_job.m_map; in and out
 * must not overlap.  radius in [0, 32], m_max finite, v_half > 0; the size
 * limits of fllf_job apply.  Asynchronous on hip_stream; ctx names the device. */
fllf_status fourier_llf_boost_map(fllf_ctx *ctx, const float *in, int32_t width, int32_t height, int64_t row_pitch,
                                  int32_t radius, double m_max, double v_half, float *out, void *hip_stream);

/* ---- kernel timing (benchmarks) ------------------------------------------ */

/* (Measurement; no passage of the paper.)
 * Aggregated device time of one kernel class over the launches recorded since
 * timing was enabled (or last read). */
typedef struct {
  char name[32];      /* kernel class: "down_l<l>" (REDUCE from level l), "up_l<l>"
                         (product-sum and collapse at level l; a job whose level 1 is
                         large enough for the fused form has no "up_l1": its level-1
                         collapse runs inside "up_l0"), "bdown_l<l>" / "bup_l<l>"
                         (batched launches), "half_l<l>" (re-parameterisation), "copy" */
  int32_t launches;   /* number of launches */
  double total_ms;    /* summed hipEvent durations */
  double bytes;       /* summed algorithmic HBM bytes of those launches */
} fllf_kernel_time;

/* enable != 0: fourier_llf_run brackets every kernel launch with a pair of
 * hipEvents recorded on the run's stream (adds a few microseconds per launch).
 * enable == 0: stop recording.  Recorded events are kept until read. */
fllf_status fourier_llf_timing_enable(fllf_ctx *ctx, int enable);

/* Waits for the recorded events, aggregates them per kernel class into
 * out[0..max-1] (sorted by total time, largest first), sets *n to the number of
 * classes and clears the record.  Fails with FLLF_EDEVICE if an event failed. */
fllf_status fourier_llf_timing_read(fllf_ctx *ctx, fllf_kernel_time *out, int max, int *n);

/* ---- host-only helpers (no device needed) -------------------------------- */

/* Series fit of Eq. (9)-(12) in float64.  If T_in > 0 it is used as the period,
 * else T = argmin_{T > R} erfc(pi sigma_r (2K+1)/T) + erfc((T-R)/sigma_r).
 * Writes *T_out and, for k = 1..K, omega[k-1] = 2 pi k / T and
 * alpha_tilde[k-1] = 2 sigma_r^2 alpha_k omega_k (arrays of length >= K,
 * either may be NULL). */
fllf_status fourier_llf_fit(double sigma_r, int K, double range_R, double T_in, double *T_out,
                            double *omega, double *alpha_tilde);

/* One period T for every range scale in [sigma_lo, sigma_hi] (pixel-by-pixel
 * alpha~_{k,p}, Sec. III-B: the Fourier pyramids depend on T, so all pixels share
 * it): T = argmin_{T > R} erfc(pi sigma_lo (2K+1)/T) + erfc((T-R)/sigma_hi), each
 * term of Eq. (12) at the scale where it is largest; with sigma_lo = sigma_hi it
 * is fourier_llf_fit's T.  The period a job with a sigma_map uses. */
fllf_status fourier_llf_fit_range(double sigma_lo, double sigma_hi, int K, double range_R, double *T_out);

/* The levels |L| of Sec. II-A, counting the residual level.
 * Largest valid level count for an image: 1 + floor(log2(min(height, width))),
 * capped at FLLF_MAX_LEVELS; 0 for non-positive sizes. */
int fourier_llf_max_levels(int height, int width);

/* The problem statement of Sec. II-A as fourier_llf_run checks it:
 * the parameter checks of fourier_llf_run without any device work
 * (pointers are checked for NULL only). */
fllf_status fourier_llf_validate(const fllf_job *jobs, int n, fllf_storage storage);

/* The pyramids of Eq. (14), as fourier_llf_workspace_size counts them.
 * Workspace bytes for these jobs with pyramid storage `storage`, without a
 * context or device (the same number fourier_llf_workspace_size returns).
 * Used for admission by device-memory footprint. */
fllf_status fourier_llf_footprint(const fllf_job *jobs, int n, fllf_storage storage, size_t *bytes);

/* Version of this library as major*10000 + minor*100 + patch. */
int fourier_llf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FOURIER_LLF_H */
