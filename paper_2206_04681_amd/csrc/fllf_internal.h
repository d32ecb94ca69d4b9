// Internal declarations shared by the host planner (fllf_host.cpp) and the
// gfx950 kernels (fllf_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "fourier_llf.h"

namespace fllf {

constexpr int kMaxK = FLLF_MAX_K;
constexpr int kMaxLevels = FLLF_MAX_LEVELS;
constexpr size_t kAlign = 256;  // every plane starts on a 256-byte boundary

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Coefficients of the Fourier remap (Eq. (11)) in the form the kernels use:
// angle of term k at intensity v is 2 pi k (v * inv_T); the product-sum weight of
// term k is boost * at[k] where at[k] = alpha~_{k+1} (Eq. (11)).
//
// Pixel-by-pixel range scale (Sec. III-B): at[k] is alpha~_k at the reference
// scale sref (the smallest in the map), and a pixel of scale s weighs term k by
//   alpha~_k(s) / alpha~_k(sref) = (s / sref)^3 Q^(k^2),
//   Q = exp(-qk (s^2 - sref^2)),  qk = (2 pi / T)^2 / 2           (Eq. (9), (11)),
// which is 1 for every k at s = sref.
struct Coefs {
  float inv_T;
  float m;          // scalar boost (used when the job has no m_map)
  int K;
  int has_mmap;     // 1: per-pixel boost read from the level's m plane
  int has_smap;     // 1: per-pixel range scale read from the level's sigma plane
  float sref, inv_sref, qk;
  // fast LLF (the comparator of Sec. II-C): n samples tau j, j = 0 .. n-1, of the
  // remap r(i, g) = i + m (i - g) exp(-(i - g)^2 rc), rc = 1 / (2 sigma_r^2); the
  // records hold the pyramids of r(I, tau j) as n / 2 pairs (at[] = 1)
  int fast;
  float tau, inv_tau, rc, nm1;  // tau = R / (n - 1); nm1 = n - 1
  float at[kMaxK];  // alpha~_1 .. alpha~_K
  float wt[kMaxK];  // re-parameterisation: new / resident alpha~_k (1 otherwise)
};

// Geometry and workspace placement of one pyramid level of one job.
struct Level {
  int w, h;
  int pitch;         // elements per row: level 0 = the input's row pitch,
                     // levels >= 1 = w rounded up to 64 (aligned, even: vector loads)
  size_t n;          // w * h
  // byte offsets into the workspace (levels >= 1), per-channel strides in elements
  size_t off_g;      // G_l[I]            float32, channels x plane
  size_t off_cs;     // (C~, S~)_{l,k}    storage pair, channels x K x plane
  size_t off_o;      // O_l (collapse)    float32, channels x plane   (1 <= l < top)
  size_t off_m;      // G_l[m_map]        float32, one plane           (1 <= l < top)
  size_t off_s;      // G_l[sigma_map]    float32, one plane           (1 <= l < top)
  size_t g_cstride;  // elements between channels of G and O
  size_t cs_kstride; // pair elements between consecutive k (1: the K pairs of a pixel are contiguous)
  size_t cs_cstride; // pair elements between channels
};

// A strided image copy (a job with a single level: the output is the input):
// C planes of h rows of w_bytes each; pitches and strides in bytes.
struct CopyDesc {
  const void *src;
  void *dst;
  size_t w_bytes, h, spitch, dpitch, sstride, dstride;
  int C;
};
hipError_t copy_image(const CopyDesc &d, hipStream_t stream);

struct JobPlan {
  int levels, K, C;  // K: pairs per record (Fourier terms; for fast LLF, samples / 2)
  bool fast;         // fast LLF comparator
  int dwp;           // dwords per stored (C~, S~) pair: 2 (float32) or 1 (16-bit)
  Level lv[kMaxLevels];
  size_t bytes;      // workspace bytes of this job
  Coefs coefs;
  const float *in;
  float *out;
  const float *m_map;
  const float *s_map;  // per-pixel range scales (sigma_map) or null
  // level-0 images: element pitches of the caller's rows and channels (the
  // input's row pitch is also lv[0].pitch); the maps have dense rows
  size_t in_cs, out_cs;
  int out_pitch;
  CopyDesc copy;     // the whole job when levels == 1
};

// Element pitches of a job's images with the dense defaults applied.
inline int64_t job_in_rp(const fllf_job &j) { return j.row_pitch > 0 ? j.row_pitch : j.width; }
inline int64_t job_in_pp(const fllf_job &j) { return j.plane_pitch > 0 ? j.plane_pitch : job_in_rp(j) * j.height; }
inline int64_t job_out_rp(const fllf_job &j) { return j.out_row_pitch > 0 ? j.out_row_pitch : j.width; }
inline int64_t job_out_pp(const fllf_job &j) {
  return j.out_plane_pitch > 0 ? j.out_plane_pitch : job_out_rp(j) * j.height;
}
// Bytes from an image's first element to one past its last (the span overlap
// checks use): channels x rows x width at the given element pitches.
inline size_t image_span(const fllf_job &j, int64_t rp, int64_t pp) {
  return (size_t)((int64_t)(j.channels - 1) * pp + (int64_t)(j.height - 1) * rp + j.width) * sizeof(float);
}
inline size_t in_span(const fllf_job &j) { return image_span(j, job_in_rp(j), job_in_pp(j)); }
inline size_t out_span(const fllf_job &j) { return image_span(j, job_out_rp(j), job_out_pp(j)); }
inline size_t map_span(const fllf_job &j) { return (size_t)j.width * j.height * sizeof(float); }
// True when [p, p + a) and [q, q + b) share a byte (null pointers share none).
inline bool spans_overlap(const void *p, size_t a, const void *q, size_t b) {
  const char *x = (const char *)p, *y = (const char *)q;
  return x && y && x < y + b && y < x + a;
}

// Host fit in float64 (Eq. (9)-(12)).
double fit_period(double sigma_r, int K, double R);
// One period for range scales in [sigma_lo, sigma_hi]: Eq. (12) with its
// truncation term at sigma_lo and its aliasing term at sigma_hi.
double fit_period_range(double sigma_lo, double sigma_hi, int K, double R);
void fourier_terms(double sigma_r, int K, double T, double *omega, double *alpha_tilde);

// Plans one job: level sizes and workspace offsets starting at byte `base`.
void plan_job(const fllf_job &job, fllf_storage storage, size_t base, JobPlan *plan);

// Optional per-launch timing: called before and after every kernel launch with
// the kernel class name and its algorithmic HBM bytes.
struct LaunchHook {
  virtual ~LaunchHook() = default;
  virtual void before(hipStream_t s) = 0;
  virtual void after(hipStream_t s, const char *name, double bytes) = 0;
};

// Timing names of the per-level kernels ("down_l<l>", "up_l<l>"; "bdown_l<l>",
// "bup_l<l>" for the batched launches).
extern const char *const kDownNames[kMaxLevels];
extern const char *const kUpNames[kMaxLevels];
extern const char *const kBatchDownNames[kMaxLevels];
extern const char *const kBatchUpNames[kMaxLevels];
extern const char *const kHalfNames[kMaxLevels];  // "half_l<l>": re-parameterisation

// Launch-shape parameters.  waves[i] is the number of waves a pass aims for when
// it picks its segment length (the kinds: 0 = down(0), 1 = down(l >= 1),
// 2 = up(0), 3 = up(l >= 1)); grid_cap > 0 caps a batched launch at grid_cap
// times the blocks that fit on the device at once (a persistent launch);
// nt_stores is a bit set of pass kinds (kNt*) whose stores are non-temporal.
enum { kTuneDown0 = 0, kTuneDown = 1, kTuneUp0 = 2, kTuneUp = 3, kTuneGridCap = 4, kTuneNtStores = 5, kTuneParams = 6 };
// Bits of the non-temporal-store parameter: the pass kinds whose stores skip
// cache reuse.
enum { kNtDown0 = 0, kNtDownFused = 1, kNtDown = 2, kNtUp0 = 3, kNtUp = 4, kNtAll = 31 };
struct Tuning {
  int p[kTuneParams];
};
Tuning default_tuning(fllf_storage storage);

// Enqueues the whole filter for one planned job on `stream`.
hipError_t launch_job(const JobPlan &plan, fllf_storage storage, char *ws, hipStream_t stream,
                      LaunchHook *hook, const Tuning &tune);
// The same per pyramid storage type (one compilation unit each).
hipError_t launch_job_f32(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_job_f16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_job_bf16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);

// Re-parameterised filter of a job whose pyramids are resident in ws (exact
// K = 4, 8, 16; coefs.at / coefs.wt / coefs.m hold the new parameters).
hipError_t launch_reparam(const JobPlan &plan, fllf_storage storage, char *ws, hipStream_t stream,
                          LaunchHook *hook, const Tuning &tune);
hipError_t launch_reparam_f32(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_reparam_f16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_reparam_bf16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);

// ---------------------------------------------------------------------------
// Batched form: every pass (down(l), then up(l)) of all jobs that reach level
// l + 1 runs as one launch per kernel class (K loop, boost map, top level).
// The per-job arguments and wave offsets of all launches form one table that
// lives at the start of the workspace.
// ---------------------------------------------------------------------------
struct BatchLaunch {
  int kind;           // 0 = down, 1 = up, 2 = copy (single-level job: in -> out)
  int level;          // l of down(l) / up(l)
  bool l0, map, hasd; // level-0 variant, boost map, O_{l+1} present (up)
  bool fuse;          // fused level: down finishes L_l[O]; up is the collapse
  int km;             // K loop length (4, 8, 16 or 32)
  bool ex;            // K == km exactly
  int njobs;
  uint32_t waves;     // total waves over the jobs
  size_t args_off;    // byte offsets of the argument array and of the njobs + 1 wave offsets
  size_t start_off;
  double bytes;       // algorithmic bytes of the launch
  CopyDesc copy;      // kind 2
};

struct BatchSchedule {
  size_t table_bytes = 0;          // bytes of the table (a multiple of kAlign)
  std::vector<unsigned char> blob; // host image of the table
  std::vector<BatchLaunch> launches;
};

// Plans the table and the launches of n planned jobs whose workspaces follow a
// table at byte offset 0 of ws.  Storage decides the record size.  With
// ws == nullptr only the sizes are planned (the argument records stay zero).
void build_batch(const JobPlan *plans, int n, fllf_storage storage, char *ws, const Tuning &tune,
                 BatchSchedule *out);
// One pass of one job: down(l) or up(l).
struct PassItem {
  const JobPlan *P;
  int l;
  bool down;
};
// The launches of independent passes of different jobs (one serving step): one
// launch per kernel class, levels mixed; the table starts at byte 0 of the blob.
void build_step(const PassItem *items, int n, fllf_storage storage, char *ws, const Tuning &tune,
                BatchSchedule *out);
// Upper bound of build_step's table bytes for n items.
size_t step_table_bound(int n);
// Bytes the batch table of these jobs needs (0 for a single job, which uses no table).
size_t batch_table_bytes(const JobPlan *plans, int n, fllf_storage storage);
// Enqueues a schedule whose table is already in the workspace (ws + 0).
hipError_t launch_batch(const BatchSchedule &s, fllf_storage storage, char *ws, hipStream_t stream,
                        LaunchHook *hook, const Tuning &tune);
hipError_t launch_batch_f32(const BatchSchedule &s, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_batch_f16(const BatchSchedule &s, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);
hipError_t launch_batch_bf16(const BatchSchedule &s, char *ws, hipStream_t stream, LaunchHook *hook, const Tuning &tune);

// ---------------------------------------------------------------------------
// Context access for the other host units (the context is defined in fllf_host.cpp).
// ---------------------------------------------------------------------------
fllf_storage ctx_storage(const fllf_ctx *ctx);
int ctx_device(const fllf_ctx *ctx);
const Tuning &ctx_tuning(const fllf_ctx *ctx);
LaunchHook *ctx_hook(fllf_ctx *ctx);
// Records the message as the thread's (and the context's) last error; returns st.
fllf_status ctx_fail(fllf_ctx *ctx, fllf_status st, const char *fmt, ...);
// The parameter checks of fourier_llf_run.
fllf_status validate_jobs(fllf_ctx *ctx, const fllf_job *jobs, int n, fllf_storage storage);
// Validates, plans and enqueues one job in the workspace ws (ws_bytes long), with
// no heap, pinned or device allocation and no timing hook; `who` names the
// entry point in error messages.
fllf_status run_single(fllf_ctx *ctx, const char *who, const fllf_job &job, void *ws, size_t ws_bytes,
                       hipStream_t stream);

}  // namespace fllf
