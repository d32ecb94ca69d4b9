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
struct Coefs {
  float inv_T;
  float m;          // scalar boost (used when the job has no m_map)
  int K;
  int has_map;      // 1: per-pixel boost read from the level's m plane
  float at[kMaxK];  // alpha~_1 .. alpha~_K
  float wt[kMaxK];  // re-parameterisation: new / resident alpha~_k (1 otherwise)
};

// Geometry and workspace placement of one pyramid level of one job.
struct Level {
  int w, h;
  int pitch;         // elements per row: level 0 = the caller's dense rows (w),
                     // levels >= 1 = w rounded up to 64 (aligned, even: vector loads)
  size_t n;          // w * h
  // byte offsets into the workspace (levels >= 1), per-channel strides in elements
  size_t off_g;      // G_l[I]            float32, channels x plane
  size_t off_cs;     // (C~, S~)_{l,k}    storage pair, channels x K x plane
  size_t off_o;      // O_l (collapse)    float32, channels x plane   (1 <= l < top)
  size_t off_m;      // G_l[m_map]        float32, one plane           (1 <= l < top)
  size_t g_cstride;  // elements between channels of G and O
  size_t cs_kstride; // pair elements between consecutive k (1: the K pairs of a pixel are contiguous)
  size_t cs_cstride; // pair elements between channels
};

struct JobPlan {
  int levels, K, C;
  int dwp;           // dwords per stored (C~, S~) pair: 2 (float32) or 1 (16-bit)
  Level lv[kMaxLevels];
  size_t bytes;      // workspace bytes of this job
  Coefs coefs;
  const float *in;
  float *out;
  const float *m_map;
};

// Host fit in float64 (Eq. (9)-(12)).
double fit_period(double sigma_r, int K, double R);
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
// times the blocks that fit on the device at once (a persistent launch).
enum { kTuneDown0 = 0, kTuneDown = 1, kTuneUp0 = 2, kTuneUp = 3, kTuneGridCap = 4, kTuneParams = 5 };
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
  const void *copy_src;  // kind 2
  void *copy_dst;
  size_t copy_bytes;
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

}  // namespace fllf
