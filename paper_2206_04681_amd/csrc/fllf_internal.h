// Internal declarations shared by the host planner (fllf_host.cpp) and the
// gfx950 kernels (fllf_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

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

// Timing names of the per-level kernels ("down_l<l>", "up_l<l>").
extern const char *const kDownNames[kMaxLevels];
extern const char *const kUpNames[kMaxLevels];

// Enqueues the whole filter for one planned job on `stream`.
hipError_t launch_job(const JobPlan &plan, fllf_storage storage, char *ws, hipStream_t stream,
                      LaunchHook *hook);
// The same per pyramid storage type (one compilation unit each).
hipError_t launch_job_f32(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook);
hipError_t launch_job_f16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook);
hipError_t launch_job_bf16(const JobPlan &plan, char *ws, hipStream_t stream, LaunchHook *hook);

}  // namespace fllf
