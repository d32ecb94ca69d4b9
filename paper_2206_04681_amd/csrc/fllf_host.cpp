// Host side of libfourier_llf.so: the C ABI, parameter validation, the float64
// series fit (Eq. (9)-(12)) and workspace planning.  Kernels live in
// fllf_kernels.hip; this file only decides what to launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <string>
#include <vector>

#include "fllf_internal.h"

namespace {

// Records a hipEvent pair around every launch (when timing is enabled).
struct EventTimer : fllf::LaunchHook {
  struct Rec {
    const char *name;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t pending = nullptr;
  hipError_t err = hipSuccess;

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) err = r;
    return e;
  }
  void before(hipStream_t s) override {
    pending = get();
    if (pending) {
      hipError_t r = hipEventRecord(pending, s);
      if (r != hipSuccess) err = r;
    }
  }
  void after(hipStream_t s, const char *name, double bytes) override {
    hipEvent_t e = get();
    if (e && pending) {
      hipError_t r = hipEventRecord(e, s);
      if (r != hipSuccess) err = r;
      recs.push_back({name, bytes, pending, e});
    }
    pending = nullptr;
  }
  ~EventTimer() override {
    for (auto &r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

}  // namespace

struct fllf_ctx {
  int device;
  fllf_storage storage;
  std::string last_error;
  EventTimer *timer = nullptr;  // records kept until read
  bool timing_on = false;       // launches are bracketed only while enabled
  fllf::Tuning tune;
  // pinned host staging of the batch table; stage_ev marks the end of its last copy
  void *stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
};

struct fllf_graph {
  int device;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string g_last_error;

fllf_status fail(fllf_ctx *ctx, fllf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  if (ctx) ctx->last_error = buf;
  return st;
}

int storage_bytes(fllf_storage s) { return s == FLLF_STORE_F32 ? 4 : 2; }

bool is_finite(double x) { return std::isfinite(x); }

}  // namespace

namespace fllf {

// ---------------------------------------------------------------------------
// Series fit.  Eq. (12) asks for T minimising
//   E(T) = erfc(a / T) + erfc((T - R) / s),  a = pi s (2K + 1),  T > R.
// E'(T) = 2/sqrt(pi) * [ (a/T^2) exp(-a^2/T^2) - (1/s) exp(-(T-R)^2/s^2) ], so the
// sign of E' is the sign of
//   F(T) = ln(a s / T^2) - a^2 / T^2 + (T - R)^2 / s^2,
// which has no underflow even where both erfc terms are below 1e-300.  The
// minimum is the first crossing of F from negative to positive; it is bracketed
// on a uniform grid and refined by bisection to full double precision.
// With a range of scales [s_lo, s_hi] (one T for every pixel, Sec. III-B) the
// truncation term is taken at s_lo (a = pi s_lo (2K + 1)) and the aliasing term
// at s_hi (s = s_hi): each at the scale where it is largest.
// ---------------------------------------------------------------------------
static double stationarity(double T, double a, double s, double R) {
  return std::log(a * s / (T * T)) - (a * a) / (T * T) + (T - R) * (T - R) / (s * s);
}

static double period_error(double T, double a, double s, double R) {
  return std::erfc(a / T) + std::erfc((T - R) / s);
}

static double fit_period_as(double a, double s, double R) {
  const double lo = R, hi = R + 20.0 * s + 4.0 * a;
  const int n = 4096;
  double prev_T = lo + (hi - lo) / n, prev_F = stationarity(prev_T, a, s, R);
  for (int i = 2; i <= n; ++i) {
    double T = lo + (hi - lo) * i / n;
    double F = stationarity(T, a, s, R);
    if (prev_F < 0.0 && F >= 0.0) {
      double x0 = prev_T, x1 = T;
      for (int it = 0; it < 200 && x1 - x0 > 0.0; ++it) {
        double xm = 0.5 * (x0 + x1);
        if (xm <= x0 || xm >= x1) break;
        if (stationarity(xm, a, s, R) < 0.0) x0 = xm; else x1 = xm;
      }
      return 0.5 * (x0 + x1);
    }
    prev_T = T;
    prev_F = F;
  }
  // E' never changes sign from - to +: take the smallest E on the grid.
  double best_T = lo + (hi - lo) / n, best_E = period_error(best_T, a, s, R);
  for (int i = 2; i <= n; ++i) {
    double T = lo + (hi - lo) * i / n, E = period_error(T, a, s, R);
    if (E < best_E) { best_E = E; best_T = T; }
  }
  return best_T;
}

double fit_period(double s, int K, double R) { return fit_period_as(M_PI * s * (2.0 * K + 1.0), s, R); }

double fit_period_range(double s_lo, double s_hi, int K, double R) {
  return fit_period_as(M_PI * s_lo * (2.0 * K + 1.0), s_hi, R);
}

// omega_k = 2 pi k / T; alpha_k = s sqrt(2 pi) / T exp(-(omega_k s)^2 / 2) (Eq. (9));
// alpha~_k = 2 s^2 alpha_k omega_k (Eq. (11)).
void fourier_terms(double s, int K, double T, double *omega, double *alpha_tilde) {
  for (int k = 1; k <= K; ++k) {
    double w = 2.0 * M_PI * k / T;
    double alpha = s * std::sqrt(2.0 * M_PI) / T * std::exp(-0.5 * (w * s) * (w * s));
    if (omega) omega[k - 1] = w;
    if (alpha_tilde) alpha_tilde[k - 1] = 2.0 * s * s * alpha * w;
  }
}

// Workspace layout of one job, all planes 256-byte aligned, rows padded to 64 pixels:
//   for l = 1..top : G_l      [C][h_l][pitch_l] float32
//                    CS_l     [C][h_l][pitch_l][K] pairs (C~_{l,k}, S~_{l,k}) of the storage
//                             type, times alpha~_k: the K pairs of a pixel are one record
//   for l = 1..top-1: O_l     [C][h_l][pitch_l] float32   (collapse of levels >= l)
//                     M_l     [h_l][pitch_l] float32      (only with a per-pixel boost map)
void plan_job(const fllf_job &job, fllf_storage storage, size_t base, JobPlan *p) {
  std::memset(p, 0, sizeof(*p));
  p->levels = job.levels;
  p->fast = (job.flags & FLLF_FLAG_FAST_LLF) != 0;
  p->K = p->fast ? job.K / 2 : job.K;
  // With a per-pixel map, 9 to 15 terms run the exact 16-term loop with the
  // extra terms' weights zero (alpha~_k = 0 for k >= K below): their records are
  // zero and add exact zeros to every sum, while the guarded 16-term loop with
  // maps kept about 0.9 KB per lane in scratch memory.
  if (!p->fast && (job.m_map || job.sigma_map) && job.K > 8 && job.K < 16) p->K = 16;
  p->C = job.channels;
  p->dwp = storage == FLLF_STORE_F32 ? 2 : 1;
  p->in = job.in;
  p->out = job.out;
  p->m_map = job.m_map;
  p->s_map = job.sigma_map;
  const size_t pair_bytes = 2 * (size_t)storage_bytes(storage);
  int w = job.width, h = job.height;
  size_t off = base;
  for (int l = 0; l < job.levels; ++l) {
    Level &L = p->lv[l];
    L.w = w;
    L.h = h;
    L.pitch = l == 0 ? (int)job_in_rp(job) : (int)align_up((size_t)w, 64);
    L.n = (size_t)w * h;
    const size_t g_plane = align_up((size_t)L.pitch * h * 4);
    const size_t cs_plane = align_up((size_t)L.pitch * h * pair_bytes * p->K);
    L.g_cstride = g_plane / 4;
    L.cs_kstride = 1;
    L.cs_cstride = cs_plane / pair_bytes;
    if (l >= 1) {
      L.off_g = off;
      off += g_plane * job.channels;
      L.off_cs = off;
      off += cs_plane * job.channels;
      if (l < job.levels - 1) {
        L.off_o = off;
        off += g_plane * job.channels;
        if (job.m_map) {
          L.off_m = off;
          off += g_plane;
        }
        if (job.sigma_map) {
          L.off_s = off;
          off += g_plane;
        }
      }
    }
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  p->bytes = off - base;
  p->in_cs = (size_t)job_in_pp(job);
  p->out_cs = (size_t)job_out_pp(job);
  p->out_pitch = (int)job_out_rp(job);
  CopyDesc &cp = p->copy;
  cp.src = job.in;
  cp.dst = job.out;
  cp.w_bytes = (size_t)job.width * sizeof(float);
  cp.h = (size_t)job.height;
  cp.spitch = (size_t)job_in_rp(job) * sizeof(float);
  cp.dpitch = (size_t)job_out_rp(job) * sizeof(float);
  cp.sstride = p->in_cs * sizeof(float);
  cp.dstride = p->out_cs * sizeof(float);
  cp.C = job.channels;

  if (p->fast) {  // the sampled remap: no period, no alpha~
    const int n = job.K;
    p->coefs.m = (float)job.m;
    p->coefs.K = p->K;
    p->coefs.fast = 1;
    p->coefs.tau = (float)(job.range_R / (n - 1));
    p->coefs.inv_tau = (float)((n - 1) / job.range_R);
    p->coefs.rc = (float)(1.0 / (2.0 * job.sigma_r * job.sigma_r));
    p->coefs.nm1 = (float)(n - 1);
    for (int k = 0; k < kMaxK; ++k) p->coefs.at[k] = p->coefs.wt[k] = 1.0f;
    return;
  }
  const double T = job.period_T > 0.0 ? job.period_T
                   : job.sigma_map  ? fit_period_range(job.sigma_r, job.sigma_max, job.K, job.range_R)
                                    : fit_period(job.sigma_r, job.K, job.range_R);
  double at[kMaxK];
  fourier_terms(job.sigma_r, job.K, T, nullptr, at);
  p->coefs.inv_T = (float)(1.0 / T);
  p->coefs.m = (float)job.m;
  p->coefs.K = p->K;
  p->coefs.has_mmap = job.m_map ? 1 : 0;
  p->coefs.has_smap = job.sigma_map ? 1 : 0;
  p->coefs.sref = (float)job.sigma_r;
  p->coefs.inv_sref = (float)(1.0 / job.sigma_r);
  p->coefs.qk = (float)(0.5 * (2.0 * M_PI / T) * (2.0 * M_PI / T));
  for (int k = 0; k < kMaxK; ++k) {
    p->coefs.at[k] = k < job.K ? (float)at[k] : 0.0f;
    p->coefs.wt[k] = 1.0f;
  }
}

const char *const kDownNames[kMaxLevels] = {
    "down_l0", "down_l1", "down_l2",  "down_l3",  "down_l4",  "down_l5",  "down_l6",  "down_l7",
    "down_l8", "down_l9", "down_l10", "down_l11", "down_l12", "down_l13", "down_l14", "down_l15"};
const char *const kUpNames[kMaxLevels] = {"up_l0", "up_l1", "up_l2",  "up_l3",  "up_l4",  "up_l5",
                                          "up_l6", "up_l7", "up_l8",  "up_l9",  "up_l10", "up_l11",
                                          "up_l12", "up_l13", "up_l14", "up_l15"};

const char *const kHalfNames[kMaxLevels] = {
    "half_l0", "half_l1", "half_l2",  "half_l3",  "half_l4",  "half_l5",  "half_l6",  "half_l7",
    "half_l8", "half_l9", "half_l10", "half_l11", "half_l12", "half_l13", "half_l14", "half_l15"};

// Dense images go as one copy, evenly spaced planes as one 2-D copy of
// C x h rows, anything else as one 2-D copy per channel.
hipError_t copy_image(const CopyDesc &d, hipStream_t st) {
  const bool dense = d.spitch == d.w_bytes && d.dpitch == d.w_bytes && d.sstride == d.w_bytes * d.h &&
                     d.dstride == d.w_bytes * d.h;
  if (dense)
    return hipMemcpyAsync(d.dst, d.src, d.w_bytes * d.h * d.C, hipMemcpyDeviceToDevice, st);
  if (d.sstride == d.spitch * d.h && d.dstride == d.dpitch * d.h)
    return hipMemcpy2DAsync(d.dst, d.dpitch, d.src, d.spitch, d.w_bytes, d.h * d.C, hipMemcpyDeviceToDevice, st);
  for (int c = 0; c < d.C; ++c) {
    const hipError_t e = hipMemcpy2DAsync((char *)d.dst + c * d.dstride, d.dpitch, (const char *)d.src + c * d.sstride,
                                          d.spitch, d.w_bytes, d.h, hipMemcpyDeviceToDevice, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reparam(const JobPlan &P, fllf_storage storage, char *ws, hipStream_t st, LaunchHook *h,
                          const Tuning &tu) {
  if (P.levels == 1) return copy_image(P.copy, st);
  switch (storage) {
    case FLLF_STORE_F16: return launch_reparam_f16(P, ws, st, h, tu);
    case FLLF_STORE_BF16: return launch_reparam_bf16(P, ws, st, h, tu);
    default: return launch_reparam_f32(P, ws, st, h, tu);
  }
}

hipError_t launch_job(const JobPlan &P, fllf_storage storage, char *ws, hipStream_t st, LaunchHook *h,
                      const Tuning &tu) {
  if (P.levels == 1) return copy_image(P.copy, st);
  switch (storage) {
    case FLLF_STORE_F16: return launch_job_f16(P, ws, st, h, tu);
    case FLLF_STORE_BF16: return launch_job_bf16(P, ws, st, h, tu);
    default: return launch_job_f32(P, ws, st, h, tu);
  }
}

}  // namespace fllf

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int fourier_llf_version(void) { return 10000; }

int fourier_llf_max_levels(int height, int width) {
  if (height <= 0 || width <= 0) return 0;
  int m = height < width ? height : width;
  int L = 1;
  while ((m >> L) >= 1) ++L;  // 1 + floor(log2(m))
  return L > FLLF_MAX_LEVELS ? FLLF_MAX_LEVELS : L;
}

static fllf_status validate(fllf_ctx *ctx, const fllf_job *jobs, int n, fllf_storage storage) {
  if (storage != FLLF_STORE_F32 && storage != FLLF_STORE_F16 && storage != FLLF_STORE_BF16)
    return fail(ctx, FLLF_EINVAL, "unknown storage mode %d", (int)storage);
  if (!jobs || n < 1) return fail(ctx, FLLF_EINVAL, "jobs must be non-NULL and n >= 1 (n=%d)", n);
  for (int i = 0; i < n; ++i) {
    const fllf_job &j = jobs[i];
    if (!j.in || !j.out) return fail(ctx, FLLF_EINVAL, "job %d: in/out must be non-NULL", i);
    if (j.width < 1 || j.height < 1 || j.channels < 1)
      return fail(ctx, FLLF_EINVAL, "job %d: width, height, channels must be >= 1 (%d x %d x %d)", i,
                  j.width, j.height, j.channels);
    if (j.width > 65536 || j.height > 65536 || (int64_t)j.width * j.height > (int64_t)1 << 30 ||
        j.channels > 65535)
      return fail(ctx, FLLF_EINVAL, "job %d: image too large (%d x %d x %d)", i, j.width, j.height,
                  j.channels);
    const int maxL = fourier_llf_max_levels(j.height, j.width);
    if (j.levels < 1 || j.levels > maxL)
      return fail(ctx, FLLF_EINVAL, "job %d: levels=%d outside [1, %d] for %d x %d", i, j.levels, maxL,
                  j.width, j.height);
    if (j.flags & ~FLLF_FLAG_FAST_LLF) return fail(ctx, FLLF_EINVAL, "job %d: unknown flags 0x%x", i, j.flags);
    const bool fast = (j.flags & FLLF_FLAG_FAST_LLF) != 0;
    if (fast) {
      if (j.K < 2 || j.K > 32 || (j.K & 1))
        return fail(ctx, FLLF_EINVAL, "job %d: fast LLF needs an even number of samples K in [2, 32] (K=%d)", i, j.K);
      if (j.period_T != 0.0) return fail(ctx, FLLF_EINVAL, "job %d: fast LLF has no period (period_T must be 0)", i);
      if (j.m_map || j.sigma_map) return fail(ctx, FLLF_EUNSUPPORTED, "job %d: fast LLF takes no per-pixel maps", i);
      if (n > 1) return fail(ctx, FLLF_EUNSUPPORTED, "job %d: fast LLF runs as a single job", i);
    } else if (j.K < 1 || j.K > FLLF_MAX_K) {
      return fail(ctx, FLLF_EINVAL, "job %d: K=%d outside [1, %d]", i, j.K, FLLF_MAX_K);
    }
    const int pairs = fast ? j.K / 2 : j.K;  // (cos, sin) pairs, or pairs of samples, per record
    if (!is_finite(j.sigma_r) || j.sigma_r <= 0.0)
      return fail(ctx, FLLF_EINVAL, "job %d: sigma_r must be finite and > 0", i);
    if (!is_finite(j.m)) return fail(ctx, FLLF_EINVAL, "job %d: m must be finite", i);
    if (!is_finite(j.range_R) || j.range_R <= 0.0)
      return fail(ctx, FLLF_EINVAL, "job %d: range_R must be finite and > 0", i);
    if (!is_finite(j.period_T) || (j.period_T != 0.0 && j.period_T <= j.range_R))
      return fail(ctx, FLLF_EINVAL, "job %d: period_T must be 0 (fit) or > range_R", i);
    // kernels address one channel's plane with 32-bit byte offsets: the largest
    // (the level-1 record plane) must stay below 4 GiB
    if (j.levels >= 2) {
      const uint64_t w1 = (uint64_t)(j.width + 1) / 2, h1 = (uint64_t)(j.height + 1) / 2;
      const uint64_t rec_plane = fllf::align_up(w1, 64) * h1 * (uint64_t)pairs * 2u * storage_bytes(storage);
      if (rec_plane >= ((uint64_t)1 << 32))
        return fail(ctx, FLLF_EINVAL, "job %d: %d x %d with K=%d needs a level-1 plane of %llu bytes (limit 4 GiB)",
                    i, j.width, j.height, j.K, (unsigned long long)rec_plane);
    }
    // pitches: rows at least as long as the image; the output's channels must
    // not share an element (stacked planes or row-interleaved channels); every
    // plane is addressed with 32-bit byte offsets from its first element
    if (j.row_pitch < 0 || (j.row_pitch > 0 && j.row_pitch < j.width) || j.plane_pitch < 0 ||
        j.out_row_pitch < 0 || (j.out_row_pitch > 0 && j.out_row_pitch < j.width) || j.out_plane_pitch < 0)
      return fail(ctx, FLLF_EINVAL, "job %d: pitches must be 0 (dense) or rows of at least width=%d elements", i,
                  j.width);
    const int64_t irp = fllf::job_in_rp(j), orp = fllf::job_out_rp(j), opp = fllf::job_out_pp(j);
    const int64_t kPlaneLimit = (int64_t)1 << 30;  // elements: 4 GiB of float32
    if (irp > kPlaneLimit || orp > kPlaneLimit || (int64_t)(j.height - 1) * irp + j.width > kPlaneLimit ||
        (int64_t)(j.height - 1) * orp + j.width > kPlaneLimit || fllf::job_in_pp(j) > ((int64_t)1 << 46) ||
        opp > ((int64_t)1 << 46))
      return fail(ctx, FLLF_EINVAL, "job %d: a channel plane spans more than 2^30 elements", i);
    if (j.channels > 1) {
      const bool stacked = opp >= (int64_t)(j.height - 1) * orp + j.width;
      const bool interleaved = opp >= j.width && orp >= (int64_t)(j.channels - 1) * opp + j.width;
      if (!stacked && !interleaved)
        return fail(ctx, FLLF_EINVAL, "job %d: out_plane_pitch %lld makes the output's channels overlap", i,
                    (long long)opp);
    }
    if (fllf::spans_overlap(j.in, fllf::in_span(j), j.out, fllf::out_span(j)))
      return fail(ctx, FLLF_EINVAL, "job %d: in and out overlap", i);
    if (fllf::spans_overlap(j.m_map, fllf::map_span(j), j.out, fllf::out_span(j)))
      return fail(ctx, FLLF_EINVAL, "job %d: m_map and out overlap", i);
    if (fllf::spans_overlap(j.sigma_map, fllf::map_span(j), j.out, fllf::out_span(j)))
      return fail(ctx, FLLF_EINVAL, "job %d: sigma_map and out overlap", i);
    if (j.sigma_map && (!is_finite(j.sigma_max) || j.sigma_max < j.sigma_r))
      return fail(ctx, FLLF_EINVAL, "job %d: with sigma_map, sigma_max must be finite and >= sigma_r", i);
  }
  // in a batch every output must be disjoint from every other job's images
  for (int i = 0; i < n && n > 1; ++i) {
    const size_t bi = fllf::out_span(jobs[i]);
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const fllf_job &b = jobs[j];
      if (fllf::spans_overlap(jobs[i].out, bi, b.in, fllf::in_span(b)) ||
          fllf::spans_overlap(jobs[i].out, bi, b.out, fllf::out_span(b)) ||
          fllf::spans_overlap(jobs[i].out, bi, b.m_map, fllf::map_span(b)) ||
          fllf::spans_overlap(jobs[i].out, bi, b.sigma_map, fllf::map_span(b)))
        return fail(ctx, FLLF_EINVAL, "job %d: output overlaps job %d's images", i, j);
    }
  }
  return FLLF_OK;
}

}  // extern "C"

namespace fllf {

fllf_storage ctx_storage(const fllf_ctx *ctx) { return ctx->storage; }
int ctx_device(const fllf_ctx *ctx) { return ctx->device; }
const Tuning &ctx_tuning(const fllf_ctx *ctx) { return ctx->tune; }
LaunchHook *ctx_hook(fllf_ctx *ctx) { return ctx->timing_on ? ctx->timer : nullptr; }

fllf_status ctx_fail(fllf_ctx *ctx, fllf_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return fail(ctx, st, "%s", buf);
}

fllf_status validate_jobs(fllf_ctx *ctx, const fllf_job *jobs, int n, fllf_storage storage) {
  return validate(ctx, jobs, n, storage);
}

}  // namespace fllf

extern "C" {

fllf_status fourier_llf_validate(const fllf_job *jobs, int n, fllf_storage storage) {
  return validate(nullptr, jobs, n, storage);
}

fllf_status fourier_llf_fit(double sigma_r, int K, double range_R, double T_in, double *T_out,
                            double *omega, double *alpha_tilde) {
  if (!is_finite(sigma_r) || sigma_r <= 0.0 || K < 1 || K > FLLF_MAX_K || !is_finite(range_R) ||
      range_R <= 0.0 || !is_finite(T_in) || (T_in != 0.0 && T_in <= range_R))
    return fail(nullptr, FLLF_EINVAL, "fit: need sigma_r > 0, 1 <= K <= %d, R > 0, T = 0 or T > R",
                FLLF_MAX_K);
  const double T = T_in > 0.0 ? T_in : fllf::fit_period(sigma_r, K, range_R);
  if (T_out) *T_out = T;
  fllf::fourier_terms(sigma_r, K, T, omega, alpha_tilde);
  return FLLF_OK;
}

fllf_status fourier_llf_fit_range(double sigma_lo, double sigma_hi, int K, double range_R, double *T_out) {
  if (!T_out || !is_finite(sigma_lo) || sigma_lo <= 0.0 || !is_finite(sigma_hi) || sigma_hi < sigma_lo || K < 1 ||
      K > FLLF_MAX_K || !is_finite(range_R) || range_R <= 0.0)
    return fail(nullptr, FLLF_EINVAL, "fit_range: need 0 < sigma_lo <= sigma_hi, 1 <= K <= %d, R > 0, T_out",
                FLLF_MAX_K);
  *T_out = fllf::fit_period_range(sigma_lo, sigma_hi, K, range_R);
  return FLLF_OK;
}

fllf_status fourier_llf_create(fllf_ctx **out, int device, fllf_storage storage) {
  if (!out) return fail(nullptr, FLLF_EINVAL, "create: out must be non-NULL");
  *out = nullptr;
  if (storage != FLLF_STORE_F32 && storage != FLLF_STORE_F16 && storage != FLLF_STORE_BF16)
    return fail(nullptr, FLLF_EINVAL, "create: unknown storage mode %d", (int)storage);
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count <= 0)
    return fail(nullptr, FLLF_EDEVICE, "create: no HIP device (%s)", hipGetErrorString(e));
  if (device < 0 || device >= count)
    return fail(nullptr, FLLF_EINVAL, "create: device %d outside [0, %d)", device, count);
  fllf_ctx *c = new fllf_ctx();
  c->device = device;
  c->storage = storage;
  c->tune = fllf::default_tuning(storage);
  *out = c;
  return FLLF_OK;
}

void fourier_llf_destroy(fllf_ctx *ctx) {
  if (!ctx) return;
  if (ctx->stage_ev) {
    (void)hipEventSynchronize(ctx->stage_ev);
    (void)hipEventDestroy(ctx->stage_ev);
  }
  if (ctx->stage) (void)hipHostFree(ctx->stage);
  delete ctx->timer;
  delete ctx;
}

fllf_status fourier_llf_timing_enable(fllf_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "timing_enable: ctx is NULL");
  if (enable && !ctx->timer) ctx->timer = new EventTimer();
  ctx->timing_on = enable != 0;
  // disabled: no further launch is hooked; unread records stay for timing_read
  if (!enable && ctx->timer) ctx->timer->pending = nullptr;
  return FLLF_OK;
}

fllf_status fourier_llf_timing_read(fllf_ctx *ctx, fllf_kernel_time *out, int max, int *n) {
  if (!ctx || !n || (max > 0 && !out)) return fail(ctx, FLLF_EINVAL, "timing_read: bad arguments");
  *n = 0;
  if (!ctx->timer) return FLLF_OK;
  EventTimer &t = *ctx->timer;
  if (t.err != hipSuccess) {
    hipError_t e = t.err;
    t.err = hipSuccess;
    return fail(ctx, FLLF_EDEVICE, "timing: event error %s", hipGetErrorString(e));
  }
  std::map<std::string, fllf_kernel_time> agg;
  for (auto &r : t.recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "timing: %s", hipGetErrorString(e));
    fllf_kernel_time &k = agg[r.name];
    std::snprintf(k.name, sizeof(k.name), "%s", r.name);
    k.launches += 1;
    k.total_ms += ms;
    k.bytes += r.bytes;
    t.pool.push_back(r.a);
    t.pool.push_back(r.b);
  }
  t.recs.clear();
  std::vector<fllf_kernel_time> v;
  for (auto &kv : agg) v.push_back(kv.second);
  std::sort(v.begin(), v.end(),
            [](const fllf_kernel_time &a, const fllf_kernel_time &b) { return a.total_ms > b.total_ms; });
  const int m = (int)v.size() < max ? (int)v.size() : max;
  for (int i = 0; i < m; ++i) out[i] = v[i];
  *n = (int)v.size();
  return FLLF_OK;
}

const char *fourier_llf_last_error(const fllf_ctx *ctx) {
  (void)ctx;
  return g_last_error.c_str();
}

// Plans every job; the jobs' workspaces follow the batch table (n >= 2).
static void plan_all(const fllf_job *jobs, int n, fllf_storage storage, std::vector<fllf::JobPlan> *plans,
                     size_t *table, size_t *total) {
  plans->resize(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    fllf::plan_job(jobs[i], storage, off, &(*plans)[i]);
    off += (*plans)[i].bytes;
  }
  *table = fllf::batch_table_bytes(plans->data(), n, storage);
  off = *table;
  for (int i = 0; i < n; ++i) {
    fllf::plan_job(jobs[i], storage, off, &(*plans)[i]);
    off += (*plans)[i].bytes;
  }
  *total = off;
}

static fllf_status footprint(fllf_ctx *c, const fllf_job *jobs, int n, fllf_storage storage,
                             size_t *bytes) {
  if (!bytes) return fail(c, FLLF_EINVAL, "workspace size: bytes is NULL");
  fllf_status st = validate(c, jobs, n, storage);
  if (st != FLLF_OK) return st;
  std::vector<fllf::JobPlan> plans;
  size_t table = 0;
  plan_all(jobs, n, storage, &plans, &table, bytes);
  return FLLF_OK;
}

fllf_status fourier_llf_footprint(const fllf_job *jobs, int n, fllf_storage storage, size_t *bytes) {
  return footprint(nullptr, jobs, n, storage, bytes);
}

fllf_status fourier_llf_workspace_size(const fllf_ctx *ctx, const fllf_job *jobs, int n,
                                       size_t *bytes) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "workspace_size: ctx is NULL");
  return footprint(const_cast<fllf_ctx *>(ctx), jobs, n, ctx->storage, bytes);
}

// The workspace checks shared by every entry point that launches work (need =
// the planned workspace bytes), then the device made current.
static fllf_status check_workspace(fllf_ctx *ctx, const char *who, const fllf_job *jobs, int n, void *workspace,
                                   size_t ws_bytes, size_t need) {
  if (need > 0 && !workspace) return fail(ctx, FLLF_EINVAL, "%s: workspace is NULL", who);
  if (ws_bytes < need)
    return fail(ctx, FLLF_ENOMEM, "%s: workspace has %zu bytes, %zu needed", who, ws_bytes, need);
  if (((uintptr_t)workspace) % fllf::kAlign != 0)
    return fail(ctx, FLLF_EINVAL, "%s: workspace must be %zu-byte aligned", who, fllf::kAlign);
  // the workspace is written before the images are read: it must not overlap any of them
  const char *wsb = (const char *)workspace;
  auto hits = [&](const void *p, size_t bytes) {
    const char *q = (const char *)p;
    return need > 0 && q && q < wsb + need && wsb < q + bytes;
  };
  for (int i = 0; i < n; ++i) {
    if (hits(jobs[i].out, fllf::out_span(jobs[i])))
      return fail(ctx, FLLF_EINVAL, "%s: job %d output overlaps the workspace", who, i);
    if (hits(jobs[i].in, fllf::in_span(jobs[i])))
      return fail(ctx, FLLF_EINVAL, "%s: job %d input overlaps the workspace", who, i);
    if (hits(jobs[i].m_map, fllf::map_span(jobs[i])))
      return fail(ctx, FLLF_EINVAL, "%s: job %d boost map overlaps the workspace", who, i);
    if (hits(jobs[i].sigma_map, fllf::map_span(jobs[i])))
      return fail(ctx, FLLF_EINVAL, "%s: job %d range-scale map overlaps the workspace", who, i);
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "%s: hipSetDevice: %s", who, hipGetErrorString(e));
  e = hipGetLastError();  // surface earlier asynchronous faults
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "%s: pending HIP error: %s", who, hipGetErrorString(e));
  return FLLF_OK;
}

// Checks shared by run, autotune and graph capture; plans the jobs.
static fllf_status prepare(fllf_ctx *ctx, const char *who, const fllf_job *jobs, int n, void *workspace,
                           size_t ws_bytes, std::vector<fllf::JobPlan> *plans) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "%s: ctx is NULL", who);
  fllf_status st = validate(ctx, jobs, n, ctx->storage);
  if (st != FLLF_OK) return st;
  size_t table = 0, need = 0;
  plan_all(jobs, n, ctx->storage, plans, &table, &need);
  return check_workspace(ctx, who, jobs, n, workspace, ws_bytes, need);
}

}  // extern "C"

namespace fllf {

// One job planned on the stack and launched with no timing hook: no heap, pinned
// or device allocation on the success path.
fllf_status run_single(fllf_ctx *ctx, const char *who, const fllf_job &job, void *ws, size_t ws_bytes,
                       hipStream_t stream) {
  fllf_status st = validate(ctx, &job, 1, ctx->storage);
  if (st != FLLF_OK) return st;
  JobPlan P;
  plan_job(job, ctx->storage, 0, &P);
  if (P.bytes > ws_bytes)
    return fail(ctx, FLLF_ENOMEM, "%s: the job needs %zu bytes of workspace; the limit is %zu", who, P.bytes,
                ws_bytes);
  st = check_workspace(ctx, who, &job, 1, ws, ws_bytes, P.bytes);
  if (st != FLLF_OK) return st;
  const hipError_t e = launch_job(P, ctx->storage, (char *)ws, stream, nullptr, ctx->tune);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "%s: launch failed: %s", who, hipGetErrorString(e));
  return FLLF_OK;
}

}  // namespace fllf

extern "C" {

// Copies a batch table into the workspace on `stream` through the context's
// pinned staging buffer.
static fllf_status upload_table(fllf_ctx *ctx, const fllf::BatchSchedule &s, void *ws, hipStream_t stream) {
  if (s.table_bytes == 0) return FLLF_OK;
  hipError_t e = hipSuccess;
  if (ctx->stage_ev) e = hipEventSynchronize(ctx->stage_ev);  // the previous copy has read the buffer
  if (e == hipSuccess && ctx->stage_cap < s.table_bytes) {
    if (ctx->stage) e = hipHostFree(ctx->stage);
    ctx->stage = nullptr;
    ctx->stage_cap = 0;
    const size_t cap = std::max(s.table_bytes, (size_t)1 << 20);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->stage, cap, hipHostMallocDefault);
    if (e == hipSuccess) ctx->stage_cap = cap;
  }
  if (e == hipSuccess && !ctx->stage_ev) e = hipEventCreateWithFlags(&ctx->stage_ev, hipEventDisableTiming);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "batch table staging: %s", hipGetErrorString(e));
  std::memcpy(ctx->stage, s.blob.data(), s.table_bytes);
  e = hipMemcpyAsync(ws, ctx->stage, s.table_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipEventRecord(ctx->stage_ev, stream);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "batch table upload: %s", hipGetErrorString(e));
  return FLLF_OK;
}

// Enqueues planned jobs with the given tuning (no validation).
static fllf_status enqueue(fllf_ctx *ctx, const std::vector<fllf::JobPlan> &plans, void *workspace,
                           hipStream_t stream, const fllf::Tuning &tu, fllf::LaunchHook *hook) {
  const int n = (int)plans.size();
  hipError_t e = hipSuccess;
  if (n == 1) {
    e = fllf::launch_job(plans[0], ctx->storage, (char *)workspace, stream, hook, tu);
    if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "run: launch failed: %s", hipGetErrorString(e));
    return FLLF_OK;
  }
  fllf::BatchSchedule sched;
  fllf::build_batch(plans.data(), n, ctx->storage, (char *)workspace, tu, &sched);
  fllf_status st = upload_table(ctx, sched, workspace, stream);
  if (st != FLLF_OK) return st;
  e = fllf::launch_batch(sched, ctx->storage, (char *)workspace, stream, hook, tu);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "run: batched launch failed: %s", hipGetErrorString(e));
  return FLLF_OK;
}

fllf_status fourier_llf_run(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                            size_t ws_bytes, void *hip_stream) {
  std::vector<fllf::JobPlan> plans;
  fllf_status st = prepare(ctx, "run", jobs, n, workspace, ws_bytes, &plans);
  if (st != FLLF_OK) return st;
  return enqueue(ctx, plans, workspace, (hipStream_t)hip_stream, ctx->tune, fllf::ctx_hook(ctx));
}

fllf_status fourier_llf_reparam(fllf_ctx *ctx, const fllf_job *prev, const fllf_job *next, void *workspace,
                                size_t ws_bytes, void *hip_stream) {
  if (!prev || !next) return fail(ctx, FLLF_EINVAL, "reparam: prev and next must be non-NULL");
  std::vector<fllf::JobPlan> plans;
  fllf_status st = prepare(ctx, "reparam", next, 1, workspace, ws_bytes, &plans);
  if (st != FLLF_OK) return st;
  st = validate(ctx, prev, 1, ctx->storage);
  if (st != FLLF_OK) return st;
  const fllf_job &a = *prev, &b = *next;
  if (a.in != b.in || a.width != b.width || a.height != b.height || a.channels != b.channels ||
      a.levels != b.levels || a.K != b.K || a.range_R != b.range_R)
    return fail(ctx, FLLF_EINVAL, "reparam: input, size, channels, levels, K and R must match the resident job");
  if (a.m_map || b.m_map || a.sigma_map || b.sigma_map)
    return fail(ctx, FLLF_EUNSUPPORTED, "reparam: per-pixel maps are not supported");
  if (a.flags || b.flags) return fail(ctx, FLLF_EUNSUPPORTED, "reparam: Fourier LLF jobs only");
  if (b.K != 4 && b.K != 8 && b.K != 16) return fail(ctx, FLLF_EUNSUPPORTED, "reparam: K must be 4, 8 or 16");
  const double T = a.period_T > 0.0 ? a.period_T : fllf::fit_period(a.sigma_r, a.K, a.range_R);
  if (b.period_T != 0.0 && b.period_T != T)
    return fail(ctx, FLLF_EINVAL, "reparam: the period T (%.17g) must stay that of the resident pyramids", T);
  double at_prev[fllf::kMaxK], at_next[fllf::kMaxK];
  fllf::fourier_terms(a.sigma_r, a.K, T, nullptr, at_prev);
  fllf::fourier_terms(b.sigma_r, b.K, T, nullptr, at_next);
  fllf::JobPlan &P = plans[0];
  P.coefs.inv_T = (float)(1.0 / T);
  for (int k = 0; k < b.K; ++k) {
    const float stored = (float)at_prev[k];  // the factor the resident pyramids carry
    if (stored == 0.0f || !std::isfinite(at_next[k] / (double)stored)) {
      if ((float)at_next[k] != 0.0f)
        return fail(ctx, FLLF_EUNSUPPORTED, "reparam: term %d vanished in the resident pyramids", k + 1);
      P.coefs.wt[k] = 0.0f;
    } else {
      P.coefs.wt[k] = (float)(at_next[k] / (double)stored);
    }
    P.coefs.at[k] = (float)at_next[k];
  }
  hipError_t e = fllf::launch_reparam(P, ctx->storage, (char *)workspace, (hipStream_t)hip_stream, fllf::ctx_hook(ctx),
                                      ctx->tune);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "reparam: launch failed: %s", hipGetErrorString(e));
  return FLLF_OK;
}

fllf_status fourier_llf_set_tuning(fllf_ctx *ctx, const int32_t *params) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "set_tuning: ctx is NULL");
  const fllf::Tuning d = fllf::default_tuning(ctx->storage);
  fllf::Tuning t = d;
  if (params) {
    for (int i = 0; i < fllf::kTuneGridCap; ++i) t.p[i] = params[i] > 0 ? params[i] : d.p[i];
    if (params[fllf::kTuneGridCap] < 0 || params[fllf::kTuneGridCap] > 1024)
      return fail(ctx, FLLF_EINVAL, "set_tuning: grid cap %d outside [0, 1024]", params[fllf::kTuneGridCap]);
    t.p[fllf::kTuneGridCap] = params[fllf::kTuneGridCap];
    if (params[fllf::kTuneNtStores] > fllf::kNtAll)
      return fail(ctx, FLLF_EINVAL, "set_tuning: nt_stores %d outside [0, %d]", params[fllf::kTuneNtStores],
                  fllf::kNtAll);
    if (params[fllf::kTuneNtStores] >= 0) t.p[fllf::kTuneNtStores] = params[fllf::kTuneNtStores];
  }
  ctx->tune = t;
  return FLLF_OK;
}

fllf_status fourier_llf_get_tuning(const fllf_ctx *ctx, int32_t *params) {
  if (!ctx || !params) return fail(nullptr, FLLF_EINVAL, "get_tuning: ctx and params must be non-NULL");
  for (int i = 0; i < fllf::kTuneParams; ++i) params[i] = ctx->tune.p[i];
  return FLLF_OK;
}

fllf_status fourier_llf_autotune(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                 size_t ws_bytes, void *hip_stream, int reps, int32_t *chosen) {
  std::vector<fllf::JobPlan> plans;
  fllf_status st = prepare(ctx, "autotune", jobs, n, workspace, ws_bytes, &plans);
  if (st != FLLF_OK) return st;
  if (reps < 1 || reps > 1000) return fail(ctx, FLLF_EINVAL, "autotune: reps=%d outside [1, 1000]", reps);
  hipStream_t stream = (hipStream_t)hip_stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return fail(ctx, FLLF_EDEVICE, "autotune: %s", hipGetErrorString(e));
  }
  // milliseconds per run with tuning t, or a negative status
  auto timed = [&](const fllf::Tuning &t, float *ms) -> fllf_status {
    fllf_status s2 = enqueue(ctx, plans, workspace, stream, t, nullptr);
    if (s2 != FLLF_OK) return s2;
    hipError_t r = hipEventRecord(e0, stream);
    for (int i = 0; i < reps && r == hipSuccess && s2 == FLLF_OK; ++i)
      s2 = enqueue(ctx, plans, workspace, stream, t, nullptr);
    if (s2 != FLLF_OK) return s2;
    if (r == hipSuccess) r = hipEventRecord(e1, stream);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
    if (r != hipSuccess) return fail(ctx, FLLF_EDEVICE, "autotune: %s", hipGetErrorString(r));
    *ms /= reps;
    return FLLF_OK;
  };
  static const int kWaves[] = {512, 1024, 1536, 3072, 6144, 12288, 24576};
  static const int kCaps[] = {0, 1, 2, 4};
  using fllf::kNtDown0, fllf::kNtDownFused, fllf::kNtUp0, fllf::kNtUp;
  static const int kNt[] = {0, 1 << kNtUp0, (1 << kNtDownFused) | (1 << kNtUp0), (1 << kNtDown0) | (1 << kNtUp0),
                            (1 << kNtDown0) | (1 << kNtDownFused) | (1 << kNtUp0),
                            (1 << kNtDownFused) | (1 << kNtUp0) | (1 << kNtUp), fllf::kNtAll};
  fllf::Tuning best = ctx->tune;
  float best_ms = 0.f;
  st = timed(best, &best_ms);
  for (int p = 0; p < fllf::kTuneParams && st == FLLF_OK; ++p) {
    if (p == fllf::kTuneGridCap && n == 1) continue;  // single jobs launch one wave per work item
    const int *cand = p == fllf::kTuneGridCap ? kCaps : p == fllf::kTuneNtStores ? kNt : kWaves;
    const int nc = p == fllf::kTuneGridCap ? 4 : 7;
    for (int i = 0; i < nc && st == FLLF_OK; ++i) {
      if (cand[i] == best.p[p]) continue;
      fllf::Tuning t = best;
      t.p[p] = cand[i];
      float ms = 0.f;
      st = timed(t, &ms);
      if (st == FLLF_OK && ms < best_ms) {
        best_ms = ms;
        best = t;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FLLF_OK) return st;
  ctx->tune = best;
  if (chosen)
    for (int i = 0; i < fllf::kTuneParams; ++i) chosen[i] = best.p[i];
  return FLLF_OK;
}

// Key of a job set's launch shape: FNV-1a over the device (architecture and
// compute units), the storage and, per job, everything planning depends on.
static uint64_t tuning_key(const fllf_ctx *ctx, const fllf_job *jobs, int n) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t len) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) {
    mix(prop.gcnArchName, std::strlen(prop.gcnArchName));
    mix(&prop.multiProcessorCount, sizeof(prop.multiProcessorCount));
  }
  const int st = (int)ctx->storage;
  mix(&st, sizeof(st));
  mix(&n, sizeof(n));
  for (int i = 0; i < n; ++i) {
    const fllf_job &j = jobs[i];
    const int32_t v[9] = {j.width, j.height, j.channels, j.levels, j.K, j.flags, j.m_map ? 1 : 0,
                          j.sigma_map ? 1 : 0, 0};
    mix(v, sizeof(v));
  }
  return h;
}

fllf_status fourier_llf_autotune_cached(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                        size_t ws_bytes, void *hip_stream, int reps, const char *cache_path,
                                        int32_t *chosen) {
  if (!ctx || !cache_path) return fail(ctx, FLLF_EINVAL, "autotune_cached: ctx and cache_path must be non-NULL");
  std::vector<fllf::JobPlan> plans;
  fllf_status st = prepare(ctx, "autotune_cached", jobs, n, workspace, ws_bytes, &plans);
  if (st != FLLF_OK) return st;
  char key[32];
  std::snprintf(key, sizeof(key), "%016llx", (unsigned long long)tuning_key(ctx, jobs, n));
  if (FILE *f = std::fopen(cache_path, "r")) {
    char line[256];
    bool found = false;
    int32_t p[fllf::kTuneParams] = {0};
    while (!found && std::fgets(line, sizeof(line), f)) {
      char k[32];
      int v[fllf::kTuneParams];
      static_assert(fllf::kTuneParams == 6, "the cache line format lists every parameter");
      if (std::sscanf(line, "%31s %d %d %d %d %d %d", k, &v[0], &v[1], &v[2], &v[3], &v[4], &v[5]) ==
              1 + fllf::kTuneParams &&
          std::strcmp(k, key) == 0) {
        for (int i = 0; i < fllf::kTuneParams; ++i) p[i] = v[i];
        found = true;
      }
    }
    std::fclose(f);
    if (found) {
      st = fourier_llf_set_tuning(ctx, p);  // checks the values read
      if (st == FLLF_OK && chosen)
        for (int i = 0; i < fllf::kTuneParams; ++i) chosen[i] = ctx->tune.p[i];
      return st;
    }
  }
  int32_t best[fllf::kTuneParams];
  st = fourier_llf_autotune(ctx, jobs, n, workspace, ws_bytes, hip_stream, reps, best);
  if (st != FLLF_OK) return st;
  if (chosen)
    for (int i = 0; i < fllf::kTuneParams; ++i) chosen[i] = best[i];
  FILE *f = std::fopen(cache_path, "a");
  if (!f) return fail(ctx, FLLF_EINVAL, "autotune_cached: cannot append to %s", cache_path);
  char line[128];
  const int len = std::snprintf(line, sizeof(line), "%s %d %d %d %d %d %d\n", key, best[0], best[1], best[2],
                                best[3], best[4], best[5]);
  const bool ok = std::fwrite(line, 1, (size_t)len, f) == (size_t)len;
  if (std::fclose(f) != 0 || !ok) return fail(ctx, FLLF_EINVAL, "autotune_cached: cannot write %s", cache_path);
  return FLLF_OK;
}

fllf_status fourier_llf_graph_create(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                                     size_t ws_bytes, fllf_graph **out) {
  if (!out) return fail(ctx, FLLF_EINVAL, "graph_create: out is NULL");
  *out = nullptr;
  std::vector<fllf::JobPlan> plans;
  fllf_status st = prepare(ctx, "graph_create", jobs, n, workspace, ws_bytes, &plans);
  if (st != FLLF_OK) return st;
  fllf::BatchSchedule sched;
  hipError_t e = hipSuccess;
  if (n > 1) {
    fllf::build_batch(plans.data(), n, ctx->storage, (char *)workspace, ctx->tune, &sched);
    e = hipMemcpy(workspace, sched.blob.data(), sched.table_bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "graph_create: table upload: %s", hipGetErrorString(e));
  }
  hipStream_t cs = nullptr;
  e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "graph_create: stream: %s", hipGetErrorString(e));
  fllf_graph *g = new fllf_graph();
  g->device = ctx->device;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    e = n == 1 ? fllf::launch_job(plans[0], ctx->storage, (char *)workspace, cs, nullptr, ctx->tune)
               : fllf::launch_batch(sched, ctx->storage, (char *)workspace, cs, nullptr, ctx->tune);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);
    g->graph = graph;
    if (e == hipSuccess) e = e2;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    fourier_llf_graph_destroy(g);
    return fail(ctx, FLLF_EDEVICE, "graph_create: capture: %s", hipGetErrorString(e));
  }
  *out = g;
  return FLLF_OK;
}

fllf_status fourier_llf_graph_launch(fllf_graph *g, void *hip_stream) {
  if (!g || !g->exec) return fail(nullptr, FLLF_EINVAL, "graph_launch: graph is NULL");
  hipError_t e = hipSetDevice(g->device);
  if (e == hipSuccess) e = hipGraphLaunch(g->exec, (hipStream_t)hip_stream);
  if (e != hipSuccess) return fail(nullptr, FLLF_EDEVICE, "graph_launch: %s", hipGetErrorString(e));
  return FLLF_OK;
}

void fourier_llf_graph_destroy(fllf_graph *g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
