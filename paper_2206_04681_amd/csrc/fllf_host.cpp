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
  EventTimer *timer = nullptr;
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
// ---------------------------------------------------------------------------
static double stationarity(double T, double a, double s, double R) {
  return std::log(a * s / (T * T)) - (a * a) / (T * T) + (T - R) * (T - R) / (s * s);
}

static double period_error(double T, double a, double s, double R) {
  return std::erfc(a / T) + std::erfc((T - R) / s);
}

double fit_period(double s, int K, double R) {
  const double a = M_PI * s * (2.0 * K + 1.0);
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
  p->K = job.K;
  p->C = job.channels;
  p->in = job.in;
  p->out = job.out;
  p->m_map = job.m_map;
  const size_t pair_bytes = 2 * (size_t)storage_bytes(storage);
  int w = job.width, h = job.height;
  size_t off = base;
  for (int l = 0; l < job.levels; ++l) {
    Level &L = p->lv[l];
    L.w = w;
    L.h = h;
    L.pitch = l == 0 ? w : (int)align_up((size_t)w, 64);
    L.n = (size_t)w * h;
    const size_t g_plane = align_up((size_t)L.pitch * h * 4);
    const size_t cs_plane = align_up((size_t)L.pitch * h * pair_bytes * job.K);
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
      }
    }
    w = (w + 1) / 2;
    h = (h + 1) / 2;
  }
  p->bytes = off - base;

  const double T = job.period_T > 0.0 ? job.period_T : fit_period(job.sigma_r, job.K, job.range_R);
  double at[kMaxK];
  fourier_terms(job.sigma_r, job.K, T, nullptr, at);
  p->coefs.inv_T = (float)(1.0 / T);
  p->coefs.m = (float)job.m;
  p->coefs.K = job.K;
  p->coefs.has_map = job.m_map ? 1 : 0;
  for (int k = 0; k < kMaxK; ++k) p->coefs.at[k] = k < job.K ? (float)at[k] : 0.0f;
}

const char *const kDownNames[kMaxLevels] = {
    "down_l0", "down_l1", "down_l2",  "down_l3",  "down_l4",  "down_l5",  "down_l6",  "down_l7",
    "down_l8", "down_l9", "down_l10", "down_l11", "down_l12", "down_l13", "down_l14", "down_l15"};
const char *const kUpNames[kMaxLevels] = {"up_l0", "up_l1", "up_l2",  "up_l3",  "up_l4",  "up_l5",
                                          "up_l6", "up_l7", "up_l8",  "up_l9",  "up_l10", "up_l11",
                                          "up_l12", "up_l13", "up_l14", "up_l15"};

hipError_t launch_job(const JobPlan &P, fllf_storage storage, char *ws, hipStream_t st, LaunchHook *h) {
  if (P.levels == 1)
    return hipMemcpyAsync(P.out, P.in, P.lv[0].n * P.C * sizeof(float), hipMemcpyDeviceToDevice, st);
  switch (storage) {
    case FLLF_STORE_F16: return launch_job_f16(P, ws, st, h);
    case FLLF_STORE_BF16: return launch_job_bf16(P, ws, st, h);
    default: return launch_job_f32(P, ws, st, h);
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
    if (j.K < 1 || j.K > FLLF_MAX_K)
      return fail(ctx, FLLF_EINVAL, "job %d: K=%d outside [1, %d]", i, j.K, FLLF_MAX_K);
    if (j.flags != 0) return fail(ctx, FLLF_EINVAL, "job %d: flags must be 0", i);
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
      const uint64_t rec_plane = fllf::align_up(w1, 64) * h1 * (uint64_t)j.K * 2u * storage_bytes(storage);
      if (rec_plane >= ((uint64_t)1 << 32))
        return fail(ctx, FLLF_EINVAL, "job %d: %d x %d with K=%d needs a level-1 plane of %llu bytes (limit 4 GiB)",
                    i, j.width, j.height, j.K, (unsigned long long)rec_plane);
    }
    const size_t bytes = (size_t)j.width * j.height * j.channels * sizeof(float);
    const char *a = (const char *)j.in, *b = (const char *)j.out;
    if (a < b + bytes && b < a + bytes)
      return fail(ctx, FLLF_EINVAL, "job %d: in and out overlap", i);
  }
  return FLLF_OK;
}

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
  *out = c;
  return FLLF_OK;
}

void fourier_llf_destroy(fllf_ctx *ctx) {
  if (!ctx) return;
  delete ctx->timer;
  delete ctx;
}

fllf_status fourier_llf_timing_enable(fllf_ctx *ctx, int enable) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "timing_enable: ctx is NULL");
  if (enable && !ctx->timer) ctx->timer = new EventTimer();
  if (!enable && ctx->timer && ctx->timer->recs.empty()) {
    delete ctx->timer;
    ctx->timer = nullptr;
  }
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

static fllf_status footprint(fllf_ctx *c, const fllf_job *jobs, int n, fllf_storage storage,
                             size_t *bytes) {
  if (!bytes) return fail(c, FLLF_EINVAL, "workspace size: bytes is NULL");
  fllf_status st = validate(c, jobs, n, storage);
  if (st != FLLF_OK) return st;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    fllf::JobPlan p;
    fllf::plan_job(jobs[i], storage, total, &p);
    total += p.bytes;
  }
  *bytes = total;
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

fllf_status fourier_llf_run(fllf_ctx *ctx, const fllf_job *jobs, int n, void *workspace,
                            size_t ws_bytes, void *hip_stream) {
  if (!ctx) return fail(nullptr, FLLF_EINVAL, "run: ctx is NULL");
  fllf_status st = validate(ctx, jobs, n, ctx->storage);
  if (st != FLLF_OK) return st;
  size_t need = 0;
  fourier_llf_workspace_size(ctx, jobs, n, &need);
  if (need > 0 && !workspace) return fail(ctx, FLLF_EINVAL, "run: workspace is NULL");
  if (ws_bytes < need)
    return fail(ctx, FLLF_ENOMEM, "run: workspace has %zu bytes, %zu needed", ws_bytes, need);
  if (((uintptr_t)workspace) % fllf::kAlign != 0)
    return fail(ctx, FLLF_EINVAL, "run: workspace must be %zu-byte aligned", fllf::kAlign);
  for (int i = 0; i < n; ++i) {
    const char *wsb = (const char *)workspace, *o = (const char *)jobs[i].out;
    size_t ob = (size_t)jobs[i].width * jobs[i].height * jobs[i].channels * sizeof(float);
    if (need > 0 && o < wsb + need && wsb < o + ob)
      return fail(ctx, FLLF_EINVAL, "run: job %d output overlaps the workspace", i);
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "run: hipSetDevice: %s", hipGetErrorString(e));
  e = hipGetLastError();  // surface earlier asynchronous faults
  if (e != hipSuccess) return fail(ctx, FLLF_EDEVICE, "run: pending HIP error: %s", hipGetErrorString(e));
  hipStream_t stream = (hipStream_t)hip_stream;
  size_t base = 0;
  for (int i = 0; i < n; ++i) {
    fllf::JobPlan p;
    fllf::plan_job(jobs[i], ctx->storage, base, &p);
    base += p.bytes;
    e = fllf::launch_job(p, ctx->storage, (char *)workspace, stream, ctx->timer);
    if (e != hipSuccess)
      return fail(ctx, FLLF_EDEVICE, "run: launch of job %d failed: %s", i, hipGetErrorString(e));
  }
  return FLLF_OK;
}

}  // extern "C"
