// gfx950 kernels of the Fourier local Laplacian filter.
//
// Per job and channel the filter runs, level by level:
//   down(0):   I -> level 1 of the 2K+1 pyramids.  cos/sin(omega_k I) are formed in
//              registers (never stored); REDUCE of Eq. (1) on every plane.
//   down(l):   level l -> level l+1 of the 2K+1 pyramids (l >= 1).
//   up(l):     for l = top-1 .. 0: the output Laplacian level of Eq. (14) at every
//              level-l pixel (EXPAND of Eq. (2) of all coarse planes + product-sum with
//              cos/sin(omega_k G_l[I])), plus the collapse step of Eq. (4):
//              O_l = L_l[O] + EXPAND(O_{l+1}).
#include <hip/hip_runtime.h>

#include "fllf_internal.h"

namespace fllf {

// --------------------------------------------------------------------------
// Storage of the (C~, S~) pairs.  Arithmetic is always float32.
// --------------------------------------------------------------------------
template <int S> struct PairStore;

template <> struct PairStore<FLLF_STORE_F32> {
  using T = float2;
  __device__ static inline float2 ld(const T *p) { return *p; }
  __device__ static inline void st(T *p, float2 v) { *p = v; }
};

template <> struct PairStore<FLLF_STORE_F16> {
  using T = uint32_t;
  __device__ static inline float2 ld(const T *p) {
    uint32_t u = *p;
    _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
    _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
    return make_float2((float)lo, (float)hi);
  }
  __device__ static inline void st(T *p, float2 v) {
    uint16_t lo = __builtin_bit_cast(uint16_t, (_Float16)v.x);
    uint16_t hi = __builtin_bit_cast(uint16_t, (_Float16)v.y);
    *p = (uint32_t)lo | ((uint32_t)hi << 16);
  }
};

template <> struct PairStore<FLLF_STORE_BF16> {
  using T = uint32_t;
  // round to nearest even; inputs are finite
  __device__ static inline uint32_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
  }
  __device__ static inline float2 ld(const T *p) {
    uint32_t u = *p;
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  }
  __device__ static inline void st(T *p, float2 v) { *p = to_bf16(v.x) | (to_bf16(v.y) << 16); }
};

// Reflect-101 fold onto [0, n):  ... 2 1 | 0 1 2 ... n-1 | n-2 ...
__device__ inline int fold(int i, int n) {
  if (n == 1) return 0;
  const int p = 2 * n - 2;
  i %= p;
  if (i < 0) i += p;
  return i > n - 1 ? p - i : i;
}

__device__ inline float binom(int d) {  // [1 4 6 4 1] / 16, d = 0..4
  return d == 2 ? 0.375f : (d == 1 || d == 3) ? 0.25f : 0.0625f;
}

// --------------------------------------------------------------------------
// down(0): one thread per level-1 pixel; 5x5 taps of I with the trig terms
// formed per tap from one accurate sincos and the angle-addition recurrence.
// --------------------------------------------------------------------------
template <int S, int KM>
__global__ void __launch_bounds__(256)
down0_kernel(const float *__restrict__ in, int W0, int H0, float *__restrict__ G1,
             typename PairStore<S>::T *__restrict__ CS1, int W1, int H1, size_t g_cs, size_t cs_ks,
             size_t cs_cs, Coefs cf, const float *__restrict__ mmap, float *__restrict__ M1) {
  using PS = PairStore<S>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int c = blockIdx.z;
  if (x >= W1 || y >= H1) return;
  const float *I = in + (size_t)c * W0 * H0;
  float g = 0.f, mm = 0.f;
  float ac[KM], as[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) ac[k] = as[k] = 0.f;
  for (int dy = 0; dy < 5; ++dy) {
    const int yy = fold(2 * y + dy - 2, H0);
    for (int dx = 0; dx < 5; ++dx) {
      const int xx = fold(2 * x + dx - 2, W0);
      const float wt = binom(dy) * binom(dx);
      const float v = I[(size_t)yy * W0 + xx];
      g += wt * v;
      if (mmap) mm += wt * mmap[(size_t)yy * W0 + xx];
      float s1, c1;
      sincospif(2.0f * v * cf.inv_T, &s1, &c1);
      float ck = c1, sk = s1;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < cf.K) {
          ac[k] += wt * ck;
          as[k] += wt * sk;
        }
        const float cn = ck * c1 - sk * s1;
        sk = sk * c1 + ck * s1;
        ck = cn;
      }
    }
  }
  const size_t p = (size_t)y * W1 + x;
  G1[c * g_cs + p] = g;
  for (int k = 0; k < cf.K && k < KM; ++k) PS::st(CS1 + c * cs_cs + k * cs_ks + p, make_float2(ac[k], as[k]));
  if (M1 && c == 0) M1[p] = mm;
}

// --------------------------------------------------------------------------
// down(l), l >= 1: one thread per level-(l+1) pixel, 5x5 taps of each plane.
// --------------------------------------------------------------------------
template <int S, int KM>
__global__ void __launch_bounds__(256)
down_kernel(const float *__restrict__ Gf, const typename PairStore<S>::T *__restrict__ CSf, int Wf,
            int Hf, size_t gf_cs, size_t csf_ks, size_t csf_cs, float *__restrict__ Gc,
            typename PairStore<S>::T *__restrict__ CSc, int Wc, int Hc, size_t gc_cs, size_t csc_ks,
            size_t csc_cs, int K, const float *__restrict__ Mf, float *__restrict__ Mc) {
  using PS = PairStore<S>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int c = blockIdx.z;
  if (x >= Wc || y >= Hc) return;
  int xs[5], ys[5];
#pragma unroll
  for (int d = 0; d < 5; ++d) {
    xs[d] = fold(2 * x + d - 2, Wf);
    ys[d] = fold(2 * y + d - 2, Hf);
  }
  const size_t p = (size_t)y * Wc + x;
  {
    const float *G = Gf + c * gf_cs;
    float g = 0.f;
    for (int dy = 0; dy < 5; ++dy)
      for (int dx = 0; dx < 5; ++dx) g += binom(dy) * binom(dx) * G[(size_t)ys[dy] * Wf + xs[dx]];
    Gc[c * gc_cs + p] = g;
  }
  if (Mf && Mc && c == 0) {
    float g = 0.f;
    for (int dy = 0; dy < 5; ++dy)
      for (int dx = 0; dx < 5; ++dx) g += binom(dy) * binom(dx) * Mf[(size_t)ys[dy] * Wf + xs[dx]];
    Mc[p] = g;
  }
  for (int k = 0; k < K; ++k) {
    const typename PS::T *P = CSf + c * csf_cs + k * csf_ks;
    float2 a = make_float2(0.f, 0.f);
    for (int dy = 0; dy < 5; ++dy)
      for (int dx = 0; dx < 5; ++dx) {
        const float wt = binom(dy) * binom(dx);
        const float2 v = PS::ld(P + (size_t)ys[dy] * Wf + xs[dx]);
        a.x += wt * v.x;
        a.y += wt * v.y;
      }
    PS::st(CSc + c * csc_cs + k * csc_ks + p, a);
  }
}

// --------------------------------------------------------------------------
// up(l): one thread per level-l pixel.  EXPAND of every coarse plane by the
// zero-insertion definition (taps that land on even positions of the folded
// fine grid), then the Eq. (14) product-sum and the collapse step.
// --------------------------------------------------------------------------
template <int S, int KM>
__global__ void __launch_bounds__(256)
up_kernel(int level0, const float *__restrict__ Gf, const typename PairStore<S>::T *__restrict__ CSf,
          int Wf, int Hf, size_t gf_cs, size_t csf_ks, size_t csf_cs, const float *__restrict__ Gc,
          const typename PairStore<S>::T *__restrict__ CSc, const float *__restrict__ Oc, int Wc,
          int Hc, size_t gc_cs, size_t csc_ks, size_t csc_cs, float *__restrict__ Of, size_t of_cs,
          const float *__restrict__ Mf, Coefs cf) {
  using PS = PairStore<S>;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int c = blockIdx.z;
  if (x >= Wf || y >= Hf) return;
  float eg = 0.f, eo = 0.f;
  float ec[KM], es[KM];
#pragma unroll
  for (int k = 0; k < KM; ++k) ec[k] = es[k] = 0.f;
  for (int dy = 0; dy < 5; ++dy) {
    const int qy = fold(y + dy - 2, Hf);
    if (qy & 1) continue;
    for (int dx = 0; dx < 5; ++dx) {
      const int qx = fold(x + dx - 2, Wf);
      if (qx & 1) continue;
      const float wt = 4.0f * binom(dy) * binom(dx);
      const size_t ci = (size_t)(qy >> 1) * Wc + (qx >> 1);
      eg += wt * Gc[c * gc_cs + ci];
      eo += wt * Oc[c * gc_cs + ci];
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < cf.K) {
          const float2 v = PS::ld(CSc + c * csc_cs + k * csc_ks + ci);
          ec[k] += wt * v.x;
          es[k] += wt * v.y;
        }
      }
    }
  }
  const size_t p = (size_t)y * Wf + x;
  const float g = Gf[c * gf_cs + p];
  float s1, c1;
  sincospif(2.0f * g * cf.inv_T, &s1, &c1);
  float ck = c1, sk = s1, acc = 0.f;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k < cf.K) {
      if (level0) {
        // Eq. (14), l = 0: + sum_k at_k (sin(w_k g) C~_{1,k}^ - cos(w_k g) S~_{1,k}^)
        acc += cf.at[k] * (sk * ec[k] - ck * es[k]);
      } else {
        // Eq. (14), 1 <= l < top: - sum_k at_k (sin(w_k g) L_l[C] - cos(w_k g) L_l[S])
        const float2 v = PS::ld(CSf + c * csf_cs + k * csf_ks + p);
        acc -= cf.at[k] * (sk * (v.x - ec[k]) - ck * (v.y - es[k]));
      }
    }
    const float cn = ck * c1 - sk * s1;
    sk = sk * c1 + ck * s1;
    ck = cn;
  }
  const float mp = cf.has_map ? Mf[p] : cf.m;
  Of[c * of_cs + p] = (g - eg) + mp * acc + eo;
}

// --------------------------------------------------------------------------
// Host-side launch sequence of one job.
// --------------------------------------------------------------------------
template <int S, int KM>
static hipError_t launch_typed(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *hook) {
  using T = typename PairStore<S>::T;
  const double pb = 2.0 * (S == FLLF_STORE_F32 ? 4 : 2) * P.K;  // bytes of the K pairs per pixel
  const double C = P.C;
  auto pre = [&]() { if (hook) hook->before(st); };
  auto post = [&](const char *name, double bytes) { if (hook) hook->after(st, name, bytes); };
  const int L = P.levels;
  const dim3 blk(16, 16, 1);
  auto grid = [&](int w, int h) { return dim3((w + 15) / 16, (h + 15) / 16, P.C); };
  auto G = [&](int l) { return (float *)(ws + P.lv[l].off_g); };
  auto CS = [&](int l) { return (T *)(ws + P.lv[l].off_cs); };
  auto O = [&](int l) { return (float *)(ws + P.lv[l].off_o); };
  auto M = [&](int l) -> float * {
    if (!P.m_map) return nullptr;
    if (l == 0) return const_cast<float *>(P.m_map);
    return l < L - 1 ? (float *)(ws + P.lv[l].off_m) : nullptr;
  };
  const Level *lv = P.lv;
  // Algorithmic bytes: every plane element a launch must read or write, once.
  // down(0)
  pre();
  down0_kernel<S, KM><<<grid(lv[1].w, lv[1].h), blk, 0, st>>>(
      P.in, lv[0].w, lv[0].h, G(1), CS(1), lv[1].w, lv[1].h, lv[1].g_cstride, lv[1].cs_kstride,
      lv[1].cs_cstride, P.coefs, P.m_map, M(1));
  post("down0", C * (4.0 * lv[0].n + (4.0 + pb) * lv[1].n));
  for (int l = 1; l + 1 < L; ++l) {
    pre();
    down_kernel<S, KM><<<grid(lv[l + 1].w, lv[l + 1].h), blk, 0, st>>>(
        G(l), CS(l), lv[l].w, lv[l].h, lv[l].g_cstride, lv[l].cs_kstride, lv[l].cs_cstride, G(l + 1),
        CS(l + 1), lv[l + 1].w, lv[l + 1].h, lv[l + 1].g_cstride, lv[l + 1].cs_kstride,
        lv[l + 1].cs_cstride, P.K, M(l), M(l + 1));
    post("down", C * (4.0 + pb) * (lv[l].n + lv[l + 1].n));
  }
  for (int l = L - 2; l >= 0; --l) {
    const float *Gf = l == 0 ? P.in : G(l);
    const T *CSf = l == 0 ? nullptr : CS(l);
    const size_t gf_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    const float *Oc = (l + 1 == L - 1) ? G(l + 1) : O(l + 1);
    float *Of = l == 0 ? P.out : O(l);
    const size_t of_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    pre();
    up_kernel<S, KM><<<grid(lv[l].w, lv[l].h), blk, 0, st>>>(
        l == 0, Gf, CSf, lv[l].w, lv[l].h, gf_cs, lv[l].cs_kstride, lv[l].cs_cstride, G(l + 1),
        CS(l + 1), Oc, lv[l + 1].w, lv[l + 1].h, lv[l + 1].g_cstride, lv[l + 1].cs_kstride,
        lv[l + 1].cs_cstride, Of, of_cs, M(l), P.coefs);
    const double fine = l == 0 ? 4.0 : 4.0 + pb;                    // I, or G_l and the K pairs
    const double coarse = 4.0 + pb + (l + 1 == L - 1 ? 0.0 : 4.0);  // G, pairs, O_{l+1}
    post(l == 0 ? "up0" : "up", C * ((fine + 4.0) * lv[l].n + coarse * lv[l + 1].n));
  }
  return hipGetLastError();
}

template <int S>
static hipError_t launch_k(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h) {
  if (P.K <= 4) return launch_typed<S, 4>(P, ws, st, h);
  if (P.K <= 8) return launch_typed<S, 8>(P, ws, st, h);
  if (P.K <= 16) return launch_typed<S, 16>(P, ws, st, h);
  return launch_typed<S, 32>(P, ws, st, h);
}

hipError_t launch_job(const JobPlan &P, fllf_storage storage, char *ws, hipStream_t st, LaunchHook *h) {
  if (P.levels == 1) {
    return hipMemcpyAsync(P.out, P.in, P.lv[0].n * P.C * sizeof(float), hipMemcpyDeviceToDevice, st);
  }
  switch (storage) {
    case FLLF_STORE_F16: return launch_k<FLLF_STORE_F16>(P, ws, st, h);
    case FLLF_STORE_BF16: return launch_k<FLLF_STORE_BF16>(P, ws, st, h);
    default: return launch_k<FLLF_STORE_F32>(P, ws, st, h);
  }
}

}  // namespace fllf
