// gfx950 kernels of the Fourier local Laplacian filter.
//
// Per job the filter runs, level by level (all channels of a job in one launch):
//   down(0):  I -> level 1 of the 2K+1 pyramids G_l[I], C~_{l,k}, S~_{l,k}.
//             cos/sin(omega_k I) are formed in registers and never stored
//             (REDUCE of Eq. (1) on every plane).
//   down(l):  level l -> level l+1 of the 2K+1 pyramids, l >= 1.  The same pass
//             also evaluates, at every level-l pixel p, the level-l half of
//             Eq. (14):  A_l = G_l - m sum_k at_k (sin(w_k g) C~_{l,k} - cos(w_k g) S~_{l,k}),
//             g = G_l[I]_p, into the O_l slot (it reads those planes anyway).
//   up(l):    l = top-1 .. 0: O_l = A_l + EXPAND(O_{l+1} - G_{l+1})
//                                   + m sum_k at_k (sin(w_k g) C~^_{l+1,k} - cos(w_k g) S~^_{l+1,k})
//             which is L_l[O] of Eq. (14) plus the collapse step of Eq. (4)
//             (level 0: A_0 = I and the level-0 Fourier terms vanish, first case of Eq. (14)).
//
// Memory-bound multi-plane stencils; no LDS and no MFMA.  One wave64 owns a
// column strip of 62 coarse columns (lane t <-> coarse column j0 + t - 1; lanes 0
// and 63 are halo) and streams down a segment of coarse rows.  Horizontal taps
// come from the neighbouring lanes through DPP wave shifts; vertical taps are
// register-resident running sums.  Borders are reflect-101 (REDUCE) and the
// matching fold on the coarse grid (EXPAND).
#include <hip/hip_runtime.h>

#include "fllf_internal.h"

namespace fllf {

// --------------------------------------------------------------------------
// Storage of the (C~, S~) pairs.  Arithmetic is always float32.
// --------------------------------------------------------------------------
template <int S> struct PairStore;

template <> struct PairStore<FLLF_STORE_F32> {
  using T = float2;
  __device__ static inline void st(T *p, float c, float s) { *p = make_float2(c, s); }
  __device__ static inline float2 ld(const T *p) { return *p; }
  // the pairs at columns x0, x0+1 of a row (vec: contiguous and aligned)
  __device__ static inline void ld2(const T *row, int x0, int f0, int f1, bool vec, float2 &a, float2 &b) {
    if (vec) {
      const float4 v = *reinterpret_cast<const float4 *>(row + x0);
      a = make_float2(v.x, v.y);
      b = make_float2(v.z, v.w);
    } else {
      a = row[f0];
      b = row[f1];
    }
  }
};

__device__ inline float2 h2_to_f2(uint32_t u) {
  const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(u & 0xffffu));
  const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(u >> 16));
  return make_float2((float)lo, (float)hi);
}

template <> struct PairStore<FLLF_STORE_F16> {
  using T = uint32_t;
  __device__ static inline void st(T *p, float c, float s) {
    const uint16_t lo = __builtin_bit_cast(uint16_t, (_Float16)c);
    const uint16_t hi = __builtin_bit_cast(uint16_t, (_Float16)s);
    *p = (uint32_t)lo | ((uint32_t)hi << 16);
  }
  __device__ static inline float2 ld(const T *p) { return h2_to_f2(*p); }
  __device__ static inline void ld2(const T *row, int x0, int f0, int f1, bool vec, float2 &a, float2 &b) {
    if (vec) {
      const uint2 v = *reinterpret_cast<const uint2 *>(row + x0);
      a = h2_to_f2(v.x);
      b = h2_to_f2(v.y);
    } else {
      a = h2_to_f2(row[f0]);
      b = h2_to_f2(row[f1]);
    }
  }
};

__device__ inline float2 b2_to_f2(uint32_t u) {
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

template <> struct PairStore<FLLF_STORE_BF16> {
  using T = uint32_t;
  __device__ static inline uint32_t to_bf16(float f) {  // round to nearest even; finite inputs
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
  }
  __device__ static inline void st(T *p, float c, float s) { *p = to_bf16(c) | (to_bf16(s) << 16); }
  __device__ static inline float2 ld(const T *p) { return b2_to_f2(*p); }
  __device__ static inline void ld2(const T *row, int x0, int f0, int f1, bool vec, float2 &a, float2 &b) {
    if (vec) {
      const uint2 v = *reinterpret_cast<const uint2 *>(row + x0);
      a = b2_to_f2(v.x);
      b = b2_to_f2(v.y);
    } else {
      a = b2_to_f2(row[f0]);
      b = b2_to_f2(row[f1]);
    }
  }
};

// --------------------------------------------------------------------------
// Index helpers
// --------------------------------------------------------------------------
// Reflect-101 fold of a fine-grid index onto [0, n):  ... 2 1 | 0 1 2 ... n-1 | n-2 ...
__device__ inline int fold(int i, int n) {
  if (n == 1) return 0;
  const int p = 2 * n - 2;
  i %= p;
  if (i < 0) i += p;
  return i > n - 1 ? p - i : i;
}

// Coarse index feeding EXPAND to a fine axis of nf samples (nc = ceil(nf/2), nf >= 2).
// Reflect-101 on the zero-inserted fine grid sends the tap left of coarse 0 to
// coarse 1 and the tap right of coarse nc-1 to nc-1 (nf even) or nc-2 (nf odd).
// Indices further out only feed lanes whose outputs are discarded: clamp them.
__device__ inline int cfold(int i, int nc, int nf) {
  if (i < 0) return nc >= 2 ? 1 : 0;
  if (i == nc) return (nf & 1) ? nc - 2 : nc - 1;
  return i > nc ? nc - 1 : i;
}

// DPP wave shifts: lane t receives lane t-1 (from_left) or lane t+1 (from_right).
__device__ inline float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}
__device__ inline float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, false));
}

// sin and cos of 2 pi u (u in revolutions, |u| < 256: hardware range).
__device__ inline void sincos2pi(float u, float &s, float &c) {
  s = __builtin_amdgcn_sinf(u);
  c = __builtin_amdgcn_cosf(u);
}

// Unnormalised horizontal REDUCE at the lane's even fine column 2j from the lane's
// samples (v0 at 2j, v1 at 2j+1) and its neighbours': taps [1 4 6 4 1].
__device__ inline float hred(float v0, float v1) {
  const float l0 = from_left(v0), l1 = from_left(v1), r0 = from_right(v0);
  return fmaf(6.f, v0, fmaf(4.f, l1 + v1, l0 + r0));
}

__device__ inline float2 ld_f2(const float *row, int x0, int f0, int f1, bool vec) {
  if (vec) return *reinterpret_cast<const float2 *>(row + x0);
  return make_float2(row[f0], row[f1]);
}

// --------------------------------------------------------------------------
// Kernel arguments
// --------------------------------------------------------------------------
struct Geom {
  int Wf, Hf, Wc, Hc;  // fine and coarse sizes
  int pf, pc;          // row pitches (elements) of the fine and coarse planes
  int nstrips, nsegs;  // column strips (62 coarse columns each) and row segments
  int S;               // coarse rows per segment
  int C;               // channels
};

template <typename PT> struct DownArgs {
  const float *gf; size_t gf_cs;         // G_l (the input I at level 0)
  const PT *csf; size_t csf_ks, csf_cs;  // level-l pairs (l >= 1)
  const float *mf;                       // level-l boost plane (m_map at level 0)
  float *gc; size_t gc_cs;               // G_{l+1}
  PT *csc; size_t csc_ks, csc_cs;        // level-(l+1) pairs
  float *mc;                             // level-(l+1) boost plane or null
  float *af; size_t af_cs;               // A_l (l >= 1), stored in the O_l slot
  Geom g;
  Coefs cf;
};

// Vertical REDUCE as running sums over a stream of horizontally reduced rows.
// P0 accumulates coarse row i, P1 coarse row i+1.  Weights [1 4 6 4 1]/256
// carry the 2-D normalisation.  Roles (row of the stream):
//   0: 2 i0 - 2     1: 2 i0 - 1     2: 2 i0
//   3: 2 i + 1      4: 2 i + 2  (completes coarse row i, returned in out)
template <int ROLE>
__device__ inline void vstep(float h, float &P0, float &P1, float &out) {
  constexpr float w1 = 1.f / 256.f, w4 = 4.f / 256.f, w6 = 6.f / 256.f;
  if (ROLE == 0) {
    P0 = w1 * h;
  } else if (ROLE == 1) {
    P0 = fmaf(w4, h, P0);
  } else if (ROLE == 2) {
    P0 = fmaf(w6, h, P0);
    P1 = w1 * h;
  } else if (ROLE == 3) {
    P0 = fmaf(w4, h, P0);
    P1 = fmaf(w4, h, P1);
  } else {
    out = fmaf(w1, h, P0);
    P0 = fmaf(w6, h, P1);
    P1 = w1 * h;
  }
}

template <int ST, int KM, bool L0, bool MAP>
struct DownWave {
  using PS = PairStore<ST>;
  using PT = typename PS::T;
  const DownArgs<PT> &a;
  int lane, c, j, i0, i1, x0, f0, f1, K;
  bool writer, contig, vec_in;
  const float *gf, *mf;
  const PT *csf;
  float PG0, PG1, PM0, PM1;
  float PC0[KM], PC1[KM], PS0[KM], PS1[KM];

  __device__ DownWave(const DownArgs<PT> &args, int lane_, int c_, int strip, int seg) : a(args) {
    lane = lane_;
    c = c_;
    K = a.cf.K;
    j = strip * 62 + lane - 1;
    i0 = seg * a.g.S;
    i1 = min(i0 + a.g.S, a.g.Hc);
    writer = lane >= 1 && lane <= 62 && j < a.g.Wc;
    x0 = 2 * j;
    f0 = fold(x0, a.g.Wf);
    f1 = fold(x0 + 1, a.g.Wf);
    contig = x0 >= 0 && x0 + 1 < a.g.Wf;
    gf = a.gf + (size_t)c * a.gf_cs;
    mf = a.mf;
    csf = L0 ? nullptr : a.csf + (size_t)c * a.csf_cs;
    // the caller's image has arbitrary row pitch: vector loads only when aligned
    vec_in = contig && (!L0 || (((a.g.pf & 1) == 0) && ((reinterpret_cast<uintptr_t>(gf) & 7) == 0)));
  }

  // Process fine row r (stream role ROLE); for ROLE 4 store coarse row ci.
  template <int ROLE>
  __device__ inline void row(int r, int ci) {
    const int fr = fold(r, a.g.Hf);
    const float2 gv = ld_f2(gf + (size_t)fr * a.g.pf, x0, f0, f1, vec_in);
    float2 mv = make_float2(0.f, 0.f);
    float out, outm = 0.f;
    vstep<ROLE>(hred(gv.x, gv.y), PG0, PG1, out);
    if (MAP) {
      const bool vm = contig && (!L0 || (((a.g.pf & 1) == 0) && ((reinterpret_cast<uintptr_t>(mf) & 7) == 0)));
      mv = ld_f2(mf + (size_t)fr * a.g.pf, x0, f0, f1, vm);
      vstep<ROLE>(hred(mv.x, mv.y), PM0, PM1, outm);
    }
    const bool store = ROLE == 4 && writer;
    const size_t cp = (size_t)ci * a.g.pc + j;
    if (store) {
      a.gc[(size_t)c * a.gc_cs + cp] = out;
      if (MAP && a.mc && c == 0) a.mc[cp] = outm;
    }
    PT *csc = a.csc + (size_t)c * a.csc_cs + cp;
    // angle of term 1 at the two pixels, in revolutions; terms k from the
    // angle-addition recurrence (k+1) = (k) rotated by (1)
    float s10, c10, s11, c11;
    sincos2pi(gv.x * a.cf.inv_T, s10, c10);
    sincos2pi(gv.y * a.cf.inv_T, s11, c11);
    float ck0 = c10, sk0 = s10, ck1 = c11, sk1 = s11;
    if (L0) {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < K) {
          float oc, os;
          vstep<ROLE>(hred(ck0, ck1), PC0[k], PC1[k], oc);
          vstep<ROLE>(hred(sk0, sk1), PS0[k], PS1[k], os);
          if (store) PS::st(csc + k * a.csc_ks, oc, os);
          const float n0 = fmaf(ck0, c10, -sk0 * s10);
          sk0 = fmaf(sk0, c10, ck0 * s10);
          ck0 = n0;
          const float n1 = fmaf(ck1, c11, -sk1 * s11);
          sk1 = fmaf(sk1, c11, ck1 * s11);
          ck1 = n1;
        }
      }
    } else {
      const PT *prow = csf + (size_t)fr * a.g.pf;
      float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k < K) {
          float2 p0, p1;
          PS::ld2(prow + k * a.csf_ks, x0, f0, f1, contig, p0, p1);
          float oc, os;
          vstep<ROLE>(hred(p0.x, p1.x), PC0[k], PC1[k], oc);
          vstep<ROLE>(hred(p0.y, p1.y), PS0[k], PS1[k], os);
          if (store) PS::st(csc + k * a.csc_ks, oc, os);
          // level-l half of Eq. (14) at the lane's two fine pixels
          const float at = a.cf.at[k];
          acc0 = fmaf(at, fmaf(sk0, p0.x, -ck0 * p0.y), acc0);
          acc1 = fmaf(at, fmaf(sk1, p1.x, -ck1 * p1.y), acc1);
          const float n0 = fmaf(ck0, c10, -sk0 * s10);
          sk0 = fmaf(sk0, c10, ck0 * s10);
          ck0 = n0;
          const float n1 = fmaf(ck1, c11, -sk1 * s11);
          sk1 = fmaf(sk1, c11, ck1 * s11);
          ck1 = n1;
        }
      }
      // this lane owns fine columns x0, x0+1 of rows [2 i0, 2 i1)
      if (writer && r >= 2 * i0 && r < 2 * i1 && r < a.g.Hf) {
        const float m0 = MAP ? mv.x : a.cf.m, m1 = MAP ? mv.y : a.cf.m;
        float *arow = a.af + (size_t)c * a.af_cs + (size_t)r * a.g.pf;
        const float A0 = fmaf(-m0, acc0, gv.x), A1 = fmaf(-m1, acc1, gv.y);
        if (x0 + 1 < a.g.Wf) {
          *reinterpret_cast<float2 *>(arow + x0) = make_float2(A0, A1);
        } else {
          arow[x0] = A0;
        }
      }
    }
  }

  __device__ inline void run() {
    row<0>(2 * i0 - 2, 0);
    row<1>(2 * i0 - 1, 0);
    row<2>(2 * i0, 0);
    for (int i = i0; i < i1; ++i) {
      row<3>(2 * i + 1, i);
      row<4>(2 * i + 2, i);
    }
  }
};

template <int ST, int KM, bool L0, bool MAP>
__global__ void __launch_bounds__(256) down_kernel(DownArgs<typename PairStore<ST>::T> a) {
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int strip = wv % a.g.nstrips;
  const int rest = wv / a.g.nstrips;
  const int seg = rest % a.g.nsegs;
  const int c = rest / a.g.nsegs;
  if (c >= a.g.C) return;  // uniform per wave
  DownWave<ST, KM, L0, MAP> w(a, lane, c, strip, seg);
  w.run();
}

// --------------------------------------------------------------------------
// up(l)
// --------------------------------------------------------------------------
template <typename PT> struct UpArgs {
  const float *base; size_t base_cs;     // A_l, or I at level 0 (may alias out)
  const float *gf; size_t gf_cs;         // G_l, or I at level 0
  const float *mf;                       // level-l boost plane, or m_map at level 0
  const float *gc; size_t gc_cs;         // G_{l+1}
  const float *oc; size_t oc_cs;         // O_{l+1} (null when l+1 is the top level)
  const PT *csc; size_t csc_ks, csc_cs;  // level-(l+1) pairs
  float *out; size_t out_cs;             // O_l (the caller's output at level 0)
  Geom g;
  Coefs cf;
};

template <int ST, int KM, bool L0, bool MAP, bool HASD>
__global__ void __launch_bounds__(256) up_kernel(UpArgs<typename PairStore<ST>::T> a) {
  using PS = PairStore<ST>;
  using PT = typename PS::T;
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
  const Geom &g = a.g;
  const int strip = wv % g.nstrips;
  const int rest = wv / g.nstrips;
  const int seg = rest % g.nsegs;
  const int c = rest / g.nsegs;
  if (c >= g.C) return;
  const int K = a.cf.K;
  const int j = strip * 62 + lane - 1;
  const int cj = cfold(j, g.Wc, g.Wf);
  const int i0 = seg * g.S, i1 = min(i0 + g.S, g.Hc);
  const bool writer = lane >= 1 && lane <= 62 && j < g.Wc;
  const int x0 = 2 * j;
  const bool two = x0 + 1 < g.Wf;  // the odd fine column exists
  const bool vec_f = two && (!L0 || (((g.pf & 1) == 0) && ((reinterpret_cast<uintptr_t>(a.gf) & 7) == 0)));
  const float *gc = a.gc + (size_t)c * a.gc_cs;
  const float *oc = HASD ? a.oc + (size_t)c * a.oc_cs : nullptr;
  const PT *csc = a.csc + (size_t)c * a.csc_cs;
  const float *base = a.base + (size_t)c * a.base_cs;
  const float *gfp = a.gf + (size_t)c * a.gf_cs;
  float *outp = a.out + (size_t)c * a.out_cs;

  // coarse rows i-1, i (and i+1 loaded per step) of every plane at column cj
  float Dm = 0.f, D0 = 0.f;
  float Cm[KM], C0[KM], Sm[KM], S0[KM];
  auto load_row = [&](int i, float &D, float *Cr, float *Sr) {
    const size_t q = (size_t)cfold(i, g.Hc, g.Hf) * g.pc + cj;
    if (HASD) D = oc[q] - gc[q];
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (k < K) {
        const float2 v = PS::ld(csc + k * a.csc_ks + q);
        Cr[k] = v.x;
        Sr[k] = v.y;
      }
    }
  };
  load_row(i0 - 1, Dm, Cm, Sm);
  load_row(i0, D0, C0, S0);

  // EXPAND weights: (1 6 1)/8 at even and (1 1)/2 at odd fine positions per axis
  constexpr float sc00 = 1.f / 64.f, sc01 = 1.f / 16.f, sc11 = 1.f / 4.f;
  for (int i = i0; i < i1; ++i) {
    float Dp = 0.f;
    float Cp[KM], Sp[KM];
    load_row(i + 1, Dp, Cp, Sp);
    const int r0 = 2 * i, r1 = 2 * i + 1;
    const bool row1 = r1 < g.Hf;
    // fine samples of the lane's 2x2 block (rows r0, r1; columns x0, x0+1)
    float b[4] = {0.f, 0.f, 0.f, 0.f}, gg[4] = {0.f, 0.f, 0.f, 0.f}, mm[4];
    if (writer) {
      const int rr[2] = {r0, row1 ? r1 : r0};
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const size_t o = (size_t)rr[q] * g.pf + x0;
        float2 gv;
        if (vec_f) {
          gv = *reinterpret_cast<const float2 *>(gfp + o);
        } else {
          gv.x = gfp[o];
          gv.y = two ? gfp[o + 1] : gv.x;
        }
        gg[2 * q] = gv.x;
        gg[2 * q + 1] = gv.y;
        if (L0) {
          b[2 * q] = gv.x;
          b[2 * q + 1] = gv.y;
        } else {
          const float2 bv = two ? *reinterpret_cast<const float2 *>(base + o) : make_float2(base[o], base[o]);
          b[2 * q] = bv.x;
          b[2 * q + 1] = bv.y;
        }
        if (MAP) {
          mm[2 * q] = a.mf[o];
          mm[2 * q + 1] = two ? a.mf[o + 1] : mm[2 * q];
        }
      }
    }
    if (!MAP) mm[0] = mm[1] = mm[2] = mm[3] = a.cf.m;
    // unnormalised EXPAND of one plane to the lane's 2x2 fine block
    auto expand4 = [&](float xm, float x0v, float xp, float *e) {
      const float ve = fmaf(6.f, x0v, xm + xp);
      const float vo = x0v + xp;
      const float re = from_right(ve), ro = from_right(vo);
      e[0] = fmaf(6.f, ve, from_left(ve) + re);
      e[1] = ve + re;
      e[2] = fmaf(6.f, vo, from_left(vo) + ro);
      e[3] = vo + ro;
    };
    float ED[4] = {0.f, 0.f, 0.f, 0.f};
    if (HASD) expand4(Dm, D0, Dp, ED);
    float s1[4], c1[4], sk[4], ck[4], acc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      sincos2pi(gg[p] * a.cf.inv_T, s1[p], c1[p]);
      sk[p] = s1[p];
      ck[p] = c1[p];
      acc[p] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (k < K) {
        float EC[4], ES[4];
        expand4(Cm[k], C0[k], Cp[k], EC);
        expand4(Sm[k], S0[k], Sp[k], ES);
        const float at = a.cf.at[k];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          acc[p] = fmaf(at, fmaf(sk[p], EC[p], -ck[p] * ES[p]), acc[p]);
          const float n = fmaf(ck[p], c1[p], -sk[p] * s1[p]);
          sk[p] = fmaf(sk[p], c1[p], ck[p] * s1[p]);
          ck[p] = n;
        }
      }
    }
    if (writer) {
      const float scl[4] = {sc00, sc01, sc01, sc11};
      float o[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) o[p] = fmaf(scl[p], fmaf(mm[p], acc[p], ED[p]), b[p]);
      const size_t o0 = (size_t)r0 * g.pf + x0;
      if (L0 || !two) {
        outp[o0] = o[0];
        if (two) outp[o0 + 1] = o[1];
        if (row1) {
          outp[o0 + g.pf] = o[2];
          if (two) outp[o0 + g.pf + 1] = o[3];
        }
      } else {
        *reinterpret_cast<float2 *>(outp + o0) = make_float2(o[0], o[1]);
        if (row1) *reinterpret_cast<float2 *>(outp + o0 + g.pf) = make_float2(o[2], o[3]);
      }
    }
    Dm = D0;
    D0 = Dp;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      Cm[k] = C0[k];
      C0[k] = Cp[k];
      Sm[k] = S0[k];
      S0[k] = Sp[k];
    }
  }
}

// --------------------------------------------------------------------------
// Host-side launch sequence of one job.
// --------------------------------------------------------------------------
static Geom make_geom(const Level &f, const Level &cl, int C, int S) {
  Geom g;
  g.Wf = f.w;
  g.Hf = f.h;
  g.Wc = cl.w;
  g.Hc = cl.h;
  g.pf = f.pitch;
  g.pc = cl.pitch;
  g.nstrips = (cl.w + 61) / 62;
  g.S = S;
  g.nsegs = (cl.h + S - 1) / S;
  g.C = C;
  return g;
}

// Coarse rows per wave: long segments amortise the halo rows, short ones give
// the 256 CUs enough waves.
static int pick_segment(const Level &cl, int C) {
  const long strips = (cl.w + 61) / 62;
  int S = 32;
  while (S > 4 && strips * ((cl.h + S - 1) / S) * C < 8192) S /= 2;
  return S;
}

static dim3 grid_for(const Geom &g) {
  const long waves = (long)g.nstrips * g.nsegs * g.C;
  return dim3((unsigned)((waves + 3) / 4), 1, 1);
}

template <int ST, int KM, bool MAP>
static hipError_t launch_typed(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *hook) {
  using T = typename PairStore<ST>::T;
  const int L = P.levels;
  const double pb = 2.0 * (ST == FLLF_STORE_F32 ? 4 : 2) * P.K;  // bytes of the K pairs per pixel
  const double C = P.C;
  auto pre = [&]() { if (hook) hook->before(st); };
  auto post = [&](const char *name, double bytes) { if (hook) hook->after(st, name, bytes); };
  auto G = [&](int l) { return (float *)(ws + P.lv[l].off_g); };
  auto CS = [&](int l) { return (T *)(ws + P.lv[l].off_cs); };
  auto O = [&](int l) { return (float *)(ws + P.lv[l].off_o); };
  auto M = [&](int l) -> float * {
    if (!MAP) return nullptr;
    if (l == 0) return const_cast<float *>(P.m_map);
    return l < L - 1 ? (float *)(ws + P.lv[l].off_m) : nullptr;
  };
  const Level *lv = P.lv;
  const dim3 blk(256, 1, 1);
  const double mapb = MAP ? 4.0 : 0.0;

  // Algorithmic bytes: every plane element a launch must read or write, once.
  for (int l = 0; l + 1 < L; ++l) {
    DownArgs<T> a{};
    a.gf = l == 0 ? P.in : G(l);
    a.gf_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    a.csf = l == 0 ? nullptr : CS(l);
    a.csf_ks = lv[l].cs_kstride;
    a.csf_cs = lv[l].cs_cstride;
    a.mf = M(l);
    a.gc = G(l + 1);
    a.gc_cs = lv[l + 1].g_cstride;
    a.csc = CS(l + 1);
    a.csc_ks = lv[l + 1].cs_kstride;
    a.csc_cs = lv[l + 1].cs_cstride;
    a.mc = M(l + 1);
    a.af = l == 0 ? nullptr : O(l);
    a.af_cs = lv[l].g_cstride;
    a.g = make_geom(lv[l], lv[l + 1], P.C, pick_segment(lv[l + 1], P.C));
    a.cf = P.coefs;
    pre();
    if (l == 0) {
      down_kernel<ST, KM, true, MAP><<<grid_for(a.g), blk, 0, st>>>(a);
      post("down0", C * (4.0 * lv[0].n + (4.0 + pb) * lv[1].n) + mapb * (lv[0].n + lv[1].n));
    } else {
      down_kernel<ST, KM, false, MAP><<<grid_for(a.g), blk, 0, st>>>(a);
      post("down", C * ((4.0 + pb + 4.0) * lv[l].n + (4.0 + pb) * lv[l + 1].n) +
                       mapb * (lv[l].n + lv[l + 1].n));
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    UpArgs<T> a{};
    a.base = l == 0 ? P.in : O(l);
    a.base_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    a.gf = l == 0 ? P.in : G(l);
    a.gf_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    a.mf = M(l);
    a.gc = G(l + 1);
    a.gc_cs = lv[l + 1].g_cstride;
    const bool hasd = l + 1 < L - 1;
    a.oc = hasd ? O(l + 1) : nullptr;
    a.oc_cs = lv[l + 1].g_cstride;
    a.csc = CS(l + 1);
    a.csc_ks = lv[l + 1].cs_kstride;
    a.csc_cs = lv[l + 1].cs_cstride;
    a.out = l == 0 ? P.out : O(l);
    a.out_cs = l == 0 ? lv[0].n : lv[l].g_cstride;
    a.g = make_geom(lv[l], lv[l + 1], P.C, pick_segment(lv[l + 1], P.C));
    a.cf = P.coefs;
    pre();
    if (l == 0) {
      if (hasd) up_kernel<ST, KM, true, MAP, true><<<grid_for(a.g), blk, 0, st>>>(a);
      else up_kernel<ST, KM, true, MAP, false><<<grid_for(a.g), blk, 0, st>>>(a);
    } else {
      if (hasd) up_kernel<ST, KM, false, MAP, true><<<grid_for(a.g), blk, 0, st>>>(a);
      else up_kernel<ST, KM, false, MAP, false><<<grid_for(a.g), blk, 0, st>>>(a);
    }
    const double fine = l == 0 ? 4.0 : 8.0;                         // I, or A_l and G_l
    const double coarse = 4.0 + pb + (hasd ? 4.0 : 0.0);            // G, pairs, O_{l+1}
    post(l == 0 ? "up0" : "up", C * ((fine + 4.0) * lv[l].n + coarse * lv[l + 1].n) + mapb * lv[l].n);
  }
  return hipGetLastError();
}

template <int ST>
static hipError_t launch_k(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h) {
  const bool map = P.m_map != nullptr;
  if (P.K <= 4) return map ? launch_typed<ST, 4, true>(P, ws, st, h) : launch_typed<ST, 4, false>(P, ws, st, h);
  if (P.K <= 8) return map ? launch_typed<ST, 8, true>(P, ws, st, h) : launch_typed<ST, 8, false>(P, ws, st, h);
  if (P.K <= 16) return map ? launch_typed<ST, 16, true>(P, ws, st, h) : launch_typed<ST, 16, false>(P, ws, st, h);
  return map ? launch_typed<ST, 32, true>(P, ws, st, h) : launch_typed<ST, 32, false>(P, ws, st, h);
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
