// gfx950 kernels of the Fourier local Laplacian filter (templates; instantiated
// once per pyramid storage type in fllf_kernels_{f32,f16,bf16}.hip).
//
// Per job the filter runs, level by level (all channels of a job in one launch):
//   down(0):  I -> level 1 of the 2K+1 pyramids G_l[I], C~_{l,k}, S~_{l,k}
//             (REDUCE of Eq. (1) on every plane).  cos/sin(omega_k I) are formed
//             in registers and never stored.
//   down(l):  level l -> level l+1 of the 2K+1 pyramids, l >= 1.  The same pass
//             evaluates, at every level-l pixel p, the level-l half of Eq. (14):
//               A_l = G_l - m sum_k at_k (sin(w_k g) C~_{l,k} - cos(w_k g) S~_{l,k}),
//             g = G_l[I]_p, into the O_l slot (it reads those planes anyway).
//   up(l):    l = top-1 .. 0:
//               O_l = A_l + EXPAND(O_{l+1} - G_{l+1})
//                         + m sum_k at_k (sin(w_k g) EXPAND(C~_{l+1,k}) - cos(w_k g) EXPAND(S~_{l+1,k}))
//             = L_l[O] of Eq. (14) plus the collapse step of Eq. (4); at level 0,
//             A_0 = I and the level-0 Fourier terms vanish (first case of Eq. (14)).
//
// Fused levels (large levels >= 1, see fused_level): down(l) also finishes
// L_l[O] = A_l - EXPAND(G_{l+1}) + m sum_k at_k (sin EXPAND(C~) - cos EXPAND(S~))
// from the coarse rows it has just reduced, and up(l) is the one-plane collapse
// O_l = L_l[O] + EXPAND(O_{l+1}).
//
// The Fourier pyramids are stored pre-multiplied by at_k = alpha~_k (REDUCE and
// EXPAND are linear, so every level carries the same factor); the product-sum
// then needs no per-term multiply.  The K (C~, S~) pairs of a pixel form one
// contiguous record, so a wave reads one contiguous run of records per row.
//
// Memory-bound multi-plane stencils; no MFMA, and LDS only as wave-private
// staging that turns record rows into 1 KB accesses.  One wave64 owns a strip of
// 62 coarse columns (lane t <-> coarse column 62 s + t - 1; lanes 0 and 63 are
// halo; the fused down pass uses 60 columns and two halo lanes a side) and
// streams down a segment of coarse rows.  Horizontal taps come
// from neighbouring lanes by DPP wave shifts; vertical taps are register
// running sums.  Each row's loads are issued one row ahead.  All memory access
// is through buffer resources: plane bases and row offsets live in scalar
// registers, each lane adds one 32-bit column offset.  Borders: reflect-101 for
// REDUCE and the matching fold of the coarse grid for EXPAND.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fllf_internal.h"

namespace fllf {

// --------------------------------------------------------------------------
// Buffer-resource memory access.  A Plane is a uniform 128-bit descriptor of a
// window starting at `base`; accesses are base + soff (uniform) + voff (lane).
// Callers keep every offset inside the plane they address.
// --------------------------------------------------------------------------
// The scalar offset operand must live in an SGPR.  Every soff passed here is
// wave-uniform by construction (row offsets), but values that went through
// VALU arithmetic sit in VGPRs; readfirstlane moves them to an SGPR so no
// per-lane waterfall loop is generated around the access.
__device__ inline uint32_t sgpr(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// A lane offset the optimiser may not treat as loop-invariant: offset + const
// is then formed at each access and folded into the instruction's immediate
// offset, so adjacent dword accesses share one VGPR and merge into dwordx2/x4.
// (Empty asm, no instruction is emitted.)
__device__ inline uint32_t opaque(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Stores through a Plane made with nt = true are non-temporal (the nt cache
// policy: the line is not kept for reuse); nt is wave-uniform.
struct Plane {
  __amdgpu_buffer_rsrc_t r;
  bool nt;
  __device__ explicit Plane(const void *base, bool nt_ = false)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, -1, 0x00020000)), nt(nt_) {}
  __device__ inline float ld1(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, sgpr(soff), 0));
  }
  __device__ inline uint32_t ldu(uint32_t voff, uint32_t soff) const {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, sgpr(soff), 0);
  }
  // 8-byte loads are written as two adjacent dword loads, which the backend
  // merges into one buffer_load_dwordx2.  (On this toolchain the 64- and
  // 128-bit buffer-load builtins return only dword 0 correctly.)
  __device__ inline float2 ld2(uint32_t voff, uint32_t soff) const {
    return make_float2(ld1(voff, soff), ld1(voff + 4u, soff));
  }
  __device__ inline void stu(uint32_t x, uint32_t voff, uint32_t soff) const {
    if (nt) __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, sgpr(soff), 2);
    else __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, sgpr(soff), 0);
  }
  __device__ inline void st1(float x, uint32_t voff, uint32_t soff) const {
    stu(__builtin_bit_cast(uint32_t, x), voff, soff);
  }
  // 16 bytes as four adjacent dword stores with cache policy POL (2 = nt), which
  // the backend merges into one buffer_store_dwordx4 (voff must be opaque()).
  template <int POL>
  __device__ inline void st4p(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t voff, uint32_t soff) const {
    __builtin_amdgcn_raw_buffer_store_b32(a, r, voff, sgpr(soff), POL);
    __builtin_amdgcn_raw_buffer_store_b32(b, r, voff + 4u, sgpr(soff), POL);
    __builtin_amdgcn_raw_buffer_store_b32(c, r, voff + 8u, sgpr(soff), POL);
    __builtin_amdgcn_raw_buffer_store_b32(d, r, voff + 12u, sgpr(soff), POL);
  }
  __device__ inline void st2(float2 x, uint32_t voff, uint32_t soff) const {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2 v = {__builtin_bit_cast(uint32_t, x.x), __builtin_bit_cast(uint32_t, x.y)};
    if (nt) __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, sgpr(soff), 2);
    else __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, sgpr(soff), 0);
  }
};

// --------------------------------------------------------------------------
// Storage of the (C, S) pairs, as DW dwords each.  Arithmetic is always
// float32; records are loaded as raw dwords (a prefetch does not wait for the
// data) and converted at the point of use.
// --------------------------------------------------------------------------
template <int S> struct PairStore;

template <> struct PairStore<FLLF_STORE_F32> {
  static constexpr int DW = 2;
  __device__ static inline float2 cvt(const uint32_t *d) {
    return make_float2(__builtin_bit_cast(float, d[0]), __builtin_bit_cast(float, d[1]));
  }
  __device__ static inline void pack(float c, float s, uint32_t *d) {
    d[0] = __builtin_bit_cast(uint32_t, c);
    d[1] = __builtin_bit_cast(uint32_t, s);
  }
};

// The 16-bit forms pack a pair with one conversion of two floats (round to
// nearest even), C in the low half and S in the high half.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));

template <> struct PairStore<FLLF_STORE_F16> {
  static constexpr int DW = 1;
  __device__ static inline float2 cvt(const uint32_t *d) {
    const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(d[0] & 0xffffu));
    const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(d[0] >> 16));
    return make_float2((float)lo, (float)hi);
  }
  __device__ static inline void pack(float c, float s, uint32_t *d) {
    const half2_t v = {(_Float16)c, (_Float16)s};
    d[0] = __builtin_bit_cast(uint32_t, v);
  }
};

template <> struct PairStore<FLLF_STORE_BF16> {
  static constexpr int DW = 1;
  __device__ static inline float2 cvt(const uint32_t *d) {
    return make_float2(__uint_as_float(d[0] << 16), __uint_as_float(d[0] & 0xffff0000u));
  }
  __device__ static inline void pack(float c, float s, uint32_t *d) {
    const bf162_t v = {(__bf16)c, (__bf16)s};
    d[0] = __builtin_bit_cast(uint32_t, v);
  }
};

// One pixel record: the first n dwords (n = K * DW) at voff; adjacent dword
// accesses are merged by the backend into dwordx4 (voff must be opaque()).
template <int NMAX, bool EX>
__device__ inline void ld_record(const Plane &p, uint32_t voff, uint32_t soff, int n, uint32_t *d) {
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (EX || i < n) d[i] = p.ldu(voff + 4u * i, soff);
}
template <int NMAX, bool EX>
__device__ inline void st_record(const Plane &p, uint32_t voff, uint32_t soff, int n, const uint32_t *d) {
#pragma unroll
  for (int i = 0; i < NMAX; ++i)
    if (EX || i < n) p.stu(d[i], voff + 4u * i, soff);
}

// Stores the records of the wave's writer lanes (lanes FIRST .. FIRST + nw - 1,
// NR dwords each, NR a multiple of 4) to one contiguous run starting at byte
// voff0 of row soff of the record plane p (non-temporal stores when p.nt).  The
// records go through the wave's LDS slice (lane L's record at L * (NR + 4)
// dwords; the pad spreads the lanes over the LDS banks) so that every store
// instruction writes 64 consecutive 16-byte pieces (whole cache lines) instead
// of one piece per record.  Only this wave touches its slice and LDS operations
// of one wave are performed in order; the wavefront-scope fences keep the
// compiler from reordering the slice accesses.
template <int NR>
constexpr int staged_slice_dwords() { return 64 * (NR + 4); }

template <int NR, int FIRST, int POL>
__device__ inline void st_staged_pieces(const Plane &p, uint32_t soff, uint32_t voff0, int lane, int total,
                                        const uint32_t *slice) {
  constexpr int PIECES = NR / 4, STRIDE = NR + 4, ITER = (62 * PIECES + 63) / 64;
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int q = 0; q < ITER; ++q) {
    const int t = min(q * 64 + lane, total - 1);
    const int r = t / PIECES + FIRST, part = t - (r - FIRST) * PIECES;
    const u4 v = *reinterpret_cast<const u4 *>(slice + r * STRIDE + 4 * part);
    if (q * 64 + lane < total) p.st4p<POL>(v.x, v.y, v.z, v.w, opaque(voff0 + 16u * (uint32_t)t), soff);
  }
}

template <int NR, int FIRST = 1>
__device__ inline void st_records_staged(const Plane &p, uint32_t soff, uint32_t voff0, int lane, int nw,
                                         const uint32_t *d, uint32_t *slice) {
  static_assert(NR % 4 == 0, "records must be whole 16-byte pieces");
  constexpr int PIECES = NR / 4, STRIDE = NR + 4;
#pragma unroll
  for (int i = 0; i < PIECES; ++i)
    *reinterpret_cast<uint4 *>(slice + lane * STRIDE + 4 * i) =
        make_uint4(d[4 * i], d[4 * i + 1], d[4 * i + 2], d[4 * i + 3]);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  const int total = nw * PIECES;  // 16-byte pieces to store, record of lane FIRST first
  // two loops whose stores differ in their cache-policy immediate (a runtime
  // choice between two otherwise equal stores would be merged into one)
  if (p.nt) st_staged_pieces<NR, FIRST, 2>(p, soff, voff0, lane, total, slice);
  else st_staged_pieces<NR, FIRST, 0>(p, soff, voff0, lane, total, slice);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Coalesced record rows.  On interior strips the records a wave needs from one
// row are one contiguous span: lane t owns records PER t .. PER t + PER - 1
// (D = NR PER dwords).  Loading lane t's own records makes every load
// instruction touch 64 cache lines; instead lane t loads 16-byte chunks
// t, t + 64, ... of the span (1 KB per instruction) and the wave transposes
// them through LDS.  In LDS each lane's D dwords are followed by 4 pad dwords,
// which keeps both the chunk writes and the ds_read_b128 read-back free of
// bank conflicts for every record size.
template <int D>
constexpr int span_slice_dwords() { return 64 * (D + 4); }

template <int D>
__device__ inline void ld_span(const Plane &p, uint32_t soff, int lane, uint32_t *q) {
  static_assert(D % 4 == 0, "whole 16-byte chunks");
  const uint32_t v = opaque(16u * (uint32_t)lane);
#pragma unroll
  for (int c = 0; c < D / 4; ++c) {
    const uint32_t so = soff + 1024u * (uint32_t)c;
#pragma unroll
    for (int e = 0; e < 4; ++e) q[4 * c + e] = p.ldu(v + 4u * e, so);
  }
}

// A run whose first n 16-byte chunks only are in bounds (a border strip's
// row): chunks past n load chunk n - 1 again; their values are never picked.
template <int D>
__device__ inline void ld_span_n(const Plane &p, uint32_t soff, int lane, uint32_t n, uint32_t *q) {
  static_assert(D % 4 == 0, "whole 16-byte chunks");
  const uint32_t last = 16u * (n - 1u);
#pragma unroll
  for (int c = 0; c < D / 4; ++c) {
    const uint32_t v = opaque(min(16u * (uint32_t)(64 * c + lane), last));
#pragma unroll
    for (int e = 0; e < 4; ++e) q[4 * c + e] = p.ldu(v + 4u * e, soff);
  }
}

// The chunks go to LDS at their place in the span: slot u holds dwords
// u D .. u D + D - 1 of the span, followed by 4 pad dwords.
template <int D>
__device__ inline void span_to_slice(const uint32_t *q, uint32_t *slice, int lane) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  constexpr int LD = D + 4;  // LDS dwords per lane
#pragma unroll
  for (int c = 0; c < D / 4; ++c) {
    const int w = 4 * (64 * c + lane);  // dword of the span this chunk starts at
    const int u = w / D, off = w - u * D;
    *reinterpret_cast<u4 *>(slice + u * LD + off) = u4{q[4 * c], q[4 * c + 1], q[4 * c + 2], q[4 * c + 3]};
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// Border strips: lane t takes its two records of R dwords (the span holds two
// per slot) from slice dword offsets o0 and o1, those of its folded columns.
template <int R>
__device__ inline void transpose_span_pick(uint32_t *q, uint32_t *slice, int lane, uint32_t o0, uint32_t o1) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  span_to_slice<2 * R>(q, slice, lane);
#pragma unroll
  for (int c = 0; c < R / 4; ++c) {
    const u4 v = *reinterpret_cast<const u4 *>(slice + o0 + 4 * c);
    const u4 w = *reinterpret_cast<const u4 *>(slice + o1 + 4 * c);
    q[4 * c] = v.x; q[4 * c + 1] = v.y; q[4 * c + 2] = v.z; q[4 * c + 3] = v.w;
    q[R + 4 * c] = w.x; q[R + 4 * c + 1] = w.y; q[R + 4 * c + 2] = w.z; q[R + 4 * c + 3] = w.w;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

template <int D>
__device__ inline void transpose_span(uint32_t *q, uint32_t *slice, int lane) {
  typedef uint32_t u4 __attribute__((ext_vector_type(4)));
  constexpr int LD = D + 4;  // LDS dwords per lane
  span_to_slice<D>(q, slice, lane);
#pragma unroll
  for (int c = 0; c < D / 4; ++c) {
    const u4 v = *reinterpret_cast<const u4 *>(slice + lane * LD + 4 * c);
    q[4 * c] = v.x;
    q[4 * c + 1] = v.y;
    q[4 * c + 2] = v.z;
    q[4 * c + 3] = v.w;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}

// --------------------------------------------------------------------------
// Index helpers
// --------------------------------------------------------------------------
// Reflect-101 fold onto [0, n):  ... 2 1 | 0 1 2 ... n-1 | n-2 ...  (any i; no division)
__device__ inline int reflect(int i, int n) {
  if (n == 1) return 0;
  while (i < 0 || i >= n) i = i < 0 ? -i : 2 * n - 2 - i;
  return i;
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

// DPP wave shifts: lane t receives lane t-1 (from_left) or lane t+1 (from_right);
// the lane that has no source gets 0 (bound_ctrl), which only halo lanes see.
__device__ inline float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ inline float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}

// sin and cos of 2 pi u, u in revolutions (|u| < 256: the hardware range).
__device__ inline void sincos2pi(float u, float &s, float &c) {
  s = __builtin_amdgcn_sinf(u);
  c = __builtin_amdgcn_cosf(u);
}

// cos/sin of k theta for k = 1, 2, ... from cos/sin theta by the three-term
// (Chebyshev) recurrence x_{k+1} = 2 cos(theta) x_k - x_{k-1}: two FMAs per term.
struct Harmonics {
  float t, cp, sp, c, s;  // 2 cos(theta); terms k-1 and k
  __device__ inline void init(float c1, float s1) {
    t = 2.f * c1;
    cp = 1.f;
    sp = 0.f;
    c = c1;
    s = s1;
  }
  __device__ inline void next() {
    const float cn = fmaf(t, c, -cp), sn = fmaf(t, s, -sp);
    cp = c;
    sp = s;
    c = cn;
    s = sn;
  }
};

// Pixel-by-pixel range scale (Sec. III-B): the factor alpha~_k(s) / alpha~_k(sref)
// = rho^3 Q^(k^2) of a pixel of scale s (see Coefs), for k = 1, 2, ... by the
// recurrence Q^((k+1)^2) = Q^(k^2) Q^(2k+1), Q^(2k+3) = Q^(2k+1) Q^2; rho^3 is
// applied once to the sum over k.  At s = sref every factor is exactly 1.
struct TermScale {
  float e, r, q2, r3;  // Q^(k^2), Q^(2k+1), Q^2, rho^3
  __device__ inline void init(float s, const Coefs &cf) {
    const float q = expf(-cf.qk * (s * s - cf.sref * cf.sref));
    e = q;
    q2 = q * q;
    r = q2 * q;
    const float rho = s * cf.inv_sref;
    r3 = cf.has_smap ? rho * rho * rho : 1.f;
  }
  __device__ inline void next() {
    e *= r;
    r *= q2;
  }
};

// Fast LLF (Sec. II-C): the remap sampled at g, and the interpolation weight of
// sample j at t = g / tau (clamped to [0, n-1]): the hat max(0, 1 - |t - j|),
// which is (1 - a) at j = floor(t) and a at j + 1, a = t - j.
__device__ inline float remap_at(float v, float g, const Coefs &cf) {
  const float d = v - g;
  return fmaf(cf.m * d, expf(-d * d * cf.rc), v);
}
__device__ inline float hat(float t, float j) { return fmaxf(0.f, 1.f - fabsf(t - j)); }
__device__ inline float sample_pos(float g, const Coefs &cf) { return fminf(fmaxf(g * cf.inv_tau, 0.f), cf.nm1); }
// Level 0: the interpolation of r(v, tau j) over j at g = v itself.
__device__ inline float fast_level0(float v, const Coefs &cf) {
  const float t = sample_pos(v, cf);
  const float j = fminf(floorf(t), cf.nm1 - 1.f), w = t - j;
  return fmaf(w, remap_at(v, (j + 1.f) * cf.tau, cf), (1.f - w) * remap_at(v, j * cf.tau, cf));
}

// Unnormalised horizontal REDUCE at the lane's even fine column 2j from its
// samples v0 (2j), v1 (2j+1) and its neighbours': taps [1 4 6 4 1].
// Each lane shift feeds exactly one add (folded into a DPP add), and the result
// is pinned where it is computed so that no part of the sum sinks into a
// conditional block away from its shifts.
__device__ inline float hred(float v0, float v1) {
  const float t = from_right(v0) + v0;  // v_{2j} + v_{2j+2}
  float h = fmaf(5.f, v0, fmaf(4.f, from_left(v1) + v1, from_left(v0) + t));
  asm volatile("" : "+v"(h));
  return h;
}

// Unnormalised EXPAND of one plane onto the lane's 2x2 fine block from coarse
// rows i-1, i, i+1 at the lane's column (xm, x0, xp) and the neighbour lanes'.
// e[0..3] = (2i, 2j), (2i, 2j+1), (2i+1, 2j), (2i+1, 2j+1).
// Written so that every neighbour value is used by exactly one add, which
// the backend folds into a DPP add (no separate lane-shift moves).
__device__ inline void expand4(float xm, float x0, float xp, float *e) {
  const float ve = fmaf(6.f, x0, xm + xp);
  const float vo = x0 + xp;
  e[1] = from_right(ve) + ve;                  // ve_j + ve_{j+1}
  e[0] = fmaf(5.f, ve, from_left(ve) + e[1]);  // ve_{j-1} + 6 ve_j + ve_{j+1}
  e[3] = from_right(vo) + vo;
  e[2] = fmaf(5.f, vo, from_left(vo) + e[3]);
}

// Vertical REDUCE as running sums over a stream of horizontally reduced rows.
// P0 accumulates coarse row i, P1 coarse row i+1.  Weights [1 4 6 4 1]/256
// carry the 2-D normalisation.  Roles (row of the stream):
//   0: 2 i0 - 2 (seeds P1 for coarse row i0; P0 is then a dummy)
//   3: 2 i + 1      4: 2 i + 2  (completes coarse row i, returned in out)
template <int ROLE>
__device__ inline void vstep(float h, float &P0, float &P1, float &out) {
  constexpr float w1 = 1.f / 256.f, w4 = 4.f / 256.f, w6 = 6.f / 256.f;
  if (ROLE == 0) {
    P0 = 0.f;
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

// Minimum waves per SIMD a kernel is compiled for: 2 (<= 256 VGPRs) up to 8
// terms; with 16 or 32 terms the pyramid rows need the whole register file.
constexpr int min_waves_per_simd(int KM) { return KM <= 8 ? 2 : 1; }
// The fused down pass with per-pixel maps carries the maps' ring as well: one
// wave per SIMD, so that it keeps its state in registers.
constexpr int down_waves_per_simd(int KM, bool MAP, bool FUSE) { return MAP && FUSE ? 1 : min_waves_per_simd(KM); }


// --------------------------------------------------------------------------
// Kernel arguments
// --------------------------------------------------------------------------
struct Geom {
  int Wf, Hf, Wc, Hc;  // fine and coarse sizes
  int pf, pc;          // row pitches (pixels) of the fine and coarse planes
  int po, pm;          // row pitches of the fine output (up passes) and of the fine
                       // boost plane: pf, except at level 0 (the caller's images)
  int nstrips, nsegs;  // column strips (62 coarse columns each) and row segments
  int S;               // coarse rows per segment
  int C;               // channels
  int nt;              // 1: the pass's stores are non-temporal
};

struct DownArgs {
  const float *gf; size_t gf_cs;         // G_l (the input I at level 0)
  const uint32_t *csf; size_t csf_cs;    // level-l pair records (l >= 1), dwords per channel
  const float *mf;                       // level-l boost plane (m_map at level 0)
  const float *sf;                       // level-l range-scale plane (sigma_map at level 0)
  float *gc; size_t gc_cs;               // G_{l+1}
  uint32_t *csc; size_t csc_cs;          // level-(l+1) pair records
  float *mc;                             // level-(l+1) boost plane or null
  float *sc;                             // level-(l+1) range-scale plane or null
  float *af; size_t af_cs;               // A_l (l >= 1), stored in the O_l slot
  int minus_g;                           // fused level 1: store L_1[O] - G_1 (see UpArgs::oc_minus_g)
  Geom g;
  Coefs cf;
};

struct UpArgs {
  const float *base; size_t base_cs;     // A_l, or I at level 0 (may alias out)
  const float *gf; size_t gf_cs;         // G_l, or I at level 0
  const float *mf;                       // level-l boost plane, or m_map at level 0
  const float *sf;                       // level-l range-scale plane, or sigma_map at level 0
  const float *gc; size_t gc_cs;         // G_{l+1}
  const float *oc; size_t oc_cs;         // O_{l+1} (null when l+1 is the top level)
  const uint32_t *csc; size_t csc_cs;    // level-(l+1) pair records
  float *out; size_t out_cs;             // O_l (the caller's output at level 0)
  int oc_minus_g;                        // oc holds O_{l+1} - G_{l+1}: G_{l+1} is not read
  // up(0) with the level-1 collapse folded in: oc holds L_1[O] - G_1 and the pass
  // adds EXPAND(O_2) itself; o2 is O_2 (G_2 when level 2 is the top), w2 x h2, pitch p2
  const float *o2; size_t o2_cs;
  int w2, h2, p2;
  Geom g;
  Coefs cf;
};

// Wave -> (strip, segment, channel), all wave-uniform in scalar registers;
// false when the wave has no work.
__device__ inline bool wave_coords(const Geom &g, int &lane, int &strip, int &seg, int &c) {
  lane = threadIdx.x & 63;
  // blocks of four waves, or of one (small passes)
  const int wv = blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  strip = __builtin_amdgcn_readfirstlane(wv % g.nstrips);
  const int rest = wv / g.nstrips;
  seg = __builtin_amdgcn_readfirstlane(rest % g.nsegs);
  c = __builtin_amdgcn_readfirstlane(rest / g.nsegs);
  return c < g.C;
}

// Batched launches: the waves of all jobs of one pass are numbered 0 .. total-1,
// job j owning [start[j], start[j+1]).  A wave walks that range with a grid
// stride, so the grid may be smaller than the work (persistent launch).
__device__ inline uint32_t first_wave() {
  return blockIdx.x * 4u + (uint32_t)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// The job of wave w: the largest j with start[j] <= w (scalar binary search).
__device__ inline int find_job(const uint32_t *__restrict__ start, int n, uint32_t w) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= w) lo = mid; else hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

__device__ inline void job_coords(const Geom &g, uint32_t wv, int &strip, int &seg, int &c) {
  strip = __builtin_amdgcn_readfirstlane((int)(wv % (uint32_t)g.nstrips));
  const uint32_t rest = wv / (uint32_t)g.nstrips;
  seg = __builtin_amdgcn_readfirstlane((int)(rest % (uint32_t)g.nsegs));
  c = __builtin_amdgcn_readfirstlane((int)(rest / (uint32_t)g.nsegs));
}

// A wave touches columns outside [0, Wf) only in the first strip and in the
// strips whose lane 63 (coarse column 62 s + 62) reaches fine column Wf - 1.
__device__ inline bool border_strip(int strip, int Wf, int sw = 62, int hl = 1) {
  return strip == 0 || 2 * (sw * strip + 63 - hl) + 1 >= Wf;
}

// --------------------------------------------------------------------------
// down(l)
// --------------------------------------------------------------------------
// State of the fused down pass: coarse rows ci-2, ci-1, ci (G and the
// at_k-weighted pairs) and, for fine rows 2ci-2 .. 2ci+1 at the lane's two
// columns, the level-l half A, cos/sin(omega_1 g) and the boost, waiting for
// coarse row ci.  A separate member so that the other passes carry none of it.
template <int KM>
struct FuseRing {
  float Gm, G0, Gp, Cm[KM], C0[KM], Cp[KM], Sm[KM], S0[KM], Sp[KM];
  float pA[4][2], pc[4][2], ps[4][2], pm[4][2], pq[4][2];  // pq: range scale (maps only)
};
struct NoRing {};

// Pyramid records the fused pass keeps in registers without spilling: exact
// K loops of at most 16 dwords per record (float32 K <= 8, 16-bit K <= 16).
constexpr bool fusable(int K, int dwp) { return (K == 4 || K == 8 || K == 16) && K * dwp <= 16; }
// ... except 16 terms with per-pixel maps: their ring plus the maps' values
// exceed the register file (16-bit storage: 1.5 KB per lane in scratch memory;
// 4K RGB K=16 with a range-scale map 3.2 ms fused against 0.8 ms separate).
constexpr bool fusable(int K, int dwp, bool map) { return fusable(K, dwp) && !(map && K == 16); }

// FAST: the fast LLF comparator (Sec. II-C): the records hold the pyramids of the
// sampled remaps r(I, tau j) (level 0: formed in registers), and the level-l
// half interpolates them at G_l[I] (separate form only, no maps).
template <int ST, int KM, bool EX, bool L0, bool MAP, bool FUSE, bool FAST = false>
struct DownWave {
  static_assert(!(L0 && FUSE), "level 0 has no Laplacian to finish");
  static_assert(!(FAST && (MAP || FUSE)), "fast LLF runs the separate passes without maps");
  using PS = PairStore<ST>;
  static constexpr int DW = PS::DW;
  static constexpr int NR = KM * DW;  // dwords of a full record
  struct RowIn {  // one fine row as loaded (raw), for the one-row-ahead prefetch
    float g0, g1, m0, m1, s0, s1;  // G (or I), boost, range scale at the two columns
    uint32_t q[2 * NR];  // records of fine columns x0 and x0 + 1
  };
  // With exact K the coarse records are written through LDS (whole lines per
  // store), and on interior strips the fine records are read as coalesced spans.
  static constexpr bool STAGED = EX;
  static constexpr bool SPAN = EX && !L0 && NR <= 16;
  static constexpr int SLICE = !EX ? 1 : SPAN ? span_slice_dwords<2 * NR>() : staged_slice_dwords<NR>();
  // FUSE (levels >= 1): the pass also finishes the level-l Laplacian of the
  // output from the fresh coarse rows: strips of 60 coarse columns with two
  // halo lanes a side, so that the coarse values EXPAND needs (lanes 1 .. 62)
  // are exact.  Otherwise levels >= 1 store the level-l half A_l only.
  static constexpr int SW = FUSE ? 60 : 62;  // coarse columns per strip
  // Level 0 of the 16-bit forms, which is bound by its ALU work, reads the two
  // input columns of a lane as two 4-byte loads (at their folded offsets, the
  // columns themselves on interior strips) rather than one 8-byte load: 4K RGB
  // K=8 down(0) float16 83.8 -> 81.7 us, bfloat16 84.1 -> 81.3 us (float32,
  // bound by its traffic, 104.7 -> 106.2 us keeps the 8-byte load).
  static constexpr bool SPLIT2 = L0 && ST != FLLF_STORE_F32;
  static constexpr int HL = FUSE ? 2 : 1;    // halo lanes on each side
  const DownArgs &a;
  int c, K, nr, j, i0, i1, x0, lane, nw;
  bool writer, border, two;
  uint32_t rec;                                        // bytes per pair record
  uint32_t vx, vf0, vf1, vpx, vpf0, vpf1, vcj, vpcj;  // lane byte offsets
  uint32_t vrun;                                       // record offset of the first writer lane's coarse column
  uint32_t vspan;                                      // record offset of lane 0's fine column x0
  uint32_t *slice;                                     // this wave's LDS staging slice
  // Border strips of the fused (large-level) passes read the in-bounds part of
  // each row's run of records as a span as well, and every lane picks the
  // records of its folded columns from the slice: per-lane record loads touch
  // 64 cache lines per instruction against 8, and made the border waves the
  // last to finish (4K RGB float32 down(1): 119 us, 106 us with those waves
  // idle, 113.5 us with spans).  On the small levels, bound by latency, the
  // slice round trip costs more than it saves, so they keep per-lane loads.
  // With at least 6 in-bounds fine columns, the folded columns of every lane
  // that feeds a writer (two lanes past the last one, whose columns fold back
  // at most 6 from the edge) lie in the span; narrower strips load per lane.
  // Loops of 16 terms keep per-lane border loads: their fused pass is at the
  // edge of the register file, and a third row loop put its row buffers in
  // scratch memory (float16 K=16 4K RGB: 0.64 -> 2.7 ms).
  static constexpr bool BSPAN = SPAN && FUSE && KM <= 8;
  bool bspan;
  uint32_t bchunks;       // in-bounds 16-byte chunks of the span
  uint32_t boff0, boff1;  // slice dword offsets of the lane's two records
  const float *gf;
  const uint32_t *csf;
  float PG0, PG1, PM0, PM1, PQ0, PQ1;
  float PC0[KM], PC1[KM], PS0[KM], PS1[KM];
  typename std::conditional<FUSE, FuseRing<KM>, NoRing>::type z;

  __device__ DownWave(const DownArgs &args, int lane_, int c_, int strip, int seg, uint32_t *slice_)
      : a(args) {
    lane = lane_;
    slice = slice_;
    c = c_;
    K = EX ? KM : a.cf.K;
    nr = K * DW;
    rec = 4u * (uint32_t)nr;
    j = strip * SW + lane - HL;
    i0 = seg * a.g.S;
    i1 = min(i0 + a.g.S, a.g.Hc);
    writer = lane >= HL && lane <= 63 - HL && j < a.g.Wc;
    nw = min(SW, a.g.Wc - strip * SW);  // writer lanes are HL .. HL + nw - 1
    vrun = (uint32_t)(strip * SW) * rec;
    border = sgpr(border_strip(strip, a.g.Wf, SW, HL));  // uniform
    x0 = 2 * j;
    two = x0 + 1 < a.g.Wf;
    vspan = border ? 0u : (uint32_t)(2 * (strip * SW - HL)) * rec;
    if constexpr (FUSE) {
      z.Gm = z.G0 = z.Gp = 0.f;
#pragma unroll
      for (int k = 0; k < KM; ++k) z.Cm[k] = z.C0[k] = z.Cp[k] = z.Sm[k] = z.S0[k] = z.Sp[k] = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        for (int e = 0; e < 2; ++e) z.pA[q][e] = z.pc[q][e] = z.ps[q][e] = z.pm[q][e] = z.pq[q][e] = 0.f;
    }
    const int f0 = reflect(x0, a.g.Wf), f1 = reflect(x0 + 1, a.g.Wf);
    vx = (uint32_t)max(x0, 0) * 4u;
    vf0 = (uint32_t)f0 * 4u;
    vf1 = (uint32_t)f1 * 4u;
    vpx = (uint32_t)max(x0, 0) * rec;
    vpf0 = (uint32_t)f0 * rec;
    vpf1 = (uint32_t)f1 * rec;
    vcj = (uint32_t)max(j, 0) * 4u;
    vpcj = (uint32_t)max(j, 0) * rec;
    bspan = false;
    bchunks = 0u;
    boff0 = boff1 = 0u;
    if (BSPAN && border) {
      const int c0 = 2 * (strip * SW - HL);  // fine column of lane 0's first record
      const int s0 = max(c0, 0), cnt = min(c0 + 128, a.g.Wf) - s0;  // wave-uniform
      if (cnt >= 6) {
        bspan = true;
        vspan = (uint32_t)s0 * rec;
        bchunks = (uint32_t)(cnt * NR / 4);
        const int r0 = min(max(f0 - s0, 0), cnt - 1), r1 = min(max(f1 - s0, 0), cnt - 1);
        boff0 = (uint32_t)((r0 >> 1) * (2 * NR + 4) + (r0 & 1) * NR);
        boff1 = (uint32_t)((r1 >> 1) * (2 * NR + 4) + (r1 & 1) * NR);
      }
    }
    gf = a.gf + (size_t)c * a.gf_cs;
    csf = L0 ? nullptr : a.csf + (size_t)c * a.csf_cs;
  }

  // Two fine samples (columns x0, x0+1) of one float row: folded columns in
  // border strips, one contiguous 8-byte access otherwise.
  template <bool BORDER>
  __device__ inline void ld_f2(const Plane &p, uint32_t soff, float &x, float &y) const {
    if (BORDER || SPLIT2) {
      x = p.ld1(vf0, soff);
      y = p.ld1(vf1, soff);
    } else {
      const float2 v = p.ld2(opaque(vx), soff);
      x = v.x;
      y = v.y;
    }
  }

  template <bool BORDER, bool BS = false>
  __device__ inline void load(RowIn &d, int r) const {
    const uint32_t fr = (uint32_t)reflect(r, a.g.Hf);
    ld_f2<BORDER>(Plane(gf), fr * (uint32_t)a.g.pf * 4u, d.g0, d.g1);
    if (MAP) {  // either map may be absent (wave-uniform): its scalar then
      const uint32_t sm = fr * (uint32_t)a.g.pm * 4u;
      if (a.mf) ld_f2<BORDER>(Plane(a.mf), sm, d.m0, d.m1);
      else d.m0 = d.m1 = a.cf.m;
      if (a.sf) ld_f2<BORDER>(Plane(a.sf), sm, d.s0, d.s1);
      else d.s0 = d.s1 = a.cf.sref;
    }
    if (!L0) {
      const Plane p(csf);
      const uint32_t so = fr * (uint32_t)a.g.pf * rec;
      if (BORDER && !(SPAN && BS)) {
        ld_record<NR, EX>(p, opaque(vpf0), so, nr, d.q);
        ld_record<NR, EX>(p, opaque(vpf1), so, nr, d.q + NR);
      } else if (SPAN && BORDER) {
        ld_span_n<2 * NR>(p, so + vspan, lane, bchunks, d.q);  // picked before use
      } else if (SPAN) {
        ld_span<2 * NR>(p, so + vspan, lane, d.q);  // transposed before use
      } else {
        const uint32_t vo = opaque(vpx);
        ld_record<NR, EX>(p, vo, so, nr, d.q);
        ld_record<NR, EX>(p, vo + rec, so, nr, d.q + NR);
      }
    }
  }

  // The loaded span chunks become this lane's two records (border strips: those
  // of its folded columns).
  template <bool BORDER, bool BS = false>
  __device__ inline void ready(RowIn &d) {
    if (SPAN && !BORDER) transpose_span<2 * NR>(d.q, slice, lane);
    else if (SPAN && BS) transpose_span_pick<NR>(d.q, slice, lane, boff0, boff1);
  }

  // Consume fine row r (stream role ROLE); ROLE 4 emits coarse row ci.
  template <int ROLE>
  __device__ inline void process(const RowIn &d, int r, int ci) {
    float og = 0.f, om = 0.f;
    float oc[KM], os[KM];
    vstep<ROLE>(hred(d.g0, d.g1), PG0, PG1, og);
    float oq = 0.f;
    if (MAP) vstep<ROLE>(hred(d.m0, d.m1), PM0, PM1, om);
    if (MAP) vstep<ROLE>(hred(d.s0, d.s1), PQ0, PQ1, oq);
    if (L0 && FAST) {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {  // pair k: samples 2k and 2k + 1
          const float ga = (float)(2 * k) * a.cf.tau, gb = (float)(2 * k + 1) * a.cf.tau;
          vstep<ROLE>(hred(remap_at(d.g0, ga, a.cf), remap_at(d.g1, ga, a.cf)), PC0[k], PC1[k], oc[k]);
          vstep<ROLE>(hred(remap_at(d.g0, gb, a.cf), remap_at(d.g1, gb, a.cf)), PS0[k], PS1[k], os[k]);
        }
      }
    } else if (L0) {
      float s, cc;
      sincos2pi(d.g0 * a.cf.inv_T, s, cc);
      Harmonics h0;
      h0.init(cc, s);
      sincos2pi(d.g1 * a.cf.inv_T, s, cc);
      Harmonics h1;
      h1.init(cc, s);
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          vstep<ROLE>(hred(h0.c, h1.c), PC0[k], PC1[k], oc[k]);
          vstep<ROLE>(hred(h0.s, h1.s), PS0[k], PS1[k], os[k]);
          h0.next();
          h1.next();
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          const float2 q0 = PS::cvt(&d.q[k * DW]), q1 = PS::cvt(&d.q[NR + k * DW]);
          vstep<ROLE>(hred(q0.x, q1.x), PC0[k], PC1[k], oc[k]);
          vstep<ROLE>(hred(q0.y, q1.y), PS0[k], PS1[k], os[k]);
        }
      }
    }
    // the level-l half of Eq. (14), A = G_l - m sum_k at_k (sin C~ - cos S~), on
    // the fine rows [2 i0, 2 i1) this wave owns (not on the rows above or below
    // that only feed the running sums); wave-uniform
    float A0 = 0.f, A1 = 0.f, c0 = 0.f, s0 = 0.f, c1 = 0.f, s1 = 0.f;
    const float m0 = MAP ? d.m0 : a.cf.m, m1 = MAP ? d.m1 : a.cf.m;
    if (FAST && !L0 && r >= 2 * i0 && r < 2 * i1 && r < a.g.Hf) {
      // the level-l half of fast LLF: the sampled remaps' level l interpolated at g
      const float t0 = sample_pos(d.g0, a.cf), t1 = sample_pos(d.g1, a.cf);
      float acc0 = 0.f, acc1 = 0.f;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          const float2 q0 = PS::cvt(&d.q[k * DW]), q1 = PS::cvt(&d.q[NR + k * DW]);
          const float ja = (float)(2 * k), jb = (float)(2 * k + 1);
          acc0 = fmaf(hat(t0, ja), q0.x, fmaf(hat(t0, jb), q0.y, acc0));
          acc1 = fmaf(hat(t1, ja), q1.x, fmaf(hat(t1, jb), q1.y, acc1));
        }
      }
      if (writer) {
        const Plane ap(a.af + (size_t)c * a.af_cs, a.g.nt);
        const uint32_t so = (uint32_t)r * (uint32_t)a.g.pf * 4u;
        if (two) ap.st2(make_float2(acc0, acc1), vx, so);
        else ap.st1(acc0, vx, so);
      }
    } else if (!L0 && r >= 2 * i0 && r < 2 * i1 && r < a.g.Hf) {
      sincos2pi(d.g0 * a.cf.inv_T, s0, c0);
      Harmonics h0;
      h0.init(c0, s0);
      sincos2pi(d.g1 * a.cf.inv_T, s1, c1);
      Harmonics h1;
      h1.init(c1, s1);
      float acc0 = 0.f, acc1 = 0.f;
      TermScale t0, t1;
      if (MAP) {
        t0.init(d.s0, a.cf);
        t1.init(d.s1, a.cf);
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          const float2 q0 = PS::cvt(&d.q[k * DW]), q1 = PS::cvt(&d.q[NR + k * DW]);
          // pairs carry at_k; with maps, each term takes the pixel's factor
          if (MAP) {
            acc0 = fmaf(t0.e, fmaf(h0.s, q0.x, -h0.c * q0.y), acc0);
            acc1 = fmaf(t1.e, fmaf(h1.s, q1.x, -h1.c * q1.y), acc1);
            t0.next();
            t1.next();
          } else {
            acc0 = fmaf(h0.s, q0.x, fmaf(-h0.c, q0.y, acc0));
            acc1 = fmaf(h1.s, q1.x, fmaf(-h1.c, q1.y, acc1));
          }
          h0.next();
          h1.next();
        }
      }
      if (MAP) {
        acc0 *= t0.r3;
        acc1 *= t1.r3;
      }
      // with minus_g (fused level 1) the pass leaves L_1[O] - G_1, whose collapse
      // is the O_1 - G_1 that up(0) expands: it then need not read G_1
      const float b0 = FUSE && a.minus_g ? 0.f : d.g0, b1 = FUSE && a.minus_g ? 0.f : d.g1;
      A0 = fmaf(-m0, acc0, b0);
      A1 = fmaf(-m1, acc1, b1);
      if (!FUSE && writer) {  // this lane owns fine columns x0, x0+1
        const Plane ap(a.af + (size_t)c * a.af_cs, a.g.nt);
        const uint32_t so = (uint32_t)r * (uint32_t)a.g.pf * 4u;
        if (two) ap.st2(make_float2(A0, A1), vx, so);
        else ap.st1(A0, vx, so);
      }
    }
    if constexpr (FUSE && ROLE == 3) {
      z.pA[3][0] = A0; z.pA[3][1] = A1;
      z.pc[3][0] = c0; z.pc[3][1] = c1;
      z.ps[3][0] = s0; z.ps[3][1] = s1;
      z.pm[3][0] = m0; z.pm[3][1] = m1;
      if (MAP) { z.pq[3][0] = d.s0; z.pq[3][1] = d.s1; }
    }
    if (ROLE == 4 && ci >= i0 && (!FUSE || ci < i1)) {  // wave-uniform
      const uint32_t so = (uint32_t)ci * (uint32_t)a.g.pc;
      if (writer) {
        Plane(a.gc + (size_t)c * a.gc_cs, a.g.nt).st1(og, vcj, so * 4u);
        if (MAP && a.mc && c == 0) Plane(a.mc, a.g.nt).st1(om, vcj, so * 4u);
        if (MAP && a.sc && c == 0) Plane(a.sc, a.g.nt).st1(oq, vcj, so * 4u);
      }
      uint32_t q[NR];
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          // level 1 is where the pyramids take their at_k factor
          const float w = L0 ? a.cf.at[k] : 1.f;
          PS::pack(w * oc[k], w * os[k], &q[k * DW]);
        }
      }
      const Plane cp(a.csc + (size_t)c * a.csc_cs, a.g.nt);
      if (STAGED) {
        st_records_staged<NR, HL>(cp, so * rec, vrun, lane, nw, q, slice);
      } else if (writer) {
        st_record<NR, EX>(cp, opaque(vpcj), so * rec, nr, q);
      }
    }
    if constexpr (FUSE && ROLE == 4) {
      z.Gm = z.G0;
      z.G0 = z.Gp;
      z.Gp = og;
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          z.Cm[k] = z.C0[k];
          z.C0[k] = z.Cp[k];
          z.Cp[k] = oc[k];
          z.Sm[k] = z.S0[k];
          z.S0[k] = z.Sp[k];
          z.Sp[k] = os[k];
        }
      }
      if (ci >= i0 + 1) finish(ci);  // wave-uniform
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        z.pA[0][e] = z.pA[2][e]; z.pA[1][e] = z.pA[3][e];
        z.pc[0][e] = z.pc[2][e]; z.pc[1][e] = z.pc[3][e];
        z.ps[0][e] = z.ps[2][e]; z.ps[1][e] = z.ps[3][e];
        z.pm[0][e] = z.pm[2][e]; z.pm[1][e] = z.pm[3][e];
        if (MAP) { z.pq[0][e] = z.pq[2][e]; z.pq[1][e] = z.pq[3][e]; }
      }
      z.pA[2][0] = A0; z.pA[2][1] = A1;
      z.pc[2][0] = c0; z.pc[2][1] = c1;
      z.ps[2][0] = s0; z.ps[2][1] = s1;
      z.pm[2][0] = m0; z.pm[2][1] = m1;
      if (MAP) { z.pq[2][0] = d.s0; z.pq[2][1] = d.s1; }
    }
  }

  // FUSE: the level-l Laplacian of the output at fine rows 2 ci - 2 (even) and
  // 2 ci - 1 (odd), from coarse rows ci - 2, ci - 1, ci of level l + 1:
  //   L_l[O] = A - E(G_{l+1}) + m sum_k (sin E(C~_{l+1,k}) - cos E(S~_{l+1,k}))
  // (Eq. (14)), stored in the O_l slot; the collapse then adds E(O_{l+1}).
  __device__ inline void finish(int ci) {
    float EG[4];
    expand4(z.Gm, z.G0, z.Gp, EG);
    Harmonics hm[4];
    TermScale ts[4];
    float acc[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      hm[p].init(z.pc[p >> 1][p & 1], z.ps[p >> 1][p & 1]);
      if (MAP) ts[p].init(z.pq[p >> 1][p & 1], a.cf);
      acc[p] = 0.f;
    }
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      if (EX || k < K) {
        float EC[4], ES[4];
        expand4(z.Cm[k], z.C0[k], z.Cp[k], EC);
        expand4(z.Sm[k], z.S0[k], z.Sp[k], ES);
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          if (MAP) {
            acc[p] = fmaf(ts[p].e, fmaf(hm[p].s, EC[p], -hm[p].c * ES[p]), acc[p]);
            ts[p].next();
          } else {
            acc[p] = fmaf(hm[p].s, EC[p], fmaf(-hm[p].c, ES[p], acc[p]));
          }
          hm[p].next();
        }
      }
    }
    if (MAP) {
#pragma unroll
      for (int p = 0; p < 4; ++p) acc[p] *= ts[p].r3;
    }
    // EXPAND weights (1 6 1)/8 and (1 1)/2 per axis, by the block position
    const float scl[4] = {1.f / 64.f, 1.f / 16.f, 1.f / 16.f, 1.f / 4.f};
    float o[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      o[p] = fmaf(scl[p], fmaf(z.pm[p >> 1][p & 1], acc[p], -EG[p]), z.pA[p >> 1][p & 1]);
      asm volatile("" : "+v"(o[p]));  // keeps the arithmetic next to its lane shifts
    }
    if (!writer) return;
    const Plane op(a.af + (size_t)c * a.af_cs, a.g.nt);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = 2 * ci - 2 + q;
      if (r >= 2 * i0 && r < 2 * i1 && r < a.g.Hf) {
        const uint32_t so = (uint32_t)r * (uint32_t)a.g.pf * 4u;
        if (two) op.st2(make_float2(o[2 * q], o[2 * q + 1]), vx, so);
        else op.st1(o[2 * q], vx, so);
      }
    }
  }

  // Row 2 i0 - 2 only seeds P1 (the running sum of coarse row i0); the loop
  // then starts one coarse row early, and its first emission (coarse row
  // i0 - 1, incomplete) is not stored.  A single steady-state loop body keeps
  // the register peak that of one row plus the prefetched next row.
  template <bool BORDER, bool BS = false>
  __device__ inline void stream() {
    // FUSE also needs coarse rows i0 - 1 and i1 (EXPAND halo): one coarse row
    // more on each side
    const int first = FUSE ? i0 - 2 : i0 - 1, last = FUSE ? i1 + 1 : i1;
    RowIn A, B;
    load<BORDER, BS>(A, 2 * first);
    load<BORDER, BS>(B, 2 * first + 1);
    ready<BORDER, BS>(A);
    process<0>(A, 2 * first, first);
    for (int i = first; i < last; ++i) {
      load<BORDER, BS>(A, 2 * i + 2);
      ready<BORDER, BS>(B);
      process<3>(B, 2 * i + 1, i);
      load<BORDER, BS>(B, 2 * i + 3);
      ready<BORDER, BS>(A);
      process<4>(A, 2 * i + 2, i);
    }
  }

  // one wave-uniform branch selects the row loop of interior strips, of border
  // strips read as spans, or of border strips read per lane
  __device__ inline void run() {
    if (!border) {
      stream<false>();
    } else if constexpr (BSPAN) {
      if (bspan) stream<true, true>(); else stream<true>();
    } else {
      stream<true>();
    }
  }
};

template <int ST, int KM, bool EX, bool L0, bool MAP, bool FUSE, bool FAST = false>
__global__ void __launch_bounds__(256, down_waves_per_simd(KM, MAP, FUSE)) down_kernel(DownArgs a) {
  using W = DownWave<ST, KM, EX, L0, MAP, FUSE, FAST>;
  constexpr int SLICE = W::SLICE;
  __shared__ __attribute__((aligned(16))) uint32_t stage[4 * SLICE];
  int lane, strip, seg, c;
  if (!wave_coords(a.g, lane, strip, seg, c)) return;  // uniform per wave
  W w(a, lane, c, strip, seg, stage + (threadIdx.x >> 6) * SLICE);
  w.run();
}

template <int ST, int KM, bool EX, bool L0, bool MAP, bool FUSE>
__global__ void __launch_bounds__(256, down_waves_per_simd(KM, MAP, FUSE))
down_batch_kernel(const DownArgs *__restrict__ jobs, const uint32_t *__restrict__ start, int n,
                  uint32_t total) {
  using W = DownWave<ST, KM, EX, L0, MAP, FUSE>;
  constexpr int SLICE = W::SLICE;
  __shared__ __attribute__((aligned(16))) uint32_t stage[4 * SLICE];
  const int lane = threadIdx.x & 63;
  const uint32_t stride = gridDim.x * 4u;
  for (uint32_t w = first_wave(); w < total; w += stride) {
    const int j = find_job(start, n, w);
    const DownArgs &a = jobs[j];
    int strip, seg, c;
    job_coords(a.g, w - start[j], strip, seg, c);
    W wv(a, lane, c, strip, seg, stage + (threadIdx.x >> 6) * SLICE);
    wv.run();
  }
}

// --------------------------------------------------------------------------
// Collapse at levels l >= 1 (Eq. (4)): O_l = L_l[O] + EXPAND(O_{l+1}), in place
// in the O_l slot (which holds L_l[O] from down(l)); O_{l+1} = G_{l+1} when
// level l + 1 is the top.  One plane in, one plane out.  Standard strips.
// --------------------------------------------------------------------------
struct CollapseWave {
  const UpArgs &a;
  int i0, i1, x0;
  bool writer, two, border;
  uint32_t vcj, vx, vxa, vxb;
  const float *oc;
  float *outp;

  __device__ CollapseWave(const UpArgs &args, int lane, int c, int strip, int seg) : a(args) {
    const Geom &g = a.g;
    const int j = strip * 62 + lane - 1;
    vcj = (uint32_t)cfold(j, g.Wc, g.Wf) * 4u;
    i0 = seg * g.S;
    i1 = min(i0 + g.S, g.Hc);
    writer = lane >= 1 && lane <= 62 && j < g.Wc;
    border = sgpr(border_strip(strip, g.Wf));
    x0 = 2 * j;
    two = x0 + 1 < g.Wf;
    vx = (uint32_t)max(x0, 0) * 4u;
    vxa = (uint32_t)min(max(x0, 0), g.Wf - 1) * 4u;
    vxb = (uint32_t)min(max(x0 + 1, 0), g.Wf - 1) * 4u;
    oc = a.oc + (size_t)c * a.oc_cs;
    outp = a.out + (size_t)c * a.out_cs;
  }

  __device__ inline float load_c(int i) const {
    const uint32_t ci = (uint32_t)cfold(i, a.g.Hc, a.g.Hf) * (uint32_t)a.g.pc;
    return Plane(oc).ld1(vcj, ci * 4u);
  }

  template <bool BORDER>
  __device__ inline void load_f(float *f, int i) const {
    const Plane op(outp);
    const uint32_t r0 = 2 * i, r1 = min(2 * i + 1, a.g.Hf - 1);
    const uint32_t s0 = r0 * (uint32_t)a.g.pf * 4u, s1 = r1 * (uint32_t)a.g.pf * 4u;
    if (BORDER) {
      f[0] = op.ld1(vxa, s0);
      f[1] = op.ld1(vxb, s0);
      f[2] = op.ld1(vxa, s1);
      f[3] = op.ld1(vxb, s1);
    } else {
      const float2 u = op.ld2(opaque(vx), s0), v = op.ld2(opaque(vx), s1);
      f[0] = u.x;
      f[1] = u.y;
      f[2] = v.x;
      f[3] = v.y;
    }
  }

  template <bool BORDER>
  __device__ inline void stream() {
    const Geom &g = a.g;
    float Dm = load_c(i0 - 1), D0 = load_c(i0), Dp = load_c(i0 + 1);
    float fa[4], fb[4];
    load_f<BORDER>(fa, i0);
    const Plane op(outp, a.g.nt);
    const float scl[4] = {1.f / 64.f, 1.f / 16.f, 1.f / 16.f, 1.f / 4.f};
    for (int i = i0; i < i1; ++i) {
      const float Dn = load_c(i + 2);
      load_f<BORDER>(fb, i + 1 < i1 ? i + 1 : i);
      float E[4], o[4];
      expand4(Dm, D0, Dp, E);
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        o[p] = fmaf(scl[p], E[p], fa[p]);
        asm volatile("" : "+v"(o[p]));  // keeps the arithmetic next to its lane shifts
      }
      if (writer) {
        const uint32_t r0 = 2 * i;
        const bool row1 = (int)r0 + 1 < g.Hf;
        const uint32_t s0 = r0 * (uint32_t)g.pf * 4u, s1 = s0 + (uint32_t)g.pf * 4u;
        if (two) {
          op.st2(make_float2(o[0], o[1]), vx, s0);
          if (row1) op.st2(make_float2(o[2], o[3]), vx, s1);
        } else {
          op.st1(o[0], vx, s0);
          if (row1) op.st1(o[2], vx, s1);
        }
      }
      Dm = D0;
      D0 = Dp;
      Dp = Dn;
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[p] = fb[p];
    }
  }

  __device__ inline void run() {
    if (border) stream<true>(); else stream<false>();
  }
};

template <int ST>
__global__ void __launch_bounds__(256, 2) collapse_kernel(UpArgs a) {
  int lane, strip, seg, c;
  if (!wave_coords(a.g, lane, strip, seg, c)) return;  // uniform per wave
  CollapseWave w(a, lane, c, strip, seg);
  w.run();
}

template <int ST>
__global__ void __launch_bounds__(256, 2)
collapse_batch_kernel(const UpArgs *__restrict__ jobs, const uint32_t *__restrict__ start, int n, uint32_t total) {
  const int lane = threadIdx.x & 63;
  const uint32_t stride = gridDim.x * 4u;
  for (uint32_t w = first_wave(); w < total; w += stride) {
    const int j = find_job(start, n, w);
    const UpArgs &a = jobs[j];
    int strip, seg, c;
    job_coords(a.g, w - start[j], strip, seg, c);
    CollapseWave wv(a, lane, c, strip, seg);
    wv.run();
  }
}

// --------------------------------------------------------------------------
// up(l)
// --------------------------------------------------------------------------

// RW: re-parameterisation; the resident records carry the previous alpha~_k
// and every term is reweighted by wt[k] (new / previous alpha~_k).
// FOLD (level 0 only): the collapse of level 1 is done here, on the fly:
// O_1 - G_1 = (L_1[O] - G_1) + EXPAND(O_2) at every level-1 sample the pass reads.
// FAST: the fast LLF comparator: O_l = A_l - sum_j w_j(G_l[I]) EXPAND(G_{l+1}[r(I, tau j)])
// + EXPAND(O_{l+1}) (O_top = G_top[I], passed as oc with oc_minus_g); at level 0
// A_0 is the interpolation of r(I_p, tau j) at I_p.
template <int ST, int KM, bool EX, bool L0, bool MAP, bool HASD, bool RW = false, bool FOLD = false,
          bool FAST = false>
struct UpWave {
  static_assert(!FOLD || (L0 && HASD && !RW), "the level-1 collapse folds into up(0) only");
  static_assert(!FAST || (HASD && !MAP && !RW && !FOLD), "fast LLF: separate passes, O_{l+1} always given");
  using PS = PairStore<ST>;
  static constexpr int DW = PS::DW;
  static constexpr int NR = KM * DW;
  struct CRow {  // coarse row as loaded (raw): O_{l+1}, G_{l+1}, pair record, at column cj
    float o, g;
    float e[FOLD ? 9 : 1];  // FOLD: O_2 at rows p-1..p+1 x columns q-1..q+1 around (ci, cj)
    int par;                // FOLD: parity of the level-1 row ci
    uint32_t q[NR];
  };
  struct FBlk {  // fine 2x2 block as loaded: G (or I), A (or I), boost, range scale
    float g[4], b[4], m[4], s[4];
  };
  // Each lane loads its own records (16-byte loads).  Unlike the down passes,
  // the up passes read them faster this way than as a coalesced span
  // transposed through LDS (4K RGB K=8 up(0): float32 133.5 -> 132 us,
  // float16 93 -> 92 us).
  const UpArgs &a;
  int c, K, nr, j, i0, i1, x0, lane;
  bool writer, two, border, vec_f;
  uint32_t rec, vcj, vpcj, vx, vxa, vxb;  // record bytes, lane byte offsets
  const float *gc, *oc, *base, *gfp;
  const uint32_t *csc;
  float *outp;
  const float *o2p;   // FOLD: O_2 of this channel
  uint32_t vq[3];     // FOLD: byte offsets of the level-2 columns q-1, q, q+1 (folded)
  float wx[3];        // FOLD: their EXPAND weights at the lane's level-1 column

  __device__ UpWave(const UpArgs &args, int lane_, int c_, int strip, int seg) : a(args) {
    const Geom &g = a.g;
    lane = lane_;
    c = c_;
    K = EX ? KM : a.cf.K;
    nr = K * DW;
    rec = 4u * (uint32_t)nr;
    j = strip * 62 + lane - 1;
    const int cj = cfold(j, g.Wc, g.Wf);
    vcj = (uint32_t)cj * 4u;
    vpcj = (uint32_t)cj * rec;
    i0 = seg * g.S;
    i1 = min(i0 + g.S, g.Hc);
    writer = lane >= 1 && lane <= 62 && j < g.Wc;
    border = sgpr(border_strip(strip, g.Wf));  // uniform
    x0 = 2 * j;
    two = x0 + 1 < g.Wf;
    // border waves read clamped columns (values of non-writer lanes are unused)
    vx = (uint32_t)max(x0, 0) * 4u;
    vxa = (uint32_t)min(max(x0, 0), g.Wf - 1) * 4u;
    vxb = (uint32_t)min(max(x0 + 1, 0), g.Wf - 1) * 4u;
    gfp = a.gf + (size_t)c * a.gf_cs;
    outp = a.out + (size_t)c * a.out_cs;
    // the caller's output (level 0) has arbitrary pitch and alignment
    vec_f = !L0 || (((g.po & 1) == 0) && ((reinterpret_cast<uintptr_t>(outp) & 7) == 0));
    gc = a.gc + (size_t)c * a.gc_cs;
    oc = HASD ? a.oc + (size_t)c * a.oc_cs : nullptr;
    csc = a.csc + (size_t)c * a.csc_cs;
    base = a.base + (size_t)c * a.base_cs;
    if (FOLD) {
      o2p = a.o2 + (size_t)c * a.o2_cs;
      const int q = cj >> 1;
      const bool odd = cj & 1;
#pragma unroll
      for (int d = 0; d < 3; ++d) vq[d] = (uint32_t)cfold(q + d - 1, a.w2, g.Wc) * 4u;
      wx[0] = odd ? 0.f : 0.125f;
      wx[1] = odd ? 0.5f : 0.75f;
      wx[2] = odd ? 0.5f : 0.125f;
    }
  }

  template <bool BORDER>
  __device__ inline void load_c(CRow &d, int i) const {
    const int cr = cfold(i, a.g.Hc, a.g.Hf);
    const uint32_t ci = (uint32_t)cr * (uint32_t)a.g.pc;
    if (HASD) {
      d.o = Plane(oc).ld1(vcj, ci * 4u);
      d.g = a.oc_minus_g ? 0.f : Plane(gc).ld1(vcj, ci * 4u);  // wave-uniform
    }
    if (FOLD) {  // the 3 x 3 level-2 neighbourhood that EXPAND takes to (cr, cj)
      d.par = cr & 1;
      const Plane p2(o2p);
#pragma unroll
      for (int dy = 0; dy < 3; ++dy) {
        const uint32_t ro = (uint32_t)cfold((cr >> 1) + dy - 1, a.h2, a.g.Hc) * (uint32_t)a.p2 * 4u;
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) d.e[3 * dy + dx] = p2.ld1(vq[dx], ro);
      }
    }
    ld_record<NR, EX>(Plane(csc), opaque(vpcj), ci * rec, nr, d.q);
  }

  // O_{l+1} - G_{l+1} at a coarse sample (FOLD: the level-1 collapse, on the fly;
  // EXPAND weights (1 6 1)/8 at even and (0 4 4)/8 at odd level-1 positions)
  __device__ inline float dval(const CRow &d) const {
    if (!FOLD) return d.o - d.g;
    const float w0 = d.par ? 0.f : 0.125f, w1 = d.par ? 0.5f : 0.75f, w2 = d.par ? 0.5f : 0.125f;
    float h[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
      h[dy] = fmaf(wx[0], d.e[3 * dy], fmaf(wx[1], d.e[3 * dy + 1], wx[2] * d.e[3 * dy + 2]));
    return d.o + fmaf(w0, h[0], fmaf(w1, h[1], w2 * h[2]));
  }

  // pair k of a coarse record as float32 (reweighted when re-parameterising)
  __device__ inline float2 term(const uint32_t *q, int k) const {
    const float2 v = PS::cvt(&q[k * DW]);
    if (!RW) return v;
    return make_float2(v.x * a.cf.wt[k], v.y * a.cf.wt[k]);
  }

  // Two fine samples of one float row: clamped columns in border strips, one
  // contiguous 8-byte access otherwise.
  template <bool BORDER>
  __device__ inline void ld_f2(const Plane &p, uint32_t so, float &x, float &y) const {
    if (BORDER) {
      x = p.ld1(vxa, so);
      y = p.ld1(vxb, so);
    } else {
      const float2 v = p.ld2(opaque(vx), so);
      x = v.x;
      y = v.y;
    }
  }

  template <bool BORDER>
  __device__ inline void load_f(FBlk &d, int i) const {
    const uint32_t r0 = 2 * i, r1 = min(2 * i + 1, a.g.Hf - 1);
    const uint32_t rr[2] = {r0, r1};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t so = rr[q] * (uint32_t)a.g.pf * 4u;
      ld_f2<BORDER>(Plane(gfp), so, d.g[2 * q], d.g[2 * q + 1]);
      if (!L0) ld_f2<BORDER>(Plane(base), so, d.b[2 * q], d.b[2 * q + 1]);
      if (MAP) {  // either map may be absent (wave-uniform): its scalar then
        const uint32_t sm = rr[q] * (uint32_t)a.g.pm * 4u;
        if (a.mf) ld_f2<BORDER>(Plane(a.mf), sm, d.m[2 * q], d.m[2 * q + 1]);
        else d.m[2 * q] = d.m[2 * q + 1] = a.cf.m;
        if (a.sf) ld_f2<BORDER>(Plane(a.sf), sm, d.s[2 * q], d.s[2 * q + 1]);
        else d.s[2 * q] = d.s[2 * q + 1] = a.cf.sref;
      }
    }
  }

  // one wave-uniform branch selects the row loop of border or interior strips
  __device__ inline void run() {
    if (border) stream<true>(); else stream<false>();
  }

  template <bool BORDER>
  __device__ inline void stream() {
    const Geom &g = a.g;
    // coarse rows i-1 and i as float32, row i+1 raw (prefetched one step ahead)
    float Dm = 0.f, D0 = 0.f, Cm[KM], C0[KM], Sm[KM], S0[KM];
    CRow rp, rn;
    FBlk fa, fb;
    {
      // the first three coarse rows and the first fine block are all in flight at once
      CRow t0, t1;
      load_c<BORDER>(t0, i0 - 1);
      load_c<BORDER>(t1, i0);
      load_c<BORDER>(rp, i0 + 1);
      load_f<BORDER>(fa, i0);
      if (HASD) Dm = dval(t0);
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (EX || k < K) { const float2 v = term(t0.q, k); Cm[k] = v.x; Sm[k] = v.y; }
      if (HASD) D0 = dval(t1);
#pragma unroll
      for (int k = 0; k < KM; ++k)
        if (EX || k < K) { const float2 v = term(t1.q, k); C0[k] = v.x; S0[k] = v.y; }
    }
    const Plane op(outp, a.g.nt);
    for (int i = i0; i < i1; ++i) {
      const bool more = i + 1 < i1;  // wave-uniform: the next rows are needed
      if (more) load_c<BORDER>(rn, i + 2);
      if (more) load_f<BORDER>(fb, i + 1);
      const float Dp = HASD ? dval(rp) : 0.f;
      float ED[4] = {0.f, 0.f, 0.f, 0.f};
      if (HASD) expand4(Dm, D0, Dp, ED);
      Harmonics hm[4];
      TermScale ts[4];
      float acc[4];
      float tp[4];  // FAST: sample positions of G_l[I]
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (FAST) {
          tp[p] = sample_pos(fa.g[p], a.cf);
        } else {
          float s, cc;
          sincos2pi(fa.g[p] * a.cf.inv_T, s, cc);
          hm[p].init(cc, s);
        }
        if (MAP) ts[p].init(fa.s[p], a.cf);
        acc[p] = 0.f;
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (EX || k < K) {
          const float2 v = term(rp.q, k);
          float EC[4], ES[4];
          expand4(Cm[k], C0[k], v.x, EC);
          expand4(Sm[k], S0[k], v.y, ES);
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            if (FAST) {
              acc[p] = fmaf(hat(tp[p], (float)(2 * k)), EC[p], fmaf(hat(tp[p], (float)(2 * k + 1)), ES[p], acc[p]));
            } else if (MAP) {
              acc[p] = fmaf(ts[p].e, fmaf(hm[p].s, EC[p], -hm[p].c * ES[p]), acc[p]);
              ts[p].next();
            } else {
              acc[p] = fmaf(hm[p].s, EC[p], fmaf(-hm[p].c, ES[p], acc[p]));
            }
            if (!FAST) hm[p].next();
          }
          Cm[k] = C0[k];
          C0[k] = v.x;
          Sm[k] = S0[k];
          S0[k] = v.y;
        }
      }
      if (MAP) {
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[p] *= ts[p].r3;
      }
      // EXPAND weights (1 6 1)/8 and (1 1)/2 per axis, by the block position
      const float scl[4] = {1.f / 64.f, 1.f / 16.f, 1.f / 16.f, 1.f / 4.f};
      float o[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        // fast LLF subtracts the interpolated EXPAND of the sampled remaps
        const float mp = FAST ? -1.f : MAP ? fa.m[p] : a.cf.m;
        const float bp = L0 ? (FAST ? fast_level0(fa.g[p], a.cf) : fa.g[p]) : fa.b[p];
        o[p] = fmaf(scl[p], fmaf(mp, acc[p], ED[p]), bp);
        // computed by every lane here: keeps the arithmetic next to its lane
        // shifts, which then fold into DPP adds (else it sinks into the
        // writers-only block below and every shift stays a separate move)
        asm volatile("" : "+v"(o[p]));
      }
      if (writer) {
        const uint32_t r0 = 2 * i;
        const bool row1 = (int)r0 + 1 < g.Hf;
        const uint32_t s0 = r0 * (uint32_t)g.po * 4u, s1 = s0 + (uint32_t)g.po * 4u;
        if (two && vec_f) {
          op.st2(make_float2(o[0], o[1]), vx, s0);
          if (row1) op.st2(make_float2(o[2], o[3]), vx, s1);
        } else {
          op.st1(o[0], vx, s0);
          if (two) op.st1(o[1], vx + 4u, s0);
          if (row1) {
            op.st1(o[2], vx, s1);
            if (two) op.st1(o[3], vx + 4u, s1);
          }
        }
      }
      Dm = D0;
      D0 = Dp;
      rp = rn;
      fa = fb;
    }
  }
};

template <int ST, int KM, bool EX, bool L0, bool MAP, bool HASD, bool RW = false, bool FOLD = false,
          bool FAST = false>
__global__ void __launch_bounds__(256, min_waves_per_simd(KM)) up_kernel(UpArgs a) {
  using W = UpWave<ST, KM, EX, L0, MAP, HASD, RW, FOLD, FAST>;
  int lane, strip, seg, c;
  if (!wave_coords(a.g, lane, strip, seg, c)) return;  // uniform per wave
  W w(a, lane, c, strip, seg);
  w.run();
}

template <int ST, int KM, bool EX, bool L0, bool MAP, bool HASD, bool FOLD = false>
__global__ void __launch_bounds__(256, min_waves_per_simd(KM))
up_batch_kernel(const UpArgs *__restrict__ jobs, const uint32_t *__restrict__ start, int n, uint32_t total) {
  using W = UpWave<ST, KM, EX, L0, MAP, HASD, false, FOLD>;
  const int lane = threadIdx.x & 63;
  const uint32_t stride = gridDim.x * 4u;
  for (uint32_t w = first_wave(); w < total; w += stride) {
    const int j = find_job(start, n, w);
    const UpArgs &a = jobs[j];
    int strip, seg, c;
    job_coords(a.g, w - start[j], strip, seg, c);
    W wv(a, lane, c, strip, seg);
    wv.run();
  }
}

// --------------------------------------------------------------------------
// Re-parameterisation: the level-l half of Eq. (14) from resident pyramids,
//   A_l = G_l - m sum_k wt_k (sin(w_k g) C~_{l,k} - cos(w_k g) S~_{l,k}),
// per pixel (no stencil), for a new boost m and new alpha~_k = wt_k x the
// resident ones.  One wave per 64 pixels of a row; rows are padded to 64, so
// a wave's records are always one in-bounds span (read coalesced).
// --------------------------------------------------------------------------
struct HalfArgs {
  const float *g; size_t g_cs;        // G_l
  const uint32_t *cs; size_t cs_cs;   // level-l records (dwords per channel)
  float *a; size_t a_cs;              // A_l (the O_l slot)
  int w, h, pitch, C, blocks;         // blocks = pitch / 64 per row
  Coefs cf;
};

template <int ST, int KM>
__global__ void __launch_bounds__(256) half_kernel(HalfArgs a) {
  using PS = PairStore<ST>;
  constexpr int DW = PS::DW, NR = KM * DW;
  __shared__ __attribute__((aligned(16))) uint32_t stage[4 * span_slice_dwords<NR>()];
  const int lane = threadIdx.x & 63;
  const int wv = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int blk = __builtin_amdgcn_readfirstlane(wv % a.blocks);
  const int rest = wv / a.blocks;
  const int y = __builtin_amdgcn_readfirstlane(rest % a.h);
  const int c = __builtin_amdgcn_readfirstlane(rest / a.h);
  if (c >= a.C) return;  // uniform per wave
  const uint32_t rec = 4u * NR;
  const uint32_t px0 = (uint32_t)y * (uint32_t)a.pitch + 64u * (uint32_t)blk;
  const int x = 64 * blk + lane;
  const float g = Plane(a.g + (size_t)c * a.g_cs).ld1(opaque(4u * (uint32_t)lane), px0 * 4u);
  uint32_t q[NR];
  ld_span<NR>(Plane(a.cs + (size_t)c * a.cs_cs), px0 * rec, lane, q);
  transpose_span<NR>(q, stage + (threadIdx.x >> 6) * span_slice_dwords<NR>(), lane);
  float sn, cs;
  sincos2pi(g * a.cf.inv_T, sn, cs);
  Harmonics h;
  h.init(cs, sn);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    const float2 v = PS::cvt(&q[k * DW]);
    acc = fmaf(a.cf.wt[k] * h.s, v.x, fmaf(-a.cf.wt[k] * h.c, v.y, acc));
    h.next();
  }
  if (x < a.w) Plane(a.a + (size_t)c * a.a_cs).st1(fmaf(-a.cf.m, acc, g), 4u * (uint32_t)lane, px0 * 4u);
}

// --------------------------------------------------------------------------
// Host-side launch sequence of one job.
// --------------------------------------------------------------------------
inline Geom make_geom(const Level &f, const Level &cl, int C, int S, int sw) {
  Geom g;
  g.Wf = f.w;
  g.Hf = f.h;
  g.Wc = cl.w;
  g.Hc = cl.h;
  g.pf = f.pitch;
  g.pc = cl.pitch;
  g.po = f.pitch;
  g.pm = f.pitch;
  g.nstrips = (cl.w + sw - 1) / sw;
  g.S = S;
  g.nsegs = (cl.h + S - 1) / S;
  g.C = C;
  g.nt = 0;
  return g;
}

// Rows per wave segment.  Shorter segments give more waves (latency hiding,
// fewer idle SIMDs in the last round) but re-read more halo rows; the target
// wave count of each pass kind is a tuning parameter.
inline int pick_segment(const Level &cl, int C, long target, int sw) {
  const long strips = (cl.w + sw - 1) / sw;
  int S = 64;
  while (S > 1 && strips * ((cl.h + S - 1) / S) * C < target) S /= 2;
  return S;
}

inline long geom_waves(const Geom &g) { return (long)g.nstrips * g.nsegs * g.C; }

// Levels l >= 1 of a job whose level l holds at least this many samples (all
// channels), with records the fused pass can hold (fusable), run the fused
// form: down(l) finishes L_l[O] and up(l) is the one-plane collapse.  Smaller levels are latency-bound: there the two extra
// coarse halo rows of every fused down wave cost more than the collapse saves,
// and they keep the separate form (down(l) stores A_l, up(l) does the EXPAND
// products and the collapse).  A property of the job alone, so that a job's
// result does not depend on the jobs batched with it.  At 2^19 rather than 2^20
// the 64-image batch runs 6.37 instead of 6.48 ms and a 1280x720 RGB image 104
// instead of 109 us (float32; float16 and the 4K image unchanged); at 2^18
// float16 is slower.
constexpr double kFuseMinSamples = 1 << 19;
inline bool fused_level(const JobPlan &P, int l) {
  const bool map = P.m_map != nullptr || P.s_map != nullptr;
  return l >= 1 && !P.fast && fusable(P.K, P.dwp, map) && (double)P.lv[l].n * P.C >= kFuseMinSamples;
}

// A fused level 1 below the top has its collapse folded into up(0), which then
// reads L_1[O] - G_1 and O_2 instead of O_1 - G_1 (one level-1 plane less to
// write and read, and one launch less).
inline bool fold_level1(const JobPlan &P) { return P.levels > 2 && fused_level(P, 1); }

// Segment target of the re-parameterised up passes: they evaluate the whole
// product-sum at every level from the resident records, which wants long
// segments (the autotuner times normal runs only, so this one is built in).
constexpr long kReparamUpWaves = 1536;

// Shortest segment of up(0): each segment re-reads two rows of level-1 records
// around it, which on small images (few columns, so one-row segments under a
// high wave target) would triple the record traffic.  The 3840x2160 workload
// takes 8-row segments anyway; a 64-image batch of 0.15-8.8 Mpixel images runs
// 7.07 ms instead of 7.82 (float32, built-in targets).
constexpr int kUp0MinSegment = 8;

// Geometry of pass down(l) / up(l) of a job: coarse columns per strip (the
// fused down(l) uses strips of 60) and the tuned segment length.  The up passes
// that evaluate the product-sum (level 0 and levels that are not fused) share
// one segment target; the one-plane collapse of the fused levels has its own.
inline Geom pass_geom(const JobPlan &P, int l, bool down, const Tuning &tu, bool reparam = false) {
  const bool collapse = !down && !reparam && fused_level(P, l);
  const int kind = down ? (l == 0 ? kTuneDown0 : kTuneDown) : (collapse ? kTuneUp : kTuneUp0);
  const long target = !down && reparam ? kReparamUpWaves : (long)tu.p[kind];
  const int sw = down && fused_level(P, l) ? 60 : 62;
  int S = pick_segment(P.lv[l + 1], P.C, target, sw);
  if (!down && l == 0 && !reparam && S < kUp0MinSegment) S = kUp0MinSegment;
  Geom g = make_geom(P.lv[l], P.lv[l + 1], P.C, S, sw);
  // non-temporal stores by pass kind (bits of the tuning parameter)
  const int bit = down ? (l == 0 ? kNtDown0 : fused_level(P, l) ? kNtDownFused : kNtDown) : (l == 0 ? kNtUp0 : kNtUp);
  g.nt = (tu.p[kTuneNtStores] >> bit) & 1;
  return g;
}

// Launch shape of a single-job pass: blocks of four waves, or of one wave when
// the pass has few waves.  A small level's pass is bound by the memory pipeline
// of the few compute units it occupies: one wave per block spreads it over four
// times as many (4K RGB float32: down passes at levels 4-6 from 10.2-11.0 to
// 7.3-8.8 us).  From about 800 waves on, four-wave blocks are faster again.
constexpr long kSmallPassWaves = 512;
inline dim3 block_for(const Geom &g) { return dim3(geom_waves(g) < kSmallPassWaves ? 64 : 256, 1, 1); }
inline dim3 grid_for(const Geom &g) {
  const long w = geom_waves(g);
  return dim3((unsigned)(w < kSmallPassWaves ? w : (w + 3) / 4), 1, 1);
}

// Arguments of down(l) / up(l) of one planned job whose workspace is ws.
inline DownArgs make_down_args(const JobPlan &P, int l, char *ws, int dwp, const Tuning &tu) {
  const Level *lv = P.lv;
  const int L = P.levels;
  // the Gaussian pyramid of a per-pixel map: the caller's map at level 0, the
  // workspace plane at levels 1 .. top-1 (the top level has no product-sum)
  auto M = [&](const float *map0, size_t Level::*off, int k) -> float * {
    if (!map0) return nullptr;
    if (k == 0) return const_cast<float *>(map0);
    return k < L - 1 ? (float *)(ws + lv[k].*off) : nullptr;
  };
  DownArgs a{};
  a.gf = l == 0 ? P.in : (const float *)(ws + lv[l].off_g);
  a.gf_cs = l == 0 ? P.in_cs : lv[l].g_cstride;
  a.csf = l == 0 ? nullptr : (const uint32_t *)(ws + lv[l].off_cs);
  a.csf_cs = lv[l].cs_cstride * dwp;
  a.mf = M(P.m_map, &Level::off_m, l);
  a.sf = M(P.s_map, &Level::off_s, l);
  a.gc = (float *)(ws + lv[l + 1].off_g);
  a.gc_cs = lv[l + 1].g_cstride;
  a.csc = (uint32_t *)(ws + lv[l + 1].off_cs);
  a.csc_cs = lv[l + 1].cs_cstride * dwp;
  a.mc = M(P.m_map, &Level::off_m, l + 1);
  a.sc = M(P.s_map, &Level::off_s, l + 1);
  a.af = l == 0 ? nullptr : (float *)(ws + lv[l].off_o);
  a.af_cs = lv[l].g_cstride;
  a.minus_g = l == 1 && fused_level(P, 1) && L > 2 ? 1 : 0;
  a.g = pass_geom(P, l, true, tu);
  if (l == 0) a.g.pm = lv[0].w;  // the caller's map has dense rows
  a.cf = P.coefs;
  return a;
}

inline UpArgs make_up_args(const JobPlan &P, int l, char *ws, int dwp, const Tuning &tu, bool reparam = false) {
  const Level *lv = P.lv;
  const int L = P.levels;
  UpArgs a{};
  a.base = l == 0 ? P.in : (const float *)(ws + lv[l].off_o);
  a.base_cs = l == 0 ? P.in_cs : lv[l].g_cstride;
  a.gf = l == 0 ? P.in : (const float *)(ws + lv[l].off_g);
  a.gf_cs = l == 0 ? P.in_cs : lv[l].g_cstride;
  a.mf = !P.m_map ? nullptr : l == 0 ? P.m_map : (const float *)(ws + lv[l].off_m);
  a.sf = !P.s_map ? nullptr : l == 0 ? P.s_map : (const float *)(ws + lv[l].off_s);
  a.gc = (const float *)(ws + lv[l + 1].off_g);
  a.gc_cs = lv[l + 1].g_cstride;
  const bool hasd = l + 1 < L - 1;
  a.oc = hasd ? (const float *)(ws + lv[l + 1].off_o) : nullptr;
  a.oc_cs = lv[l + 1].g_cstride;
  a.csc = (const uint32_t *)(ws + lv[l + 1].off_cs);
  a.csc_cs = lv[l + 1].cs_cstride * dwp;
  a.out = l == 0 ? P.out : (float *)(ws + lv[l].off_o);
  a.out_cs = l == 0 ? P.out_cs : lv[l].g_cstride;
  // the normal sequence leaves L_1[O] - G_1 in the O_1 slot when level 1 is
  // fused; up(0) adds EXPAND(O_2) itself
  a.oc_minus_g = l == 0 && hasd && !reparam && fused_level(P, 1) ? 1 : 0;
  if (a.oc_minus_g) {
    a.o2 = (const float *)(ws + (2 < L - 1 ? lv[2].off_o : lv[2].off_g));
    a.o2_cs = lv[2].g_cstride;
    a.w2 = lv[2].w;
    a.h2 = lv[2].h;
    a.p2 = lv[2].pitch;
  }
  if (P.fast) {  // O_{l+1}, or G_top[I] (the residual level) at the top; G_{l+1} is not subtracted
    a.oc = (const float *)(ws + (hasd ? lv[l + 1].off_o : lv[l + 1].off_g));
    a.oc_minus_g = 1;
  }
  a.g = pass_geom(P, l, false, tu, reparam);
  if (l == 0) {  // the caller's output and map rows
    a.g.po = P.out_pitch;
    a.g.pm = lv[0].w;
  }
  a.cf = P.coefs;
  return a;
}

// Algorithmic bytes: every plane element a launch must read or write, once.
inline double down_bytes(const JobPlan &P, int l, int dwp) {
  const Level *lv = P.lv;
  const double pb = 4.0 * dwp * P.K, C = P.C, mapb = (P.m_map ? 4.0 : 0.0) + (P.s_map ? 4.0 : 0.0);
  if (l == 0) return C * (4.0 * lv[0].n + (4.0 + pb) * lv[1].n) + mapb * (lv[0].n + lv[1].n);
  return C * ((4.0 + pb + 4.0) * lv[l].n + (4.0 + pb) * lv[l + 1].n) + mapb * (lv[l].n + lv[l + 1].n);
}

inline double up_bytes(const JobPlan &P, int l, int dwp, bool reparam = false) {
  const Level *lv = P.lv;
  const double pb = 4.0 * dwp * P.K, C = P.C, mapb = (P.m_map ? 4.0 : 0.0) + (P.s_map ? 4.0 : 0.0);
  const bool hasd = l + 1 < P.levels - 1;
  if (!reparam && fused_level(P, l)) return C * (8.0 * lv[l].n + 4.0 * lv[l + 1].n);  // L_l, O_l; O_{l+1}
  const bool fold = l == 0 && hasd && !reparam && fused_level(P, 1);  // L_1[O] - G_1, and O_2
  const double fine = l == 0 ? 4.0 : 8.0;                               // I, or A_l and G_l
  const double coarse = P.fast ? pb + 4.0                               // pairs, O_{l+1} (G_top)
                               : (fold ? 0.0 : 4.0) + pb + (hasd ? 4.0 : 0.0);  // G, pairs, O_{l+1}
  const double o2 = fold ? 4.0 * lv[2].n : 0.0;
  return C * ((fine + 4.0) * lv[l].n + coarse * lv[l + 1].n + o2) + mapb * lv[l].n;  // + O_l written
}

// The fused down pass exists for the fusable K loops only (fused_level never
// selects it for the others).
template <int ST, int KM, bool EX, bool MAP>
void launch_fused_down(const DownArgs &a, hipStream_t st) {
  if constexpr (EX && fusable(KM, PairStore<ST>::DW, MAP))
    down_kernel<ST, KM, EX, false, MAP, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
}

// up(0) with the level-1 collapse folded in: exists for the fusable K loops only
// (fold_level1 implies a fused level 1).
template <int ST, int KM, bool EX, bool MAP>
void launch_fold_up(const UpArgs &a, hipStream_t st) {
  if constexpr (EX && fusable(KM, PairStore<ST>::DW, MAP))
    up_kernel<ST, KM, EX, true, MAP, true, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
}

template <int ST, int KM, bool EX, bool MAP>
hipError_t launch_typed(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *hook, const Tuning &tu) {
  const int L = P.levels;
  const int dwp = PairStore<ST>::DW;  // dwords per pair
  auto pre = [&]() { if (hook) hook->before(st); };
  auto post = [&](const char *name, double bytes) { if (hook) hook->after(st, name, bytes); };
  for (int l = 0; l + 1 < L; ++l) {
    const DownArgs a = make_down_args(P, l, ws, dwp, tu);
    pre();
    if (l == 0) down_kernel<ST, KM, EX, true, MAP, false><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    else if (fused_level(P, l)) launch_fused_down<ST, KM, EX, MAP>(a, st);
    else down_kernel<ST, KM, EX, false, MAP, false><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    post(kDownNames[l], down_bytes(P, l, dwp));
  }
  for (int l = L - 2; l >= 0; --l) {
    if (l == 1 && fold_level1(P)) continue;  // done inside up(0)
    const UpArgs a = make_up_args(P, l, ws, dwp, tu);
    const bool hasd = a.oc != nullptr;
    pre();
    if (fused_level(P, l)) {
      UpArgs ca = a;
      if (!hasd) ca.oc = ca.gc;  // O_{l+1} is G_{l+1} at the top
      collapse_kernel<ST><<<grid_for(ca.g), block_for(ca.g), 0, st>>>(ca);
    } else if (l == 0) {
      if (a.o2) launch_fold_up<ST, KM, EX, MAP>(a, st);
      else if (hasd) up_kernel<ST, KM, EX, true, MAP, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
      else up_kernel<ST, KM, EX, true, MAP, false><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    } else {
      if (hasd) up_kernel<ST, KM, EX, false, MAP, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
      else up_kernel<ST, KM, EX, false, MAP, false><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    }
    post(kUpNames[l], up_bytes(P, l, dwp));
  }
  return hipGetLastError();
}

// Fast LLF (single jobs): the separate down and up passes with the sampled-remap
// basis; every up pass expands O_{l+1} (G_top[I] at the top).
template <int ST, int KM, bool EX>
hipError_t launch_fast_typed(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *hook, const Tuning &tu) {
  const int L = P.levels;
  const int dwp = PairStore<ST>::DW;
  for (int l = 0; l + 1 < L; ++l) {
    const DownArgs a = make_down_args(P, l, ws, dwp, tu);
    if (hook) hook->before(st);
    if (l == 0) down_kernel<ST, KM, EX, true, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    else down_kernel<ST, KM, EX, false, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    if (hook) hook->after(st, kDownNames[l], down_bytes(P, l, dwp));
  }
  for (int l = L - 2; l >= 0; --l) {
    const UpArgs a = make_up_args(P, l, ws, dwp, tu);
    if (hook) hook->before(st);
    if (l == 0)
      up_kernel<ST, KM, EX, true, false, true, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    else
      up_kernel<ST, KM, EX, false, false, true, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    if (hook) hook->after(st, kUpNames[l], up_bytes(P, l, dwp));
  }
  return hipGetLastError();
}

// The K loop of a job: K == 4, 8, 16 run exact loops; other K run the next
// larger loop with guards.
inline void k_class(int K, int *km, bool *ex) {
  if (K == 4 || K == 8 || K == 16) { *km = K; *ex = true; return; }
  *ex = false;
  *km = K < 8 ? 8 : K < 16 ? 16 : 32;
}

template <int ST>
hipError_t launch_storage(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  const bool map = P.m_map != nullptr || P.s_map != nullptr;  // per-pixel parameters
  int km;
  bool ex;
  k_class(P.K, &km, &ex);
  if (P.fast) {  // at most 16 pairs (32 samples)
    if (ex) return km == 4 ? launch_fast_typed<ST, 4, true>(P, ws, st, h, tu)
                           : km == 8 ? launch_fast_typed<ST, 8, true>(P, ws, st, h, tu)
                                     : launch_fast_typed<ST, 16, true>(P, ws, st, h, tu);
    return km == 8 ? launch_fast_typed<ST, 8, false>(P, ws, st, h, tu) : launch_fast_typed<ST, 16, false>(P, ws, st, h, tu);
  }
#define FLLF_LAUNCH(KM, EX) \
  return map ? launch_typed<ST, KM, EX, true>(P, ws, st, h, tu) : launch_typed<ST, KM, EX, false>(P, ws, st, h, tu)
  if (ex) {
    if (km == 4) FLLF_LAUNCH(4, true);
    if (km == 8) FLLF_LAUNCH(8, true);
    FLLF_LAUNCH(16, true);
  }
  if (km == 8) FLLF_LAUNCH(8, false);
  if (km == 16) {  // with a map, 9 to 15 terms are planned as the exact 16-term loop
    if (map) return hipErrorInvalidValue;
    return launch_typed<ST, 16, false, false>(P, ws, st, h, tu);
  }
  FLLF_LAUNCH(32, false);
#undef FLLF_LAUNCH
}

// Re-parameterised filter of a job whose pyramids are resident in ws: the
// half pass at levels 1 .. top-1, then the reweighted collapse passes.
template <int ST, int KM>
hipError_t launch_reparam_typed(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *hook, const Tuning &tu) {
  const int L = P.levels;
  const int dwp = PairStore<ST>::DW;
  const dim3 blk(256, 1, 1);
  const double pb = 4.0 * dwp * P.K;
  for (int l = 1; l + 1 < L; ++l) {
    const Level &lv = P.lv[l];
    HalfArgs a{};
    a.g = (const float *)(ws + lv.off_g);
    a.g_cs = lv.g_cstride;
    a.cs = (const uint32_t *)(ws + lv.off_cs);
    a.cs_cs = lv.cs_cstride * dwp;
    a.a = (float *)(ws + lv.off_o);
    a.a_cs = lv.g_cstride;
    a.w = lv.w;
    a.h = lv.h;
    a.pitch = lv.pitch;
    a.C = P.C;
    a.blocks = lv.pitch / 64;
    a.cf = P.coefs;
    const long waves = (long)a.blocks * lv.h * P.C;
    if (hook) hook->before(st);
    half_kernel<ST, KM><<<dim3((unsigned)((waves + 3) / 4)), blk, 0, st>>>(a);
    if (hook) hook->after(st, kHalfNames[l], (double)P.C * lv.n * (8.0 + pb));
  }
  for (int l = L - 2; l >= 0; --l) {
    const UpArgs a = make_up_args(P, l, ws, dwp, tu, true);
    const bool hasd = a.oc != nullptr;
    if (hook) hook->before(st);
    if (l == 0) {
      if (hasd) up_kernel<ST, KM, true, true, false, true, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
      else up_kernel<ST, KM, true, true, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    } else {
      if (hasd) up_kernel<ST, KM, true, false, false, true, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
      else up_kernel<ST, KM, true, false, false, false, true><<<grid_for(a.g), block_for(a.g), 0, st>>>(a);
    }
    if (hook) hook->after(st, kUpNames[l], up_bytes(P, l, dwp, true));
  }
  return hipGetLastError();
}

template <int ST>
hipError_t launch_reparam_storage(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  switch (P.K) {
    case 4: return launch_reparam_typed<ST, 4>(P, ws, st, h, tu);
    case 8: return launch_reparam_typed<ST, 8>(P, ws, st, h, tu);
    case 16: return launch_reparam_typed<ST, 16>(P, ws, st, h, tu);
    default: return hipErrorInvalidValue;  // the caller admits K = 4, 8, 16 only
  }
}

// --------------------------------------------------------------------------
// Batched launches
// --------------------------------------------------------------------------
// Blocks of 256 threads of `kernel` that fit on the device at once.
inline long resident_blocks(const void *kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess) return 0;
  return (long)cus * per_cu;
}

inline dim3 batch_grid(const BatchLaunch &b, const void *kernel, const Tuning &tu) {
  long blocks = ((long)b.waves + 3) / 4;
  if (tu.p[kTuneGridCap] > 0) {
    const long cap = resident_blocks(kernel) * tu.p[kTuneGridCap];
    if (cap > 0 && cap < blocks) blocks = cap;
  }
  return dim3((unsigned)blocks, 1, 1);
}

template <int ST, int KM, bool EX, bool MAP>
hipError_t launch_batch_typed(const BatchLaunch &b, char *ws, hipStream_t st, const Tuning &tu) {
  const dim3 blk(256, 1, 1);
  const uint32_t *start = (const uint32_t *)(ws + b.start_off);
  if (b.kind == 0) {
    const DownArgs *args = (const DownArgs *)(ws + b.args_off);
#define FLLF_DOWN(L0, FUSE)                                                             \
  {                                                                                     \
    auto k = down_batch_kernel<ST, KM, EX, L0, MAP, FUSE>;                              \
    k<<<batch_grid(b, (const void *)k, tu), blk, 0, st>>>(args, start, b.njobs, b.waves); \
  }
    if (b.l0) {
      FLLF_DOWN(true, false)
    } else if (b.fuse) {
      if constexpr (EX && fusable(KM, PairStore<ST>::DW, MAP)) FLLF_DOWN(false, true)
    } else {
      FLLF_DOWN(false, false)
    }
#undef FLLF_DOWN
  } else {
    const UpArgs *args = (const UpArgs *)(ws + b.args_off);
#define FLLF_UP(L0, HASD, FOLD)                                                         \
  {                                                                                     \
    auto k = up_batch_kernel<ST, KM, EX, L0, MAP, HASD, FOLD>;                          \
    k<<<batch_grid(b, (const void *)k, tu), blk, 0, st>>>(args, start, b.njobs, b.waves); \
  }
    // the product-sum and collapse (fused levels run collapse_batch_kernel); at
    // level 0, fuse marks the jobs whose level-1 collapse is folded in
    if (b.l0) {
      if (b.fuse) {
        if constexpr (EX && fusable(KM, PairStore<ST>::DW, MAP)) FLLF_UP(true, true, true)
      } else if (b.hasd) {
        FLLF_UP(true, true, false)
      } else {
        FLLF_UP(true, false, false)
      }
    } else {
      if (b.hasd) FLLF_UP(false, true, false) else FLLF_UP(false, false, false)
    }
#undef FLLF_UP
  }
  return hipGetLastError();
}

template <int ST>
hipError_t launch_batch_storage(const BatchSchedule &s, char *ws, hipStream_t st, LaunchHook *hook,
                                const Tuning &tu) {
  for (const BatchLaunch &b : s.launches) {
    if (hook) hook->before(st);
    hipError_t e = hipSuccess;
    if (b.kind == 2) {
      e = copy_image(b.copy, st);
    } else if (b.kind == 1 && b.fuse && !b.l0) {  // the collapse does not depend on K
      const UpArgs *args = (const UpArgs *)(ws + b.args_off);
      const uint32_t *start = (const uint32_t *)(ws + b.start_off);
      auto k = collapse_batch_kernel<ST>;
      k<<<batch_grid(b, (const void *)k, tu), dim3(256, 1, 1), 0, st>>>(args, start, b.njobs, b.waves);
      e = hipGetLastError();
    } else {
#define FLLF_B(KM, EX) \
  e = b.map ? launch_batch_typed<ST, KM, EX, true>(b, ws, st, tu) : launch_batch_typed<ST, KM, EX, false>(b, ws, st, tu)
      if (b.ex) {
        if (b.km == 4) FLLF_B(4, true);
        else if (b.km == 8) FLLF_B(8, true);
        else FLLF_B(16, true);
      } else {
        if (b.km == 8) FLLF_B(8, false);
        else if (b.km == 16 && !b.map) e = launch_batch_typed<ST, 16, false, false>(b, ws, st, tu);
        else if (b.km == 16) e = hipErrorInvalidValue;  // planned as the exact 16-term loop
        else FLLF_B(32, false);
      }
#undef FLLF_B
    }
    if (e != hipSuccess) return e;
    if (hook)
      hook->after(st, b.kind == 0 ? kBatchDownNames[b.level] : b.kind == 1 ? kBatchUpNames[b.level] : "copy",
                  b.bytes);
  }
  return hipSuccess;
}

}  // namespace fllf
