// Boost map for pixel-by-pixel enhancement driven by local variance (Sec. IV,
// the discussion of the pixel-by-pixel enhancement figure: the enhancement of
// a pixel follows the variance of the pixels in a window around it, small where
// the variance is low).  Reading: the window is the (2r+1) x (2r+1) square
// around p with reflect-101 borders, v_p its population variance, and
//   m_p = m_max v_p / (v_p + v_half)
// (0 on flat areas, m_max / 2 at v_p = v_half, towards m_max on strong texture).
//
// One block of 256 threads per 64 x 16 tile of the map: the tile and its halo
// of r samples are staged in LDS with folded coordinates, then every thread
// computes four outputs of one column, each in two passes over its window (the
// mean first, then the mean squared deviation from it: no cancellation).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fllf_internal.h"

namespace fllf {

constexpr int kTileW = 64, kTileH = 16;

// Reflect-101 fold onto [0, n) for any i (n >= 1).
__device__ inline int fold(int i, int n) {
  if (n == 1) return 0;
  const int p = 2 * n - 2;
  i %= p;
  if (i < 0) i += p;
  return i > n - 1 ? p - i : i;
}

__global__ void __launch_bounds__(256) boost_map_kernel(const float *__restrict__ in, int64_t pitch, int w, int h,
                                                          int r, float m_max, float v_half, float *__restrict__ out) {
  extern __shared__ float tile[];  // (kTileH + 2r) rows of (kTileW + 2r)
  const int tw = kTileW + 2 * r, th = kTileH + 2 * r;
  const int x0 = blockIdx.x * kTileW, y0 = blockIdx.y * kTileH;
  for (int i = threadIdx.x; i < tw * th; i += blockDim.x) {
    const int ty = i / tw, tx = i - ty * tw;
    const int gy = fold(y0 + ty - r, h), gx = fold(x0 + tx - r, w);
    tile[i] = in[(int64_t)gy * pitch + gx];
  }
  __syncthreads();
  const int lx = threadIdx.x & (kTileW - 1), ly0 = (threadIdx.x >> 6) * 4;
  const int x = x0 + lx;
  const float inv_n = 1.f / (float)((2 * r + 1) * (2 * r + 1));
  for (int q = 0; q < 4; ++q) {
    const int ly = ly0 + q, y = y0 + ly;
    if (x >= w || y >= h) continue;
    float s = 0.f;
    for (int dy = 0; dy <= 2 * r; ++dy)
      for (int dx = 0; dx <= 2 * r; ++dx) s += tile[(ly + dy) * tw + lx + dx];
    const float mean = s * inv_n;
    float d2 = 0.f;
    for (int dy = 0; dy <= 2 * r; ++dy)
      for (int dx = 0; dx <= 2 * r; ++dx) {
        const float d = tile[(ly + dy) * tw + lx + dx] - mean;
        d2 = fmaf(d, d, d2);
      }
    const float v = d2 * inv_n;
    out[(int64_t)y * w + x] = m_max * v / (v + v_half);
  }
}


}  // namespace fllf

extern "C" fllf_status fourier_llf_boost_map(fllf_ctx *ctx, const float *in, int32_t width, int32_t height,
                                             int64_t row_pitch, int32_t radius, double m_max, double v_half,
                                             float *out, void *hip_stream) {
  if (!ctx) return fllf::ctx_fail(nullptr, FLLF_EINVAL, "boost_map: ctx is NULL");
  if (!in || !out) return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: in and out must be non-NULL");
  if (width < 1 || height < 1 || width > 65536 || height > 65536 || (int64_t)width * height > ((int64_t)1 << 30))
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: bad size %d x %d", width, height);
  const int64_t pitch = row_pitch > 0 ? row_pitch : width;
  if (row_pitch < 0 || pitch < width)
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: row_pitch must be 0 or >= width");
  if (radius < 0 || radius > 32) return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: radius %d outside [0, 32]", radius);
  if (!std::isfinite(m_max) || !std::isfinite(v_half) || v_half <= 0.0)
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: need a finite m_max and v_half > 0");
  const size_t in_bytes = (size_t)((int64_t)(height - 1) * pitch + width) * sizeof(float);
  if (fllf::spans_overlap(in, in_bytes, out, (size_t)width * height * sizeof(float)))
    return fllf::ctx_fail(ctx, FLLF_EINVAL, "boost_map: in and out overlap");
  hipError_t e = hipSetDevice(fllf::ctx_device(ctx));
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "boost_map: %s", hipGetErrorString(e));
  const int tw = fllf::kTileW, th = fllf::kTileH;
  const dim3 grid((unsigned)((width + tw - 1) / tw), (unsigned)((height + th - 1) / th), 1);
  const size_t lds = sizeof(float) * (size_t)(tw + 2 * radius) * (th + 2 * radius);
  fllf::boost_map_kernel<<<grid, dim3(256, 1, 1), lds, (hipStream_t)hip_stream>>>(
      in, pitch, width, height, radius, (float)m_max, (float)v_half, out);
  e = hipGetLastError();
  if (e != hipSuccess) return fllf::ctx_fail(ctx, FLLF_EDEVICE, "boost_map: launch: %s", hipGetErrorString(e));
  return FLLF_OK;
}
