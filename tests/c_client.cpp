// A host program that uses the library through its C interface only (no
// Python, no torch): reads a planar float32 image from a file, filters it on
// device 0 and writes the output.
//
//   c_client IN OUT WIDTH HEIGHT CHANNELS LEVELS SIGMA_R M K STORAGE
//
// STORAGE is f32, f16 or bf16.  Exit status 0 on success; otherwise the
// library's message is printed and the status is 2 (bad arguments or file),
// 3 (library error) or 4 (HIP error).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "fourier_llf.h"

static int hip_fail(hipError_t e, const char *what) {
  std::fprintf(stderr, "c_client: %s: %s\n", what, hipGetErrorString(e));
  return 4;
}

int main(int argc, char **argv) {
  if (argc != 11) {
    std::fprintf(stderr, "usage: %s IN OUT WIDTH HEIGHT CHANNELS LEVELS SIGMA_R M K STORAGE\n", argv[0]);
    return 2;
  }
  const int W = std::atoi(argv[3]), H = std::atoi(argv[4]), C = std::atoi(argv[5]), L = std::atoi(argv[6]);
  const double sigma_r = std::atof(argv[7]), m = std::atof(argv[8]);
  const int K = std::atoi(argv[9]);
  fllf_storage storage;
  if (!std::strcmp(argv[10], "f32")) storage = FLLF_STORE_F32;
  else if (!std::strcmp(argv[10], "f16")) storage = FLLF_STORE_F16;
  else if (!std::strcmp(argv[10], "bf16")) storage = FLLF_STORE_BF16;
  else {
    std::fprintf(stderr, "c_client: unknown storage %s\n", argv[10]);
    return 2;
  }
  if (W < 1 || H < 1 || C < 1) {
    std::fprintf(stderr, "c_client: bad image size\n");
    return 2;
  }
  const size_t n = (size_t)W * H * C;
  std::vector<float> host(n);
  FILE *f = std::fopen(argv[1], "rb");
  if (!f || std::fread(host.data(), sizeof(float), n, f) != n) {
    std::fprintf(stderr, "c_client: cannot read %zu floats from %s\n", n, argv[1]);
    if (f) std::fclose(f);
    return 2;
  }
  std::fclose(f);

  fllf_ctx *ctx = nullptr;
  fllf_status st = fourier_llf_create(&ctx, 0, storage);
  if (st != FLLF_OK) {
    std::fprintf(stderr, "c_client: fourier_llf_create: status %d: %s\n", (int)st, fourier_llf_last_error(ctx));
    fourier_llf_destroy(ctx);
    return 3;
  }
  float *d_in = nullptr, *d_out = nullptr;
  void *d_ws = nullptr;
  hipStream_t stream = nullptr;
  int rc = 0;
  fllf_job job;
  std::memset(&job, 0, sizeof(job));
  job.width = W;
  job.height = H;
  job.channels = C;
  job.levels = L;
  job.K = K;
  job.sigma_r = sigma_r;
  job.m = m;
  job.range_R = 1.0;
  job.period_T = 0.0;  // fitted by Eq. (12)
  size_t ws_bytes = 0;
  hipError_t e;
  // the job is validated as a whole (pointers included) before the workspace is sized
  if ((e = hipMalloc((void **)&d_in, n * sizeof(float))) != hipSuccess) {
    rc = hip_fail(e, "hipMalloc(in)");
  } else if ((e = hipMalloc((void **)&d_out, n * sizeof(float))) != hipSuccess) {
    rc = hip_fail(e, "hipMalloc(out)");
  } else if (job.in = d_in, job.out = d_out,
             (st = fourier_llf_workspace_size(ctx, &job, 1, &ws_bytes)) != FLLF_OK) {
    std::fprintf(stderr, "c_client: fourier_llf_workspace_size: status %d: %s\n", (int)st, fourier_llf_last_error(ctx));
    rc = 3;
  } else if ((e = hipMalloc(&d_ws, ws_bytes)) != hipSuccess) {
    rc = hip_fail(e, "hipMalloc(workspace)");
  } else if ((e = hipStreamCreate(&stream)) != hipSuccess) {
    rc = hip_fail(e, "hipStreamCreate");
  } else if ((e = hipMemcpy(d_in, host.data(), n * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) {
    rc = hip_fail(e, "hipMemcpy(in)");
  } else {
    if ((st = fourier_llf_run(ctx, &job, 1, d_ws, ws_bytes, stream)) != FLLF_OK) {
      std::fprintf(stderr, "c_client: fourier_llf_run: status %d: %s\n", (int)st, fourier_llf_last_error(ctx));
      rc = 3;
    } else if ((e = hipStreamSynchronize(stream)) != hipSuccess) {
      rc = hip_fail(e, "hipStreamSynchronize");
    } else if ((e = hipMemcpy(host.data(), d_out, n * sizeof(float), hipMemcpyDeviceToHost)) != hipSuccess) {
      rc = hip_fail(e, "hipMemcpy(out)");
    } else {
      FILE *g = std::fopen(argv[2], "wb");
      if (!g || std::fwrite(host.data(), sizeof(float), n, g) != n) {
        std::fprintf(stderr, "c_client: cannot write %s\n", argv[2]);
        rc = 2;
      }
      if (g) std::fclose(g);
    }
  }
  if (stream) (void)hipStreamDestroy(stream);
  if (d_ws) (void)hipFree(d_ws);
  if (d_out) (void)hipFree(d_out);
  if (d_in) (void)hipFree(d_in);
  fourier_llf_destroy(ctx);
  return rc;
}
