// Kernels of the Fourier local Laplacian filter with bf16 pyramid storage.
#include "fllf_kernels.h"

namespace fllf {

hipError_t launch_job_bf16(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h) {
  return launch_storage<FLLF_STORE_BF16>(P, ws, st, h);
}

}  // namespace fllf
