// Kernels of the Fourier local Laplacian filter with f16 pyramid storage.
#include "fllf_kernels.h"

namespace fllf {

hipError_t launch_job_f16(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_storage<FLLF_STORE_F16>(P, ws, st, h, tu);
}

hipError_t launch_batch_f16(const BatchSchedule &s, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_batch_storage<FLLF_STORE_F16>(s, ws, st, h, tu);
}

hipError_t launch_reparam_f16(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_reparam_storage<FLLF_STORE_F16>(P, ws, st, h, tu);
}

}  // namespace fllf
