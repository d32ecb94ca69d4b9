// Kernels of the Fourier local Laplacian filter with f32 pyramid storage.
#include "fllf_kernels.h"

namespace fllf {

hipError_t launch_job_f32(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_storage<FLLF_STORE_F32>(P, ws, st, h, tu);
}

hipError_t launch_batch_f32(const BatchSchedule &s, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_batch_storage<FLLF_STORE_F32>(s, ws, st, h, tu);
}

hipError_t launch_reparam_f32(const JobPlan &P, char *ws, hipStream_t st, LaunchHook *h, const Tuning &tu) {
  return launch_reparam_storage<FLLF_STORE_F32>(P, ws, st, h, tu);
}

}  // namespace fllf
