// Launchers of the step kernels.  Every (lattice, precision) pair is built in
// an object of its own (step_launch.hip compiled once per pair), so the many
// compile-time variants of the step kernel compile in parallel.  Not part of
// the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace lbm {
namespace host {

// Run-time choice of the step kernel's compile-time variant.
struct StepVariant {
  bool flux;       // also write the per-word x-momentum partials
  bool linear;     // linear (Stokes) equilibrium
  bool off32;      // 32-bit group-relative offsets
  bool periodic;   // six periodic faces and a body force
  bool trt;        // two-relaxation-time collision
};

// One step of one domain: k_step over `grid` blocks on stream st.
template <class Lat, class T>
void launch_step_kernel(const StepArgs<T>& a, int grid, hipStream_t st, StepVariant v);

// One step of a batch: k_step_batch over `grid` blocks with the argument and
// owner tables in device memory.
template <class Lat, class T>
void launch_batch_step_kernel(const StepArgs<T>* args, const int2* owner, int flip, int grid,
                              hipStream_t st, StepVariant v);

#define LBM_STEP_LAUNCH_EXTERN(LAT, T)                                                  \
  extern template void launch_step_kernel<LAT, T>(const StepArgs<T>&, int, hipStream_t, \
                                                  StepVariant);                        \
  extern template void launch_batch_step_kernel<LAT, T>(const StepArgs<T>*, const int2*, \
                                                        int, int, hipStream_t, StepVariant);
LBM_STEP_LAUNCH_EXTERN(D2Q9, float)
LBM_STEP_LAUNCH_EXTERN(D2Q9, double)
LBM_STEP_LAUNCH_EXTERN(D3Q19, float)
LBM_STEP_LAUNCH_EXTERN(D3Q19, double)
#undef LBM_STEP_LAUNCH_EXTERN

}  // namespace host
}  // namespace lbm
