// Step-kernel launchers of one (lattice, precision) pair, chosen at build time
// by LBM_LAT (D2Q9 or D3Q19) and LBM_REAL (float or double): the build
// compiles this file once per pair.
#include "step_launch.h"

#if !defined(LBM_LAT) || !defined(LBM_REAL)
#error "build with -DLBM_LAT=<D2Q9|D3Q19> -DLBM_REAL=<float|double>"
#endif

namespace lbm {
namespace host {
namespace {

// Calls f.run<B...>() with the run-time flags turned into template arguments.
template <bool... Bs, class F>
void with_flags(F& f) {
  f.template run<Bs...>();
}
template <bool... Bs, class F, class... Rest>
void with_flags(F& f, bool b, Rest... rest) {
  if (b) with_flags<Bs..., true>(f, rest...);
  else with_flags<Bs..., false>(f, rest...);
}

template <class Lat, class T>
struct Single {
  const StepArgs<T>& a;
  int grid;
  hipStream_t st;
  template <bool FLUX, bool LIN, bool O32, bool PER, bool TRT>
  void run() {
    k_step<Lat, T, FLUX, LIN, O32, PER, TRT><<<grid, dim3(kWave, kRows), 0, st>>>(a);
  }
};

template <class Lat, class T>
struct Batched {
  const StepArgs<T>* args;
  const int2* owner;
  int flip, grid;
  hipStream_t st;
  template <bool FLUX, bool LIN, bool O32, bool PER, bool TRT>
  void run() {
    k_step_batch<Lat, T, FLUX, LIN, O32, PER, TRT><<<grid, dim3(kWave, kRows), 0, st>>>(
        args, owner, flip);
  }
};

}  // namespace

template <class Lat, class T>
void launch_step_kernel(const StepArgs<T>& a, int grid, hipStream_t st, StepVariant v) {
  Single<Lat, T> f{a, grid, st};
  with_flags(f, v.flux, v.linear, v.off32, v.periodic, v.trt);
}

template <class Lat, class T>
void launch_batch_step_kernel(const StepArgs<T>* args, const int2* owner, int flip, int grid,
                              hipStream_t st, StepVariant v) {
  Batched<Lat, T> f{args, owner, flip, grid, st};
  with_flags(f, v.flux, v.linear, v.off32, v.periodic, v.trt);
}

template void launch_step_kernel<LBM_LAT, LBM_REAL>(const StepArgs<LBM_REAL>&, int, hipStream_t,
                                                    StepVariant);
template void launch_batch_step_kernel<LBM_LAT, LBM_REAL>(const StepArgs<LBM_REAL>*,
                                                          const int2*, int, int, hipStream_t,
                                                          StepVariant);

}  // namespace host
}  // namespace lbm
