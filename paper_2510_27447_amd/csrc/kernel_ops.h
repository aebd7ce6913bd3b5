// Type-erased launch table of one cell model: the host library dispatches on
// (model, precision, node count) at run time through these entries; each
// model's kernels are instantiated in a translation unit of their own.
#pragma once

#include <hip/hip_runtime.h>

#include "sdc_kernel.h"

namespace ionic {

struct LaunchCommon {
  double S[kMaxNodes - 1][kMaxNodes];
  double dc[kMaxNodes - 1];
  double tol;
  int maxit;
  int n_sims;
  AdaptCtl* ctl;
  ErrSlot* err;
  void* state_alt;
  SimDesc sims[kMaxBatch];
};

using SdcLaunch = hipError_t (*)(int M, const void* params, const LaunchCommon& c, int blocks,
                                 hipStream_t st);

struct ModelOps {
  int n_states;
  int n_fp64;  // leading planes in double under the mixed layout
  int n_params;
  const char* const* param_names;
  const double* param_defaults;  // n_params (+ trailing fixed entries)
  int n_raw;                     // length of the raw parameter vector
  const double* scale;           // n_states: the Newton stop's per-state scale
  const char* const* state_names;
  size_t params_bytes[2];        // sizeof(Params<double>), sizeof(Params<float>)
  void (*derive)(const double* raw, void* p64, void* p32);
  // fused step kernels, [precision policy: double, mixed][predictor: Newton, ROS2, Rush-Larsen]
  SdcLaunch sdc[2][3];
  hipError_t (*pack)(int prec, const double* src, long long ld, void* state, long long stride,
                     long long first, long long count, hipStream_t st);
  hipError_t (*unpack)(int prec, const void* state, long long stride, long long first,
                       long long count, double* dst, long long ld, hipStream_t st);
  hipError_t (*steady)(int prec, const void* params, void* state, long long stride, long long n,
                       hipStream_t st);
  // resting state (computed in double into rest_out, N doubles) broadcast to
  // every vertex of the state in precision `prec`
  hipError_t (*rest)(int prec, const void* params64, double* rest_out, void* state,
                     long long stride, long long n, hipStream_t st);
  hipError_t (*debug_jac)(int prec, const void* params, const void* state, long long stride,
                          long long v, double stim, double diff, double* out, hipStream_t st);
};

// The step kernels of the cell models live in translation units of their own
// (one per model, precision policy and predictor) so they compile in
// parallel.
hipError_t tt06_sdc_fp64_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_fp64_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_newton(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_ros2(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_fp64_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t tt06_sdc_mixed_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_fp64_rl(int, const void*, const LaunchCommon&, int, hipStream_t);
hipError_t lr91_sdc_mixed_rl(int, const void*, const LaunchCommon&, int, hipStream_t);

// Adaptive step control (control.hip).
hipError_t adapt_init(AdaptCtl* c, ErrSlot* err, double t0, double t_end, double dt_init,
                      double dt_max, double tol, double dt_min, double t_on, double t_off,
                      long long max_attempts, hipStream_t st);
hipError_t adapt_control(AdaptCtl* c, ErrSlot* err, double* history, long long history_len,
                         hipStream_t st);

extern const ModelOps kOpsLR91;
extern const ModelOps kOpsTT06;
extern const ModelOps kOpsTestLinear;
extern const ModelOps kOpsTestLogistic;

}  // namespace ionic
