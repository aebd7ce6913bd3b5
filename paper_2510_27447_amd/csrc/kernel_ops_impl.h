// Instantiation helpers behind ModelOps (included by one .hip file per model).
#pragma once

#include "kernel_ops.h"

namespace ionic {

template <class Model>
struct OpsImpl {
  static constexpr int kAuxBlock = 256;

  static void derive(const double* raw, void* p64, void* p32) {
    *static_cast<typename Model::template Params<double>*>(p64) = Model::template derive<double>(raw);
    *static_cast<typename Model::template Params<float>*>(p32) = Model::template derive<float>(raw);
  }

  template <class Prec, int Pred, int M>
  static hipError_t launch_m(const void* params, const LaunchCommon& c, int blocks, hipStream_t st) {
    using P = typename Model::template Params<typename Prec::TE>;
    LaunchArgs<P> a;
    a.params = *static_cast<const P*>(params);
    for (int m = 0; m < kMaxNodes - 1; ++m) {
      a.dc[m] = c.dc[m];
      for (int j = 0; j < kMaxNodes; ++j) a.S[m][j] = c.S[m][j];
    }
    a.tol = c.tol;
    a.maxit = c.maxit;
    a.n_sims = c.n_sims;
    a.ctl = c.ctl;
    a.err = c.err;
    a.state_alt = c.state_alt;
    for (int s = 0; s < kMaxBatch; ++s) a.sims[s] = c.sims[s];
    static_assert(sizeof(LaunchArgs<P>) <= 3800, "kernel arguments must fit the kernarg segment");
    // the two-wavefront build only when the launch gives every SIMD two
    // wavefronts (256 compute units x 4 SIMDs x 2)
    constexpr int kTwoWaveBlocks = 2048;
    if constexpr (StepPolicy<Model, Prec, M, Pred>::waves == 2) {
      if (blocks >= kTwoWaveBlocks) {
        hipLaunchKernelGGL((sdc_kernel<Model, Prec, M, Pred, 2>), dim3(blocks), dim3(kBlock), 0, st,
                           a);
        return hipGetLastError();
      }
    }
    hipLaunchKernelGGL((sdc_kernel<Model, Prec, M, Pred, 1>), dim3(blocks), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  }

  // node count dispatch of one (precision policy, predictor) pair
  template <class Prec, int Pred>
  static hipError_t sdc(int M, const void* params, const LaunchCommon& c, int blocks,
                        hipStream_t st) {
    switch (M) {
      case 2: return launch_m<Prec, Pred, 2>(params, c, blocks, st);
      case 3: return launch_m<Prec, Pred, 3>(params, c, blocks, st);
      case 4: return launch_m<Prec, Pred, 4>(params, c, blocks, st);
      case 5: return launch_m<Prec, Pred, 5>(params, c, blocks, st);
      default: return hipErrorInvalidValue;
    }
  }

  static int grid(long long count) { return int((count + kAuxBlock - 1) / kAuxBlock); }

  static hipError_t pack(int prec, const double* src, long long ld, void* state, long long stride,
                         long long first, long long count, hipStream_t st) {
    if (prec == 0)
      hipLaunchKernelGGL((pack_kernel<Model, Fp64>), dim3(grid(count)), dim3(kAuxBlock), 0, st, src,
                         ld, state, stride, first, count);
    else
      hipLaunchKernelGGL((pack_kernel<Model, Mixed>), dim3(grid(count)), dim3(kAuxBlock), 0, st,
                         src, ld, state, stride, first, count);
    return hipGetLastError();
  }
  static hipError_t unpack(int prec, const void* state, long long stride, long long first,
                           long long count, double* dst, long long ld, hipStream_t st) {
    if (prec == 0)
      hipLaunchKernelGGL((unpack_kernel<Model, Fp64>), dim3(grid(count)), dim3(kAuxBlock), 0, st,
                         state, stride, first, count, dst, ld);
    else
      hipLaunchKernelGGL((unpack_kernel<Model, Mixed>), dim3(grid(count)), dim3(kAuxBlock), 0, st,
                         state, stride, first, count, dst, ld);
    return hipGetLastError();
  }
  static hipError_t steady(int prec, const void* params, void* state, long long stride,
                           long long n, hipStream_t st) {
    if (prec == 0)
      hipLaunchKernelGGL((steady_gates_kernel<Model, Fp64>), dim3(grid(n)), dim3(kAuxBlock), 0, st,
                         *static_cast<const typename Model::template Params<double>*>(params), state,
                         stride, n);
    else
      hipLaunchKernelGGL((steady_gates_kernel<Model, Mixed>), dim3(grid(n)), dim3(kAuxBlock), 0, st,
                         *static_cast<const typename Model::template Params<float>*>(params), state,
                         stride, n);
    return hipGetLastError();
  }
  static hipError_t rest(int prec, const void* params64, double* rest_out, void* state,
                         long long stride, long long n, hipStream_t st) {
    hipLaunchKernelGGL((rest_state_kernel<Model>), dim3(1), dim3(64), 0, st,
                       *static_cast<const typename Model::template Params<double>*>(params64),
                       rest_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (prec == 0)
      hipLaunchKernelGGL((broadcast_kernel<Model, Fp64>), dim3(grid(n)), dim3(kAuxBlock), 0, st,
                         rest_out, state, stride, n);
    else
      hipLaunchKernelGGL((broadcast_kernel<Model, Mixed>), dim3(grid(n)), dim3(kAuxBlock), 0, st,
                         rest_out, state, stride, n);
    return hipGetLastError();
  }
  static hipError_t debug_jac(int prec, const void* params, const void* state, long long stride,
                              long long v, double stim, double diff, double* out, hipStream_t st) {
    if (prec == 0)
      hipLaunchKernelGGL((debug_jacobian_kernel<Model, Fp64>), dim3(1), dim3(64), 0, st,
                         *static_cast<const typename Model::template Params<double>*>(params), state,
                         stride, v, stim, diff, out);
    else
      hipLaunchKernelGGL((debug_jacobian_kernel<Model, Mixed>), dim3(1), dim3(64), 0, st,
                         *static_cast<const typename Model::template Params<float>*>(params), state,
                         stride, v, stim, diff, out);
    return hipGetLastError();
  }

  static constexpr int n_raw() {
    return int(sizeof(Model::PARAM_DEFAULTS) / sizeof(double));
  }

  // with_step = false leaves the step kernels unset (the caller installs
  // launchers from other translation units), so none is instantiated here
  template <bool with_step = true>
  static ModelOps make(const char* const* state_names) {
    ModelOps o{};
    o.n_states = Model::N;
    o.n_fp64 = Model::N64;
    o.n_params = Model::N_PARAMS;
    o.param_names = Model::PARAM_NAMES;
    o.param_defaults = Model::PARAM_DEFAULTS;
    o.n_raw = n_raw();
    o.scale = Model::SCALE;
    o.state_names = state_names;
    o.params_bytes[0] = sizeof(typename Model::template Params<double>);
    o.params_bytes[1] = sizeof(typename Model::template Params<float>);
    o.derive = &derive;
    if constexpr (with_step) {
      o.sdc[0][kPredNewton] = &sdc<Fp64, kPredNewton>;
      o.sdc[0][kPredRos2] = &sdc<Fp64, kPredRos2>;
      o.sdc[1][kPredNewton] = &sdc<Mixed, kPredNewton>;
      o.sdc[1][kPredRos2] = &sdc<Mixed, kPredRos2>;
      o.sdc[0][kPredRushLarsen] = &sdc<Fp64, kPredRushLarsen>;
      o.sdc[1][kPredRushLarsen] = &sdc<Mixed, kPredRushLarsen>;
    }
    o.pack = &pack;
    o.unpack = &unpack;
    o.steady = &steady;
    o.rest = &rest;
    o.debug_jac = &debug_jac;
    return o;
  }
};

}  // namespace ionic
