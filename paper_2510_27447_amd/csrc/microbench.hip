// Rate microbenchmarks of the MI355X units the reaction + SDC kernels are
// bound by: fp64 and fp32 fused multiply-add, the hardware transcendental
// v_exp_f32 (raw and as the __expf the fp32 models call), the device math
// library's double exp() (a software sequence: gfx950 has no fp64 exp
// instruction) and a streaming copy through HBM.  Measurement support for
// the roofline of the step kernels; built into its own library
// (libionic_microbench.so), not part of the reaction library's C ABI.
//
//   int ionic_mb_run(int which, int64_t n_threads, int iters, double* seconds,
//                    double* ops, void* buffer, size_t buffer_bytes)
//     which: 0 fp64 FMA, 1 fp32 FMA, 2 v_exp_f32, 3 __expf, 4 fp64 exp(),
//            5 copy (buffer: 2 x n_threads doubles, read half, write half);
//     runs the kernel once untimed and once between two HIP events on a
//     stream of its own; *seconds = the timed launch, *ops = the operations
//     it performed (flops for FMA, one per transcendental call, bytes moved
//     for the copy).  Returns 0 or the hipError_t.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;   // independent dependency chains per lane
constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) fma64_kernel(double* out, int iters, double a, double b) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double x[kChains];
  for (int k = 0; k < kChains; ++k) x[k] = 1e-3 * double(threadIdx.x + k);
  for (int i = 0; i < iters; ++i)
    for (int k = 0; k < kChains; ++k) x[k] = fma(x[k], a, b);
  double s = 0.0;
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5) out[t] = s;  // keeps the chains live without a store per lane
}

__global__ void __launch_bounds__(kBlock) fma32_kernel(float* out, int iters, float a, float b) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float x[kChains];
  for (int k = 0; k < kChains; ++k) x[k] = 1e-3f * float(threadIdx.x + k);
  for (int i = 0; i < iters; ++i)
    for (int k = 0; k < kChains; ++k) x[k] = __builtin_fmaf(x[k], a, b);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5f) out[t] = s;
}

// x <- 2^(-x) converges to a fixed point in (0, 1): every call stays finite
__global__ void __launch_bounds__(kBlock) exp2raw_kernel(float* out, int iters) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float x[kChains];
  for (int k = 0; k < kChains; ++k) x[k] = 0.01f * float(k + 1);
  for (int i = 0; i < iters; ++i)
    for (int k = 0; k < kChains; ++k) x[k] = __builtin_amdgcn_exp2f(-x[k]);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5f) out[t] = s;
}

__global__ void __launch_bounds__(kBlock) expf_kernel(float* out, int iters) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  float x[kChains];
  for (int k = 0; k < kChains; ++k) x[k] = 0.01f * float(k + 1);
  for (int i = 0; i < iters; ++i)
    for (int k = 0; k < kChains; ++k) x[k] = __expf(-x[k]);
  float s = 0.0f;
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5f) out[t] = s;
}

__global__ void __launch_bounds__(kBlock) exp64_kernel(double* out, int iters) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double x[kChains];
  for (int k = 0; k < kChains; ++k) x[k] = 0.01 * double(k + 1);
  for (int i = 0; i < iters; ++i)
    for (int k = 0; k < kChains; ++k) x[k] = exp(-x[k]);
  double s = 0.0;
  for (int k = 0; k < kChains; ++k) s += x[k];
  if (s == 1234.5) out[t] = s;
}

// dst[i] = src[i] over n doubles, 16 bytes per lane and iteration
__global__ void __launch_bounds__(kBlock) copy_kernel(const double2* __restrict__ src,
                                                      double2* __restrict__ dst, int64_t n2) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n2; i += stride)
    dst[i] = src[i];
}

}  // namespace

extern "C" int ionic_mb_run(int which, int64_t n_threads, int iters, double* seconds, double* ops,
                            void* buffer, size_t buffer_bytes) {
  if (!seconds || !ops || !buffer || n_threads < kBlock || iters < 1 || which < 0 || which > 5)
    return int(hipErrorInvalidValue);
  const int64_t blocks64 = n_threads / kBlock;
  if (blocks64 > (int64_t(1) << 30)) return int(hipErrorInvalidValue);
  const int blocks = int(blocks64);
  const int64_t threads = blocks64 * kBlock;
  if (which == 5) {
    if (buffer_bytes < size_t(threads) * 2 * sizeof(double) || threads % 2) return int(hipErrorInvalidValue);
  } else if (buffer_bytes < size_t(threads) * sizeof(double)) {
    return int(hipErrorInvalidValue);
  }
  hipStream_t st;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return int(e);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  auto launch = [&]() {
    switch (which) {
      case 0: hipLaunchKernelGGL(fma64_kernel, dim3(blocks), dim3(kBlock), 0, st, (double*)buffer, iters, 0.999999, 1e-7); break;
      case 1: hipLaunchKernelGGL(fma32_kernel, dim3(blocks), dim3(kBlock), 0, st, (float*)buffer, iters, 0.9999f, 1e-4f); break;
      case 2: hipLaunchKernelGGL(exp2raw_kernel, dim3(blocks), dim3(kBlock), 0, st, (float*)buffer, iters); break;
      case 3: hipLaunchKernelGGL(expf_kernel, dim3(blocks), dim3(kBlock), 0, st, (float*)buffer, iters); break;
      case 4: hipLaunchKernelGGL(exp64_kernel, dim3(blocks), dim3(kBlock), 0, st, (double*)buffer, iters); break;
      default: {
        double* b = static_cast<double*>(buffer);
        const int64_t n2 = threads / 2;  // double2 elements per half
        const int cblocks = 256 * 16;
        hipLaunchKernelGGL(copy_kernel, dim3(cblocks), dim3(kBlock), 0, st,
                           reinterpret_cast<const double2*>(b), reinterpret_cast<double2*>(b + threads), n2);
      }
    }
  };
  launch();
  e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(st);
  if (e != hipSuccess) return int(e);
  *seconds = double(ms) * 1e-3;
  const double per = double(threads) * double(iters) * kChains;
  switch (which) {
    case 0: case 1: *ops = 2.0 * per; break;            // one FMA = 2 flops
    case 2: case 3: case 4: *ops = per; break;           // one exponential per call
    default: *ops = 2.0 * double(threads) * sizeof(double); break;  // bytes read + written
  }
  return 0;
}
