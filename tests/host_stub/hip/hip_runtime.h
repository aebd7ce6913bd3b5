/* Stand-in for the HIP runtime header: lets the host compiler build the
 * library's host-side planning code and its device-side stencil header as
 * plain C++ in the CPU tests (test_stencil_host.py, test_multigrid_host.py).
 * Qualifiers are defined away; the runtime types are opaque and never used. */
#pragma once
#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
typedef int hipError_t;
typedef struct ihipStream_t* hipStream_t;
