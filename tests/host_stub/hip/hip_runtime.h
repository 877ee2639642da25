// Stand-in for <hip/hip_runtime.h> on a machine without a GPU (see
// hip_runtime_api.h): the vector types and qualifiers the library's host
// code names, and a symbol marker that tells the stub the extent of a
// file-scope device array.
#pragma once
#include "hip_runtime_api.h"

#define __host__
#define __device__
#define __global__
#define __shared__
#define __align__(n) __attribute__((aligned(n)))

struct float2 { float x, y; };
struct double2 { double x, y; };
struct uint4 { unsigned x, y, z, w; };
struct int4 { int x, y, z, w; };

#ifdef __cplusplus
extern "C" const void* stub_symbol(const void* addr, size_t bytes);
#define HIP_SYMBOL(x) stub_symbol(&(x), sizeof(x))
#endif
