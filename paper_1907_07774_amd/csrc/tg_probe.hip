// Streaming reference for the roofline of the PCG passes: five fields read
// and two written in one pass, float4 accesses, grid-stride, no other work.
#include <hip/hip_runtime.h>

#include "tg_internal.h"

namespace tg {
namespace {
typedef float f4v __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream7(const f4v* __restrict__ a,
                                                 const f4v* __restrict__ b,
                                                 const f4v* __restrict__ c, f4v* __restrict__ d,
                                                 f4v* __restrict__ e, long long n) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    const f4v x = a[i], y = b[i], z = c[i], u = d[i], w = e[i];
    d[i] = u + 0.5f * x;
    e[i] = w - 0.25f * (y + z);
  }
}
}  // namespace

hipError_t stream7_launch(const void* a, const void* b, const void* c, void* d, void* e,
                          long long n4, hipStream_t st) {
  k_stream7<<<8192, 256, 0, st>>>((const f4v*)a, (const f4v*)b, (const f4v*)c, (f4v*)d,
                                  (f4v*)e, n4);
  return hipGetLastError();
}

}  // namespace tg
