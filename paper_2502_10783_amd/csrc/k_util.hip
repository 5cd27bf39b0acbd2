// Fill kernels (used instead of hipMemsetAsync so that the same sequence
// can be captured into a HIP graph).
#include "ipp_internal.h"
#include "kernels.h"

namespace ipp {

__global__ void k_fill_i32(int32_t* a, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

__global__ void k_fill_i64(int64_t* a, int64_t n, int64_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = v;
}

}  // namespace ipp
