// Small device utilities of libabm.  Buffers are cleared by a fill kernel
// rather than a memset node so that the same launch sequence can be captured
// into a HIP graph and replayed.
#include "abm_dev.h"
#include "abm_kernels.h"

namespace abm {

namespace {
__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* p, uint32_t v, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}
}  // namespace

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace abm
