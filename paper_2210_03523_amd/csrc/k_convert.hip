// Promotion of an FP32 state to FP64 before the truncation-error estimate: the time
// stepping may run in single precision, but the estimate is a difference of two
// residuals of nearly equal size and is formed in double precision (Section 2.3).
// Float to double is exact, so the promoted state is the stepped state itself.
#include <algorithm>

#include "common.h"

namespace dgt {

// Four values per lane: one 16-byte load, two 16-byte stores.
__global__ __launch_bounds__(256) void k_promote(const float *__restrict__ in, double *__restrict__ out,
                                                 int64_t n4) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
        const float4 v = reinterpret_cast<const float4 *>(in)[i];
        reinterpret_cast<double2 *>(out)[2 * i] = make_double2(v.x, v.y);
        reinterpret_cast<double2 *>(out)[2 * i + 1] = make_double2(v.z, v.w);
    }
}

__global__ void k_promote_tail(const float *__restrict__ in, double *__restrict__ out, int64_t first, int64_t n) {
    const int64_t i = first + threadIdx.x;
    if (i < n) out[i] = in[i];
}

hipError_t launch_promote(const float *in, double *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t n4 = n / 4;
    if (n4 > 0) {
        const int64_t blocks = std::min<int64_t>((n4 + 255) / 256, 8192);
        hipLaunchKernelGGL(k_promote, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n4);
    }
    if (n > 4 * n4) hipLaunchKernelGGL(k_promote_tail, dim3(1), dim3(4), 0, s, in, out, 4 * n4, n);
    return hipGetLastError();
}

}  // namespace dgt
