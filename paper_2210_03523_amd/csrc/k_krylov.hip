// Vector kernels of the adjoint solve (restarted GMRES on (dr/dQ)^T psi = dJ/dQ; the
// matrix-vector product is the residual VJP).  The inner product is deterministic: a
// fixed grid of KR_BLOCKS workgroups reduces fixed index ranges, then one workgroup
// sums the partials in a fixed order.
#include "common.h"

namespace dgt {

constexpr int KR_WG = 256;
constexpr int KR_BLOCKS = 1024;

__device__ __forceinline__ double block_sum(double v, double *sm) {
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) sm[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < KR_WG / 64; ++i) s += sm[i];
    return s;
}

__global__ __launch_bounds__(KR_WG) void k_dot_part(const double *__restrict__ a, const double *__restrict__ b,
                                                    int64_t n, double *__restrict__ part) {
    __shared__ double sm[KR_WG / 64];
    double v = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)KR_WG + threadIdx.x; i < n; i += (int64_t)KR_BLOCKS * KR_WG)
        v += a[i] * b[i];
    const double s = block_sum(v, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(KR_WG) void k_dot_final(const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double sm[KR_WG / 64];
    double v = 0.0;
    for (int i = threadIdx.x; i < KR_BLOCKS; i += KR_WG) v += part[i];
    const double s = block_sum(v, sm);
    if (threadIdx.x == 0) *out = s;
}

// y <- alpha x + beta y (x may be y)
__global__ __launch_bounds__(KR_WG) void k_axpby(double alpha, const double *x, double beta, double *y, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)KR_WG + threadIdx.x;
    if (i < n) y[i] = alpha * x[i] + beta * y[i];
}

hipError_t launch_dot(const double *a, const double *b, int64_t n, double *part, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_part, dim3(KR_BLOCKS), dim3(KR_WG), 0, s, a, b, n, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(KR_WG), 0, s, part, out);
    return hipGetLastError();
}

hipError_t launch_axpby(double alpha, const double *x, double beta, double *y, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + KR_WG - 1) / KR_WG)), dim3(KR_WG), 0, s, alpha, x, beta, y, n);
    return hipGetLastError();
}

int dot_partials() { return KR_BLOCKS; }

}  // namespace dgt
