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

// Non-physical nodes of a state [elem][var][node] (plan layout): partial counts per
// workgroup over fixed node ranges, then summed in a fixed order (as doubles: exact for
// counts below 2^53).
template <typename T>
__global__ __launch_bounds__(KR_WG) void k_bad_part(const ElemInfo *__restrict__ el, int E, const T *__restrict__ u,
                                                    double gm1, double *__restrict__ part) {
    __shared__ double sm[KR_WG / 64];
    double cnt = 0.0;
    for (int p = blockIdx.x; p < E; p += KR_BLOCKS) {
        const ElemInfo e = el[p];
        const int ne = e.n[0] * e.n[1] * e.n[2];
        const T *q = u + NV * e.noff;
        for (int t = threadIdx.x; t < ne; t += KR_WG) {
            const double r = (double)q[t], mx = (double)q[ne + t], my = (double)q[2 * ne + t],
                         mz = (double)q[3 * ne + t], en = (double)q[4 * ne + t];
            const double pr = gm1 * (en - 0.5 * (mx * mx + my * my + mz * mz) / r);
            const bool finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(en);
            if (!(finite && r > 0.0 && pr > 0.0)) cnt += 1.0;
        }
    }
    const double s = block_sum(cnt, sm);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
hipError_t launch_count_bad(const ElemInfo *el, int E, const T *u, double gamma, double *part, double *out,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_bad_part<T>, dim3(KR_BLOCKS), dim3(KR_WG), 0, s, el, E, u, gamma - 1.0, part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(KR_WG), 0, s, part, out);
    return hipGetLastError();
}

template hipError_t launch_count_bad<double>(const ElemInfo *, int, const double *, double, double *, double *,
                                             hipStream_t);
template hipError_t launch_count_bad<float>(const ElemInfo *, int, const float *, double, double *, double *,
                                            hipStream_t);

}  // namespace dgt
