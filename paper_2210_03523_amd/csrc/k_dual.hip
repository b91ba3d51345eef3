// Physical time derivative for the dual time-stepping truncation-error estimate
// (arXiv 2210.03523, Section 2.3, item 2).  The estimate replaces the fine operator
// term of the variational form by the discrete physical time derivative of the
// sampled solution; the sampling is linear and element-local, so forming
// dudt = -(delta_p/delta t) Q on the fine layout and passing it to the tau kernels
// gives (delta_p/delta t)(I Q) + (M^N)^-1 F^N(I Q_0).  delta_p/delta t is the backward
// difference of order k at t_{n+1} over Q(t_{n+1-j}), j = 0..k (standard BDF weights).
#include "common.h"

namespace dgt {

struct BdfStates {
    const double *q[4];
    double w[4];  // weights divided by -dt
};

__global__ __launch_bounds__(256) void k_bdf_rate(BdfStates st, int nst, int64_t n, double *__restrict__ dudt) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = st.w[0] * st.q[0][i];
    for (int j = 1; j < nst; ++j) acc += st.w[j] * st.q[j][i];
    dudt[i] = acc;
}

hipError_t launch_bdf_rate(const double *const *states, int nst, double dt, int64_t n, double *dudt, hipStream_t s) {
    static const double B[3][4] = {{1.0, -1.0, 0.0, 0.0},
                                   {1.5, -2.0, 0.5, 0.0},
                                   {11.0 / 6.0, -3.0, 1.5, -1.0 / 3.0}};
    if (nst < 2 || nst > 4) return hipErrorInvalidValue;
    if (n == 0) return hipSuccess;
    BdfStates st{};
    for (int j = 0; j < nst; ++j) {
        st.q[j] = states[j];
        st.w[j] = -B[nst - 2][j] / dt;
    }
    hipLaunchKernelGGL(k_bdf_rate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, st, nst, n, dudt);
    return hipGetLastError();
}

}  // namespace dgt
