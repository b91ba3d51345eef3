// Vector kernels of the adjoint solve (restarted GMRES on (dr/dQ)^T psi = dJ/dQ; the
// matrix-vector product is the residual VJP).  Inner products are deterministic: a
// fixed grid of KR_BLOCKS workgroups reduces fixed index ranges, then one workgroup
// per result sums the partials in a fixed order.  The Gram-Schmidt step of the Arnoldi
// process works on many Krylov vectors per pass: the inner products with up to KR_MD
// of them (and the vector's own norm) read w once, and the update w -= sum h_k x_k
// reads every x_k and w once and returns the new norm.
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
// beta = 0 overwrites y without reading it (y may hold anything, NaN bit patterns of
// uninitialised memory included)
__global__ __launch_bounds__(KR_WG) void k_axpby(double alpha, const double *x, double beta, double *y, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)KR_WG + threadIdx.x;
    if (i < n) y[i] = beta == 0.0 ? alpha * x[i] : alpha * x[i] + beta * y[i];
}

// Block reduction of KR_MD + 1 values at once: wave shuffles, one LDS row per wave,
// then thread k sums row k over the waves (fixed order); returns that sum on threads
// k < KR_MD + 1.
constexpr int KR_MD = 8;  // vectors per pass of the multi-vector inner product
__device__ __forceinline__ double block_sum_many(double (&acc)[KR_MD + 1], double (*sm)[KR_MD + 1]) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k <= KR_MD; ++k) {
        double v = acc[k];
        for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
        if (lane == 0) sm[w][k] = v;
    }
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x <= KR_MD)
        for (int i = 0; i < KR_WG / 64; ++i) s += sm[i][threadIdx.x];
    return s;
}

// Partials of x_k . w for the c <= KR_MD vectors x_k = X + k ld, and of w . w when
// self: part[k * KR_BLOCKS + block] (k = c for w . w), fixed index ranges per block.
__global__ __launch_bounds__(KR_WG) void k_mdot_part(const double *__restrict__ X, int64_t ld, int c,
                                                     const double *__restrict__ w, int self, int64_t n,
                                                     double *__restrict__ part) {
    __shared__ double sm[KR_WG / 64][KR_MD + 1];
    double acc[KR_MD + 1];
#pragma unroll
    for (int k = 0; k <= KR_MD; ++k) acc[k] = 0.0;
    // two indices per iteration: twice the loads in flight
    constexpr int64_t STEP = (int64_t)KR_BLOCKS * KR_WG;
    int64_t i = blockIdx.x * (int64_t)KR_WG + threadIdx.x;
    for (; i + STEP < n; i += 2 * STEP) {
        const double w0 = w[i], w1 = w[i + STEP];
#pragma unroll
        for (int k = 0; k < KR_MD; ++k)
            if (k < c) acc[k] += X[k * ld + i] * w0 + X[k * ld + i + STEP] * w1;
        acc[KR_MD] += w0 * w0 + w1 * w1;
    }
    if (i < n) {
        const double w0 = w[i];
#pragma unroll
        for (int k = 0; k < KR_MD; ++k)
            if (k < c) acc[k] += X[k * ld + i] * w0;
        acc[KR_MD] += w0 * w0;
    }
    const double s = block_sum_many(acc, sm);
    const int k = threadIdx.x;
    if (k < c) part[(int64_t)k * KR_BLOCKS + blockIdx.x] = s;
    if (k == KR_MD && self) part[(int64_t)c * KR_BLOCKS + blockIdx.x] = s;
}

// out[b] = the fixed-order sum of partial row b (one workgroup per row).
__global__ __launch_bounds__(KR_WG) void k_rows_final(const double *__restrict__ part, double *__restrict__ out) {
    __shared__ double sm[KR_WG / 64];
    const double *row = part + (int64_t)blockIdx.x * KR_BLOCKS;
    double v = 0.0;
    for (int i = threadIdx.x; i < KR_BLOCKS; i += KR_WG) v += row[i];
    const double s = block_sum(v, sm);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// w <- w - sum_{k < c} h_k x_k, x_k = X + k ld (h on the device), and the partials of the
// new w . w in part[0 .. KR_BLOCKS) when part is given.
__global__ __launch_bounds__(KR_WG) void k_maxpy(const double *__restrict__ X, int64_t ld, int c,
                                                 const double *__restrict__ h, double *__restrict__ w, int64_t n,
                                                 double *__restrict__ part) {
    __shared__ double sh[DG_KRYLOV_MAX];
    __shared__ double sm[KR_WG / 64];
    for (int k = threadIdx.x; k < c; k += KR_WG) sh[k] = h[k];
    __syncthreads();
    double nn = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)KR_WG + threadIdx.x; i < n; i += (int64_t)KR_BLOCKS * KR_WG) {
        double v = w[i];
        for (int k = 0; k < c; ++k) v -= sh[k] * X[k * ld + i];
        w[i] = v;
        nn += v * v;
    }
    if (part) {
        const double s = block_sum(nn, sm);
        if (threadIdx.x == 0) part[blockIdx.x] = s;
    }
}

hipError_t launch_mdot(const double *X, int64_t ld, int c, const double *w, bool self, int64_t n, double *part,
                       double *out, hipStream_t s) {
    // passes of KR_MD vectors; the last one also forms w . w (out[c]) when self
    for (int k0 = 0; k0 < c || (self && k0 == c); k0 += KR_MD) {
        const int ck = c - k0 < KR_MD ? c - k0 : KR_MD;
        const bool last = k0 + KR_MD >= c;
        const int sf = self && last ? 1 : 0;
        hipLaunchKernelGGL(k_mdot_part, dim3(KR_BLOCKS), dim3(KR_WG), 0, s, X + k0 * ld, ld, ck, w, sf, n, part);
        hipLaunchKernelGGL(k_rows_final, dim3(ck + sf), dim3(KR_WG), 0, s, part, out + k0);
        if (last) break;
    }
    return hipGetLastError();
}

hipError_t launch_maxpy(const double *X, int64_t ld, int c, const double *h, double *w, int64_t n, double *part,
                        double *nrm2, hipStream_t s) {
    if (c > DG_KRYLOV_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_maxpy, dim3(KR_BLOCKS), dim3(KR_WG), 0, s, X, ld, c, h, w, n, nrm2 ? part : nullptr);
    if (nrm2) hipLaunchKernelGGL(k_rows_final, dim3(1), dim3(KR_WG), 0, s, part, nrm2);
    return hipGetLastError();
}

int mdot_partials() { return (KR_MD + 1) * KR_BLOCKS; }

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
