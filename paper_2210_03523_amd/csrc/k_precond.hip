// Element-block Jacobi preconditioner of the adjoint operator A = (dr/du)^T for the
// GMRES adjoint solve.  The diagonal block A_ee of every element is assembled column by
// column from probing products: with v = 1 at local unknown j of every element of one
// colour (no two elements of a colour share a face), (A v) restricted to an element e of
// that colour is column j of A_ee, since the only other unknowns that the residual of e
// couples to belong to its face neighbours, which carry zeros.  The blocks (FP32,
// column-major, nd x nd, nd = 5 x nodes) are factored and inverted in place; applying
// the preconditioner is then one matrix-vector product per element.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"

namespace dgt {

// v[unknown j of element e] = val for the listed plan elements
__global__ void k_probe_set(double *__restrict__ v, const int32_t *__restrict__ elems, int nel,
                            const ElemInfo *__restrict__ el, int j, double val) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nel) return;
    v[(int64_t)NV * el[elems[i]].noff + j] = val;
}

// column j of the block of every listed element, from the product out (plan layout)
__global__ __launch_bounds__(256) void k_probe_gather(const double *__restrict__ out, float *__restrict__ blocks,
                                                      const int32_t *__restrict__ elems, const ElemInfo *__restrict__ el,
                                                      int j, int nd) {
    const int e = elems[blockIdx.x];
    const double *src = out + (int64_t)NV * el[e].noff;
    float *dst = blocks + ((int64_t)e * nd + j) * nd;
    for (int i = threadIdx.x; i < nd; i += 256) dst[i] = (float)src[i];
}

// z_e = B_e x_e per element (B_e the stored inverse, column-major); x staged in LDS, the
// columns read coalesced.  Blocks whose size nd is a multiple of 4 (16-byte aligned
// columns): a lane owns 4 consecutive rows, reads them as one 16-byte load per column and
// keeps 4 columns' loads in flight; the workgroup has a lane per row quad (nd / 4 rounded
// up to whole waves, at most 1024).  Otherwise 256 lanes of one row each per pass.
__global__ __launch_bounds__(1024) void k_bj_apply(const float *__restrict__ blocks, const double *__restrict__ x,
                                                  const double *__restrict__ t, double *__restrict__ z,
                                                  const ElemInfo *__restrict__ el, const int32_t *__restrict__ elems,
                                                  int nd) {
    extern __shared__ double sx[];
    const int e = elems ? elems[blockIdx.x] : blockIdx.x;
    const int64_t base = (int64_t)NV * el[e].noff;
    for (int i = threadIdx.x; i < nd; i += blockDim.x) sx[i] = t ? x[base + i] - t[base + i] : x[base + i];
    __syncthreads();
    const float *B = blocks + (int64_t)e * nd * nd;
    if ((nd & 3) == 0) {
        const int nq = nd >> 2;  // row quads
        for (int q = threadIdx.x; q < nq; q += blockDim.x) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            const float4 *col = (const float4 *)B + q;
#pragma unroll 4
            for (int j = 0; j < nd; ++j) {
                const float4 b = col[(int64_t)j * nq];
                const double xj = sx[j];
                a0 += (double)b.x * xj;
                a1 += (double)b.y * xj;
                a2 += (double)b.z * xj;
                a3 += (double)b.w * xj;
            }
            double *zz = z + base + 4 * q;
            zz[0] = a0;
            zz[1] = a1;
            zz[2] = a2;
            zz[3] = a3;
        }
        return;
    }
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < nd; ++j) acc += (double)B[(int64_t)j * nd + i] * sx[j];
        z[base + i] = acc;
    }
}

// Compact storage: column j of block e as FP16 values of B_ij / s_ej with the column scale
// s_ej = max_i |B_ij| in FP32 (1 for a zero column), so every stored value lies in [-1, 1].
// One workgroup per (block, 64 columns); a wave per column at a time.
__global__ __launch_bounds__(256) void k_bj_compact(const float *__restrict__ blocks, __half *__restrict__ hblocks,
                                                    float *__restrict__ scales, int nd) {
    const int e = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int j = blockIdx.x * 64 + wave; j < nd && j < (int)(blockIdx.x + 1) * 64; j += 4) {
        const float *col = blocks + ((int64_t)e * nd + j) * nd;
        float m = 0.f;
        for (int i = lane; i < nd; i += 64) m = fmaxf(m, fabsf(col[i]));
        for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
        const float sc = m > 0.f ? m : 1.f;
        __half *hc = hblocks + ((int64_t)e * nd + j) * nd;
        for (int i = lane; i < nd; i += 64) hc[i] = __float2half_rn(col[i] / sc);
        if (lane == 0) scales[(int64_t)e * nd + j] = sc;
    }
}

// z_e = B_e x_e from the compact storage: x_j s_ej staged in LDS, then as k_bj_apply
// (a lane per row quad, 8-byte loads of four FP16 values; one row per lane otherwise).
__global__ __launch_bounds__(1024) void k_bj_apply16(const __half *__restrict__ hblocks,
                                                     const float *__restrict__ scales, const double *__restrict__ x,
                                                     const double *__restrict__ t, double *__restrict__ z,
                                                     const ElemInfo *__restrict__ el,
                                                     const int32_t *__restrict__ elems, int nd) {
    extern __shared__ double sx[];
    const int e = elems ? elems[blockIdx.x] : blockIdx.x;
    const int64_t base = (int64_t)NV * el[e].noff;
    for (int i = threadIdx.x; i < nd; i += blockDim.x)
        sx[i] = (t ? x[base + i] - t[base + i] : x[base + i]) * (double)scales[(int64_t)e * nd + i];
    __syncthreads();
    const __half *B = hblocks + (int64_t)e * nd * nd;
    if ((nd & 3) == 0) {
        const int nq = nd >> 2;
        for (int q = threadIdx.x; q < nq; q += blockDim.x) {
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            const uint2 *col = (const uint2 *)B + q;
#pragma unroll 4
            for (int j = 0; j < nd; ++j) {
                const uint2 w = col[(int64_t)j * nq];
                const double xj = sx[j];
                const __half2 h01 = *(const __half2 *)&w.x, h23 = *(const __half2 *)&w.y;
                const float2 f01 = __half22float2(h01), f23 = __half22float2(h23);
                a0 += (double)f01.x * xj;
                a1 += (double)f01.y * xj;
                a2 += (double)f23.x * xj;
                a3 += (double)f23.y * xj;
            }
            double *zz = z + base + 4 * q;
            zz[0] = a0;
            zz[1] = a1;
            zz[2] = a2;
            zz[3] = a3;
        }
        return;
    }
    for (int i = threadIdx.x; i < nd; i += blockDim.x) {
        double acc = 0.0;
        for (int j = 0; j < nd; ++j) acc += (double)__half2float(B[(int64_t)j * nd + i]) * sx[j];
        z[base + i] = acc;
    }
}

hipError_t launch_bj_compact(const float *blocks, void *hblocks, float *scales, int E, int nd, hipStream_t s) {
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bj_compact, dim3((nd + 63) / 64, E), dim3(256), 0, s, blocks, (__half *)hblocks, scales, nd);
    return hipGetLastError();
}

hipError_t launch_bj_apply16(const void *hblocks, const float *scales, const double *x, double *z,
                             const ElemInfo *el, int E, int nd, hipStream_t s, const int32_t *elems,
                             const double *t) {
    if (E == 0) return hipSuccess;
    const int threads = (nd & 3) == 0 ? std::min(1024, (nd / 4 + 63) / 64 * 64) : 256;
    hipLaunchKernelGGL(k_bj_apply16, dim3(E), dim3(threads), sizeof(double) * nd, s, (const __half *)hblocks, scales,
                       x, t, z, el, elems, nd);
    return hipGetLastError();
}

hipError_t launch_probe_set(double *v, const int32_t *elems, int nel, const ElemInfo *el, int j, double val,
                            hipStream_t s) {
    if (nel == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_set, dim3((nel + 255) / 256), dim3(256), 0, s, v, elems, nel, el, j, val);
    return hipGetLastError();
}

hipError_t launch_probe_gather(const double *out, float *blocks, const int32_t *elems, int nel, const ElemInfo *el,
                               int j, int nd, hipStream_t s) {
    if (nel == 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_gather, dim3(nel), dim3(256), 0, s, out, blocks, elems, el, j, nd);
    return hipGetLastError();
}

hipError_t launch_bj_apply(const float *blocks, const double *x, double *z, const ElemInfo *el, int E, int nd,
                           hipStream_t s, const int32_t *elems, const double *t) {
    if (E == 0) return hipSuccess;
    const int threads = (nd & 3) == 0 ? std::min(1024, (nd / 4 + 63) / 64 * 64) : 256;
    hipLaunchKernelGGL(k_bj_apply, dim3(E), dim3(threads), sizeof(double) * nd, s, blocks, x, t, z, el, elems, nd);
    return hipGetLastError();
}

}  // namespace dgt
