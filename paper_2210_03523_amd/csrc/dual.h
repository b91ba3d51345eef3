// Forward-mode dual numbers with K derivative components, used to form the local
// Jacobians (flux along an axis, Riemann flux at a face node) that the adjoint
// (vector-Jacobian product) kernels transpose.  Only the operations the Euler
// flux functions use are provided.
#pragma once

#include <hip/hip_runtime.h>

namespace dgt {

// keep the double overloads visible next to the dual ones
using ::fabs;
using ::fmax;
using ::sqrt;

template <int K>
struct Dual {
    double v;
    double d[K];
    __device__ __forceinline__ Dual() {}
    __device__ __forceinline__ Dual(double x) : v(x) {
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] = 0.0;
    }
    __device__ __forceinline__ Dual &operator+=(const Dual &b) {
        v += b.v;
#pragma unroll
        for (int k = 0; k < K; ++k) d[k] += b.d[k];
        return *this;
    }
};

template <int K>
__device__ __forceinline__ Dual<K> operator+(const Dual<K> &a, const Dual<K> &b) {
    Dual<K> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K> &a, const Dual<K> &b) {
    Dual<K> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator-(const Dual<K> &a) {
    Dual<K> r;
    r.v = -a.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator*(const Dual<K> &a, const Dual<K> &b) {
    Dual<K> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> operator/(const Dual<K> &a, const Dual<K> &b) {
    Dual<K> r;
    const double ib = 1.0 / b.v;
    r.v = a.v * ib;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> sqrt(const Dual<K> &a) {
    Dual<K> r;
    r.v = ::sqrt(a.v);
    const double h = 0.5 / r.v;
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * h;
    return r;
}
// |a| with the derivative of its sign (0 at a = 0).
template <int K>
__device__ __forceinline__ Dual<K> fabs(const Dual<K> &a) {
    const double s = a.v > 0.0 ? 1.0 : (a.v < 0.0 ? -1.0 : 0.0);
    Dual<K> r;
    r.v = ::fabs(a.v);
#pragma unroll
    for (int k = 0; k < K; ++k) r.d[k] = s * a.d[k];
    return r;
}
template <int K>
__device__ __forceinline__ Dual<K> fmax(const Dual<K> &a, const Dual<K> &b) {
    return a.v >= b.v ? a : b;
}

}  // namespace dgt
