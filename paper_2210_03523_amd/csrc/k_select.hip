// Polynomial-degree selection from truncation-error maps and the degree-jump conditions
// between face neighbours (arXiv 2210.03523, Section 2.4.2 approaches 1 and 2 with the
// maximum aggregator; Section 3.1 jump conditions (a) and (b)).
//
// k_select: one wave per plan element (then the optional per-stage decrease limit).  Lanes stride over the element's combinations of
// the sweep layout (c1 fastest), each keeping its best qualifying candidate under the
// total order (degrees of freedom, map value, N1, N2, N3); a butterfly of cross-lane
// exchanges leaves the minimum in every lane.
// k_jump: one lane per element, one Jacobi step of N_e <- max(N_e, max_j bound(N_j)) over
// the face neighbours j; nmax steps reach the least fixed point, because every hop lowers
// a bound by at least one and degrees are at least one.
// k_extrapolate: one lane per (plan element, combination of the extended map), the
// tau-extrapolation of the computed map to degrees at and above the reference degree.
#include <cfloat>
#include <climits>
#include <cmath>

#include "common.h"
#include "dgtau.h"

namespace dgt {

struct SelectMaps {
    const double *p[DG_SELECT_MAX_STAGES];
};

struct Cand {
    int ndof;  // INT_MAX: none
    double t;
    int code;  // N1 * 256 + N2 * 16 + N3: lexicographic order, N1 first
};

__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
    if (a.ndof != b.ndof) return a.ndof < b.ndof;
    if (a.t != b.t) return a.t < b.t;
    return a.code < b.code;
}

__device__ __forceinline__ Cand wave_best(Cand c) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        Cand o;
        o.ndof = __shfl_xor(c.ndof, m, 64);
        o.t = __shfl_xor(c.t, m, 64);
        o.code = __shfl_xor(c.code, m, 64);
        if (better(o, c)) c = o;
    }
    return c;
}

// Best candidate of one element over maps [s0, s1): a combination qualifies when its
// value is below tau_max in every one of them; its value is their maximum.  X = 0: maps
// in the sweep layout (combinations below the reference degree P only); X > 0: extended
// maps of X^3 combinations per element, N_i in 1..X, where the extrapolation has already
// given N_i >= P_i its value (or the high value).
__device__ Cand element_best(const int P[3], int64_t off, const SelectMaps &maps, int s0, int s1, double tau_max,
                             int nmin, int nmax, int X, int lane) {
    const int C1 = X ? X : P[0] > 1 ? P[0] - 1 : 1, C2 = X ? X : P[1] > 1 ? P[1] - 1 : 1;
    const int C3 = X ? X : P[2] > 1 ? P[2] - 1 : 1;
    const int nc = C1 * C2 * C3;
    Cand best{INT_MAX, 0.0, 0};
    for (int c = lane; c < nc; c += 64) {
        const int N[3] = {c % C1 + 1, (c / C1) % C2 + 1, c / (C1 * C2) + 1};
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) ok = ok && N[d] >= nmin && N[d] <= nmax && (X || N[d] < P[d]);
        if (!ok) continue;
        double t = 0.0;
        for (int s = s0; s < s1 && ok; ++s) {
            const double v = maps.p[s][off + c];
            ok = v < tau_max;  // false for NaN
            t = s == s0 ? v : fmax(t, v);
        }
        if (!ok) continue;
        const Cand cand{(N[0] + 1) * (N[1] + 1) * (N[2] + 1), t, N[0] * 256 + N[1] * 16 + N[2]};
        if (better(cand, best)) best = cand;
    }
    return wave_best(best);
}

__global__ __launch_bounds__(256) void k_select(const ElemInfo *__restrict__ el, int E,
                                                const int64_t *__restrict__ combo_off, SelectMaps maps, int nst,
                                                double tau_max, int nmin, int nmax, int approach,
                                                const int32_t *__restrict__ prev, int max_decrease, int X,
                                                int32_t *__restrict__ orders) {
    const int p = (int)((blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6);
    const int lane = threadIdx.x & 63;
    if (p >= E) return;  // whole waves only
    const ElemInfo e = el[p];
    const int P[3] = {e.n[0] - 1, e.n[1] - 1, e.n[2] - 1};
    const int64_t off = X ? (int64_t)p * X * X * X : combo_off[p];
    int out[3];
    auto decode = [&](const Cand &c, int N[3]) {
        if (c.ndof == INT_MAX) {
            N[0] = N[1] = N[2] = nmax;
        } else {
            N[0] = c.code >> 8;
            N[1] = (c.code >> 4) & 15;
            N[2] = c.code & 15;
        }
    };
    if (approach == 2) {
        decode(element_best(P, off, maps, 0, nst, tau_max, nmin, nmax, X, lane), out);
    } else {
        out[0] = out[1] = out[2] = 0;
        for (int s = 0; s < nst; ++s) {
            int N[3];
            decode(element_best(P, off, maps, s, s + 1, tau_max, nmin, nmax, X, lane), N);
#pragma unroll
            for (int d = 0; d < 3; ++d) out[d] = max(out[d], N[d]);
        }
    }
    if (prev) {  // at most max_decrease lower than the current degrees
        const int32_t *pv = prev + 3 * (int64_t)e.nat;
#pragma unroll
        for (int d = 0; d < 3; ++d) out[d] = max(out[d], min(nmax, pv[d] - max_decrease));
    }
    if (lane == 0) {
        int32_t *o = orders + 3 * (int64_t)e.nat;
        o[0] = out[0];
        o[1] = out[1];
        o[2] = out[2];
    }
}

// One Jacobi step of the jump condition on natural orders [E][3].
// periodic: bit d set when the box is periodic along d.
__global__ __launch_bounds__(256) void k_jump(const int32_t *__restrict__ cur, int32_t *__restrict__ nxt, int nx,
                                              int ny, int nz, int periodic, int kind) {
    const int64_t E = (int64_t)nx * ny * nz;
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= E) return;
    const int n[3] = {nx, ny, nz};
    const int idx[3] = {(int)(e % nx), (int)((e / nx) % ny), (int)(e / ((int64_t)nx * ny))};
    int o[3] = {cur[3 * e], cur[3 * e + 1], cur[3 * e + 2]};
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int side = -1; side <= 1; side += 2) {
            int j[3] = {idx[0], idx[1], idx[2]};
            j[d] += side;
            if (j[d] < 0 || j[d] >= n[d]) {
                if (!((periodic >> d) & 1)) continue;
                j[d] = (j[d] + n[d]) % n[d];
            }
            const int64_t f = j[0] + (int64_t)nx * (j[1] + (int64_t)ny * j[2]);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int nb = cur[3 * f + i];
                o[i] = max(o[i], kind == 1 ? (2 * nb) / 3 : nb - 1);
            }
        }
#pragma unroll
    for (int i = 0; i < 3; ++i) nxt[3 * e + i] = o[i];
}

// acc <- max(acc, m), NaN sticky (a NaN in either operand gives NaN)
__global__ __launch_bounds__(256) void k_map_fmax(double *acc, const double *m, int64_t n) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = acc[i], b = m[i];
    double r = b > a ? b : a;
    if (b != b) r = b;
    if (a != a) r = a;
    acc[i] = r;
}

// tau-extrapolation (one lane per extended entry; C_d = max(1, P_d - 1) the computed
// degrees): entries with N_d <= C_d everywhere copy the map; otherwise, from the inner
// corner N' (N'_d = C_d where N_d > C_d), every such direction continues the decay of
// the map line through N', ln tau fitted by least squares over its last min(3, C_d)
// degrees (slope y_C - y_{C-1} for two, (y_C - y_{C-2}) / 2 for three); a direction with
// one degree, a non-positive or non-finite value there, or no decay gives +inf.
__global__ __launch_bounds__(256) void k_extrapolate(const ElemInfo *__restrict__ el, int E,
                                                     const int64_t *__restrict__ combo_off,
                                                     const double *__restrict__ map, int X,
                                                     double *__restrict__ ext) {
    const int64_t X3 = (int64_t)X * X * X;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)E * X3) return;
    const int p = (int)(t / X3);
    const int k = (int)(t - p * X3);
    const int N[3] = {k % X + 1, (k / X) % X + 1, k / (X * X) + 1};
    const ElemInfo e = el[p];
    int C[3], cn[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        C[d] = e.n[d] > 2 ? e.n[d] - 2 : 1;
        cn[d] = N[d] > C[d] ? C[d] : N[d];
    }
    const double *m = map + combo_off[p];
    auto at = [&](const int M[3]) { return m[(M[0] - 1) + C[0] * ((M[1] - 1) + C[1] * (M[2] - 1))]; };
    double v = at(cn);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (N[d] <= C[d] || v == HUGE_VAL) continue;
        const int L = C[d] < 3 ? C[d] : 3;
        if (L < 2) {
            v = HUGE_VAL;
            continue;
        }
        double y[3] = {0.0, 0.0, 0.0};
        bool ok = true;
        for (int j = 0; j < L; ++j) {
            int M[3] = {cn[0], cn[1], cn[2]};
            M[d] = C[d] - L + 1 + j;
            const double w = at(M);
            ok = ok && w > 0.0 && w <= DBL_MAX;  // false for NaN and +inf
            y[j] = ok ? log(w) : 0.0;
        }
        const double beta = L == 2 ? y[1] - y[0] : 0.5 * (y[2] - y[0]);
        v = ok && beta < 0.0 ? v * exp(beta * (double)(N[d] - C[d])) : HUGE_VAL;
    }
    ext[t] = v;
}

hipError_t launch_extrapolate(const ElemInfo *el, int E, const int64_t *combo_off, const double *map, int X,
                              double *ext, hipStream_t s) {
    const int64_t n = (int64_t)E * X * X * X;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_extrapolate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, el, E, combo_off, map, X,
                       ext);
    return hipGetLastError();
}

hipError_t launch_map_fmax(double *acc, const double *m, int64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_map_fmax, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, m, n);
    return hipGetLastError();
}

hipError_t launch_select(const ElemInfo *el, int E, const int64_t *combo_off, const double *const *maps, int nst,
                         double tau_max, int nmin, int nmax, int approach, const int32_t *prev, int max_decrease,
                         int X, int jump, int nx, int ny, int nz, int periodic, int32_t *orders, int32_t *tmp,
                         hipStream_t s) {
    if (E == 0) return hipSuccess;
    SelectMaps m{};
    for (int i = 0; i < nst; ++i) m.p[i] = maps[i];
    const int blocks = (int)((E * 64LL + 255) / 256);
    hipLaunchKernelGGL(k_select, dim3(blocks), dim3(256), 0, s, el, E, combo_off, m, nst, tau_max, nmin, nmax,
                       approach, prev, max_decrease, X, orders);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess || jump == 0) return err;
    // an even number of steps (at least nmax) ends in orders
    const int steps = nmax + (nmax & 1);
    const int jb = (E + 255) / 256;
    for (int k = 0; k < steps; k += 2) {
        hipLaunchKernelGGL(k_jump, dim3(jb), dim3(256), 0, s, orders, tmp, nx, ny, nz, periodic, jump);
        hipLaunchKernelGGL(k_jump, dim3(jb), dim3(256), 0, s, tmp, orders, nx, ny, nz, periodic, jump);
    }
    return hipGetLastError();
}

}  // namespace dgt
