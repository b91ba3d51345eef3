// Tau-estimation kernels for gfx950 (Section 2.3, variational DG estimate).
//
//   k_restrict_w : restricts the fine element polynomial of Q and of the fine time
//                derivative to the coarse orders, by sampling at the coarse
//                Gauss-Lobatto nodes or by the exact L2 projection (sum-factorised
//                A3 (x) A2 (x) A1: x in registers, y and z through LDS), writing the
//                coarse plan layout.  The coarse residual and the tau difference then run in
//                the element kernel's tau epilogue.
//   k_sweep    : the isolated truncation-error map.  One workgroup per (fine
//                element, c1, c2): the x-interpolation of Q and of the time
//                derivative is shared by every (c2, c3), the y-interpolation by
//                every c3; for each c3 the workgroup evaluates the isolated
//                coarse volume residual V/J, the difference with the restricted
//                time derivative, both forms and their maxima.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "euler.h"

namespace dgt {


// ---------------------------------------------------------------------------- restriction
// Per direction the operator is the interpolation where the order rises or stays and,
// where it falls, the table at offset `down`: T_I (sampling) or T_P (exact L2
// projection).  PROJECT: the solution transfer onto another order map (Section 2.4.1,
// down = T_P): the "coarse" element is the target, of any orders, the source element is
// found through the source plan's natural -> plan index (fine_of), one field (Q); the
// restriction itself reads the fine element's record at the coarse element's position.
// psi_new: the adjoint weight is the adjoint of the new-form residual M^-1 F, i.e. M times
// the traditional-form adjoint (M = J w_i w_j w_k of the fine element); it is divided by
// M as it is loaded (box elements: J = 1/invJ; curved: J per node from met).
// m / n for 0 <= m < 2^20 and n <= 1000 through the float reciprocal of n: the exact
// quotient of m + 1/2 sits at least 1/(2n) from an integer, far beyond the rounding of
// the product, so the truncation is the integer quotient (integer division by a
// run-time value takes tens of instructions).
__device__ __forceinline__ int qdiv(int m, float inv_n) { return (int)(((float)m + 0.5f) * inv_n); }

// One wave per (coarse element, field, variable): lane = fine x-line (j, k) of the
// element, loaded into registers (8 doubles); the x-pass runs from registers into LDS,
// the y-pass and the z-pass through LDS into the coarse plan layout, with barriers of
// one wave only.  Small waves (a few KB of LDS and registers) keep many of them
// resident per CU, so the loads of some overlap the passes of others (one workgroup of
// five waves per (element, field) was slower: 98.6 against 77.7 us on 16^3 elements,
// N = 7).  LDS: s1 [c1][f2 f3], overwritten by the y-pass result [c1 c2][f3] (held in
// registers across a barrier), then the y and z operators (read there rather than
// through the vector cache).  Elements with more than 64 fine x-lines (f2 f3 > 64) take
// them 64 at a time.
constexpr int RW_YIT = (NNMAX * NNMAX * NNMAX + 63) / 64;  // y-pass outputs per lane
template <bool PROJECT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) void k_restrict_w(const int32_t *__restrict__ fine_of,
                                                   const ElemInfo *__restrict__ cel,
                                                   const ElemInfo *__restrict__ fel, const double *__restrict__ u,
                                                   const double *__restrict__ dudt, const double *__restrict__ psi,
                                                   double *__restrict__ uc, double *__restrict__ rdc,
                                                   double *__restrict__ psic, const double *__restrict__ tab,
                                                   int cap1, int down, int psi_new, const double *__restrict__ met,
                                                   double invJ, int nfield) {
    extern __shared__ double lds[];
    double *s1 = lds, *sI = lds + cap1;  // sI: the y and z operators
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int pf = w / NV, v = w - pf * NV;
    const int p = pf / nfield, field = pf - p * nfield;
    const int lane = threadIdx.x;
    const ElemInfo C = cel[p];
    const ElemInfo F = PROJECT ? fel[fine_of[C.nat]] : fel[p];
    const int f1 = F.n[0], f2 = F.n[1], f3 = F.n[2], nl = f2 * f3, nef = f1 * nl;
    const int c1 = C.n[0], c2 = C.n[1], c3 = C.n[2], n12 = c1 * c2, nec = n12 * c3;
    const float ic1 = 1.0f / c1, ic2 = 1.0f / c2, ic12 = 1.0f / n12;
    auto op = [&](int c, int f) { return tab + (c < f ? down : T_I) + moff(c - 1, f - 1); };
    const double *I1 = op(c1, f1);
    {
        const double *g2 = op(c2, f2), *g3 = op(c3, f3);
        for (int t = lane; t < c2 * f2 + c3 * f3; t += 64)
            sI[t] = t < c2 * f2 ? g2[t] : g3[t - c2 * f2];
    }  // ordered before their first use by the barrier after the x-pass
    const double *I2 = sI, *I3 = sI + c2 * f2;
    const double *src = (field == 0 ? u : field == 1 ? dudt : psi) + NV * F.noff + (int64_t)v * nef;
    double *dst = (field == 0 ? uc : field == 1 ? rdc : psic) + NV * C.noff + (int64_t)v * nec;
    const bool scale = !PROJECT && field == 2 && psi_new;

    // x: s1[a + c1 jk] = sum_i I1[a, i] Q_v[i + f1 jk]
    for (int l0 = 0; l0 < nl; l0 += 64) {
        const int jk = l0 + lane;
        if (jk >= nl) continue;
        double ln[NNMAX];
        double sc = 1.0;
        if (scale) {
            const double *w2 = tab + T_W + xoff(f2 - 1), *w3 = tab + T_W + xoff(f3 - 1);
            const int k = qdiv(jk, 1.0f / f2);
            sc = 1.0 / (w2[jk - k * f2] * w3[k]);
        }
#pragma unroll
        for (int i = 0; i < NNMAX; ++i) {
            double x = i < f1 ? src[f1 * jk + i] : 0.0;
            if (scale && i < f1) {
                const int node = i + f1 * jk;
                const double ij = met ? 1.0 / met[10 * F.noff + 9 * nef + node] : invJ;
                x *= ij * sc / tab[T_W + xoff(f1 - 1) + i];
            }
            ln[i] = x;
        }
        for (int a = 0; a < c1; ++a) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < NNMAX; ++i)
                if (i < f1) acc += I1[a * f1 + i] * ln[i];
            s1[a + c1 * jk] = acc;
        }
    }
    __syncthreads();
    // y: s2[a + c1 (b + c2 k)] = sum_j I2[b, j] s1[a + c1 (j + f2 k)], s2 over s1
    double yv[RW_YIT];
#pragma unroll
    for (int it = 0; it < RW_YIT; ++it) {
        const int t = lane + 64 * it;
        yv[it] = 0.0;
        if (t < n12 * f3) {
            const int r = qdiv(t, ic1), a = t - r * c1, k = qdiv(r, ic2), b = r - k * c2;
            const double *x = s1 + a + c1 * f2 * k;
            const double *wy = I2 + b * f2;
            double acc = 0.0;
            for (int j = 0; j < f2; ++j) acc += wy[j] * x[c1 * j];
            yv[it] = acc;
        }
    }
    __syncthreads();
    double *s2 = s1;
#pragma unroll
    for (int it = 0; it < RW_YIT; ++it)
        if (lane + 64 * it < n12 * f3) s2[lane + 64 * it] = yv[it];
    __syncthreads();
    // z: the coarse plan layout, node a + c1 (b + c2 c)
    for (int t = lane; t < nec; t += 64) {
        const int c = qdiv(t, ic12), ab = t - c * n12;
        const double *x = s2 + ab;
        const double *wz = I3 + c * f3;
        double acc = 0.0;
        for (int k = 0; k < f3; ++k) acc += wz[k] * x[n12 * k];
        dst[t] = acc;
    }
}

hipError_t launch_restrict(int ncoarse, const ElemInfo *celems, const ElemInfo *felems,
                           const double *u, const double *dudt, const double *psi, double *uc, double *rdc,
                           double *psic, const double *tab, int capA, int capB, int restriction, int psi_new,
                           const double *met, double invJ, hipStream_t s) {
    if (ncoarse == 0) return hipSuccess;
    const int nfield = psi ? 3 : 2;
    const size_t lds = sizeof(double) * (size_t)(capA / NV + capB / NV);
    hipLaunchKernelGGL(k_restrict_w<false>, dim3(ncoarse * nfield * NV), dim3(64), lds, s, nullptr, celems, felems, u,
                       dudt, psi, uc, rdc, psic, tab, capA / NV, restriction ? T_P : T_I, psi_new, met, invJ, nfield);
    return hipGetLastError();
}

hipError_t launch_project(const int32_t *src_inv, int ntarget, const ElemInfo *tel, const ElemInfo *sel,
                          const double *u, double *ut, const double *tab, int capA, int capB, hipStream_t s) {
    if (ntarget == 0) return hipSuccess;
    const size_t lds = sizeof(double) * (size_t)(capA / NV + capB / NV);
    hipLaunchKernelGGL(k_restrict_w<true>, dim3(ntarget * NV), dim3(64), lds, s, src_inv, tel, sel, u, nullptr, nullptr,
                       ut, nullptr, nullptr, tab, capA / NV, T_P, 0, nullptr, 0.0, 1);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- sweep
__device__ __forceinline__ double wave_max(double x) {
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o));
    return x;
}

constexpr int SW_WG = 256;
constexpr int SW_NPL = 3;  // coarse nodes per lane: up to 768 (order 9 in every direction: 729)

// Dynamic LDS layout (doubles): X1 [5][m1][f2][f3] (aliased by the flux stage
// [5][m1 m2 m3]), X2Q and X2R [5][m1][m2][f3], red [2][4].
__global__ __launch_bounds__(SW_WG) void k_sweep(const SweepTask *__restrict__ tasks, int ntasks,
                                                 const ElemInfo *__restrict__ el,
                                                 const int64_t *__restrict__ combo_off,
                                                 const double *__restrict__ u, const double *__restrict__ dudt,
                                                 const double *__restrict__ tab, Geom g, double gamma,
                                                 int x1cap, int x2cap, int rt, double *__restrict__ te_new,
                                                 double *__restrict__ te_trad) {
    extern __shared__ double lds[];
    double *sX1 = lds;
    double *sX2Q = sX1 + x1cap;
    double *sX2R = sX2Q + x2cap;
    double *sRed = sX2R + x2cap;
    const SweepTask task = tasks[xcd_remap(blockIdx.x, ntasks)];
    const ElemInfo E = el[task.p];
    const int f1 = E.n[0], f2 = E.n[1], f3 = E.n[2], nef = f1 * f2 * f3;
    const int m1 = task.c1 + 1, m2 = task.c2 + 1;
    const int C1 = f1 > 2 ? f1 - 2 : 1, C2 = f2 > 2 ? f2 - 2 : 1, C3 = f3 > 2 ? f3 - 2 : 1;
    const double *I1 = tab + rt + moff(m1 - 1, f1 - 1);
    const double *I2 = tab + rt + moff(m2 - 1, f2 - 1);
    const int tid = threadIdx.x;
    const double gm1 = gamma - 1.0;

    for (int field = 0; field < 2; ++field) {
        const double *src = (field == 0 ? u : dudt) + NV * E.noff;
        double *dst = field == 0 ? sX2Q : sX2R;
        for (int t = tid; t < NV * m1 * f2 * f3; t += SW_WG) {
            const int a = t % m1, r = t / m1;  // r = v*(f2*f3) + jk
            const int v = r / (f2 * f3), jk = r - v * (f2 * f3);
            const double *row = src + v * nef + f1 * jk;
            double acc = 0.0;
            for (int i = 0; i < f1; ++i) acc += I1[a * f1 + i] * row[i];
            sX1[t] = acc;  // index a + m1*(jk + f2*f3*v)
        }
        __syncthreads();
        for (int t = tid; t < NV * m1 * m2 * f3; t += SW_WG) {
            const int a = t % m1, b = (t / m1) % m2, r = t / (m1 * m2);  // r = v*f3 + k
            const int v = r / f3, k = r - v * f3;
            double acc = 0.0;
            for (int j = 0; j < f2; ++j) acc += I2[b * f2 + j] * sX1[a + m1 * (j + f2 * (k + f3 * v))];
            dst[t] = acc;  // index a + m1*(b + m2*(k + f3*v))
        }
        __syncthreads();
    }

    const double invJ = 1.0 / g.J;
    const double *w1 = tab + T_W + xoff(m1 - 1);
    const double *w2 = tab + T_W + xoff(m2 - 1);
    double *sF = sX1;  // X1 is dead now
    for (int c3 = 1; c3 <= C3; ++c3) {
        const int m3 = c3 + 1, M = m1 * m2 * m3;
        const double *I3 = tab + rt + moff(m3 - 1, f3 - 1);
        const double *w3 = tab + T_W + xoff(m3 - 1);
        double q[SW_NPL][NV], V[SW_NPL][NV];
        int loc[SW_NPL][3];
        bool ok[SW_NPL];
#pragma unroll
        for (int k = 0; k < SW_NPL; ++k) {
            const int t = tid + k * SW_WG;
            ok[k] = t < M;
            const int tt = ok[k] ? t : 0;
            loc[k][0] = tt % m1;
            loc[k][1] = (tt / m1) % m2;
            loc[k][2] = tt / (m1 * m2);
            const int ab = loc[k][0] + m1 * loc[k][1];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double acc = 0.0;
                for (int kk = 0; kk < f3; ++kk) acc += I3[loc[k][2] * f3 + kk] * sX2Q[ab + m1 * m2 * (kk + f3 * v)];
                q[k][v] = ok[k] ? acc : 1.0;
                V[k][v] = 0.0;
            }
        }
        const int mm[3] = {m1, m2, m3};
        const int st[3] = {1, m1, m1 * m2};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double Ja = g.Ja[d];
#pragma unroll
            for (int k = 0; k < SW_NPL; ++k) {
                if (!ok[k]) continue;
                double f[NV];
                flux_axis(q[k], d, gm1, f);
#pragma unroll
                for (int v = 0; v < NV; ++v) sF[v * M + tid + k * SW_WG] = Ja * f[v];
            }
            __syncthreads();
            const double *Dm = tab + T_D + doff(mm[d] - 1);
#pragma unroll
            for (int k = 0; k < SW_NPL; ++k) {
                if (!ok[k]) continue;
                const int id = loc[k][d];
                const int tb = tid + k * SW_WG - id * st[d];
                for (int m = 0; m < mm[d]; ++m) {
                    const double dm = Dm[id * mm[d] + m];
#pragma unroll
                    for (int v = 0; v < NV; ++v) V[k][v] += dm * sF[v * M + tb + m * st[d]];
                }
            }
            __syncthreads();
        }
        double mx0 = 0.0, mx1 = 0.0;
#pragma unroll
        for (int k = 0; k < SW_NPL; ++k) {
            if (!ok[k]) continue;
            const int ab = loc[k][0] + m1 * loc[k][1];
            const double Jw = g.J * w1[loc[k][0]] * w2[loc[k][1]] * w3[loc[k][2]];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double rc = 0.0;
                for (int kk = 0; kk < f3; ++kk) rc += I3[loc[k][2] * f3 + kk] * sX2R[ab + m1 * m2 * (kk + f3 * v)];
                const double a = V[k][v] * invJ - rc;
                mx0 = fmax(mx0, fabs(a));
                mx1 = fmax(mx1, fabs(Jw * a));
            }
        }
        mx0 = wave_max(mx0);
        mx1 = wave_max(mx1);
        if ((tid & 63) == 0) {
            sRed[tid >> 6] = mx0;
            sRed[4 + (tid >> 6)] = mx1;
        }
        __syncthreads();
        if (tid == 0) {
            const double r0 = fmax(fmax(sRed[0], sRed[1]), fmax(sRed[2], sRed[3]));
            const double r1 = fmax(fmax(sRed[4], sRed[5]), fmax(sRed[6], sRed[7]));
            const int64_t slot = combo_off[task.p] + (task.c1 - 1) + C1 * ((task.c2 - 1) + C2 * (c3 - 1));
            te_new[slot] = r0;
            te_trad[slot] = r1;
        }
        __syncthreads();
    }
}

hipError_t launch_sweep_tasks(const void *tasks, int ntasks, const ElemInfo *elems, const int64_t *combo_off,
                              const double *u, const double *dudt, const double *tab, Geom g, double gamma,
                              int x1cap, int x2cap, int restriction, double *te_new, double *te_trad,
                              hipStream_t s) {
    if (ntasks == 0) return hipSuccess;
    size_t lds = sizeof(double) * (size_t)(x1cap + 2 * x2cap + 8);
    if (lds > 64 * 1024) {  // per device: set on every launch (a host-side call)
        hipError_t e = hipFuncSetAttribute((const void *)k_sweep, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           160 * 1024);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sweep, dim3(ntasks), dim3(SW_WG), lds, s, (const SweepTask *)tasks, ntasks, elems,
                       combo_off, u, dudt, tab, g, gamma, x1cap, x2cap, restriction ? T_P : T_I, te_new, te_trad);
    return hipGetLastError();
}

}  // namespace dgt

namespace dgt {

// ---------------------------------------------------------------------------- isotropic sweep
// Fast path of the isolated sweep for elements with the same fine order in every
// direction (F = N+1 nodes, F <= 8).  With C = max(1, F-2) coarse orders per
// direction and m = c+1 coarse nodes, the coarse x-rows of two orders c1 and
// C+1-c1 are stacked (at most C+3 rows) and the coarse y-rows of every c2 are
// stacked (sum_c m = C(C+3)/2 rows), so one workgroup of 256 lanes covers a
// pair of c1 values and every c2 (243 lanes at F = 8), each lane owning one
// z-line (a, b):
//   - x-interpolation of Q and dQ/dt for the pair, cooperatively, into LDS;
//   - each lane forms its y-interpolated z-line of both fields in registers;
//   - for every c3 (compile-time): z-interpolation and the z part of the
//     derivative in registers with wave-uniform coefficients; x- and y-fluxes
//     are exchanged through LDS; the tau difference and its maxima per
//     (c1, c2, c3) are folded with LDS atomics on the bit patterns.
// The lanes of one c2 (rows x (c2+1) z-lines) form a block, and the blocks are
// packed into the four waves largest first, each into the first wave with room, so
// that every x- and y-neighbour of a lane is in its own wave: the exchange then
// needs no workgroup barrier, and the waves drift apart, overlapping one wave's
// LDS reads with another's arithmetic.
template <int F>
constexpr bool iso_blocks_fit_waves() {
    constexpr int C = F > 2 ? F - 2 : 1;
    for (int pair = 0; pair < (C + 1) / 2; ++pair) {
        const int cA = pair + 1, cBr = C - pair;
        const int cB = cBr == cA ? 0 : cBr;
        const int rows = cA + 1 + (cB ? cB + 1 : 0);
        int fill[4] = {0, 0, 0, 0};
        for (int cc = C; cc >= 1; --cc) {
            const int sz = rows * (cc + 1);
            int q = 0;
            while (q < 4 && fill[q] + sz > 64) ++q;
            if (q == 4) return false;
            fill[q] += sz;
        }
    }
    return true;
}

// orders the LDS accesses of one wave (they execute in order; no hardware wait needed)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int F>
__global__ __launch_bounds__(256) void k_sweep_iso(const int2 *__restrict__ elems, int njobs, SweepProb single,
                                                   const SweepProb *__restrict__ probs,
                                                   const double *__restrict__ tab, int rt) {
    constexpr int C = F > 2 ? F - 2 : 1;        // coarse orders per direction
    constexpr int NPAIR = (C + 1) / 2;
    constexpr int RMAX = C + 3;                 // rows of a pair of x-orders
    constexpr int MM = C + 1;                   // largest coarse node count
    constexpr int NL = 256;
    constexpr int SLOTS = 2 * C * C * 2;        // [c3][c1 of the pair][c2][form]
    // row stride of X1: odd in doubles, so the lanes of different x-rows that read
    // the same (j, k) fall in different LDS banks
    constexpr int X1S = F * F + 1;
    static_assert(2 * NV * RMAX * X1S <= 2 * NV * MM * 256, "X1 fits in the staging area");
    static_assert(iso_blocks_fit_waves<F>(), "every c2 block fits in one wave");
    extern __shared__ double lds[];
    double *S = lds;                                                     // staging / X1
    unsigned long long *slot = (unsigned long long *)(lds + 2 * NV * MM * NL);

    const int job = xcd_remap(blockIdx.x, njobs);
    const int pair = job % NPAIR;
    const int2 pe = elems[job / NPAIR];
    const SweepProb P = probs ? probs[pe.x] : single;
    const double *__restrict__ u = P.u;
    const double *__restrict__ dudt = P.dudt;
    const Geom g = P.g;
    const double gamma = P.gamma;
    const int p = pe.y;
    const ElemInfo E = P.el[p];
    const int cA = pair + 1, cBr = C - pair;
    const int cB = cBr == cA ? 0 : cBr;
    const int mA = cA + 1, mB = cB ? cB + 1 : 0;
    const int rows = mA + mB;
    const int lane = threadIdx.x;
    const double gm1 = gamma - 1.0;

    for (int i = lane; i < SLOTS; i += NL) slot[i] = 0ull;

    // x-interpolation: X1[f][v][row][j][k], row over the pair's stacked coarse x-nodes
    {
        const double *IA = tab + rt + moff(mA - 1, F - 1);
        const double *IB = tab + rt + moff((mB ? mB : 2) - 1, F - 1);
        for (int r = lane; r < 2 * NV * F * F; r += NL) {
            const int f = r / (NV * F * F), rem = r - f * NV * F * F;  // rem = v*F*F + jk
            const double *src = (f == 0 ? u : dudt) + NV * E.noff + (int64_t)rem * F;
            double row[F];
#pragma unroll
            for (int i = 0; i < F; ++i) row[i] = src[i];
            const int v = rem / (F * F), jk = rem - v * F * F;
            double *dst = S + ((f * NV + v) * RMAX) * X1S + jk;
            for (int a = 0; a < mA; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < F; ++i) acc += IA[a * F + i] * row[i];
                dst[a * X1S] = acc;
            }
            for (int a = 0; a < mB; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < F; ++i) acc += IB[a * F + i] * row[i];
                dst[(mA + a) * X1S] = acc;
            }
        }
    }
    __syncthreads();

    // lane -> z-line (a, b) of the c2 block that covers it: lane = lbase + a + rows*b
    int c2 = 0, lbase = lane;
    {
        const int w = lane >> 6, off = lane & 63;
        int fill[4] = {0, 0, 0, 0};
#pragma unroll
        for (int cc = C; cc >= 1; --cc) {
            const int sz = rows * (cc + 1);
            bool placed = false;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (placed || fill[q] + sz > 64) continue;
                if (q == w && off >= fill[q] && off < fill[q] + sz) {
                    c2 = cc;
                    lbase = 64 * q + fill[q];
                }
                fill[q] += sz;
                placed = true;
            }
        }
    }
    const bool active = c2 != 0;
    if (!active) c2 = 1;
    const int a = active ? (lane - lbase) % rows : 0;
    const int b = active ? (lane - lbase) / rows : 0;
    const int m2 = c2 + 1;
    const bool inA = a < mA;
    const int c1 = inA ? cA : cB;
    const int m1 = c1 + 1;
    const int al = inA ? a : a - mA;            // local x-node
    const int a0 = inA ? 0 : mA;                // first row of this c1

    // per-lane rows of the 1D operators
    double Dx[MM], Dy[MM], I2r[F];
    {
        const double *dx = tab + T_D + doff(m1 - 1) + al * m1;
        const double *dy = tab + T_D + doff(m2 - 1) + b * m2;
        const double *i2 = tab + rt + moff(m2 - 1, F - 1) + b * F;
#pragma unroll
        for (int q = 0; q < MM; ++q) {
            Dx[q] = q < m1 ? dx[q] : 0.0;
            Dy[q] = q < m2 ? dy[q] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < F; ++j) I2r[j] = i2[j];
    }
    const double w12 = g.J * tab[T_W + xoff(m1 - 1) + al] * tab[T_W + xoff(m2 - 1) + b];

    // y-interpolated z-lines of both fields
    double XQ[NV][F], XR[NV][F];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double *x1 = S + ((f * NV + v) * RMAX + a) * X1S;
#pragma unroll
            for (int k = 0; k < F; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < F; ++j) acc += I2r[j] * x1[j + F * k];
                if (f == 0) XQ[v][k] = acc; else XR[v][k] = acc;
            }
        }
    }
    __syncthreads();  // X1 is dead; S becomes the flux staging area

    const double invJ = 1.0 / g.J;
    const double Jax = g.Ja[0], Jay = g.Ja[1], Jaz = g.Ja[2];
    const int grp = (inA ? 0 : 1) * C + (c2 - 1);
    double *Sx = S, *Sy = S + NV * MM * NL;

#pragma unroll
    for (int c3 = 1; c3 <= C; ++c3) {
        const int m3 = c3 + 1;
        const double *I3 = tab + rt + moff(m3 - 1, F - 1);
        const double *D3 = tab + T_D + doff(m3 - 1);
        const double *w3 = tab + T_W + xoff(m3 - 1);
        double V[NV][MM];
#pragma unroll
        for (int c = 0; c < MM; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v) V[v][c] = 0.0;
        // coarse state at node c of the line (z-interpolation with wave-uniform weights)
        auto node_state = [&](int c, double q[NV]) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < F; ++k) acc += I3[c * F + k] * XQ[v][k];
                q[v] = acc;
            }
        };
        // z: flux at each node, then D3 along the line (all in registers)
#pragma unroll
        for (int cp = 0; cp < MM; ++cp) {
            if (cp >= m3) continue;
            double q[NV], fz[NV];
            node_state(cp, q);
            flux_axis(q, 2, gm1, fz);
#pragma unroll
            for (int c = 0; c < MM; ++c) {
                if (c >= m3) continue;
                const double dz = D3[c * m3 + cp];
#pragma unroll
                for (int v = 0; v < NV; ++v) V[v][c] += dz * (Jaz * fz[v]);
            }
            double fx[NV], fy[NV];
            flux_axis(q, 0, gm1, fx);
            flux_axis(q, 1, gm1, fy);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Sx[(v * MM + cp) * NL + lane] = Jax * fx[v];
                Sy[(v * MM + cp) * NL + lane] = Jay * fy[v];
            }
        }
        wave_lds_sync();
        if (active) {
            // x: neighbours are the lanes of the same y-row and x-order
#pragma unroll
            for (int q = 0; q < MM; ++q) {
                if (q >= m1) continue;
                const int ln = lbase + (a0 + q) + rows * b;
                const double d = Dx[q];
#pragma unroll
                for (int c = 0; c < MM; ++c) {
                    if (c >= m3) continue;
#pragma unroll
                    for (int v = 0; v < NV; ++v) V[v][c] += d * Sx[(v * MM + c) * NL + ln];
                }
            }
#pragma unroll
            for (int q = 0; q < MM; ++q) {
                if (q >= m2) continue;
                const int ln = lbase + a + rows * q;
                const double d = Dy[q];
#pragma unroll
                for (int c = 0; c < MM; ++c) {
                    if (c >= m3) continue;
#pragma unroll
                    for (int v = 0; v < NV; ++v) V[v][c] += d * Sy[(v * MM + c) * NL + ln];
                }
            }
            double mx0 = 0.0, mx1 = 0.0;
#pragma unroll
            for (int c = 0; c < MM; ++c) {
                if (c >= m3) continue;
                const double jw = w12 * w3[c];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double rc = 0.0;
#pragma unroll
                    for (int k = 0; k < F; ++k) rc += I3[c * F + k] * XR[v][k];
                    const double t = V[v][c] * invJ - rc;
                    mx0 = fmax(mx0, fabs(t));
                    mx1 = fmax(mx1, fabs(jw * t));
                }
            }
            unsigned long long *sl = slot + ((c3 - 1) * 2 * C + grp) * 2;
            atomicMax(sl, (unsigned long long)__double_as_longlong(mx0));
            atomicMax(sl + 1, (unsigned long long)__double_as_longlong(mx1));
        }
        wave_lds_sync();
    }
    __syncthreads();
    // write the maxima of every (c1, c2, c3) of this workgroup
    for (int i = lane; i < 2 * C * C; i += NL) {
        const int c3 = i / (2 * C) + 1, gi = i % (2 * C);
        const int cc1 = gi < C ? cA : cB;
        if (cc1 == 0) continue;
        const int cc2 = gi % C + 1;
        const int64_t s = P.combo_off[p] + (cc1 - 1) + C * ((cc2 - 1) + C * (c3 - 1));
        P.te_new[s] = __longlong_as_double((long long)slot[2 * i]);
        P.te_trad[s] = __longlong_as_double((long long)slot[2 * i + 1]);
    }
}

template <int F>
static hipError_t launch_iso(const int2 *elems, int nelem, const SweepProb &single, const SweepProb *probs,
                             const double *tab, int rt, hipStream_t s) {
    constexpr int C = F > 2 ? F - 2 : 1;
    constexpr int MM = C + 1;
    constexpr int NPAIR = (C + 1) / 2;
    const size_t lds = sizeof(double) * (size_t)(2 * NV * MM * 256) + sizeof(unsigned long long) * 2 * C * C * 2;
    const int njobs = nelem * NPAIR;
    auto go = [&](auto kern) {
        // per device: set on every launch (a host-side call)
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(njobs), dim3(256), lds, s, elems, njobs, single, probs, tab, rt);
        return hipGetLastError();
    };
    return go(k_sweep_iso<F>);
}

// ---------------------------------------------------------------------------- anisotropic sweep
// The same scheme for elements whose fine orders differ between directions (fine node
// counts F1, F2 <= 8 at run time, F3 <= 8 at compile time): a job per (element, pair of
// coarse x-orders c1 and C1 + 1 - c1), a lane per coarse z-line (a, B) of the job with
// the x-rows of the pair and the y-rows of every c2 stacked, the z direction in
// registers.  A workgroup runs up to AN_JOBS jobs side by side (the host packs them so
// that their lanes, x-interpolated rows and maxima fit): job j holds lanes
// [lane0_j, lane0_j + rows_j * SUMM_j) and its x-rows at offset x1_j of the staging area.
constexpr int AN_JOBS = AN_JOBS_MAX;

// SAMPLE (the sampling restriction): the coarse LGL end nodes are fine nodes, so the
// z-interpolation at them is the fine value itself (the table rows there are unit
// vectors) and is skipped.  (The isotropic kernel keeps the table rows: there the
// shortcut changes the compiler's schedule into register spills.)
template <int F3, bool SAMPLE>
__global__ __launch_bounds__(256) void k_sweep_an(const int4 *__restrict__ wgs, int nwg,
                                                  const int4 *__restrict__ jobs, SweepProb single,
                                                  const SweepProb *__restrict__ probs,
                                                  const double *__restrict__ tab, int rt) {
    constexpr int C3 = F3 > 2 ? F3 - 2 : 1;     // coarse z-orders
    constexpr int MM = C3 + 1;                  // largest coarse z node count
    constexpr int FM = 8;                       // largest fine x and y node count
    constexpr int MX = FM - 1;                  // largest coarse x and y node count
    constexpr int CM = FM - 2;                  // largest number of coarse x or y orders
    constexpr int NSL = 2 * C3 * 2 * CM;        // maxima slots of one job: [c3][c1 of the pair][c2][form]
    constexpr int NL = 256;
    extern __shared__ double lds[];
    double *S = lds;                                                     // staging / X1
    unsigned long long *slot = (unsigned long long *)(lds + 2 * NV * MM * NL);

    const int4 W = wgs[xcd_remap(blockIdx.x, nwg)];  // (first job, job count, problem, 0)
    const SweepProb P = probs ? probs[W.z] : single;
    const ElemInfo *__restrict__ el = P.el;
    const double *__restrict__ u = P.u;
    const double *__restrict__ dudt = P.dudt;
    const Geom g = P.g;
    const int lane = threadIdx.x;
    const double gm1 = P.gamma - 1.0;

    for (int i = lane; i < W.y * NSL; i += NL) slot[i] = 0ull;

    // x-interpolation of every job: X1[f][v][row][j][k] at the job's offset
    for (int jb = 0; jb < W.y; ++jb) {
        const int4 J = jobs[W.x + jb];
        const ElemInfo E = el[J.x];
        const int F1 = E.n[0], F2 = E.n[1];
        const int C1 = F1 > 2 ? F1 - 2 : 1;
        const int cA = J.y + 1, cBr = C1 - J.y;
        const int cB = cBr == cA ? 0 : cBr;
        const int mA = cA + 1, mB = cB ? cB + 1 : 0, rows = mA + mB;
        const int X1S = F2 * F3 + 1;            // odd row stride (LDS banks)
        const double *IA = tab + rt + moff(mA - 1, F1 - 1);
        const double *IB = tab + rt + moff((mB ? mB : 2) - 1, F1 - 1);
        const int nl = F2 * F3;
        double *X1 = S + J.w;
        for (int r = lane; r < 2 * NV * nl; r += NL) {
            const int f = r / (NV * nl), rem = r - f * NV * nl;  // rem = v*nl + jk
            const double *src = (f == 0 ? u : dudt) + NV * E.noff + (int64_t)rem * F1;
            double row[FM];
#pragma unroll
            for (int i = 0; i < FM; ++i) row[i] = i < F1 ? src[i] : 0.0;
            const int v = rem / nl, jk = rem - v * nl;
            double *dst = X1 + ((f * NV + v) * rows) * X1S + jk;
            for (int a = 0; a < mA; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    if (i < F1) acc += IA[a * F1 + i] * row[i];
                dst[a * X1S] = acc;
            }
            for (int a = 0; a < mB; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    if (i < F1) acc += IB[a * F1 + i] * row[i];
                dst[(mA + a) * X1S] = acc;
            }
        }
    }
    __syncthreads();

    // lane -> job, then z-line (a, B) of the job
    int jb = 0;
    while (jb + 1 < W.y && lane >= jobs[W.x + jb + 1].z) ++jb;
    const int4 J = jobs[W.x + jb];
    const ElemInfo E = el[J.x];
    const int F1 = E.n[0], F2 = E.n[1];
    const int C1 = F1 > 2 ? F1 - 2 : 1, C2 = F2 > 2 ? F2 - 2 : 1;
    const int SUMM = C2 * (C2 + 3) / 2;         // stacked coarse y-rows over every c2
    const int X1S = F2 * F3 + 1;
    const int cA = J.y + 1, cBr = C1 - J.y;
    const int cB = cBr == cA ? 0 : cBr;
    const int mA = cA + 1, mB = cB ? cB + 1 : 0;
    const int rows = mA + mB;
    const int lj = lane - J.z;                  // lane within the job
    const bool active = lj >= 0 && lj < rows * SUMM;
    const int a = active ? lj % rows : 0;
    const int B = active ? lj / rows : 0;
    int c2 = 1, b = B;
    while (c2 < C2 && b >= c2 + 1) {
        b -= c2 + 1;
        ++c2;
    }
    const int m2 = c2 + 1;
    const int B0 = B - b;                       // first stacked row of this c2
    const bool inA = a < mA;
    const int c1 = inA ? cA : cB;
    const int m1 = c1 + 1;
    const int al = inA ? a : a - mA;            // local x-node
    const int a0 = J.z + (inA ? 0 : mA);        // lane of the first row of this c1

    double Dx[MX], Dy[MX], I2r[FM];
    {
        const double *dx = tab + T_D + doff(m1 - 1) + al * m1;
        const double *dy = tab + T_D + doff(m2 - 1) + b * m2;
        const double *i2 = tab + rt + moff(m2 - 1, F2 - 1) + b * F2;
#pragma unroll
        for (int q = 0; q < MX; ++q) {
            Dx[q] = q < m1 ? dx[q] : 0.0;
            Dy[q] = q < m2 ? dy[q] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < FM; ++j) I2r[j] = j < F2 ? i2[j] : 0.0;
    }
    const double w12 = g.J * tab[T_W + xoff(m1 - 1) + al] * tab[T_W + xoff(m2 - 1) + b];

    // y-interpolated z-lines of both fields
    double XQ[NV][F3], XR[NV][F3];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double *x1 = S + J.w + ((f * NV + v) * rows + a) * X1S;
#pragma unroll
            for (int k = 0; k < F3; ++k) {
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < FM; ++j)
                    if (j < F2) acc += I2r[j] * x1[j + F2 * k];
                if (f == 0) XQ[v][k] = acc; else XR[v][k] = acc;
            }
        }
    }
    __syncthreads();  // X1 is dead; S becomes the flux staging area

    const double invJ = 1.0 / g.J;
    const double Jax = g.Ja[0], Jay = g.Ja[1], Jaz = g.Ja[2];
    const int grp = (inA ? 0 : 1) * CM + (c2 - 1);
    double *Sx = S, *Sy = S + NV * MM * NL;

#pragma unroll
    for (int c3 = 1; c3 <= C3; ++c3) {
        const int m3 = c3 + 1;
        const double *I3 = tab + rt + moff(m3 - 1, F3 - 1);
        const double *D3 = tab + T_D + doff(m3 - 1);
        const double *w3 = tab + T_W + xoff(m3 - 1);
        double V[NV][MM];
#pragma unroll
        for (int c = 0; c < MM; ++c)
#pragma unroll
            for (int v = 0; v < NV; ++v) V[v][c] = 0.0;
#pragma unroll
        for (int cp = 0; cp < MM; ++cp) {
            if (cp >= m3) continue;
            double q[NV], fz[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (SAMPLE && (cp == 0 || cp == m3 - 1)) {
                    q[v] = XQ[v][cp == 0 ? 0 : F3 - 1];
                    continue;
                }
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < F3; ++k) acc += I3[cp * F3 + k] * XQ[v][k];
                q[v] = acc;
            }
            flux_axis(q, 2, gm1, fz);
#pragma unroll
            for (int c = 0; c < MM; ++c) {
                if (c >= m3) continue;
                const double dz = D3[c * m3 + cp];
#pragma unroll
                for (int v = 0; v < NV; ++v) V[v][c] += dz * (Jaz * fz[v]);
            }
            double fx[NV], fy[NV];
            flux_axis(q, 0, gm1, fx);
            flux_axis(q, 1, gm1, fy);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                Sx[(v * MM + cp) * NL + lane] = Jax * fx[v];
                Sy[(v * MM + cp) * NL + lane] = Jay * fy[v];
            }
        }
        __syncthreads();
        if (active) {
#pragma unroll
            for (int q = 0; q < MX; ++q) {
                if (q >= m1) continue;
                const int ln = (a0 + q) + rows * B;
                const double d = Dx[q];
#pragma unroll
                for (int c = 0; c < MM; ++c) {
                    if (c >= m3) continue;
#pragma unroll
                    for (int v = 0; v < NV; ++v) V[v][c] += d * Sx[(v * MM + c) * NL + ln];
                }
            }
#pragma unroll
            for (int q = 0; q < MX; ++q) {
                if (q >= m2) continue;
                const int ln = J.z + a + rows * (B0 + q);
                const double d = Dy[q];
#pragma unroll
                for (int c = 0; c < MM; ++c) {
                    if (c >= m3) continue;
#pragma unroll
                    for (int v = 0; v < NV; ++v) V[v][c] += d * Sy[(v * MM + c) * NL + ln];
                }
            }
            double mx0 = 0.0, mx1 = 0.0;
#pragma unroll
            for (int c = 0; c < MM; ++c) {
                if (c >= m3) continue;
                const double jw = w12 * w3[c];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    double rc = 0.0;
                    if (SAMPLE && (c == 0 || c == m3 - 1)) {
                        rc = XR[v][c == 0 ? 0 : F3 - 1];
                    } else {
#pragma unroll
                        for (int k = 0; k < F3; ++k) rc += I3[c * F3 + k] * XR[v][k];
                    }
                    const double t = V[v][c] * invJ - rc;
                    mx0 = fmax(mx0, fabs(t));
                    mx1 = fmax(mx1, fabs(jw * t));
                }
            }
            unsigned long long *sl = slot + jb * NSL + ((c3 - 1) * 2 * CM + grp) * 2;
            atomicMax(sl, (unsigned long long)__double_as_longlong(mx0));
            atomicMax(sl + 1, (unsigned long long)__double_as_longlong(mx1));
        }
        __syncthreads();
    }
    // every job's maxima
    for (int i = lane; i < W.y * (NSL / 2); i += NL) {
        const int j = i / (NSL / 2), r = i - j * (NSL / 2);
        const int4 Jj = jobs[W.x + j];
        const ElemInfo Ej = el[Jj.x];
        const int C1j = Ej.n[0] > 2 ? Ej.n[0] - 2 : 1, C2j = Ej.n[1] > 2 ? Ej.n[1] - 2 : 1;
        const int cAj = Jj.y + 1, cBrj = C1j - Jj.y;
        const int cBj = cBrj == cAj ? 0 : cBrj;
        const int c3 = r / (2 * CM) + 1, gi = r % (2 * CM);
        const int cc1 = gi < CM ? cAj : cBj;
        const int cc2 = gi % CM + 1;
        if (cc1 == 0 || cc2 > C2j) continue;
        const int64_t sidx_ = P.combo_off[Jj.x] + (cc1 - 1) + C1j * ((cc2 - 1) + C2j * (c3 - 1));
        P.te_new[sidx_] = __longlong_as_double((long long)slot[j * NSL + 2 * r]);
        P.te_trad[sidx_] = __longlong_as_double((long long)slot[j * NSL + 2 * r + 1]);
    }
}

template <int F3>
static hipError_t launch_an(const int4 *wgs, int nwg, const int4 *jobs, const SweepProb &single,
                            const SweepProb *probs, const double *tab, int rt, hipStream_t s) {
    constexpr int C3 = F3 > 2 ? F3 - 2 : 1;
    const size_t lds = sizeof(double) * (size_t)an_stage_doubles(F3) +
                       sizeof(unsigned long long) * AN_JOBS * 2 * C3 * 2 * 6;
    auto go = [&](auto kern) {
        hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(256), lds, s, wgs, nwg, jobs, single, probs, tab, rt);
        return hipGetLastError();
    };
    return rt == T_I ? go(k_sweep_an<F3, true>) : go(k_sweep_an<F3, false>);
}

hipError_t launch_sweep_an(int F3, const int4 *wgs, int nwg, const int4 *jobs, const SweepProb &single,
                           const SweepProb *probs, const double *tab, int restriction, hipStream_t s) {
    if (nwg == 0) return hipSuccess;
    const int rt = restriction ? T_P : T_I;
    switch (F3) {
        case 2: return launch_an<2>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 3: return launch_an<3>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 4: return launch_an<4>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 5: return launch_an<5>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 6: return launch_an<6>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 7: return launch_an<7>(wgs, nwg, jobs, single, probs, tab, rt, s);
        case 8: return launch_an<8>(wgs, nwg, jobs, single, probs, tab, rt, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_iso(int F, const int2 *elems, int nelem, const SweepProb &single, const SweepProb *probs,
                            const double *tab, int restriction, hipStream_t s) {
    if (nelem == 0) return hipSuccess;
    const int rt = restriction ? T_P : T_I;
    switch (F) {
        case 2: return launch_iso<2>(elems, nelem, single, probs, tab, rt, s);
        case 3: return launch_iso<3>(elems, nelem, single, probs, tab, rt, s);
        case 4: return launch_iso<4>(elems, nelem, single, probs, tab, rt, s);
        case 5: return launch_iso<5>(elems, nelem, single, probs, tab, rt, s);
        case 6: return launch_iso<6>(elems, nelem, single, probs, tab, rt, s);
        case 7: return launch_iso<7>(elems, nelem, single, probs, tab, rt, s);
        case 8: return launch_iso<8>(elems, nelem, single, probs, tab, rt, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace dgt
