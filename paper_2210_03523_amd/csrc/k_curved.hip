// Curved elements (Section 2.1: every element mapped onto the reference cube; the
// fluxes are contravariant, Ft^d = Ja^d . f, and J is the Jacobian of the map).
//
//   k_face_curved      : Riemann flux on the mortar with the scaled normal m (the minus
//                        side's Ja^d interpolated onto the mortar nodes, precomputed per
//                        face), F* = |m| [ f*(Q_L, Q_R, m/|m|) - (1/2)(f^v_L + f^v_R).m/|m| ],
//                        projected back onto both faces (the plus side negated).
//   k_face_avg_curved  : BR1 face data of the gradient pass, s P[ qhat m_l ] for l = x, y, z
//                        (the normal multiplied in before the projection).
//   k_elem_grad_curved : J dQ/dx_l = sum_d D_d[(Ja^d)_l Q] + sum_faces (s P[qhat m_l] - Q s (Ja^d)_l)/w_end.
//   k_sweep_curved     : one workgroup per (element, coarse combination) of the isolated
//                        sweep: restriction of Q, dQ/dt and the node coordinates, metric terms
//                        of the coarse element from its coordinates, BR1 gradients (Navier-Stokes),
//                        contravariant fluxes, volume term, tau difference and its maxima.
// The element pass of curved plans is the common element kernel with per-node metric terms.
#include <hip/hip_runtime.h>

#include "common.h"
#include "euler.h"

namespace dgt {

namespace {


__device__ __forceinline__ int face_node_c(const int32_t *n, int d, int side, int a, int b) {
    int idx[3];
    idx[d] = side > 0 ? n[d] - 1 : 0;
    idx[d == 0 ? 1 : 0] = a;
    idx[d == 2 ? 1 : 2] = b;
    return idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
}

template <typename T>
__device__ __forceinline__ T unit_normal(const T m[3], T nh[3]) {
    const T len = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    const T il = T(1) / len;
#pragma unroll
    for (int c = 0; c < 3; ++c) nh[c] = m[c] * il;
    return len;
}

template <typename T>
__device__ __forceinline__ void ghost(const T qin[NV], const T nh[3], int bc, const PhysParams &ph, T qg[NV]) {
    if (bc == 1) {  // slip wall: mirror the normal momentum
        const T mn = qin[1] * nh[0] + qin[2] * nh[1] + qin[3] * nh[2];
        qg[0] = qin[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) qg[1 + k] = qin[1 + k] - T(2) * mn * nh[k];
        qg[4] = qin[4];
    } else {  // far field
#pragma unroll
        for (int v = 0; v < NV; ++v) qg[v] = (T)ph.qfar[v];
    }
}

// Interpolate NF staged trace fields (na x nb, field stride FN) to mortar node (A, B).
template <typename T, int NF, int FN>
__device__ __forceinline__ void to_mortar_node(const T (*S)[FN], int na, int nb, int K1, int K2, int A, int B,
                                               const T *__restrict__ tab, T x[NF]) {
    if (na == K1 && nb == K2) {
#pragma unroll
        for (int c = 0; c < NF; ++c) x[c] = S[c][A + K1 * B];
        return;
    }
    const T *S1 = tab + T_I + moff(K1 - 1, na - 1) + A * na;
    const T *S2 = tab + T_I + moff(K2 - 1, nb - 1) + B * nb;
#pragma unroll
    for (int c = 0; c < NF; ++c) x[c] = T(0);
    for (int b = 0; b < nb; ++b)
        for (int a = 0; a < na; ++a) {
            const T w = S1[a] * S2[b];
#pragma unroll
            for (int c = 0; c < NF; ++c) x[c] += w * S[c][a + na * b];
        }
}

// Project NO mortar fields (field stride FN) back onto face node (a, b) of an na x nb face.
template <typename T, int NO, int FN>
__device__ __forceinline__ void from_mortar_node(const T (*F)[FN], int na, int nb, int K1, int K2, int a, int b,
                                                 const T *__restrict__ tab, T acc[NO]) {
    if (na == K1 && nb == K2) {
#pragma unroll
        for (int c = 0; c < NO; ++c) acc[c] = F[c][a + na * b];
        return;
    }
    const T *P1 = tab + T_P + moff(na - 1, K1 - 1) + a * K1;
    const T *P2 = tab + T_P + moff(nb - 1, K2 - 1) + b * K2;
#pragma unroll
    for (int c = 0; c < NO; ++c) acc[c] = T(0);
    for (int B = 0; B < K2; ++B)
        for (int A = 0; A < K1; ++A) {
            const T w = P1[A] * P2[B];
#pragma unroll
            for (int c = 0; c < NO; ++c) acc[c] += w * F[c][A + K1 * B];
        }
}

}  // namespace

// ---------------------------------------------------------------------------- face flux
// D: the face direction as a compile-time constant (a wave-uniform branch in the kernel),
// so no register array is indexed at run time.
template <typename T, int FN, bool VISC, int D>
__device__ __forceinline__ void face_curved_d(const Face f, const T *__restrict__ mt, const ElemInfo *__restrict__ el,
                                              const T *__restrict__ u, const T *__restrict__ grad,
                                              T *__restrict__ ff, const T *__restrict__ tab, const PhysParams &ph,
                                              T (*sL)[FN], T (*sR)[FN], T (*sF)[FN]) {
    constexpr int NF = VISC ? 4 * NV : NV;  // Q and, for Navier-Stokes, its three gradient components
    constexpr int d = D, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const T gam = (T)ph.gamma, mu = (T)ph.mu, kappa = (T)ph.kappa;
    const int lane = threadIdx.x;
    auto load = [&](const ElemInfo &E, int node, T *x) {
        const int ne = E.n[0] * E.n[1] * E.n[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = u[NV * E.noff + v * ne + node];
        if (VISC) {
#pragma unroll
            for (int c = 0; c < 3 * NV; ++c) x[NV + c] = grad[3 * NV * E.noff + (int64_t)c * ne + node];
        }
    };
    if (f.bc != 0) {
        const int e = f.eL >= 0 ? f.eL : f.eR;
        const int s = f.eL >= 0 ? 1 : -1;
        const ElemInfo E = el[e];
        const int na = E.n[t1], nb = E.n[t2];
        T *out = ff + E.foff + fslot(E.n, d, s);
        for (int m = lane; m < na * nb; m += 64) {
            T x[NF], qg[NV], F[NV], mv[3], nh[3];
            load(E, face_node_c(E.n, d, s, m % na, m / na), x);
#pragma unroll
            for (int c = 0; c < 3; ++c) mv[c] = mt[3 * m + c];
            const T len = unit_normal(mv, nh);
            ghost(x, nh, f.bc, ph, qg);
            numflux_n(x, qg, nh, gam, ph.flux, F);
            if (VISC) {
                T fv1[NV], fv2[NV];
                viscous_n(x, x + NV, nh, gam, mu, kappa, fv1);
                viscous_n(qg, x + NV, nh, gam, mu, kappa, fv2);
#pragma unroll
                for (int v = 0; v < NV; ++v) F[v] -= T(0.5) * (fv1[v] + fv2[v]);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * na * nb + m] = len * F[v];
        }
        return;
    }
    const ElemInfo L = el[f.eL], R = el[f.eR];
    const int aL = L.n[t1], bL = L.n[t2], aR = R.n[t1], bR = R.n[t2];
    const int K1 = aL > aR ? aL : aR, K2 = bL > bR ? bL : bR;
    for (int m = lane; m < aL * bL; m += 64) {
        T x[NF];
        load(L, face_node_c(L.n, d, 1, m % aL, m / aL), x);
#pragma unroll
        for (int c = 0; c < NF; ++c) sL[c][m] = x[c];
    }
    for (int m = lane; m < aR * bR; m += 64) {
        T x[NF];
        load(R, face_node_c(R.n, d, -1, m % aR, m / aR), x);
#pragma unroll
        for (int c = 0; c < NF; ++c) sR[c][m] = x[c];
    }
    __syncthreads();
    for (int m = lane; m < K1 * K2; m += 64) {
        const int A = m % K1, B = m / K1;
        T xl[NF], xr[NF], F[NV], mv[3], nh[3];
        to_mortar_node<T, NF, FN>(sL, aL, bL, K1, K2, A, B, tab, xl);
        to_mortar_node<T, NF, FN>(sR, aR, bR, K1, K2, A, B, tab, xr);
#pragma unroll
        for (int c = 0; c < 3; ++c) mv[c] = mt[3 * m + c];
        const T len = unit_normal(mv, nh);
        numflux_n(xl, xr, nh, gam, ph.flux, F);
        if (VISC) {
            T fvL[NV], fvR[NV];
            viscous_n(xl, xl + NV, nh, gam, mu, kappa, fvL);
            viscous_n(xr, xr + NV, nh, gam, mu, kappa, fvR);
#pragma unroll
            for (int v = 0; v < NV; ++v) F[v] -= T(0.5) * (fvL[v] + fvR[v]);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v][m] = len * F[v];
    }
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const ElemInfo &E = side == 0 ? L : R;
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        const T sg = side == 0 ? T(1) : T(-1);
        T *out = ff + E.foff + fslot(E.n, d, side == 0 ? 1 : -1);
        for (int m = lane; m < na * nb; m += 64) {
            T acc[NV];
            from_mortar_node<T, NV, FN>(sF, na, nb, K1, K2, m % na, m / na, tab, acc);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * na * nb + m] = sg * acc[v];
        }
    }
}

template <typename T, int FN, bool VISC>
__global__ __launch_bounds__(64) void k_face_curved(const Face *__restrict__ faces, const int64_t *__restrict__ fmo,
                                                    const T *__restrict__ fmet, const ElemInfo *__restrict__ el,
                                                    const T *__restrict__ u, const T *__restrict__ grad,
                                                    T *__restrict__ ff, const T *__restrict__ tab, PhysParams ph) {
    constexpr int NF = VISC ? 4 * NV : NV;
    __shared__ T sL[NF][FN], sR[NF][FN], sF[NV][FN];
    const int fi = xcd_remap(blockIdx.x, gridDim.x);  // XCD-contiguous face ranges
    const Face f = faces[fi];
    const T *mt = fmet + 3 * fmo[fi];
    if (f.d == 0) face_curved_d<T, FN, VISC, 0>(f, mt, el, u, grad, ff, tab, ph, sL, sR, sF);
    else if (f.d == 1) face_curved_d<T, FN, VISC, 1>(f, mt, el, u, grad, ff, tab, ph, sL, sR, sF);
    else face_curved_d<T, FN, VISC, 2>(f, mt, el, u, grad, ff, tab, ph, sL, sR, sF);
}

// ---------------------------------------------------------------------------- BR1 face data
// Output per own face node: 15 values (l*NV + v) at 3*E.foff + 3*fslot(E.n, d, s).
template <typename T, int FN, int D>
__device__ __forceinline__ void face_avg_curved_d(const Face f, const T *__restrict__ mt,
                                                  const ElemInfo *__restrict__ el, const T *__restrict__ u,
                                                  T *__restrict__ fq, const T *__restrict__ tab, const PhysParams &ph,
                                                  T (*sL)[FN], T (*sR)[FN], T (*sP)[FN]) {
    constexpr int NP = 3 * NV;
    constexpr int d = D, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int lane = threadIdx.x;
    if (f.bc != 0) {
        const int e = f.eL >= 0 ? f.eL : f.eR;
        const int s = f.eL >= 0 ? 1 : -1;
        const ElemInfo E = el[e];
        const int na = E.n[t1], nb = E.n[t2], ne = E.n[0] * E.n[1] * E.n[2];
        T *out = fq + 3 * (E.foff + fslot(E.n, d, s));
        for (int m = lane; m < na * nb; m += 64) {
            const int node = face_node_c(E.n, d, s, m % na, m / na);
            T qin[NV], qg[NV], mv[3], nh[3];
#pragma unroll
            for (int v = 0; v < NV; ++v) qin[v] = u[NV * E.noff + v * ne + node];
#pragma unroll
            for (int c = 0; c < 3; ++c) mv[c] = mt[3 * m + c];
            unit_normal(mv, nh);
            ghost(qin, nh, f.bc, ph, qg);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const T qh = T(0.5) * (qin[v] + qg[v]);
#pragma unroll
                for (int l = 0; l < 3; ++l) out[(l * NV + v) * na * nb + m] = qh * mv[l];
            }
        }
        return;
    }
    const ElemInfo L = el[f.eL], R = el[f.eR];
    const int aL = L.n[t1], bL = L.n[t2], aR = R.n[t1], bR = R.n[t2];
    const int K1 = aL > aR ? aL : aR, K2 = bL > bR ? bL : bR;
    const int neL = L.n[0] * L.n[1] * L.n[2], neR = R.n[0] * R.n[1] * R.n[2];
    for (int m = lane; m < aL * bL; m += 64) {
        const int node = face_node_c(L.n, d, 1, m % aL, m / aL);
#pragma unroll
        for (int v = 0; v < NV; ++v) sL[v][m] = u[NV * L.noff + v * neL + node];
    }
    for (int m = lane; m < aR * bR; m += 64) {
        const int node = face_node_c(R.n, d, -1, m % aR, m / aR);
#pragma unroll
        for (int v = 0; v < NV; ++v) sR[v][m] = u[NV * R.noff + v * neR + node];
    }
    __syncthreads();
    for (int m = lane; m < K1 * K2; m += 64) {
        const int A = m % K1, B = m / K1;
        T xl[NV], xr[NV];
        to_mortar_node<T, NV, FN>(sL, aL, bL, K1, K2, A, B, tab, xl);
        to_mortar_node<T, NV, FN>(sR, aR, bR, K1, K2, A, B, tab, xr);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const T qh = T(0.5) * (xl[v] + xr[v]);
#pragma unroll
            for (int l = 0; l < 3; ++l) sP[l * NV + v][m] = qh * mt[3 * m + l];
        }
    }
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const ElemInfo &E = side == 0 ? L : R;
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        const T sg = side == 0 ? T(1) : T(-1);
        T *out = fq + 3 * (E.foff + fslot(E.n, d, side == 0 ? 1 : -1));
        for (int m = lane; m < na * nb; m += 64) {
            T acc[NP];
            from_mortar_node<T, NP, FN>(sP, na, nb, K1, K2, m % na, m / na, tab, acc);
#pragma unroll
            for (int c = 0; c < NP; ++c) out[c * na * nb + m] = sg * acc[c];
        }
    }
}

template <typename T, int FN>
__global__ __launch_bounds__(64) void k_face_avg_curved(const Face *__restrict__ faces,
                                                        const int64_t *__restrict__ fmo, const T *__restrict__ fmet,
                                                        const ElemInfo *__restrict__ el, const T *__restrict__ u,
                                                        T *__restrict__ fq, const T *__restrict__ tab, PhysParams ph) {
    __shared__ T sL[NV][FN], sR[NV][FN], sP[3 * NV][FN];
    const int fi = xcd_remap(blockIdx.x, gridDim.x);  // XCD-contiguous face ranges
    const Face f = faces[fi];
    const T *mt = fmet + 3 * fmo[fi];
    if (f.d == 0) face_avg_curved_d<T, FN, 0>(f, mt, el, u, fq, tab, ph, sL, sR, sP);
    else if (f.d == 1) face_avg_curved_d<T, FN, 1>(f, mt, el, u, fq, tab, ph, sL, sR, sP);
    else face_avg_curved_d<T, FN, 2>(f, mt, el, u, fq, tab, ph, sL, sR, sP);
}

// ---------------------------------------------------------------------------- gradient pass
template <typename T, int NPT>
__global__ __launch_bounds__(WG) void k_elem_grad_curved(const Tile *__restrict__ tiles, int tile0, int ntiles,
                                                         const ElemInfo *__restrict__ el, const T *__restrict__ u,
                                                         const T *__restrict__ met, const T *__restrict__ fq,
                                                         T *__restrict__ grad, const T *__restrict__ tab,
                                                         int isolated) {
    __shared__ T sQ[NV][WG * NPT];
    __shared__ T sD[3 * NNMAX * NNMAX];  // the tile's derivative matrices (per-lane rows)
    const int tid = threadIdx.x;
    const Tile tl = tiles[tile0 + blockIdx.x];
    const ElemInfo E0 = el[tl.first];
    const int n1 = E0.n[0], n2 = E0.n[1], n3 = E0.n[2];
    {
        const int ns[3] = {n1, n2, n3};
#pragma unroll
        for (int d = 0; d < 3; ++d)
            for (int t = tid; t < ns[d] * ns[d]; t += WG) sD[d * NNMAX * NNMAX + t] = tab[T_D + doff(ns[d] - 1) + t];
    }
    const int npe = n1 * n2 * n3, total = tl.count * npe;
    const int64_t fblk = fblock(E0.n);
    const int nn[3] = {n1, n2, n3};
    const int stride[3] = {1, n1, n1 * n2};
    T q[NPT][NV], M[NPT][10], G[NPT][3 * NV];
    int loc[NPT][3], le[NPT], nd[NPT];
    bool ok[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int t = tid + k * WG;
        ok[k] = t < total;
        le[k] = ok[k] ? t / npe : 0;
        nd[k] = ok[k] ? t - le[k] * npe : 0;
        loc[k][0] = nd[k] % n1;
        loc[k][1] = (nd[k] / n1) % n2;
        loc[k][2] = nd[k] / (n1 * n2);
        const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le[k] * npe);
        const T *mp = met + (int64_t)10 * (E0.noff + (int64_t)le[k] * npe) + nd[k];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[k][v] = ok[k] ? u[base + v * npe + nd[k]] : T(0);
#pragma unroll
        for (int c = 0; c < 10; ++c) M[k][c] = ok[k] ? mp[(int64_t)c * npe] : T(c == 9 ? 1 : 0);
#pragma unroll
        for (int c = 0; c < 3 * NV; ++c) G[k][c] = T(0);
    }
    // volume part: D_d applied to (Ja^d)_l Q, one (d, l) pair at a time
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                const int t = tid + k * WG;
                if (ok[k]) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) sQ[v][t] = M[k][3 * d + l] * q[k][v];
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < NPT; ++k) {
                if (!ok[k]) continue;
                const int t = tid + k * WG;
                const int id = loc[k][d], nl = nn[d];
                const T *Drow = sD + d * NNMAX * NNMAX + id * nl;
                const int tb = t - id * stride[d];
                for (int m = 0; m < nl; ++m) {
                    const T dm = Drow[m];
#pragma unroll
                    for (int v = 0; v < NV; ++v) G[k][l * NV + v] += dm * sQ[v][tb + m * stride[d]];
                }
            }
            __syncthreads();
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!ok[k]) continue;
        if (!isolated) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int id = loc[k][d], nl = nn[d];
                if (id != 0 && id != nl - 1) continue;
                const int s = id == 0 ? -1 : 1;
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                const int na = nn[t1], nb = nn[t2];
                const T *fs = fq + 3 * (E0.foff + le[k] * fblk + fslot(E0.n, d, s));
                const int fm = loc[k][t1] + na * loc[k][t2];
                const T iw = T(1) / tab[T_W + xoff(nl - 1)];
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const T ml = T(s) * M[k][3 * d + l];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        G[k][l * NV + v] += (fs[(l * NV + v) * na * nb + fm] - q[k][v] * ml) * iw;
                }
            }
        }
        const T iJ = T(1) / M[k][9];
        T *Gp = grad + (int64_t)3 * NV * (E0.noff + (int64_t)le[k] * npe) + nd[k];
#pragma unroll
        for (int c = 0; c < 3 * NV; ++c) Gp[(int64_t)c * npe] = G[k][c] * iJ;
    }
}

template <typename T>
hipError_t launch_face_curved(const Face *faces, const int64_t *fmo, const T *fmet, int nfaces, const ElemInfo *el,
                              const T *u, const T *grad, T *ff, const T *tab, PhysParams ph, int max_order,
                              hipStream_t s) {
    if (nfaces == 0) return hipSuccess;
    const bool visc = grad != nullptr;
    if (max_order <= 7) {
        if (visc)
            hipLaunchKernelGGL((k_face_curved<T, 64, true>), dim3(nfaces), dim3(64), 0, s, faces, fmo, fmet, el, u,
                               grad, ff, tab, ph);
        else
            hipLaunchKernelGGL((k_face_curved<T, 64, false>), dim3(nfaces), dim3(64), 0, s, faces, fmo, fmet, el, u,
                               grad, ff, tab, ph);
    } else {
        if (visc) return hipErrorInvalidValue;  // Navier-Stokes plans hold orders up to 7
        hipLaunchKernelGGL((k_face_curved<T, 100, false>), dim3(nfaces), dim3(64), 0, s, faces, fmo, fmet, el, u,
                           grad, ff, tab, ph);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_grad_curved(const Face *faces, const int64_t *fmo, const T *fmet, int nfaces, const Tile *tiles,
                              int tile0, int ntiles, int npt, bool do_faces, const ElemInfo *el, const T *u,
                              const T *met, T *fq, T *grad, const T *tab, PhysParams ph, int isolated,
                              hipStream_t s) {
    if (do_faces && !isolated && nfaces > 0)
        hipLaunchKernelGGL((k_face_avg_curved<T, 64>), dim3(nfaces), dim3(64), 0, s, faces, fmo, fmet, el, u, fq, tab,
                           ph);
    if (ntiles == 0) return hipGetLastError();
    switch (npt) {
        case 1: hipLaunchKernelGGL((k_elem_grad_curved<T, 1>), dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, met, fq, grad, tab, isolated); break;
        case 2: hipLaunchKernelGGL((k_elem_grad_curved<T, 2>), dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, met, fq, grad, tab, isolated); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_face_curved<double>(const Face *, const int64_t *, const double *, int, const ElemInfo *,
                                               const double *, const double *, double *, const double *, PhysParams,
                                               int, hipStream_t);
template hipError_t launch_face_curved<float>(const Face *, const int64_t *, const float *, int, const ElemInfo *,
                                              const float *, const float *, float *, const float *, PhysParams, int,
                                              hipStream_t);
template hipError_t launch_grad_curved<double>(const Face *, const int64_t *, const double *, int, const Tile *, int,
                                               int, int, bool, const ElemInfo *, const double *, const double *,
                                               double *, double *, const double *, PhysParams, int, hipStream_t);
template hipError_t launch_grad_curved<float>(const Face *, const int64_t *, const float *, int, const Tile *, int,
                                              int, int, bool, const ElemInfo *, const float *, const float *, float *,
                                              float *, const float *, PhysParams, int, hipStream_t);

// ---------------------------------------------------------------------------- sweep
// One workgroup per task (fine plan element p, coarse orders c1, c2, c3).  LDS holds
//   A: [13][m1][f2][f3] after the x-restriction, later the coarse fields [13][nc]
//      (Q, dQ/dt, node coordinates);
//   B: [13][m1][m2][f3] after the y-restriction, later the coarse metric terms [10][nc];
//   S: [15][nc] staging of products and contravariant fluxes (and of the reduction).
constexpr int NFLD = NFLD_SWEEP;

template <int BS, int NPT>
__global__ __launch_bounds__(BS) void k_sweep_curved(const int4 *__restrict__ tasks, const ElemInfo *__restrict__ el,
                                                     const int64_t *__restrict__ combo_off,
                                                     const double *__restrict__ u, const double *__restrict__ dudt,
                                                     const double *__restrict__ xyz, const double *__restrict__ tab,
                                                     PhysParams ph, int capA, int capB, int viscous, int rt,
                                                     double *__restrict__ te_new, double *__restrict__ te_trad) {
    extern __shared__ double lds[];
    double *A = lds, *B = lds + capA, *S = lds + capA + capB;
    const int4 tk = tasks[blockIdx.x];
    const ElemInfo E = el[tk.x];
    const int f1 = E.n[0], f2 = E.n[1], f3 = E.n[2], nf = f1 * f2 * f3;
    const int c[3] = {tk.y, tk.z, tk.w};
    const int m1 = c[0] + 1, m2 = c[1] + 1, m3 = c[2] + 1, nc = m1 * m2 * m3;
    const int mm[3] = {m1, m2, m3};
    const int tid = threadIdx.x;
    const double gam = ph.gamma, gm1 = gam - 1.0, mu = ph.mu, kappa = ph.kappa;
    auto field = [&](int fld) -> const double * {
        if (fld < NV) return u + NV * E.noff + (int64_t)fld * nf;
        if (fld < 2 * NV) return dudt + NV * E.noff + (int64_t)(fld - NV) * nf;
        return xyz + 3 * E.noff + (int64_t)(fld - 2 * NV) * nf;
    };
    // restriction, one direction at a time: Q and dQ/dt by the estimate's operator (sampling
    // at the coarse nodes or L2 projection), the node coordinates always by sampling
    {
        const double *I1 = tab + T_I + moff(c[0], f1 - 1), *R1 = tab + rt + moff(c[0], f1 - 1);
        for (int r = tid; r < NFLD * m1 * f2 * f3; r += BS) {
            const int a = r % m1, jk = (r / m1) % (f2 * f3), fld = r / (m1 * f2 * f3);
            const double *src = field(fld) + (int64_t)jk * f1;
            const double *w = (fld < 2 * NV ? R1 : I1) + a * f1;
            double acc = 0.0;
            for (int i = 0; i < f1; ++i) acc += w[i] * src[i];
            A[r] = acc;  // [fld][jk][a]
        }
    }
    __syncthreads();
    {
        const double *I2 = tab + T_I + moff(c[1], f2 - 1), *R2 = tab + rt + moff(c[1], f2 - 1);
        for (int r = tid; r < NFLD * m1 * m2 * f3; r += BS) {
            const int a = r % m1, b = (r / m1) % m2, k = (r / (m1 * m2)) % f3, fld = r / (m1 * m2 * f3);
            const double *w = (fld < 2 * NV ? R2 : I2) + b * f2;
            double acc = 0.0;
            for (int j = 0; j < f2; ++j) acc += w[j] * A[((fld * f3 + k) * f2 + j) * m1 + a];
            B[r] = acc;  // [fld][k][b][a]
        }
    }
    __syncthreads();
    {
        const double *I3 = tab + T_I + moff(c[2], f3 - 1), *R3 = tab + rt + moff(c[2], f3 - 1);
        for (int r = tid; r < NFLD * nc; r += BS) {
            const int ab = r % (m1 * m2), cc = (r / (m1 * m2)) % m3, fld = r / nc;
            const double *w = (fld < 2 * NV ? R3 : I3) + cc * f3;
            double acc = 0.0;
            for (int k = 0; k < f3; ++k) acc += w[k] * B[(fld * f3 + k) * m1 * m2 + ab];
            A[r] = acc;  // coarse fields [fld][node], node = a + m1 (b + m2 cc)
        }
    }
    __syncthreads();
    const double *Dm[3] = {tab + T_D + doff(c[0]), tab + T_D + doff(c[1]), tab + T_D + doff(c[2])};
    const int stride[3] = {1, m1, m1 * m2};
    // metric terms of the coarse element from its coordinates (cross-product form)
    for (int t = tid; t < nc; t += BS) {
        const int idx[3] = {t % m1, (t / m1) % m2, t / (m1 * m2)};
        double a[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double *Drow = Dm[r] + idx[r] * mm[r];
            const int tb = t - idx[r] * stride[r];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                double acc = 0.0;
                for (int q = 0; q < mm[r]; ++q) acc += Drow[q] * A[(2 * NV + cc) * nc + tb + q * stride[r]];
                a[r][cc] = acc;
            }
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *p = a[(d + 1) % 3], *q = a[(d + 2) % 3];
            B[(3 * d + 0) * nc + t] = p[1] * q[2] - p[2] * q[1];
            B[(3 * d + 1) * nc + t] = p[2] * q[0] - p[0] * q[2];
            B[(3 * d + 2) * nc + t] = p[0] * q[1] - p[1] * q[0];
        }
        B[9 * nc + t] = a[0][0] * B[0 * nc + t] + a[0][1] * B[1 * nc + t] + a[0][2] * B[2 * nc + t];
    }
    __syncthreads();
    // at most NPT coarse nodes per thread (nc <= NPT * BS)
    double G[NPT][3 * NV], V[NPT][NV];
#pragma unroll
    for (int k = 0; k < NPT; ++k)
#pragma unroll
        for (int x = 0; x < 3 * NV; ++x) G[k][x] = 0.0;
    if (viscous) {
        // isolated BR1 gradient: J dQ/dx_l = sum_d D_d[(Ja^d)_l Q]
        for (int d = 0; d < 3; ++d)
            for (int l = 0; l < 3; ++l) {
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    const int t = tid + k * BS;
                    if (t < nc)
#pragma unroll
                        for (int v = 0; v < NV; ++v) S[v * nc + t] = B[(3 * d + l) * nc + t] * A[v * nc + t];
                }
                __syncthreads();
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    const int t = tid + k * BS;
                    if (t >= nc) continue;
                    const int id = d == 0 ? t % m1 : (d == 1 ? (t / m1) % m2 : t / (m1 * m2));
                    const double *Drow = Dm[d] + id * mm[d];
                    const int tb = t - id * stride[d];
                    for (int q = 0; q < mm[d]; ++q)
#pragma unroll
                        for (int v = 0; v < NV; ++v) G[k][l * NV + v] += Drow[q] * S[v * nc + tb + q * stride[d]];
                }
                __syncthreads();
            }
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int t = tid + k * BS;
            if (t >= nc) continue;
            const double iJ = 1.0 / B[9 * nc + t];
#pragma unroll
            for (int x = 0; x < 3 * NV; ++x) G[k][x] *= iJ;
        }
    }
    // contravariant fluxes Ja^d . (f^a - f^v), staged for all three directions
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int t = tid + k * BS;
#pragma unroll
        for (int v = 0; v < NV; ++v) V[k][v] = 0.0;
        if (t >= nc) continue;
        double q[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) q[v] = A[v * nc + t];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double n[3] = {B[(3 * d) * nc + t], B[(3 * d + 1) * nc + t], B[(3 * d + 2) * nc + t]};
            double f[NV];
            flux_n(q, n, gm1, f);
            if (viscous) {
                double fv[NV];
                viscous_n(q, G[k], n, gam, mu, kappa, fv);
#pragma unroll
                for (int v = 0; v < NV; ++v) f[v] -= fv[v];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) S[(d * NV + v) * nc + t] = f[v];
        }
    }
    __syncthreads();
    double mx0 = 0.0, mx1 = 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int t = tid + k * BS;
        if (t >= nc) continue;
        const int idx[3] = {t % m1, (t / m1) % m2, t / (m1 * m2)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double *Drow = Dm[d] + idx[d] * mm[d];
            const int tb = t - idx[d] * stride[d];
            for (int q = 0; q < mm[d]; ++q)
#pragma unroll
                for (int v = 0; v < NV; ++v) V[k][v] += Drow[q] * S[(d * NV + v) * nc + tb + q * stride[d]];
        }
        const double J = B[9 * nc + t];
        const double www = tab[T_W + xoff(c[0]) + idx[0]] * tab[T_W + xoff(c[1]) + idx[1]] *
                           tab[T_W + xoff(c[2]) + idx[2]];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double a = V[k][v] / J - A[(NV + v) * nc + t];
            mx0 = fmax(mx0, fabs(a));
            mx1 = fmax(mx1, fabs(J * www * a));
        }
    }
    // workgroup maxima
    __syncthreads();
    S[tid] = mx0;
    S[BS + tid] = mx1;
    __syncthreads();
    for (int h = BS / 2; h > 0; h >>= 1) {
        if (tid < h) {
            S[tid] = fmax(S[tid], S[tid + h]);
            S[BS + tid] = fmax(S[BS + tid], S[BS + tid + h]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int C1 = E.n[0] > 2 ? E.n[0] - 2 : 1, C2 = E.n[1] > 2 ? E.n[1] - 2 : 1;
        const int64_t slot = combo_off[tk.x] + (c[0] - 1) + (int64_t)C1 * ((c[1] - 1) + (int64_t)C2 * (c[2] - 1));
        te_new[slot] = S[0];
        te_trad[slot] = S[BS];
    }
}

// Workgroup shape from the largest combination: 128 lanes x 1 node up to 128 coarse
// nodes, 256 x 1 up to 256, 256 x 2 up to 512 (the sweep's fine orders are at most 7).
template <int BS, int NPT>
static hipError_t launch_sweep_curved_bs(const int4 *tasks, int ntasks, const ElemInfo *el, const int64_t *combo_off,
                                         const double *u, const double *dudt, const double *xyz, const double *tab,
                                         PhysParams ph, int capA, int capB, int capS, int viscous, int rt,
                                         double *te_new, double *te_trad, hipStream_t s) {
    const size_t lds = sizeof(double) * (size_t)(capA + capB + capS);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void *)k_sweep_curved<BS, NPT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_sweep_curved<BS, NPT>), dim3(ntasks), dim3(BS), lds, s, tasks, el, combo_off, u, dudt, xyz,
                       tab, ph, capA, capB, viscous, rt, te_new, te_trad);
    return hipGetLastError();
}

hipError_t launch_sweep_curved(const int4 *tasks, int ntasks, const ElemInfo *el, const int64_t *combo_off,
                               const double *u, const double *dudt, const double *xyz, const double *tab,
                               PhysParams ph, int capA, int capB, int capS, int max_nc, int viscous, int restriction,
                               double *te_new, double *te_trad, hipStream_t s) {
    if (ntasks == 0) return hipSuccess;
    const int rt = restriction ? T_P : T_I;
    if (capS < 2 * WG) return hipErrorInvalidValue;  // the maxima reduction stages 2 BS values
    if (max_nc <= 128)
        return launch_sweep_curved_bs<128, 1>(tasks, ntasks, el, combo_off, u, dudt, xyz, tab, ph, capA, capB, capS,
                                              viscous, rt, te_new, te_trad, s);
    if (max_nc <= 256)
        return launch_sweep_curved_bs<256, 1>(tasks, ntasks, el, combo_off, u, dudt, xyz, tab, ph, capA, capB, capS,
                                              viscous, rt, te_new, te_trad, s);
    if (max_nc <= 512)
        return launch_sweep_curved_bs<256, 2>(tasks, ntasks, el, combo_off, u, dudt, xyz, tab, ph, capA, capB, capS,
                                              viscous, rt, te_new, te_trad, s);
    return hipErrorInvalidValue;
}

}  // namespace dgt
