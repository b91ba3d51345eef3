// DGSEM residual kernels for gfx950 (Section 2.1, strong form on Gauss-Lobatto nodes):
//
//   J dQ/dt = -( sum_d D_d Ft^d + SAT ),  Ft^d = |Ja^d| f_d(Q),
//   SAT(face node of face (d,s)) = (F*_out - s Ft^d) / w_end.
//
// Two passes:
//   k_face  : one wavefront per face.  Gathers both traces, interpolates them onto
//             the mortar (K = max order per tangential direction) when the orders
//             differ, evaluates the Riemann flux once in the canonical orientation
//             (left = minus side, normal +e_d), projects it back onto both faces
//             (L2 projection; the plus side takes the minus sign) and stores the
//             outward fluxes F*_out into per-element face slots.
//   k_elem  : one workgroup per tile (consecutive plan elements with identical
//             orders).  Loads Q once, stages the directional fluxes through LDS,
//             applies the 1D derivative matrices (sum factorisation), adds the
//             lifted surface terms and finishes with an epilogue: the residual in
//             new or traditional form, a fused low-storage RK3 stage, or the
//             tau difference of the estimate with per-element maxima.
#include <hip/hip_runtime.h>

#include "common.h"
#include "euler.h"

namespace dgt {

__device__ __forceinline__ int face_node(const int32_t *n, int d, int side, int a, int b) {
    int idx[3];
    idx[d] = side > 0 ? n[d] - 1 : 0;
    idx[d == 0 ? 1 : 0] = a;
    idx[d == 2 ? 1 : 2] = b;
    return idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
}

// ---------------------------------------------------------------------------- faces
// FN = largest number of nodes of a face (and of a mortar) the launch may meet:
// 64 for orders up to 7, 100 up to 9.  It sizes the LDS staging and so the number
// of faces resident per CU.
template <typename T, int FN>
struct FaceSmem {
    // FP32 faces stage their mortar operators (S1, S2, P1, P2 of each side) in LDS; FP64
    // ones read them through the cache (their larger LDS would cost occupancy)
    static constexpr int OPS = sizeof(T) == 4 ? 8 : 1;
    T QL[NV][FN];   // left trace, later the left projection intermediate
    T QR[NV][FN];   // right trace, later the right projection intermediate
    T TL[NV][FN];   // left trace interpolated along the first tangential direction
    T TR[NV][FN];
    T F[NV][FN];    // Riemann flux on the mortar
    T op[OPS][FN];  // [side]: S1; [2 + side]: S2; [4 + side]: P1; [6 + side]: P2
};

// One face, processed by one wavefront (64 lanes).  Mortar interpolation S2 (x) S1 and
// projection P2 (x) P1 are applied one tangential direction at a time, and only in a
// direction where the two sides' orders differ.
// m = a + n b split into (a, b) for m < 2^20 and n <= 1000 through the float reciprocal
// of n (the exact quotient of m + 1/2 sits at least 1/(2n) from an integer, far beyond
// the rounding): the face loops split their lane index this way instead of by integer
// division, which takes tens of instructions.
__device__ __forceinline__ void split2(int m, int n, float inv, int &a, int &b) {
    b = (int)(((float)m + 0.5f) * inv);
    a = m - b * n;
}

// MODE 0: outward Riemann flux F*_out (plus side negated).  MODE 1: the BR1 trace of the
// solution, (Q_L + Q_R)/2 on the mortar projected back onto both sides (no sign, no
// metric), the face input of the gradient pass.
// D: the face direction as a compile-time constant (see face_body below).
// L, R: the elements of the two sides (a boundary face passes its one element in both).
// UP, FP: pointer types of the state and the face fluxes (generic, or in the global
// address space where the pointers come from a descriptor in memory: the compiler cannot
// tell their address space then and would issue flat accesses, which also count against
// the LDS wait counter and need 64-bit address arithmetic per access).
template <typename T, int FN, int MODE, int D, typename UP, typename FP>
__device__ __forceinline__ void face_body_d(const Face f, const ElemInfo &L, const ElemInfo &R, UP __restrict__ u,
                                            FP __restrict__ ff, const T *__restrict__ tab, const Geom &g,
                                            const PhysParams &ph, FaceSmem<T, FN> &sm) {
    constexpr int d = D, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const T Ja = (T)g.Ja[d];
    const T gam = (T)ph.gamma;
    const int lane = threadIdx.x;

    if (f.bc != 0) {
        const int s = f.eL >= 0 ? 1 : -1;
        const ElemInfo &E = f.eL >= 0 ? L : R;
        const int na = E.n[t1], nb = E.n[t2], ne = E.n[0] * E.n[1] * E.n[2];
        const UP Q = u + NV * E.noff;
        const FP out = ff + E.foff + fslot(E.n, d, s);
        const float ina = 1.0f / na;
        for (int m = lane; m < na * nb; m += 64) {
            int ma, mb;
            split2(m, na, ina, ma, mb);
            int node = face_node(E.n, d, s, ma, mb);
            T qin[NV], qg[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) qin[v] = Q[v * ne + node];
            if (f.bc == 1) {  // slip wall: mirror the normal momentum
#pragma unroll
                for (int v = 0; v < NV; ++v) qg[v] = qin[v];
                qg[1 + d] = -qin[1 + d];
            } else {  // far field
#pragma unroll
                for (int v = 0; v < NV; ++v) qg[v] = (T)ph.qfar[v];
            }
            if (MODE == 0) {
                numflux_axis(qin, qg, d, (T)s, gam, ph.flux, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) out[v * na * nb + m] = Ja * F[v];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) out[v * na * nb + m] = T(0.5) * (qin[v] + qg[v]);
            }
        }
        return;
    }

    const int aL = L.n[t1], bL = L.n[t2], aR = R.n[t1], bR = R.n[t2];
    const int K1 = aL > aR ? aL : aR, K2 = bL > bR ? bL : bR;
    const float iaL = 1.0f / aL, iaR = 1.0f / aR, iK1 = 1.0f / K1;
    const int neL = L.n[0] * L.n[1] * L.n[2], neR = R.n[0] * R.n[1] * R.n[2];
    const FP oL = ff + L.foff + fslot(L.n, d, 1);
    const FP oR = ff + R.foff + fslot(R.n, d, -1);

    if (aL == aR && bL == bR) {
        // conforming face: one node pair per lane, no staging
        for (int m = lane; m < aL * bL; m += 64) {
            int ma, mb;
            split2(m, aL, iaL, ma, mb);
            const int nl = face_node(L.n, d, 1, ma, mb);
            const int nr = face_node(R.n, d, -1, ma, mb);
            T qL[NV], qR[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                qL[v] = u[NV * L.noff + v * neL + nl];
                qR[v] = u[NV * R.noff + v * neR + nr];
            }
            if (MODE == 0) {
                numflux_axis(qL, qR, d, T(1), gam, ph.flux, F);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    oL[v * aL * bL + m] = Ja * F[v];
                    oR[v * aL * bL + m] = -Ja * F[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T h = T(0.5) * (qL[v] + qR[v]);
                    oL[v * aL * bL + m] = h;
                    oR[v * aL * bL + m] = h;
                }
            }
        }
        return;
    }

    for (int m = lane; m < aL * bL; m += 64) {
        int ma, mb;
        split2(m, aL, iaL, ma, mb);
        int node = face_node(L.n, d, 1, ma, mb);
#pragma unroll
        for (int v = 0; v < NV; ++v) sm.QL[v][m] = u[NV * L.noff + v * neL + node];
    }
    for (int m = lane; m < aR * bR; m += 64) {
        int ma, mb;
        split2(m, aR, iaR, ma, mb);
        int node = face_node(R.n, d, -1, ma, mb);
#pragma unroll
        for (int v = 0; v < NV; ++v) sm.QR[v][m] = u[NV * R.noff + v * neR + node];
    }
    const bool stage = FaceSmem<T, FN>::OPS == 8;
    if (stage) {
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
            if (na != K1) {
                const T *s1 = tab + T_I + moff(K1 - 1, na - 1), *p1 = tab + T_P + moff(na - 1, K1 - 1);
                for (int t = lane; t < K1 * na; t += 64) {
                    sm.op[side][t] = s1[t];
                    sm.op[4 + side][t] = p1[t];
                }
            }
            if (nb != K2) {
                const T *s2 = tab + T_I + moff(K2 - 1, nb - 1), *p2 = tab + T_P + moff(nb - 1, K2 - 1);
                for (int t = lane; t < K2 * nb; t += 64) {
                    sm.op[2 + side][t] = s2[t];
                    sm.op[6 + side][t] = p2[t];
                }
            }
        }
    }
    __syncthreads();
    // first tangential direction: T[A + K1 b] = sum_a S1[A][a] Q[a + na b]
    for (int side = 0; side < 2; ++side) {
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        if (na == K1) continue;
        T(*Q)[FN] = side == 0 ? sm.QL : sm.QR;
        T(*Tt)[FN] = side == 0 ? sm.TL : sm.TR;
        const T *S1 = stage ? sm.op[side & (FaceSmem<T, FN>::OPS - 1)] : tab + T_I + moff(K1 - 1, na - 1);
        for (int m = lane; m < K1 * nb; m += 64) {
            int A, b;
            split2(m, K1, iK1, A, b);
            T acc[NV] = {T(0), T(0), T(0), T(0), T(0)};
            for (int a = 0; a < na; ++a) {
                const T s1 = S1[A * na + a];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] += s1 * Q[v][a + na * b];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) Tt[v][m] = acc[v];
        }
    }
    __syncthreads();
    // second tangential direction, then the Riemann flux on the mortar
    for (int m = lane; m < K1 * K2; m += 64) {
        int A, B;
        split2(m, K1, iK1, A, B);
        T q[2][NV], F[NV];
        for (int side = 0; side < 2; ++side) {
            const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
            T(*src)[FN] = na == K1 ? (side == 0 ? sm.QL : sm.QR) : (side == 0 ? sm.TL : sm.TR);
            if (nb == K2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) q[side][v] = src[v][A + K1 * B];
            } else {
                const T *S2 = (stage ? sm.op[(2 + side) & (FaceSmem<T, FN>::OPS - 1)]
                                     : tab + T_I + moff(K2 - 1, nb - 1)) + B * nb;
                T acc[NV] = {T(0), T(0), T(0), T(0), T(0)};
                for (int b = 0; b < nb; ++b) {
                    const T s2 = S2[b];
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[v] += s2 * src[v][A + K1 * b];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) q[side][v] = acc[v];
            }
        }
        if (MODE == 0) {
            numflux_axis(q[0], q[1], d, T(1), gam, ph.flux, F);
#pragma unroll
            for (int v = 0; v < NV; ++v) sm.F[v][m] = Ja * F[v];
        } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) sm.F[v][m] = T(0.5) * (q[0][v] + q[1][v]);
        }
    }
    __syncthreads();
    // projection, first tangential direction: U[a + na B] = sum_A P1[a][A] F[A + K1 B]
    for (int side = 0; side < 2; ++side) {
        const int na = side == 0 ? aL : aR;
        if (na == K1) continue;
        T(*U)[FN] = side == 0 ? sm.QL : sm.QR;
        const T *P1 = stage ? sm.op[(4 + side) & (FaceSmem<T, FN>::OPS - 1)] : tab + T_P + moff(na - 1, K1 - 1);
        for (int m = lane; m < na * K2; m += 64) {
            int a, B;
            split2(m, na, 1.0f / na, a, B);
            T acc[NV] = {T(0), T(0), T(0), T(0), T(0)};
            for (int A = 0; A < K1; ++A) {
                const T p1 = P1[a * K1 + A];
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] += p1 * sm.F[v][A + K1 * B];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) U[v][m] = acc[v];
        }
    }
    __syncthreads();
    // second tangential direction, outward sign (+ for L, - for R)
    for (int side = 0; side < 2; ++side) {
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        const FP out = side == 0 ? oL : oR;
        const T sg = (side == 0 || MODE == 1) ? T(1) : T(-1);
        const bool x1 = na != K1;  // the first pass ran: intermediate in QL/QR as [a + na B]
        T(*U)[FN] = x1 ? (side == 0 ? sm.QL : sm.QR) : sm.F;
        const int ld = x1 ? na : K1;
        const T *P2 = stage ? sm.op[(6 + side) & (FaceSmem<T, FN>::OPS - 1)] : tab + T_P + moff(nb - 1, K2 - 1);
        for (int m = lane; m < na * nb; m += 64) {
            int a, b;
            split2(m, na, 1.0f / na, a, b);
            T acc[NV];
            if (nb == K2) {
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = U[v][a + ld * b];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = T(0);
                for (int B = 0; B < K2; ++B) {
                    const T p2 = P2[b * K2 + B];
#pragma unroll
                    for (int v = 0; v < NV; ++v) acc[v] += p2 * U[v][a + ld * B];
                }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * na * nb + m] = sg * acc[v];
        }
    }
}

// The face direction selects register-array elements all through the face body; it is
// made a compile-time constant by a wave-uniform branch, so nothing is indexed at run
// time (which would put the arrays in scratch memory).
template <typename T, int FN, int MODE = 0, typename UP = const T *, typename FP = T *>
__device__ __forceinline__ void face_body(const Face f, const ElemInfo &L, const ElemInfo &R, UP u, FP ff,
                                          const T *__restrict__ tab, const Geom &g, const PhysParams &ph,
                                          FaceSmem<T, FN> &sm) {
    if (f.d == 0) face_body_d<T, FN, MODE, 0>(f, L, R, u, ff, tab, g, ph, sm);
    else if (f.d == 1) face_body_d<T, FN, MODE, 1>(f, L, R, u, ff, tab, g, ph, sm);
    else face_body_d<T, FN, MODE, 2>(f, L, R, u, ff, tab, g, ph, sm);
}

// The two sides' elements of a face (a boundary face's one element twice), loaded side
// by side rather than one after the other.
__device__ __forceinline__ void face_elems(const Face &f, const ElemInfo *__restrict__ el, ElemInfo &L,
                                           ElemInfo &R) {
    L = el[f.eL >= 0 ? f.eL : f.eR];
    R = el[f.eR >= 0 ? f.eR : f.eL];
}

template <typename T, int FN>
__global__ __launch_bounds__(64) void k_face(const Face *__restrict__ faces, const ElemInfo *__restrict__ el,
                                             const T *__restrict__ u, T *__restrict__ ff,
                                             const T *__restrict__ tab, Geom g, PhysParams ph) {
    __shared__ FaceSmem<T, FN> sm;
    // XCD-contiguous face ranges: both sides' element blocks stay in one L2
    const Face f = faces[xcd_remap(blockIdx.x, gridDim.x)];
    ElemInfo L, R;
    face_elems(f, el, L, R);
    face_body<T, FN>(f, L, R, u, ff, tab, g, ph, sm);
}

template <typename T>
hipError_t launch_face_flux(const Face *faces, int nfaces, const ElemInfo *elems, const T *u, T *fflux,
                            const T *tab, Geom g, PhysParams ph, int max_order, hipStream_t s) {
    if (nfaces == 0) return hipSuccess;
    if (max_order <= 7)
        hipLaunchKernelGGL((k_face<T, 64>), dim3(nfaces), dim3(64), 0, s, faces, elems, u, fflux, tab, g, ph);
    else
        hipLaunchKernelGGL((k_face<T, 100>), dim3(nfaces), dim3(64), 0, s, faces, elems, u, fflux, tab, g, ph);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- elements
// One tile of elements, processed by one workgroup of BS lanes (NPT nodes per lane).
// u is not __restrict__: the RK epilogue writes the stage update in place.
// CURVED: per-node metric terms (epi.met), contravariant fluxes Ja^d . f and per-node J.
// VISC: Navier-Stokes (gradients in epi.grad); the Euler instances carry no viscous registers.
// sD (LDS, 3 NNMAX^2): the tile's derivative matrices, staged so that the per-lane rows are
// read from LDS rather than through vector memory loads.
// E0: the descriptor of the tile's first element (every element of a tile has its orders).
// sF: elem_rows<T, BS * NPT>() rows of elem_cols<T>(BS * NPT) values.  With three flux
// sets of rows the fluxes of all three directions are staged at once, behind one barrier;
// with one set the directions take turns (tiles too large for 64 KB of LDS).
// FP64 flux rows hold a node's value at sidx(node) = node + node / 32, one pad slot per
// 32 values, so that the x-derivative's reads (eight rows of 8 doubles, one address per
// row) do not fall two to a bank; FP32 rows are unpadded (measured: 96.6 against 103.9 us
// for the FP64 residual of 16^3 elements at N = 7, FP32 faster without the pad).  The
// derivative matrices sit in LDS with rows of odd stride dstride(n) for the same reason.
template <typename T>
__device__ __forceinline__ int sidx(int t) {
    return sizeof(T) == 8 ? t + (t >> 5) : t;
}
template <typename T>
constexpr int elem_cols(int N) {
    return sizeof(T) == 8 ? N + N / 32 : N;
}
constexpr int DSTR = NNMAX * (NNMAX + 1);  // per direction
__device__ __forceinline__ int dstride(int n) { return n | 1; }
template <typename T, int N>
constexpr int elem_rows() {
    return (3 * NV * elem_cols<T>(N) + 3 * DSTR) * (int)sizeof(T) <= 64 * 1024 ? 3 * NV : NV;
}

// What the element body reads from global memory for its nodes before any work (the
// EARLY form, box Euler elements): the state, the face fluxes of the node's faces and
// the RK register.  A persistent loop requests them for the next tile before the
// current tile's work, so their latency overlaps it.
template <typename T, int NPT>
struct ElemPre {
    T q[NPT][NV];
    T fe[NPT][3][NV];
    T ge[NPT][NV];
};

template <typename T, int NPT, int BS>
__device__ __forceinline__ void elem_preload(const Tile tl, const ElemInfo E0, const T *u, const T *__restrict__ ff,
                                             const EpiArgs &epi, ElemPre<T, NPT> &P) {
    const int tid = threadIdx.x;
    const int n1 = E0.n[0], n2 = E0.n[1], n3 = E0.n[2];
    const int npe = n1 * n2 * n3, total = tl.count * npe;
    const int64_t fblk = fblock(E0.n);
    const bool rk = epi.mode == EPI_RK && epi.rkA != 0.0;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int t = tid + k * BS;
        const bool ok = t < total;
        const int le = ok ? t / npe : 0, nd = ok ? t - le * npe : 0;
        const int loc[3] = {nd % n1, (nd / n1) % n2, nd / (n1 * n2)};
        const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le * npe);
#pragma unroll
        for (int v = 0; v < NV; ++v) P.q[k][v] = ok ? ((const gmem<T> *)u)[base + v * npe + nd] : T(1);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = loc[d], nd_ = d == 0 ? n1 : d == 1 ? n2 : n3;
            const bool on = ok && !epi.isolated && (id == 0 || id == nd_ - 1);
            const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
            const int na = t1 == 0 ? n1 : n2;
            const int ab = (d == 0 ? n2 * n3 : d == 1 ? n1 * n3 : n1 * n2);
            const gmem<T> *fp =
                (const gmem<T> *)ff + E0.foff + le * fblk + fslot(E0.n, d, id == 0 ? -1 : 1) + loc[t1] + na * loc[t2];
#pragma unroll
            for (int v = 0; v < NV; ++v) P.fe[k][d][v] = on ? fp[v * ab] : T(0);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) P.ge[k][v] = (ok && rk) ? ((const gmem<T> *)epi.g)[base + v * npe + nd] : T(0);
    }
}

// Workgroup barrier of the element body.  LDS_ONLY: the wave's own LDS accesses are
// completed (lgkmcnt) and the compiler keeps memory accesses on their side of it, but
// vector-memory loads in flight -- the next tile's, requested before this tile's work --
// are not waited for, as the full barrier's memory fence would; the body shares nothing
// between lanes through global memory.
template <bool LDS_ONLY>
__device__ __forceinline__ void elem_sync() {
    if (LDS_ONLY) {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left alone
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    } else {
        __syncthreads();
    }
}

// EARLY: the face fluxes of the node's faces and the RK register are requested right
// after the state, so their latency overlaps the volume terms (more registers).
// PRE (with EARLY): those values come from pre, requested earlier by elem_preload; the
// body's barriers then order LDS only.
template <typename T, int NPT, bool CURVED = false, int BS = WG, bool VISC = true, bool EARLY = false,
          bool PRE = false>
__device__ __forceinline__ void elem_body(const Tile tl, const ElemInfo E0, const T *u,
                                          const T *__restrict__ ff, const T *__restrict__ tab, const Geom &g,
                                          const PhysParams &ph, const EpiArgs &epi, T (*sF)[elem_cols<T>(BS * NPT)],
                                          T *sD, const ElemPre<T, NPT> *pre = nullptr) {
    static_assert(!PRE || (EARLY && !CURVED && !VISC), "preloaded values are those of the EARLY box form");
    constexpr bool ALLD = elem_rows<T, BS * NPT>() == 3 * NV;
    const int tid = threadIdx.x;
    const int n1 = E0.n[0], n2 = E0.n[1], n3 = E0.n[2];
    {
        const int ns[3] = {n1, n2, n3};
#pragma unroll
        for (int d = 0; d < 3; ++d)
            for (int t = tid; t < ns[d] * ns[d]; t += BS) {
                const int row = t / ns[d], col = t - row * ns[d];
                sD[d * DSTR + row * dstride(ns[d]) + col] = tab[T_D + doff(ns[d] - 1) + t];
            }
    }  // ordered before the first read by the barrier after the first flux staging
    const int npe = n1 * n2 * n3;
    const int total = tl.count * npe;
    const T gm1 = (T)ph.gamma - T(1);  // as the face fluxes form it (equal states: zero jump)
    const int64_t fblk = fblock(E0.n);

    T q[NPT][NV], V[NPT][NV];
    T M[CURVED ? NPT : 1][10];  // curved: Ja^1, Ja^2, Ja^3, J at the node
    int loc[NPT][3], le[NPT], nd[NPT];
    bool ok[NPT];
    const bool visc = VISC && epi.grad != nullptr;
    const T mu = (T)epi.mu, kappa = (T)epi.kappa, gam = (T)ph.gamma;
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int t = tid + k * BS;
        ok[k] = t < total;
        le[k] = ok[k] ? t / npe : 0;
        nd[k] = ok[k] ? t - le[k] * npe : 0;
        loc[k][0] = nd[k] % n1;
        loc[k][1] = (nd[k] / n1) % n2;
        loc[k][2] = nd[k] / (n1 * n2);
        const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le[k] * npe);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            q[k][v] = PRE ? pre->q[k][v] : ok[k] ? ((const gmem<T> *)u)[base + v * npe + nd[k]] : T(1);
            V[k][v] = T(0);
        }
        if (CURVED) {
            const T *mp = (const T *)epi.met + (int64_t)10 * (E0.noff + (int64_t)le[k] * npe) + nd[k];
#pragma unroll
            for (int c = 0; c < 10; ++c) M[CURVED ? k : 0][c] = ok[k] ? mp[(int64_t)c * npe] : T(c == 9 ? 1 : 0);
        }
    }
    // the face flux of face (d, side of the node) at this thread's k-th node, variable v
    auto face_ptr = [&](int k, int d) -> const gmem<T> * {
        const int id = loc[k][d], nd_ = d == 0 ? n1 : d == 1 ? n2 : n3;
        if (id != 0 && id != nd_ - 1) return nullptr;
        const int s = id == 0 ? -1 : 1;
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        const int na = t1 == 0 ? n1 : n2;
        const int fm = loc[k][t1] + na * loc[k][t2];
        return (const gmem<T> *)ff + E0.foff + le[k] * fblk + fslot(E0.n, d, s) + fm;
    };
    constexpr int NE = EARLY ? NPT : 1;
    T fe[NE][3][NV];  // EARLY: face fluxes (per direction; zero off the faces)
    T ge[NE][NV];     // EARLY: the RK register
    if (PRE) {
#pragma unroll
        for (int k = 0; k < NE; ++k)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                fe[k][0][v] = pre->fe[PRE ? k : 0][0][v];
                fe[k][1][v] = pre->fe[PRE ? k : 0][1][v];
                fe[k][2][v] = pre->fe[PRE ? k : 0][2][v];
                ge[k][v] = pre->ge[PRE ? k : 0][v];
            }
    } else if (EARLY) {
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le[k] * npe);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const gmem<T> *fp = (ok[k] && !epi.isolated) ? face_ptr(k, d) : nullptr;
                const int ab = (d == 0 ? n2 * n3 : d == 1 ? n1 * n3 : n1 * n2);
#pragma unroll
                for (int v = 0; v < NV; ++v) fe[k][d][v] = fp ? fp[v * ab] : T(0);
            }
#pragma unroll
            for (int v = 0; v < NV; ++v)
                ge[k][v] = (ok[k] && epi.mode == EPI_RK && epi.rkA != 0.0) ? ((const gmem<T> *)epi.g)[base + v * npe + nd[k]]
                                                                           : T(0);
        }
    }
    // contravariant total flux along d at this thread's k-th node, Ja^d . (f^a - f^v):
    // |Ja^d| (f^a_d - f^v_d) on box elements
    auto total_flux = [&](int k, int d, T f[NV]) {
        T G[15];
        if (visc && ok[k]) {
            const T *Gp = (const T *)epi.grad + (int64_t)3 * NV * (E0.noff + (int64_t)le[k] * npe) + nd[k];
#pragma unroll
            for (int c = 0; c < 15; ++c) G[c] = Gp[(int64_t)c * npe];
        }
        if (CURVED) {
            const T *m = M[CURVED ? k : 0];
            const T n[3] = {m[3 * d], m[3 * d + 1], m[3 * d + 2]};
            flux_n(q[k], n, gm1, f);
            if (visc && ok[k]) {
                T fv[NV];
                viscous_n(q[k], G, n, gam, mu, kappa, fv);
#pragma unroll
                for (int v = 0; v < NV; ++v) f[v] -= fv[v];
            }
            return;
        }
        flux_axis(q[k], d, gm1, f);
        if (visc && ok[k]) {
            T fv[NV];
            viscous_axis(q[k], G, d, gam, mu, kappa, fv);
#pragma unroll
            for (int v = 0; v < NV; ++v) f[v] -= fv[v];
        }
        const T Ja = (T)g.Ja[d];
#pragma unroll
        for (int v = 0; v < NV; ++v) f[v] = Ja * f[v];
    };
    const int nn[3] = {n1, n2, n3};
    const int stride[3] = {1, n1, n1 * n2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (!ALLD || d == 0) {
#pragma unroll
            for (int dd = 0; dd < (ALLD ? 3 : 1); ++dd) {
                const int df = ALLD ? dd : d;  // direction of the staged flux
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    T f[NV];
                    total_flux(k, df, f);
                    const int t = tid + k * BS;
                    if (ok[k]) {
#pragma unroll
                        for (int v = 0; v < NV; ++v) sF[(ALLD ? df * NV : 0) + v][sidx<T>(t)] = f[v];
                    }
                }
            }
            elem_sync<PRE>();
        }
        const int nd_ = nn[d];
        const T *Dm = sD + d * DSTR;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!ok[k]) continue;
            const int t = tid + k * BS;
            const int id = loc[k][d];
            const T *Drow = Dm + id * dstride(nd_);
            const int tb = t - id * stride[d];
            // FP32: the flux at the line's first node is subtracted inside every term (the
            // rows of D sum to zero, so the derivative is unchanged in exact arithmetic),
            // which keeps the near-constant part of the flux out of the rounding
            T ref[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) ref[v] = sizeof(T) == 4 ? sF[(ALLD ? d * NV : 0) + v][sidx<T>(tb)] : T(0);
            for (int m = 0; m < nd_; ++m) {
                const T dm = Drow[m];
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    V[k][v] += dm * (sF[(ALLD ? d * NV : 0) + v][sidx<T>(tb + m * stride[d])] - ref[v]);
            }
        }
        // the next direction's staging (or, after the last, the next tile of a persistent
        // loop and the epilogue's reduction) overwrites sF only after this barrier
        if (!ALLD || d == 2) elem_sync<PRE>();
    }
    // lifted surface terms from the face pass
    if (!epi.isolated) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!ok[k]) continue;
            const T *fb = ff + E0.foff + le[k] * fblk;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int id = loc[k][d];
                const int nd_ = nn[d];
                if (id != 0 && id != nd_ - 1) continue;
                const int s = id == 0 ? -1 : 1;
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                const int na = nn[t1], nb = nn[t2];
                const int fm = loc[k][t1] + na * loc[k][t2];
                const T *fs = fb + fslot(E0.n, d, s);
                const T iw = T(1) / tab[T_W + xoff(nd_ - 1)];
                T f[NV];
                total_flux(k, d, f);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const T fv = EARLY ? fe[EARLY ? k : 0][d][v] : fs[v * na * nb + fm];
                    V[k][v] += (fv - T(s) * f[v]) * iw;
                }
            }
        }
    }
    // epilogue
    const T invJbox = (T)(1.0 / g.J);
    T mx[NPT][3];
    T vmx[NPT][2][NV];  // per-variable |tau_new|, |tau_trad| (tau with varnorms)
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        mx[k][0] = T(0);
        mx[k][1] = T(0);
        mx[k][2] = T(0);
#pragma unroll
        for (int v = 0; v < NV; ++v) vmx[k][0][v] = vmx[k][1][v] = T(0);
        if (!ok[k]) continue;
        const T Jn = CURVED ? M[CURVED ? k : 0][9] : (T)g.J;
        const T invJ = CURVED ? T(1) / Jn : invJbox;
        const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le[k] * npe);
        const T www = tab[T_W + xoff(n1 - 1) + loc[k][0]] * tab[T_W + xoff(n2 - 1) + loc[k][1]] *
                      tab[T_W + xoff(n3 - 1) + loc[k][2]];
        if (epi.mode == EPI_RESIDUAL) {
            gmem<T> *r = (gmem<T> *)epi.out;
#pragma unroll
            for (int v = 0; v < NV; ++v) r[base + v * npe + nd[k]] = epi.form == 0 ? V[k][v] * invJ : www * V[k][v];
        } else if (epi.mode == EPI_RK) {
            gmem<T> *uu = (gmem<T> *)u;
            gmem<T> *G = (gmem<T> *)epi.g;
            const T A = (T)epi.rkA, B = (T)epi.rkB, dt = (T)epi.dt;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int64_t x = base + v * npe + nd[k];
                const T r = V[k][v] * invJ;
                const T gold = EARLY ? ge[EARLY ? k : 0][v] : (epi.rkA == 0.0 ? T(0) : G[x]);
                const T gn = (epi.rkA == 0.0) ? -dt * r : A * gold - dt * r;
                G[x] = gn;
                uu[x] = q[k][v] + B * gn;
            }
        } else {  // EPI_TAU
            // no contraction: the coarse residual is rounded exactly as the stored
            // fine one, so tau vanishes bitwise when the coarse orders equal the fine
#pragma clang fp contract(off)
            const T *rd = (const T *)epi.rdc;
            T *tn = (T *)epi.out;
            T *tt = (T *)epi.out2;
            const T Jw = Jn * www;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int64_t x = base + v * npe + nd[k];
                const T a = V[k][v] * invJ - rd[x];
                const T b = Jw * a;
                if (tn) tn[x] = a;
                if (tt) tt[x] = b;
                mx[k][0] = fmax(mx[k][0], fabs(a));
                mx[k][1] = fmax(mx[k][1], fabs(b));
                vmx[k][0][v] = fabs(a);
                vmx[k][1][v] = fabs(b);
                if (epi.psic) mx[k][2] += ((const T *)epi.psic)[x] * b;
            }
        }
    }
    if (epi.mode != EPI_TAU) return;
    // Per-element reduction of three per-node values (two maxima and a sum): stage in
    // LDS, then reduce each element's segment in a fixed order; emit(elem, m0, m1, s2).
    auto reduce = [&](auto val, auto emit) {
        elem_sync<PRE>();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int t = tid + k * BS;
            sF[0][t] = val(k, 0);
            sF[1][t] = val(k, 1);
            sF[2][t] = val(k, 2);
        }
        elem_sync<PRE>();
        if (tl.count == 1) {
            for (int s = BS * NPT / 2; s > 0; s >>= 1) {
#pragma unroll
                for (int k = 0; k < NPT; ++k) {
                    const int t = tid + k * BS;
                    if (t < s) {
                        sF[0][t] = fmax(sF[0][t], sF[0][t + s]);
                        sF[1][t] = fmax(sF[1][t], sF[1][t + s]);
                        sF[2][t] = sF[2][t] + sF[2][t + s];
                    }
                }
                elem_sync<PRE>();
            }
            if (tid == 0) emit((int64_t)tl.first, sF[0][0], sF[1][0], sF[2][0]);
        } else if (tid < tl.count) {
            T m0 = T(0), m1 = T(0), e2 = T(0);
            for (int i = 0; i < npe; ++i) {
                m0 = fmax(m0, sF[0][tid * npe + i]);
                m1 = fmax(m1, sF[1][tid * npe + i]);
                e2 += sF[2][tid * npe + i];
            }
            emit((int64_t)(tl.first + tid), m0, m1, e2);
        }
    };
    if (epi.norms || epi.eta)
        reduce([&](int k, int j) { return mx[k][j]; },
               [&](int64_t e, T m0, T m1, T e2) {
                   if (epi.norms) {
                       epi.norms[2 * e] = (double)m0;
                       epi.norms[2 * e + 1] = (double)m1;
                   }
                   if (epi.eta) epi.eta[e] = (double)e2;
               });
    if (epi.varnorms)
#pragma unroll
        for (int v = 0; v < NV; ++v)
            reduce([&](int k, int j) { return j < 2 ? vmx[k][j][v] : T(0); },
                   [&](int64_t e, T m0, T m1, T) {
                       epi.varnorms[(2 * e) * NV + v] = (double)m0;
                       epi.varnorms[(2 * e + 1) * NV + v] = (double)m1;
                   });
}

// One node per lane for tiles of up to 256 and 512 nodes (BS = 256, 512 lanes): the
// register footprint of one node per lane keeps several waves per SIMD.  Tiles of up to
// 1024 nodes take 1024 lanes on box elements and 512 lanes of two nodes on curved ones
// (whose per-node metric terms do not fit the register budget of 1024-lane groups).
template <typename T, int NPT, bool CURVED, bool VISC, int BS>
__global__ __launch_bounds__(BS) void k_elem(const Tile *__restrict__ tiles, int tile0, int ntiles,
                                             const ElemInfo *__restrict__ el, const T *u,
                                             const T *__restrict__ ff, const T *__restrict__ tab, Geom g,
                                             PhysParams ph, EpiArgs epi) {
    __shared__ T sF[elem_rows<T, BS * NPT>()][elem_cols<T>(BS * NPT)];
    __shared__ T sD[3 * DSTR];
    const Tile tl = tiles[tile0 + xcd_remap(blockIdx.x, ntiles)];
    // early loads pay for FP32 box Euler tiles (31.1 -> 32.2 GDOF/s at 16^3, N = 7); the
    // FP64 pass was slower with them (98 -> 111 us)
    constexpr bool EARLY = !CURVED && !VISC && sizeof(T) == 4;
    elem_body<T, NPT, CURVED, BS, VISC, EARLY>(tl, el[tl.first], u, ff, tab, g, ph, epi, sF, sD);
}

template <typename T>
hipError_t launch_element(const Tile *tiles, int tile0, int ntiles, int npt, const ElemInfo *elems, const T *u,
                          const T *fflux, const T *tab, Geom g, PhysParams ph, EpiArgs epi, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    dim3 grid(ntiles);
    const bool curved = epi.met != nullptr;
    const bool visc = epi.grad != nullptr;
#define DGT_ELEM(NP, CU, BSZ)                                                                                  \
    do {                                                                                                       \
        if (visc)                                                                                              \
            hipLaunchKernelGGL((k_elem<T, NP, CU, true, BSZ>), grid, dim3(BSZ), 0, s, tiles, tile0, ntiles,    \
                               elems, u, fflux, tab, g, ph, epi);                                              \
        else                                                                                                   \
            hipLaunchKernelGGL((k_elem<T, NP, CU, false, BSZ>), grid, dim3(BSZ), 0, s, tiles, tile0, ntiles,   \
                               elems, u, fflux, tab, g, ph, epi);                                              \
    } while (0)
    switch (npt * 2 + (curved ? 1 : 0)) {
        case 2: DGT_ELEM(1, false, WG); break;
        case 3: DGT_ELEM(1, true, WG); break;
        case 4: DGT_ELEM(1, false, 2 * WG); break;
        case 5: DGT_ELEM(1, true, 2 * WG); break;
        case 8: DGT_ELEM(1, false, 4 * WG); break;
        case 9: DGT_ELEM(2, true, 2 * WG); break;
        default: return hipErrorInvalidValue;
    }
#undef DGT_ELEM
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- Navier-Stokes (BR1)
// Pass 1 (faces): BR1 solution trace qhat = (Q_L + Q_R)/2 on the mortar, projected back.
// Pass 2 (elements): J dQ/dx_l = |Ja^l| [ D_l Q + sum_s s (qhat - Q) / w_end on the l-faces ]
//   (affine elements: only the l-derivative and the l-faces contribute).
// Pass 3 (faces): F*_out = |Ja^d| [ Roe(Q_L, Q_R) - (f^v(Q_L, G_L) + f^v(Q_R, G_R))/2 ] . e_d on the
//   mortar (traces of Q and of the 15 gradient components interpolated), projected back.
// Pass 4: the element pass with total flux f^a - f^v.
template <typename T, int FN>
__global__ __launch_bounds__(64) void k_face_avg(const Face *__restrict__ faces, const ElemInfo *__restrict__ el,
                                                 const T *__restrict__ u, T *__restrict__ fq,
                                                 const T *__restrict__ tab, Geom g, PhysParams ph) {
    __shared__ FaceSmem<T, FN> sm;
    const Face f = faces[xcd_remap(blockIdx.x, gridDim.x)];
    ElemInfo L, R;
    face_elems(f, el, L, R);
    face_body<T, FN, 1>(f, L, R, u, fq, tab, g, ph, sm);
}

template <typename T, int NPT>
__global__ __launch_bounds__(WG) void k_elem_grad(const Tile *__restrict__ tiles, int tile0, int ntiles,
                                                  const ElemInfo *__restrict__ el, const T *__restrict__ u,
                                                  const T *__restrict__ fq, T *__restrict__ grad,
                                                  const T *__restrict__ tab, Geom g, int isolated) {
    __shared__ T sQ[NV][WG * NPT];
    __shared__ T sD[3 * NNMAX * NNMAX];  // the tile's derivative matrices (per-lane rows)
    const int tid = threadIdx.x;
    const Tile tl = tiles[tile0 + xcd_remap(blockIdx.x, ntiles)];
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
    T q[NPT][NV];
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
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            q[k][v] = ok[k] ? u[base + v * npe + nd[k]] : T(0);
            if (ok[k]) sQ[v][t] = q[k][v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!ok[k]) continue;
        const int t = tid + k * WG;
        T *Gp = grad + (int64_t)3 * NV * (E0.noff + (int64_t)le[k] * npe) + nd[k];
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const int id = loc[k][l], nl = nn[l];
            const T *Drow = sD + l * NNMAX * NNMAX + id * nl;
            const int tb = t - id * stride[l];
            T G[NV] = {T(0), T(0), T(0), T(0), T(0)};
            for (int m = 0; m < nl; ++m) {
                const T dm = Drow[m];
#pragma unroll
                for (int v = 0; v < NV; ++v) G[v] += dm * sQ[v][tb + m * stride[l]];
            }
            if (!isolated && (id == 0 || id == nl - 1)) {
                const int s = id == 0 ? -1 : 1;
                const int t1 = l == 0 ? 1 : 0, t2 = l == 2 ? 1 : 2;
                const int na = nn[t1], nb = nn[t2];
                const T *fs = fq + E0.foff + le[k] * fblk + fslot(E0.n, l, s);
                const int fm = loc[k][t1] + na * loc[k][t2];
                const T iw = T(1) / tab[T_W + xoff(nl - 1)];
#pragma unroll
                for (int v = 0; v < NV; ++v) G[v] += T(s) * (fs[v * na * nb + fm] - q[k][v]) * iw;
            }
            const T sc = (T)(g.Ja[l] / g.J);
#pragma unroll
            for (int v = 0; v < NV; ++v) Gp[(int64_t)(l * NV + v) * npe] = sc * G[v];
        }
    }
}

template <typename T, int FN, int D>
__device__ __forceinline__ void face_ns_d(const Face f, const ElemInfo *__restrict__ el, const T *__restrict__ u,
                                          const T *__restrict__ grad, T *__restrict__ ff,
                                          const T *__restrict__ tab, const Geom &g, const PhysParams &ph,
                                          T (*sL)[FN], T (*sR)[FN], T (*sF)[FN]) {
    constexpr int NF = 4 * NV;  // Q and its three gradient components
    constexpr int d = D, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const T Ja = (T)g.Ja[d], gam = (T)ph.gamma, mu = (T)ph.mu, kappa = (T)ph.kappa;
    const int lane = threadIdx.x;
    auto load = [&](const ElemInfo &E, int node, T *x) {
        const int ne = E.n[0] * E.n[1] * E.n[2];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = u[NV * E.noff + v * ne + node];
#pragma unroll
        for (int c = 0; c < 3 * NV; ++c) x[NV + c] = grad[3 * NV * E.noff + (int64_t)c * ne + node];
    };
    if (f.bc != 0) {
        const int e = f.eL >= 0 ? f.eL : f.eR;
        const int s = f.eL >= 0 ? 1 : -1;
        const ElemInfo E = el[e];
        const int na = E.n[t1], nb = E.n[t2];
        T *out = ff + E.foff + fslot(E.n, d, s);
        for (int m = lane; m < na * nb; m += 64) {
            T x[NF], qg[NV], F[NV], fv1[NV], fv2[NV];
            load(E, face_node(E.n, d, s, m % na, m / na), x);
            if (f.bc == 1) {
#pragma unroll
                for (int v = 0; v < NV; ++v) qg[v] = x[v];
                qg[1 + d] = -x[1 + d];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) qg[v] = (T)ph.qfar[v];
            }
            numflux_axis(x, qg, d, (T)s, gam, ph.flux, F);
            viscous_axis(x, x + NV, d, gam, mu, kappa, fv1);
            viscous_axis(qg, x + NV, d, gam, mu, kappa, fv2);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * na * nb + m] = Ja * (F[v] - T(s) * T(0.5) * (fv1[v] + fv2[v]));
        }
        return;
    }
    const ElemInfo L = el[f.eL], R = el[f.eR];
    const int aL = L.n[t1], bL = L.n[t2], aR = R.n[t1], bR = R.n[t2];
    const int K1 = aL > aR ? aL : aR, K2 = bL > bR ? bL : bR;
    for (int m = lane; m < aL * bL; m += 64) {
        T x[NF];
        load(L, face_node(L.n, d, 1, m % aL, m / aL), x);
#pragma unroll
        for (int c = 0; c < NF; ++c) sL[c][m] = x[c];
    }
    for (int m = lane; m < aR * bR; m += 64) {
        T x[NF];
        load(R, face_node(R.n, d, -1, m % aR, m / aR), x);
#pragma unroll
        for (int c = 0; c < NF; ++c) sR[c][m] = x[c];
    }
    __syncthreads();
    for (int m = lane; m < K1 * K2; m += 64) {
        const int A = m % K1, B = m / K1;
        T x[2][NF], F[NV], fvL[NV], fvR[NV];
        for (int side = 0; side < 2; ++side) {
            const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
            T(*S)[FN] = side == 0 ? sL : sR;
            if (na == K1 && nb == K2) {
#pragma unroll
                for (int c = 0; c < NF; ++c) x[side][c] = S[c][m];
                continue;
            }
            const T *S1 = tab + T_I + moff(K1 - 1, na - 1) + A * na;
            const T *S2 = tab + T_I + moff(K2 - 1, nb - 1) + B * nb;
#pragma unroll
            for (int c = 0; c < NF; ++c) x[side][c] = T(0);
            for (int b = 0; b < nb; ++b)
                for (int a = 0; a < na; ++a) {
                    const T w = S1[a] * S2[b];
#pragma unroll
                    for (int c = 0; c < NF; ++c) x[side][c] += w * S[c][a + na * b];
                }
        }
        numflux_axis(x[0], x[1], d, T(1), gam, ph.flux, F);
        viscous_axis(x[0], x[0] + NV, d, gam, mu, kappa, fvL);
        viscous_axis(x[1], x[1] + NV, d, gam, mu, kappa, fvR);
#pragma unroll
        for (int v = 0; v < NV; ++v) sF[v][m] = Ja * (F[v] - T(0.5) * (fvL[v] + fvR[v]));
    }
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const ElemInfo &E = side == 0 ? L : R;
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        const T sg = side == 0 ? T(1) : T(-1);
        T *out = ff + E.foff + fslot(E.n, d, side == 0 ? 1 : -1);
        const bool conf = na == K1 && nb == K2;
        const T *P1 = tab + T_P + moff(na - 1, K1 - 1);
        const T *P2 = tab + T_P + moff(nb - 1, K2 - 1);
        for (int m = lane; m < na * nb; m += 64) {
            const int a = m % na, b = m / na;
            T acc[NV] = {T(0), T(0), T(0), T(0), T(0)};
            if (conf) {
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] = sF[v][m];
            } else {
                for (int B = 0; B < K2; ++B)
                    for (int A = 0; A < K1; ++A) {
                        const T w = P1[a * K1 + A] * P2[b * K2 + B];
#pragma unroll
                        for (int v = 0; v < NV; ++v) acc[v] += w * sF[v][A + K1 * B];
                    }
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) out[v * na * nb + m] = sg * acc[v];
        }
    }
}

template <typename T, int FN>
__global__ __launch_bounds__(64) void k_face_ns(const Face *__restrict__ faces, const ElemInfo *__restrict__ el,
                                                const T *__restrict__ u, const T *__restrict__ grad,
                                                T *__restrict__ ff, const T *__restrict__ tab, Geom g,
                                                PhysParams ph) {
    __shared__ T sL[4 * NV][FN], sR[4 * NV][FN], sF[NV][FN];
    const Face f = faces[xcd_remap(blockIdx.x, gridDim.x)];
    if (f.d == 0) face_ns_d<T, FN, 0>(f, el, u, grad, ff, tab, g, ph, sL, sR, sF);
    else if (f.d == 1) face_ns_d<T, FN, 1>(f, el, u, grad, ff, tab, g, ph, sL, sR, sF);
    else face_ns_d<T, FN, 2>(f, el, u, grad, ff, tab, g, ph, sL, sR, sF);
}

template <typename T>
hipError_t launch_ns_gradient(const Face *faces, int nfaces, const Tile *tiles, int tile0, int ntiles, int npt,
                              bool do_faces, const ElemInfo *el, const T *u, T *fq, T *grad, const T *tab, Geom g,
                              PhysParams ph, int max_order, int isolated, hipStream_t s) {
    if (do_faces && !isolated && nfaces > 0) {
        if (max_order <= 7)
            hipLaunchKernelGGL((k_face_avg<T, 64>), dim3(nfaces), dim3(64), 0, s, faces, el, u, fq, tab, g, ph);
        else
            hipLaunchKernelGGL((k_face_avg<T, 100>), dim3(nfaces), dim3(64), 0, s, faces, el, u, fq, tab, g, ph);
    }
    if (ntiles == 0) return hipGetLastError();
    switch (npt) {
        case 1: hipLaunchKernelGGL((k_elem_grad<T, 1>), dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, fq, grad, tab, g, isolated); break;
        case 2: hipLaunchKernelGGL((k_elem_grad<T, 2>), dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, fq, grad, tab, g, isolated); break;
        case 4: hipLaunchKernelGGL((k_elem_grad<T, 4>), dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, fq, grad, tab, g, isolated); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_ns_faces(const Face *faces, int nfaces, const ElemInfo *el, const T *u, const T *grad, T *ff,
                           const T *tab, Geom g, PhysParams ph, hipStream_t s) {
    if (nfaces == 0) return hipSuccess;
    hipLaunchKernelGGL((k_face_ns<T, 64>), dim3(nfaces), dim3(64), 0, s, faces, el, u, grad, ff, tab, g, ph);
    return hipGetLastError();
}

template hipError_t launch_ns_gradient<double>(const Face *, int, const Tile *, int, int, int, bool, const ElemInfo *,
                                               const double *, double *, double *, const double *, Geom, PhysParams,
                                               int, int, hipStream_t);
template hipError_t launch_ns_gradient<float>(const Face *, int, const Tile *, int, int, int, bool, const ElemInfo *,
                                              const float *, float *, float *, const float *, Geom, PhysParams, int,
                                              int, hipStream_t);
template hipError_t launch_ns_faces<double>(const Face *, int, const ElemInfo *, const double *, const double *,
                                            double *, const double *, Geom, PhysParams, hipStream_t);
template hipError_t launch_ns_faces<float>(const Face *, int, const ElemInfo *, const float *, const float *, float *,
                                           const float *, Geom, PhysParams, hipStream_t);

// ---------------------------------------------------------------------------- batches
// Persistent forms, so one launch covers every problem of a batch (no atomics).  Faces
// (listed problem by problem, neighbours close together) go in contiguous ranges, one
// per workgroup, and the workgroups of one XCD take neighbouring ranges, so both sides'
// element blocks stay in that XCD's L2; element tiles (sorted by cost) go cyclically.
// Each face record carries the face and both sides' element descriptors, so a face
// waits on two loads (its record, then its problem's descriptor) before its data.
template <typename T>
__global__ __launch_bounds__(64) void k_face_batch(const BatchFace *__restrict__ faces, int nfaces,
                                                   const ProbDesc<T> *__restrict__ probs, const T *__restrict__ tab) {
    __shared__ FaceSmem<T, 64> sm;  // batches hold orders up to 7
    const int chunk = (nfaces + gridDim.x - 1) / gridDim.x;
    const int i0 = xcd_remap(blockIdx.x, gridDim.x) * chunk;
    const int i1 = min(nfaces, i0 + chunk);
    for (int i = i0; i < i1; ++i) {
        const BatchFace bf = faces[i];
        const ProbDesc<T> pd = probs[bf.prob];
        face_body<T, 64>(bf.f, bf.L, bf.R, (const gmem<T> *)pd.u, (gmem<T> *)pd.ff, tab, pd.geom, pd.phys, sm);
        __syncthreads();
    }
}

template <typename T, int BS, int NPT>
__global__ __launch_bounds__(BS) void k_elem_batch(const BatchTile *__restrict__ tiles, int ntiles,
                                                   const ProbDesc<T> *__restrict__ probs, const T *__restrict__ tab,
                                                   EpiArgs epi0) {
    __shared__ T sF[elem_rows<T, BS * NPT>()][elem_cols<T>(BS * NPT)];
    __shared__ T sD[3 * DSTR];
    __shared__ T sTab[T_I];  // node, weight and derivative tables of every order
    const int G = gridDim.x;
    int i = blockIdx.x;
    if (i >= ntiles) return;
    if (sizeof(T) == 8) {  // FP64: the pipeline's registers would cost a wave per SIMD
        for (; i < ntiles; i += G) {
            const BatchTile bt = tiles[i];
            const ProbDesc<T> pd = probs[bt.prob];
            EpiArgs epi = epi0;
            epi.out = pd.out;
            epi.g = pd.g;
            elem_body<T, NPT, false, BS, false, true>(Tile{bt.first, bt.count}, bt.e0, pd.u, pd.ff, tab, pd.geom,
                                                     pd.phys, epi, sF, sD);
            __syncthreads();
        }
        return;
    }
    // A software pipeline over the workgroup's tiles i, i + G, ...: while tile j is
    // processed, the state, face fluxes and RK register of tile j + 1 are in flight, the
    // descriptor of tile j + 2 and the record of tile j + 3.  The tables are read from
    // LDS, so the body waits on no global load of its own (vector loads complete in
    // order: a wait for a later load would wait for the prefetch as well).
    for (int t = threadIdx.x; t < T_I; t += BS) sTab[t] = tab[t];
    auto at = [&](int k) { return k < ntiles ? k : ntiles - 1; };
    auto epi_of = [&](const ProbDesc<T> &pd) {
        EpiArgs e = epi0;
        e.out = pd.out;
        e.g = pd.g;
        return e;
    };
    BatchTile r0 = tiles[i], r1 = tiles[at(i + G)], r2 = tiles[at(i + 2 * G)];
    ProbDesc<T> p0 = probs[r0.prob], p1 = probs[r1.prob];
    ElemPre<T, NPT> d0;
    elem_preload<T, NPT, BS>(Tile{r0.first, r0.count}, r0.e0, p0.u, p0.ff, epi_of(p0), d0);
    __syncthreads();  // sTab
    for (; i < ntiles; i += G) {
        ElemPre<T, NPT> d1;
        elem_preload<T, NPT, BS>(Tile{r1.first, r1.count}, r1.e0, p1.u, p1.ff, epi_of(p1), d1);
        const ProbDesc<T> p2 = probs[r2.prob];
        const BatchTile r3 = tiles[at(i + 3 * G)];
        elem_body<T, NPT, false, BS, false, true, true>(Tile{r0.first, r0.count}, r0.e0, p0.u, p0.ff, sTab,
                                                       p0.geom, p0.phys, epi_of(p0), sF, sD, &d0);
        elem_sync<true>();
        r0 = r1;
        r1 = r2;
        r2 = r3;
        p0 = p1;
        p1 = p2;
        d0 = d1;
    }
}

template <typename T>
hipError_t launch_face_batch(const BatchFace *faces, int nfaces, const ProbDesc<T> *probs, const T *tab, int grid,
                             hipStream_t s) {
    if (nfaces == 0) return hipSuccess;
    hipLaunchKernelGGL(k_face_batch<T>, dim3(grid), dim3(64), 0, s, faces, nfaces, probs, tab);
    return hipGetLastError();
}

// Element-kernel shapes of the batch (tiles of at most 256 or 512 nodes):
// 0: 256 lanes x 1 node, 1: 256 lanes x 2 nodes, 2: 512 lanes x 1 node.
template <typename T>
hipError_t launch_elem_batch(const BatchTile *tiles, int ntiles, const ProbDesc<T> *probs, const T *tab, int grid,
                             int shape, EpiArgs epi, hipStream_t s) {
    if (ntiles == 0) return hipSuccess;
    switch (shape) {
        case 0:
            hipLaunchKernelGGL((k_elem_batch<T, WG, 1>), dim3(grid), dim3(WG), 0, s, tiles, ntiles, probs, tab, epi);
            break;
        case 1:
            hipLaunchKernelGGL((k_elem_batch<T, WG, 2>), dim3(grid), dim3(WG), 0, s, tiles, ntiles, probs, tab, epi);
            break;
        case 2:
            hipLaunchKernelGGL((k_elem_batch<T, 2 * WG, 1>), dim3(grid), dim3(2 * WG), 0, s, tiles, ntiles, probs,
                               tab, epi);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Uniform admissible state (rho, rho u, rho v, rho w, rho E) = (1, 0.1, 0, 0, 2.505) in every
// element: scratch input of the schedule search.
template <typename T>
__global__ void k_fill_state(const ElemInfo *__restrict__ el, T *__restrict__ u) {
    const ElemInfo E = el[blockIdx.x];
    const int npe = E.n[0] * E.n[1] * E.n[2];
    const T q[NV] = {T(1), T(0.1), T(0), T(0), T(2.505)};
    for (int t = threadIdx.x; t < NV * npe; t += blockDim.x) u[NV * E.noff + t] = q[t / npe];
}

template <typename T>
hipError_t launch_fill_state(const ElemInfo *el, int E, T *u, hipStream_t s) {
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_state<T>, dim3(E), dim3(256), 0, s, el, u);
    return hipGetLastError();
}

template hipError_t launch_face_batch<double>(const BatchFace *, int, const ProbDesc<double> *, const double *, int,
                                              hipStream_t);
template hipError_t launch_face_batch<float>(const BatchFace *, int, const ProbDesc<float> *, const float *, int,
                                             hipStream_t);
template hipError_t launch_elem_batch<double>(const BatchTile *, int, const ProbDesc<double> *, const double *, int, int,
                                              EpiArgs, hipStream_t);
template hipError_t launch_elem_batch<float>(const BatchTile *, int, const ProbDesc<float> *, const float *, int, int,
                                             EpiArgs, hipStream_t);
template hipError_t launch_fill_state<double>(const ElemInfo *, int, double *, hipStream_t);
template hipError_t launch_fill_state<float>(const ElemInfo *, int, float *, hipStream_t);

template hipError_t launch_face_flux<double>(const Face *, int, const ElemInfo *, const double *, double *,
                                             const double *, Geom, PhysParams, int, hipStream_t);
template hipError_t launch_face_flux<float>(const Face *, int, const ElemInfo *, const float *, float *,
                                            const float *, Geom, PhysParams, int, hipStream_t);
template hipError_t launch_element<double>(const Tile *, int, int, int, const ElemInfo *, const double *,
                                           const double *, const double *, Geom, PhysParams, EpiArgs, hipStream_t);
template hipError_t launch_element<float>(const Tile *, int, int, int, const ElemInfo *, const float *,
                                          const float *, const float *, Geom, PhysParams, EpiArgs, hipStream_t);

// ---------------------------------------------------------------------------- coordinates
__global__ void k_coords(const ElemInfo *__restrict__ el, int nx, int ny, const double *__restrict__ tab, Geom g,
                         double *__restrict__ xyz) {
    const ElemInfo E = el[blockIdx.x];
    const int npe = E.n[0] * E.n[1] * E.n[2];
    const int c[3] = {E.nat % nx, (E.nat / nx) % ny, E.nat / (nx * ny)};
    for (int t = threadIdx.x; t < npe; t += blockDim.x) {
        const int id[3] = {t % E.n[0], (t / E.n[0]) % E.n[1], t / (E.n[0] * E.n[1])};
        for (int d = 0; d < 3; ++d) {
            const double xi = tab[T_X + xoff(E.n[d] - 1) + id[d]];
            xyz[3 * E.noff + d * npe + t] = g.lo[d] + g.h[d] * (c[d] + 0.5 * (xi + 1.0));
        }
    }
}

hipError_t launch_coords(const ElemInfo *elems, int E, int nx, int ny, const double *tab, Geom g, double *xyz,
                         hipStream_t s) {
    if (E == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coords, dim3(E), dim3(128), 0, s, elems, nx, ny, tab, g, xyz);
    return hipGetLastError();
}

}  // namespace dgt
