// Adjoint kernels for gfx950: the vector-Jacobian product of the DGSEM residual
// (out = (dr/dQ)^T v, r in the new or traditional form of Section 2.1), the
// x-pressure force on slip walls with its gradient, and helpers.
//
// r_n = c_n [ sum_d sum_m D^d_{n m} |Ja^d| f_d(Q_m) + SAT_n ],  c_n = 1/J (new form)
// or w_i w_j w_k (traditional form).  With vt = c v:
//   volume     : out_m += sum_d |Ja^d| A_d(Q_m)^T (sum_n D^d_{n m} vt_n)      (D transposed)
//   inner trace: out_m -= s |Ja^d| A_d(Q_m)^T vt_m / w_end  at face nodes of face (d, s)
//   Riemann    : the face pass transposes P (projection), the Riemann-flux Jacobian
//                (its reverse-mode derivative) and S (mortar interpolation), and
//                stores each side's share in per-element face slots, which the
//                element pass gathers -- no atomics, deterministic.
// The transposed Jacobians A_d^T = (df_d/dQ)^T act through the fluxes' reverse-mode
// derivatives (euler_adj.h), never formed as matrices.
#include <hip/hip_runtime.h>

#include "common.h"
#include "euler.h"
#include "euler_adj.h"

namespace dgt {

__device__ __forceinline__ int vjp_face_node(const int32_t *n, int d, int side, int a, int b) {
    int idx[3];
    idx[d] = side > 0 ? n[d] - 1 : 0;
    idx[d == 0 ? 1 : 0] = a;
    idx[d == 2 ? 1 : 2] = b;
    return idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
}


// Residual-form weight c_n at a node.
__device__ __forceinline__ double form_weight(const ElemInfo &E, int node, const double *tab, int form,
                                              double invJ) {
    if (form == 0) return invJ;
    const int i = node % E.n[0], j = (node / E.n[0]) % E.n[1], k = node / (E.n[0] * E.n[1]);
    return tab[T_W + xoff(E.n[0] - 1) + i] * tab[T_W + xoff(E.n[1] - 1) + j] * tab[T_W + xoff(E.n[2] - 1) + k];
}

// ---------------------------------------------------------------------------- faces
// D: the face direction as a compile-time constant (a wave-uniform branch in the kernel),
// so no register array is indexed at run time; KIND: the Riemann flux (0 Roe, 1 Rusanov)
// as a compile-time constant, so the register budget is that of one flux.  The LDS
// arrays hold [5][fnv] doubles each, fnv the plan's largest face node count.
template <int D, int KIND>
__device__ __forceinline__ void face_vjp_d(const Face f, const ElemInfo *__restrict__ el, const double *__restrict__ u,
                                           const double *__restrict__ v, double *__restrict__ fa,
                                           const double *__restrict__ tab, const Geom &g, const PhysParams &ph,
                                           int form, double *sQL, double *sQR, double *sLL, double *sLR, double *sAL,
                                           double *sAR, int fnv) {
    constexpr int d = D, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double Ja = g.Ja[d], invJ = 1.0 / g.J;
    const int lane = threadIdx.x;

    if (f.bc != 0) {
        const int e = f.eL >= 0 ? f.eL : f.eR;
        const int s = f.eL >= 0 ? 1 : -1;
        const ElemInfo E = el[e];
        const int na = E.n[t1], nb = E.n[t2], ne = E.n[0] * E.n[1] * E.n[2];
        const double iw = 1.0 / tab[T_W + xoff(E.n[d] - 1)];
        double *out = fa + E.foff + fslot(E.n, d, s);
        for (int m = lane; m < na * nb; m += 64) {
            const int node = vjp_face_node(E.n, d, s, m % na, m / na);
            const double c = form_weight(E, node, tab, form, invJ) * iw;
            double q0[NV], lam[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                q0[k] = u[NV * E.noff + k * ne + node];
                lam[k] = c * v[NV * E.noff + k * ne + node];
            }
            // lam^T dF/dq of the boundary flux; a wall's ghost is the mirrored state, so
            // its cotangent returns through the mirror; the far-field state is fixed
            double qg[NV], gI[NV], gG[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) qg[k] = f.bc == 1 ? q0[k] : ph.qfar[k];
            if (f.bc == 1) qg[1 + d] = -q0[1 + d];
            numflux_axis_adj_d<d>(q0, qg, (double)s, ph.gamma, KIND, lam, gI, gG);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                if (f.bc == 1) gI[k] += k == 1 + d ? -gG[k] : gG[k];
                out[k * na * nb + m] = Ja * gI[k];
            }
        }
        return;
    }

    const ElemInfo L = el[f.eL], R = el[f.eR];
    const int aL = L.n[t1], bL = L.n[t2], aR = R.n[t1], bR = R.n[t2];
    const int K1 = aL > aR ? aL : aR, K2 = bL > bR ? bL : bR;
    const int neL = L.n[0] * L.n[1] * L.n[2], neR = R.n[0] * R.n[1] * R.n[2];
    const double iwL = 1.0 / tab[T_W + xoff(L.n[d] - 1)], iwR = 1.0 / tab[T_W + xoff(R.n[d] - 1)];
    if (aL == aR && bL == bR) {
        // conforming face: the mortar is both traces, so every lane works on its own node
        // from global memory to global memory (no staging, no barrier)
        double *outL = fa + L.foff + fslot(L.n, d, 1), *outR = fa + R.foff + fslot(R.n, d, -1);
        for (int m = lane; m < aL * bL; m += 64) {
            const int a = m % aL, b = m / aL;
            const int nL = vjp_face_node(L.n, d, 1, a, b), nR = vjp_face_node(R.n, d, -1, a, b);
            const double cL = form_weight(L, nL, tab, form, invJ) * iwL;
            const double cR = form_weight(R, nR, tab, form, invJ) * iwR;
            double qL[NV], qR[NV], gK[NV], gL[NV], gR[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                qL[k] = u[NV * L.noff + k * neL + nL];
                qR[k] = u[NV * R.noff + k * neR + nR];
                gK[k] = cL * v[NV * L.noff + k * neL + nL] - cR * v[NV * R.noff + k * neR + nR];
            }
            numflux_axis_adj_d<d>(qL, qR, 1.0, ph.gamma, KIND, gK, gL, gR);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                outL[k * aL * bL + m] = Ja * gL[k];
                outR[k * aL * bL + m] = Ja * gR[k];
            }
        }
        return;
    }
    for (int m = lane; m < aL * bL; m += 64) {
        const int node = vjp_face_node(L.n, d, 1, m % aL, m / aL);
        const double c = form_weight(L, node, tab, form, invJ) * iwL;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            sQL[k * fnv + m] = u[NV * L.noff + k * neL + node];
            sLL[k * fnv + m] = c * v[NV * L.noff + k * neL + node];
        }
    }
    for (int m = lane; m < aR * bR; m += 64) {
        const int node = vjp_face_node(R.n, d, -1, m % aR, m / aR);
        const double c = form_weight(R, node, tab, form, invJ) * iwR;
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            sQR[k * fnv + m] = u[NV * R.noff + k * neR + node];
            sLR[k * fnv + m] = c * v[NV * R.noff + k * neR + node];
        }
    }
    __syncthreads();
    const bool confL = (aL == K1 && bL == K2), confR = (aR == K1 && bR == K2);
    for (int m = lane; m < K1 * K2; m += 64) {
        const int A = m % K1, B = m / K1;
        double qL[NV], qR[NV], gK[NV];
        // mortar traces (forward interpolation) and the mortar adjoint weight
        // gK = P_L^T lambda_L - P_R^T lambda_R (unrolled: q and gK stay in registers)
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
            const bool conf = side == 0 ? confL : confR;
            double *sQ = side == 0 ? sQL : sQR;
            double *sL = side == 0 ? sLL : sLR;
            double *q = side == 0 ? qL : qR;
            const double sg = side == 0 ? 1.0 : -1.0;
            if (conf) {
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    q[k] = sQ[k * fnv + m];
                    gK[k] = (side == 0 ? 0.0 : gK[k]) + sg * sL[k * fnv + m];
                }
                continue;
            }
            const double *S1 = tab + T_I + moff(K1 - 1, na - 1) + A * na;
            const double *S2 = tab + T_I + moff(K2 - 1, nb - 1) + B * nb;
            const double *P1 = tab + T_P + moff(na - 1, K1 - 1);
            const double *P2 = tab + T_P + moff(nb - 1, K2 - 1);
            double qa[NV] = {0, 0, 0, 0, 0}, ga[NV] = {0, 0, 0, 0, 0};
            for (int b = 0; b < nb; ++b) {
                double qi[NV] = {0, 0, 0, 0, 0}, gi[NV] = {0, 0, 0, 0, 0};
                for (int a = 0; a < na; ++a) {
                    const double s1 = S1[a], p1 = P1[a * K1 + A];
#pragma unroll
                    for (int k = 0; k < NV; ++k) {
                        qi[k] += s1 * sQ[k * fnv + a + na * b];
                        gi[k] += p1 * sL[k * fnv + a + na * b];
                    }
                }
                const double s2 = S2[b], p2 = P2[b * K2 + B];
#pragma unroll
                for (int k = 0; k < NV; ++k) {
                    qa[k] += s2 * qi[k];
                    ga[k] += p2 * gi[k];
                }
            }
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                q[k] = qa[k];
                gK[k] = (side == 0 ? 0.0 : gK[k]) + sg * ga[k];
            }
        }
        // gK^T dF/dq for both traces, by the flux's reverse-mode derivative
        double gL[NV], gR[NV];
        numflux_axis_adj_d<d>(qL, qR, 1.0, ph.gamma, KIND, gK, gL, gR);
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            sAL[k * fnv + m] = Ja * gL[k];
            sAR[k * fnv + m] = Ja * gR[k];
        }
    }
    __syncthreads();
    // transpose of the mortar interpolation back onto each side's face nodes
    for (int side = 0; side < 2; ++side) {
        const ElemInfo &E = side == 0 ? L : R;
        const int na = side == 0 ? aL : aR, nb = side == 0 ? bL : bR;
        const bool conf = side == 0 ? confL : confR;
        double *sA = side == 0 ? sAL : sAR;
        double *out = fa + E.foff + fslot(E.n, d, side == 0 ? 1 : -1);
        const double *S1 = tab + T_I + moff(K1 - 1, na - 1);
        const double *S2 = tab + T_I + moff(K2 - 1, nb - 1);
        for (int m = lane; m < na * nb; m += 64) {
            const int a = m % na, b = m / na;
            if (conf) {
#pragma unroll
                for (int k = 0; k < NV; ++k) out[k * na * nb + m] = sA[k * fnv + m];
                continue;
            }
            double acc[NV] = {0, 0, 0, 0, 0};
            for (int B = 0; B < K2; ++B) {
                double in[NV] = {0, 0, 0, 0, 0};
                for (int A = 0; A < K1; ++A) {
                    const double s1 = S1[A * na + a];
#pragma unroll
                    for (int k = 0; k < NV; ++k) in[k] += s1 * sA[k * fnv + A + K1 * B];
                }
                const double s2 = S2[B * nb + b];
#pragma unroll
                for (int k = 0; k < NV; ++k) acc[k] += s2 * in[k];
            }
#pragma unroll
            for (int k = 0; k < NV; ++k) out[k * na * nb + m] = acc[k];
        }
    }
}

// Two waves per SIMD: the Roe flux with its reverse-mode derivative needs about 200
// registers, which the budget of two waves holds without spills.
template <int KIND>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_face_vjp(
    const Face *__restrict__ faces, const ElemInfo *__restrict__ el, const double *__restrict__ u,
    const double *__restrict__ v, double *__restrict__ fa, const double *__restrict__ tab, Geom g, PhysParams ph,
    int form, int fnv) {
    extern __shared__ double lds[];
    double *sQL = lds, *sQR = lds + NV * fnv, *sLL = lds + 2 * NV * fnv, *sLR = lds + 3 * NV * fnv;
    double *sAL = lds + 4 * NV * fnv, *sAR = lds + 5 * NV * fnv;
    const Face f = faces[xcd_remap(blockIdx.x, gridDim.x)];  // XCD-contiguous face ranges
    if (f.d == 0) face_vjp_d<0, KIND>(f, el, u, v, fa, tab, g, ph, form, sQL, sQR, sLL, sLR, sAL, sAR, fnv);
    else if (f.d == 1) face_vjp_d<1, KIND>(f, el, u, v, fa, tab, g, ph, form, sQL, sQR, sLL, sLR, sAL, sAR, fnv);
    else face_vjp_d<2, KIND>(f, el, u, v, fa, tab, g, ph, form, sQL, sQR, sLL, sLR, sAL, sAR, fnv);
}

// ---------------------------------------------------------------------------- elements
// One node per lane: five waves per SIMD (86 registers, no spills), more element tiles
// in flight to cover the load-compute-store phases; the multi-node instances keep the
// default budget, which they need without spills.
template <int NPT>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(NPT == 1 ? 5 : 1))) void k_elem_vjp(const Tile *__restrict__ tiles, int tile0, int ntiles,
                                                 const ElemInfo *__restrict__ el, const double *__restrict__ u,
                                                 const double *__restrict__ v, const double *__restrict__ fa,
                                                 double *__restrict__ out, const double *__restrict__ tab, Geom g,
                                                 PhysParams ph, int form, int isolated) {
    __shared__ double sV[NV][WG * NPT];
    __shared__ double sD[3 * NNMAX * NNMAX];  // the tile's derivative matrices (per-lane columns)
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
    const double invJ = 1.0 / g.J, gm1 = ph.gamma - 1.0;
    const int nn[3] = {n1, n2, n3};
    const int stride[3] = {1, n1, n1 * n2};

    double q[NPT][NV], vt[NPT][NV];
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
        const double c = form_weight(E0, nd[k], tab, form, invJ);
#pragma unroll
        for (int w = 0; w < NV; ++w) {
            q[k][w] = ok[k] ? u[base + w * npe + nd[k]] : 1.0;
            vt[k][w] = ok[k] ? c * v[base + w * npe + nd[k]] : 0.0;
            if (ok[k]) sV[w][t] = vt[k][w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!ok[k]) continue;
        const int t = tid + k * WG;
        double acc[NV] = {0, 0, 0, 0, 0}, yd[3][NV];
        const int64_t base = (int64_t)NV * (E0.noff + (int64_t)le[k] * npe);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int id = loc[k][d], nd_ = nn[d];
            const double *Dm = sD + d * NNMAX * NNMAX;
            const int tb = t - id * stride[d];
            double y[NV] = {0, 0, 0, 0, 0};
            for (int m = 0; m < nd_; ++m) {
                const double dm = Dm[m * nd_ + id];
#pragma unroll
                for (int w = 0; w < NV; ++w) y[w] += dm * sV[w][tb + m * stride[d]];
            }
            if (!isolated && (id == 0 || id == nd_ - 1)) {
                const double s = id == 0 ? -1.0 : 1.0;
                const double iw = 1.0 / tab[T_W + xoff(nd_ - 1)];
#pragma unroll
                for (int w = 0; w < NV; ++w) y[w] -= s * vt[k][w] * iw;
            }
            const double Ja = g.Ja[d];
#pragma unroll
            for (int w = 0; w < NV; ++w) yd[d][w] = Ja * y[w];
            // Riemann-flux share gathered from the face pass
            if (!isolated && (id == 0 || id == nd_ - 1)) {
                const int side = id == 0 ? -1 : 1;
                const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                const int na = nn[t1], nb = nn[t2];
                const double *fs = fa + E0.foff + le[k] * fblk + fslot(E0.n, d, side);
                const int fm = loc[k][t1] + na * loc[k][t2];
#pragma unroll
                for (int kk = 0; kk < NV; ++kk) acc[kk] += fs[kk * na * nb + fm];
            }
        }
        // sum_d A_d(Q)^T (Ja_d y_d), one reverse-mode pass over the three axis fluxes
        flux3_adj(q[k], gm1, yd, acc);
#pragma unroll
        for (int kk = 0; kk < NV; ++kk) out[base + kk * npe + nd[k]] = acc[kk];
    }
}

hipError_t launch_vjp(const Face *faces, int nfaces, const Tile *tiles, int tile0, int ntiles, int npt,
                      const ElemInfo *el, const double *u, const double *v, double *fa, double *out,
                      const double *tab, Geom g, PhysParams ph, int form, int isolated, bool do_faces, int max_order,
                      hipStream_t s) {
    if (do_faces && nfaces > 0) {
        const int fnv = (max_order + 1) * (max_order + 1);  // largest face node count
        const size_t lds = sizeof(double) * 6 * NV * (size_t)fnv;
        if (ph.flux == 1)
            hipLaunchKernelGGL(k_face_vjp<1>, dim3(nfaces), dim3(64), lds, s, faces, el, u, v, fa, tab, g, ph, form,
                               fnv);
        else
            hipLaunchKernelGGL(k_face_vjp<0>, dim3(nfaces), dim3(64), lds, s, faces, el, u, v, fa, tab, g, ph, form,
                               fnv);
    }
    if (ntiles == 0) return hipGetLastError();
    switch (npt) {
        case 1: hipLaunchKernelGGL(k_elem_vjp<1>, dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, v, fa, out, tab, g, ph, form, isolated); break;
        case 2: hipLaunchKernelGGL(k_elem_vjp<2>, dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, v, fa, out, tab, g, ph, form, isolated); break;
        case 4: hipLaunchKernelGGL(k_elem_vjp<4>, dim3(ntiles), dim3(WG), 0, s, tiles, tile0, ntiles, el, u, v, fa, out, tab, g, ph, form, isolated); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------- force functional
// x-pressure force on slip walls: per wall face, sum of w_a w_b |Ja^1| s p(Q) over its
// nodes (one wavefront), then a fixed-order sum of the face partials.
__device__ __forceinline__ double wsum(double x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__global__ __launch_bounds__(64) void k_functional(const Face *__restrict__ faces, const int32_t *__restrict__ wall,
                                                   const ElemInfo *__restrict__ el, const double *__restrict__ u,
                                                   const double *__restrict__ tab, Geom g, double gamma,
                                                   double *__restrict__ part, double *__restrict__ dJdu) {
    const Face f = faces[wall[blockIdx.x]];
    const int e = f.eL >= 0 ? f.eL : f.eR;
    const int s = f.eL >= 0 ? 1 : -1;
    const ElemInfo E = el[e];
    const int na = E.n[1], nb = E.n[2], ne = E.n[0] * E.n[1] * E.n[2];
    const double *wa = tab + T_W + xoff(na - 1), *wb = tab + T_W + xoff(nb - 1);
    double acc = 0.0;
    for (int m = threadIdx.x; m < na * nb; m += 64) {
        const int a = m % na, b = m / na;
        const int node = vjp_face_node(E.n, 0, s, a, b);
        const double *Q = u + NV * E.noff;
        const double rho = Q[node], mx = Q[ne + node], my = Q[2 * ne + node], mz = Q[3 * ne + node];
        const double rE = Q[4 * ne + node];
        const double ux = mx / rho, uy = my / rho, uz = mz / rho;
        const double p = (gamma - 1.0) * (rE - 0.5 * (mx * ux + my * uy + mz * uz));
        const double wgt = wa[a] * wb[b] * g.Ja[0] * (double)s;
        acc += wgt * p;
        if (dJdu) {
            double *D = dJdu + NV * E.noff;
            D[node] = wgt * (gamma - 1.0) * 0.5 * (ux * ux + uy * uy + uz * uz);
            D[ne + node] = -wgt * (gamma - 1.0) * ux;
            D[2 * ne + node] = -wgt * (gamma - 1.0) * uy;
            D[3 * ne + node] = -wgt * (gamma - 1.0) * uz;
            D[4 * ne + node] = wgt * (gamma - 1.0);
        }
    }
    acc = wsum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_sum_parts(const double *__restrict__ part, int n, double *__restrict__ J) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) acc += part[i];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) J[0] = s[0];
}

__global__ void k_zero(double *__restrict__ x, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 0.0;
}

hipError_t launch_functional(const Face *faces, const int32_t *wall, int nwall, const ElemInfo *el,
                             const double *u, const double *tab, Geom g, double gamma, double *part, double *J,
                             double *dJdu, int64_t n_vals, hipStream_t s) {
    if (dJdu) hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, s, dJdu, n_vals);
    if (nwall > 0)
        hipLaunchKernelGGL(k_functional, dim3(nwall), dim3(64), 0, s, faces, wall, el, u, tab, g, gamma, part, dJdu);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, part, nwall, J);
    return hipGetLastError();
}

}  // namespace dgt
