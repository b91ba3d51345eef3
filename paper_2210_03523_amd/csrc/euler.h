// Device physics of the compressible Euler equations: physical flux along a
// coordinate axis and the numerical fluxes at an axis-aligned face.
//
// Roe's approximate Riemann solver (the advective flux of the paper's
// numerical set-up at the start of Section 3): F = (f_L + f_R)/2 - (1/2) sum_k |lam_k| alpha_k r_k
// with Roe averages, acoustic waves u_n -/+ c, an entropy wave and both shear
// waves combined; no entropy fix.  The Rusanov (local Lax-Friedrichs) flux is
// the alternative: F = (f_L + f_R)/2 - (s/2)(Q_R - Q_L), s = max(|u_n| + c).
#pragma once

#include <hip/hip_runtime.h>

namespace dgt {

// The direction index d selects register array elements: every function below is
// written for a compile-time direction D, and the runtime-d entry points dispatch to
// the three instances (a wave-uniform branch), so no private array is ever indexed by
// a runtime value (which would place it in scratch memory).

// Flux f_d(q) along the coordinate direction d (unit normal e_d).
template <int d, typename T>
__device__ __forceinline__ void flux_axis_d(const T q[5], T gm1, T f[5]) {
    T ri = T(1) / q[0];
    T ud = q[1 + d] * ri;
    T p = gm1 * (q[4] - T(0.5) * ri * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
    f[0] = q[1 + d];
    f[1] = q[1] * ud;
    f[2] = q[2] * ud;
    f[3] = q[3] * ud;
    f[1 + d] += p;
    f[4] = (q[4] + p) * ud;
}

template <typename T>
__device__ __forceinline__ void flux_axis(const T q[5], int d, T gm1, T f[5]) {
    if (d == 0) flux_axis_d<0>(q, gm1, f);
    else if (d == 1) flux_axis_d<1>(q, gm1, f);
    else flux_axis_d<2>(q, gm1, f);
}

// Numerical flux through a face with normal s * e_d (s = +-1): returns F . n.
template <int d, typename T>
__device__ __forceinline__ void numflux_axis_d(const T qL[5], const T qR[5], T s, T gamma, int kind, T F[5]) {
    const T gm1 = gamma - T(1);
    T fL[5], fR[5];
    flux_axis_d<d>(qL, gm1, fL);
    flux_axis_d<d>(qR, gm1, fR);
    const T riL = T(1) / qL[0], riR = T(1) / qR[0];
    T uL[3] = {qL[1] * riL, qL[2] * riL, qL[3] * riL};
    T uR[3] = {qR[1] * riR, qR[2] * riR, qR[3] * riR};
    T pL = gm1 * (qL[4] - T(0.5) * qL[0] * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
    T pR = gm1 * (qR[4] - T(0.5) * qR[0] * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
    if (kind == 1) {
        T cL = sqrt(gamma * pL * riL), cR = sqrt(gamma * pR * riR);
        T sp = fmax(fabs(uL[d]) + cL, fabs(uR[d]) + cR);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = s * T(0.5) * (fL[v] + fR[v]) - T(0.5) * sp * (qR[v] - qL[v]);
        return;
    }
    T sL = sqrt(qL[0]), sR = sqrt(qR[0]);
    T ws = T(1) / (sL + sR);
    T ut[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = (sL * uL[k] + sR * uR[k]) * ws;
    T HL = (qL[4] + pL) * riL, HR = (qR[4] + pR) * riR;
    T Ht = (sL * HL + sR * HR) * ws;
    T rt = sL * sR;
    T q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    T c2 = gm1 * (Ht - T(0.5) * q2);
    T c = sqrt(c2);
    T un = s * ut[d];
    T du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
    T dun = s * du[d];
    du[d] = T(0);  // tangential part of the velocity jump
    T drho = qR[0] - qL[0], dp = pR - pL;
    T i2c2 = T(1) / (T(2) * c2);
    T a1 = (dp - rt * c * dun) * i2c2;
    T a2 = drho - dp / c2;
    T a4 = (dp + rt * c * dun) * i2c2;
    T l1 = fabs(un - c) * a1, l2 = fabs(un), l4 = fabs(un + c) * a4;
    T w2 = l2 * a2, w3 = l2 * rt;
    T cn = s * c;
    T utdut = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
    T diss[5];
    diss[0] = l1 + w2 + l4;
#pragma unroll
    for (int k = 0; k < 3; ++k) diss[1 + k] = (l1 + w2 + l4) * ut[k] + w3 * du[k];
    diss[1 + d] += (l4 - l1) * cn;
    diss[4] = l1 * (Ht - c * un) + w2 * T(0.5) * q2 + w3 * utdut + l4 * (Ht + c * un);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = s * T(0.5) * (fL[v] + fR[v]) - T(0.5) * diss[v];
}

template <typename T>
__device__ __forceinline__ void numflux_axis(const T qL[5], const T qR[5], int d, T s, T gamma, int kind,
                                             T F[5]) {
    if (d == 0) numflux_axis_d<0>(qL, qR, s, gamma, kind, F);
    else if (d == 1) numflux_axis_d<1>(qL, qR, s, gamma, kind, F);
    else numflux_axis_d<2>(qL, qR, s, gamma, kind, F);
}

// Flux along an arbitrary vector n (not normalised): f(q) . n = sum_l n_l f_l(q), the
// contravariant flux Ja^d . f of a curved element when n = Ja^d.
template <typename T>
__device__ __forceinline__ void flux_n(const T q[5], const T n[3], T gm1, T f[5]) {
    const T ri = T(1) / q[0];
    const T un = (q[1] * n[0] + q[2] * n[1] + q[3] * n[2]) * ri;
    const T p = gm1 * (q[4] - T(0.5) * ri * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]));
    f[0] = q[0] * un;
    f[1] = q[1] * un + p * n[0];
    f[2] = q[2] * un + p * n[1];
    f[3] = q[3] * un + p * n[2];
    f[4] = (q[4] + p) * un;
}

// Numerical flux through a face with unit normal nh (left state on the side nh
// points away from): Roe (kind 0) or Rusanov (kind 1), returns F . nh.
template <typename T>
__device__ __forceinline__ void numflux_n(const T qL[5], const T qR[5], const T nh[3], T gamma, int kind, T F[5]) {
    const T gm1 = gamma - T(1);
    T fL[5], fR[5];
    flux_n(qL, nh, gm1, fL);
    flux_n(qR, nh, gm1, fR);
    const T riL = T(1) / qL[0], riR = T(1) / qR[0];
    const T uL[3] = {qL[1] * riL, qL[2] * riL, qL[3] * riL};
    const T uR[3] = {qR[1] * riR, qR[2] * riR, qR[3] * riR};
    const T pL = gm1 * (qL[4] - T(0.5) * qL[0] * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
    const T pR = gm1 * (qR[4] - T(0.5) * qR[0] * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
    if (kind == 1) {
        const T cL = sqrt(gamma * pL * riL), cR = sqrt(gamma * pR * riR);
        const T unL = uL[0] * nh[0] + uL[1] * nh[1] + uL[2] * nh[2];
        const T unR = uR[0] * nh[0] + uR[1] * nh[1] + uR[2] * nh[2];
        const T sp = fmax(fabs(unL) + cL, fabs(unR) + cR);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (fL[v] + fR[v]) - T(0.5) * sp * (qR[v] - qL[v]);
        return;
    }
    const T sL = sqrt(qL[0]), sR = sqrt(qR[0]);
    const T ws = T(1) / (sL + sR);
    T ut[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = (sL * uL[k] + sR * uR[k]) * ws;
    const T HL = (qL[4] + pL) * riL, HR = (qR[4] + pR) * riR;
    const T Ht = (sL * HL + sR * HR) * ws;
    const T rt = sL * sR;
    const T q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    const T c2 = gm1 * (Ht - T(0.5) * q2);
    const T c = sqrt(c2);
    const T un = ut[0] * nh[0] + ut[1] * nh[1] + ut[2] * nh[2];
    T du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
    const T dun = du[0] * nh[0] + du[1] * nh[1] + du[2] * nh[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) du[k] -= dun * nh[k];  // tangential part of the velocity jump
    const T drho = qR[0] - qL[0], dp = pR - pL;
    const T i2c2 = T(1) / (T(2) * c2);
    const T a1 = (dp - rt * c * dun) * i2c2;
    const T a2 = drho - dp / c2;
    const T a4 = (dp + rt * c * dun) * i2c2;
    const T l1 = fabs(un - c) * a1, l2 = fabs(un), l4 = fabs(un + c) * a4;
    const T w2 = l2 * a2, w3 = l2 * rt;
    const T utdut = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
    T diss[5];
    diss[0] = l1 + w2 + l4;
#pragma unroll
    for (int k = 0; k < 3; ++k) diss[1 + k] = (l1 + w2 + l4) * ut[k] + w3 * du[k] + (l4 - l1) * c * nh[k];
    diss[4] = l1 * (Ht - c * un) + w2 * T(0.5) * q2 + w3 * utdut + l4 * (Ht + c * un);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = T(0.5) * (fL[v] + fR[v]) - T(0.5) * diss[v];
}

// Viscous flux f^v_d(Q, G) of the Navier-Stokes equations along direction d
// (BR1: G[l*5 + v] = d(conserved v)/dx_l): Stokes stress with constant mu and Fourier
// heat flux kappa grad T on T = p/rho, kappa = mu gamma / ((gamma-1) Pr).
template <int d, typename T>
__device__ __forceinline__ void viscous_axis_d(const T q[5], const T G[15], T gamma, T mu, T kappa, T f[5]) {
    const T ri = T(1) / q[0];
    const T u[3] = {q[1] * ri, q[2] * ri, q[3] * ri};
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T p = (gamma - T(1)) * (q[4] - T(0.5) * q[0] * uu);
    const T Tt = p * ri;
    T du[3][3], dT[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const T *Gl = G + 5 * l;
#pragma unroll
        for (int k = 0; k < 3; ++k) du[k][l] = (Gl[1 + k] - u[k] * Gl[0]) * ri;
        const T dp = (gamma - T(1)) * (Gl[4] - (u[0] * Gl[1] + u[1] * Gl[2] + u[2] * Gl[3]) + T(0.5) * uu * Gl[0]);
        dT[l] = (dp - Tt * Gl[0]) * ri;
    }
    const T div = du[0][0] + du[1][1] + du[2][2];
    T tau[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) tau[k] = mu * (du[k][d] + du[d][k]);
    tau[d] -= T(2.0 / 3.0) * mu * div;
    f[0] = T(0);
    f[1] = tau[0];
    f[2] = tau[1];
    f[3] = tau[2];
    f[4] = u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + kappa * dT[d];
}

template <typename T>
__device__ __forceinline__ void viscous_axis(const T q[5], const T G[15], int d, T gamma, T mu, T kappa,
                                             T f[5]) {
    if (d == 0) viscous_axis_d<0>(q, G, gamma, mu, kappa, f);
    else if (d == 1) viscous_axis_d<1>(q, G, gamma, mu, kappa, f);
    else viscous_axis_d<2>(q, G, gamma, mu, kappa, f);
}

// Viscous flux along an arbitrary vector n: sum_l n_l f^v_l(Q, G) (same model).
template <typename T>
__device__ __forceinline__ void viscous_n(const T q[5], const T G[15], const T n[3], T gamma, T mu, T kappa,
                                          T f[5]) {
    const T ri = T(1) / q[0];
    const T u[3] = {q[1] * ri, q[2] * ri, q[3] * ri};
    const T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const T p = (gamma - T(1)) * (q[4] - T(0.5) * q[0] * uu);
    const T Tt = p * ri;
    T du[3][3], dT[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        const T *Gl = G + 5 * l;
#pragma unroll
        for (int k = 0; k < 3; ++k) du[k][l] = (Gl[1 + k] - u[k] * Gl[0]) * ri;
        const T dp = (gamma - T(1)) * (Gl[4] - (u[0] * Gl[1] + u[1] * Gl[2] + u[2] * Gl[3]) + T(0.5) * uu * Gl[0]);
        dT[l] = (dp - Tt * Gl[0]) * ri;
    }
    const T div = du[0][0] + du[1][1] + du[2][2];
    T tn[3];  // (tau n)_k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < 3; ++l) acc += (du[k][l] + du[l][k]) * n[l];
        tn[k] = mu * acc - T(2.0 / 3.0) * mu * div * n[k];
    }
    f[0] = T(0);
    f[1] = tn[0];
    f[2] = tn[1];
    f[3] = tn[2];
    f[4] = u[0] * tn[0] + u[1] * tn[1] + u[2] * tn[2] + kappa * (dT[0] * n[0] + dT[1] * n[1] + dT[2] * n[2]);
}

}  // namespace dgt
