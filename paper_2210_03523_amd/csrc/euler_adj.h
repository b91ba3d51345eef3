// Reverse-mode (adjoint) derivatives of the Euler fluxes in euler.h, written out by
// hand: for a cotangent y of the flux they return y^T (df/dq), the transposed
// Jacobian applied to y, at the cost of about one more flux evaluation (instead of one
// forward-mode pass per input component).  Each backward statement mirrors one
// forward statement of euler.h, in reverse order.  At the non-smooth points:
// d|x|/dx = sign(x) with 0 at x = 0, and max(a, b) follows a when a >= b.
#pragma once

#include <hip/hip_runtime.h>

namespace dgt {

__device__ __forceinline__ double sgn(double x) { return x > 0.0 ? 1.0 : (x < 0.0 ? -1.0 : 0.0); }

// g += sum_d (Ja_d y_d)^T df_d/dq: the three axis fluxes of one node, each with its own
// cotangent y[d] (already scaled by the metric term).
__device__ __forceinline__ void flux3_adj(const double q[5], double gm1, const double y[3][5], double g[5]) {
    const double ri = 1.0 / q[0];
    const double u[3] = {q[1] * ri, q[2] * ri, q[3] * ri};
    const double m2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const double p = gm1 * (q[4] - 0.5 * ri * m2);
    double pb = 0.0, rib = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double *yd = y[d];
        // f0 = q[1+d], f[1+k] = q[1+k] u_d (+ p for k = d), f4 = (q4 + p) u_d
        const double udb = yd[1] * q[1] + yd[2] * q[2] + yd[3] * q[3] + yd[4] * (q[4] + p);
        pb += yd[1 + d] + yd[4] * u[d];
        g[1] += yd[1] * u[d];
        g[2] += yd[2] * u[d];
        g[3] += yd[3] * u[d];
        g[4] += yd[4] * u[d];
        g[1 + d] += yd[0] + udb * ri;  // u_d = q[1+d] ri
        rib += udb * q[1 + d];
    }
    // p = gm1 (q4 - ri m2 / 2)
    g[4] += gm1 * pb;
    rib -= 0.5 * gm1 * m2 * pb;
#pragma unroll
    for (int k = 1; k < 4; ++k) g[k] -= gm1 * ri * q[k] * pb;
    g[0] -= ri * ri * rib;
}

// gL = lam^T dF/dqL, gR = lam^T dF/dqR for the numerical flux F = numflux_axis_d<d>(qL,
// qR, s, gamma, kind) of euler.h (Roe for kind 0, Rusanov for kind 1).
template <int d>
__device__ __forceinline__ void numflux_axis_adj_d(const double qL[5], const double qR[5], double s, double gamma,
                                                   int kind, const double lam[5], double gL[5], double gR[5]) {
    const double gm1 = gamma - 1.0;
    // ---- forward values
    const double riL = 1.0 / qL[0], riR = 1.0 / qR[0];
    const double uL[3] = {qL[1] * riL, qL[2] * riL, qL[3] * riL};
    const double uR[3] = {qR[1] * riR, qR[2] * riR, qR[3] * riR};
    const double kL = uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2];
    const double kR = uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2];
    const double pL = gm1 * (qL[4] - 0.5 * qL[0] * kL), pR = gm1 * (qR[4] - 0.5 * qR[0] * kR);

    // the central part s (f_L + f_R) / 2: the physical flux's adjoint on each side
    double half[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        half[v] = 0.5 * s * lam[v];
        gL[v] = 0.0;
        gR[v] = 0.0;
    }
    {
        double y[3][5];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int v = 0; v < 5; ++v) y[a][v] = a == d ? half[v] : 0.0;
        flux3_adj(qL, gm1, y, gL);
        flux3_adj(qR, gm1, y, gR);
    }

    // adjoints of the primitive quantities, filled by the dissipation below
    double uLb[3] = {0, 0, 0}, uRb[3] = {0, 0, 0}, pLb = 0.0, pRb = 0.0, riLb = 0.0, riRb = 0.0;
    if (kind == 1) {
        // F -= sp (qR - qL) / 2, sp = max(|uL_d| + cL, |uR_d| + cR), c = sqrt(gamma p ri)
        const double cL = sqrt(gamma * pL * riL), cR = sqrt(gamma * pR * riR);
        const double eL = fabs(uL[d]) + cL, eR = fabs(uR[d]) + cR;
        const double sp = eL >= eR ? eL : eR;
        double spb = 0.0;
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            spb -= 0.5 * lam[v] * (qR[v] - qL[v]);
            gR[v] -= 0.5 * sp * lam[v];
            gL[v] += 0.5 * sp * lam[v];
        }
        if (eL >= eR) {
            uLb[d] += spb * sgn(uL[d]);
            const double zb = spb * 0.5 / cL;  // z = gamma pL riL
            pLb += zb * gamma * riL;
            riLb += zb * gamma * pL;
        } else {
            uRb[d] += spb * sgn(uR[d]);
            const double zb = spb * 0.5 / cR;
            pRb += zb * gamma * riR;
            riRb += zb * gamma * pR;
        }
    } else {
        // ---- Roe: forward values of the dissipation
        const double sL = sqrt(qL[0]), sR = sqrt(qR[0]);
        const double ws = 1.0 / (sL + sR);
        double ut[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ut[k] = (sL * uL[k] + sR * uR[k]) * ws;
        const double HL = (qL[4] + pL) * riL, HR = (qR[4] + pR) * riR;
        const double Ht = (sL * HL + sR * HR) * ws;
        const double rt = sL * sR;
        const double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
        const double c2 = gm1 * (Ht - 0.5 * q2);
        const double c = sqrt(c2);
        const double un = s * ut[d];
        double du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
        const double dun = s * du[d];
        du[d] = 0.0;  // tangential part
        const double drho = qR[0] - qL[0], dp = pR - pL;
        const double i2c2 = 1.0 / (2.0 * c2);
        const double X = rt * c * dun;
        const double a1 = (dp - X) * i2c2;
        const double a2 = drho - dp / c2;
        const double a4 = (dp + X) * i2c2;
        const double e1 = un - c, e4 = un + c;
        const double l1 = fabs(e1) * a1, l2 = fabs(un), l4 = fabs(e4) * a4;
        const double w2 = l2 * a2, w3 = l2 * rt;
        const double cn = s * c;
        const double utdut = ut[0] * du[0] + ut[1] * du[1] + ut[2] * du[2];
        const double S = l1 + w2 + l4;

        // ---- backward: F -= diss / 2
        double db[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) db[v] = -0.5 * lam[v];
        double utb[3], dub[3];
        double Sb = db[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Sb += db[1 + k] * ut[k];
            utb[k] = db[1 + k] * S;
            dub[k] = db[1 + k] * (k == d ? 0.0 : w3);  // du[d] was zeroed
        }
        double w3b = db[1] * du[0] + db[2] * du[1] + db[3] * du[2];
        double l1b = -db[1 + d] * cn, l4b = db[1 + d] * cn;
        double cb = s * db[1 + d] * (l4 - l1);  // cn = s c
        // diss4 = l1 (Ht - c un) + w2 q2 / 2 + w3 utdut + l4 (Ht + c un)
        l1b += db[4] * (Ht - c * un);
        l4b += db[4] * (Ht + c * un);
        double Htb = db[4] * (l1 + l4);
        cb += db[4] * un * (l4 - l1);
        double unb = db[4] * c * (l4 - l1);
        double w2b = db[4] * 0.5 * q2;
        double q2b = db[4] * 0.5 * w2;
        w3b += db[4] * utdut;
        const double utdutb = db[4] * w3;
        // S = l1 + w2 + l4
        l1b += Sb;
        w2b += Sb;
        l4b += Sb;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            utb[k] += utdutb * du[k];
            dub[k] += k == d ? 0.0 : utdutb * ut[k];
        }
        // w3 = l2 rt, w2 = l2 a2
        double l2b = w3b * rt + w2b * a2;
        double rtb = w3b * l2;
        const double a2b = w2b * l2;
        // l4 = |e4| a4, l2 = |un|, l1 = |e1| a1
        const double a4b = l4b * fabs(e4), e4b = l4b * a4 * sgn(e4);
        const double a1b = l1b * fabs(e1), e1b = l1b * a1 * sgn(e1);
        unb += e4b + e1b + l2b * sgn(un);
        cb += e4b - e1b;
        // a4 = (dp + X) i2c2, a2 = drho - dp / c2, a1 = (dp - X) i2c2
        double dpb = (a4b + a1b) * i2c2 - a2b / c2;
        const double Xb = (a4b - a1b) * i2c2;
        const double i2c2b = a4b * (dp + X) + a1b * (dp - X);
        double c2b = a2b * dp / (c2 * c2) - 2.0 * i2c2 * i2c2 * i2c2b;
        const double drhob = a2b;
        // X = rt c dun
        rtb += Xb * c * dun;
        cb += Xb * rt * dun;
        const double dunb = Xb * rt * c;
        // drho, dp, du (dun = s du_d)
        gR[0] += drhob;
        gL[0] -= drhob;
        pRb += dpb;
        pLb -= dpb;
        dub[d] = s * dunb;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uRb[k] += dub[k];
            uLb[k] -= dub[k];
        }
        // un = s ut_d, c = sqrt(c2), c2 = gm1 (Ht - q2 / 2), q2 = |ut|^2
        utb[d] += s * unb;
        c2b += cb * 0.5 / c;
        Htb += gm1 * c2b;
        q2b -= 0.5 * gm1 * c2b;
#pragma unroll
        for (int k = 0; k < 3; ++k) utb[k] += 2.0 * ut[k] * q2b;
        // rt = sL sR, Ht = (sL HL + sR HR) ws, ut = (sL uL + sR uR) ws
        double sLb = rtb * sR + Htb * HL * ws, sRb = rtb * sL + Htb * HR * ws;
        double wsb = Htb * (sL * HL + sR * HR);
        const double HLb = Htb * sL * ws, HRb = Htb * sR * ws;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uLb[k] += utb[k] * sL * ws;
            uRb[k] += utb[k] * sR * ws;
            sLb += utb[k] * uL[k] * ws;
            sRb += utb[k] * uR[k] * ws;
            wsb += utb[k] * (sL * uL[k] + sR * uR[k]);
        }
        // HL = (qL4 + pL) riL
        gL[4] += HLb * riL;
        pLb += HLb * riL;
        riLb += HLb * (qL[4] + pL);
        gR[4] += HRb * riR;
        pRb += HRb * riR;
        riRb += HRb * (qR[4] + pR);
        // ws = 1 / (sL + sR), s = sqrt(rho)
        sLb -= ws * ws * wsb;
        sRb -= ws * ws * wsb;
        gL[0] += sLb * 0.5 / sL;
        gR[0] += sRb * 0.5 / sR;
    }
    // p = gm1 (q4 - rho |u|^2 / 2), u = q[1..3] ri, ri = 1 / rho
    gL[4] += gm1 * pLb;
    gL[0] -= 0.5 * gm1 * kL * pLb;
    gR[4] += gm1 * pRb;
    gR[0] -= 0.5 * gm1 * kR * pRb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        uLb[k] -= gm1 * qL[0] * uL[k] * pLb;
        uRb[k] -= gm1 * qR[0] * uR[k] * pRb;
        gL[1 + k] += uLb[k] * riL;
        gR[1 + k] += uRb[k] * riR;
        riLb += uLb[k] * qL[1 + k];
        riRb += uRb[k] * qR[1 + k];
    }
    gL[0] -= riL * riL * riLb;
    gR[0] -= riR * riR * riRb;
}

}  // namespace dgt
