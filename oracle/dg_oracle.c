/*
 * dg_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see dg_oracle.h).
 *
 * What it follows in arXiv 2210.03523:
 *   - DGSEM semi-discretisation, Section 2.1 (eqs. DGSEMsystem, DGMassMatrixLeft /
 *     DGMassMatrixRight): tensor-product Lagrange basis on Gauss-Lobatto nodes,
 *     collocated quadrature, diagonal mass matrix M = diag(J_j w_j).
 *   - New and traditional truncation-error forms, Section 2.2 (eqs. TEtildedef,
 *     TEdef): tau_new = M^-1 F^N(I q) - I F(q), tau_trad = M tau_new.
 *   - Isolated truncation error, end of Section 2.2: surface numerical fluxes
 *     replaced by the inner flux (all surface terms vanish on Gauss-Lobatto nodes).
 *   - Tau-estimation, Section 2.3: fine solution injected into every coarser
 *     anisotropic order; unsteady "variational DG" estimate of I F(q) by the
 *     sampled fine time derivative I (M^P)^-1 F^P(q^P).
 *   - Roe advective flux and Williamson low-storage RK3, Section 3 (set-up).
 *
 * The residual is written in the strong form, which on Gauss-Lobatto nodes is
 * algebraically identical to the weak form of Section 2.1 (summation by parts):
 *   J dQ/dt = -( sum_d D_d Ft^d + SAT ),   Ft^d = Ja^d . f(Q),
 *   SAT at a face node of face (d, s) = (F*_out - s Ft^d) / w_end.
 * Faces whose tangential orders differ are coupled on a mortar of order
 * K = max per tangential direction: both traces are interpolated onto the
 * mortar, the Riemann flux is evaluated once there (left = element on the
 * minus side; scaled normal = its Ja^d interpolated onto the mortar, e_d |Ja^d|
 * on box elements), and each side takes the L2 projection back onto its own
 * face nodes (the right side with a minus sign).  Curved elements carry their
 * metric terms per node (see elem_metrics).
 */
#include "dg_oracle.h"

#include <complex.h>
/* The name I is used for interpolation matrices below; the imaginary unit of the
 * complex-step derivatives is written _Complex_I. */
#undef I
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define NV 5

/* ------------------------------------------------------------------------ */
/* 1D Legendre-Gauss-Lobatto tables (computed once in long double).          */

static double g_x[ORC_NMAX + 1][ORC_NMAX + 1];
static double g_w[ORC_NMAX + 1][ORC_NMAX + 1];
static long double g_xl[ORC_NMAX + 1][ORC_NMAX + 1];
static long double g_lam[ORC_NMAX + 1][ORC_NMAX + 1];
static double g_D[ORC_NMAX + 1][(ORC_NMAX + 1) * (ORC_NMAX + 1)];
static int g_ready = 0;

/* Legendre polynomial L_N and its derivative at x (three-term recurrence). */
static void legendre(int N, long double x, long double *L, long double *dL)
{
    long double p0 = 1.0L, p1 = x, d0 = 0.0L, d1 = 1.0L;
    if (N == 0) { *L = 1.0L; *dL = 0.0L; return; }
    for (int k = 2; k <= N; ++k) {
        long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        long double d2 = d0 + (2 * k - 1) * p1;
        p0 = p1; p1 = p2; d0 = d1; d1 = d2;
    }
    *L = p1; *dL = d1;
}

static void build_tables(void)
{
    for (int N = 1; N <= ORC_NMAX; ++N) {
        long double *x = g_xl[N];
        x[0] = -1.0L; x[N] = 1.0L;
        /* interior nodes: roots of L'_N, Newton from Chebyshev-Lobatto guesses */
        for (int j = 1; j < N; ++j) {
            long double t = -cosl(3.14159265358979323846264338327950288L * j / N);
            for (int it = 0; it < 100; ++it) {
                long double L, dL;
                legendre(N, t, &L, &dL);
                /* (1-t^2) L'' = 2 t L' - N(N+1) L */
                long double d2 = (2.0L * t * dL - N * (N + 1.0L) * L) / (1.0L - t * t);
                long double dt = dL / d2;
                t -= dt;
                if (fabsl(dt) < 1e-30L) break;
            }
            x[j] = t;
        }
        /* enforce exact symmetry, and 0 at the centre for even N */
        for (int j = 0; j <= N / 2; ++j) {
            long double s = 0.5L * (x[N - j] - x[j]);
            x[j] = -s; x[N - j] = s;
        }
        if (N % 2 == 0) x[N / 2] = 0.0L;
        for (int j = 0; j <= N; ++j) {
            long double L, dL;
            legendre(N, x[j], &L, &dL);
            g_x[N][j] = (double)x[j];
            g_w[N][j] = (double)(2.0L / (N * (N + 1.0L) * L * L));
        }
        /* barycentric weights */
        for (int j = 0; j <= N; ++j) {
            long double p = 1.0L;
            for (int k = 0; k <= N; ++k)
                if (k != j) p *= (x[j] - x[k]);
            g_lam[N][j] = 1.0L / p;
        }
        /* derivative matrix D_jk = l_k'(x_j) */
        for (int j = 0; j <= N; ++j) {
            long double diag = 0.0L;
            for (int k = 0; k <= N; ++k) {
                if (k == j) continue;
                long double djk = (g_lam[N][k] / g_lam[N][j]) / (x[j] - x[k]);
                g_D[N][j * (N + 1) + k] = (double)djk;
                diag -= djk;
            }
            g_D[N][j * (N + 1) + j] = (double)diag;
        }
    }
    g_ready = 1;
}

static void ensure_tables(void)
{
    if (!g_ready) {
#pragma omp critical(orc_tables)
        if (!g_ready) build_tables();
    }
}

int orc_lgl(int N, double *x, double *w)
{
    if (N < 1 || N > ORC_NMAX) return -1;
    ensure_tables();
    for (int j = 0; j <= N; ++j) { x[j] = g_x[N][j]; w[j] = g_w[N][j]; }
    return 0;
}

int orc_dmat(int N, double *D)
{
    if (N < 1 || N > ORC_NMAX) return -1;
    ensure_tables();
    memcpy(D, g_D[N], sizeof(double) * (N + 1) * (N + 1));
    return 0;
}

/* Lagrange basis of order N evaluated at the order-M nodes (barycentric form). */
int orc_interp(int M, int N, double *I)
{
    if (M < 1 || M > ORC_NMAX || N < 1 || N > ORC_NMAX) return -1;
    ensure_tables();
    for (int a = 0; a <= M; ++a) {
        long double xa = g_xl[M][a];
        int hit = -1;
        for (int k = 0; k <= N; ++k)
            if (xa == g_xl[N][k]) hit = k;
        if (hit >= 0) {
            for (int k = 0; k <= N; ++k) I[a * (N + 1) + k] = (k == hit) ? 1.0 : 0.0;
            continue;
        }
        long double den = 0.0L;
        for (int k = 0; k <= N; ++k) den += g_lam[N][k] / (xa - g_xl[N][k]);
        for (int k = 0; k <= N; ++k)
            I[a * (N + 1) + k] = (double)((g_lam[N][k] / (xa - g_xl[N][k])) / den);
    }
    return 0;
}

/* L2 projection from order K onto order N <= K:  P = (S^T W_K S)^-1 S^T W_K,
 * S = interpolation from order N to the order-K nodes (an exact embedding). */
int orc_proj(int N, int K, double *P)
{
    if (N < 1 || K < N || K > ORC_NMAX) return -1;
    ensure_tables();
    int n = N + 1, k = K + 1;
    if (N == K) {
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) P[a * n + b] = (a == b) ? 1.0 : 0.0;
        return 0;
    }
    double S[(ORC_NMAX + 1) * (ORC_NMAX + 1)];
    orc_interp(K, N, S); /* k x n */
    long double A[ORC_NMAX + 1][ORC_NMAX + 1];       /* S^T W S  (n x n) */
    long double B[ORC_NMAX + 1][ORC_NMAX + 1];       /* S^T W    (n x k) */
    for (int a = 0; a < n; ++a) {
        for (int b = 0; b < n; ++b) {
            long double s = 0.0L;
            for (int q = 0; q < k; ++q) s += (long double)S[q * n + a] * g_w[K][q] * S[q * n + b];
            A[a][b] = s;
        }
        for (int q = 0; q < k; ++q) B[a][q] = (long double)S[q * n + a] * g_w[K][q];
    }
    /* Gauss-Jordan elimination with partial pivoting: A X = B */
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int r = c + 1; r < n; ++r)
            if (fabsl(A[r][c]) > fabsl(A[piv][c])) piv = r;
        if (piv != c) {
            for (int j = 0; j < n; ++j) { long double t = A[c][j]; A[c][j] = A[piv][j]; A[piv][j] = t; }
            for (int j = 0; j < k; ++j) { long double t = B[c][j]; B[c][j] = B[piv][j]; B[piv][j] = t; }
        }
        long double inv = 1.0L / A[c][c];
        for (int j = 0; j < n; ++j) A[c][j] *= inv;
        for (int j = 0; j < k; ++j) B[c][j] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            long double f = A[r][c];
            if (f == 0.0L) continue;
            for (int j = 0; j < n; ++j) A[r][j] -= f * A[c][j];
            for (int j = 0; j < k; ++j) B[r][j] -= f * B[c][j];
        }
    }
    for (int a = 0; a < n; ++a)
        for (int q = 0; q < k; ++q) P[a * k + q] = (double)B[a][q];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Physics: compressible Euler.                                              */

static double pressure(const double *q, double g)
{
    double ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    return (g - 1.0) * (q[4] - ke);
}

void orc_flux_n(const double *q, const double *n, double g, double *f)
{
    double rho = q[0];
    double u = q[1] / rho, v = q[2] / rho, w = q[3] / rho;
    double p = pressure(q, g);
    double un = u * n[0] + v * n[1] + w * n[2];
    f[0] = rho * un;
    f[1] = q[1] * un + p * n[0];
    f[2] = q[2] * un + p * n[1];
    f[3] = q[3] * un + p * n[2];
    f[4] = (q[4] + p) * un;
}

/* Roe's approximate Riemann solver: eigenvalues and wave vectors alpha_k r_k of
 * the Roe-averaged Jacobian, with both shear waves combined into one vector. */
void orc_roe_waves(const double *qL, const double *qR, const double *n, double g,
                   double *lam, double *wave)
{
    double rL = qL[0], rR = qR[0];
    double uL[3] = {qL[1] / rL, qL[2] / rL, qL[3] / rL};
    double uR[3] = {qR[1] / rR, qR[2] / rR, qR[3] / rR};
    double pL = pressure(qL, g), pR = pressure(qR, g);
    double HL = (qL[4] + pL) / rL, HR = (qR[4] + pR) / rR;
    double sL = sqrt(rL), sR = sqrt(rR);
    double ut[3];
    for (int d = 0; d < 3; ++d) ut[d] = (sL * uL[d] + sR * uR[d]) / (sL + sR);
    double Ht = (sL * HL + sR * HR) / (sL + sR);
    double rt = sL * sR;
    double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    double c2 = (g - 1.0) * (Ht - 0.5 * q2);
    double c = sqrt(c2);
    double un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
    double du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
    double dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
    double dut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
    double drho = rR - rL, dp = pR - pL;
    double a1 = (dp - rt * c * dun) / (2.0 * c2);
    double a2 = drho - dp / c2;
    double a4 = (dp + rt * c * dun) / (2.0 * c2);
    lam[0] = un - c; lam[1] = un; lam[2] = un; lam[3] = un + c;
    /* k = 1: acoustic wave moving with u_n - c */
    wave[0] = a1;
    for (int d = 0; d < 3; ++d) wave[1 + d] = a1 * (ut[d] - c * n[d]);
    wave[4] = a1 * (Ht - c * un);
    /* k = 2: entropy wave */
    wave[5] = a2;
    for (int d = 0; d < 3; ++d) wave[6 + d] = a2 * ut[d];
    wave[9] = a2 * 0.5 * q2;
    /* k = 3: both shear waves, strength rho~ */
    wave[10] = 0.0;
    for (int d = 0; d < 3; ++d) wave[11 + d] = rt * dut[d];
    wave[14] = rt * (ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2]);
    /* k = 4: acoustic wave moving with u_n + c */
    wave[15] = a4;
    for (int d = 0; d < 3; ++d) wave[16 + d] = a4 * (ut[d] + c * n[d]);
    wave[19] = a4 * (Ht + c * un);
}

void orc_numflux(const double *qL, const double *qR, const double *n, double g, int kind,
                 double *f)
{
    double fL[NV], fR[NV];
    orc_flux_n(qL, n, g, fL);
    orc_flux_n(qR, n, g, fR);
    if (kind == 0) {
        double lam[4], wave[20];
        orc_roe_waves(qL, qR, n, g, lam, wave);
        for (int v = 0; v < NV; ++v) {
            double diss = 0.0;
            for (int k = 0; k < 4; ++k) diss += fabs(lam[k]) * wave[k * NV + v];
            f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * diss;
        }
    } else {
        double rL = qL[0], rR = qR[0];
        double unL = (qL[1] * n[0] + qL[2] * n[1] + qL[3] * n[2]) / rL;
        double unR = (qR[1] * n[0] + qR[2] * n[1] + qR[3] * n[2]) / rR;
        double cL = sqrt(g * pressure(qL, g) / rL), cR = sqrt(g * pressure(qR, g) / rR);
        double s = fmax(fabs(unL) + cL, fabs(unR) + cR);
        for (int v = 0; v < NV; ++v) f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * s * (qR[v] - qL[v]);
    }
}

/* ------------------------------------------------------------------------ */
/* Mesh helpers.                                                             */

static int nnodes(const int *o) { return (o[0] + 1) * (o[1] + 1) * (o[2] + 1); }

long orc_num_nodes(int E, const int *orders)
{
    long s = 0;
    for (int e = 0; e < E; ++e) s += nnodes(orders + 3 * e);
    return s;
}

static long *node_offsets(int E, const int *orders)
{
    long *off = (long *)malloc(sizeof(long) * (E + 1));
    off[0] = 0;
    for (int e = 0; e < E; ++e) off[e + 1] = off[e] + nnodes(orders + 3 * e);
    return off;
}

static int check_orders(int E, const int *orders)
{
    for (int i = 0; i < 3 * E; ++i)
        if (orders[i] < 1 || orders[i] > ORC_NMAX) return -1;
    return 0;
}

static int check_mesh(const orc_mesh *m)
{
    if (m->nx < 1 || m->ny < 1 || m->nz < 1) return -1;
    if (m->map_kind == 0) return 0;
    if (m->map_kind != 1) return -1;
    for (int d = 0; d < 3; ++d)
        if (m->geo_order[d] < 1 || m->geo_order[d] > ORC_NMAX) return -1;
    return 0;
}

static void elem_ijk(const orc_mesh *m, int e, int *c)
{
    c[0] = e % m->nx;
    c[1] = (e / m->nx) % m->ny;
    c[2] = e / (m->nx * m->ny);
}

static int elem_index(const orc_mesh *m, const int *c) { return c[0] + m->nx * (c[1] + m->ny * c[2]); }

/* Affine geometry of a uniform box element: h_d, J = h1h2h3/8, |Ja^d| = J*2/h_d. */
static void geometry(const orc_mesh *m, double *h, double *J, double *Ja)
{
    int nd[3] = {m->nx, m->ny, m->nz};
    for (int d = 0; d < 3; ++d) h[d] = (m->hi[d] - m->lo[d]) / nd[d];
    *J = h[0] * h[1] * h[2] / 8.0;
    Ja[0] = h[1] * h[2] / 4.0;
    Ja[1] = h[0] * h[2] / 4.0;
    Ja[2] = h[0] * h[1] / 4.0;
}

/* The curvilinear map (map_kind 1): (x, y, z) -> (x + f, y + f, z). */
static void map_point(const orc_mesh *m, const double *xb, double *X)
{
    const double twopi = 6.28318530717958647692528676655900577;
    double f = m->map_amp * sin(twopi * (xb[0] - m->lo[0]) / (m->hi[0] - m->lo[0])) *
               sin(twopi * (xb[1] - m->lo[1]) / (m->hi[1] - m->lo[1]));
    X[0] = xb[0] + f;
    X[1] = xb[1] + f;
    X[2] = xb[2];
}

/* Node coordinates of element e at orders o: X[d*ne + node].  Box elements: the
 * affine map of the reference cube.  Curved elements: the map sampled at the
 * Gauss-Lobatto nodes of the geometry order, interpolated to the element's nodes. */
static void elem_coords(const orc_mesh *m, const int *o, int e, double *X)
{
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    int c[3];
    elem_ijk(m, e, c);
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    if (m->map_kind == 0) {
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    int node = i + n[0] * (j + n[1] * k);
                    int idx[3] = {i, j, k};
                    for (int d = 0; d < 3; ++d)
                        X[d * ne + node] = m->lo[d] + h[d] * (c[d] + 0.5 * (g_x[o[d]][idx[d]] + 1.0));
                }
        return;
    }
    const int *G = m->geo_order;
    int g[3] = {G[0] + 1, G[1] + 1, G[2] + 1}, ng = g[0] * g[1] * g[2];
    double *P = malloc(sizeof(double) * 3 * ng);
    for (int kc = 0; kc < g[2]; ++kc)
        for (int kb = 0; kb < g[1]; ++kb)
            for (int ka = 0; ka < g[0]; ++ka) {
                int gi[3] = {ka, kb, kc};
                double xb[3], Xm[3];
                for (int d = 0; d < 3; ++d) xb[d] = m->lo[d] + h[d] * (c[d] + 0.5 * (g_x[G[d]][gi[d]] + 1.0));
                map_point(m, xb, Xm);
                for (int d = 0; d < 3; ++d) P[d * ng + ka + g[0] * (kb + g[1] * kc)] = Xm[d];
            }
    double I1[(ORC_NMAX + 1) * (ORC_NMAX + 1)], I2[(ORC_NMAX + 1) * (ORC_NMAX + 1)],
        I3[(ORC_NMAX + 1) * (ORC_NMAX + 1)];
    orc_interp(o[0], G[0], I1);
    orc_interp(o[1], G[1], I2);
    orc_interp(o[2], G[2], I3);
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    double acc = 0.0;
                    for (int kc = 0; kc < g[2]; ++kc)
                        for (int kb = 0; kb < g[1]; ++kb)
                            for (int ka = 0; ka < g[0]; ++ka)
                                acc += I1[i * g[0] + ka] * I2[j * g[1] + kb] * I3[k * g[2] + kc] *
                                       P[d * ng + ka + g[0] * (kb + g[1] * kc)];
                    X[d * ne + i + n[0] * (j + n[1] * k)] = acc;
                }
    free(P);
}

/* Metric terms from node coordinates: covariant vectors a_i = D_i X (collocation
 * derivative along reference direction i), contravariant Ja^1 = a_2 x a_3,
 * Ja^2 = a_3 x a_1, Ja^3 = a_1 x a_2, Jacobian J = a_1 . (a_2 x a_3).
 * Ja[(d*3 + l)*ne + node] = (Ja^d)_l.  For maps whose third coordinate is an affine
 * function of the third reference coordinate alone (the box and the sine map), this
 * cross-product form satisfies the discrete metric identities sum_d D_d (Ja^d)_l = 0
 * up to rounding, which free-stream preservation needs. */
static void metrics_from_coords(const int *o, const double *X, double *Ja, double *J)
{
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int idx[3] = {i, j, k};
                int node = i + n[0] * (j + n[1] * k);
                double a[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int c = 0; c < 3; ++c) {
                        double acc = 0.0;
                        for (int q = 0; q < n[r]; ++q) {
                            int id2[3] = {i, j, k};
                            id2[r] = q;
                            acc += g_D[o[r]][idx[r] * n[r] + q] * X[c * ne + id2[0] + n[0] * (id2[1] + n[1] * id2[2])];
                        }
                        a[r][c] = acc;
                    }
                for (int d = 0; d < 3; ++d) {
                    const double *p = a[(d + 1) % 3], *q = a[(d + 2) % 3];
                    Ja[(d * 3 + 0) * ne + node] = p[1] * q[2] - p[2] * q[1];
                    Ja[(d * 3 + 1) * ne + node] = p[2] * q[0] - p[0] * q[2];
                    Ja[(d * 3 + 2) * ne + node] = p[0] * q[1] - p[1] * q[0];
                }
                J[node] = a[0][0] * Ja[0 * ne + node] + a[0][1] * Ja[1 * ne + node] + a[0][2] * Ja[2 * ne + node];
            }
}

/* Metric terms of element e at orders o (box elements: the closed forms). */
static void elem_metrics(const orc_mesh *m, const int *o, int e, double *Ja, double *J)
{
    int ne = nnodes(o);
    if (m->map_kind == 0) {
        double h[3], Jm, Jd[3];
        geometry(m, h, &Jm, Jd);
        for (int x = 0; x < ne; ++x) {
            J[x] = Jm;
            for (int d = 0; d < 3; ++d)
                for (int l = 0; l < 3; ++l) Ja[(d * 3 + l) * ne + x] = (l == d) ? Jd[d] : 0.0;
        }
        return;
    }
    double *X = malloc(sizeof(double) * 3 * ne);
    elem_coords(m, o, e, X);
    metrics_from_coords(o, X, Ja, J);
    free(X);
}

int orc_node_coords(const orc_mesh *m, const int *orders, double *xyz)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders)) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e) elem_coords(m, orders + 3 * e, e, xyz + 3 * off[e]);
    free(off);
    return 0;
}

int orc_metrics(const orc_mesh *m, const int *orders, double *met)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders)) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e) {
        int ne = nnodes(orders + 3 * e);
        double *M = met + 10 * off[e];
        elem_metrics(m, orders + 3 * e, e, M, M + 9 * ne);
    }
    free(off);
    return 0;
}

/* Volume node index of face node (a,b) on face (d, side). */
static int face_node(const int *n, int d, int side, int a, int b)
{
    int idx[3];
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    idx[d] = side > 0 ? n[d] - 1 : 0;
    idx[t1] = a;
    idx[t2] = b;
    return idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
}

/* Neighbour of element e across face (d, s): returns its index, or -1 with *bc set. */
static int neighbour(const orc_mesh *m, int e, int d, int s, int *bc)
{
    int c[3], nd[3] = {m->nx, m->ny, m->nz};
    elem_ijk(m, e, c);
    c[d] += s;
    *bc = 0;
    if (c[d] < 0 || c[d] >= nd[d]) {
        *bc = m->bc[2 * d + (s > 0 ? 1 : 0)];
        if (*bc != 0) return -1;
        c[d] = (c[d] + nd[d]) % nd[d];
    }
    return elem_index(m, c);
}

/* Ghost state of a boundary face with unit outward normal nout: slip wall (the
 * normal momentum mirrored) or far field (the free stream). */
static void ghost_state(const orc_mesh *m, int bc, const double *nout, const double *qin, double *qg)
{
    if (bc == 1) {
        double mn = qin[1] * nout[0] + qin[2] * nout[1] + qin[3] * nout[2];
        qg[0] = qin[0];
        for (int k = 0; k < 3; ++k) qg[1 + k] = qin[1 + k] - 2.0 * mn * nout[k];
        qg[4] = qin[4];
    } else {
        for (int v = 0; v < NV; ++v) qg[v] = m->qfar[v];
    }
}

/* Interpolate a face trace (nv fields of na*nb nodes, field stride na*nb) onto
 * the K1 x K2 mortar: out[v*K1*K2 + A + K1*B]. */
static void to_mortar(int nv, int na, int nb, int K1, int K2, const double *in, double *out)
{
    double *S1 = malloc(sizeof(double) * K1 * na), *S2 = malloc(sizeof(double) * K2 * nb);
    orc_interp(K1 - 1, na - 1, S1);
    orc_interp(K2 - 1, nb - 1, S2);
    for (int v = 0; v < nv; ++v)
        for (int B = 0; B < K2; ++B)
            for (int A = 0; A < K1; ++A) {
                double acc = 0.0;
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) acc += S1[A * na + a] * S2[B * nb + b] * in[v * na * nb + a + na * b];
                out[v * K1 * K2 + A + K1 * B] = acc;
            }
    free(S1);
    free(S2);
}

/* L2 projection of nv mortar fields back onto an na x nb face. */
static void from_mortar(int nv, int na, int nb, int K1, int K2, const double *in, double *out)
{
    double *P1 = malloc(sizeof(double) * na * K1), *P2 = malloc(sizeof(double) * nb * K2);
    orc_proj(na - 1, K1 - 1, P1);
    orc_proj(nb - 1, K2 - 1, P2);
    for (int v = 0; v < nv; ++v)
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < na; ++a) {
                double acc = 0.0;
                for (int B = 0; B < K2; ++B)
                    for (int A = 0; A < K1; ++A) acc += P1[a * K1 + A] * P2[b * K2 + B] * in[v * K1 * K2 + A + K1 * B];
                out[v * na * nb + a + na * b] = acc;
            }
    free(P1);
    free(P2);
}

/* Gather the face trace of nv fields (field stride ne) of element data X on face (d, s). */
static void face_trace(const int *n, int d, int s, int nv, const double *X, double *out)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    int na = n[t1], nb = n[t2], ne = n[0] * n[1] * n[2];
    for (int v = 0; v < nv; ++v)
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < na; ++a) out[v * na * nb + a + na * b] = X[v * ne + face_node(n, d, s, a, b)];
}

/* Scaled normal of a face on its mortar, mK[c*K1*K2 + x] (c = x, y, z): the minus-side
 * element's Ja^d (outward from it) interpolated onto the mortar nodes.  Box elements:
 * the constant |Ja^d| e_d. */
static void mortar_metric(const orc_mesh *m, const int *oL, int eL, int d, int K1, int K2, double *mK)
{
    int KK = K1 * K2;
    if (m->map_kind == 0) {
        double h[3], J, Ja[3];
        geometry(m, h, &J, Ja);
        for (int c = 0; c < 3; ++c)
            for (int x = 0; x < KK; ++x) mK[c * KK + x] = (c == d) ? Ja[d] : 0.0;
        return;
    }
    int n[3] = {oL[0] + 1, oL[1] + 1, oL[2] + 1}, ne = n[0] * n[1] * n[2];
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    double *Ja = malloc(sizeof(double) * 9 * ne), *J = malloc(sizeof(double) * ne);
    double *tr = malloc(sizeof(double) * 3 * n[t1] * n[t2]);
    elem_metrics(m, oL, eL, Ja, J);
    face_trace(n, d, +1, 3, Ja + 3 * d * ne, tr);
    to_mortar(3, n[t1], n[t2], K1, K2, tr, mK);
    free(Ja); free(J); free(tr);
}

/* Split a scaled normal into its length and the unit normal. */
static double unit_normal(const double *mv, double *nh)
{
    double len = sqrt(mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2]);
    for (int c = 0; c < 3; ++c) nh[c] = mv[c] / len;
    return len;
}

/* ------------------------------------------------------------------------ */
/* Residual: contravariant fluxes, volume term, surface terms.               */

/* Contravariant flux Ft^d = sum_l (Ja^d)_l (f^a_l - f^v_l) at every node,
 * Ft[(d*NV + v)*ne + node].  G (nullable: Euler) holds the gradients [3][5][node]. */
static void contravariant_flux(const orc_mesh *m, const int *o, const double *Q, const double *G, double mu,
                               double Pr, const double *Ja, double *Ft)
{
    int ne = nnodes(o);
    for (int node = 0; node < ne; ++node) {
        double q[NV], f[3][NV], Gn[3 * NV];
        for (int v = 0; v < NV; ++v) q[v] = Q[v * ne + node];
        if (G)
            for (int l = 0; l < 3; ++l)
                for (int v = 0; v < NV; ++v) Gn[5 * l + v] = G[(l * NV + v) * ne + node];
        for (int l = 0; l < 3; ++l) {
            double el[3] = {0, 0, 0};
            el[l] = 1.0;
            orc_flux_n(q, el, m->gamma, f[l]);
            if (G) {
                double fv[NV];
                orc_viscous_flux(q, Gn, l, m->gamma, mu, Pr, fv);
                for (int v = 0; v < NV; ++v) f[l][v] = f[l][v] - fv[v];
            }
        }
        for (int d = 0; d < 3; ++d)
            for (int v = 0; v < NV; ++v) {
                double acc = 0.0;
                for (int l = 0; l < 3; ++l) acc += Ja[(d * 3 + l) * ne + node] * f[l][v];
                Ft[(d * NV + v) * ne + node] = acc;
            }
    }
}

/* Volume term V = sum_d D^{N_d} Ft^d along direction d, V[v*ne + node]. */
static void volume_term(const int *o, const double *Ft, double *V)
{
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int node = i + n[0] * (j + n[1] * k);
                for (int v = 0; v < NV; ++v) {
                    double acc = 0.0;
                    for (int q = 0; q < n[0]; ++q)
                        acc += g_D[o[0]][i * n[0] + q] * Ft[(0 * NV + v) * ne + q + n[0] * (j + n[1] * k)];
                    for (int q = 0; q < n[1]; ++q)
                        acc += g_D[o[1]][j * n[1] + q] * Ft[(1 * NV + v) * ne + i + n[0] * (q + n[1] * k)];
                    for (int q = 0; q < n[2]; ++q)
                        acc += g_D[o[2]][k * n[2] + q] * Ft[(2 * NV + v) * ne + i + n[0] * (j + n[1] * q)];
                    V[v * ne + node] = acc;
                }
            }
}

/* Outward numerical flux F*_out at the own face nodes of face (d, s) of element e:
 * fout[v*(na*nb) + a + na*b].  JaOwn: the element's metric terms.  With G (the
 * gradients, Navier-Stokes) the BR1 viscous trace is subtracted:
 *   F* = |m| [ f*(Q_L, Q_R, n) - (1/2) sum_l n_l (f^v_l(Q_L, G_L) + f^v_l(Q_R, G_R)) ],
 * with m the scaled normal (Ja^d of the minus side on the mortar), n = m/|m|; at
 * boundaries the ghost state carries the inner gradient. */
static void face_flux(const orc_mesh *m, const int *orders, const long *off, const double *u,
                      const double *grad, double mu, double Pr, int e, int d, int s, const double *JaOwn,
                      double *fout)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1};
    int na = n[t1], nb = n[t2], ne = n[0] * n[1] * n[2];
    const int nf = grad ? 4 * NV : NV; /* Q (and the three gradient components) */
    double g = m->gamma;
    double *own = malloc(sizeof(double) * nf * na * nb);
    face_trace(n, d, s, NV, u + NV * off[e], own);
    if (grad) face_trace(n, d, s, 3 * NV, grad + 3 * NV * off[e], own + NV * na * nb);

    int bc;
    int nbr = neighbour(m, e, d, s, &bc);
    if (nbr < 0) {
        double *mo = malloc(sizeof(double) * 3 * na * nb);
        face_trace(n, d, s, 3, JaOwn + 3 * d * ne, mo);
        for (int x = 0; x < na * nb; ++x) {
            double mv[3], nh[3], qin[NV], qg[NV], fa[NV], Gin[3 * NV];
            for (int c = 0; c < 3; ++c) mv[c] = (double)s * mo[c * na * nb + x];
            double len = unit_normal(mv, nh);
            for (int v = 0; v < NV; ++v) qin[v] = own[v * na * nb + x];
            ghost_state(m, bc, nh, qin, qg);
            orc_numflux(qin, qg, nh, g, m->flux, fa);
            if (grad) {
                double vs[NV] = {0, 0, 0, 0, 0};
                for (int c = 0; c < 3 * NV; ++c) Gin[c] = own[(NV + c) * na * nb + x];
                for (int l = 0; l < 3; ++l) {
                    double fv1[NV], fv2[NV];
                    orc_viscous_flux(qin, Gin, l, g, mu, Pr, fv1);
                    orc_viscous_flux(qg, Gin, l, g, mu, Pr, fv2);
                    for (int v = 0; v < NV; ++v) vs[v] += nh[l] * (fv1[v] + fv2[v]);
                }
                for (int v = 0; v < NV; ++v) fout[v * na * nb + x] = len * (fa[v] - 0.5 * vs[v]);
            } else {
                for (int v = 0; v < NV; ++v) fout[v * na * nb + x] = len * fa[v];
            }
        }
        free(mo);
        free(own);
        return;
    }

    const int *on = orders + 3 * nbr;
    int nn[3] = {on[0] + 1, on[1] + 1, on[2] + 1};
    int ma = nn[t1], mb = nn[t2];
    double *oth = malloc(sizeof(double) * nf * ma * mb);
    face_trace(nn, d, -s, NV, u + NV * off[nbr], oth);
    if (grad) face_trace(nn, d, -s, 3 * NV, grad + 3 * NV * off[nbr], oth + NV * ma * mb);
    int K1 = na > ma ? na : ma, K2 = nb > mb ? nb : mb, KK = K1 * K2;
    double *A = malloc(sizeof(double) * nf * KK), *B = malloc(sizeof(double) * nf * KK);
    to_mortar(nf, na, nb, K1, K2, own, A);
    to_mortar(nf, ma, mb, K1, K2, oth, B);
    /* left = element on the minus side of the face, right = plus side */
    double *L = s > 0 ? A : B, *R = s > 0 ? B : A;
    double *mK = malloc(sizeof(double) * 3 * KK);
    if (s > 0) mortar_metric(m, o, e, d, K1, K2, mK);
    else mortar_metric(m, on, nbr, d, K1, K2, mK);
    double *FK = malloc(sizeof(double) * NV * KK);
    for (int x = 0; x < KK; ++x) {
        double mv[3] = {mK[x], mK[KK + x], mK[2 * KK + x]}, nh[3];
        double len = unit_normal(mv, nh);
        double qL[NV], qR[NV], fa[NV];
        for (int v = 0; v < NV; ++v) {
            qL[v] = L[v * KK + x];
            qR[v] = R[v * KK + x];
        }
        orc_numflux(qL, qR, nh, g, m->flux, fa);
        if (grad) {
            double GL[3 * NV], GR[3 * NV], vs[NV] = {0, 0, 0, 0, 0};
            for (int c = 0; c < 3 * NV; ++c) {
                GL[c] = L[(NV + c) * KK + x];
                GR[c] = R[(NV + c) * KK + x];
            }
            for (int l = 0; l < 3; ++l) {
                double fvL[NV], fvR[NV];
                orc_viscous_flux(qL, GL, l, g, mu, Pr, fvL);
                orc_viscous_flux(qR, GR, l, g, mu, Pr, fvR);
                for (int v = 0; v < NV; ++v) vs[v] += nh[l] * (fvL[v] + fvR[v]);
            }
            for (int v = 0; v < NV; ++v) FK[v * KK + x] = len * (fa[v] - 0.5 * vs[v]);
        } else {
            for (int v = 0; v < NV; ++v) FK[v * KK + x] = len * fa[v];
        }
    }
    /* project back onto the own face (L2 projection), outward sign */
    from_mortar(NV, na, nb, K1, K2, FK, fout);
    for (int x = 0; x < NV * na * nb; ++x) fout[x] *= (double)s;
    free(own); free(oth); free(A); free(B); free(mK); free(FK);
}

/* Residual of one element of orders o with data Q (natural layout of element e):
 * r = (V + SAT)/J (form 0) or w_i w_j w_k (V + SAT) (form 1).  G: gradients (NS) or
 * NULL (Euler).  Surface terms need the whole mesh (orders, off, u, grad); isolated
 * evaluations pass isolated = 1 and may leave those NULL. */
static void residual_core(const orc_mesh *m, const int *orders, const long *off, const double *u,
                          const double *grad, double mu, double Pr, const int *o, int e, const double *Q,
                          const double *G, int form, int isolated, double *r)
{
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    double *Ja = malloc(sizeof(double) * 9 * ne), *Jn = malloc(sizeof(double) * ne);
    elem_metrics(m, o, e, Ja, Jn);
    double *Ft = malloc(sizeof(double) * 3 * NV * ne);  /* [d][v][node] */
    double *V = malloc(sizeof(double) * NV * ne);       /* [v][node] */
    contravariant_flux(m, o, Q, G, mu, Pr, Ja, Ft);
    volume_term(o, Ft, V);
    if (!isolated) {
        for (int d = 0; d < 3; ++d) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int na = n[t1], nb = n[t2];
            double wend = g_w[o[d]][0];
            double *fout = malloc(sizeof(double) * NV * na * nb);
            for (int s = -1; s <= 1; s += 2) {
                face_flux(m, orders, off, u, grad, mu, Pr, e, d, s, Ja, fout);
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) {
                        int node = face_node(n, d, s, a, b);
                        for (int v = 0; v < NV; ++v)
                            V[v * ne + node] += (fout[v * na * nb + a + na * b] -
                                                 (double)s * Ft[(d * NV + v) * ne + node]) / wend;
                    }
            }
            free(fout);
        }
    }
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int node = i + n[0] * (j + n[1] * k);
                double www = g_w[o[0]][i] * g_w[o[1]][j] * g_w[o[2]][k];
                for (int v = 0; v < NV; ++v)
                    r[v * ne + node] = form == 0 ? V[v * ne + node] / Jn[node] : www * V[v * ne + node];
            }
    free(Ja); free(Jn); free(Ft); free(V);
}

int orc_residual(const orc_mesh *m, const int *orders, const double *u, double *r, int form,
                 int isolated)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders) || (form != 0 && form != 1)) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e)
        residual_core(m, orders, off, u, NULL, 0.0, 0.0, orders + 3 * e, e, u + NV * off[e], NULL, form, isolated,
                      r + NV * off[e]);
    free(off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Navier-Stokes: BR1 gradients and viscous fluxes.                           */

void orc_viscous_flux(const double *q, const double *G, int d, double g, double mu, double Pr, double *f)
{
    double rho = q[0], u[3] = {q[1] / q[0], q[2] / q[0], q[3] / q[0]};
    double p = pressure(q, g), T = p / rho;
    double du[3][3]; /* du[k][l] = d u_k / d x_l */
    double dT[3];
    for (int l = 0; l < 3; ++l) {
        const double *Gl = G + 5 * l;
        for (int k = 0; k < 3; ++k) du[k][l] = (Gl[1 + k] - u[k] * Gl[0]) / rho;
        double dp = (g - 1.0) * (Gl[4] - (u[0] * Gl[1] + u[1] * Gl[2] + u[2] * Gl[3]) +
                                 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * Gl[0]);
        dT[l] = (dp - T * Gl[0]) / rho;
    }
    double div = du[0][0] + du[1][1] + du[2][2];
    double tau[3]; /* tau[k] = tau_{k d} */
    for (int k = 0; k < 3; ++k) tau[k] = mu * (du[k][d] + du[d][k]) - (k == d ? 2.0 / 3.0 * mu * div : 0.0);
    double kappa = mu * g / ((g - 1.0) * Pr);
    f[0] = 0.0;
    for (int k = 0; k < 3; ++k) f[1 + k] = tau[k];
    f[4] = u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + kappa * dT[d];
}

/* BR1 surface data of face (d, s) of element e on its own face nodes, for the
 * gradient pass.  qhat = (1/2)(Q_in + Q_out) on the mortar (the ghost state at
 * boundaries).  Box elements: out[v][node] = qhat projected back (the metric is the
 * constant |Ja^d| e_d and is applied by the caller).  Curved elements:
 * out[(l*NV + v)][node] = s P[qhat m_l], the outward scaled normal m (Ja^d of the
 * minus side on the mortar) multiplied in before the projection, l = x, y, z. */
static void br1_face(const orc_mesh *m, const int *orders, const long *off, const double *u, int e, int d, int s,
                     const double *JaOwn, double *out)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1};
    int na = n[t1], nb = n[t2], ne = n[0] * n[1] * n[2], F = na * nb;
    const int curved = m->map_kind != 0;
    double *own = malloc(sizeof(double) * NV * F);
    face_trace(n, d, s, NV, u + NV * off[e], own);
    int bc;
    int nbr = neighbour(m, e, d, s, &bc);
    if (nbr < 0) {
        double *mo = malloc(sizeof(double) * 3 * F);
        face_trace(n, d, s, 3, JaOwn + 3 * d * ne, mo);
        for (int x = 0; x < F; ++x) {
            double qin[NV], qg[NV], mv[3], nh[3];
            for (int c = 0; c < 3; ++c) mv[c] = (double)s * mo[c * F + x];
            unit_normal(mv, nh);
            for (int v = 0; v < NV; ++v) qin[v] = own[v * F + x];
            ghost_state(m, bc, nh, qin, qg);
            for (int v = 0; v < NV; ++v) {
                double qh = 0.5 * (qin[v] + qg[v]);
                if (!curved) out[v * F + x] = qh;
                else
                    for (int l = 0; l < 3; ++l) out[(l * NV + v) * F + x] = qh * mv[l];
            }
        }
        free(mo);
        free(own);
        return;
    }
    const int *on = orders + 3 * nbr;
    int nn[3] = {on[0] + 1, on[1] + 1, on[2] + 1};
    int ma = nn[t1], mb = nn[t2];
    int K1 = na > ma ? na : ma, K2 = nb > mb ? nb : mb, KK = K1 * K2;
    double *oth = malloc(sizeof(double) * NV * ma * mb);
    face_trace(nn, d, -s, NV, u + NV * off[nbr], oth);
    double *A = malloc(sizeof(double) * NV * KK), *B = malloc(sizeof(double) * NV * KK);
    to_mortar(NV, na, nb, K1, K2, own, A);
    to_mortar(NV, ma, mb, K1, K2, oth, B);
    for (int x = 0; x < NV * KK; ++x) A[x] = 0.5 * (A[x] + B[x]);
    if (!curved) {
        from_mortar(NV, na, nb, K1, K2, A, out);
    } else {
        double *mK = malloc(sizeof(double) * 3 * KK), *prod = malloc(sizeof(double) * 3 * NV * KK);
        if (s > 0) mortar_metric(m, o, e, d, K1, K2, mK);
        else mortar_metric(m, on, nbr, d, K1, K2, mK);
        for (int l = 0; l < 3; ++l)
            for (int v = 0; v < NV; ++v)
                for (int x = 0; x < KK; ++x) prod[(l * NV + v) * KK + x] = (double)s * A[v * KK + x] * mK[l * KK + x];
        from_mortar(3 * NV, na, nb, K1, K2, prod, out);
        free(mK);
        free(prod);
    }
    free(own); free(oth); free(A); free(B);
}

/* BR1 gradient of element e (orders o, data Q), grad[(l*NV + v)*ne + node] = d(var v)/dx_l.
 *   Box elements:    J dQ/dx_l = |Ja^l| [ D_l Q + sum_s s (qhat - Q) / w_end on the l-faces ].
 *   Curved elements: J dQ/dx_l = sum_d D_d[(Ja^d)_l Q]
 *                                + sum over faces (d, s) of (s P[qhat m_l] - Q s (Ja^d)_l) / w_end.
 * isolated drops the surface terms (then orders, off and u may be NULL). */
static void gradient_core(const orc_mesh *m, const int *orders, const long *off, const double *u, const int *o,
                          int e, const double *Q, int isolated, double *grad)
{
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    if (m->map_kind == 0) {
        double h[3], J, Ja[3];
        geometry(m, h, &J, Ja);
        double *Jfull = NULL;
        if (!isolated) {
            Jfull = malloc(sizeof(double) * 10 * ne);
            elem_metrics(m, o, e, Jfull, Jfull + 9 * ne);
        }
        for (int l = 0; l < 3; ++l) {
            double *Gl = grad + (size_t)l * NV * ne;
            for (int k = 0; k < n[2]; ++k)
                for (int j = 0; j < n[1]; ++j)
                    for (int i = 0; i < n[0]; ++i) {
                        int idx[3] = {i, j, k};
                        int node = i + n[0] * (j + n[1] * k);
                        for (int v = 0; v < NV; ++v) {
                            double acc = 0.0;
                            for (int q = 0; q < n[l]; ++q) {
                                int id2[3] = {i, j, k};
                                id2[l] = q;
                                acc += g_D[o[l]][idx[l] * n[l] + q] * Q[v * ne + id2[0] + n[0] * (id2[1] + n[1] * id2[2])];
                            }
                            Gl[v * ne + node] = acc;
                        }
                    }
            if (!isolated) {
                int t1 = (l == 0) ? 1 : 0, t2 = (l == 2) ? 1 : 2;
                int na = n[t1], nb = n[t2];
                double *qh = malloc(sizeof(double) * NV * na * nb);
                for (int s = -1; s <= 1; s += 2) {
                    br1_face(m, orders, off, u, e, l, s, Jfull, qh);
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < na; ++a) {
                            int node = face_node(n, l, s, a, b);
                            for (int v = 0; v < NV; ++v)
                                Gl[v * ne + node] += (double)s * (qh[v * na * nb + a + na * b] - Q[v * ne + node]) /
                                                     g_w[o[l]][0];
                        }
                }
                free(qh);
            }
            for (int x = 0; x < NV * ne; ++x) Gl[x] *= Ja[l] / J;
        }
        free(Jfull);
        return;
    }
    double *Ja = malloc(sizeof(double) * 9 * ne), *Jn = malloc(sizeof(double) * ne);
    double *P = malloc(sizeof(double) * NV * ne);
    elem_metrics(m, o, e, Ja, Jn);
    for (int l = 0; l < 3; ++l) {
        double *Gl = grad + (size_t)l * NV * ne;
        for (int x = 0; x < NV * ne; ++x) Gl[x] = 0.0;
        for (int d = 0; d < 3; ++d) {
            /* P = (Ja^d)_l Q, differentiated along d */
            for (int v = 0; v < NV; ++v)
                for (int x = 0; x < ne; ++x) P[v * ne + x] = Ja[(d * 3 + l) * ne + x] * Q[v * ne + x];
            for (int k = 0; k < n[2]; ++k)
                for (int j = 0; j < n[1]; ++j)
                    for (int i = 0; i < n[0]; ++i) {
                        int idx[3] = {i, j, k};
                        int node = i + n[0] * (j + n[1] * k);
                        for (int v = 0; v < NV; ++v) {
                            double acc = 0.0;
                            for (int q = 0; q < n[d]; ++q) {
                                int id2[3] = {i, j, k};
                                id2[d] = q;
                                acc += g_D[o[d]][idx[d] * n[d] + q] * P[v * ne + id2[0] + n[0] * (id2[1] + n[1] * id2[2])];
                            }
                            Gl[v * ne + node] += acc;
                        }
                    }
        }
    }
    if (!isolated) {
        for (int d = 0; d < 3; ++d) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int na = n[t1], nb = n[t2], F = na * nb;
            double *bf = malloc(sizeof(double) * 3 * NV * F);
            for (int s = -1; s <= 1; s += 2) {
                br1_face(m, orders, off, u, e, d, s, Ja, bf);
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) {
                        int node = face_node(n, d, s, a, b);
                        for (int l = 0; l < 3; ++l) {
                            double ml = (double)s * Ja[(d * 3 + l) * ne + node];
                            for (int v = 0; v < NV; ++v)
                                grad[(l * NV + v) * ne + node] +=
                                    (bf[(l * NV + v) * F + a + na * b] - Q[v * ne + node] * ml) / g_w[o[d]][0];
                        }
                    }
            }
            free(bf);
        }
    }
    for (int l = 0; l < 3; ++l)
        for (int v = 0; v < NV; ++v)
            for (int x = 0; x < ne; ++x) grad[(l * NV + v) * ne + x] /= Jn[x];
    free(Ja); free(Jn); free(P);
}

int orc_gradient(const orc_mesh *m, const int *orders, const double *u, int isolated, double *grad)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders)) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e)
        gradient_core(m, orders, off, u, orders + 3 * e, e, u + NV * off[e], isolated, grad + 3 * NV * off[e]);
    free(off);
    return 0;
}

int orc_residual_ns(const orc_mesh *m, const int *orders, const double *u, double mu, double Pr, double *r,
                    int form, int isolated)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders) || (form != 0 && form != 1)) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
    double *grad = malloc(sizeof(double) * 3 * NV * off[E]);
    orc_gradient(m, orders, u, isolated, grad);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e)
        residual_core(m, orders, off, u, grad, mu, Pr, orders + 3 * e, e, u + NV * off[e], grad + 3 * NV * off[e],
                      form, isolated, r + NV * off[e]);
    free(grad);
    free(off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Tau-estimation.                                                           */

/* Sample the order-(nf) element polynomial at the order-(nc) nodes:
 * out[a,b,c] = sum_{i,j,k} I1[a,i] I2[b,j] I3[c,k] in[i,j,k], for each variable. */
static void restrict_element(const int *of, const int *oc, const double *in, double *out)
{
    int nf[3] = {of[0] + 1, of[1] + 1, of[2] + 1};
    int nc[3] = {oc[0] + 1, oc[1] + 1, oc[2] + 1};
    int nef = nf[0] * nf[1] * nf[2], nec = nc[0] * nc[1] * nc[2];
    double I1[(ORC_NMAX + 1) * (ORC_NMAX + 1)], I2[(ORC_NMAX + 1) * (ORC_NMAX + 1)],
        I3[(ORC_NMAX + 1) * (ORC_NMAX + 1)];
    orc_interp(oc[0], of[0], I1);
    orc_interp(oc[1], of[1], I2);
    orc_interp(oc[2], of[2], I3);
    for (int v = 0; v < NV; ++v)
        for (int c = 0; c < nc[2]; ++c)
            for (int b = 0; b < nc[1]; ++b)
                for (int a = 0; a < nc[0]; ++a) {
                    double acc = 0.0;
                    for (int k = 0; k < nf[2]; ++k)
                        for (int j = 0; j < nf[1]; ++j)
                            for (int i = 0; i < nf[0]; ++i)
                                acc += I1[a * nf[0] + i] * I2[b * nf[1] + j] * I3[c * nf[2] + k] *
                                       in[v * nef + i + nf[0] * (j + nf[1] * k)];
                    out[v * nec + a + nc[0] * (b + nc[1] * c)] = acc;
                }
}

int orc_restrict(int E, const int *fine_orders, const int *coarse_orders, const double *u,
                 double *uc)
{
    if (E <= 0 || check_orders(E, fine_orders) || check_orders(E, coarse_orders)) return -1;
    ensure_tables();
    long *off = node_offsets(E, fine_orders), *offc = node_offsets(E, coarse_orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e)
        restrict_element(fine_orders + 3 * e, coarse_orders + 3 * e, u + NV * off[e], uc + NV * offc[e]);
    free(off);
    free(offc);
    return 0;
}

/* Solution transfer onto a new order map (Section 2.4.1: storage reallocated and the
 * solution projected onto the new polynomial spaces): per direction, the 1D operator is
 * the interpolation I^{M<-N} when the order rises or stays (the old polynomial lies in
 * the new space, so this is its exact L2 projection), and the exact L2 projection
 * P^{M<-N} when it falls; the element operator is their tensor product (the L2 projection
 * onto the tensor-product space of the reference cube). */
static void project_element(const int *from, const int *to, const double *in, double *out)
{
    int nf[3] = {from[0] + 1, from[1] + 1, from[2] + 1};
    int nt[3] = {to[0] + 1, to[1] + 1, to[2] + 1};
    int nef = nf[0] * nf[1] * nf[2], net = nt[0] * nt[1] * nt[2];
    double A[3][(ORC_NMAX + 1) * (ORC_NMAX + 1)];
    for (int d = 0; d < 3; ++d) {
        if (to[d] >= from[d])
            orc_interp(to[d], from[d], A[d]);
        else
            orc_proj(to[d], from[d], A[d]);
    }
    for (int v = 0; v < NV; ++v)
        for (int c = 0; c < nt[2]; ++c)
            for (int b = 0; b < nt[1]; ++b)
                for (int a = 0; a < nt[0]; ++a) {
                    double acc = 0.0;
                    for (int k = 0; k < nf[2]; ++k)
                        for (int j = 0; j < nf[1]; ++j)
                            for (int i = 0; i < nf[0]; ++i)
                                acc += A[0][a * nf[0] + i] * A[1][b * nf[1] + j] * A[2][c * nf[2] + k] *
                                       in[v * nef + i + nf[0] * (j + nf[1] * k)];
                    out[v * net + a + nt[0] * (b + nt[1] * c)] = acc;
                }
}

int orc_project(int E, const int *from_orders, const int *to_orders, const double *u, double *ut)
{
    if (E <= 0 || check_orders(E, from_orders) || check_orders(E, to_orders)) return -1;
    ensure_tables();
    long *off = node_offsets(E, from_orders), *offt = node_offsets(E, to_orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e)
        project_element(from_orders + 3 * e, to_orders + 3 * e, u + NV * off[e], ut + NV * offt[e]);
    free(off);
    free(offt);
    return 0;
}

int orc_tau(const orc_mesh *m, const int *fine_orders, const int *coarse_orders, const double *u,
            const double *dudt, int isolated, int restriction, double *tau_new, double *tau_trad,
            double *norms, double *varnorms)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, fine_orders) || check_orders(E, coarse_orders)) return -1;
    for (int i = 0; i < 3 * E; ++i)
        if (coarse_orders[i] > fine_orders[i]) return -1;
    ensure_tables();
    long nc = orc_num_nodes(E, coarse_orders);
    double *uc = malloc(sizeof(double) * NV * nc);
    double *rdc = malloc(sizeof(double) * NV * nc);
    /* I^N q^P and I^N (M^P)^-1 F^P(q^P), I^N the sampling or the exact L2 projection
     * (Section 2.3: I^N maps the solution from one space to another) */
    if (restriction != 0 && restriction != 1) {
        free(uc);
        free(rdc);
        return -1;
    }
    if (restriction) {
        orc_project(E, fine_orders, coarse_orders, u, uc);
        orc_project(E, fine_orders, coarse_orders, dudt, rdc);
    } else {
        orc_restrict(E, fine_orders, coarse_orders, u, uc);
        orc_restrict(E, fine_orders, coarse_orders, dudt, rdc);
    }
    /* (M^N)^-1 F^N (I^N q^P) on the coarse mesh */
    orc_residual(m, coarse_orders, uc, tau_new, 0, isolated);
    long *offc = node_offsets(E, coarse_orders);
    for (int e = 0; e < E; ++e) {
        const int *o = coarse_orders + 3 * e;
        int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
        double *Ja = malloc(sizeof(double) * 9 * ne), *Jn = malloc(sizeof(double) * ne);
        elem_metrics(m, o, e, Ja, Jn);
        double *tn = tau_new + NV * offc[e], *tt = tau_trad + NV * offc[e];
        const double *rd = rdc + NV * offc[e];
        double mx[2] = {0, 0}, vm[2][NV] = {{0}};
        for (int v = 0; v < NV; ++v)
            for (int k = 0; k < n[2]; ++k)
                for (int j = 0; j < n[1]; ++j)
                    for (int i = 0; i < n[0]; ++i) {
                        int node = i + n[0] * (j + n[1] * k);
                        int x = v * ne + node;
                        tn[x] = tn[x] - rd[x];
                        tt[x] = Jn[node] * g_w[o[0]][i] * g_w[o[1]][j] * g_w[o[2]][k] * tn[x];
                        double a0 = fabs(tn[x]), a1 = fabs(tt[x]);
                        if (a0 > vm[0][v]) vm[0][v] = a0;
                        if (a1 > vm[1][v]) vm[1][v] = a1;
                    }
        for (int v = 0; v < NV; ++v) {
            if (vm[0][v] > mx[0]) mx[0] = vm[0][v];
            if (vm[1][v] > mx[1]) mx[1] = vm[1][v];
        }
        norms[2 * e] = mx[0];
        norms[2 * e + 1] = mx[1];
        if (varnorms)
            for (int f = 0; f < 2; ++f)
                for (int v = 0; v < NV; ++v) varnorms[(2 * e + f) * NV + v] = vm[f][v];
        free(Ja);
        free(Jn);
    }
    free(offc);
    free(uc);
    free(rdc);
    return 0;
}

int orc_num_combos(const int *o)
{
    int c = 1;
    for (int d = 0; d < 3; ++d) c *= o[d] > 1 ? o[d] - 1 : 1;
    return c;
}

/* Isolated sweep, Euler (viscous = 0) or Navier-Stokes: for every combination the
 * element's isolated coarse residual (its geometry sampled at the coarse nodes)
 * minus the restricted fine time derivative, both forms, maxima. */
static int sweep_impl(const orc_mesh *m, const int *orders, const double *u, const double *dudt, int viscous,
                      double mu, double Pr, int restriction, const int *elems, int nelems, double *te_new,
                      double *te_trad)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders) || (restriction != 0 && restriction != 1)) return -1;
    for (int i = 0; i < nelems; ++i)
        if (elems[i] < 0 || elems[i] >= E) return -1;
    ensure_tables();
    long *off = node_offsets(E, orders);
    long *cofs = malloc(sizeof(long) * (nelems + 1));
    cofs[0] = 0;
    for (int i = 0; i < nelems; ++i) cofs[i + 1] = cofs[i] + orc_num_combos(orders + 3 * elems[i]);

#pragma omp parallel for schedule(guided)
    for (int i = 0; i < nelems; ++i) {
        int e = elems[i];
        const int *of = orders + 3 * e;
        int cmax[3];
        for (int d = 0; d < 3; ++d) cmax[d] = of[d] > 1 ? of[d] - 1 : 1;
        int nef = nnodes(of);
        const double *Q = u + NV * off[e], *R = dudt + NV * off[e];
        double *qc = malloc(sizeof(double) * NV * nef), *rc = malloc(sizeof(double) * NV * nef);
        double *res = malloc(sizeof(double) * NV * nef), *G = malloc(sizeof(double) * 3 * NV * nef);
        double *Ja = malloc(sizeof(double) * 9 * nef), *Jn = malloc(sizeof(double) * nef);
        long slot = cofs[i];
        for (int c3 = 1; c3 <= cmax[2]; ++c3)
            for (int c2 = 1; c2 <= cmax[1]; ++c2)
                for (int c1 = 1; c1 <= cmax[0]; ++c1) {
                    int oc[3] = {c1, c2, c3};
                    int n[3] = {c1 + 1, c2 + 1, c3 + 1}, ne = n[0] * n[1] * n[2];
                    if (restriction) {
                        project_element(of, oc, Q, qc);
                        project_element(of, oc, R, rc);
                    } else {
                        restrict_element(of, oc, Q, qc);
                        restrict_element(of, oc, R, rc);
                    }
                    if (viscous) gradient_core(m, NULL, NULL, NULL, oc, e, qc, 1, G);
                    residual_core(m, NULL, NULL, NULL, NULL, mu, Pr, oc, e, qc, viscous ? G : NULL, 0, 1, res);
                    elem_metrics(m, oc, e, Ja, Jn);
                    double mx0 = 0.0, mx1 = 0.0;
                    for (int v = 0; v < NV; ++v)
                        for (int k = 0; k < n[2]; ++k)
                            for (int j = 0; j < n[1]; ++j)
                                for (int ii = 0; ii < n[0]; ++ii) {
                                    int node = ii + n[0] * (j + n[1] * k);
                                    int x = v * ne + node;
                                    double tn = res[x] - rc[x];
                                    double tt = Jn[node] * g_w[c1][ii] * g_w[c2][j] * g_w[c3][k] * tn;
                                    if (fabs(tn) > mx0) mx0 = fabs(tn);
                                    if (fabs(tt) > mx1) mx1 = fabs(tt);
                                }
                    te_new[slot] = mx0;
                    te_trad[slot] = mx1;
                    ++slot;
                }
        free(qc); free(rc); free(res); free(G); free(Ja); free(Jn);
    }
    free(cofs);
    free(off);
    return 0;
}

int orc_sweep(const orc_mesh *m, const int *orders, const double *u, const double *dudt, int restriction,
              const int *elems, int nelems, double *te_new, double *te_trad)
{
    return sweep_impl(m, orders, u, dudt, 0, 0.0, 0.0, restriction, elems, nelems, te_new, te_trad);
}

int orc_sweep_ns(const orc_mesh *m, const int *orders, const double *u, const double *dudt, double mu,
                 double Pr, int restriction, const int *elems, int nelems, double *te_new, double *te_trad)
{
    return sweep_impl(m, orders, u, dudt, 1, mu, Pr, restriction, elems, nelems, te_new, te_trad);
}

/* Weights of the backward-difference rate at t_{n+1} from k+1 equally spaced samples
 * Q(t_{n+1-j}), j = 0..k: the derivative at s = 0 of the Lagrange polynomial through the
 * abscissae s_j = -j (in units of the step), w_j = l_j'(0). */
int orc_bdf_weights(int k, double *w)
{
    if (k < 1 || k > 6) return -1;
    for (int j = 0; j <= k; ++j) {
        /* l_j(s) = prod_{m != j} (s - s_m) / (s_j - s_m); l_j'(0) = sum_{m != j} 1/(s_j - s_m) prod_{q != j,m} (0 - s_q)/(s_j - s_q) */
        long double sj = -j, acc = 0.0L;
        for (int m = 0; m <= k; ++m) {
            if (m == j) continue;
            long double term = 1.0L / (sj - (long double)(-m));
            for (int q = 0; q <= k; ++q) {
                if (q == j || q == m) continue;
                term *= (0.0L - (long double)(-q)) / (sj - (long double)(-q));
            }
            acc += term;
        }
        w[j] = (double)acc;
    }
    return 0;
}

/* Dual time-stepping estimate (Section 2.3, item 2): the physical time derivative
 * discretised by the backward difference of order nstates-1 over the stored fine
 * solutions states[j] = Q^P(t_{n+1-j}) at step dt, applied to the sampled coarse
 * solutions:  new form  tau_new = (delta_p/delta t)(I Q) + (M^N)^-1 F^N(I Q_0),
 *             traditional tau_trad = J w_i w_j w_k tau_new  (coarse weights). */
int orc_tau_dual(const orc_mesh *m, const int *fine_orders, const int *coarse_orders, const double *const *states,
                 int nstates, double dt, int isolated, double *tau_new, double *tau_trad)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, fine_orders) || check_orders(E, coarse_orders)) return -1;
    if (nstates < 2 || nstates > 7 || !(dt > 0.0)) return -1;
    for (int i = 0; i < 3 * E; ++i)
        if (coarse_orders[i] > fine_orders[i]) return -1;
    double w[8];
    orc_bdf_weights(nstates - 1, w);
    long nc = orc_num_nodes(E, coarse_orders);
    double *qc = malloc(sizeof(double) * NV * nc), *rate = calloc(NV * nc, sizeof(double));
    for (int j = 0; j < nstates; ++j) {
        orc_restrict(E, fine_orders, coarse_orders, states[j], qc);
        for (long i = 0; i < NV * nc; ++i) rate[i] += w[j] * qc[i] / dt;
    }
    orc_restrict(E, fine_orders, coarse_orders, states[0], qc);
    orc_residual(m, coarse_orders, qc, tau_new, 0, isolated);
    long *offc = node_offsets(E, coarse_orders);
    for (int e = 0; e < E; ++e) {
        const int *o = coarse_orders + 3 * e;
        int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
        double *Ja = malloc(sizeof(double) * 9 * ne), *Jn = malloc(sizeof(double) * ne);
        elem_metrics(m, o, e, Ja, Jn);
        for (int v = 0; v < NV; ++v)
            for (int c = 0; c < n[2]; ++c)
                for (int b = 0; b < n[1]; ++b)
                    for (int a = 0; a < n[0]; ++a) {
                        int node = a + n[0] * (b + n[1] * c);
                        long x = NV * offc[e] + (long)v * ne + node;
                        tau_new[x] += rate[x];
                        tau_trad[x] = Jn[node] * g_w[o[0]][a] * g_w[o[1]][b] * g_w[o[2]][c] * tau_new[x];
                    }
        free(Ja);
        free(Jn);
    }
    free(offc);
    free(qc);
    free(rate);
    return 0;
}

int orc_tau_eta(const orc_mesh *m, const int *fine_orders, const int *coarse_orders, const double *u,
                const double *dudt, int isolated, int restriction, const double *psi, int psi_form, double *eta)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, fine_orders) || check_orders(E, coarse_orders)) return -1;
    if (psi_form != 0 && psi_form != 1) return -1;
    ensure_tables();
    long nc = orc_num_nodes(E, coarse_orders);
    double *tn = malloc(sizeof(double) * NV * nc), *tt = malloc(sizeof(double) * NV * nc);
    double *norms = malloc(sizeof(double) * 2 * E), *psic = malloc(sizeof(double) * NV * nc);
    int rc = orc_tau(m, fine_orders, coarse_orders, u, dudt, isolated, restriction, tn, tt, norms, NULL);
    const double *pt = psi;
    double *scaled = NULL;
    if (rc == 0 && psi_form == 0) {
        /* the adjoint of the new form, (d(M^-1 F)/du)^T psi = g, is M times the adjoint of
         * the traditional form: back to the nodal field psi / (J w_i w_j w_k) (fine map) */
        long *off = node_offsets(E, fine_orders);
        scaled = malloc(sizeof(double) * NV * off[E]);
        for (int e = 0; e < E; ++e) {
            const int *o = fine_orders + 3 * e;
            int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
            double *Ja = malloc(sizeof(double) * 9 * ne), *Jn = malloc(sizeof(double) * ne);
            elem_metrics(m, o, e, Ja, Jn);
            for (int k = 0; k < n[2]; ++k)
                for (int j = 0; j < n[1]; ++j)
                    for (int i = 0; i < n[0]; ++i) {
                        int node = i + n[0] * (j + n[1] * k);
                        double mass = Jn[node] * g_w[o[0]][i] * g_w[o[1]][j] * g_w[o[2]][k];
                        for (int v = 0; v < NV; ++v)
                            scaled[NV * off[e] + v * ne + node] = psi[NV * off[e] + v * ne + node] / mass;
                    }
            free(Ja);
            free(Jn);
        }
        free(off);
        pt = scaled;
    }
    if (rc == 0) {
        if (restriction)
            orc_project(E, fine_orders, coarse_orders, pt, psic);
        else
            orc_restrict(E, fine_orders, coarse_orders, pt, psic);
        long *offc = node_offsets(E, coarse_orders);
        for (int e = 0; e < E; ++e) {
            long a = NV * offc[e], b = NV * offc[e + 1];
            double acc = 0.0;
            for (long x = a; x < b; ++x) acc += psic[x] * tt[x];
            eta[e] = acc;
        }
        free(offc);
    }
    free(tn); free(tt); free(norms); free(psic); free(scaled);
    return rc;
}

int orc_functional(const orc_mesh *m, const int *orders, const double *u, double *J, double *dJdu)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || m->map_kind != 0 || check_orders(E, orders)) return -1;
    ensure_tables();
    double h[3], Jm, Ja[3];
    geometry(m, h, &Jm, Ja);
    long *off = node_offsets(E, orders);
    if (dJdu) memset(dJdu, 0, sizeof(double) * NV * off[E]);
    double g = m->gamma, total = 0.0;
    for (int e = 0; e < E; ++e) {
        int c[3];
        elem_ijk(m, e, c);
        const int *o = orders + 3 * e;
        int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
        for (int s = -1; s <= 1; s += 2) {
            int at_wall = (s < 0 && c[0] == 0 && m->bc[0] == 1) || (s > 0 && c[0] == m->nx - 1 && m->bc[1] == 1);
            if (!at_wall) continue;
            /* face normal to x: tangential directions y (a) and z (b) */
            for (int b = 0; b < n[2]; ++b)
                for (int a = 0; a < n[1]; ++a) {
                    int node = face_node(n, 0, s, a, b);
                    const double *Q = u + NV * off[e];
                    double q[NV];
                    for (int v = 0; v < NV; ++v) q[v] = Q[v * ne + node];
                    double wgt = g_w[o[1]][a] * g_w[o[2]][b] * Ja[0] * (double)s;
                    total += wgt * pressure(q, g);
                    if (dJdu) {
                        double *D = dJdu + NV * off[e];
                        double ux = q[1] / q[0], uy = q[2] / q[0], uz = q[3] / q[0];
                        D[0 * ne + node] = wgt * (g - 1.0) * 0.5 * (ux * ux + uy * uy + uz * uz);
                        D[1 * ne + node] = -wgt * (g - 1.0) * ux;
                        D[2 * ne + node] = -wgt * (g - 1.0) * uy;
                        D[3 * ne + node] = -wgt * (g - 1.0) * uz;
                        D[4 * ne + node] = wgt * (g - 1.0);
                    }
                }
        }
    }
    *J = total;
    free(off);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Williamson (1980) low-storage third-order Runge-Kutta.                    */

int orc_rk3(const orc_mesh *m, const int *orders, double *u, double dt, int nsteps)
{
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || check_orders(E, orders) || nsteps < 0) return -1;
    long n = NV * orc_num_nodes(E, orders);
    double *r = malloc(sizeof(double) * n), *G = malloc(sizeof(double) * n);
    for (int step = 0; step < nsteps; ++step)
        for (int k = 0; k < 3; ++k) {
            orc_residual(m, orders, u, r, 0, 0); /* r = -dQ/dt */
            for (long x = 0; x < n; ++x) {
                G[x] = (k == 0) ? -dt * r[x] : A[k] * G[x] - dt * r[x];
                u[x] += B[k] * G[x];
            }
        }
    free(r);
    free(G);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Derivatives of the residual (box Euler meshes).                           */
/*
 * The adjoint-weighted estimate (the remark of Section 2.2 relating the truncation
 * error to functional errors) needs the transpose of the residual's Jacobian.  Two
 * routes are written here, independently of each other:
 *
 *   - The directional derivative (d r / d u) d by complex step (Squire and Trapp, 1998):
 *     the residual evaluated in complex arithmetic at u + i h d, whose imaginary part
 *     divided by h is the derivative, with no subtraction and hence exact to rounding
 *     for h = 1e-30.  |x| continues as x sign(Re x) (0 at 0) and max by the real parts
 *     (the first argument on ties).
 *   - The vector-Jacobian product (d r / d u)^T v, each step of the residual transposed
 *     by hand: the form's diagonal scaling, D^T along every direction, the transposed
 *     lifting, the transposed mortar projection P^T and interpolation S^T, the
 *     transposed Jacobian of the physical flux (closed form), of the Riemann flux (its
 *     5 x 10 Jacobian by complex step at each mortar node) and of the boundary ghost
 *     states (slip wall: the mirror, a reflection; far field: a constant).
 *
 * The two agree through <v, (d r/d u) d> = <(d r/d u)^T v, d>; the transposed product
 * also keeps the discrete conservation of the residual (mass-weighted sums of a
 * variable over a periodic mesh are independent of the state).
 */

typedef double _Complex zdbl;

static const double CSTEP_H = 1e-30;

static zdbl z_abs(zdbl x)
{
    double r = creal(x);
    return r > 0.0 ? x : (r < 0.0 ? -x : 0.0);
}

static zdbl z_max(zdbl a, zdbl b) { return creal(a) >= creal(b) ? a : b; }

static zdbl z_pressure(const zdbl *q, double g)
{
    zdbl ke = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
    return (g - 1.0) * (q[4] - ke);
}

static void z_flux_n(const zdbl *q, const double *n, double g, zdbl *f)
{
    zdbl rho = q[0];
    zdbl u = q[1] / rho, v = q[2] / rho, w = q[3] / rho;
    zdbl p = z_pressure(q, g);
    zdbl un = u * n[0] + v * n[1] + w * n[2];
    f[0] = rho * un;
    f[1] = q[1] * un + p * n[0];
    f[2] = q[2] * un + p * n[1];
    f[3] = q[3] * un + p * n[2];
    f[4] = (q[4] + p) * un;
}

/* The numerical flux of orc_numflux in complex arithmetic (same steps, same order). */
static void z_numflux(const zdbl *qL, const zdbl *qR, const double *n, double g, int kind, zdbl *f)
{
    zdbl fL[NV], fR[NV];
    z_flux_n(qL, n, g, fL);
    z_flux_n(qR, n, g, fR);
    if (kind == 0) {
        zdbl rL = qL[0], rR = qR[0];
        zdbl uL[3] = {qL[1] / rL, qL[2] / rL, qL[3] / rL};
        zdbl uR[3] = {qR[1] / rR, qR[2] / rR, qR[3] / rR};
        zdbl pL = z_pressure(qL, g), pR = z_pressure(qR, g);
        zdbl HL = (qL[4] + pL) / rL, HR = (qR[4] + pR) / rR;
        zdbl sL = csqrt(rL), sR = csqrt(rR);
        zdbl ut[3];
        for (int d = 0; d < 3; ++d) ut[d] = (sL * uL[d] + sR * uR[d]) / (sL + sR);
        zdbl Ht = (sL * HL + sR * HR) / (sL + sR);
        zdbl rt = sL * sR;
        zdbl q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
        zdbl c2 = (g - 1.0) * (Ht - 0.5 * q2);
        zdbl c = csqrt(c2);
        zdbl un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
        zdbl du[3] = {uR[0] - uL[0], uR[1] - uL[1], uR[2] - uL[2]};
        zdbl dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
        zdbl dut[3] = {du[0] - dun * n[0], du[1] - dun * n[1], du[2] - dun * n[2]};
        zdbl drho = rR - rL, dp = pR - pL;
        zdbl a1 = (dp - rt * c * dun) / (2.0 * c2);
        zdbl a2 = drho - dp / c2;
        zdbl a4 = (dp + rt * c * dun) / (2.0 * c2);
        zdbl lam[4] = {un - c, un, un, un + c};
        zdbl wave[20];
        wave[0] = a1;
        for (int d = 0; d < 3; ++d) wave[1 + d] = a1 * (ut[d] - c * n[d]);
        wave[4] = a1 * (Ht - c * un);
        wave[5] = a2;
        for (int d = 0; d < 3; ++d) wave[6 + d] = a2 * ut[d];
        wave[9] = a2 * 0.5 * q2;
        wave[10] = 0.0;
        for (int d = 0; d < 3; ++d) wave[11 + d] = rt * dut[d];
        wave[14] = rt * (ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2]);
        wave[15] = a4;
        for (int d = 0; d < 3; ++d) wave[16 + d] = a4 * (ut[d] + c * n[d]);
        wave[19] = a4 * (Ht + c * un);
        for (int v = 0; v < NV; ++v) {
            zdbl diss = 0.0;
            for (int k = 0; k < 4; ++k) diss += z_abs(lam[k]) * wave[k * NV + v];
            f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * diss;
        }
    } else {
        zdbl rL = qL[0], rR = qR[0];
        zdbl unL = (qL[1] * n[0] + qL[2] * n[1] + qL[3] * n[2]) / rL;
        zdbl unR = (qR[1] * n[0] + qR[2] * n[1] + qR[3] * n[2]) / rR;
        zdbl cL = csqrt(g * z_pressure(qL, g) / rL), cR = csqrt(g * z_pressure(qR, g) / rR);
        zdbl s = z_max(z_abs(unL) + cL, z_abs(unR) + cR);
        for (int v = 0; v < NV; ++v) f[v] = 0.5 * (fL[v] + fR[v]) - 0.5 * s * (qR[v] - qL[v]);
    }
}

/* Ghost state of a boundary face in complex arithmetic (as ghost_state). */
static void z_ghost_state(const orc_mesh *m, int bc, const double *nout, const zdbl *qin, zdbl *qg)
{
    if (bc == 1) {
        zdbl mn = qin[1] * nout[0] + qin[2] * nout[1] + qin[3] * nout[2];
        qg[0] = qin[0];
        for (int k = 0; k < 3; ++k) qg[1 + k] = qin[1 + k] - 2.0 * mn * nout[k];
        qg[4] = qin[4];
    } else {
        for (int v = 0; v < NV; ++v) qg[v] = m->qfar[v];
    }
}

/* Apply the real tensor-product operator A1 (rows x na) (x) A2 (cols x nb) to nv complex
 * face fields: out[v][r + R1*c] = sum A1[r][a] A2[c][b] in[v][a + na*b]. */
static void z_face_apply(int nv, int na, int nb, int R1, int R2, const double *A1, const double *A2, const zdbl *in,
                         zdbl *out)
{
    for (int v = 0; v < nv; ++v)
        for (int c = 0; c < R2; ++c)
            for (int r = 0; r < R1; ++r) {
                zdbl acc = 0.0;
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) acc += A1[r * na + a] * A2[c * nb + b] * in[v * na * nb + a + na * b];
                out[v * R1 * R2 + r + R1 * c] = acc;
            }
}

/* Outward numerical flux of face (d, s) of element e in complex arithmetic (box Euler;
 * the steps of face_flux). */
static void z_face_flux(const orc_mesh *m, const int *orders, const long *off, const zdbl *u, int e, int d, int s,
                        zdbl *fout)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1};
    int na = n[t1], nb = n[t2], ne = n[0] * n[1] * n[2];
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    const double g = m->gamma;
    zdbl *own = malloc(sizeof(zdbl) * NV * na * nb);
    for (int v = 0; v < NV; ++v)
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < na; ++a) own[v * na * nb + a + na * b] = u[NV * off[e] + v * ne + face_node(n, d, s, a, b)];
    int bc;
    int nbr = neighbour(m, e, d, s, &bc);
    if (nbr < 0) {
        double mv[3] = {0.0, 0.0, 0.0}, nh[3];
        mv[d] = (double)s * Ja[d];
        double len = unit_normal(mv, nh);
        for (int x = 0; x < na * nb; ++x) {
            zdbl qin[NV], qg[NV], fa[NV];
            for (int v = 0; v < NV; ++v) qin[v] = own[v * na * nb + x];
            z_ghost_state(m, bc, nh, qin, qg);
            z_numflux(qin, qg, nh, g, m->flux, fa);
            for (int v = 0; v < NV; ++v) fout[v * na * nb + x] = len * fa[v];
        }
        free(own);
        return;
    }
    const int *on = orders + 3 * nbr;
    int nn[3] = {on[0] + 1, on[1] + 1, on[2] + 1}, nen = nn[0] * nn[1] * nn[2];
    int ma = nn[t1], mb = nn[t2];
    zdbl *oth = malloc(sizeof(zdbl) * NV * ma * mb);
    for (int v = 0; v < NV; ++v)
        for (int b = 0; b < mb; ++b)
            for (int a = 0; a < ma; ++a)
                oth[v * ma * mb + a + ma * b] = u[NV * off[nbr] + v * nen + face_node(nn, d, -s, a, b)];
    int K1 = na > ma ? na : ma, K2 = nb > mb ? nb : mb, KK = K1 * K2;
    double *S1 = malloc(sizeof(double) * K1 * na), *S2 = malloc(sizeof(double) * K2 * nb);
    double *T1 = malloc(sizeof(double) * K1 * ma), *T2 = malloc(sizeof(double) * K2 * mb);
    double *P1 = malloc(sizeof(double) * na * K1), *P2 = malloc(sizeof(double) * nb * K2);
    orc_interp(K1 - 1, na - 1, S1);
    orc_interp(K2 - 1, nb - 1, S2);
    orc_interp(K1 - 1, ma - 1, T1);
    orc_interp(K2 - 1, mb - 1, T2);
    orc_proj(na - 1, K1 - 1, P1);
    orc_proj(nb - 1, K2 - 1, P2);
    zdbl *A = malloc(sizeof(zdbl) * NV * KK), *B = malloc(sizeof(zdbl) * NV * KK), *FK = malloc(sizeof(zdbl) * NV * KK);
    z_face_apply(NV, na, nb, K1, K2, S1, S2, own, A);
    z_face_apply(NV, ma, mb, K1, K2, T1, T2, oth, B);
    zdbl *L = s > 0 ? A : B, *R = s > 0 ? B : A;
    double mv[3] = {0.0, 0.0, 0.0}, nh[3];
    mv[d] = Ja[d];
    double len = unit_normal(mv, nh);
    for (int x = 0; x < KK; ++x) {
        zdbl qL[NV], qR[NV], fa[NV];
        for (int v = 0; v < NV; ++v) {
            qL[v] = L[v * KK + x];
            qR[v] = R[v * KK + x];
        }
        z_numflux(qL, qR, nh, g, m->flux, fa);
        for (int v = 0; v < NV; ++v) FK[v * KK + x] = len * fa[v];
    }
    z_face_apply(NV, K1, K2, na, nb, P1, P2, FK, fout);
    for (int x = 0; x < NV * na * nb; ++x) fout[x] *= (double)s;
    free(own); free(oth); free(S1); free(S2); free(T1); free(T2); free(P1); free(P2);
    free(A); free(B); free(FK);
}

/* Residual of box element e in complex arithmetic (the steps of residual_core for the
 * Euler equations: Ft^d = |Ja^d| f_d, V = sum_d D_d Ft^d, lifting, form scaling). */
static void z_residual_elem(const orc_mesh *m, const int *orders, const long *off, const zdbl *u, int e, int form,
                            int isolated, zdbl *r)
{
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    const zdbl *Q = u + NV * off[e];
    zdbl *Ft = malloc(sizeof(zdbl) * 3 * NV * ne), *V = malloc(sizeof(zdbl) * NV * ne);
    for (int node = 0; node < ne; ++node) {
        zdbl q[NV], f[NV];
        for (int v = 0; v < NV; ++v) q[v] = Q[v * ne + node];
        for (int d = 0; d < 3; ++d) {
            double ed[3] = {0.0, 0.0, 0.0};
            ed[d] = 1.0;
            z_flux_n(q, ed, m->gamma, f);
            for (int v = 0; v < NV; ++v) Ft[(d * NV + v) * ne + node] = Ja[d] * f[v];
        }
    }
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int node = i + n[0] * (j + n[1] * k);
                for (int v = 0; v < NV; ++v) {
                    zdbl acc = 0.0;
                    for (int q = 0; q < n[0]; ++q)
                        acc += g_D[o[0]][i * n[0] + q] * Ft[(0 * NV + v) * ne + q + n[0] * (j + n[1] * k)];
                    for (int q = 0; q < n[1]; ++q)
                        acc += g_D[o[1]][j * n[1] + q] * Ft[(1 * NV + v) * ne + i + n[0] * (q + n[1] * k)];
                    for (int q = 0; q < n[2]; ++q)
                        acc += g_D[o[2]][k * n[2] + q] * Ft[(2 * NV + v) * ne + i + n[0] * (j + n[1] * q)];
                    V[v * ne + node] = acc;
                }
            }
    if (!isolated) {
        for (int d = 0; d < 3; ++d) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int na = n[t1], nb = n[t2];
            double wend = g_w[o[d]][0];
            zdbl *fout = malloc(sizeof(zdbl) * NV * na * nb);
            for (int s = -1; s <= 1; s += 2) {
                z_face_flux(m, orders, off, u, e, d, s, fout);
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) {
                        int node = face_node(n, d, s, a, b);
                        for (int v = 0; v < NV; ++v)
                            V[v * ne + node] += (fout[v * na * nb + a + na * b] -
                                                 (double)s * Ft[(d * NV + v) * ne + node]) / wend;
                    }
            }
            free(fout);
        }
    }
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int node = i + n[0] * (j + n[1] * k);
                double www = g_w[o[0]][i] * g_w[o[1]][j] * g_w[o[2]][k];
                for (int v = 0; v < NV; ++v)
                    r[v * ne + node] = form == 0 ? V[v * ne + node] / J : www * V[v * ne + node];
            }
    free(Ft);
    free(V);
}

static int check_box_euler(const orc_mesh *m, const int *orders, int form)
{
    int E = m->nx * m->ny * m->nz;
    if (check_mesh(m) || m->map_kind != 0 || check_orders(E, orders) || (form != 0 && form != 1)) return -1;
    return 0;
}

int orc_residual_cstep(const orc_mesh *m, const int *orders, const double *u, const double *dir, double h,
                       double *r_re, double *r_im, int form, int isolated)
{
    if (check_box_euler(m, orders, form)) return -1;
    ensure_tables();
    int E = m->nx * m->ny * m->nz;
    long *off = node_offsets(E, orders);
    long N = NV * off[E];
    zdbl *zu = malloc(sizeof(zdbl) * N), *zr = malloc(sizeof(zdbl) * N);
    for (long x = 0; x < N; ++x) zu[x] = u[x] + h * dir[x] * _Complex_I;
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e) z_residual_elem(m, orders, off, zu, e, form, isolated, zr + NV * off[e]);
    for (long x = 0; x < N; ++x) {
        if (r_re) r_re[x] = creal(zr[x]);
        if (r_im) r_im[x] = cimag(zr[x]);
    }
    free(zu);
    free(zr);
    free(off);
    return 0;
}

int orc_residual_jvp(const orc_mesh *m, const int *orders, const double *u, const double *dir, double *out, int form,
                     int isolated)
{
    int rc = orc_residual_cstep(m, orders, u, dir, CSTEP_H, NULL, out, form, isolated);
    if (rc == 0) {
        long N = NV * orc_num_nodes(m->nx * m->ny * m->nz, orders);
        for (long x = 0; x < N; ++x) out[x] /= CSTEP_H;
    }
    return rc;
}

/* Jacobian of the physical flux f.n in the conserved variables (closed form; e.g.
 * Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 3):
 * A[i*5 + j] = d (f.n)_i / d q_j, with u the velocity, u_n = u.n, H the total enthalpy
 * and phi = (gamma - 1) |u|^2 / 2. */
void orc_flux_jacobian(const double *q, const double *n, double g, double *A)
{
    double rho = q[0], u[3] = {q[1] / q[0], q[2] / q[0], q[3] / q[0]};
    double p = pressure(q, g), H = (q[4] + p) / rho;
    double un = u[0] * n[0] + u[1] * n[1] + u[2] * n[2];
    double phi = 0.5 * (g - 1.0) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    A[0] = 0.0;
    for (int l = 0; l < 3; ++l) A[1 + l] = n[l];
    A[4] = 0.0;
    for (int k = 0; k < 3; ++k) {
        double *row = A + 5 * (1 + k);
        row[0] = -u[k] * un + phi * n[k];
        for (int l = 0; l < 3; ++l) row[1 + l] = (k == l ? un : 0.0) + u[k] * n[l] - (g - 1.0) * u[l] * n[k];
        row[4] = (g - 1.0) * n[k];
    }
    double *row = A + 20;
    row[0] = un * (phi - H);
    for (int l = 0; l < 3; ++l) row[1 + l] = H * n[l] - (g - 1.0) * u[l] * un;
    row[4] = g * un;
}

/* Jacobians of the numerical flux with respect to either state, column by column by
 * complex step: AL[i*5 + j] = d f*_i / d qL_j, AR[i*5 + j] = d f*_i / d qR_j. */
void orc_numflux_jacobian(const double *qL, const double *qR, const double *n, double g, int kind, double *AL,
                          double *AR)
{
    for (int side = 0; side < 2; ++side)
        for (int j = 0; j < NV; ++j) {
            zdbl zl[NV], zr[NV], f[NV];
            for (int v = 0; v < NV; ++v) {
                zl[v] = qL[v];
                zr[v] = qR[v];
            }
            if (side == 0) zl[j] += CSTEP_H * _Complex_I;
            else zr[j] += CSTEP_H * _Complex_I;
            z_numflux(zl, zr, n, g, kind, f);
            double *Aout = side == 0 ? AL : AR;
            for (int i = 0; i < NV; ++i) Aout[i * NV + j] = cimag(f[i]) / CSTEP_H;
        }
}

/* Transpose of face_flux on a box Euler mesh.  Fb[v][a + na*b] is the adjoint of the
 * outward flux F*_out on the own face nodes of face (d, s) of element e; the
 * contributions to the adjoints of the own face trace are added to bo[v][a + na*b], and
 * those of the neighbour's face trace to bn[v][a' + ma*b'] (untouched at boundaries). */
static void face_flux_vjp(const orc_mesh *m, const int *orders, const long *off, const double *u, int e, int d, int s,
                          const double *Fb, double *bo, double *bn)
{
    int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1};
    int na = n[t1], nb = n[t2];
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    const double g = m->gamma;
    double *own = malloc(sizeof(double) * NV * na * nb);
    face_trace(n, d, s, NV, u + NV * off[e], own);
    int bc;
    int nbr = neighbour(m, e, d, s, &bc);
    double AL[NV * NV], AR[NV * NV];
    if (nbr < 0) {
        /* F*_out = len f*(q, ghost(q), n): adjoint len (AL + AR G)^T Fb, G the ghost Jacobian */
        double mv[3] = {0.0, 0.0, 0.0}, nh[3];
        mv[d] = (double)s * Ja[d];
        double len = unit_normal(mv, nh);
        double G[NV * NV];
        for (int i = 0; i < NV * NV; ++i) G[i] = 0.0;
        if (bc == 1) {
            G[0] = 1.0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) G[(1 + k) * NV + 1 + l] = (k == l ? 1.0 : 0.0) - 2.0 * nh[k] * nh[l];
            G[4 * NV + 4] = 1.0;
        }
        for (int x = 0; x < na * nb; ++x) {
            double qin[NV], qg[NV];
            for (int v = 0; v < NV; ++v) qin[v] = own[v * na * nb + x];
            ghost_state(m, bc, nh, qin, qg);
            orc_numflux_jacobian(qin, qg, nh, g, m->flux, AL, AR);
            for (int w = 0; w < NV; ++w) {
                double acc = 0.0;
                for (int v = 0; v < NV; ++v) {
                    double dfdq = AL[v * NV + w];
                    for (int k = 0; k < NV; ++k) dfdq += AR[v * NV + k] * G[k * NV + w];
                    acc += Fb[v * na * nb + x] * dfdq;
                }
                bo[w * na * nb + x] += len * acc;
            }
        }
        free(own);
        return;
    }
    const int *on = orders + 3 * nbr;
    int nn[3] = {on[0] + 1, on[1] + 1, on[2] + 1};
    int ma = nn[t1], mb = nn[t2];
    double *oth = malloc(sizeof(double) * NV * ma * mb);
    face_trace(nn, d, -s, NV, u + NV * off[nbr], oth);
    int K1 = na > ma ? na : ma, K2 = nb > mb ? nb : mb, KK = K1 * K2;
    double *S1 = malloc(sizeof(double) * K1 * na), *S2 = malloc(sizeof(double) * K2 * nb);
    double *T1 = malloc(sizeof(double) * K1 * ma), *T2 = malloc(sizeof(double) * K2 * mb);
    double *P1 = malloc(sizeof(double) * na * K1), *P2 = malloc(sizeof(double) * nb * K2);
    orc_interp(K1 - 1, na - 1, S1);
    orc_interp(K2 - 1, nb - 1, S2);
    orc_interp(K1 - 1, ma - 1, T1);
    orc_interp(K2 - 1, mb - 1, T2);
    orc_proj(na - 1, K1 - 1, P1);
    orc_proj(nb - 1, K2 - 1, P2);
    /* forward: A = (S1 x S2) own, B = (T1 x T2) oth on the mortar */
    double *A = malloc(sizeof(double) * NV * KK), *B = malloc(sizeof(double) * NV * KK);
    to_mortar(NV, na, nb, K1, K2, own, A);
    to_mortar(NV, ma, mb, K1, K2, oth, B);
    const double *Lq = s > 0 ? A : B, *Rq = s > 0 ? B : A;
    /* forward: F*_out = s (P1 x P2) FK; adjoint FKb = s (P1 x P2)^T Fb */
    double *FKb = malloc(sizeof(double) * NV * KK);
    for (int v = 0; v < NV; ++v)
        for (int Bm = 0; Bm < K2; ++Bm)
            for (int Am = 0; Am < K1; ++Am) {
                double acc = 0.0;
                for (int b = 0; b < nb; ++b)
                    for (int a = 0; a < na; ++a) acc += P1[a * K1 + Am] * P2[b * K2 + Bm] * Fb[v * na * nb + a + na * b];
                FKb[v * KK + Am + K1 * Bm] = (double)s * acc;
            }
    /* forward: FK = len f*(L, R, e_d) per mortar node; adjoints of L and R */
    double mv[3] = {0.0, 0.0, 0.0}, nh[3];
    mv[d] = Ja[d];
    double len = unit_normal(mv, nh);
    double *Lb = malloc(sizeof(double) * NV * KK), *Rb = malloc(sizeof(double) * NV * KK);
    for (int x = 0; x < KK; ++x) {
        double qL[NV], qR[NV];
        for (int v = 0; v < NV; ++v) {
            qL[v] = Lq[v * KK + x];
            qR[v] = Rq[v * KK + x];
        }
        orc_numflux_jacobian(qL, qR, nh, g, m->flux, AL, AR);
        for (int w = 0; w < NV; ++w) {
            double aL = 0.0, aR = 0.0;
            for (int v = 0; v < NV; ++v) {
                aL += AL[v * NV + w] * FKb[v * KK + x];
                aR += AR[v * NV + w] * FKb[v * KK + x];
            }
            Lb[w * KK + x] = len * aL;
            Rb[w * KK + x] = len * aR;
        }
    }
    const double *Ab = s > 0 ? Lb : Rb, *Bb = s > 0 ? Rb : Lb;
    /* adjoint of the interpolations onto the mortar: (S1 x S2)^T and (T1 x T2)^T */
    for (int w = 0; w < NV; ++w) {
        for (int b = 0; b < nb; ++b)
            for (int a = 0; a < na; ++a) {
                double acc = 0.0;
                for (int Bm = 0; Bm < K2; ++Bm)
                    for (int Am = 0; Am < K1; ++Am) acc += S1[Am * na + a] * S2[Bm * nb + b] * Ab[w * KK + Am + K1 * Bm];
                bo[w * na * nb + a + na * b] += acc;
            }
        for (int b = 0; b < mb; ++b)
            for (int a = 0; a < ma; ++a) {
                double acc = 0.0;
                for (int Bm = 0; Bm < K2; ++Bm)
                    for (int Am = 0; Am < K1; ++Am) acc += T1[Am * ma + a] * T2[Bm * mb + b] * Bb[w * KK + Am + K1 * Bm];
                bn[w * ma * mb + a + ma * b] += acc;
            }
    }
    free(own); free(oth); free(S1); free(S2); free(T1); free(T2); free(P1); free(P2);
    free(A); free(B); free(FKb); free(Lb); free(Rb);
}

/* Form scaling of the residual at the nodes of element orders o: 1/J (new form) or
 * w_i w_j w_k (traditional form). */
static void form_scale(const orc_mesh *m, const int *o, int form, double *sc)
{
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1};
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i)
                sc[i + n[0] * (j + n[1] * k)] = form == 0 ? 1.0 / J : g_w[o[0]][i] * g_w[o[1]][j] * g_w[o[2]][k];
}

/* (d r / d u)^T v restricted to the unknowns of element e: the transposed steps of e's
 * own residual, plus, through each shared face, the transposed face flux of the
 * neighbour's residual (which reads e's face trace). */
static void vjp_elem(const orc_mesh *m, const int *orders, const long *off, const double *u, const double *v, int e,
                     int form, int isolated, double *out)
{
    const int *o = orders + 3 * e;
    int n[3] = {o[0] + 1, o[1] + 1, o[2] + 1}, ne = n[0] * n[1] * n[2];
    double h[3], J, Ja[3];
    geometry(m, h, &J, Ja);
    const double *Q = u + NV * off[e];
    double *sc = malloc(sizeof(double) * ne), *vt = malloc(sizeof(double) * NV * ne);
    double *Ftb = malloc(sizeof(double) * 3 * NV * ne);
    form_scale(m, o, form, sc);
    for (int w = 0; w < NV; ++w)
        for (int x = 0; x < ne; ++x) vt[w * ne + x] = sc[x] * v[NV * off[e] + w * ne + x];
    /* V = sum_d D_d Ft^d: adjoint Ftb^d = D_d^T vt along d */
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                int node = i + n[0] * (j + n[1] * k);
                for (int w = 0; w < NV; ++w) {
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
                    for (int q = 0; q < n[0]; ++q) a0 += g_D[o[0]][q * n[0] + i] * vt[w * ne + q + n[0] * (j + n[1] * k)];
                    for (int q = 0; q < n[1]; ++q) a1 += g_D[o[1]][q * n[1] + j] * vt[w * ne + i + n[0] * (q + n[1] * k)];
                    for (int q = 0; q < n[2]; ++q) a2 += g_D[o[2]][q * n[2] + k] * vt[w * ne + i + n[0] * (j + n[1] * q)];
                    Ftb[(0 * NV + w) * ne + node] = a0;
                    Ftb[(1 * NV + w) * ne + node] = a1;
                    Ftb[(2 * NV + w) * ne + node] = a2;
                }
            }
    /* lifting -s Ft^d / w_end at the face nodes: adjoint -s vt / w_end */
    if (!isolated)
        for (int d = 0; d < 3; ++d) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            double wend = g_w[o[d]][0];
            for (int s = -1; s <= 1; s += 2)
                for (int b = 0; b < n[t2]; ++b)
                    for (int a = 0; a < n[t1]; ++a) {
                        int node = face_node(n, d, s, a, b);
                        for (int w = 0; w < NV; ++w) Ftb[(d * NV + w) * ne + node] -= (double)s * vt[w * ne + node] / wend;
                    }
        }
    /* Ft^d = |Ja^d| f_d(Q): adjoint |Ja^d| A_d(Q)^T Ftb^d */
    for (int x = 0; x < ne; ++x) {
        double q[NV], A[NV * NV];
        for (int w = 0; w < NV; ++w) q[w] = Q[w * ne + x];
        for (int w = 0; w < NV; ++w) out[w * ne + x] = 0.0;
        for (int d = 0; d < 3; ++d) {
            double ed[3] = {0.0, 0.0, 0.0};
            ed[d] = 1.0;
            orc_flux_jacobian(q, ed, m->gamma, A);
            for (int w = 0; w < NV; ++w) {
                double acc = 0.0;
                for (int vv = 0; vv < NV; ++vv) acc += A[vv * NV + w] * Ftb[(d * NV + vv) * ne + x];
                out[w * ne + x] += Ja[d] * acc;
            }
        }
    }
    if (!isolated) {
        for (int d = 0; d < 3; ++d) {
            int t1 = (d == 0) ? 1 : 0, t2 = (d == 2) ? 1 : 2;
            int na = n[t1], nb = n[t2];
            double wend = g_w[o[d]][0];
            double *Fb = malloc(sizeof(double) * NV * (ORC_NMAX + 1) * (ORC_NMAX + 1));
            double *bo = malloc(sizeof(double) * NV * (ORC_NMAX + 1) * (ORC_NMAX + 1));
            double *bn = malloc(sizeof(double) * NV * (ORC_NMAX + 1) * (ORC_NMAX + 1));
            for (int s = -1; s <= 1; s += 2) {
                /* e's own surface term (F*_out / w_end at its face nodes) */
                for (int w = 0; w < NV; ++w)
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < na; ++a) {
                            Fb[w * na * nb + a + na * b] = vt[w * ne + face_node(n, d, s, a, b)] / wend;
                            bo[w * na * nb + a + na * b] = 0.0;
                        }
                /* (the neighbour's share of e's own surface term is collected by the
                 * neighbour itself; bn is only a sink here) */
                for (int x = 0; x < NV * (ORC_NMAX + 1) * (ORC_NMAX + 1); ++x) bn[x] = 0.0;
                face_flux_vjp(m, orders, off, u, e, d, s, Fb, bo, bn);
                for (int w = 0; w < NV; ++w)
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < na; ++a) out[w * ne + face_node(n, d, s, a, b)] += bo[w * na * nb + a + na * b];
                /* the neighbour's surface term on the same face reads e's trace */
                int bc;
                int nbr = neighbour(m, e, d, s, &bc);
                if (nbr < 0) continue;
                const int *on = orders + 3 * nbr;
                int nn[3] = {on[0] + 1, on[1] + 1, on[2] + 1}, nen = nn[0] * nn[1] * nn[2];
                int ma = nn[t1], mb = nn[t2];
                double *scn = malloc(sizeof(double) * nen);
                form_scale(m, on, form, scn);
                double wendn = g_w[on[d]][0];
                for (int w = 0; w < NV; ++w)
                    for (int b = 0; b < mb; ++b)
                        for (int a = 0; a < ma; ++a) {
                            int node = face_node(nn, d, -s, a, b);
                            Fb[w * ma * mb + a + ma * b] = scn[node] * v[NV * off[nbr] + w * nen + node] / wendn;
                            bo[w * ma * mb + a + ma * b] = 0.0;
                        }
                for (int x = 0; x < NV * na * nb; ++x) bn[x] = 0.0;
                face_flux_vjp(m, orders, off, u, nbr, d, -s, Fb, bo, bn);
                for (int w = 0; w < NV; ++w)
                    for (int b = 0; b < nb; ++b)
                        for (int a = 0; a < na; ++a) out[w * ne + face_node(n, d, s, a, b)] += bn[w * na * nb + a + na * b];
                free(scn);
            }
            free(Fb);
            free(bo);
            free(bn);
        }
    }
    free(sc);
    free(vt);
    free(Ftb);
}

int orc_residual_vjp(const orc_mesh *m, const int *orders, const double *u, const double *v, double *out, int form,
                     int isolated)
{
    if (check_box_euler(m, orders, form)) return -1;
    ensure_tables();
    int E = m->nx * m->ny * m->nz;
    long *off = node_offsets(E, orders);
#pragma omp parallel for schedule(guided)
    for (int e = 0; e < E; ++e) vjp_elem(m, orders, off, u, v, e, form, isolated, out + NV * off[e]);
    free(off);
    return 0;
}

/* Threads of the OpenMP loops over elements (timing on a stated core count). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
