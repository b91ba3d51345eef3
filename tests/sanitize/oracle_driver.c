/* Runs the oracle's entry points on small mixed-order meshes (box with periodic, wall and
 * far-field faces; the sine-mapped curved mesh; Navier-Stokes) so that a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer checks every access and operation they
 * make.  Exit status 0 when every call returns 0. */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/dg_oracle.h"

static unsigned long long rng = 88172645463325252ull;
static double urand(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

static void state(long n, const int *o, int E, double *u) {
    long off = 0;
    for (int e = 0; e < E; ++e) {
        long ne = (long)(o[3 * e] + 1) * (o[3 * e + 1] + 1) * (o[3 * e + 2] + 1);
        for (long k = 0; k < ne; ++k) {
            double rho = 0.8 + 0.4 * urand(), vx = 0.6 * urand() - 0.3, vy = 0.6 * urand() - 0.3;
            double vz = 0.6 * urand() - 0.3, p = 0.8 + 0.4 * urand();
            double *b = u + 5 * off;
            b[0 * ne + k] = rho;
            b[1 * ne + k] = rho * vx;
            b[2 * ne + k] = rho * vy;
            b[3 * ne + k] = rho * vz;
            b[4 * ne + k] = p / 0.4 + 0.5 * rho * (vx * vx + vy * vy + vz * vz);
        }
        off += ne;
    }
    (void)n;
}

#define CHECK(x)                                                    \
    do {                                                            \
        if ((x) != 0) {                                             \
            fprintf(stderr, "%s failed at line %d\n", #x, __LINE__); \
            return 1;                                               \
        }                                                           \
    } while (0)

static int run(orc_mesh *m, int lo, int hi, int ns, int derivs) {
    const int E = m->nx * m->ny * m->nz;
    int *o = malloc(sizeof(int) * 3 * E), *co = malloc(sizeof(int) * 3 * E);
    for (int i = 0; i < 3 * E; ++i) {
        o[i] = lo + (int)(urand() * (hi - lo + 1));
        if (m->map_kind && o[i] < m->geo_order[i % 3]) o[i] = m->geo_order[i % 3];
        co[i] = 1 + (int)(urand() * o[i]);
        if (co[i] > o[i]) co[i] = o[i];
    }
    const long n = orc_num_nodes(E, o), nc = orc_num_nodes(E, co);
    double *u = malloc(sizeof(double) * 5 * n), *r = malloc(sizeof(double) * 5 * n);
    double *v = malloc(sizeof(double) * 5 * n), *w = malloc(sizeof(double) * 5 * n);
    double *tn = malloc(sizeof(double) * 5 * nc), *tt = malloc(sizeof(double) * 5 * nc);
    double *norms = malloc(sizeof(double) * 2 * E), *vn = malloc(sizeof(double) * 10 * E);
    double *eta = malloc(sizeof(double) * E), *xyz = malloc(sizeof(double) * 3 * n);
    double *met = malloc(sizeof(double) * 10 * n);
    state(n, o, E, u);
    for (long i = 0; i < 5 * n; ++i) v[i] = urand() - 0.5;
    CHECK(orc_node_coords(m, o, xyz) < 0);
    CHECK(orc_metrics(m, o, met) < 0);
    for (int form = 0; form < 2; ++form)
        for (int iso = 0; iso < 2; ++iso) CHECK(orc_residual(m, o, u, r, form, iso));
    CHECK(orc_residual(m, o, u, r, 0, 0));
    for (int iso = 0; iso < 2; ++iso)
        for (int rs = 0; rs < 2; ++rs) CHECK(orc_tau(m, o, co, u, r, iso, rs, tn, tt, norms, vn));
    CHECK(orc_tau_eta(m, o, co, u, r, 0, 0, v, 0, eta));
    long nt = 0;
    for (int e = 0; e < E; ++e) nt += orc_num_combos(o + 3 * e);
    double *te = malloc(sizeof(double) * nt), *te2 = malloc(sizeof(double) * nt);
    int *el = malloc(sizeof(int) * E);
    for (int e = 0; e < E; ++e) el[e] = e;
    CHECK(orc_sweep(m, o, u, r, 0, el, E, te, te2));
    if (ns) {
        CHECK(orc_residual_ns(m, o, u, 0.01, 0.72, w, 0, 0));
        CHECK(orc_sweep_ns(m, o, u, w, 0.01, 0.72, 1, el, E, te, te2));
    }
    if (derivs) {
        CHECK(orc_residual_jvp(m, o, u, v, w, 0, 0));
        CHECK(orc_residual_vjp(m, o, u, v, w, 1, 0));
        double J;
        CHECK(orc_functional(m, o, u, &J, w));
        CHECK(orc_rk3(m, o, u, 1e-4, 2));
        CHECK(orc_project(E, o, co, u, tn));
    }
    free(o); free(co); free(u); free(r); free(v); free(w); free(tn); free(tt); free(norms); free(vn);
    free(eta); free(xyz); free(met); free(te); free(te2); free(el);
    return 0;
}

int main(void) {
    orc_mesh box = {3, 2, 2, {0, 0, 0}, {1, 0.7, 1.3}, {1, 2, 0, 0, 0, 0}, 0, 1.4, {1.1, 0.3, 0.1, -0.2, 2.6},
                    0, 0.0, {1, 1, 1}};
    if (run(&box, 1, 7, 1, 1)) return 1;
    box.flux = 1;
    box.bc[0] = box.bc[1] = 0;
    box.bc[2] = 2; box.bc[3] = 1;
    if (run(&box, 1, 9, 0, 1)) return 1;
    orc_mesh curved = {2, 2, 2, {0, 0, 0}, {1, 1, 1}, {0, 0, 0, 0, 0, 0}, 0, 1.4, {1, 0.3, 0, 0, 2.5},
                       1, 0.05, {2, 2, 1}};
    if (run(&curved, 2, 6, 1, 0)) return 1;
    printf("oracle driver ok\n");
    return 0;
}
