/*
 * dg_oracle.h -- plain, slow FP64 CPU oracle for the DGSEM residual and the
 * anisotropic truncation-error (tau) estimate of Rueda-Ramirez, Ferrer, Rubio
 * et al., "Truncation error-based anisotropic p-adaptation for unsteady flows
 * for high-order discontinuous Galerkin methods" (arXiv 2210.03523).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * Conventions (all arrays are host memory owned by the caller):
 *   - Box mesh of nx*ny*nz equal hexahedra on [lo,hi]; element e = ix + nx*(iy + ny*iz).
 *   - orders[e*3 + d] = polynomial order N_d (1..ORC_NMAX) of element e in direction d.
 *   - Natural ragged layout: element e occupies 5*n_e doubles starting at
 *     5*noff(e), noff = prefix sum of n_e = (N1+1)(N2+1)(N3+1); inside the
 *     element [var][node], node = i + n1*(j + n2*k).
 *   - Conserved variables (rho, rho u, rho v, rho w, rho E).
 *   - Return value 0 on success, -1 on invalid arguments.
 */
#ifndef DG_ORACLE_H
#define DG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NMAX 12

typedef struct {
    int nx, ny, nz;
    double lo[3], hi[3];
    int bc[6];       /* faces -x,+x,-y,+y,-z,+z: 0 periodic, 1 slip wall, 2 far field */
    int flux;        /* 0 Roe, 1 Lax-Friedrichs (Rusanov) */
    double gamma;
    double qfar[5];  /* far-field state (conserved) */
    /* Geometry.  map_kind 0: the box elements themselves (affine).  map_kind 1: the
     * box point (x, y, z) is moved to (x + f, y + f, z) with
     *   f = map_amp sin(2 pi (x - lo_x)/(hi_x - lo_x)) sin(2 pi (y - lo_y)/(hi_y - lo_y)),
     * each element's geometry being the tensor-product Gauss-Lobatto interpolant of
     * that map of order geo_order[d] (sampled at the element's own nodes), and the
     * metric terms Ja^d and J the cross products of the collocation derivatives of the
     * node coordinates (Section 2.1: the mapping of each element onto the reference
     * cube).  Curved elements need orders >= geo_order in every direction for the
     * fine solution; coarse maps of the tau-estimate may go lower (their geometry is
     * the same interpolant sampled at the coarse nodes). */
    int map_kind;
    double map_amp;
    int geo_order[3];
} orc_mesh;

/* 1D tables on Legendre-Gauss-Lobatto nodes. x,w: N+1 entries; D: (N+1)^2 row-major. */
int orc_lgl(int N, double *x, double *w);
int orc_dmat(int N, double *D);
/* I[a*(N+1)+k] = l^N_k(x^M_a): samples the order-N interpolant at the order-M nodes. */
int orc_interp(int M, int N, double *I);
/* L2 projection from order K to order N (N <= K), (N+1)x(K+1) row-major. */
int orc_proj(int N, int K, double *P);

/* Physical flux f.n and numerical flux (kind 0 Roe, 1 LF). */
void orc_flux_n(const double *q, const double *n, double gamma, double *f);
void orc_numflux(const double *qL, const double *qR, const double *n, double gamma,
                 int kind, double *f);
/* Roe wave decomposition: lam[4], wave[4*5] = alpha_k * r_k. */
void orc_roe_waves(const double *qL, const double *qR, const double *n, double gamma,
                   double *lam, double *wave);

/* Node coordinates, natural ragged layout [e][3][node]. */
int orc_node_coords(const orc_mesh *m, const int *orders, double *xyz);
/* Metric terms, natural ragged layout [e][10][node]: Ja^1 (x,y,z), Ja^2, Ja^3, J. */
int orc_metrics(const orc_mesh *m, const int *orders, double *met);
long orc_num_nodes(int E, const int *orders);

/* Spatial residual. form 0: new form r = M^-1 F^N = -dQ/dt; form 1: traditional
 * F^N = M r.  isolated != 0 drops every surface term. */
int orc_residual(const orc_mesh *m, const int *orders, const double *u, double *r,
                 int form, int isolated);

/* Element-wise restriction (sampling of the fine polynomial at coarse nodes). */
int orc_restrict(int E, const int *fine_orders, const int *coarse_orders,
                 const double *u, double *uc);

/* Transfer of a solution onto another order map: per element and direction,
 * interpolation where the order rises or stays, exact L2 projection where it falls
 * (Section 2.4.1, the solution projected onto the new polynomial spaces). */
int orc_project(int E, const int *from_orders, const int *to_orders, const double *u, double *ut);

/* Coupled (isolated=0) or isolated tau-estimate on one coarse order map.
 * dudt: fine r = -dQ/dt (new form, non-isolated residual of u on the fine map).
 * restriction: the operator I^N of the estimate (Section 2.3), 0 = sampling at the
 * coarse nodes, 1 = exact L2 projection onto the coarse tensor-product space.
 * Outputs in the coarse natural ragged layout; norms[e*2+{0,1}] = max |tau_new|,
 * max |tau_trad| over nodes and variables; varnorms[(e*2+f)*5+v] (nullable). */
int orc_tau(const orc_mesh *m, const int *fine_orders, const int *coarse_orders,
            const double *u, const double *dudt, int isolated, int restriction,
            double *tau_new, double *tau_trad, double *norms, double *varnorms);

/* Backward-difference weights: rate at t_{n+1} = (1/dt) sum_j w[j] Q(t_{n+1-j}),
 * j = 0..k (exact for polynomials of degree k in time). */
int orc_bdf_weights(int k, double *w);
/* Dual time-stepping estimate (Section 2.3, item 2) with the backward difference of
 * order nstates-1 over stored fine solutions states[j] = Q^P(t_{n+1-j}):
 * tau_new = (delta_p/delta t)(I Q) + (M^N)^-1 F^N(I Q_0); tau_trad = J w w w tau_new. */
int orc_tau_dual(const orc_mesh *m, const int *fine_orders, const int *coarse_orders, const double *const *states,
                 int nstates, double dt, int isolated, double *tau_new, double *tau_trad);

/* Number of coarse combinations of an element: prod_d max(1, N_d - 1). */
int orc_num_combos(const int *order3);
/* Threads of the OpenMP loops over elements (for timing on a stated core count). */
void orc_set_threads(int n);
int orc_max_threads(void);
/* Isolated sweep over every coarse combination (c1 fastest, then c2, then c3;
 * c_d in 1..max(1,N_d-1)) for the listed elements (natural indices); restriction as
 * for orc_tau.
 * te_new/te_trad: for list entry i, the combos of element elems[i] are stored
 * contiguously, entries ordered as the list. */
int orc_sweep(const orc_mesh *m, const int *orders, const double *u, const double *dudt, int restriction,
              const int *elems, int nelems, double *te_new, double *te_trad);

/* The isolated sweep for the Navier-Stokes equations (BR1 gradients with the
 * isolated flag, viscous flux of constant mu and Prandtl number Pr). */
int orc_sweep_ns(const orc_mesh *m, const int *orders, const double *u, const double *dudt, double mu,
                 double Pr, int restriction, const int *elems, int nelems, double *te_new, double *te_trad);

/* Adjoint-weighted truncation error (used with an adjoint state psi on the fine
 * layout): eta[e] = sum over coarse nodes and variables of (I psi_t) * tau_trad, where
 * psi_t is the adjoint of the traditional-form residual F (a nodal field): psi itself for
 * psi_form 1, and psi / (J w_i w_j w_k) for psi_form 0, the adjoint of the new form
 * M^-1 F (which is M psi_t).  The estimate of the functional error is -sum(eta). */
int orc_tau_eta(const orc_mesh *m, const int *fine_orders, const int *coarse_orders,
                const double *u, const double *dudt, int isolated, int restriction, const double *psi,
                int psi_form, double *eta);

/* Pressure force along x on the slip walls: J = sum over slip-wall faces with
 * normal +-e_x of sum_{a,b} w_a w_b |Ja^1| p(Q) n_x; dJdu (nullable, natural
 * layout) receives dJ/dQ (zero away from those faces). */
int orc_functional(const orc_mesh *m, const int *orders, const double *u, double *J, double *dJdu);

/* Navier-Stokes with the BR1 viscous discretisation (first-order system of
 * Section 2.1, eqs. SystemAdvDiff and DGSEMsystem:2).  Gradients of the conserved
 * variables: grad natural layout [e][3][5][node] (d(var)/dx_l at each node).
 * Constant viscosity mu, Stokes hypothesis, heat conductivity mu gamma/((gamma-1) Pr)
 * acting on T = p/rho.  isolated drops every surface term of both passes. */
int orc_gradient(const orc_mesh *m, const int *orders, const double *u, int isolated, double *grad);
int orc_residual_ns(const orc_mesh *m, const int *orders, const double *u, double mu, double Pr,
                    double *r, int form, int isolated);
/* Viscous flux f^v_d(Q, G) along direction d, G[l*5 + v] = d(var v)/dx_l. */
void orc_viscous_flux(const double *q, const double *G, int d, double gamma, double mu, double Pr, double *f);

/* Derivatives of the residual (box Euler meshes, map_kind 0; form and isolated as for
 * orc_residual).  Natural layout for u, dir, v and the outputs.
 *   orc_residual_cstep: real and imaginary parts of the residual evaluated in complex
 *     arithmetic at u + i h dir (r_re or r_im may be NULL).
 *   orc_residual_jvp: (d r / d u) dir by complex step (h = 1e-30), exact to rounding.
 *   orc_residual_vjp: (d r / d u)^T v, every step of the residual transposed by hand. */
int orc_residual_cstep(const orc_mesh *m, const int *orders, const double *u, const double *dir, double h,
                       double *r_re, double *r_im, int form, int isolated);
int orc_residual_jvp(const orc_mesh *m, const int *orders, const double *u, const double *dir, double *out, int form,
                     int isolated);
int orc_residual_vjp(const orc_mesh *m, const int *orders, const double *u, const double *v, double *out, int form,
                     int isolated);
/* Jacobian of the physical flux f.n, A[i*5 + j] = d (f.n)_i / d q_j (closed form). */
void orc_flux_jacobian(const double *q, const double *n, double gamma, double *A);
/* Jacobians of the numerical flux (kind 0 Roe, 1 LF) in either state by complex step,
 * AL[i*5 + j] = d f*_i / d qL_j and AR likewise. */
void orc_numflux_jacobian(const double *qL, const double *qR, const double *n, double gamma, int kind, double *AL,
                          double *AR);

/* Williamson low-storage RK3, nsteps steps of size dt, in place on u. */
int orc_rk3(const orc_mesh *m, const int *orders, double *u, double dt, int nsteps);

#ifdef __cplusplus
}
#endif
#endif
