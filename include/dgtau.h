/*
 * dgtau.h -- C ABI of the MI355X (gfx950) DGSEM residual and anisotropic
 * truncation-error estimation library.
 *
 * Method: Rueda-Ramirez, Ferrer, Rubio et al., "Truncation error-based
 * anisotropic p-adaptation for unsteady flows for high-order discontinuous
 * Galerkin methods" (arXiv 2210.03523).
 *
 * General rules
 *   - Every function returns a dg_status; DG_OK == 0.  On failure the text of
 *     the error is available from dg_last_error() (thread-local).  Nothing
 *     throws across this interface.
 *   - Device pointers are HIP device memory owned by the caller; host pointers
 *     are marked "host".  Device arrays must be 16-byte aligned (every hipMalloc
 *     or torch allocation is); a misaligned one returns DG_EINVAL.  Compute calls
 *     are asynchronous on the given stream (NULL = the legacy default stream) and
 *     allocate no device memory.  The exception is the first RK3 call with a new
 *     (u, g, dt) pointer set: it captures and instantiates a HIP graph (host-side
 *     runtime allocations); each plan and batch keeps at most 8 such graphs and
 *     destroys the least recently used one, after a device synchronisation, to
 *     make room.  Set-up calls allocate where their comments say so (plan and
 *     batch creation, the adaptation loops, the adjoint preconditioner's
 *     factorisation workspace).
 *   - Plans own only their internal device buffers (tables, tiles, face lists,
 *     face-flux and tau scratch).  A plan is immutable after creation; because
 *     it holds scratch buffers, one plan must not be used by two streams at once.
 *   - Device state arrays use the PLAN LAYOUT: elements stable-sorted by
 *     (node-count class, N1, N2, N3, natural index); element p occupies
 *     5 * n_p consecutive values starting at 5 * node_offset[p], ordered
 *     [var][node] with node = i + n1*(j + n2*k), n_d = N_d + 1, variables
 *     (rho, rho u, rho v, rho w, rho E).  dg_plan_layout() returns the
 *     permutation and offsets.
 */
#ifndef DGTAU_H
#define DGTAU_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dg_status;
enum {
    DG_OK = 0,
    DG_EINVAL = -1,       /* invalid argument (null pointer, bad order, size mismatch) */
    DG_ENOMEM = -2,       /* device or host allocation failed (plan creation only) */
    DG_EHIP = -3,         /* a HIP runtime call failed; message in dg_last_error() */
    DG_EUNSUPPORTED = -4, /* valid request this build does not implement */
    DG_ENONPHYSICAL = -5  /* a state holds non-physical values (dg_check_state) */
};

enum { DG_BC_PERIODIC = 0, DG_BC_SLIP_WALL = 1, DG_BC_FARFIELD = 2 };
enum { DG_EULER = 0, DG_NAVIER_STOKES = 1 };
enum { DG_FLUX_ROE = 0, DG_FLUX_LF = 1 };
enum { DG_MAP_BOX = 0, DG_MAP_SINE = 1 };
enum { DG_F64 = 0, DG_F32 = 1 };
/* Residual forms (Section 2.2): NEW = M^-1 F^N(Q) = -dQ/dt, TRAD = F^N(Q) = M * NEW. */
enum { DG_FORM_NEW = 0, DG_FORM_TRAD = 1 };
/* Restriction operator I of the tau-estimate (Section 2.3, the operator of eq.
 * TEderivation1 that maps the fine solution into the coarse space): sampling of the
 * fine element polynomial at the coarse Gauss-Lobatto nodes (the paper's choice), or
 * the exact L2 projection onto the coarse tensor-product space of the reference cube. */
enum { DG_RESTRICT_SAMPLE = 0, DG_RESTRICT_L2 = 1 };
/* Capacity, in doubles, of the static scratch of dg_residual_noalloc (64 MiB). */
#define DG_NOALLOC_SCRATCH_DOUBLES (8 * 1024 * 1024)

#define DG_NMAX 9 /* polynomial orders 1..DG_NMAX in every direction */

typedef struct dg_plan_s *dg_plan;

/* Structured box mesh of nx*ny*nz equal hexahedra on [lo, hi]; natural element
 * index e = ix + nx*(iy + ny*iz).  bc[] per box face in the order -x,+x,-y,+y,-z,+z;
 * a periodic pair must be periodic on both sides.
 * Geometry (Section 2.1: each element is mapped onto the reference cube, fluxes are
 * contravariant, Ft^d = Ja^d . f, and J is the Jacobian of the map):
 *   map_kind DG_MAP_BOX: the axis-aligned box elements (constant metric terms).
 *   map_kind DG_MAP_SINE: the box point (x, y, z) moves to (x + f, y + f, z),
 *     f = map_amp sin(2 pi (x - lo_x)/(hi_x - lo_x)) sin(2 pi (y - lo_y)/(hi_y - lo_y));
 *     each element's geometry is the tensor-product Gauss-Lobatto interpolant of the
 *     map of order geo_order (sampled at the element's nodes); the metric terms are
 *     the cross products of the collocation derivatives of the node coordinates
 *     (exact discrete metric identities for this quasi-2D map).  Fine orders must be
 *     >= geo_order per direction; coarse plans sample the same geometry at their
 *     nodes.  On faces the minus side's Ja^d, interpolated onto the mortar, is the
 *     scaled normal of the Riemann problem. */
typedef struct {
    int32_t nx, ny, nz;
    double lo[3], hi[3];
    int32_t bc[6];
    int32_t flux;     /* DG_FLUX_ROE (the paper's advective flux) or DG_FLUX_LF */
    double gamma;     /* ratio of specific heats */
    double q_far[5];  /* conserved far-field state for DG_BC_FARFIELD faces */
    int32_t equation; /* DG_EULER or DG_NAVIER_STOKES (BR1, Section 2.1 eqs. SystemAdvDiff) */
    double mu;        /* Navier-Stokes: constant dynamic viscosity (nondimensional, 1/Re) */
    double Pr;        /* Navier-Stokes: Prandtl number; heat conductivity mu gamma/((gamma-1) Pr) on T = p/rho */
    int32_t map_kind; /* DG_MAP_BOX or DG_MAP_SINE */
    double map_amp;   /* DG_MAP_SINE: amplitude of f */
    int32_t geo_order[3]; /* DG_MAP_SINE: geometry order per direction, 1..DG_NMAX */
} dg_mesh_desc;

/* Build a plan for the compressible Euler or Navier-Stokes DGSEM (Section 2.1) on
 * the mesh with per-element anisotropic orders.  Navier-Stokes uses the BR1 scheme
 * of the paper's set-up: gradients of the conserved variables from the averaged
 * solution trace, viscous face flux = average of both sides' viscous fluxes; at
 * boundaries the ghost state carries the inner gradient.  Navier-Stokes plans
 * support orders up to 7, and neither the VJP nor batches (DG_EUNSUPPORTED).
 * Curved (DG_MAP_SINE) plans need orders >= the geometry order and support the
 * residual, RK3, the tau-estimate (coupled: coarse orders >= the geometry order too,
 * so that the coarse faces stay watertight) and the sweep (fine orders up to 7); the
 * VJP, the functional and batches return DG_EUNSUPPORTED.
 *   orders_host: host int32 [E][3], natural element order, each in 1..DG_NMAX.
 *   out: receives the plan (release with dg_plan_destroy).
 * Errors: DG_EINVAL (bad mesh, orders or periodic pairing), DG_ENOMEM, DG_EHIP. */
dg_status dg_plan_create(const dg_mesh_desc *mesh, const int32_t *orders_host, dg_plan *out);

/* Build the coarse plan of a tau-estimate (Section 2.3): the same mesh with
 * coarse orders 1 <= Nc <= Nf per element and direction.  The coarse plan keeps
 * a reference to the fine one; destroy it before the fine plan. */
dg_status dg_plan_create_coarse(dg_plan fine, const int32_t *coarse_orders_host, dg_plan *out);

dg_status dg_plan_destroy(dg_plan plan);

/* Layout queries (host outputs, any may be NULL):
 *   n_elems, n_nodes: element and node counts;
 *   perm[E]: natural index of plan element p;
 *   node_offset[E+1]: first node of plan element p (prefix sums of n_p);
 *   orders[E*3]: orders of plan element p. */
dg_status dg_plan_layout(dg_plan plan, int64_t *n_elems, int64_t *n_nodes, int64_t *perm,
                         int64_t *node_offset, int32_t *orders);

/* Node coordinates in the plan layout, device double [E] blocks of [3][n_p]
 * (x, y, z of every node, same node order as the state). */
dg_status dg_node_coords(dg_plan plan, double *xyz, hipStream_t stream);

/* Metric terms in the plan layout, device double [E] blocks of [10][n_p]:
 * Ja^1 (x, y, z), Ja^2 (x, y, z), Ja^3 (x, y, z), J at every node (Section 2.1). */
dg_status dg_plan_metrics(dg_plan plan, double *met, hipStream_t stream);

/* Spatial residual of the DGSEM semi-discretisation (Section 2.1, eqs.
 * DGSEMsystem, DGMassMatrixLeft/Right), strong form on Gauss-Lobatto nodes:
 *   form DG_FORM_NEW:  r = M^-1 F^N(u)  (= -du/dt)
 *   form DG_FORM_TRAD: r = F^N(u)        (= M * new form)
 * isolated != 0 evaluates the isolated operator (end of Section 2.2): surface
 * numerical fluxes replaced by the inner flux, i.e. no surface terms.
 *   u, r: device arrays of 5*n_nodes values of type dtype (DG_F64: double,
 *   DG_F32: float), plan layout; u and r must not overlap. */
dg_status dg_residual(dg_plan plan, const void *u, void *r, int32_t dtype, int32_t form,
                      int32_t isolated, hipStream_t stream);

/* Allocation-free residual, for callers that cannot allocate device memory or call
 * anything that may (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same computation and arguments as dg_residual, with
 * the face-flux and BR1-gradient scratch taken from one static device array of
 * DG_NOALLOC_SCRATCH_DOUBLES doubles (64 MiB) per GPU instead of the plan's buffers.
 * The array is held by every GPU the call runs on until the process ends; its device
 * address is looked up on the first call on each device.  A plan needing more
 * scratch (6 face slots x 5 variables x face nodes per element, tripled for curved
 * Navier-Stokes plans, plus 15 doubles per node for Navier-Stokes gradients; the 16^3
 * order-7 mesh needs 7.9 Mi doubles) returns DG_EINVAL.  All calls on one GPU share
 * the array: calls that overlap on one GPU (two streams, or two host threads) race,
 * and the caller must serialise them.  The plan's device must be current. */
dg_status dg_residual_noalloc(dg_plan plan, const void *u, void *r, int32_t dtype, int32_t form, int32_t isolated,
                              hipStream_t stream);

/* Tau-estimate on the coarse order map of `coarse` (Section 2.3, eqs. TEtildedef
 * and TEdef with the variational DG estimate I F(q) ~ I (M^P)^-1 F^P(q^P)):
 *   tau_new  = r^Nc(I u) - I dudt        (new form, "without the mass matrix")
 *   tau_trad = J w_i w_j w_k * tau_new    (traditional form, coarse weights)
 * I = the restriction operator: DG_RESTRICT_SAMPLE or DG_RESTRICT_L2.
 *   u: device double, fine plan layout (5*n_fine values).
 *   dudt: device double fine new-form residual -du/dt (non-isolated), or NULL to
 *         have it computed here into the fine plan's scratch.
 *   isolated: 0 coupled coarse residual (mortars between coarse orders), 1 isolated.
 *   restriction: DG_RESTRICT_SAMPLE or DG_RESTRICT_L2, for u, dudt and psi alike.
 *   tau_new, tau_trad: device double, coarse plan layout (either may be NULL).
 *   norms: device double [E_coarse][2], max |tau_new|, max |tau_trad| over nodes and
 *          the 5 variables of each coarse plan element (may be NULL).
 *   varnorms: device double [E_coarse][2][5], the same maxima per variable (max over
 *          nodes of |tau_new| for each of the 5 conserved variables, then of |tau_trad|);
 *          may be NULL.
 *   psi, eta: optional adjoint weighting (both NULL or both set): psi is a fine-layout
 *          device double field, the adjoint of a functional (e.g. dg_adjoint_solve's
 *          solution for dg_functional's gradient) for the residual of form psi_form;
 *          eta[E_coarse] receives sum over coarse nodes and variables of (I psi_t) * tau_trad,
 *          psi_t the traditional-form adjoint, a nodal field: psi itself for
 *          psi_form = DG_FORM_TRAD; for DG_FORM_NEW the adjoint of M^-1 F, which is M psi_t,
 *          so psi is divided by the fine mass matrix M = J w_i w_j w_k before the
 *          restriction.  Either consistent pair gives the same eta (Section 2.2: the
 *          truncation error and functional errors); the functional error estimate is
 *          -sum(eta).
 *   psi_form: DG_FORM_TRAD or DG_FORM_NEW (ignored without psi).
 * Errors: DG_EINVAL (null u, foreign coarse plan, psi without eta, bad restriction or
 * psi_form, misaligned arrays), DG_EUNSUPPORTED (coupled estimate on a curved mesh with a
 * coarse order below the geometry order), DG_EHIP. */
dg_status dg_tau_estimate(dg_plan fine, dg_plan coarse, const double *u, const double *dudt,
                          int32_t isolated, int32_t restriction, double *tau_new, double *tau_trad,
                          double *norms, double *varnorms, const double *psi, int32_t psi_form, double *eta,
                          hipStream_t stream);

/* Number of coarse combinations per fine plan element for the sweep:
 * prod_d max(1, N_d - 1); combo_offset[E+1] (host) gets their prefix sums. */
dg_status dg_sweep_layout(dg_plan fine, int64_t *combo_offset);

/* Isolated anisotropic truncation-error map (Section 2.3 and Section 2.4.2,
 * approach 2): for every fine plan element and every coarse combination
 * (c1, c2, c3), c_d in 1..max(1, N_d - 1), enumerated c1 fastest, the maxima
 * over nodes and variables of |tau_new| and |tau_trad| of the isolated estimate
 * (Euler or Navier-Stokes; on curved plans the element's geometry sampled at the
 * coarse nodes whatever the restriction).  Fine orders up to 9 (7 for Navier-Stokes
 * and curved plans).
 *   u, dudt: device double, fine plan layout (dudt as for dg_tau_estimate,
 *            NULL computes it).
 *   restriction: DG_RESTRICT_SAMPLE or DG_RESTRICT_L2 (of u and dudt).
 *   te_new, te_trad: device double [combo_offset[E]] (dg_sweep_layout). */
dg_status dg_tau_sweep(dg_plan fine, const double *u, const double *dudt, int32_t restriction,
                       double *te_new, double *te_trad, hipStream_t stream);

/* Polynomial-degree selection from truncation-error maps (Section 2.4.2, static
 * p-adaptation, approaches 1 and 2 with the maximum aggregator F_max; jump
 * conditions of Section 3.1, eqs. (a) N >= floor(2/3 N_j) and (b) N >= N_j - 1).
 *
 * A combination (N1, N2, N3) of a map qualifies when its value is below tau_max and every
 * N_i lies in [nmin, nmax].  Maps in the sweep layout (ext_nmax = 0) hold the
 * combinations below the plan's orders P only: those at or above P have the high value
 * of the paper's fallback.  Extended maps (ext_nmax > 0, from dg_tau_extrapolate) hold
 * every N_i in 1..ext_nmax, with the extrapolated value or the high value at N_i >= P_i.
 * Among the qualifying combinations the one with the fewest degrees of freedom
 * prod (N_i + 1) is selected; ties go to the smaller map value, then to the smaller
 * (N1, N2, N3) compared lexicographically (N1 first).  An element without a qualifying
 * combination gets (nmax, nmax, nmax).
 *   approach 1: select per map (one map per estimation stage), then the maximum
 *               over the stages in every direction;
 *   approach 2: a combination qualifies when it does in every map (the F_max total
 *               map below tau_max); its value is the maximum over the maps.
 * With prev (the current degrees, device int32 [E][3] natural order), no degree falls
 * by more than max_decrease: N_i >= min(nmax, prev_i - max_decrease) (Section 3.2,
 * dynamic adaptation: one order per stage).
 * The jump condition (jump 1: (a), jump 2: (b), 0: none) is then enforced against
 * the face neighbours (across periodic box faces too), in the matching direction,
 * by raising degrees to the least fixed point.  Integer results are exact; a NaN in
 * a map never qualifies.
 *   maps: host array of nstages (1..DG_SELECT_MAX_STAGES) device double pointers,
 *         each a map in the layout of dg_tau_sweep (te_new or te_trad), or with
 *         ext_nmax > 0 in the extended layout of dg_tau_extrapolate.
 *   orders: device int32 [E][3], natural element order (the layout dg_plan_create
 *           takes), written by the call; the plan's own scratch holds the
 *           intermediate degrees, so one plan runs one selection at a time.
 * Errors: DG_EINVAL for null arguments, nstages outside 1..DG_SELECT_MAX_STAGES,
 * approach not 1 or 2, jump not 0..2, 1 <= nmin <= nmax <= DG_NMAX violated, a
 * NaN tau_max, a negative max_decrease, or ext_nmax outside 0..DG_NMAX or below nmax
 * when positive; DG_EHIP for launch failures.  Asynchronous on stream. */
#define DG_SELECT_MAX_STAGES 32
typedef struct {
    double tau_max;
    int32_t nmin, nmax;
    int32_t approach; /* 1 or 2 */
    int32_t jump;     /* 0 none, 1 (a), 2 (b) */
    const int32_t *prev;  /* NULL, or current degrees (device, [E][3] natural) */
    int32_t max_decrease; /* with prev: largest decrease per direction, >= 0 */
    int32_t ext_nmax;     /* 0: maps in the sweep layout; > 0: extended maps of that nmax */
} dg_select_params;

dg_status dg_select_orders(dg_plan fine, const double *const *maps, int32_t nstages,
                           const dg_select_params *params, int32_t *orders, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Adaptation loops (Section 2.4): the flowcharts of dynamic and static
 * p-adaptation, every step in this library's kernels: RK3 steps (as
 * dg_rk3_step, launched directly), the isolated truncation-error map
 * (dg_tau_sweep, the fine time derivative computed from the state), the degree
 * selection (dg_select_orders), a new plan for the selected degrees and the
 * projection of the state onto it (dg_project).
 * ------------------------------------------------------------------------- */
typedef struct {
    double dt;                /* RK3 time step */
    int32_t steps_per_stage;  /* RK3 steps between estimations (Delta t_e), >= 0 */
    int32_t nstages;          /* estimation stages, 1..DG_SELECT_MAX_STAGES */
    int32_t steps_after;      /* static loop: RK3 steps after the adaptation (to the final time) */
    int32_t restriction;      /* DG_RESTRICT_SAMPLE or DG_RESTRICT_L2 */
    int32_t form;             /* map used for the selection: DG_FORM_NEW (te_new) or DG_FORM_TRAD */
    dg_select_params select;  /* tau_max, nmin, nmax, approach (static loop), jump, max_decrease
                                 (dynamic loop); prev and ext_nmax must be 0 */
} dg_adapt_params;

typedef struct {
    int64_t steps;      /* S: RK3 steps taken */
    double ndof_dyn;    /* (1/S) sum over the steps of the step's number of degrees of freedom
                           (nodes), the weighted average of Section 3.2 */
    int64_t ndof_final; /* nodes of the final plan */
} dg_adapt_report;

/* Dynamic p-adaptation (Section 2.4.1 and its flowchart; the decrease limit of Section
 * 3.2): nstages times { advance steps_per_stage RK3 steps; estimate the isolated map
 * on the current plan; select degrees from it (prev = the current degrees, no degree
 * falling by more than select.max_decrease, then the jump condition); build the plan of
 * the selected degrees and project the state onto it }.
 *   plan: in, the initial plan (never destroyed); out, the final plan, a new plan owned
 *         by the caller when any stage changed the degrees (intermediate plans are
 *         destroyed).  Box meshes; orders and select.nmax <= 7 for Navier-Stokes.
 *   u: device double of capacity values: in, the state in the initial plan's layout;
 *      out, the state in the final plan's layout.  work: device double of capacity
 *      values (RK register and projection scratch).  capacity >= 5 E (nmax+1)^3 and
 *      >= 5 n_nodes of the initial plan.
 *   stage_orders: host int32 [nstages][E][3] (nullable), the degrees selected at every
 *      stage (natural element order).  report: nullable.
 * Allocates the loop's maps and degree buffers and each stage's plan (the storage
 * reallocation the paper names); synchronous on stream (each stage reads its degrees
 * back).  Errors: DG_EINVAL, DG_EUNSUPPORTED (curved plans, orders above the sweep's),
 * DG_ENOMEM, DG_EHIP. */
dg_status dg_adapt_dynamic(dg_plan *plan, double *u, double *work, int64_t capacity, const dg_adapt_params *params,
                           int32_t *stage_orders, dg_adapt_report *report, hipStream_t stream);

/* Static p-adaptation (Section 2.4.2 and its flowchart): nstages times { advance
 * steps_per_stage RK3 steps; estimate the isolated map and store it } on the initial
 * plan; at T_e one selection from all stored maps (select.approach 1: per map then the
 * maximum per direction; 2: the F_max total map, eq. totalTruncMap), the jump
 * condition, the plan of the selected degrees and the projection onto it; then
 * steps_after RK3 steps on the new plan.  Arguments as dg_adapt_dynamic, except
 *   orders: host int32 [E][3] (nullable), the degrees of the adaptation;
 *   select.max_decrease is ignored.
 * Errors as dg_adapt_dynamic. */
dg_status dg_adapt_static(dg_plan *plan, double *u, double *work, int64_t capacity, const dg_adapt_params *params,
                          int32_t *orders, dg_adapt_report *report, hipStream_t stream);

/* Total truncation-error map of static adaptation (Section 2.4.2, eq. totalTruncMap with
 * F_max): acc <- max(acc, map) entry by entry, over the sweep layout of the plan
 * (dg_sweep_layout, ext_nmax = 0) or the extended layout of dg_tau_extrapolate
 * (ext_nmax > 0); a NaN in either operand gives NaN (it never qualifies in
 * dg_select_orders).  Selecting from the accumulated map equals approach 2 over the
 * individual stage maps.  acc, map: device double; they may be the same array.
 * Errors: DG_EINVAL for null arguments or ext_nmax outside 0..DG_NMAX.  Asynchronous
 * on stream. */
dg_status dg_map_fmax(dg_plan fine, double *acc, const double *map, int32_t ext_nmax, hipStream_t stream);

/* tau-extrapolation of an isolated truncation-error map to degrees at and above the
 * reference degree (Sections 1 and 2.3: the truncation error of smooth solutions decays
 * exponentially with the degree, so the map computed below P can be extended; Section
 * 2.4.2, last paragraph: approach 2 works on the extrapolated maps, and a direction
 * outside the asymptotic range gives the high value).  The paper cites the method
 * without stating it; this library's reading, per plan element of fine orders P with
 * computed degrees C_d = max(1, P_d - 1):
 *   - N_d <= C_d in every direction: the computed value;
 *   - otherwise, from the inner corner N' (N'_d = C_d where N_d > C_d, N_d elsewhere),
 *     along every direction d with N_d > C_d the map line through N' is fitted over its
 *     last L = min(3, C_d) degrees by least squares, ln tau = a + b_d n; the value is
 *     tau(N') prod_d exp(b_d (N_d - C_d)); a direction with L < 2, a value of its window
 *     that is not positive and finite, or b_d >= 0 gives +inf (the high value).
 *   map: device double, sweep layout of the plan (te_new or te_trad of dg_tau_sweep).
 *   nmax: 1..DG_NMAX, the largest degree of the extended map.
 *   ext: device double [E][nmax^3], plan element order, (N1, N2, N3) with N1 fastest,
 *        N_d in 1..nmax; not overlapping map.
 * Errors: DG_EINVAL (null or misaligned arrays, nmax outside 1..DG_NMAX).  Asynchronous
 * on stream. */
dg_status dg_tau_extrapolate(dg_plan fine, const double *map, int32_t nmax, double *ext, hipStream_t stream);

/* Solution transfer onto another order map of the same mesh (Section 2.4.1: after an
 * adaptation the solution is projected onto the new polynomial spaces).  Per element
 * and direction the 1D operator is the interpolation from the old to the new
 * Gauss-Lobatto nodes where the order rises or stays (the old polynomial belongs to the
 * new space) and the exact L2 projection where it falls; the element operator is their
 * tensor product, i.e. the L2 projection onto the new tensor-product space of the
 * reference element.
 *   from, to: plans of the same mesh (any orders; coarse plans allowed).
 *   u: device double, layout of from; ut: device double, layout of to (5 * n_nodes(to)),
 *      not overlapping u.
 * Errors: DG_EINVAL for null arguments or plans of different meshes.  FP64 only.
 * Asynchronous on stream. */
dg_status dg_project(dg_plan from, dg_plan to, const double *u, double *ut, hipStream_t stream);

/* Physical time derivative of the dual time-stepping estimate (Section 2.3, item 2):
 * dudt = -(1/dt) sum_j b_j states[j], the backward difference of order nstates-1 at
 * t_{n+1} over stored solutions states[j] = Q(t_{n+1-j}) on one plan (BDF1: b = (1, -1);
 * BDF2: (3/2, -2, 1/2); BDF3: (11/6, -3, 3/2, -1/3)).  Passed as dudt to dg_tau_estimate
 * or dg_tau_sweep it gives the dual time-stepping estimate
 * (delta_p/delta t)(I Q) + (M^N)^-1 F^N(I Q_0) (the sampling I is linear and element-local;
 * u of those calls is states[0]).
 *   states: host array of nstates (2..4) device double pointers, plan layout.
 *   dudt: device double, plan layout (5 n_nodes), not aliasing a state.
 * Errors: DG_EINVAL for null arguments, nstates outside 2..4 or dt <= 0.
 * Asynchronous on stream. */
dg_status dg_bdf_rate(dg_plan plan, const double *const *states, int32_t nstates, double dt, double *dudt,
                      hipStream_t stream);

/* Vector-Jacobian product of the residual: out = (d r / d u)^T v, r the form and
 * operator of dg_residual (FP64 only).  Written by hand: transposed derivative
 * matrices, transposed lifting, transposed mortar interpolation and projection, and
 * the transposed Jacobians of the physical and Riemann fluxes applied per node by
 * their reverse-mode derivatives (never formed as matrices).
 * Deterministic: the face pass stores per-element shares that the element pass
 * gathers.  u, v, out: device double, plan layout; out must not overlap u or v. */
dg_status dg_residual_vjp(dg_plan plan, const double *u, const double *v, double *out, int32_t form,
                          int32_t isolated, hipStream_t stream);

/* Adjoint solve (the adjoint problem behind the adjoint-weighted estimate: psi of
 * dg_tau_estimate): (d r / d u)^T psi = g, r the residual of the given form and
 * operator of dg_residual at the state u (box Euler plans), g e.g. dJ/du of
 * dg_functional.  Restarted GMRES (Givens rotations) whose matrix-vector product is
 * dg_residual_vjp; each Arnoldi step orthogonalises by classical Gram-Schmidt (one
 * pass for all inner products, one for the update), repeated once when the first round
 * removes more than 99 % of the vector's squared norm.  Inner products are
 * deterministic device reductions (fixed partition, fixed summation order).  The problem must be non-singular: on fully periodic meshes the discrete
 * conservation makes (d r / d u)^T singular, so use wall or far-field boundaries.
 *   psi: device double, plan layout; initial guess in, solution out.
 *   work: device double of dg_adjoint_workspace(plan, restart) values (caller-owned;
 *         nothing is allocated here).
 *   iters, relres (host, nullable): products done and the final ||g - A^T psi|| / ||g||.
 *   precond (in params, nullable): an element-block preconditioner built by
 *         dg_adjoint_precond_build (or its compact form) for the same plan, state, form
 *         and isolated flag, applied on the right (the Krylov space is that of A^T M^-1;
 *         the stopping test stays on the true residual) as params.precond_sweep says.
 *         The Gauss-Seidel sweep uses the workspace's spare vectors as its scratch.
 * Stops at relres <= rtol or after max_iter products.  SYNCHRONOUS: the host drives the
 * iteration and waits on stream once or twice per Arnoldi step.
 * Errors: DG_EINVAL (null arguments, restart outside 1..DG_ADJOINT_MAX_RESTART,
 * negative max_iter or rtol, unknown form, psi overlapping u or g, a preconditioner of
 * another plan, an unknown precond_sweep), DG_EUNSUPPORTED (Navier-Stokes or curved
 * plans), DG_EHIP. */
#define DG_ADJOINT_MAX_RESTART 200
/* How the solve applies its element-block preconditioner: DG_PRECOND_JACOBI, z = D^-1 x
 * (D the diagonal blocks); DG_PRECOND_GAUSS_SEIDEL, z = (D + L)^-1 x with L the
 * couplings of each element to the elements of the colours before its own (the colours
 * of the preconditioner's colouring, in order): one more dg_residual_vjp per colour
 * after the first, on the adjoint workloads here well under half the products. */
enum { DG_PRECOND_JACOBI = 0, DG_PRECOND_GAUSS_SEIDEL = 1 };
typedef struct {
    int32_t restart;     /* Krylov vectors per cycle */
    int32_t max_iter;    /* largest number of matrix-vector products */
    double rtol;         /* relative residual target */
    int32_t form;        /* DG_FORM_NEW or DG_FORM_TRAD */
    int32_t isolated;
    const void *precond; /* dg_adjoint_precond_build's memory (either form), or NULL */
    int32_t precond_sweep; /* DG_PRECOND_JACOBI or DG_PRECOND_GAUSS_SEIDEL */
} dg_adjoint_params;

dg_status dg_adjoint_workspace(dg_plan plan, int32_t restart, int64_t *doubles);
dg_status dg_adjoint_solve(dg_plan plan, const double *u, const double *g, double *psi,
                           const dg_adjoint_params *params, double *work, int32_t *iters,
                           double *relres, hipStream_t stream);

/* Element-block Jacobi preconditioner of the adjoint operator A = (d r / d u)^T at u
 * (Section 2.2's adjoint problem; restarted GMRES alone stalls on transport-dominated
 * states): M = the block diagonal of A, one block of nd x nd per element (nd = 5 x the
 * element's nodes), its inverse stored in FP32.  Each block is assembled from probing
 * products: with v = 1 at local unknown j of every element of one colour (a colouring of
 * the elements in which face neighbours differ: two colours when every periodic
 * direction has an even element count), (A v) on an element of that colour is column j
 * of its block.  colours x nd products of dg_residual_vjp, then an LU factorisation with
 * partial pivoting and the inverse of every block (rocSOLVER's batched getrf / getri).
 * Box Euler plans of one order triple with nd <= DG_PRECOND_MAX_ND.
 *   bytes (precond_bytes): the size of the caller-owned preconditioner memory.
 *   pc: device memory of that size, 256-byte aligned; filled here (its header, the
 *       colouring, pivots and the inverted blocks).
 *   work: device double[2 x 5 n_nodes] scratch.
 * SYNCHRONOUS; allocates only the rocBLAS handle and the factorisation's workspace
 * (set-up, not a hot call).  Errors: DG_EINVAL (null or misaligned arguments, a singular
 * block), DG_EUNSUPPORTED (curved or Navier-Stokes plans, mixed orders, nd too large),
 * DG_EHIP. */
#define DG_PRECOND_MAX_ND 4096
dg_status dg_adjoint_precond_bytes(dg_plan plan, int64_t *bytes);
dg_status dg_adjoint_precond_build(dg_plan plan, const double *u, int32_t form, int32_t isolated, void *pc,
                                   double *work, hipStream_t stream);
/* Compact form of a built preconditioner: every inverse block stored as FP16 values of
 * B_ij / s_j with the column scale s_j = max_i |B_ij| in FP32 (half the bytes each
 * application reads; the preconditioner's entries are then known to about 2^-11 of their
 * column's largest, which right preconditioning tolerates: the iteration and its
 * stopping test stay FP64).
 *   compact_bytes: the size of the compact form's caller-owned memory.
 *   pc: a preconditioner built by dg_adjoint_precond_build for this plan (left as it is;
 *       the caller may free it afterwards).  pc16: device memory of compact_bytes,
 *       256-byte aligned, distinct from pc.
 * The compact form is accepted wherever a preconditioner is (dg_adjoint_precond_apply,
 * dg_adjoint_params.precond).  SYNCHRONOUS; allocates nothing.  Errors: DG_EINVAL (null
 * or misaligned arguments, pc of another plan or already compact), DG_EUNSUPPORTED (as
 * dg_adjoint_precond_bytes), DG_EHIP. */
dg_status dg_adjoint_precond_compact_bytes(dg_plan plan, int64_t *bytes);
dg_status dg_adjoint_precond_compact(dg_plan plan, const void *pc, void *pc16, hipStream_t stream);
/* z = M^-1 x with a built preconditioner, either form (x, z: device double, plan layout,
 * distinct). */
dg_status dg_adjoint_precond_apply(dg_plan plan, const void *pc, const double *x, double *z, hipStream_t stream);
/* z = (D + L)^-1 x, the colour-ordered block Gauss-Seidel sweep of the solve's
 * DG_PRECOND_GAUSS_SEIDEL (u, form, isolated: those the preconditioner was built for;
 * work: device double[5 n_nodes] scratch; x, z, work distinct). */
dg_status dg_adjoint_precond_apply_gs(dg_plan plan, const void *pc, const double *u, int32_t form, int32_t isolated,
                                      const double *x, double *z, double *work, hipStream_t stream);
/* The preconditioner's colouring (host output colour[natural element]): face neighbours
 * differ in colour; the Gauss-Seidel sweep visits the colours in increasing order. */
dg_status dg_adjoint_precond_colours(dg_plan plan, const void *pc, int32_t *colour);

/* Pressure force along x on the slip walls (faces normal to x):
 *   J = sum over those faces of sum_{a,b} w_a w_b |Ja^1| p(Q_ab) n_x,
 * the quadrature of the face integral of p n_x with the face's own nodes.
 *   J: device double[1]; dJdu: device double, plan layout (nullable), receives
 *   dJ/du (zero away from the wall nodes).  Deterministic reduction. */
dg_status dg_functional(dg_plan plan, const double *u, double *J, double *dJdu, hipStream_t stream);

/* nsteps steps of Williamson's low-storage RK3 (set-up of Section 3):
 * for k = 0,1,2:  g = A_k g - dt * r(u);  u = u + B_k g,
 * A = (0, -5/9, -153/128), B = (1/3, 15/16, 8/15), r = dg_residual new form.
 *   u, g: device arrays (dtype) of 5*n_nodes values, updated in place; g is
 *   scratch (its input value is ignored).  One step is captured once into a
 *   HIP graph per (u, g, dt, dtype) and replayed. */
dg_status dg_rk3_step(dg_plan plan, void *u, void *g, double dt, int32_t nsteps, int32_t dtype,
                      hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Batches: many independent problems (plans) advanced by the same launches.
 * Each residual evaluation / RK3 stage of a batch is one persistent face launch
 * and one persistent element launch over the cost-sorted work lists of every
 * problem.  The schedule (tile capacity in nodes, element-kernel shape, grid sizes)
 * is chosen at creation by timing candidates on a uniform scratch state (the
 * library's own autotuner), and cached for the process by device architecture and
 * compute-unit count, precision and batch composition (per problem the element and
 * face counts and the element count of every order triple): a later batch of the
 * same composition takes the cached schedule without timing.  The plans must
 * outlive the batch and must not be used on another stream while the batch runs
 * (their face-flux scratch is shared); for the same reason a plan may appear only
 * once in a batch (problems on the same mesh each need a plan of their own).
 * ------------------------------------------------------------------------- */
typedef struct dg_batch_s *dg_batch;

/* plans: host array of n plans with orders <= 7; dtype DG_F64 or DG_F32 fixes the
 * state type of every later call.  Allocates and frees scratch for the schedule
 * search, and allocates the problem-descriptor slots later calls use.  Errors:
 * DG_EINVAL (null or repeated plan handle, checked before any plan is read),
 * DG_EUNSUPPORTED (order > 7), DG_ENOMEM, DG_EHIP. */
dg_status dg_batch_create(const dg_plan *plans, int32_t n, int32_t dtype, dg_batch *out);
dg_status dg_batch_destroy(dg_batch batch);
/* The schedule the autotuner chose (host outputs, any may be NULL): tile capacity in
 * nodes, element and face grid sizes, element-kernel shape (0: 256 lanes x 1 node,
 * 1: 256 x 2, 2: 512 x 1), and from_cache = 1 when it came from the cache. */
dg_status dg_batch_schedule(dg_batch batch, int32_t *tile_cap, int32_t *elem_grid, int32_t *face_grid,
                            int32_t *shape, int32_t *from_cache);
/* Replace the autotuner's schedule (for reproducible timings and tests): tile_cap 256
 * with shape 0, or 512 with shape 1 or 2, at least the largest element's node count;
 * positive grid sizes.  Every schedule gives the same results bit for bit.  SYNCHRONOUS:
 * waits for the device, drops the batch's captured RK3 graphs (they hold the old tiles
 * and grids) and rebuilds its tile list (a device allocation: set-up, not a hot call).
 * Errors: DG_EINVAL (null batch, a shape / capacity pair not listed, a capacity below an
 * element's node count, a non-positive grid), DG_EHIP. */
dg_status dg_batch_set_schedule(dg_batch batch, int32_t tile_cap, int32_t elem_grid, int32_t face_grid,
                                int32_t shape);
/* New-form residual of every problem (Section 2.1): u[i], r[i] device arrays of
 * problem i in its plan layout (host arrays of n device pointers).  The pointer
 * arrays are staged through a ring of four pinned descriptor slots; the call
 * blocks only when the call four before it has not yet finished on the device. */
dg_status dg_batch_residual(dg_batch batch, const void *const *u, void *const *r, hipStream_t stream);
/* Every problem's state in FP64 for the truncation-error estimate (Section 2.3; the
 * estimate is a difference of two nearly equal residuals and is formed in double
 * precision whatever precision the time stepping uses): u[i] in the batch's dtype,
 * u64[i] device double[5 n_nodes(i)] (plan layout, caller-owned, not overlapping u[i]).
 * An FP32 batch promotes (exactly) with one launch per problem; an FP64 batch copies. */
dg_status dg_batch_to_f64(dg_batch batch, const void *const *u, double *const *u64, hipStream_t stream);
/* FP64 isolated truncation-error map of every problem (Section 2.3 and Section 2.4.2;
 * as dg_tau_sweep with dudt = NULL): the FP64 non-isolated fine residual of every
 * problem in one batched face and element pass, into each plan's scratch, then the
 * sweeps of all problems in one launch per fine node count (the plans' work lists
 * merged at batch creation).  u64[i] as produced by dg_batch_to_f64; te_new[i],
 * te_trad[i] device double[combo_offset[E_i]] of problem i's sweep layout
 * (dg_sweep_layout), 16-byte aligned.  The pointers are staged through the ring of
 * descriptor slots of dg_batch_residual.  Errors as dg_tau_sweep. */
dg_status dg_batch_tau_sweep(dg_batch batch, const double *const *u64, int32_t restriction,
                             double *const *te_new, double *const *te_trad, hipStream_t stream);
/* nsteps Williamson RK3 steps of every problem (as dg_rk3_step), in place on u[i],
 * g[i] scratch; one step is captured once per (u, g, dt) pointer set into a HIP graph
 * of three stages, each one persistent face launch and one persistent element launch. */
dg_status dg_batch_rk3_step(dg_batch batch, void *const *u, void *const *g, double dt, int32_t nsteps,
                            hipStream_t stream);

/* Synchronise the device and report a deferred HIP error, if any. */
dg_status dg_check(void);

/* Admissibility of a state: counts the nodes where rho <= 0, the pressure
 * (gamma - 1)(rho E - |rho u|^2 / (2 rho)) <= 0, or any variable is not finite (the
 * Euler and Navier-Stokes fluxes are defined only for positive density and pressure).
 *   u: device array of 5 n_nodes values of type dtype (DG_F64 or DG_F32), plan layout.
 *   bad (host, nullable): receives the count.
 * Returns DG_ENONPHYSICAL when the count is positive.  SYNCHRONOUS on stream (the count
 * is read back); the reduction is deterministic and allocates nothing (it uses the
 * plan's scratch, so one plan runs one check at a time). */
dg_status dg_check_state(dg_plan plan, const void *u, int32_t dtype, int64_t *bad, hipStream_t stream);

/* Message of the last non-OK status on this thread ("" if none). */
const char *dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
