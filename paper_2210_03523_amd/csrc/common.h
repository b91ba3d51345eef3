// Internal definitions shared by the host plan code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgt {

constexpr int NV = 5;        // conserved variables
constexpr int NMAX = 9;      // maximum polynomial order
constexpr int NNMAX = NMAX + 1;
constexpr int WG = 256;      // threads per workgroup of the element kernels

// 1D tables, packed: orders 1..NMAX, n = N+1 values per order.
// xoff(N) = sum_{k=1}^{N-1} (k+1)
__host__ __device__ constexpr inline int xoff(int N) { return (N - 1) * (N + 4) / 2; }
// doff(N) = sum_{k=1}^{N-1} (k+1)^2
__host__ __device__ constexpr inline int doff(int N) { return N * (N + 1) * (2 * N + 1) / 6 - 1; }
constexpr int XTOT = xoff(NMAX + 1);            // 54
constexpr int DTOT = doff(NMAX + 1);            // 384
// Matrices indexed by an order pair (A, B) with (A+1) rows and (B+1) columns.
__host__ __device__ constexpr inline int moff(int A, int B) { return xoff(A) * XTOT + (A + 1) * xoff(B); }
constexpr int MTOT = XTOT * XTOT;               // 2916

// Table block layout (one block per precision): nodes, weights, D, I, P.
constexpr int T_X = 0;
constexpr int T_W = T_X + XTOT;
constexpr int T_D = T_W + XTOT;
constexpr int T_I = T_D + DTOT;                 // I^{A<-B}: samples order-B basis at order-A nodes
constexpr int T_P = T_I + MTOT;                 // P^{A<-B}: L2 projection from order B onto order A (A <= B)
constexpr int T_TOT = T_P + MTOT;

// Workgroup id -> work item such that each XCD (dispatch is round-robin over the 8
// XCDs) takes a contiguous range of the G items and keeps neighbours in its own L2.
// A bijection of [0, G).
__device__ __forceinline__ int xcd_remap(int bid, int G) {
    int q = G >> 3, r = G & 7;
    int x = bid & 7, l = bid >> 3;
    return (x < r) ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// A value in the global address space.  Pointers read from a descriptor in memory are
// cast to `gmem<T> *` before use, so that their accesses compile to global (not flat)
// memory instructions.
template <typename T>
using gmem = __attribute__((address_space(1))) T;

// Per plan element record (device).
struct ElemInfo {
    int32_t n[3];     // nodes per direction (order + 1)
    int32_t nat;      // natural element index
    int64_t noff;     // first node of the element
    int64_t foff;     // first value of the element's face-flux block
};

// Face between plan elements eL (minus side) and eR (plus side) along direction d.
// Boundary faces have eL < 0 (box face at the minus end) or eR < 0 (plus end), and bc != 0.
struct Face {
    int32_t eL, eR;
    int32_t d, bc;
};

// A tile: `count` consecutive plan elements with identical orders.
struct Tile {
    int32_t first, count;
};

// Offset of the face-flux slot (d, side) inside an element's face-flux block.
__host__ __device__ inline int64_t fslot(const int32_t *n, int d, int side) {
    int64_t off = 0;
    for (int dd = 0; dd < d; ++dd) {
        int a = n[dd == 0 ? 1 : 0], b = n[dd == 2 ? 1 : 2];
        off += 2 * NV * a * b;
    }
    int a = n[d == 0 ? 1 : 0], b = n[d == 2 ? 1 : 2];
    return off + (side > 0 ? NV * a * b : 0);
}
__host__ __device__ inline int64_t fblock(const int32_t *n) {
    return 2 * NV * ((int64_t)n[1] * n[2] + (int64_t)n[0] * n[2] + (int64_t)n[0] * n[1]);
}

// Uniform affine geometry of the box elements.
struct Geom {
    double J;        // h1 h2 h3 / 8
    double Ja[3];    // |Ja^d| = J * 2 / h_d
    double h[3];
    double lo[3];
};

struct PhysParams {
    double gamma;
    int32_t flux;
    int32_t pad;
    double qfar[NV];
    double mu, kappa;   // Navier-Stokes (mu = 0: Euler)
};

// Host-side launch wrappers (defined in the .hip files).
template <typename T>
hipError_t launch_face_flux(const Face *faces, int nfaces, const ElemInfo *elems, const T *u, T *fflux,
                            const T *tab, Geom g, PhysParams ph, int max_order, hipStream_t s);

enum EpiMode { EPI_RESIDUAL = 0, EPI_RK = 1, EPI_TAU = 2 };

struct EpiArgs {
    int mode;
    int form;           // residual: 0 new, 1 traditional
    int isolated;
    double rkA, rkB, dt;
    void *out;          // residual output / tau_new
    void *out2;         // tau_trad
    void *g;            // RK register
    const void *rdc;    // restricted fine time derivative (tau)
    double *norms;      // [E][2] (tau)
    const void *psic;   // restricted adjoint weight (tau, optional)
    double *eta;        // [E] sum of psic * tau_trad (tau, optional)
    double *varnorms;   // [E][2][5] per-variable maxima of |tau_new|, |tau_trad| (tau, optional)
    const void *grad;   // Navier-Stokes: BR1 gradients [elem][3][5][node] (null for Euler)
    double mu, kappa;   // viscosity and heat conductivity
    const void *met;    // curved elements: metric terms [elem][10][node] (Ja^1, Ja^2, Ja^3, J)
};

template <typename T>
hipError_t launch_element(const Tile *tiles, int tile0, int ntiles, int npt, const ElemInfo *elems, const T *u,
                          const T *fflux, const T *tab, Geom g, PhysParams ph, EpiArgs epi, hipStream_t s);

// capA, capB: LDS capacities of the restriction, NV times the doubles of its two areas
// maximised over the target plan's elements (restrict_cap_a, restrict_cap_b of the
// target orders c and source orders f).  restriction:
// 0 samples at the coarse nodes, 1 takes the exact L2 projection (also for the sweeps).
// psi_new: psi is the new-form adjoint and is divided by the fine mass matrix J w w w
// (met: curved metric terms [elem][10][node], or null with invJ = 1/J of box elements).
// staging of one variable: the x-pass [c1][f2 f3], overwritten by the y-pass [c1 c2][f3]
inline int restrict_cap_a(const int32_t *c, const int32_t *f) {
    return NV * (c[0] + 1) * (f[1] > c[1] ? f[1] + 1 : c[1] + 1) * (f[2] + 1);
}
// the y and z operators, (c2 + 1)(f2 + 1) + (c3 + 1)(f3 + 1) doubles
inline int restrict_cap_b(const int32_t *c, const int32_t *f) {
    return NV * ((c[1] + 1) * (f[1] + 1) + (c[2] + 1) * (f[2] + 1));
}
// felems: per coarse element the record of its fine element.
hipError_t launch_restrict(int ncoarse, const ElemInfo *celems, const ElemInfo *felems,
                           const double *u, const double *dudt, const double *psi, double *uc, double *rdc,
                           double *psic, const double *tab, int capA, int capB, int restriction, int psi_new,
                           const double *met, double invJ, hipStream_t s);

// Solution transfer onto another order map: target plan elements tel, source plan
// elements sel, src_inv[natural] = source plan position; capA = max 5 t1 s2 s3,
// capB = max 5 max(t1 t2 s3, s1 s2 s3) over the elements.
hipError_t launch_project(const int32_t *src_inv, int ntarget, const ElemInfo *tel, const ElemInfo *sel,
                          const double *u, double *ut, const double *tab, int capA, int capB, hipStream_t s);

hipError_t launch_vjp(const Face *faces, int nfaces, const Tile *tiles, int tile0, int ntiles, int npt,
                      const ElemInfo *el, const double *u, const double *v, double *fa, double *out,
                      const double *tab, Geom g, PhysParams ph, int form, int isolated, bool do_faces, int max_order,
                      hipStream_t s);
hipError_t launch_functional(const Face *faces, const int32_t *wall, int nwall, const ElemInfo *el,
                             const double *u, const double *tab, Geom g, double gamma, double *part, double *J,
                             double *dJdu, int64_t n_vals, hipStream_t s);

hipError_t launch_coords(const ElemInfo *elems, int E, int nx, int ny, const double *tab, Geom g, double *xyz,
                         hipStream_t s);

// One workgroup of the isolated sweep: fine plan element p and coarse orders (c1, c2).
struct SweepTask {
    int32_t p, c1, c2, pad;
};

// Anisotropic sweep: workgroups (first job, job count, problem, 0) over jobs (element,
// pair of x-orders, first lane, offset of the x-rows in the staging area), packed by the host
// within AN_LANES lanes and an_stage_doubles(F3) doubles of x-rows, AN_JOBS_MAX jobs.
constexpr int AN_LANES = 256;
constexpr int AN_JOBS_MAX = 8;
__host__ __device__ constexpr inline int an_stage_doubles(int F3) {
    return 2 * NV * ((F3 > 2 ? F3 - 2 : 1) + 1) * AN_LANES;
}
// Inputs and outputs of one problem of the isolated sweep.  The sweep kernels take one by
// value (single) or, for a batch of problems, an array indexed by the problem of each work
// record (probs, or null).
struct SweepProb {
    const ElemInfo *el;
    const int64_t *combo_off;
    const double *u, *dudt;
    double *te_new, *te_trad;
    Geom g;
    double gamma;
};
hipError_t launch_sweep_an(int F3, const int4 *wgs, int nwg, const int4 *jobs, const SweepProb &single,
                           const SweepProb *probs, const double *tab, int restriction, hipStream_t s);
hipError_t launch_sweep_tasks(const void *tasks, int ntasks, const ElemInfo *elems, const int64_t *combo_off,
                              const double *u, const double *dudt, const double *tab, Geom g, double gamma,
                              int x1cap, int x2cap, int restriction, double *te_new, double *te_trad,
                              hipStream_t s);

// Isotropic fast path of the sweep (fine nodes F per direction, 2 <= F <= 8).
// Degree selection from truncation-error maps (maps: host array of nst device pointers)
// and nmax Jacobi steps of the jump condition; orders natural [E][3]; tmp: [E][3] scratch.
// X = 0: maps in the sweep layout; X > 0: extended maps [E][X^3] (plan order, N1 fastest).
hipError_t launch_select(const ElemInfo *el, int E, const int64_t *combo_off, const double *const *maps, int nst,
                         double tau_max, int nmin, int nmax, int approach, const int32_t *prev, int max_decrease,
                         int X, int jump, int nx, int ny, int nz, int periodic, int32_t *orders, int32_t *tmp,
                         hipStream_t s);
hipError_t launch_map_fmax(double *acc, const double *m, int64_t n, hipStream_t s);
// tau-extrapolation of a sweep-layout map into the extended layout [E][X^3]
hipError_t launch_extrapolate(const ElemInfo *el, int E, const int64_t *combo_off, const double *map, int X,
                              double *ext, hipStream_t s);
// Krylov vector operations: out[0] = sum a b (part: dot_partials() doubles of scratch);
// y <- alpha x + beta y (x may equal y)
hipError_t launch_dot(const double *a, const double *b, int64_t n, double *part, double *out, hipStream_t s);
// element-block Jacobi preconditioner of the adjoint solve (k_precond.hip)
hipError_t launch_probe_set(double *v, const int32_t *elems, int nel, const ElemInfo *el, int j, double val,
                            hipStream_t s);
hipError_t launch_probe_gather(const double *out, float *blocks, const int32_t *elems, int nel, const ElemInfo *el,
                               int j, int nd, hipStream_t s);
hipError_t launch_bj_apply(const float *blocks, const double *x, double *z, const ElemInfo *el, int E, int nd,
                           hipStream_t s, const int32_t *elems = nullptr, const double *t = nullptr);
// Compact FP16 storage of the inverse blocks with per-column FP32 scales, and its apply.
hipError_t launch_bj_compact(const float *blocks, void *hblocks, float *scales, int E, int nd, hipStream_t s);
hipError_t launch_bj_apply16(const void *hblocks, const float *scales, const double *x, double *z,
                             const ElemInfo *el, int E, int nd, hipStream_t s, const int32_t *elems = nullptr,
                             const double *t = nullptr);
hipError_t launch_axpby(double alpha, const double *x, double beta, double *y, int64_t n, hipStream_t s);
int dot_partials();
// Gram-Schmidt passes over Krylov vectors x_k = X + k ld, k < c: out[k] = x_k . w (and
// out[c] = w . w when self); w <- w - sum h_k x_k (h on the device, c <= DG_KRYLOV_MAX)
// and *nrm2 = the new w . w when nrm2 is given.  part: mdot_partials() doubles.
constexpr int DG_KRYLOV_MAX = 201;  // restart + 1 vectors for the largest restart, 200
hipError_t launch_mdot(const double *X, int64_t ld, int c, const double *w, bool self, int64_t n, double *part,
                       double *out, hipStream_t s);
hipError_t launch_maxpy(const double *X, int64_t ld, int c, const double *h, double *w, int64_t n, double *part,
                        double *nrm2, hipStream_t s);
int mdot_partials();
// Count of non-physical nodes (rho <= 0, p <= 0 or not finite) into out[0]; part holds
// dot_partials() doubles of scratch.
template <typename T>
hipError_t launch_count_bad(const ElemInfo *el, int E, const T *u, double gamma, double *part, double *out,
                            hipStream_t s);
// dudt = -(1/dt) sum_j b_j states[j], backward difference of order nst-1 (nst in 2..4)
hipError_t launch_bdf_rate(const double *const *states, int nst, double dt, int64_t n, double *dudt, hipStream_t s);
hipError_t launch_promote(const float *in, double *out, int64_t n, hipStream_t s);
// Isotropic sweep of elements (problem, element) with F fine nodes per direction.
hipError_t launch_sweep_iso(int F, const int2 *elems, int nelem, const SweepProb &single, const SweepProb *probs,
                            const double *tab, int restriction, hipStream_t s);

// ---------------------------------------------------------------------------- batches
// One independent problem of a batch, as seen by the persistent kernels.
template <typename T>
struct ProbDesc {
    const ElemInfo *el;
    const Face *faces;
    T *u;        // state (read; updated in place by the RK epilogue)
    T *out;      // residual output
    T *g;        // RK register
    T *ff;       // face-flux scratch of the problem's plan
    Geom geom;
    PhysParams phys;
};

// A face of a batch: the face of problem `prob` with both sides' element descriptors
// (a boundary face's one element in both).
struct BatchFace {
    Face f;
    ElemInfo L, R;
    int32_t prob, pad[3];
};

// A tile of a batch: `count` consecutive plan elements of problem `prob`, e0 the
// descriptor of the first.
struct BatchTile {
    int32_t prob, first, count, pad;
    ElemInfo e0;
};

template <typename T>
hipError_t launch_face_batch(const BatchFace *faces, int nfaces, const ProbDesc<T> *probs, const T *tab, int grid,
                             hipStream_t s);
// shape: 0 = 256 lanes x 1 node, 1 = 256 x 2, 2 = 512 x 1 (tile capacity 256 for shape 0, 512 otherwise)
template <typename T>
hipError_t launch_elem_batch(const BatchTile *tiles, int ntiles, const ProbDesc<T> *probs, const T *tab, int grid,
                             int shape, EpiArgs epi, hipStream_t s);
template <typename T>
hipError_t launch_fill_state(const ElemInfo *el, int E, T *u, hipStream_t s);

// Navier-Stokes (BR1) passes: BR1 solution trace on the faces, gradients, viscous face fluxes.
template <typename T>
hipError_t launch_ns_gradient(const Face *faces, int nfaces, const Tile *tiles, int tile0, int ntiles, int npt,
                              bool do_faces, const ElemInfo *el, const T *u, T *fq, T *grad, const T *tab, Geom g,
                              PhysParams ph, int max_order, int isolated, hipStream_t s);
template <typename T>
hipError_t launch_ns_faces(const Face *faces, int nfaces, const ElemInfo *el, const T *u, const T *grad, T *ff,
                           const T *tab, Geom g, PhysParams ph, hipStream_t s);

// Fields restricted per combination by the curved sweep: Q, dQ/dt, node coordinates.
constexpr int NFLD_SWEEP = 2 * NV + 3;

// Curved elements (k_curved.hip): face fluxes with per-face scaled normals (fmet, 3 values
// per mortar / boundary-face node starting at node offset fmo[face]), the BR1 face data and
// gradient pass, and the isolated sweep with per-combination coarse geometry.
template <typename T>
hipError_t launch_face_curved(const Face *faces, const int64_t *fmo, const T *fmet, int nfaces, const ElemInfo *el,
                              const T *u, const T *grad, T *ff, const T *tab, PhysParams ph, int max_order,
                              hipStream_t s);
template <typename T>
hipError_t launch_grad_curved(const Face *faces, const int64_t *fmo, const T *fmet, int nfaces, const Tile *tiles,
                              int tile0, int ntiles, int npt, bool do_faces, const ElemInfo *el, const T *u,
                              const T *met, T *fq, T *grad, const T *tab, PhysParams ph, int isolated,
                              hipStream_t s);
hipError_t launch_sweep_curved(const int4 *tasks, int ntasks, const ElemInfo *el, const int64_t *combo_off,
                               const double *u, const double *dudt, const double *xyz, const double *tab,
                               PhysParams ph, int capA, int capB, int capS, int max_nc, int viscous, int restriction,
                               double *te_new, double *te_trad, hipStream_t s);

// Host tables (tables.cpp): fills T_TOT values.
void build_tables(double *tab64, float *tab32);

}  // namespace dgt
