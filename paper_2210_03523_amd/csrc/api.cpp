// C ABI of the library (declared in include/dgtau.h): plan construction (order
// buckets, tiles, face lists, tables, scratch) and the host side of every entry
// point.  All numerical work runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include <rocsolver/rocsolver.h>

#include "../../include/dgtau.h"
#include "common.h"

using namespace dgt;

namespace {

thread_local std::string g_err;

dg_status fail(dg_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(DG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));         \
    } while (0)

// Nodal tables, one copy per device, kept until the process ends.
struct DevTables {
    double *t64 = nullptr;
    float *t32 = nullptr;
};
std::mutex g_tab_mu;
std::map<int, DevTables> g_tabs;

dg_status device_tables(DevTables *out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tab_mu);
    auto it = g_tabs.find(dev);
    if (it != g_tabs.end()) {
        *out = it->second;
        return DG_OK;
    }
    std::vector<double> h64(T_TOT);
    std::vector<float> h32(T_TOT);
    build_tables(h64.data(), h32.data());
    DevTables t;
    HIP_TRY(hipMalloc(&t.t64, sizeof(double) * T_TOT));
    HIP_TRY(hipMalloc(&t.t32, sizeof(float) * T_TOT));
    HIP_TRY(hipMemcpy(t.t64, h64.data(), sizeof(double) * T_TOT, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(t.t32, h32.data(), sizeof(float) * T_TOT, hipMemcpyHostToDevice));
    g_tabs[dev] = t;
    *out = t;
    return DG_OK;
}

struct TileClass {
    int npt, first, count;
};

// RK3 graphs kept per plan and per batch; the least recently used one is destroyed
// (after a device synchronisation, so no launch of it is in flight) to make room.
constexpr size_t kGraphCache = 8;

template <typename Map>
typename Map::iterator lru_victim(Map &m) {
    auto v = m.begin();
    for (auto it = m.begin(); it != m.end(); ++it)
        if (it->second.second < v->second.second) v = it;
    return v;
}

struct GraphKey {
    void *u, *g;
    double dt;
    int dtype;
    bool operator<(const GraphKey &o) const {
        return std::tie(u, g, dt, dtype) < std::tie(o.u, o.g, o.dt, o.dtype);
    }
};

}  // namespace

struct dg_plan_s {
    dg_mesh_desc mesh;
    int device = 0;
    int E = 0;
    int64_t n_nodes = 0, ff_len = 0;
    std::vector<int32_t> ord;   // plan order [E][3]
    std::vector<int64_t> perm;  // plan -> natural
    std::vector<int64_t> inv;   // natural -> plan
    std::vector<int64_t> noff;  // [E+1]
    std::vector<TileClass> classes;
    Geom geom{};
    PhysParams phys{};
    DevTables tabs;
    int nfaces = 0;
    ElemInfo *d_el = nullptr;
    Face *d_faces = nullptr;
    Tile *d_tiles = nullptr;
    void *d_ff = nullptr;        // face fluxes, sized for doubles
    double *d_dudt = nullptr;    // fine time-derivative scratch (tau without dudt)
    // coarse plans
    dg_plan_s *parent = nullptr;
    ElemInfo *d_fine_el = nullptr;  // coarse plans: the fine element's record per element (foff unused)
    double *d_uc = nullptr, *d_rdc = nullptr, *d_psic = nullptr;
    bool ns = false;              // Navier-Stokes plan
    void *d_grad = nullptr;       // BR1 gradients [elem][3][5][node], sized for doubles
    // curved elements: per-node metric terms [elem][10][node] (double and float copies),
    // scaled face normals (3 values per mortar / boundary-face node from node offset
    // fmo[face]); node coordinates [elem][3][node] of curved and Navier-Stokes plans
    bool curved = false;
    std::vector<double> xyz_h;
    double *d_xyz = nullptr;
    double *d_met64 = nullptr, *d_fmet64 = nullptr;
    float *d_met32 = nullptr, *d_fmet32 = nullptr;
    int64_t *d_fmo = nullptr;
    // sweep of curved and Navier-Stokes plans: one task per (element, c1, c2, c3)
    int4 *d_ctasks = nullptr;
    int nctasks = 0, capA = 0, capB = 0, capS = 0, max_nc = 0;
    // restriction from the fine plan (coarse plans): LDS staging capacities
    int rcapA = 0, rcapB = 0;
    // x-force functional: boundary faces on slip walls normal to x, and their partial sums
    int32_t *d_wallx = nullptr;
    int nwallx = 0;
    double *d_part = nullptr;
    // sweep
    std::vector<int64_t> combo_off;
    int64_t *d_combo_off = nullptr;
    SweepTask *d_tasks = nullptr;
    int ntasks = 0, x1cap = 0, x2cap = 0, max_order = 0;
    int2 *d_iso = nullptr;              // isotropic elements (0, element) grouped by fine node count F
    int32_t *d_sel = nullptr;           // degree selection: [E][3] intermediate of the jump steps
    int32_t *d_inv = nullptr;           // natural element -> plan position
    double *d_red = nullptr;            // reduction partials of dg_check_state
    int iso_first[NNMAX + 1] = {0}, iso_count[NNMAX + 1] = {0};
    int4 *d_an = nullptr;               // anisotropic sweep jobs (element, pair, lane0, x1 offset)
    int4 *d_anw = nullptr;              // their workgroups (first job, job count, 0, 0) grouped by F3
    std::vector<int2> h_iso;            // host copies of the three sweep lists (for batches)
    std::vector<int4> h_an, h_anw;
    int an_first[NNMAX + 1] = {0}, an_count[NNMAX + 1] = {0};
    void *d_arena = nullptr;  // the one device allocation every device buffer lives in
    // RK3 graphs: at most kGraphCache, each with the call count of its last use
    hipStream_t cap_stream = nullptr;
    std::map<GraphKey, std::pair<hipGraphExec_t, uint64_t>> graphs;
    uint64_t graph_clock = 0;
};

namespace {

template <typename T>
dg_status upload(T **dst, const std::vector<T> &src) {
    if (src.empty()) return DG_OK;
    HIP_TRY(hipMalloc((void **)dst, sizeof(T) * src.size()));
    HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return DG_OK;
}

// One device allocation per plan: the uploaded tables (one host image, one copy) followed
// by the scratch buffers, each 256-byte aligned.  Empty uploads leave their pointer null.
struct Arena {
    struct Slot {
        void **dst;
        size_t off;
    };
    std::vector<Slot> slots;
    std::vector<char> image;  // host image of the uploaded part
    size_t off = 0;
    static size_t align(size_t x) { return (x + 255) & ~size_t(255); }
    template <typename T>
    void upload(T **dst, const std::vector<T> &v) {
        if (v.empty()) return;
        off = align(off);
        slots.push_back({(void **)dst, off});
        const size_t bytes = sizeof(T) * v.size();
        image.resize(off + bytes);
        memcpy(image.data() + off, v.data(), bytes);
        off += bytes;
    }
    template <typename T>
    void scratch(T **dst, size_t bytes) {  // after every upload
        off = align(off);
        slots.push_back({(void **)dst, off});
        off += std::max<size_t>(bytes, 8);
    }
    dg_status commit(void **base) {
        if (hipMalloc(base, std::max<size_t>(off, 256)) != hipSuccess) return fail(DG_ENOMEM, "device allocation failed");
        if (!image.empty() && hipMemcpy(*base, image.data(), image.size(), hipMemcpyHostToDevice) != hipSuccess)
            return fail(DG_EHIP, "plan upload failed");
        for (const Slot &sl : slots) *sl.dst = (char *)*base + sl.off;
        return DG_OK;
    }
};

void destroy_plan(dg_plan p) {
    if (!p) return;
    for (auto &kv : p->graphs) (void)hipGraphExecDestroy(kv.second.first);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_arena) (void)hipFree(p->d_arena);
    delete p;
}

int npt_class(int npe) { return npe <= WG ? 1 : (npe <= 2 * WG ? 2 : 4); }

// ---------------------------------------------------------------------------- host geometry
// Node coordinates X[3][ne] of the element at box position c with nodes n[3]: box
// elements are the affine image of the reference cube; DG_MAP_SINE moves the box point
// (x, y, z) to (x + f, y + f, z) and takes the Gauss-Lobatto interpolant of order
// geo_order of that map, sampled at the element's nodes.
void element_coords(const dg_mesh_desc &m, const double *tab, const int c[3], const int32_t n[3], double *X) {
    const int nd[3] = {m.nx, m.ny, m.nz};
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = (m.hi[d] - m.lo[d]) / nd[d];
    const int ne = n[0] * n[1] * n[2];
    if (m.map_kind == DG_MAP_BOX) {
        for (int k = 0; k < n[2]; ++k)
            for (int j = 0; j < n[1]; ++j)
                for (int i = 0; i < n[0]; ++i) {
                    const int idx[3] = {i, j, k};
                    for (int d = 0; d < 3; ++d)
                        X[d * ne + i + n[0] * (j + n[1] * k)] =
                            m.lo[d] + h[d] * (c[d] + 0.5 * (tab[T_X + xoff(n[d] - 1) + idx[d]] + 1.0));
                }
        return;
    }
    const double two_pi = 6.283185307179586476925286766559;
    const int G[3] = {m.geo_order[0], m.geo_order[1], m.geo_order[2]};
    const int g[3] = {G[0] + 1, G[1] + 1, G[2] + 1}, ng = g[0] * g[1] * g[2];
    std::vector<double> P(3 * (size_t)ng);
    for (int kc = 0; kc < g[2]; ++kc)
        for (int kb = 0; kb < g[1]; ++kb)
            for (int ka = 0; ka < g[0]; ++ka) {
                const int gi[3] = {ka, kb, kc};
                double xb[3];
                for (int d = 0; d < 3; ++d) xb[d] = m.lo[d] + h[d] * (c[d] + 0.5 * (tab[T_X + xoff(G[d]) + gi[d]] + 1.0));
                const double f = m.map_amp * std::sin(two_pi * (xb[0] - m.lo[0]) / (m.hi[0] - m.lo[0])) *
                                 std::sin(two_pi * (xb[1] - m.lo[1]) / (m.hi[1] - m.lo[1]));
                const int gn = ka + g[0] * (kb + g[1] * kc);
                P[gn] = xb[0] + f;
                P[ng + gn] = xb[1] + f;
                P[2 * ng + gn] = xb[2];
            }
    const double *I1 = tab + T_I + moff(n[0] - 1, G[0]);
    const double *I2 = tab + T_I + moff(n[1] - 1, G[1]);
    const double *I3 = tab + T_I + moff(n[2] - 1, G[2]);
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
}

// Metric terms Mt[10][ne] from node coordinates: a_r = D_r X along reference direction r,
// Ja^1 = a_2 x a_3, Ja^2 = a_3 x a_1, Ja^3 = a_1 x a_2, J = a_1 . Ja^1.
void element_metrics(const double *tab, const int32_t n[3], const double *X, double *Mt) {
    const int ne = n[0] * n[1] * n[2];
    const int stride[3] = {1, n[0], n[0] * n[1]};
    for (int t = 0; t < ne; ++t) {
        const int idx[3] = {t % n[0], (t / n[0]) % n[1], t / (n[0] * n[1])};
        double a[3][3];
        for (int r = 0; r < 3; ++r) {
            const double *Drow = tab + T_D + doff(n[r] - 1) + idx[r] * n[r];
            const int tb = t - idx[r] * stride[r];
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int q = 0; q < n[r]; ++q) acc += Drow[q] * X[c * ne + tb + q * stride[r]];
                a[r][c] = acc;
            }
        }
        for (int d = 0; d < 3; ++d) {
            const double *p = a[(d + 1) % 3], *q = a[(d + 2) % 3];
            Mt[(3 * d + 0) * ne + t] = p[1] * q[2] - p[2] * q[1];
            Mt[(3 * d + 1) * ne + t] = p[2] * q[0] - p[0] * q[2];
            Mt[(3 * d + 2) * ne + t] = p[0] * q[1] - p[1] * q[0];
        }
        Mt[9 * ne + t] = a[0][0] * Mt[0 * ne + t] + a[0][1] * Mt[1 * ne + t] + a[0][2] * Mt[2 * ne + t];
    }
}

int face_node_h(const int32_t *n, int d, int side, int a, int b) {
    int idx[3];
    idx[d] = side > 0 ? n[d] - 1 : 0;
    idx[d == 0 ? 1 : 0] = a;
    idx[d == 2 ? 1 : 2] = b;
    return idx[0] + n[0] * (idx[1] + n[1] * idx[2]);
}

dg_status build_plan(const dg_mesh_desc *mesh, const int32_t *orders, dg_plan parent, dg_plan *out) {
    if (!mesh || !orders || !out) return fail(DG_EINVAL, "null argument");
    if (mesh->nx < 1 || mesh->ny < 1 || mesh->nz < 1) return fail(DG_EINVAL, "mesh needs at least one element per direction");
    const int64_t E64 = (int64_t)mesh->nx * mesh->ny * mesh->nz;
    if (E64 > (1 << 30)) return fail(DG_EINVAL, "too many elements");
    for (int d = 0; d < 3; ++d) {
        if (!(mesh->hi[d] > mesh->lo[d])) return fail(DG_EINVAL, "mesh extent must be positive");
        int a = mesh->bc[2 * d], b = mesh->bc[2 * d + 1];
        if (a < 0 || a > 2 || b < 0 || b > 2) return fail(DG_EINVAL, "unknown boundary condition");
        if ((a == DG_BC_PERIODIC) != (b == DG_BC_PERIODIC)) return fail(DG_EINVAL, "periodic faces must come in pairs");
    }
    if (mesh->flux != DG_FLUX_ROE && mesh->flux != DG_FLUX_LF) return fail(DG_EINVAL, "unknown flux");
    if (!(mesh->gamma > 1.0)) return fail(DG_EINVAL, "gamma must exceed 1");
    if (mesh->equation != DG_EULER && mesh->equation != DG_NAVIER_STOKES) return fail(DG_EINVAL, "unknown equation");
    if (mesh->equation == DG_NAVIER_STOKES && !(mesh->mu >= 0.0 && mesh->Pr > 0.0))
        return fail(DG_EINVAL, "Navier-Stokes needs mu >= 0 and Pr > 0");
    if (mesh->map_kind != DG_MAP_BOX && mesh->map_kind != DG_MAP_SINE) return fail(DG_EINVAL, "unknown map");
    if (mesh->map_kind == DG_MAP_SINE) {
        for (int d = 0; d < 3; ++d)
            if (mesh->geo_order[d] < 1 || mesh->geo_order[d] > DG_NMAX)
                return fail(DG_EINVAL, "geometry orders must be in 1..9");
        if (!(std::fabs(mesh->map_amp) < 1e3)) return fail(DG_EINVAL, "map amplitude out of range");
    }
    const int E = (int)E64;
    for (int i = 0; i < 3 * E; ++i)
        if (orders[i] < 1 || orders[i] > DG_NMAX) return fail(DG_EINVAL, "orders must be in 1..9");
    if (mesh->map_kind == DG_MAP_SINE && !parent)
        for (int i = 0; i < 3 * E; ++i)
            if (orders[i] < mesh->geo_order[i % 3])
                return fail(DG_EINVAL, "curved elements need orders >= the geometry order");

    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(DG_EHIP, "no current device");
    dg_plan p = new dg_plan_s();
    p->mesh = *mesh;
    p->E = E;
    p->device = device;
    dg_status st = DG_OK;

    // stable sort by (tile class, N1, N2, N3), ties by natural index
    std::vector<int64_t> perm(E);
    std::iota(perm.begin(), perm.end(), 0);
    auto key = [&](int64_t e) {
        const int32_t *o = orders + 3 * e;
        int npe = (o[0] + 1) * (o[1] + 1) * (o[2] + 1);
        return std::make_tuple(npt_class(npe), o[0], o[1], o[2]);
    };
    std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
    p->perm = perm;
    p->inv.assign(E, 0);
    for (int i = 0; i < E; ++i) p->inv[perm[i]] = i;
    p->ord.resize(3 * E);
    p->noff.assign(E + 1, 0);
    std::vector<ElemInfo> el(E);
    int64_t foff = 0;
    for (int i = 0; i < E; ++i) {
        const int32_t *o = orders + 3 * perm[i];
        ElemInfo &x = el[i];
        for (int d = 0; d < 3; ++d) {
            p->ord[3 * i + d] = o[d];
            x.n[d] = o[d] + 1;
            p->max_order = std::max(p->max_order, (int)o[d]);
        }
        x.nat = (int32_t)perm[i];
        x.noff = p->noff[i];
        x.foff = foff;
        p->noff[i + 1] = p->noff[i] + (int64_t)x.n[0] * x.n[1] * x.n[2];
        foff += fblock(x.n);
    }
    p->n_nodes = p->noff[E];
    p->ff_len = foff;

    // tiles: runs of equal orders, chunked to fill a workgroup
    std::vector<Tile> tiles;
    for (int i = 0; i < E;) {
        int j = i;
        while (j < E && p->ord[3 * j] == p->ord[3 * i] && p->ord[3 * j + 1] == p->ord[3 * i + 1] &&
               p->ord[3 * j + 2] == p->ord[3 * i + 2])
            ++j;
        const int npe = el[i].n[0] * el[i].n[1] * el[i].n[2];
        const int cls = npt_class(npe);
        const int cap = npe <= WG ? WG / npe : 1;
        if (p->classes.empty() || p->classes.back().npt != cls)
            p->classes.push_back({cls, (int)tiles.size(), 0});
        for (int k = i; k < j; k += cap) {
            tiles.push_back({k, std::min(cap, j - k)});
            p->classes.back().count++;
        }
        i = j;
    }

    // faces: the + face of every element in every direction, plus boundary faces at the minus ends
    std::vector<Face> faces;
    const int nd[3] = {mesh->nx, mesh->ny, mesh->nz};
    for (int e = 0; e < E; ++e) {
        int c[3] = {e % mesh->nx, (e / mesh->nx) % mesh->ny, e / (mesh->nx * mesh->ny)};
        for (int d = 0; d < 3; ++d) {
            int cn[3] = {c[0], c[1], c[2]};
            if (c[d] == 0 && mesh->bc[2 * d] != DG_BC_PERIODIC)
                faces.push_back({-1, (int32_t)p->inv[e], d, mesh->bc[2 * d]});
            if (c[d] == nd[d] - 1) {
                if (mesh->bc[2 * d + 1] != DG_BC_PERIODIC) {
                    faces.push_back({(int32_t)p->inv[e], -1, d, mesh->bc[2 * d + 1]});
                    continue;
                }
                cn[d] = 0;
            } else {
                cn[d] = c[d] + 1;
            }
            int en = cn[0] + mesh->nx * (cn[1] + mesh->ny * cn[2]);
            faces.push_back({(int32_t)p->inv[e], (int32_t)p->inv[en], d, 0});
        }
    }
    p->nfaces = (int)faces.size();
    std::vector<int32_t> wallx;
    for (int f = 0; f < p->nfaces; ++f)
        if (faces[f].bc == DG_BC_SLIP_WALL && faces[f].d == 0) wallx.push_back(f);
    p->nwallx = (int)wallx.size();

    // geometry and physics
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = (mesh->hi[d] - mesh->lo[d]) / nd[d];
    p->geom.J = h[0] * h[1] * h[2] / 8.0;
    p->geom.Ja[0] = h[1] * h[2] / 4.0;
    p->geom.Ja[1] = h[0] * h[2] / 4.0;
    p->geom.Ja[2] = h[0] * h[1] / 4.0;
    for (int d = 0; d < 3; ++d) {
        p->geom.h[d] = h[d];
        p->geom.lo[d] = mesh->lo[d];
    }
    p->phys.gamma = mesh->gamma;
    p->phys.flux = mesh->flux;
    p->ns = mesh->equation == DG_NAVIER_STOKES;
    if (p->ns) {
        p->phys.mu = mesh->mu;
        p->phys.kappa = mesh->mu * mesh->gamma / ((mesh->gamma - 1.0) * mesh->Pr);
    }
    if (p->ns && p->max_order > 7) {
        destroy_plan(p);
        return fail(DG_EUNSUPPORTED, "Navier-Stokes plans support orders up to 7");
    }
    for (int v = 0; v < NV; ++v) p->phys.qfar[v] = mesh->q_far[v];

    // geometry of curved plans (and node coordinates of Navier-Stokes plans, for the sweep)
    p->curved = mesh->map_kind == DG_MAP_SINE;
    std::vector<double> met_h, fmet_h;
    std::vector<int64_t> fmo;
    if (p->curved || p->ns) {
        std::vector<double> tab(T_TOT);
        std::vector<float> tab32(T_TOT);
        build_tables(tab.data(), tab32.data());
        p->xyz_h.assign(3 * (size_t)p->n_nodes, 0.0);
        for (int i = 0; i < E; ++i) {
            const int nat = (int)perm[i];
            const int c[3] = {nat % mesh->nx, (nat / mesh->nx) % mesh->ny, nat / (mesh->nx * mesh->ny)};
            double *X = p->xyz_h.data() + 3 * p->noff[i];
            if (!parent) {
                element_coords(*mesh, tab.data(), c, el[i].n, X);
                continue;
            }
            // coarse plan: the fine element's coordinates sampled at the coarse nodes
            const int fi = (int)parent->inv[nat];
            const int32_t nf[3] = {parent->ord[3 * fi] + 1, parent->ord[3 * fi + 1] + 1, parent->ord[3 * fi + 2] + 1};
            const double *Xf = parent->xyz_h.data() + 3 * parent->noff[fi];
            const int32_t *nc = el[i].n;
            const int nef = nf[0] * nf[1] * nf[2], nec = nc[0] * nc[1] * nc[2];
            const double *I1 = tab.data() + T_I + moff(nc[0] - 1, nf[0] - 1);
            const double *I2 = tab.data() + T_I + moff(nc[1] - 1, nf[1] - 1);
            const double *I3 = tab.data() + T_I + moff(nc[2] - 1, nf[2] - 1);
            for (int d = 0; d < 3; ++d)
                for (int k = 0; k < nc[2]; ++k)
                    for (int j = 0; j < nc[1]; ++j)
                        for (int a = 0; a < nc[0]; ++a) {
                            double acc = 0.0;
                            for (int kk = 0; kk < nf[2]; ++kk)
                                for (int jj = 0; jj < nf[1]; ++jj)
                                    for (int ii = 0; ii < nf[0]; ++ii)
                                        acc += I1[a * nf[0] + ii] * I2[j * nf[1] + jj] * I3[k * nf[2] + kk] *
                                               Xf[d * nef + ii + nf[0] * (jj + nf[1] * kk)];
                            X[d * nec + a + nc[0] * (j + nc[1] * k)] = acc;
                        }
        }
        if (p->curved) {
            met_h.assign(10 * (size_t)p->n_nodes, 0.0);
            for (int i = 0; i < E; ++i) {
                double *Mt = met_h.data() + 10 * p->noff[i];
                element_metrics(tab.data(), el[i].n, p->xyz_h.data() + 3 * p->noff[i], Mt);
                const int ne = el[i].n[0] * el[i].n[1] * el[i].n[2];
                for (int t = 0; t < ne; ++t)
                    if (!(Mt[9 * ne + t] > 0.0)) {
                        destroy_plan(p);
                        return fail(DG_EINVAL, "the map folds an element (non-positive Jacobian)");
                    }
            }
            // scaled normals: minus side's Ja^d on the mortar, own outward s Ja^d on boundaries
            fmo.assign(p->nfaces + 1, 0);
            for (int fi = 0; fi < p->nfaces; ++fi) {
                const Face &f = faces[fi];
                const int d = f.d, t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
                if (f.bc != 0) {
                    const int e = f.eL >= 0 ? f.eL : f.eR, s = f.eL >= 0 ? 1 : -1;
                    const int32_t *n = el[e].n;
                    const int ne = n[0] * n[1] * n[2], na = n[t1], nb = n[t2];
                    const double *Mt = met_h.data() + 10 * p->noff[e];
                    for (int m = 0; m < na * nb; ++m) {
                        const int node = face_node_h(n, d, s, m % na, m / na);
                        for (int c = 0; c < 3; ++c) fmet_h.push_back(s * Mt[(3 * d + c) * ne + node]);
                    }
                    fmo[fi + 1] = fmo[fi] + na * nb;
                    continue;
                }
                const int32_t *nL = el[f.eL].n, *nR = el[f.eR].n;
                const int aL = nL[t1], bL = nL[t2];
                const int K1 = std::max(aL, (int)nR[t1]), K2 = std::max(bL, (int)nR[t2]);
                const int neL = nL[0] * nL[1] * nL[2];
                const double *Mt = met_h.data() + 10 * p->noff[f.eL];
                const double *S1 = tab.data() + T_I + moff(K1 - 1, aL - 1);
                const double *S2 = tab.data() + T_I + moff(K2 - 1, bL - 1);
                for (int B = 0; B < K2; ++B)
                    for (int A = 0; A < K1; ++A)
                        for (int c = 0; c < 3; ++c) {
                            double acc = 0.0;
                            for (int b = 0; b < bL; ++b)
                                for (int a = 0; a < aL; ++a)
                                    acc += S1[A * aL + a] * S2[B * bL + b] *
                                           Mt[(3 * d + c) * neL + face_node_h(nL, d, 1, a, b)];
                            fmet_h.push_back(acc);
                        }
                fmo[fi + 1] = fmo[fi] + K1 * K2;
            }
        }
    }

    // sweep layout: combos per element; on box Euler plans isotropic elements (F <= 8)
    // go to the isotropic fast path grouped by F, anisotropic ones with every F_d <= 8 to
    // the anisotropic kernel as (element, pair of x-orders) jobs grouped by F3, and the
    // rest (a direction of 9 or 10 nodes) to the generic (p, c1, c2) work list; curved
    // and Navier-Stokes plans take one task per (element, c1, c2, c3)
    p->combo_off.assign(E + 1, 0);
    std::vector<SweepTask> tasks;
    std::vector<int4> ctasks;
    std::vector<std::vector<int2>> iso(NNMAX + 1);
    std::vector<std::vector<int2>> an(NNMAX + 1);  // (element, pair) per F3
    for (int i = 0; i < E; ++i) {
        int C[3];
        for (int d = 0; d < 3; ++d) C[d] = std::max(1, p->ord[3 * i + d] - 1);
        p->combo_off[i + 1] = p->combo_off[i] + (int64_t)C[0] * C[1] * C[2];
        if (p->curved || p->ns) {
            for (int c3 = 1; c3 <= C[2]; ++c3)
                for (int c2 = 1; c2 <= C[1]; ++c2)
                    for (int c1 = 1; c1 <= C[0]; ++c1) ctasks.push_back(make_int4(i, c1, c2, c3));
            const int m1 = C[0] + 1, m2 = C[1] + 1, m3 = C[2] + 1, nc = m1 * m2 * m3;
            const int f2 = el[i].n[1], f3 = el[i].n[2];
            p->capA = std::max(p->capA, NFLD_SWEEP * std::max(m1 * f2 * f3, nc));
            p->capB = std::max(p->capB, std::max(NFLD_SWEEP * m1 * m2 * f3, 10 * nc));
            p->capS = std::max(p->capS, std::max(3 * NV * nc, 2 * WG));
            p->max_nc = std::max(p->max_nc, nc);
            continue;
        }
        const int F = el[i].n[0];
        if (F == el[i].n[1] && F == el[i].n[2] && F <= 8) {
            iso[F].push_back(make_int2(0, i));
            continue;
        }
        if (el[i].n[0] <= 8 && el[i].n[1] <= 8 && el[i].n[2] <= 8) {
            for (int pr = 0; pr < (C[0] + 1) / 2; ++pr) an[el[i].n[2]].push_back(make_int2(i, pr));
            continue;
        }
        for (int c2 = 1; c2 <= C[1]; ++c2)
            for (int c1 = 1; c1 <= C[0]; ++c1) tasks.push_back({i, c1, c2, 0});
        int f2 = el[i].n[1], f3 = el[i].n[2];
        int m1 = C[0] + 1, m2 = C[1] + 1;
        p->x1cap = std::max(p->x1cap, NV * m1 * f2 * f3);
        p->x2cap = std::max(p->x2cap, NV * m1 * m2 * f3);
    }
    p->ntasks = (int)tasks.size();
    std::vector<int2> iso_all;
    std::vector<int4> an_all;
    std::vector<int4> anw_all;
    for (int F = 0; F <= NNMAX; ++F) {
        p->iso_first[F] = (int)iso_all.size();
        p->iso_count[F] = (int)iso[F].size();
        iso_all.insert(iso_all.end(), iso[F].begin(), iso[F].end());
        // pack the jobs of this F3 greedily into workgroups: a job takes rows * SUMM
        // lanes and 2 * NV * rows * (F2 * F3 + 1) doubles of x-rows
        p->an_first[F] = (int)anw_all.size();
        int lanes = 0, x1 = 0;
        for (const int2 &jb : an[F]) {
            const int32_t *n = el[jb.x].n;
            const int C1 = std::max(1, n[0] - 2), C2 = std::max(1, n[1] - 2);
            const int cA = jb.y + 1, cB = C1 - jb.y == cA ? 0 : C1 - jb.y;
            const int rows = cA + 1 + (cB ? cB + 1 : 0);
            const int nl = rows * (C2 * (C2 + 3) / 2), nx = 2 * NV * rows * (n[1] * F + 1);
            if (anw_all.size() == (size_t)p->an_first[F] || anw_all.back().y == AN_JOBS_MAX ||
                lanes + nl > AN_LANES || x1 + nx > an_stage_doubles(F)) {
                anw_all.push_back(make_int4((int)an_all.size(), 0, 0, 0));
                lanes = x1 = 0;
            }
            an_all.push_back(make_int4(jb.x, jb.y, lanes, x1));
            ++anw_all.back().y;
            lanes += nl;
            x1 += nx;
        }
        p->an_count[F] = (int)anw_all.size() - p->an_first[F];
    }

    p->nctasks = (int)ctasks.size();
    std::vector<float> met32(met_h.begin(), met_h.end()), fmet32(fmet_h.begin(), fmet_h.end());
    // coarse plans: the fine element of every coarse element, restriction LDS capacities
    std::vector<ElemInfo> fine_el;
    if (parent) {
        fine_el.resize(E);
        for (int i = 0; i < E; ++i) {
            const int64_t fi = parent->inv[perm[i]];
            const int32_t *of = parent->ord.data() + 3 * fi, *oc = p->ord.data() + 3 * i;
            for (int d = 0; d < 3; ++d) fine_el[i].n[d] = of[d] + 1;
            fine_el[i].nat = (int32_t)perm[i];
            fine_el[i].noff = parent->noff[fi];
            fine_el[i].foff = 0;
            p->rcapA = std::max(p->rcapA, restrict_cap_a(oc, of));
            p->rcapB = std::max(p->rcapB, restrict_cap_b(oc, of));
        }
    }
    // device work starts here: everything above is host code
    if ((st = device_tables(&p->tabs))) {
        destroy_plan(p);
        return st;
    }
    Arena ar;
    ar.upload(&p->d_el, el);
    ar.upload(&p->d_faces, faces);
    ar.upload(&p->d_tiles, tiles);
    ar.upload(&p->d_combo_off, p->combo_off);
    ar.upload(&p->d_tasks, tasks);
    ar.upload(&p->d_iso, iso_all);
    p->h_iso = iso_all;
    p->h_an = an_all;
    p->h_anw = anw_all;
    ar.upload(&p->d_an, an_all);
    ar.upload(&p->d_anw, anw_all);
    ar.upload(&p->d_wallx, wallx);
    ar.upload(&p->d_ctasks, ctasks);
    ar.upload(&p->d_xyz, p->xyz_h);
    ar.upload(&p->d_met64, met_h);
    ar.upload(&p->d_met32, met32);
    ar.upload(&p->d_fmet64, fmet_h);
    ar.upload(&p->d_fmet32, fmet32);
    ar.upload(&p->d_fmo, fmo);
    ar.upload(&p->d_inv, std::vector<int32_t>(p->inv.begin(), p->inv.end()));
    ar.upload(&p->d_fine_el, fine_el);
    // the face buffer also carries the 15-value BR1 face data of curved Navier-Stokes plans
    const int64_t ff_alloc = std::max<int64_t>(1, (p->curved && p->ns ? 3 : 1) * p->ff_len);
    ar.scratch(&p->d_ff, sizeof(double) * ff_alloc);
    ar.scratch(&p->d_part, sizeof(double) * std::max(1, p->nwallx));
    ar.scratch(&p->d_dudt, sizeof(double) * NV * p->n_nodes);
    ar.scratch(&p->d_sel, sizeof(int32_t) * 3 * std::max(1, E));
    ar.scratch(&p->d_red, sizeof(double) * (dot_partials() + 8));
    if (p->ns) ar.scratch(&p->d_grad, sizeof(double) * 3 * NV * p->n_nodes);
    if (parent) {
        ar.scratch(&p->d_uc, sizeof(double) * NV * p->n_nodes);
        ar.scratch(&p->d_rdc, sizeof(double) * NV * p->n_nodes);
        ar.scratch(&p->d_psic, sizeof(double) * NV * p->n_nodes);
    }
    if ((st = ar.commit(&p->d_arena))) {
        destroy_plan(p);
        return st;
    }
    *out = p;
    return DG_OK;
}

// face pass + element pass with the given epilogue
template <typename T>
dg_status run_residual(dg_plan p, const T *u, EpiArgs epi, hipStream_t s, void *ff, void *gradbuf) {
    const bool f64 = std::is_same<T, double>::value;
    const T *tab = f64 ? (const T *)p->tabs.t64 : (const T *)p->tabs.t32;
    if (p->curved) {
        // curved elements: per-node metric terms, scaled face normals on the mortars
        const T *met = f64 ? (const T *)p->d_met64 : (const T *)p->d_met32;
        const T *fmet = f64 ? (const T *)p->d_fmet64 : (const T *)p->d_fmet32;
        epi.met = met;
        const T *grad = nullptr;
        if (p->ns) {
            for (size_t i = 0; i < p->classes.size(); ++i) {
                const TileClass &c = p->classes[i];
                HIP_TRY(launch_grad_curved<T>(p->d_faces, p->d_fmo, fmet, p->nfaces, p->d_tiles, c.first, c.count,
                                              c.npt, i == 0, p->d_el, u, met, (T *)ff, (T *)gradbuf, tab,
                                              p->phys, epi.isolated, s));
            }
            grad = (const T *)gradbuf;
            epi.grad = gradbuf;
            epi.mu = p->phys.mu;
            epi.kappa = p->phys.kappa;
        }
        if (!epi.isolated)
            HIP_TRY(launch_face_curved<T>(p->d_faces, p->d_fmo, fmet, p->nfaces, p->d_el, u, grad, (T *)ff, tab,
                                          p->phys, p->max_order, s));
        for (const TileClass &c : p->classes)
            HIP_TRY(launch_element<T>(p->d_tiles, c.first, c.count, c.npt, p->d_el, u, (const T *)ff, tab,
                                      p->geom, p->phys, epi, s));
        return DG_OK;
    }
    if (p->ns) {
        // BR1: solution trace, gradients, viscous face fluxes, then the element pass
        for (size_t i = 0; i < p->classes.size(); ++i) {
            const TileClass &c = p->classes[i];
            HIP_TRY(launch_ns_gradient<T>(p->d_faces, p->nfaces, p->d_tiles, c.first, c.count, c.npt, i == 0, p->d_el,
                                          u, (T *)ff, (T *)gradbuf, tab, p->geom, p->phys, p->max_order,
                                          epi.isolated, s));
        }
        if (!epi.isolated)
            HIP_TRY(launch_ns_faces<T>(p->d_faces, p->nfaces, p->d_el, u, (const T *)gradbuf, (T *)ff, tab,
                                       p->geom, p->phys, s));
        epi.grad = gradbuf;
        epi.mu = p->phys.mu;
        epi.kappa = p->phys.kappa;
        for (const TileClass &c : p->classes)
            HIP_TRY(launch_element<T>(p->d_tiles, c.first, c.count, c.npt, p->d_el, u, (const T *)ff, tab,
                                      p->geom, p->phys, epi, s));
        return DG_OK;
    }
    if (!epi.isolated)
        HIP_TRY(launch_face_flux<T>(p->d_faces, p->nfaces, p->d_el, u, (T *)ff, tab, p->geom, p->phys,
                                    p->max_order, s));
    for (const TileClass &c : p->classes)
        HIP_TRY(launch_element<T>(p->d_tiles, c.first, c.count, c.npt, p->d_el, u, (const T *)ff, tab, p->geom,
                                  p->phys, epi, s));
    return DG_OK;
}

template <typename T>
dg_status run_residual(dg_plan p, const T *u, EpiArgs epi, hipStream_t s) {
    return run_residual<T>(p, u, epi, s, p->d_ff, p->d_grad);
}

bool aligned(const void *x) { return ((uintptr_t)x & 15) == 0; }
// every non-null device array argument 16-byte aligned
template <typename... P>
bool all_aligned(P... p) {
    return ((p == nullptr || aligned((const void *)p)) && ...);
}
#define DG_ALIGNED(...) \
    if (!all_aligned(__VA_ARGS__)) return fail(DG_EINVAL, "device arrays must be 16-byte aligned")

// Scratch of the allocation-free residual (dg_residual_noalloc): the face fluxes and
// BR1 gradients live in this file-scope device array instead of the plan's buffers.
// Host code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol): the device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and that address is used.
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kNoAllocDevices] = {};

}  // namespace

static __device__ __align__(256) double scratch[DG_NOALLOC_SCRATCH_DOUBLES];

namespace {

dg_status noalloc_scratch(int dev, double **out) {
    if (dev < 0 || dev >= kNoAllocDevices) return fail(DG_EUNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DG_EHIP, std::string("address of the allocation-free scratch: ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = (double *)ptr;
    }
    *out = g_noalloc_ptr[dev];
    return DG_OK;
}

}  // namespace

extern "C" {

dg_status dg_plan_create(const dg_mesh_desc *mesh, const int32_t *orders_host, dg_plan *out) {
    return build_plan(mesh, orders_host, nullptr, out);
}

dg_status dg_plan_create_coarse(dg_plan fine, const int32_t *coarse_orders_host, dg_plan *out) {
    if (!fine || !coarse_orders_host || !out) return fail(DG_EINVAL, "null argument");
    if (fine->parent) return fail(DG_EINVAL, "the fine plan of a coarse plan must not itself be coarse");
    for (int e = 0; e < fine->E; ++e)
        for (int d = 0; d < 3; ++d) {
            int nc = coarse_orders_host[3 * e + d];
            int nf = fine->ord[3 * fine->inv[e] + d];
            if (nc < 1 || nc > nf) return fail(DG_EINVAL, "coarse orders must satisfy 1 <= Nc <= Nf");
        }
    dg_plan c = nullptr;
    dg_status st = build_plan(&fine->mesh, coarse_orders_host, fine, &c);
    if (st) return st;
    c->parent = fine;
    *out = c;
    return DG_OK;
}

dg_status dg_plan_destroy(dg_plan plan) {
    destroy_plan(plan);
    return DG_OK;
}

dg_status dg_plan_layout(dg_plan p, int64_t *n_elems, int64_t *n_nodes, int64_t *perm, int64_t *node_offset,
                         int32_t *orders) {
    if (!p) return fail(DG_EINVAL, "null plan");
    if (n_elems) *n_elems = p->E;
    if (n_nodes) *n_nodes = p->n_nodes;
    if (perm) std::copy(p->perm.begin(), p->perm.end(), perm);
    if (node_offset) std::copy(p->noff.begin(), p->noff.end(), node_offset);
    if (orders) std::copy(p->ord.begin(), p->ord.end(), orders);
    return DG_OK;
}

dg_status dg_node_coords(dg_plan p, double *xyz, hipStream_t stream) {
    if (!p || !xyz) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(xyz);
    if (p->d_xyz) {
        HIP_TRY(hipMemcpyAsync(xyz, p->d_xyz, sizeof(double) * 3 * p->n_nodes, hipMemcpyDeviceToDevice, stream));
        return DG_OK;
    }
    HIP_TRY(launch_coords(p->d_el, p->E, p->mesh.nx, p->mesh.ny, p->tabs.t64, p->geom, xyz, stream));
    return DG_OK;
}

dg_status dg_plan_metrics(dg_plan p, double *met, hipStream_t stream) {
    if (!p || !met) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(met);
    if (p->curved) {
        HIP_TRY(hipMemcpyAsync(met, p->d_met64, sizeof(double) * 10 * p->n_nodes, hipMemcpyDeviceToDevice, stream));
        return DG_OK;
    }
    // box elements: the constant metric terms, staged on the host
    std::vector<double> h(10 * (size_t)p->n_nodes, 0.0);
    for (int i = 0; i < p->E; ++i) {
        const int64_t ne = p->noff[i + 1] - p->noff[i];
        double *Mt = h.data() + 10 * p->noff[i];
        for (int64_t t = 0; t < ne; ++t) {
            for (int d = 0; d < 3; ++d) Mt[(3 * d + d) * ne + t] = p->geom.Ja[d];
            Mt[9 * ne + t] = p->geom.J;
        }
    }
    HIP_TRY(hipMemcpyAsync(met, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return DG_OK;
}

dg_status dg_residual(dg_plan p, const void *u, void *r, int32_t dtype, int32_t form, int32_t isolated,
                      hipStream_t stream) {
    if (!p || !u || !r) return fail(DG_EINVAL, "null argument");
    if (!aligned(u) || !aligned(r)) return fail(DG_EINVAL, "arrays must be 16-byte aligned");
    if (u == r) return fail(DG_EINVAL, "u and r must not overlap");
    if (form != DG_FORM_NEW && form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    EpiArgs epi{};
    epi.mode = EPI_RESIDUAL;
    epi.form = form;
    epi.isolated = isolated ? 1 : 0;
    epi.out = r;
    if (dtype == DG_F64) return run_residual<double>(p, (const double *)u, epi, stream);
    if (dtype == DG_F32) return run_residual<float>(p, (const float *)u, epi, stream);
    return fail(DG_EINVAL, "unknown dtype");
}

dg_status dg_residual_noalloc(dg_plan p, const void *u, void *r, int32_t dtype, int32_t form, int32_t isolated,
                              hipStream_t stream) {
    if (!p || !u || !r) return fail(DG_EINVAL, "null argument");
    if (!aligned(u) || !aligned(r)) return fail(DG_EINVAL, "arrays must be 16-byte aligned");
    if (u == r) return fail(DG_EINVAL, "u and r must not overlap");
    if (form != DG_FORM_NEW && form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_EINVAL, "unknown dtype");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != p->device) return fail(DG_EINVAL, "the plan's device must be the current device");
    // face fluxes first, BR1 gradients after them (256-byte aligned), both sized for doubles
    const int64_t ffd = (std::max<int64_t>(1, (p->curved && p->ns ? 3 : 1) * p->ff_len) + 31) / 32 * 32;
    const int64_t need = ffd + (p->ns ? int64_t(3) * NV * p->n_nodes : 0);
    if (need > DG_NOALLOC_SCRATCH_DOUBLES)
        return fail(DG_EINVAL, "the plan needs " + std::to_string(need) +
                                   " doubles of residual scratch; the allocation-free residual holds at most " +
                                   std::to_string((long long)DG_NOALLOC_SCRATCH_DOUBLES));
    double *base = nullptr;
    dg_status st = noalloc_scratch(dev, &base);
    if (st) return st;
    EpiArgs epi{};
    epi.mode = EPI_RESIDUAL;
    epi.form = form;
    epi.isolated = isolated ? 1 : 0;
    epi.out = r;
    if (dtype == DG_F64) return run_residual<double>(p, (const double *)u, epi, stream, base, base + ffd);
    return run_residual<float>(p, (const float *)u, epi, stream, base, base + ffd);
}

dg_status dg_tau_estimate(dg_plan fine, dg_plan coarse, const double *u, const double *dudt, int32_t isolated,
                          int32_t restriction, double *tau_new, double *tau_trad, double *norms, double *varnorms,
                          const double *psi, int32_t psi_form, double *eta, hipStream_t stream) {
    if (!fine || !coarse || !u) return fail(DG_EINVAL, "null argument");
    if (restriction != DG_RESTRICT_SAMPLE && restriction != DG_RESTRICT_L2)
        return fail(DG_EINVAL, "restriction must be DG_RESTRICT_SAMPLE or DG_RESTRICT_L2");
    DG_ALIGNED(u, dudt, tau_new, tau_trad, norms, varnorms, psi, eta);
    if (coarse->parent != fine) return fail(DG_EINVAL, "coarse plan was not built from this fine plan");
    if (fine->curved && !isolated)
        for (int i = 0; i < 3 * coarse->E; ++i)
            if (coarse->ord[i] < fine->mesh.geo_order[i % 3])
                return fail(DG_EUNSUPPORTED, "the coupled tau-estimate on curved meshes needs coarse orders >= the "
                                             "geometry order (watertight coarse faces); the isolated one takes any");
    if ((psi == nullptr) != (eta == nullptr)) return fail(DG_EINVAL, "psi and eta go together");
    if (psi_form != DG_FORM_NEW && psi_form != DG_FORM_TRAD)
        return fail(DG_EINVAL, "psi_form must be DG_FORM_NEW or DG_FORM_TRAD");
    if (!tau_new && !tau_trad && !norms && !varnorms && !eta) return DG_OK;
    if (!dudt) {
        EpiArgs epi{};
        epi.mode = EPI_RESIDUAL;
        epi.out = fine->d_dudt;
        dg_status st = run_residual<double>(fine, u, epi, stream);
        if (st) return st;
        dudt = fine->d_dudt;
    }
    HIP_TRY(launch_restrict(coarse->E, coarse->d_el, coarse->d_fine_el, u, dudt, psi, coarse->d_uc,
                            coarse->d_rdc, coarse->d_psic, fine->tabs.t64, coarse->rcapA, coarse->rcapB,
                            restriction, psi && psi_form == DG_FORM_NEW, fine->curved ? fine->d_met64 : nullptr,
                            1.0 / fine->geom.J, stream));
    EpiArgs epi{};
    epi.mode = EPI_TAU;
    epi.isolated = isolated ? 1 : 0;
    epi.out = tau_new;
    epi.out2 = tau_trad;
    epi.rdc = coarse->d_rdc;
    epi.norms = norms;
    epi.varnorms = varnorms;
    epi.psic = psi ? coarse->d_psic : nullptr;
    epi.eta = eta;
    return run_residual<double>(coarse, coarse->d_uc, epi, stream);
}

dg_status dg_sweep_layout(dg_plan p, int64_t *combo_offset) {
    if (!p || !combo_offset) return fail(DG_EINVAL, "null argument");
    std::copy(p->combo_off.begin(), p->combo_off.end(), combo_offset);
    return DG_OK;
}

dg_status dg_tau_sweep(dg_plan p, const double *u, const double *dudt, int32_t restriction, double *te_new,
                       double *te_trad, hipStream_t stream) {
    if (!p || !u || !te_new || !te_trad) return fail(DG_EINVAL, "null argument");
    if (restriction != DG_RESTRICT_SAMPLE && restriction != DG_RESTRICT_L2)
        return fail(DG_EINVAL, "restriction must be DG_RESTRICT_SAMPLE or DG_RESTRICT_L2");
    DG_ALIGNED(u, dudt, te_new, te_trad);
    if ((p->curved || p->ns) && p->max_order > 7)
        return fail(DG_EUNSUPPORTED, "the sweep of curved and Navier-Stokes plans supports fine orders up to 7");
    if (!dudt) {
        EpiArgs epi{};
        epi.mode = EPI_RESIDUAL;
        epi.out = p->d_dudt;
        dg_status st = run_residual<double>(p, u, epi, stream);
        if (st) return st;
        dudt = p->d_dudt;
    }
    if (p->curved || p->ns) {
        HIP_TRY(launch_sweep_curved(p->d_ctasks, p->nctasks, p->d_el, p->d_combo_off, u, dudt, p->d_xyz, p->tabs.t64,
                                    p->phys, p->capA, p->capB, p->capS, p->max_nc, p->ns ? 1 : 0, restriction,
                                    te_new, te_trad, stream));
        return DG_OK;
    }
    const SweepProb one{p->d_el, p->d_combo_off, u, dudt, te_new, te_trad, p->geom, p->mesh.gamma};
    for (int F = 2; F <= 8; ++F)
        if (p->an_count[F])
            HIP_TRY(launch_sweep_an(F, p->d_anw + p->an_first[F], p->an_count[F], p->d_an, one, nullptr,
                                    p->tabs.t64, restriction, stream));
    for (int F = 2; F <= 8; ++F)
        if (p->iso_count[F])
            HIP_TRY(launch_sweep_iso(F, p->d_iso + p->iso_first[F], p->iso_count[F], one, nullptr, p->tabs.t64,
                                     restriction, stream));
    HIP_TRY(launch_sweep_tasks(p->d_tasks, p->ntasks, p->d_el, p->d_combo_off, u, dudt, p->tabs.t64, p->geom,
                               p->mesh.gamma, p->x1cap, p->x2cap, restriction, te_new, te_trad, stream));
    return DG_OK;
}

dg_status dg_select_orders(dg_plan p, const double *const *maps, int32_t nstages, const dg_select_params *prm,
                           int32_t *orders, hipStream_t stream) {
    if (!p || !maps || !prm || !orders) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(orders, prm->prev);
    if (nstages < 1 || nstages > DG_SELECT_MAX_STAGES) return fail(DG_EINVAL, "nstages must be in 1..32");
    for (int s = 0; s < nstages; ++s) {
        if (!maps[s]) return fail(DG_EINVAL, "null map");
        DG_ALIGNED(maps[s]);
    }
    if (prm->approach != 1 && prm->approach != 2) return fail(DG_EINVAL, "approach must be 1 or 2");
    if (prm->jump < 0 || prm->jump > 2) return fail(DG_EINVAL, "jump must be 0, 1 or 2");
    if (prm->nmin < 1 || prm->nmin > prm->nmax || prm->nmax > DG_NMAX)
        return fail(DG_EINVAL, "degrees must satisfy 1 <= nmin <= nmax <= 9");
    if (std::isnan(prm->tau_max)) return fail(DG_EINVAL, "tau_max is NaN");
    if (prm->prev && prm->max_decrease < 0) return fail(DG_EINVAL, "max_decrease must be >= 0");
    if (prm->ext_nmax < 0 || prm->ext_nmax > DG_NMAX || (prm->ext_nmax > 0 && prm->ext_nmax < prm->nmax))
        return fail(DG_EINVAL, "ext_nmax must be 0 (sweep layout) or in nmax..9");
    const dg_mesh_desc &m = p->mesh;
    const int periodic = (m.bc[0] == DG_BC_PERIODIC ? 1 : 0) | (m.bc[2] == DG_BC_PERIODIC ? 2 : 0) |
                         (m.bc[4] == DG_BC_PERIODIC ? 4 : 0);
    HIP_TRY(launch_select(p->d_el, p->E, p->d_combo_off, maps, nstages, prm->tau_max, prm->nmin, prm->nmax,
                          prm->approach, prm->prev, prm->max_decrease, prm->ext_nmax, prm->jump, m.nx, m.ny, m.nz,
                          periodic, orders, p->d_sel, stream));
    return DG_OK;
}

dg_status dg_bdf_rate(dg_plan p, const double *const *states, int32_t nstates, double dt, double *dudt,
                      hipStream_t stream) {
    if (!p || !states || !dudt) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(dudt);
    if (nstates < 2 || nstates > 4) return fail(DG_EINVAL, "nstates must be in 2..4");
    if (!(dt > 0.0)) return fail(DG_EINVAL, "dt must be positive");
    for (int j = 0; j < nstates; ++j) {
        if (!states[j]) return fail(DG_EINVAL, "null state");
        DG_ALIGNED(states[j]);
        if (states[j] == dudt) return fail(DG_EINVAL, "dudt must not alias a state");
    }
    HIP_TRY(launch_bdf_rate(states, nstates, dt, (int64_t)NV * p->n_nodes, dudt, stream));
    return DG_OK;
}

dg_status dg_map_fmax(dg_plan p, double *acc, const double *map, int32_t ext_nmax, hipStream_t stream) {
    if (!p || !acc || !map) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(acc, map);
    if (ext_nmax < 0 || ext_nmax > DG_NMAX) return fail(DG_EINVAL, "ext_nmax must be in 0..9");
    const int64_t n = ext_nmax ? (int64_t)p->E * ext_nmax * ext_nmax * ext_nmax : p->combo_off[p->E];
    HIP_TRY(launch_map_fmax(acc, map, n, stream));
    return DG_OK;
}

dg_status dg_tau_extrapolate(dg_plan p, const double *map, int32_t nmax, double *ext, hipStream_t stream) {
    if (!p || !map || !ext) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(map, ext);
    if (nmax < 1 || nmax > DG_NMAX) return fail(DG_EINVAL, "nmax must be in 1..9");
    HIP_TRY(launch_extrapolate(p->d_el, p->E, p->d_combo_off, map, nmax, ext, stream));
    return DG_OK;
}

dg_status dg_project(dg_plan from, dg_plan to, const double *u, double *ut, hipStream_t stream) {
    if (!from || !to || !u || !ut) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, ut);
    if (from->mesh.nx != to->mesh.nx || from->mesh.ny != to->mesh.ny || from->mesh.nz != to->mesh.nz)
        return fail(DG_EINVAL, "plans of different meshes");
    int capA = 1, capB = 1;
    for (int p = 0; p < to->E; ++p) {
        const int32_t *t = &to->ord[3 * p];
        const int32_t *f = &from->ord[3 * from->inv[to->perm[p]]];
        capA = std::max(capA, restrict_cap_a(t, f));
        capB = std::max(capB, restrict_cap_b(t, f));
    }
    HIP_TRY(launch_project(from->d_inv, to->E, to->d_el, from->d_el, u, ut, from->tabs.t64, capA, capB, stream));
    return DG_OK;
}

dg_status dg_rk3_step(dg_plan p, void *u, void *g, double dt, int32_t nsteps, int32_t dtype, hipStream_t stream) {
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    if (!p || !u || !g) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, g);
    if (u == g) return fail(DG_EINVAL, "u and g must not overlap");
    if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_EINVAL, "unknown dtype");
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return DG_OK;
    GraphKey key{u, g, dt, dtype};
    auto it = p->graphs.find(key);
    if (it == p->graphs.end()) {
        if (p->graphs.size() >= kGraphCache) {
            HIP_TRY(hipDeviceSynchronize());
            auto v = lru_victim(p->graphs);
            (void)hipGraphExecDestroy(v->second.first);
            p->graphs.erase(v);
        }
        if (!p->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph;
        HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
        dg_status st = DG_OK;
        for (int k = 0; k < 3 && !st; ++k) {
            EpiArgs epi{};
            epi.mode = EPI_RK;
            epi.rkA = A[k];
            epi.rkB = B[k];
            epi.dt = dt;
            epi.g = g;
            st = dtype == DG_F64 ? run_residual<double>(p, (const double *)u, epi, p->cap_stream)
                                 : run_residual<float>(p, (const float *)u, epi, p->cap_stream);
        }
        hipError_t e = hipStreamEndCapture(p->cap_stream, &graph);
        if (st) return st;
        if (e != hipSuccess) return fail(DG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t exec;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(DG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = p->graphs.emplace(key, std::make_pair(exec, uint64_t(0))).first;
    }
    it->second.second = ++p->graph_clock;
    for (int s = 0; s < nsteps; ++s) HIP_TRY(hipGraphLaunch(it->second.first, stream));
    return DG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------- adaptation loops
namespace {

// nsteps RK3 steps launched directly (each stage one face and one element pass): the
// adaptation loops change plans from stage to stage, where a captured graph would be
// used once.
dg_status rk3_eager(dg_plan p, double *u, double *g, double dt, int nsteps, hipStream_t s) {
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    for (int n = 0; n < nsteps; ++n)
        for (int k = 0; k < 3; ++k) {
            EpiArgs epi{};
            epi.mode = EPI_RK;
            epi.rkA = A[k];
            epi.rkB = B[k];
            epi.dt = dt;
            epi.g = g;
            const dg_status st = run_residual<double>(p, u, epi, s);
            if (st) return st;
        }
    return DG_OK;
}

// Device buffers of one loop call, freed on every exit.
struct LoopBuffers {
    std::vector<void *> bufs;
    ~LoopBuffers() {
        for (void *b : bufs) (void)hipFree(b);
    }
    template <typename T>
    dg_status alloc(T **p, size_t n) {
        void *b = nullptr;
        if (hipMalloc(&b, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess)
            return fail(DG_ENOMEM, "device allocation failed");
        bufs.push_back(b);
        *p = (T *)b;
        return DG_OK;
    }
};

dg_status check_adapt(dg_plan p, const double *u, const double *work, int64_t capacity, const dg_adapt_params *prm,
                      bool dynamic) {
    if (!p || !u || !work || !prm) return fail(DG_EINVAL, "null argument");
    if (!aligned(u) || !aligned(work)) return fail(DG_EINVAL, "device arrays must be 16-byte aligned");
    if (u == work) return fail(DG_EINVAL, "u and work must be different arrays");
    if (p->parent) return fail(DG_EINVAL, "the loop runs on a fine plan, not a coarse one");
    if (p->curved) return fail(DG_EUNSUPPORTED, "the adaptation loops run box meshes");
    const dg_select_params &sp = prm->select;
    if (prm->steps_per_stage < 0 || prm->steps_after < 0) return fail(DG_EINVAL, "step counts must be >= 0");
    if (prm->nstages < 1 || prm->nstages > DG_SELECT_MAX_STAGES) return fail(DG_EINVAL, "nstages must be in 1..32");
    if (prm->restriction != DG_RESTRICT_SAMPLE && prm->restriction != DG_RESTRICT_L2)
        return fail(DG_EINVAL, "restriction must be DG_RESTRICT_SAMPLE or DG_RESTRICT_L2");
    if (prm->form != DG_FORM_NEW && prm->form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    if (sp.prev || sp.ext_nmax) return fail(DG_EINVAL, "select.prev and select.ext_nmax must be unset");
    if (sp.approach != 1 && sp.approach != 2) return fail(DG_EINVAL, "approach must be 1 or 2");
    if (sp.jump < 0 || sp.jump > 2) return fail(DG_EINVAL, "jump must be 0, 1 or 2");
    if (sp.nmin < 1 || sp.nmin > sp.nmax || sp.nmax > DG_NMAX)
        return fail(DG_EINVAL, "degrees must satisfy 1 <= nmin <= nmax <= 9");
    if (std::isnan(sp.tau_max)) return fail(DG_EINVAL, "tau_max is NaN");
    if (dynamic && sp.max_decrease < 0) return fail(DG_EINVAL, "max_decrease must be >= 0");
    const int sweep_max = p->ns ? 7 : 9;
    if (p->max_order > sweep_max || (dynamic && sp.nmax > sweep_max))
        return fail(DG_EUNSUPPORTED, "every estimated plan needs orders <= 7 for Navier-Stokes");
    const int64_t need = (int64_t)NV * p->E * (int64_t)(sp.nmax + 1) * (sp.nmax + 1) * (sp.nmax + 1);
    if (capacity < std::max<int64_t>(need, NV * p->n_nodes))
        return fail(DG_EINVAL, "capacity must hold 5 E (nmax+1)^3 doubles and the initial state");
    return DG_OK;
}

// A new plan of the same mesh for the degrees selected on the device (natural order),
// the state projected onto it through work; the previous plan is destroyed unless it is
// the caller's.
dg_status replan(dg_plan *cur, dg_plan initial, const int32_t *orders_dev, std::vector<int32_t> &orders_host,
                 double *u, double *work, hipStream_t s) {
    dg_plan p = *cur;
    HIP_TRY(hipMemcpyAsync(orders_host.data(), orders_dev, sizeof(int32_t) * orders_host.size(),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    dg_plan q = nullptr;
    dg_status st = build_plan(&p->mesh, orders_host.data(), nullptr, &q);
    if (st) return st;
    st = dg_project(p, q, u, work, s);
    if (!st && hipMemcpyAsync(u, work, sizeof(double) * NV * q->n_nodes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        st = fail(DG_EHIP, "state copy failed");
    if (st) {
        destroy_plan(q);
        return st;
    }
    if (p != initial) {
        HIP_TRY(hipStreamSynchronize(s));
        destroy_plan(p);
    }
    *cur = q;
    return DG_OK;
}

void natural_orders(dg_plan p, std::vector<int32_t> &o) {
    o.resize(3 * (size_t)p->E);
    for (int i = 0; i < p->E; ++i)
        for (int d = 0; d < 3; ++d) o[3 * p->perm[i] + d] = p->ord[3 * i + d];
}

}  // namespace

extern "C" {

dg_status dg_adapt_dynamic(dg_plan *plan, double *u, double *work, int64_t capacity, const dg_adapt_params *prm,
                           int32_t *stage_orders, dg_adapt_report *report, hipStream_t stream) {
    if (!plan) return fail(DG_EINVAL, "null argument");
    dg_status st = check_adapt(*plan, u, work, capacity, prm, true);
    if (st) return st;
    const dg_plan initial = *plan;
    const int E = initial->E;
    const int cmax = std::max(1, std::max(initial->max_order, prm->select.nmax) - 1);
    LoopBuffers lb;
    double *te[2] = {nullptr, nullptr};
    int32_t *prev = nullptr, *sel = nullptr;
    if ((st = lb.alloc(&te[0], (size_t)E * cmax * cmax * cmax)) || (st = lb.alloc(&te[1], (size_t)E * cmax * cmax * cmax)) ||
        (st = lb.alloc(&prev, 3 * (size_t)E)) || (st = lb.alloc(&sel, 3 * (size_t)E)))
        return st;
    std::vector<int32_t> oh;
    natural_orders(initial, oh);
    HIP_TRY(hipMemcpyAsync(prev, oh.data(), sizeof(int32_t) * oh.size(), hipMemcpyHostToDevice, stream));
    dg_plan cur = initial;
    double ndof_steps = 0.0;
    int64_t steps = 0;
    auto finish = [&](dg_status code) {
        if (code && cur != initial) {
            (void)hipStreamSynchronize(stream);
            destroy_plan(cur);
            cur = initial;
        }
        *plan = cur;
        return code;
    };
    for (int stage = 0; stage < prm->nstages; ++stage) {
        // advance Delta t_e (the RK register lives in work until the projection)
        if ((st = rk3_eager(cur, u, work, prm->dt, prm->steps_per_stage, stream))) return finish(st);
        ndof_steps += (double)cur->n_nodes * prm->steps_per_stage;
        steps += prm->steps_per_stage;
        // estimate the error on the current plan, then adapt the degrees
        if ((st = dg_tau_sweep(cur, u, nullptr, prm->restriction, te[0], te[1], stream))) return finish(st);
        dg_select_params sp = prm->select;
        sp.prev = prev;
        const double *map = te[prm->form == DG_FORM_NEW ? 0 : 1];
        if ((st = dg_select_orders(cur, &map, 1, &sp, sel, stream))) return finish(st);
        if ((st = replan(&cur, initial, sel, oh, u, work, stream))) return finish(st);
        if (stage_orders) std::copy(oh.begin(), oh.end(), stage_orders + (size_t)stage * oh.size());
        std::swap(prev, sel);
    }
    if (report) {
        report->steps = steps;
        report->ndof_dyn = steps ? ndof_steps / (double)steps : (double)cur->n_nodes;
        report->ndof_final = cur->n_nodes;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) return finish(fail(DG_EHIP, "stream synchronisation failed"));
    return finish(DG_OK);
}

dg_status dg_adapt_static(dg_plan *plan, double *u, double *work, int64_t capacity, const dg_adapt_params *prm,
                          int32_t *orders, dg_adapt_report *report, hipStream_t stream) {
    if (!plan) return fail(DG_EINVAL, "null argument");
    dg_status st = check_adapt(*plan, u, work, capacity, prm, false);
    if (st) return st;
    const dg_plan initial = *plan;
    const int64_t nmap = initial->combo_off[initial->E];
    LoopBuffers lb;
    std::vector<double *> maps(prm->nstages);
    double *other = nullptr;
    int32_t *sel = nullptr;
    for (auto &m : maps)
        if ((st = lb.alloc(&m, (size_t)nmap))) return st;
    if ((st = lb.alloc(&other, (size_t)nmap)) || (st = lb.alloc(&sel, 3 * (size_t)initial->E))) return st;
    // estimation stages on the fixed plan, every map stored until T_e
    for (int stage = 0; stage < prm->nstages; ++stage) {
        if ((st = rk3_eager(initial, u, work, prm->dt, prm->steps_per_stage, stream))) return st;
        double *tn = prm->form == DG_FORM_NEW ? maps[stage] : other;
        double *tt = prm->form == DG_FORM_NEW ? other : maps[stage];
        if ((st = dg_tau_sweep(initial, u, nullptr, prm->restriction, tn, tt, stream))) return st;
    }
    // one adaptation from all stored maps (approach 1 or 2), then the rest of the run
    dg_select_params sp = prm->select;
    if ((st = dg_select_orders(initial, (const double *const *)maps.data(), prm->nstages, &sp, sel, stream)))
        return st;
    std::vector<int32_t> oh(3 * (size_t)initial->E);
    dg_plan cur = initial;
    if ((st = replan(&cur, initial, sel, oh, u, work, stream))) return st;
    if (orders) std::copy(oh.begin(), oh.end(), orders);
    if ((st = rk3_eager(cur, u, work, prm->dt, prm->steps_after, stream))) {
        (void)hipStreamSynchronize(stream);
        destroy_plan(cur);
        return st;
    }
    const int64_t steps = (int64_t)prm->nstages * prm->steps_per_stage + prm->steps_after;
    if (report) {
        report->steps = steps;
        report->ndof_dyn = steps ? ((double)initial->n_nodes * prm->nstages * prm->steps_per_stage +
                                    (double)cur->n_nodes * prm->steps_after) / (double)steps
                                 : (double)cur->n_nodes;
        report->ndof_final = cur->n_nodes;
    }
    if (hipStreamSynchronize(stream) != hipSuccess) {
        destroy_plan(cur);
        return fail(DG_EHIP, "stream synchronisation failed");
    }
    *plan = cur;
    return DG_OK;
}

dg_status dg_residual_vjp(dg_plan p, const double *u, const double *v, double *out, int32_t form,
                          int32_t isolated, hipStream_t stream) {
    if (!p || !u || !v || !out) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, v, out);
    if (out == u || out == v) return fail(DG_EINVAL, "out must not overlap u or v");
    if (form != DG_FORM_NEW && form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    if (p->ns) return fail(DG_EUNSUPPORTED, "the VJP is implemented for the Euler equations");
    if (p->curved) return fail(DG_EUNSUPPORTED, "the VJP is implemented for box elements");
    for (size_t i = 0; i < p->classes.size(); ++i) {
        const TileClass &c = p->classes[i];
        HIP_TRY(launch_vjp(p->d_faces, p->nfaces, p->d_tiles, c.first, c.count, c.npt, p->d_el, u, v,
                           (double *)p->d_ff, out, p->tabs.t64, p->geom, p->phys, form, isolated ? 1 : 0,
                           i == 0 && !isolated, p->max_order, stream));
    }
    return DG_OK;
}

dg_status dg_adjoint_workspace(dg_plan p, int32_t restart, int64_t *doubles) {
    if (!p || !doubles) return fail(DG_EINVAL, "null argument");
    if (restart < 1 || restart > DG_ADJOINT_MAX_RESTART) return fail(DG_EINVAL, "restart must be in 1..200");
    const int64_t ld = ((int64_t)NV * p->n_nodes + 1) & ~(int64_t)1;  // vectors 16-byte aligned
    *doubles = (int64_t)(restart + 3) * ld + mdot_partials() + 2 * (restart + 4);
    return DG_OK;
}

// ---------------------------------------------------------------------------- adjoint preconditioner
namespace {
// Preconditioner memory: this header, then (256-byte aligned) the colour starts
// [ncolor + 1], the plan elements grouped by colour [E], the pivots [E][nd], the
// factorisation flags [E], and the inverted blocks [E][nd][nd] (FP32, column-major).
struct PrecondHeader {
    uint64_t magic;  // identifies the plan the memory was built for
    int32_t E, nd, ncolor;
    int32_t compact;  // 0: FP32 inverse blocks; 1: FP16 blocks with per-column FP32 scales
    int64_t off_first, off_elems, off_ipiv, off_info, off_blocks, bytes;
    int64_t off_scales;  // compact form only
};
constexpr int kMaxColors = 27;
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
PrecondHeader precond_layout(int E, int nd) {
    PrecondHeader h{};
    h.E = E;
    h.nd = nd;
    size_t o = align256(sizeof(PrecondHeader));
    h.off_first = (int64_t)o;
    o = align256(o + sizeof(int32_t) * (kMaxColors + 1));
    h.off_elems = (int64_t)o;
    o = align256(o + sizeof(int32_t) * E);
    h.off_ipiv = (int64_t)o;
    o = align256(o + sizeof(int32_t) * (size_t)E * nd);
    h.off_info = (int64_t)o;
    o = align256(o + sizeof(int32_t) * E);
    h.off_blocks = (int64_t)o;
    o += sizeof(float) * (size_t)E * nd * nd;
    h.bytes = (int64_t)o;
    return h;
}
uint64_t plan_magic(dg_plan p) { return 0x4247504a00000000ull ^ (uint64_t)(uintptr_t)p; }
dg_status precond_check(dg_plan p, int *nd) {
    if (p->ns || p->curved) return fail(DG_EUNSUPPORTED, "the adjoint preconditioner is built for box Euler plans");
    for (int i = 0; i < 3 * p->E; ++i)
        if (p->ord[i] != p->ord[i % 3]) return fail(DG_EUNSUPPORTED, "the adjoint preconditioner needs one order triple");
    *nd = NV * (p->ord[0] + 1) * (p->ord[1] + 1) * (p->ord[2] + 1);
    if (*nd > DG_PRECOND_MAX_ND) return fail(DG_EUNSUPPORTED, "element blocks larger than DG_PRECOND_MAX_ND");
    return DG_OK;
}
}  // namespace

dg_status dg_adjoint_precond_bytes(dg_plan p, int64_t *bytes) {
    if (!p || !bytes) return fail(DG_EINVAL, "null argument");
    int nd = 0;
    dg_status st = precond_check(p, &nd);
    if (st) return st;
    *bytes = precond_layout(p->E, nd).bytes;
    return DG_OK;
}

dg_status dg_adjoint_precond_build(dg_plan p, const double *u, int32_t form, int32_t isolated, void *pc, double *work,
                                   hipStream_t stream) {
    if (!p || !u || !pc || !work) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, work);
    if ((uintptr_t)pc & 255) return fail(DG_EINVAL, "the preconditioner memory must be 256-byte aligned");
    if (form != DG_FORM_NEW && form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    int nd = 0;
    dg_status st = precond_check(p, &nd);
    if (st) return st;
    PrecondHeader h = precond_layout(p->E, nd);
    h.magic = plan_magic(p);
    // colouring of the element grid in which face neighbours differ: per direction the
    // parity of the index, with a third colour for the last element of an odd periodic
    // direction; the parity of the index sum when every periodic direction is even
    const int nn[3] = {p->mesh.nx, p->mesh.ny, p->mesh.nz};
    int K[3];
    bool odd_periodic = false;
    for (int d = 0; d < 3; ++d) {
        const bool per = p->mesh.bc[2 * d] == DG_BC_PERIODIC && p->mesh.bc[2 * d + 1] == DG_BC_PERIODIC;
        K[d] = per && (nn[d] % 2) && nn[d] > 1 ? 3 : 2;
        odd_periodic |= K[d] == 3;
    }
    auto colour = [&](int nat) {
        int c[3] = {nat % nn[0], (nat / nn[0]) % nn[1], nat / (nn[0] * nn[1])};
        if (!odd_periodic) return (c[0] + c[1] + c[2]) & 1;
        for (int d = 0; d < 3; ++d) c[d] = (K[d] == 3 && c[d] == nn[d] - 1) ? 2 : c[d] & 1;
        return c[0] + K[0] * (c[1] + K[1] * c[2]);
    };
    h.ncolor = odd_periodic ? K[0] * K[1] * K[2] : 2;
    std::vector<std::vector<int32_t>> byc(h.ncolor);
    for (int e = 0; e < p->E; ++e) byc[colour((int)p->perm[e])].push_back(e);
    std::vector<int32_t> first(kMaxColors + 1, 0), elems;
    for (int c = 0; c < h.ncolor; ++c) {
        first[c] = (int32_t)elems.size();
        elems.insert(elems.end(), byc[c].begin(), byc[c].end());
    }
    first[h.ncolor] = (int32_t)elems.size();
    char *base = (char *)pc;
    HIP_TRY(hipMemcpy(base, &h, sizeof(h), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + h.off_first, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(base + h.off_elems, elems.data(), sizeof(int32_t) * elems.size(), hipMemcpyHostToDevice));
    const int32_t *d_elems = (const int32_t *)(base + h.off_elems);
    float *blocks = (float *)(base + h.off_blocks);
    // probing: v = e_j on one colour, (A v) gathered into column j of those blocks
    const int64_t n = (int64_t)NV * p->n_nodes;
    double *v = work, *out = work + n;
    HIP_TRY(hipMemsetAsync(v, 0, sizeof(double) * n, stream));
    for (int c = 0; c < h.ncolor; ++c) {
        const int32_t *ce = d_elems + first[c];
        const int nc = first[c + 1] - first[c];
        for (int j = 0; j < nd && nc > 0; ++j) {
            HIP_TRY(launch_probe_set(v, ce, nc, p->d_el, j, 1.0, stream));
            if ((st = dg_residual_vjp(p, u, v, out, form, isolated, stream))) return st;
            HIP_TRY(launch_probe_gather(out, blocks, ce, nc, p->d_el, j, nd, stream));
            HIP_TRY(launch_probe_set(v, ce, nc, p->d_el, j, 0.0, stream));
        }
    }
    // LU with partial pivoting and the inverse of every block
    rocblas_handle rh = nullptr;
    if (rocblas_create_handle(&rh) != rocblas_status_success) return fail(DG_EHIP, "rocBLAS handle creation failed");
    rocblas_set_stream(rh, stream);
    int32_t *ipiv = (int32_t *)(base + h.off_ipiv), *info = (int32_t *)(base + h.off_info);
    const rocblas_stride sA = (rocblas_stride)nd * nd;
    rocblas_status rs = rocsolver_sgetrf_strided_batched(rh, nd, nd, blocks, nd, sA, ipiv, nd, info, p->E);
    std::vector<int32_t> hinfo(p->E);
    if (rs == rocblas_status_success &&
        hipMemcpyAsync(hinfo.data(), info, sizeof(int32_t) * p->E, hipMemcpyDeviceToHost, stream) == hipSuccess &&
        hipStreamSynchronize(stream) == hipSuccess) {
        for (int e = 0; e < p->E; ++e)
            if (hinfo[e] != 0) {
                rocblas_destroy_handle(rh);
                return fail(DG_EINVAL, "a singular element block: the adjoint preconditioner is not defined");
            }
        rs = rocsolver_sgetri_strided_batched(rh, nd, blocks, nd, sA, ipiv, nd, info, p->E);
    }
    hipError_t he = hipStreamSynchronize(stream);
    rocblas_destroy_handle(rh);
    if (rs != rocblas_status_success) return fail(DG_EHIP, "rocSOLVER factorisation failed");
    if (he != hipSuccess) return fail(DG_EHIP, std::string("preconditioner build: ") + hipGetErrorString(he));
    return DG_OK;
}

namespace {
dg_status precond_view(dg_plan p, const void *pc, PrecondHeader *h) {
    if (hipMemcpy(h, pc, sizeof(*h), hipMemcpyDeviceToHost) != hipSuccess) return fail(DG_EHIP, "reading the preconditioner");
    if (h->magic != plan_magic(p) || h->E != p->E) return fail(DG_EINVAL, "the preconditioner was built for another plan");
    return DG_OK;
}
PrecondHeader compact_layout(int E, int nd) {
    PrecondHeader h{};
    h.E = E;
    h.nd = nd;
    h.compact = 1;
    size_t o = align256(sizeof(PrecondHeader));
    h.off_first = (int64_t)o;
    o = align256(o + sizeof(int32_t) * (kMaxColors + 1));
    h.off_elems = (int64_t)o;
    o = align256(o + sizeof(int32_t) * E);
    h.off_scales = (int64_t)o;
    o = align256(o + sizeof(float) * (size_t)E * nd);
    h.off_blocks = (int64_t)o;
    o += sizeof(uint16_t) * (size_t)E * nd * nd;
    h.bytes = (int64_t)o;
    return h;
}
// z = M^-1 x with a built preconditioner of either form; with elems (count of them) only
// for those elements, and x - t in place of x when t is given
hipError_t precond_apply(const PrecondHeader &h, const void *pc, const double *x, double *z, dg_plan p,
                         hipStream_t stream, const int32_t *elems = nullptr, int count = 0,
                         const double *t = nullptr) {
    const char *b = (const char *)pc;
    const int ne = elems ? count : p->E;
    if (h.compact)
        return launch_bj_apply16(b + h.off_blocks, (const float *)(b + h.off_scales), x, z, p->d_el, ne, h.nd,
                                 stream, elems, t);
    return launch_bj_apply((const float *)(b + h.off_blocks), x, z, p->d_el, ne, h.nd, stream, elems, t);
}
// the colour offsets of a built preconditioner (host copy): first[c]..first[c + 1] index
// the plan elements of colour c in its element list
dg_status precond_colour_offsets(const PrecondHeader &h, const void *pc, std::vector<int32_t> &first) {
    first.assign(h.ncolor + 1, 0);
    if (hipMemcpy(first.data(), (const char *)pc + h.off_first, sizeof(int32_t) * first.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return fail(DG_EHIP, "reading the preconditioner's colouring");
    return DG_OK;
}
// z = (D + L)^-1 x: the block lower triangle of A^T in colour order (colour-ordered block
// Gauss-Seidel).  z = 0; for each colour c in turn: t = A^T z (c > 0; z then holds the
// colours before c, so on an element of colour c, t is its coupling to them), and
// z_e = D_e^-1 (x_e - t_e) on the elements of colour c.  One VJP per colour after the
// first; t: device scratch of 5 n_nodes doubles.
dg_status precond_apply_gs(const PrecondHeader &h, const void *pc, const std::vector<int32_t> &first, dg_plan p,
                           const double *u, int form, int isolated, const double *x, double *z, double *t,
                           hipStream_t stream) {
    const int64_t n = (int64_t)NV * p->n_nodes;
    const int32_t *elems = (const int32_t *)((const char *)pc + h.off_elems);
    HIP_TRY(launch_axpby(0.0, x, 0.0, z, n, stream));
    for (int c = 0; c < h.ncolor; ++c) {
        const int cnt = first[c + 1] - first[c];
        if (cnt == 0) continue;
        if (c > 0) {
            dg_status st = dg_residual_vjp(p, u, z, t, form, isolated, stream);
            if (st) return st;
        }
        HIP_TRY(precond_apply(h, pc, x, z, p, stream, elems + first[c], cnt, c > 0 ? t : nullptr));
    }
    return DG_OK;
}
}  // namespace

dg_status dg_adjoint_precond_apply_gs(dg_plan p, const void *pc, const double *u, int32_t form, int32_t isolated,
                                      const double *x, double *z, double *work, hipStream_t stream) {
    if (!p || !pc || !u || !x || !z || !work) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, x, z, work);
    if (x == z || work == x || work == z) return fail(DG_EINVAL, "x, z and work must be distinct");
    if (form != DG_FORM_NEW && form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    PrecondHeader h;
    dg_status st = precond_view(p, pc, &h);
    if (st) return st;
    std::vector<int32_t> first;
    if ((st = precond_colour_offsets(h, pc, first))) return st;
    return precond_apply_gs(h, pc, first, p, u, form, isolated, x, z, work, stream);
}

dg_status dg_adjoint_precond_colours(dg_plan p, const void *pc, int32_t *colour) {
    if (!p || !pc || !colour) return fail(DG_EINVAL, "null argument");
    PrecondHeader h;
    dg_status st = precond_view(p, pc, &h);
    if (st) return st;
    std::vector<int32_t> first, elems(p->E);
    if ((st = precond_colour_offsets(h, pc, first))) return st;
    if (hipMemcpy(elems.data(), (const char *)pc + h.off_elems, sizeof(int32_t) * elems.size(),
                  hipMemcpyDeviceToHost) != hipSuccess)
        return fail(DG_EHIP, "reading the preconditioner's colouring");
    for (int c = 0; c < h.ncolor; ++c)
        for (int i = first[c]; i < first[c + 1]; ++i) colour[p->perm[elems[i]]] = c;
    return DG_OK;
}

dg_status dg_adjoint_precond_compact_bytes(dg_plan p, int64_t *bytes) {
    if (!p || !bytes) return fail(DG_EINVAL, "null argument");
    int nd = 0;
    dg_status st = precond_check(p, &nd);
    if (st) return st;
    *bytes = compact_layout(p->E, nd).bytes;
    return DG_OK;
}

dg_status dg_adjoint_precond_compact(dg_plan p, const void *pc, void *pc16, hipStream_t stream) {
    if (!p || !pc || !pc16) return fail(DG_EINVAL, "null argument");
    if ((uintptr_t)pc16 & 255) return fail(DG_EINVAL, "the preconditioner memory must be 256-byte aligned");
    if (pc == pc16) return fail(DG_EINVAL, "the compact preconditioner needs memory of its own");
    PrecondHeader h;
    dg_status st = precond_view(p, pc, &h);
    if (st) return st;
    if (h.compact) return fail(DG_EINVAL, "the preconditioner is already compact");
    PrecondHeader hc = compact_layout(p->E, h.nd);
    hc.magic = h.magic;
    hc.ncolor = h.ncolor;
    char *b = (char *)pc16;
    HIP_TRY(hipMemcpyAsync(b + hc.off_first, (const char *)pc + h.off_first, sizeof(int32_t) * (kMaxColors + 1),
                           hipMemcpyDeviceToDevice, stream));
    HIP_TRY(hipMemcpyAsync(b + hc.off_elems, (const char *)pc + h.off_elems, sizeof(int32_t) * p->E,
                           hipMemcpyDeviceToDevice, stream));
    HIP_TRY(launch_bj_compact((const float *)((const char *)pc + h.off_blocks), b + hc.off_blocks,
                              (float *)(b + hc.off_scales), p->E, h.nd, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    HIP_TRY(hipMemcpy(pc16, &hc, sizeof(hc), hipMemcpyHostToDevice));
    return DG_OK;
}

dg_status dg_adjoint_precond_apply(dg_plan p, const void *pc, const double *x, double *z, hipStream_t stream) {
    if (!p || !pc || !x || !z) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(x, z);
    if (x == z) return fail(DG_EINVAL, "x and z must be distinct");
    PrecondHeader h;
    dg_status st = precond_view(p, pc, &h);
    if (st) return st;
    HIP_TRY(precond_apply(h, pc, x, z, p, stream));
    return DG_OK;
}
static_assert(DG_KRYLOV_MAX == DG_ADJOINT_MAX_RESTART + 1, "Krylov kernels sized for the largest restart");

// Restarted GMRES on A^T psi = g, A = d r / d Q (the residual of the given form), with
// Givens rotations; the host holds the small Hessenberg system, the device the Krylov
// vectors.  Orthogonalisation: classical Gram-Schmidt (all inner products of a step in
// one pass over the vectors, then one update pass), repeated once when it removed more
// than 99 % of w's squared norm (the test of Daniel, Gragg, Kaufman and Stewart with
// kappa = 10, ||w'|| < ||w|| / 10; their kappa = sqrt 2 repeated the round in most
// steps of the adjoint solves here, for the same iteration counts and residuals), with
// one or two host waits per step instead of one per vector.
// Workspace: V_0..V_m, one spare vector, the partials, the step's coefficients.
dg_status dg_adjoint_solve(dg_plan p, const double *u, const double *g, double *psi, const dg_adjoint_params *prm,
                           double *work, int32_t *iters_out, double *relres_out, hipStream_t stream) {
    if (!p || !u || !g || !psi || !prm || !work) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, g, psi, work);
    const int m = prm->restart;
    if (m < 1 || m > DG_ADJOINT_MAX_RESTART) return fail(DG_EINVAL, "restart must be in 1..200");
    if (prm->max_iter < 0 || !(prm->rtol >= 0.0)) return fail(DG_EINVAL, "max_iter >= 0 and rtol >= 0 required");
    if (prm->form != DG_FORM_NEW && prm->form != DG_FORM_TRAD) return fail(DG_EINVAL, "unknown form");
    if (p->ns || p->curved) return fail(DG_EUNSUPPORTED, "the adjoint solve uses the VJP of box Euler plans");
    if (psi == g || psi == u) return fail(DG_EINVAL, "psi must not overlap u or g");
    const int64_t n = (int64_t)NV * p->n_nodes;
    const int64_t ld = (n + 1) & ~(int64_t)1;  // vector stride: every V_j 16-byte aligned
    double *V = work;                        // V_j = V + j ld, j = 0..m
    double *Z = work + (int64_t)(m + 2) * ld;  // M^-1 of a Krylov vector (preconditioned solves)
    double *part = work + (int64_t)(m + 3) * ld;
    PrecondHeader ph{};
    const void *pblk = nullptr;  // the preconditioner, if any (either form)
    std::vector<int32_t> pfirst;
    if (prm->precond_sweep != DG_PRECOND_JACOBI && prm->precond_sweep != DG_PRECOND_GAUSS_SEIDEL)
        return fail(DG_EINVAL, "unknown preconditioner sweep");
    const bool gs = prm->precond && prm->precond_sweep == DG_PRECOND_GAUSS_SEIDEL;
    if (prm->precond) {
        dg_status st0 = precond_view(p, prm->precond, &ph);
        if (st0) return st0;
        pblk = prm->precond;
        if (gs && (st0 = precond_colour_offsets(ph, pblk, pfirst))) return st0;
    }
    // M^-1 v into out; T: scratch of the Gauss-Seidel sweep
    auto papply = [&](const double *v, double *out, double *T) -> dg_status {
        if (gs) return precond_apply_gs(ph, pblk, pfirst, p, u, prm->form, prm->isolated, v, out, T, stream);
        HIP_TRY(precond_apply(ph, pblk, v, out, p, stream));
        return DG_OK;
    };
    double *hb = part + mdot_partials();  // 2 (m + 4) doubles: a step's coefficients and norms
    auto fetch = [&](double *dst, int count) -> dg_status {
        HIP_TRY(hipMemcpyAsync(dst, hb, sizeof(double) * count, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        return DG_OK;
    };
    auto dot = [&](const double *a, const double *b, double *out) -> dg_status {
        HIP_TRY(launch_dot(a, b, n, part, hb, stream));
        return fetch(out, 1);
    };
    auto matvec = [&](const double *v, double *out) {
        return dg_residual_vjp(p, u, v, out, prm->form, prm->isolated, stream);
    };
    // A^T M^-1 v (right preconditioning) or A^T v
    auto pmatvec = [&](const double *v, double *out) -> dg_status {
        if (!pblk) return matvec(v, out);
        dg_status s2 = papply(v, Z, V + (int64_t)(m + 1) * ld);  // V_m+1 is free during a cycle
        if (s2) return s2;
        return matvec(Z, out);
    };
    dg_status st;
    double gn2 = 0.0;
    if ((st = dot(g, g, &gn2))) return st;
    const double gnorm = std::sqrt(gn2);
    int iters = 0;
    double relres = 0.0;
    if (gnorm == 0.0) {
        HIP_TRY(launch_axpby(0.0, g, 0.0, psi, n, stream));
        if (iters_out) *iters_out = 0;
        if (relres_out) *relres_out = 0.0;
        return DG_OK;
    }
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), sv(m + 1), y(m);
    for (;;) {
        // r = g - A^T psi in V_0
        if ((st = matvec(psi, V + ld))) return st;
        HIP_TRY(launch_axpby(1.0, g, 0.0, V, n, stream));
        HIP_TRY(launch_axpby(-1.0, V + ld, 1.0, V, n, stream));
        double b2 = 0.0;
        if ((st = dot(V, V, &b2))) return st;
        const double beta = std::sqrt(b2);
        relres = beta / gnorm;
        if (relres <= prm->rtol || iters >= prm->max_iter || beta == 0.0) break;
        HIP_TRY(launch_axpby(1.0 / beta, V, 0.0, V, n, stream));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(sv.begin(), sv.end(), 0.0);
        sv[0] = beta;
        int k = 0;
        for (int j = 0; j < m && iters < prm->max_iter; ++j) {
            double *vj = V + (int64_t)j * ld, *w = V + (int64_t)(j + 1) * ld;
            if ((st = pmatvec(vj, w))) return st;
            ++iters;
            // classical Gram-Schmidt against V_0..V_j: coefficients and ||w||^2 in one
            // pass, the update with the new ||w||^2 in another, and a second round when
            // the first removed more than 99 % of the squared norm
            std::vector<double> hv(j + 3), h2v(j + 2);
            HIP_TRY(launch_mdot(V, ld, j + 1, w, true, n, part, hb, stream));
            HIP_TRY(launch_maxpy(V, ld, j + 1, hb, w, n, part, hb + j + 2, stream));
            if ((st = fetch(hv.data(), j + 3))) return st;
            double nw = hv[j + 2];
            if (nw < 0.01 * hv[j + 1]) {
                HIP_TRY(launch_mdot(V, ld, j + 1, w, false, n, part, hb, stream));
                HIP_TRY(launch_maxpy(V, ld, j + 1, hb, w, n, part, hb + j + 1, stream));
                if ((st = fetch(h2v.data(), j + 2))) return st;
                for (int i = 0; i <= j; ++i) hv[i] += h2v[i];
                nw = h2v[j + 1];
            }
            for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hv[i];
            const double h1 = std::sqrt(nw);
            H[(size_t)(j + 1) * m + j] = h1;
            if (h1 > 0.0) HIP_TRY(launch_axpby(1.0 / h1, w, 0.0, w, n, stream));
            // previous rotations on column j, then the one that zeroes H[j+1][j]
            for (int i = 0; i < j; ++i) {
                const double a = H[(size_t)i * m + j], b = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * b;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
            }
            const double a = H[(size_t)j * m + j], b = H[(size_t)(j + 1) * m + j];
            const double r = std::hypot(a, b);
            cs[j] = r > 0.0 ? a / r : 1.0;
            sn[j] = r > 0.0 ? b / r : 0.0;
            H[(size_t)j * m + j] = r;
            H[(size_t)(j + 1) * m + j] = 0.0;
            sv[j + 1] = -sn[j] * sv[j];
            sv[j] = cs[j] * sv[j];
            k = j + 1;
            if (std::fabs(sv[j + 1]) <= prm->rtol * gnorm || h1 == 0.0) break;
        }
        // y = H^-1 s (upper triangular), psi += V y
        for (int i = k - 1; i >= 0; --i) {
            double t = sv[i];
            for (int c = i + 1; c < k; ++c) t -= H[(size_t)i * m + c] * y[c];
            y[i] = H[(size_t)i * m + i] != 0.0 ? t / H[(size_t)i * m + i] : 0.0;
        }
        if (!pblk) {
            for (int i = 0; i < k; ++i) HIP_TRY(launch_axpby(y[i], V + (int64_t)i * ld, 1.0, psi, n, stream));
        } else if (k > 0) {
            // psi += M^-1 (V y): V y gathered in V_m+1 (free after the cycle), then mapped
            double *t = V + (int64_t)(m + 1) * ld;
            HIP_TRY(launch_axpby(y[0], V, 0.0, t, n, stream));
            for (int i = 1; i < k; ++i) HIP_TRY(launch_axpby(y[i], V + (int64_t)i * ld, 1.0, t, n, stream));
            if ((st = papply(t, Z, V + ld))) return st;  // V_1 is free once V y is formed
            HIP_TRY(launch_axpby(1.0, Z, 1.0, psi, n, stream));
        }
    }
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = relres;
    return DG_OK;
}

dg_status dg_functional(dg_plan p, const double *u, double *J, double *dJdu, hipStream_t stream) {
    if (!p || !u || !J) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u, J, dJdu);
    if (p->curved) return fail(DG_EUNSUPPORTED, "the functional is implemented for box elements");
    HIP_TRY(launch_functional(p->d_faces, p->d_wallx, p->nwallx, p->d_el, u, p->tabs.t64, p->geom, p->mesh.gamma,
                              p->d_part, J, dJdu, (int64_t)NV * p->n_nodes, stream));
    return DG_OK;
}

dg_status dg_check_state(dg_plan p, const void *u, int32_t dtype, int64_t *bad, hipStream_t stream) {
    if (!p || !u) return fail(DG_EINVAL, "null argument");
    DG_ALIGNED(u);
    if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_EINVAL, "unknown dtype");
    double *part = p->d_red, *out = p->d_red + dot_partials();
    if (dtype == DG_F64)
        HIP_TRY(launch_count_bad<double>(p->d_el, p->E, (const double *)u, p->mesh.gamma, part, out, stream));
    else
        HIP_TRY(launch_count_bad<float>(p->d_el, p->E, (const float *)u, p->mesh.gamma, part, out, stream));
    double cnt = 0.0;
    HIP_TRY(hipMemcpyAsync(&cnt, out, sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (bad) *bad = (int64_t)cnt;
    if (cnt > 0.0) return fail(DG_ENONPHYSICAL, "non-physical state: " + std::to_string((int64_t)cnt) + " nodes");
    return DG_OK;
}

dg_status dg_check(void) {
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipGetLastError());
    return DG_OK;
}

const char *dg_last_error(void) { return g_err.c_str(); }

}  // extern "C"

// ============================================================================ batches
// Many independent problems advanced together: one persistent face launch and one
// persistent element launch per residual evaluation (or RK3 stage) cover every
// problem.  The schedule (tile capacity, grid sizes) is chosen at creation by
// timing candidates on a uniform scratch state.

namespace {

constexpr int kEagerRing = 4;
static_assert(sizeof(ProbDesc<double>) == sizeof(ProbDesc<float>), "one descriptor size for both precisions");

struct BatchKey {
    std::vector<void *> u, g;
    double dt;
    bool operator<(const BatchKey &o) const { return std::tie(u, g, dt) < std::tie(o.u, o.g, o.dt); }
};

}  // namespace

struct dg_batch_s {
    std::vector<dg_plan> plans;
    int dtype = DG_F64;
    int tile_cap = 512, elem_grid = 1024, face_grid = 2048;
    int shape = 1;  // element-kernel shape (launch_elem_batch); valid for every tile of <= 512 nodes
    int ntiles = 0, nfaces = 0;
    BatchTile *d_tiles = nullptr;
    BatchFace *d_faces = nullptr;
    std::vector<std::vector<ElemInfo>> hel;  // element descriptors of every plan (host copies)
    hipStream_t cap_stream = nullptr;
    // Problem-descriptor arrays, allocated at creation: kGraphCache slots for the RK3
    // graphs, then kEagerRing slots for eager residual calls, staged from pinned host
    // memory; a ring slot is reused once the event recorded after its last use is done.
    void *d_desc = nullptr;
    void *h_desc = nullptr;
    hipEvent_t ring_ev[kEagerRing] = {};
    bool ring_used[kEagerRing] = {};
    int ring_next = 0;
    // RK3 graphs: key -> (descriptor slot, graph, call count of the last use)
    struct Graph {
        int slot;
        hipGraphExec_t exec;
        uint64_t last;
    };
    std::map<BatchKey, Graph> graphs;
    uint64_t graph_clock = 0;
    bool from_cache = false;  // schedule taken from the autotuner's cache
    // Isolated sweep of every problem in one launch per fine node count: the plans' work
    // lists merged, each record carrying its problem; sweep descriptors staged per call
    // through the ring slot of the call (d_sdesc, pinned h_sdesc).
    int2 *d_siso = nullptr;
    int4 *d_san = nullptr, *d_sanw = nullptr;
    int siso_first[NNMAX + 1] = {0}, siso_count[NNMAX + 1] = {0};
    int sanw_first[NNMAX + 1] = {0}, sanw_count[NNMAX + 1] = {0};
    void *d_sdesc = nullptr;
    void *h_sdesc = nullptr;
    size_t desc_bytes() const { return sizeof(ProbDesc<double>) * plans.size(); }
    size_t sdesc_bytes() const { return sizeof(SweepProb) * plans.size(); }
    void *desc_slot(int k) const { return (char *)d_desc + desc_bytes() * k; }
};

namespace {

void destroy_batch(dg_batch b) {
    if (!b) return;
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    for (hipEvent_t e : b->ring_ev)
        if (e) (void)hipEventDestroy(e);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_faces) (void)hipFree(b->d_faces);
    if (b->d_desc) (void)hipFree(b->d_desc);
    if (b->h_desc) (void)hipHostFree(b->h_desc);
    if (b->d_siso) (void)hipFree(b->d_siso);
    if (b->d_san) (void)hipFree(b->d_san);
    if (b->d_sanw) (void)hipFree(b->d_sanw);
    if (b->d_sdesc) (void)hipFree(b->d_sdesc);
    if (b->h_sdesc) (void)hipHostFree(b->h_sdesc);
    delete b;
}

// Tiles of every problem for a tile capacity, sorted by node count (largest first).
std::vector<BatchTile> batch_tiles(const std::vector<dg_plan> &plans, const std::vector<std::vector<ElemInfo>> &hel,
                                   int cap) {
    std::vector<std::pair<int, BatchTile>> t;
    for (int pi = 0; pi < (int)plans.size(); ++pi) {
        const dg_plan p = plans[pi];
        for (int i = 0; i < p->E;) {
            int j = i;
            while (j < p->E && p->ord[3 * j] == p->ord[3 * i] && p->ord[3 * j + 1] == p->ord[3 * i + 1] &&
                   p->ord[3 * j + 2] == p->ord[3 * i + 2])
                ++j;
            const int npe = (p->ord[3 * i] + 1) * (p->ord[3 * i + 1] + 1) * (p->ord[3 * i + 2] + 1);
            const int per = std::max(1, cap / npe);
            for (int k = i; k < j; k += per) {
                const int cnt = std::min(per, j - k);
                t.push_back({cnt * npe, BatchTile{pi, k, cnt, 0, hel[pi][k]}});
            }
            i = j;
        }
    }
    std::stable_sort(t.begin(), t.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<BatchTile> out(t.size());
    for (size_t i = 0; i < t.size(); ++i) out[i] = t[i].second;
    return out;
}

template <typename T>
std::vector<ProbDesc<T>> prob_descs(dg_batch b, void *const *u, void *const *out, void *const *g) {
    std::vector<ProbDesc<T>> pd(b->plans.size());
    for (size_t i = 0; i < pd.size(); ++i) {
        const dg_plan p = b->plans[i];
        pd[i].el = p->d_el;
        pd[i].faces = p->d_faces;
        pd[i].u = (T *)u[i];
        pd[i].out = out ? (T *)out[i] : nullptr;
        pd[i].g = g ? (T *)g[i] : nullptr;
        pd[i].ff = (T *)p->d_ff;
        pd[i].geom = p->geom;
        pd[i].phys = p->phys;
    }
    return pd;
}

template <typename T>
dg_status batch_pass(dg_batch b, const ProbDesc<T> *probs, EpiArgs epi, hipStream_t s) {
    const T *tab = std::is_same<T, double>::value ? (const T *)b->plans[0]->tabs.t64
                                                  : (const T *)b->plans[0]->tabs.t32;
    HIP_TRY(launch_face_batch<T>(b->d_faces, b->nfaces, probs, tab, b->face_grid, s));
    HIP_TRY(launch_elem_batch<T>(b->d_tiles, b->ntiles, probs, tab, b->elem_grid, b->shape, epi, s));
    return DG_OK;
}

// The plans' isolated-sweep work lists, merged problem by problem per fine node count.
dg_status merge_sweep_lists(dg_batch b) {
    std::vector<int2> iso;
    std::vector<int4> an, anw;
    for (int F = 0; F <= NNMAX; ++F) {
        b->siso_first[F] = (int)iso.size();
        b->sanw_first[F] = (int)anw.size();
        for (int pi = 0; pi < (int)b->plans.size(); ++pi) {
            const dg_plan p = b->plans[pi];
            for (int k = p->iso_first[F]; k < p->iso_first[F] + p->iso_count[F]; ++k)
                iso.push_back(make_int2(pi, p->h_iso[k].y));
            for (int w = p->an_first[F]; w < p->an_first[F] + p->an_count[F]; ++w) {
                const int4 W = p->h_anw[w];
                anw.push_back(make_int4((int)an.size(), W.y, pi, 0));
                an.insert(an.end(), p->h_an.begin() + W.x, p->h_an.begin() + W.x + W.y);
            }
        }
        b->siso_count[F] = (int)iso.size() - b->siso_first[F];
        b->sanw_count[F] = (int)anw.size() - b->sanw_first[F];
    }
    dg_status st = upload(&b->d_siso, iso);
    if (!st) st = upload(&b->d_san, an);
    if (!st) st = upload(&b->d_sanw, anw);
    return st;
}

dg_status set_tiles(dg_batch b, int cap) {
    auto tiles = batch_tiles(b->plans, b->hel, cap);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    b->d_tiles = nullptr;
    b->ntiles = (int)tiles.size();
    b->tile_cap = cap;
    return upload(&b->d_tiles, tiles);
}

// Time the candidate schedules on a uniform scratch state and keep the fastest.
template <typename T>
dg_status autotune(dg_batch b) {
    int64_t tot = 0;
    for (dg_plan p : b->plans) tot += p->n_nodes;
    T *su = nullptr, *sr = nullptr;
    if (hipMalloc((void **)&su, sizeof(T) * NV * tot) != hipSuccess ||
        hipMalloc((void **)&sr, sizeof(T) * NV * tot) != hipSuccess) {
        if (su) (void)hipFree(su);
        return fail(DG_ENOMEM, "device allocation failed");
    }
    std::vector<void *> up(b->plans.size()), rp(b->plans.size());
    int64_t off = 0;
    for (size_t i = 0; i < b->plans.size(); ++i) {
        up[i] = su + NV * off;
        rp[i] = sr + NV * off;
        HIP_TRY(launch_fill_state<T>(b->plans[i]->d_el, b->plans[i]->E, (T *)up[i], b->cap_stream));
        off += b->plans[i]->n_nodes;
    }
    auto pd = prob_descs<T>(b, up.data(), rp.data(), nullptr);
    ProbDesc<T> *dpd = nullptr;
    dg_status st = upload(&dpd, pd);
    if (st) return st;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int dev = 0, cus = 256;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    EpiArgs epi{};
    epi.mode = EPI_RESIDUAL;
    float best = 1e30f;
    int bc = 512, be = cus, bf = 4 * cus, bs = 1;
    // (tile capacity, element-kernel shape): 256 lanes x 1 node, 256 x 2, 512 x 1.  A
    // tile holds at least one element, so the 256-node shape needs every element to fit.
    int max_npe = 1;
    for (dg_plan p : b->plans)
        for (int e = 0; e < p->E; ++e)
            max_npe = std::max(max_npe, (p->ord[3 * e] + 1) * (p->ord[3 * e + 1] + 1) * (p->ord[3 * e + 2] + 1));
    const int cand[3][2] = {{256, 0}, {512, 1}, {512, 2}};
    for (const auto &cs : cand) {
        const int cap = cs[0];
        if (cap < max_npe) continue;
        b->shape = cs[1];
        if ((st = set_tiles(b, cap))) break;
        // persistent grids of a few waves per CU, or one workgroup per work item
        for (int eg : {2 * cus, 8 * cus, std::max(1, b->ntiles)})
            for (int fg : {16 * cus, std::max(1, b->nfaces)}) {
                b->elem_grid = eg;
                b->face_grid = fg;
                if ((st = batch_pass<T>(b, dpd, epi, b->cap_stream))) break;  // warm-up
                HIP_TRY(hipEventRecord(e0, b->cap_stream));
                for (int r = 0; r < 3 && !st; ++r) st = batch_pass<T>(b, dpd, epi, b->cap_stream);
                HIP_TRY(hipEventRecord(e1, b->cap_stream));
                HIP_TRY(hipEventSynchronize(e1));
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                if (!st && ms < best) {
                    best = ms;
                    bc = cap;
                    be = eg;
                    bf = fg;
                    bs = cs[1];
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(dpd);
    (void)hipFree(su);
    (void)hipFree(sr);
    if (st) return st;
    b->elem_grid = be;
    b->face_grid = bf;
    b->shape = bs;
    return set_tiles(b, bc);
}

// Schedules found by the autotuner, per device (architecture and compute-unit count),
// precision and batch composition (per problem: element and face counts and the number
// of elements of every order triple), so that a batch of the same shape -- for example
// one re-created after an adaptation stage that kept every problem's orders -- skips the
// timing search.  Process-wide, guarded by a mutex.
struct TunedSchedule {
    int tile_cap, shape, elem_grid, face_grid;
};
std::mutex g_tune_mu;
std::map<std::string, TunedSchedule> g_tune_cache;

std::string tune_key(dg_batch b) {
    int dev = 0;
    hipDeviceProp_t prop{};
    // a failed query leaves an empty architecture name: such a key matches no tuned
    // device, so the batch is tuned afresh
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) prop = hipDeviceProp_t{};
    std::string k = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "/" +
                    std::to_string(b->dtype);
    for (dg_plan p : b->plans) {
        std::map<std::tuple<int, int, int>, int> hist;
        for (int e = 0; e < p->E; ++e) ++hist[std::make_tuple(p->ord[3 * e], p->ord[3 * e + 1], p->ord[3 * e + 2])];
        k += "|" + std::to_string(p->E) + "," + std::to_string(p->nfaces);
        for (const auto &kv : hist)
            k += ";" + std::to_string(std::get<0>(kv.first)) + "." + std::to_string(std::get<1>(kv.first)) + "." +
                 std::to_string(std::get<2>(kv.first)) + ":" + std::to_string(kv.second);
    }
    return k;
}

}  // namespace

extern "C" {

dg_status dg_batch_create(const dg_plan *plans, int32_t n, int32_t dtype, dg_batch *out) {
    if (!plans || n <= 0 || !out) return fail(DG_EINVAL, "null argument or empty batch");
    if (dtype != DG_F64 && dtype != DG_F32) return fail(DG_EINVAL, "unknown dtype");
    // handles first (no plan is read before every handle is known to be distinct)
    for (int i = 0; i < n; ++i) {
        if (!plans[i]) return fail(DG_EINVAL, "null plan in batch");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i])
                return fail(DG_EINVAL, "a plan appears twice in the batch (each problem needs its own plan: "
                                       "the plan's face-flux scratch is written by the batched launches)");
    }
    for (int i = 0; i < n; ++i) {
        if (plans[i]->max_order > 7) return fail(DG_EUNSUPPORTED, "batched launches support orders up to 7");
        if (plans[i]->ns) return fail(DG_EUNSUPPORTED, "batched launches run the Euler equations");
        if (plans[i]->curved) return fail(DG_EUNSUPPORTED, "batched launches run box elements");
    }
    dg_batch b = new dg_batch_s();
    b->plans.assign(plans, plans + n);
    b->dtype = dtype;
    // face records: each face with both sides' element descriptors (read back once here)
    std::vector<BatchFace> faces;
    dg_status st = DG_OK;
    for (int i = 0; i < n && !st; ++i) {
        const dg_plan p = plans[i];
        std::vector<Face> pf(p->nfaces);
        std::vector<ElemInfo> pe(p->E);
        if (hipMemcpy(pf.data(), p->d_faces, sizeof(Face) * pf.size(), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(pe.data(), p->d_el, sizeof(ElemInfo) * pe.size(), hipMemcpyDeviceToHost) != hipSuccess) {
            st = fail(DG_EHIP, "reading back a plan's faces failed");
            break;
        }
        for (const Face &f : pf) {
            BatchFace r{};
            r.f = f;
            r.L = pe[f.eL >= 0 ? f.eL : f.eR];
            r.R = pe[f.eR >= 0 ? f.eR : f.eL];
            r.prob = i;
            faces.push_back(r);
        }
        b->hel.push_back(std::move(pe));
    }
    b->nfaces = (int)faces.size();
    if (!st) st = upload(&b->d_faces, faces);
    if (!st && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess)
        st = fail(DG_EHIP, "stream creation failed");
    if (!st) {
        const std::string key = tune_key(b);
        TunedSchedule ts{};
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                ts = it->second;
                hit = true;
            }
        }
        if (hit) {
            b->shape = ts.shape;
            b->elem_grid = ts.elem_grid;
            b->face_grid = ts.face_grid;
            b->from_cache = true;
            st = set_tiles(b, ts.tile_cap);
        } else {
            st = dtype == DG_F64 ? autotune<double>(b) : autotune<float>(b);
            if (!st) {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune_cache[key] = TunedSchedule{b->tile_cap, b->shape, b->elem_grid, b->face_grid};
            }
        }
    }
    if (!st) st = merge_sweep_lists(b);
    if (!st && (hipMalloc(&b->d_sdesc, b->sdesc_bytes() * kEagerRing) != hipSuccess ||
                hipHostMalloc(&b->h_sdesc, b->sdesc_bytes() * kEagerRing, hipHostMallocDefault) != hipSuccess))
        st = fail(DG_ENOMEM, "sweep descriptor allocation failed");
    if (!st && (hipMalloc(&b->d_desc, b->desc_bytes() * (kGraphCache + kEagerRing)) != hipSuccess ||
                hipHostMalloc(&b->h_desc, b->desc_bytes() * kEagerRing, hipHostMallocDefault) != hipSuccess))
        st = fail(DG_ENOMEM, "device or pinned host allocation failed");
    for (int k = 0; k < kEagerRing && !st; ++k)
        if (hipEventCreateWithFlags(&b->ring_ev[k], hipEventDisableTiming) != hipSuccess)
            st = fail(DG_EHIP, "event creation failed");
    if (st) {
        destroy_batch(b);
        return st;
    }
    *out = b;
    return DG_OK;
}

dg_status dg_batch_destroy(dg_batch b) {
    destroy_batch(b);
    return DG_OK;
}

dg_status dg_batch_schedule(dg_batch b, int32_t *tile_cap, int32_t *elem_grid, int32_t *face_grid, int32_t *shape,
                            int32_t *from_cache) {
    if (!b) return fail(DG_EINVAL, "null batch");
    if (tile_cap) *tile_cap = b->tile_cap;
    if (elem_grid) *elem_grid = b->elem_grid;
    if (face_grid) *face_grid = b->face_grid;
    if (shape) *shape = b->shape;
    if (from_cache) *from_cache = b->from_cache ? 1 : 0;
    return DG_OK;
}

dg_status dg_batch_set_schedule(dg_batch b, int32_t tile_cap, int32_t elem_grid, int32_t face_grid,
                                int32_t shape) {
    if (!b) return fail(DG_EINVAL, "null batch");
    if (shape < 0 || shape > 2) return fail(DG_EINVAL, "shape must be 0, 1 or 2");
    if (tile_cap != (shape == 0 ? 256 : 512))
        return fail(DG_EINVAL, "tile capacity 256 goes with shape 0, 512 with shapes 1 and 2");
    if (elem_grid < 1 || face_grid < 1) return fail(DG_EINVAL, "grid sizes must be positive");
    int max_npe = 1;
    for (dg_plan p : b->plans)
        for (int e = 0; e < p->E; ++e)
            max_npe = std::max(max_npe, (p->ord[3 * e] + 1) * (p->ord[3 * e + 1] + 1) * (p->ord[3 * e + 2] + 1));
    if (max_npe > tile_cap) return fail(DG_EINVAL, "an element of the batch does not fit the tile capacity");
    // work in flight and the captured RK3 graphs use the old tiles and grids
    HIP_TRY(hipDeviceSynchronize());
    for (auto &kv : b->graphs) (void)hipGraphExecDestroy(kv.second.exec);
    b->graphs.clear();
    b->shape = shape;
    b->elem_grid = elem_grid;
    b->face_grid = face_grid;
    b->from_cache = false;
    return set_tiles(b, tile_cap);
}

dg_status dg_batch_residual(dg_batch b, const void *const *u, void *const *r, hipStream_t stream) {
    if (!b || !u || !r) return fail(DG_EINVAL, "null argument");
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (!u[i] || !r[i] || u[i] == r[i] || !aligned(u[i]) || !aligned(r[i]))
            return fail(DG_EINVAL, "bad state or residual pointer (null, shared or not 16-byte aligned)");
    EpiArgs epi{};
    epi.mode = EPI_RESIDUAL;
    // descriptors staged through the next ring slot (pinned host -> device, ordered on
    // the stream); the slot's previous use must have finished first
    const int k = b->ring_next;
    b->ring_next = (k + 1) % kEagerRing;
    if (b->ring_used[k]) HIP_TRY(hipEventSynchronize(b->ring_ev[k]));
    void *hs = (char *)b->h_desc + b->desc_bytes() * k;
    void *ds = b->desc_slot((int)kGraphCache + k);
    if (b->dtype == DG_F64) {
        auto pd = prob_descs<double>(b, (void *const *)u, r, nullptr);
        memcpy(hs, pd.data(), b->desc_bytes());
    } else {
        auto pd = prob_descs<float>(b, (void *const *)u, r, nullptr);
        memcpy(hs, pd.data(), b->desc_bytes());
    }
    HIP_TRY(hipMemcpyAsync(ds, hs, b->desc_bytes(), hipMemcpyHostToDevice, stream));
    const dg_status st = b->dtype == DG_F64 ? batch_pass<double>(b, (const ProbDesc<double> *)ds, epi, stream)
                                            : batch_pass<float>(b, (const ProbDesc<float> *)ds, epi, stream);
    HIP_TRY(hipEventRecord(b->ring_ev[k], stream));
    b->ring_used[k] = true;
    return st;
}

dg_status dg_batch_to_f64(dg_batch b, const void *const *u, double *const *u64, hipStream_t stream) {
    if (!b || !u || !u64) return fail(DG_EINVAL, "null argument");
    for (size_t i = 0; i < b->plans.size(); ++i)
        if (!u[i] || !u64[i] || !aligned(u[i]) || !aligned(u64[i]) || u[i] == (const void *)u64[i])
            return fail(DG_EINVAL, "bad state pointer (null, shared or not 16-byte aligned)");
    for (size_t i = 0; i < b->plans.size(); ++i) {
        const int64_t n = NV * b->plans[i]->n_nodes;
        if (b->dtype == DG_F32)
            HIP_TRY(launch_promote((const float *)u[i], u64[i], n, stream));
        else
            HIP_TRY(hipMemcpyAsync(u64[i], u[i], sizeof(double) * n, hipMemcpyDeviceToDevice, stream));
    }
    return DG_OK;
}

dg_status dg_batch_tau_sweep(dg_batch b, const double *const *u64, int32_t restriction, double *const *te_new,
                             double *const *te_trad, hipStream_t stream) {
    if (!b || !u64 || !te_new || !te_trad) return fail(DG_EINVAL, "null argument");
    if (restriction != DG_RESTRICT_SAMPLE && restriction != DG_RESTRICT_L2)
        return fail(DG_EINVAL, "restriction must be DG_RESTRICT_SAMPLE or DG_RESTRICT_L2");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i)
        if (!u64[i] || !te_new[i] || !te_trad[i] || !aligned(u64[i]) || !aligned(te_new[i]) || !aligned(te_trad[i]))
            return fail(DG_EINVAL, "bad state or map pointer (null or not 16-byte aligned)");
    // descriptors of this call staged through the next ring slot, as for dg_batch_residual
    const int k = b->ring_next;
    b->ring_next = (k + 1) % kEagerRing;
    if (b->ring_used[k]) HIP_TRY(hipEventSynchronize(b->ring_ev[k]));
    // the FP64 fine residual of every problem, one batched face and element pass, into
    // each plan's time-derivative scratch
    std::vector<void *> uu(n), rr(n);
    for (size_t i = 0; i < n; ++i) {
        uu[i] = (void *)u64[i];
        rr[i] = b->plans[i]->d_dudt;
    }
    auto pd = prob_descs<double>(b, uu.data(), rr.data(), nullptr);
    void *hs = (char *)b->h_desc + b->desc_bytes() * k;
    void *ds = b->desc_slot((int)kGraphCache + k);
    memcpy(hs, pd.data(), b->desc_bytes());
    HIP_TRY(hipMemcpyAsync(ds, hs, b->desc_bytes(), hipMemcpyHostToDevice, stream));
    EpiArgs epi{};
    epi.mode = EPI_RESIDUAL;
    dg_status st = batch_pass<double>(b, (const ProbDesc<double> *)ds, epi, stream);
    if (st) return st;
    // every problem's sweep, one launch per fine node count
    SweepProb *hsp = (SweepProb *)((char *)b->h_sdesc + b->sdesc_bytes() * k);
    SweepProb *dsp = (SweepProb *)((char *)b->d_sdesc + b->sdesc_bytes() * k);
    for (size_t i = 0; i < n; ++i) {
        const dg_plan p = b->plans[i];
        hsp[i] = SweepProb{p->d_el, p->d_combo_off, u64[i], p->d_dudt, te_new[i], te_trad[i], p->geom, p->mesh.gamma};
    }
    HIP_TRY(hipMemcpyAsync(dsp, hsp, b->sdesc_bytes(), hipMemcpyHostToDevice, stream));
    const SweepProb none{};
    const double *tab = b->plans[0]->tabs.t64;
    for (int F = 2; F <= 8; ++F)
        HIP_TRY(launch_sweep_an(F, b->d_sanw + b->sanw_first[F], b->sanw_count[F], b->d_san, none, dsp, tab,
                                restriction, stream));
    for (int F = 2; F <= 8; ++F)
        HIP_TRY(launch_sweep_iso(F, b->d_siso + b->siso_first[F], b->siso_count[F], none, dsp, tab, restriction,
                                 stream));
    HIP_TRY(hipEventRecord(b->ring_ev[k], stream));
    b->ring_used[k] = true;
    return DG_OK;
}

dg_status dg_batch_rk3_step(dg_batch b, void *const *u, void *const *g, double dt, int32_t nsteps,
                            hipStream_t stream) {
    static const double A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
    static const double B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};
    if (!b || !u || !g) return fail(DG_EINVAL, "null argument");
    if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
    const size_t n = b->plans.size();
    for (size_t i = 0; i < n; ++i)
        if (!u[i] || !g[i] || u[i] == g[i] || !aligned(u[i]) || !aligned(g[i]))
            return fail(DG_EINVAL, "bad state or register pointer (null, shared or not 16-byte aligned)");
    if (nsteps == 0) return DG_OK;
    BatchKey key{std::vector<void *>(u, u + n), std::vector<void *>(g, g + n), dt};
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        if (b->graphs.size() >= kGraphCache) {
            HIP_TRY(hipDeviceSynchronize());
            auto v = b->graphs.begin();
            for (auto j = b->graphs.begin(); j != b->graphs.end(); ++j)
                if (j->second.last < v->second.last) v = j;
            (void)hipGraphExecDestroy(v->second.exec);
            b->graphs.erase(v);
        }
        bool taken[kGraphCache] = {};
        for (const auto &kv : b->graphs) taken[kv.second.slot] = true;
        int slot = 0;
        while (taken[slot]) ++slot;
        void *dpd = b->desc_slot(slot);
        if (b->dtype == DG_F64) {
            auto pd = prob_descs<double>(b, u, nullptr, g);
            HIP_TRY(hipMemcpy(dpd, pd.data(), b->desc_bytes(), hipMemcpyHostToDevice));
        } else {
            auto pd = prob_descs<float>(b, u, nullptr, g);
            HIP_TRY(hipMemcpy(dpd, pd.data(), b->desc_bytes(), hipMemcpyHostToDevice));
        }
        dg_status st = DG_OK;
        hipGraph_t graph;
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        for (int k = 0; k < 3 && !st; ++k) {
            EpiArgs epi{};
            epi.mode = EPI_RK;
            epi.rkA = A[k];
            epi.rkB = B[k];
            epi.dt = dt;
            st = b->dtype == DG_F64 ? batch_pass<double>(b, (const ProbDesc<double> *)dpd, epi, b->cap_stream)
                                    : batch_pass<float>(b, (const ProbDesc<float> *)dpd, epi, b->cap_stream);
        }
        hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
        if (st || e != hipSuccess) return st ? st : fail(DG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        hipGraphExec_t exec;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return fail(DG_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        it = b->graphs.emplace(key, dg_batch_s::Graph{slot, exec, 0}).first;
    }
    it->second.last = ++b->graph_clock;
    for (int s = 0; s < nsteps; ++s) HIP_TRY(hipGraphLaunch(it->second.exec, stream));
    return DG_OK;
}

}  // extern "C"
