// Runs the host side of plan creation (ordering, tiles, face lists, curved geometry and
// metrics, sweep work lists, the device image) on box, curved and Navier-Stokes meshes
// with random orders, and every refusal of invalid arguments, so that a build of the
// host code with AddressSanitizer and UndefinedBehaviorSanitizer checks it.  Without a
// GPU every valid request stops at its first device call with DG_EHIP or DG_ENOMEM;
// with one it succeeds.  Exit status 0 when every request ends as expected.
#include <cstdio>
#include <random>
#include <vector>

#include "../../include/dgtau.h"

static dg_mesh_desc box(int nx, int ny, int nz) {
    dg_mesh_desc m{};
    m.nx = nx, m.ny = ny, m.nz = nz;
    for (int d = 0; d < 3; ++d) m.lo[d] = 0.0, m.hi[d] = 1.0;
    m.map_kind = DG_MAP_BOX;
    m.geo_order[0] = m.geo_order[1] = m.geo_order[2] = 1;
    m.equation = DG_EULER;
    m.gamma = 1.4;
    m.Pr = 0.72;
    m.flux = DG_FLUX_ROE;
    const double q[5] = {1.0, 0.3, 0.1, 0.0, 2.6};
    for (int v = 0; v < 5; ++v) m.q_far[v] = q[v];
    return m;
}

int main() {
    std::mt19937 g(5);
    int bad = 0;
    auto expect = [&](const dg_mesh_desc &m, const std::vector<int32_t> &o, bool valid, const char *what) {
        dg_plan p = nullptr;
        const dg_status st = dg_plan_create(&m, o.data(), &p);
        const bool ok = valid ? (st == DG_OK || st == DG_EHIP || st == DG_ENOMEM) : st == DG_EINVAL;
        if (!ok) {
            std::printf("%s: status %d (%s)\n", what, st, dg_last_error());
            ++bad;
        }
        if (p) dg_plan_destroy(p);
    };
    auto orders = [&](int E, int lo, int hi) {
        std::vector<int32_t> o(3 * E);
        std::uniform_int_distribution<int> u(lo, hi);
        for (auto &x : o) x = u(g);
        return o;
    };
    dg_mesh_desc m = box(4, 3, 2);
    m.bc[0] = DG_BC_SLIP_WALL, m.bc[1] = DG_BC_FARFIELD;
    expect(m, orders(24, 1, 9), true, "box, wall and far field, orders 1..9");
    m = box(5, 4, 3);
    expect(m, orders(60, 1, 7), true, "periodic box, orders 1..7");
    m = box(3, 3, 2);
    m.equation = DG_NAVIER_STOKES;
    m.mu = 0.01;
    expect(m, orders(18, 1, 7), true, "Navier-Stokes box");
    m = box(4, 4, 2);
    m.map_kind = DG_MAP_SINE;
    m.map_amp = 0.05;
    m.geo_order[0] = m.geo_order[1] = 2;
    m.hi[2] = 0.5;
    std::vector<int32_t> oc = orders(32, 2, 6);
    for (int e = 0; e < 32; ++e) oc[3 * e + 2] = 1 + (e % 2);
    expect(m, oc, true, "curved, per-element orders");
    m.equation = DG_NAVIER_STOKES;
    m.mu = 0.01;
    expect(m, oc, true, "curved Navier-Stokes");
    // refusals
    m = box(2, 2, 2);
    std::vector<int32_t> o8 = orders(8, 1, 5);
    std::vector<int32_t> o8b = o8;
    o8b[5] = 10;
    expect(m, o8b, false, "order 10");
    o8b[5] = 0;
    expect(m, o8b, false, "order 0");
    dg_mesh_desc mb = m;
    mb.bc[0] = DG_BC_SLIP_WALL;
    expect(mb, o8, false, "unpaired periodic face");
    mb = m;
    mb.gamma = 1.0;
    expect(mb, o8, false, "gamma 1");
    mb = m;
    mb.nx = 0;
    expect(mb, o8, false, "no elements");
    mb = m;
    mb.map_kind = DG_MAP_SINE;
    mb.geo_order[0] = mb.geo_order[1] = 2;
    expect(mb, o8, false, "curved orders below the geometry order");
    std::printf(bad ? "plan driver: %d failures\n" : "plan driver ok\n", bad);
    return bad ? 1 : 0;
}
