// CPU-only driver of libodp's host runtime for an AddressSanitizer /
// UndefinedBehaviorSanitizer build: argument validation, grids, plans of
// single solves and of a 512-solve batch for every dynamics, precision, RK
// order and spatial order, their host images, and a tile-coverage count:
// replaying the stage kernels' block -> (solve, planes, points) mapping from
// each plan's descriptors, every (plane, hyperplane element) of every solve
// must be covered by exactly one tile; and the default chunk of single
// first-order 4D solves (one round of resident blocks).  Prints "ok" on
// success.
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "plan.h"
#include "runtime.h"

using namespace odp;

static int fails = 0;
#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::printf("check failed line %d: %s\n", __LINE__, #c);      \
            ++fails;                                                      \
        }                                                                 \
    } while (0)

static odp_grid *grid(int nd, const int64_t *n, const uint8_t *per, double lo = -4.0, double hi = 4.0) {
    double L[6], H[6];
    for (int d = 0; d < nd; ++d) { L[d] = lo; H[d] = hi; }
    odp_grid *g = nullptr;
    CHECK(odp_grid_create(nd, n, L, H, per, &g) == ODP_OK);
    return g;
}

// Replay of the stage kernel's tile mapping: tile lt of a solve covers planes
// [cid * chunk, min(+chunk, n0)), cid = lt / nqb, and, for each of its
// kBlock threads, the group of VEC consecutive hyperplane elements that
// tile_group gives tile qb = lt % nqb (row-major or brick tiles).  Every
// element must be covered exactly once, every group (also a past-the-end
// thread's) must lie inside the hyperplane, and a tile's first element must
// be the start of its threads' range.  The copy kernels' row-major groups
// must cover the hyperplane too (brick tiles are at least as many).
static int g_brick_plans = 0;  // plans whose tiles were brick tiles
static int g_quad_plans = 0;   // of which quad tiles

static void coverage(const Plan &p, const std::vector<unsigned char> &img) {
    for (size_t i = 0; i < p.items.size(); ++i) {
        SolveDesc s;
        std::memcpy(&s, img.data() + p.desc_off + i * sizeof(SolveDesc), sizeof(s));
        const int64_t Q = s.Q, n0 = s.n0;
        std::vector<uint8_t> cnt(size_t(Q * n0), 0);
        for (uint32_t lt = 0; lt < s.tiles; ++lt) {
            const uint32_t cid = lt / s.nqb, qb = lt - cid * s.nqb;
            const int i0b = int(cid) * s.chunk, i0e = std::min<int>(i0b + s.chunk, int(n0));
            CHECK(i0b < i0e);
            for (int t = 0; t < kBlock; ++t) {
                const TileGroup tg = tile_group(s, qb, uint32_t(t), uint32_t(s.vec));
                CHECK(int64_t(tg.q) + s.vec <= Q);
                // a tile's (quad: a wave's) first thread starts its range
                if ((t == 0 || (s.quad && (t & 63) == 0)) && tg.active) CHECK(tg.q == tg.q0);
                if (!tg.active) continue;
                CHECK(tg.q % uint32_t(s.vec) == 0);
                for (int j = 0; j < s.vec; ++j)
                    for (int i0 = i0b; i0 < i0e; ++i0) cnt[size_t(i0 * Q + tg.q + j)]++;
            }
        }
        bool once = true;
        for (uint8_t c : cnt) once = once && c == 1;
        CHECK(once);
        CHECK(Q % s.vec == 0);
        CHECK(int64_t(s.nqb) * kBlock * s.vec >= Q);
        CHECK(s.pitch >= s.n[s.ndim - 1] || s.ndim == 1);
        if (s.brick) {
            ++g_brick_plans;
            if (s.quad) ++g_quad_plans;
            CHECK(s.ndim == 6 && s.n[1] % int(s.brick) == 0 && s.n[2] % int(s.brick) == 0);
            CHECK(int64_t(s.cube) * s.n[1] * s.n[2] == Q);
            CHECK(!s.quad || (s.brick % 2 == 0 && s.lds == 2 && s.pitch <= 32 * s.vec));
        }
    }
}

static void plan_case(const std::vector<const odp_grid *> &gs, const std::vector<odp_dynamics> &dyns,
                      odp_solve_opts o, int chunk) {
    std::vector<PlanItem> items;
    const double tau[3] = {0.0, 0.21, 0.4};
    for (size_t i = 0; i < gs.size(); ++i) {
        PlanItem it;
        it.g = gs[i];
        it.dyn = dyns[i];
        it.V0 = (const void *)uintptr_t(4096 * (i + 1));
        it.A = (void *)uintptr_t(4096 * (i + 9000));
        it.tau.assign(tau, tau + 3);
        if (gs.size() > 1 && gs[i]->ndim >= 2 && o.space_order != 2) {
            const int64_t nl = gs[i]->n[gs[i]->ndim - 1], w = o.precision == 32 ? 4 : 2;
            if (nl % w) {
                it.pitch = int((nl + w - 1) / w * w);
                it.pad_io = true;
            }
        }
        items.push_back(it);
    }
    Plan p;
    std::vector<int> perm = plan_build(p, items, o, chunk);
    CHECK(perm.size() == gs.size());
    CHECK(p.error.empty());
    std::vector<unsigned char> img;
    plan_image(p, (unsigned char *)uintptr_t(1u << 20), img);
    CHECK(img.size() == p.upload_bytes);
    for (const PlanItem &it : p.items) {
        CHECK(it.nsteps > 0 && it.nsteps < it.max_steps);
        CHECK(it.box_cfl || int64_t(it.land.size()) == it.nsteps);
    }
    coverage(p, img);
}

// The default chunk of a single first-order 4D solve: whole tiles of one
// round of resident blocks (1024) when the whole-axis
// tiles fit one round, filled to at least 65% unless even one-plane chunks
// cannot fill it, and the fewest chunks that do.
static void default_chunk_case(const int64_t *n, int prec) {
    const uint8_t per[4] = {0, 0, 0, 1};
    odp_grid *g = grid(4, n, per);
    odp_dynamics d{};
    d.id = ODP_DYN_DYNCAR4D; d.u_mode = 1; d.p[0] = 1.0; d.p[1] = 1.0;
    odp_solve_opts o{};
    o.precision = prec;
    o.rk_order = 3;
    o.cfl = 0.8;
    o.mode = ODP_BRT;
    o.space_order = 1;
    PlanItem it;
    it.g = g;
    it.dyn = d;
    it.V0 = (const void *)uintptr_t(4096);
    it.A = (void *)uintptr_t(8192);
    it.tau = {0.0, 0.3};
    Plan p;
    plan_build(p, {it}, o, 0);
    CHECK(p.error.empty());
    const PlanItem &q = p.items[0];
    const int64_t n0 = n[0], round = 1024;
    const int64_t chunks = (n0 + q.chunk - 1) / q.chunk;
    CHECK(q.chunk >= 1 && q.chunk <= n0);
    CHECK(int64_t(q.tiles) == int64_t(q.nqb) * chunks);
    if (int64_t(q.nqb) <= round) {
        const int64_t fill = round * 13 / 20, tiles = q.tiles;
        CHECK(tiles <= round);
        for (int64_t b = 1; b <= n0; ++b) {
            const int64_t t = int64_t(q.nqb) * ((n0 + b - 1) / b);
            // filled: no chunk length giving fewer chunks fills 65% too;
            // not filled: no chunk length that fits one round has more tiles
            if (tiles >= fill && (n0 + b - 1) / b < chunks) CHECK(t < fill);
            if (tiles < fill && t <= round) CHECK(t <= tiles);
        }
    }
    odp_grid_destroy(g);
}

int main() {
    // argument validation
    {
        odp_grid *g = nullptr;
        const int64_t n[3] = {10, 2, 8};
        const double lo[3] = {0, 0, 0}, hi[3] = {1, 1, 1};
        CHECK(odp_grid_create(3, n, lo, hi, nullptr, &g) == ODP_EINVAL && !g);
        const int64_t n2[1] = {5};
        const double bad[1] = {1.0};
        CHECK(odp_grid_create(1, n2, bad, bad, nullptr, &g) == ODP_EINVAL);
        CHECK(odp_grid_create(7, n2, lo, hi, nullptr, &g) == ODP_EINVAL);
        CHECK(std::strlen(odp_last_error()) > 0);
        CHECK(odp_strerror(-99) != nullptr);
    }
    std::mt19937 rng(220405520);
    auto U = [&](int a, int b) { return int(std::uniform_int_distribution<int>(a, b)(rng)); };
    for (int prec : {32, 64})
        for (int order : {1, 2})
            for (int rk : {1, 2, 3}) {
                odp_solve_opts o;
                std::memset(&o, 0, sizeof(o));
                o.precision = prec;
                o.rk_order = rk;
                o.cfl = 0.8;
                o.mode = ODP_BRT;
                o.space_order = order;
                // single solves of every dynamics, ragged shapes, a few chunks
                const uint8_t p3[3] = {0, 0, 1}, p4[4] = {0, 0, 0, 1}, p6[6] = {0, 0, 1, 0, 0, 1};
                for (int rep = 0; rep < 3; ++rep) {
                    const int64_t n3[3] = {U(5, 40), U(5, 40), U(4, 37)};
                    const int64_t n4[4] = {U(5, 20), U(5, 20), U(5, 20), U(4, 23)};
                    const int64_t n6[6] = {U(5, 9), U(5, 9), U(4, 9), U(5, 9), U(5, 9), U(4, 11)};
                    odp_grid *g3 = grid(3, n3, p3), *g4 = grid(4, n4, p4), *g6 = grid(6, n6, p6);
                    odp_dynamics d1{}, d2{}, d3{}, d4{};
                    d1.id = ODP_DYN_DUBINS3D; d1.u_mode = 1; d1.p[0] = 1.0; d1.p[1] = 1.0;
                    d2.id = ODP_DYN_DYNCAR4D; d2.u_mode = 1; d2.p[0] = 1.0; d2.p[1] = 1.0;
                    d3.id = ODP_DYN_TWODUBINS6D; d3.u_mode = 1; d3.p[0] = 1; d3.p[1] = 1; d3.p[2] = 1; d3.p[3] = 1;
                    d4.id = ODP_DYN_PE3D; d4.u_mode = 1; d4.p[0] = 1; d4.p[1] = 1; d4.p[2] = 1; d4.p[3] = 1;
                    for (int chunk : {0, 1, 3, 5, 13}) {
                        plan_case({g3}, {d1}, o, chunk);
                        plan_case({g4}, {d2}, o, chunk);
                        plan_case({g6}, {d3}, o, chunk);
                        plan_case({g3}, {d4}, o, chunk);
                    }
                    CHECK(odp_hj_workspace_bytes(g4, &d2, (const double[]){0.0, 0.3}, 2, &o) > 0);
                    CHECK(odp_hj_workspace_bytes(g4, &d1, (const double[]){0.0, 0.3}, 2, &o) == 0);  // dim mismatch
                    odp_grid_destroy(g3);
                    odp_grid_destroy(g4);
                    odp_grid_destroy(g6);
                }
                // a batch of many small Dubins solves (padded rows) and single integrators
                std::vector<odp_grid *> owned;
                std::vector<const odp_grid *> gs;
                std::vector<odp_dynamics> ds;
                for (int i = 0; i < 96; ++i) {
                    if (i % 8 == 7) {
                        const int nd = U(1, 6);
                        int64_t n[6];
                        uint8_t per[6];
                        for (int d = 0; d < nd; ++d) { n[d] = U(3, 9); per[d] = uint8_t(U(0, 1)); }
                        owned.push_back(grid(nd, n, per));
                        odp_dynamics d{};
                        d.id = ODP_DYN_SINGLE_INTEGRATOR;
                        d.p[0] = 1.0;
                        ds.push_back(d);
                    } else {
                        const int64_t n[3] = {U(8, 40), U(8, 40), U(6, 24)};
                        owned.push_back(grid(3, n, p3));
                        odp_dynamics d{};
                        d.id = ODP_DYN_DUBINS3D;
                        d.u_mode = 1;
                        d.p[0] = 0.5 + U(0, 10) / 10.0;
                        d.p[1] = 0.5 + U(0, 15) / 10.0;
                        ds.push_back(d);
                    }
                    gs.push_back(owned.back());
                }
                plan_case(gs, ds, o, 0);
                plan_case(gs, ds, o, 4);
                for (odp_grid *g : owned) odp_grid_destroy(g);
            }
    // six-dimensional grids with cubes of axes 3..5 large enough for brick
    // tiles: quad tiles (even squares; first order), 3x3 squares (and second
    // order on either), and one that misses a condition (an axis-1 extent
    // that is not a multiple of 3)
    for (int prec : {32, 64})
        for (int order : {1, 2}) {
            odp_solve_opts o;
            std::memset(&o, 0, sizeof(o));
            o.precision = prec;
            o.rk_order = 2;
            o.cfl = 0.8;
            o.mode = ODP_BRT;
            o.space_order = order;
            const uint8_t p6[6] = {0, 0, 1, 0, 0, 1};
            for (int rep = 0; rep < 3; ++rep) {
                const int64_t n6q[6] = {U(3, 6), 6, 6, U(18, 26), U(18, 26), 4 * U(6, 8)};
                const int64_t n6b[6] = {U(3, 6), 9, 3, 24, 24, 36};
                const int64_t n6r[6] = {U(3, 6), 7, 6, U(18, 26), U(18, 26), 4 * U(6, 10)};
                const int64_t *n6 = rep == 0 ? n6q : rep == 1 ? n6b : n6r;
                odp_grid *g6 = grid(6, n6, p6);
                odp_dynamics d3{};
                d3.id = ODP_DYN_TWODUBINS6D; d3.u_mode = 1; d3.p[0] = 1; d3.p[1] = 1; d3.p[2] = 1; d3.p[3] = 1;
                for (int chunk : {0, 5}) plan_case({g6}, {d3}, o, chunk);
                odp_grid_destroy(g6);
            }
        }
    CHECK(g_brick_plans > 0 && g_quad_plans > 0 && g_quad_plans < g_brick_plans);
    // default chunks of single first-order 4D solves, cubic and ragged
    for (int prec : {32, 64}) {
        for (int64_t c = 20; c <= 100; c += 4) {
            const int64_t n[4] = {c, c, c, c};
            default_chunk_case(n, prec);
        }
        std::mt19937 rng(7);
        for (int rep = 0; rep < 40; ++rep) {
            auto V = [&](int a, int b) { return int64_t(std::uniform_int_distribution<int>(a, b)(rng)); };
            const int64_t n[4] = {V(20, 100), V(20, 100), V(20, 100), 4 * V(5, 25)};
            default_chunk_case(n, prec);
        }
    }
    // time to reach workspace, the server's argument checks (no device here)
    {
        const int64_t n[3] = {20, 20, 16};
        const uint8_t p3[3] = {0, 0, 1};
        odp_grid *g = grid(3, n, p3);
        odp_ttr_opts t{};
        t.precision = 32;
        CHECK(odp_ttr_workspace_bytes(g, &t) > 0);
        t.precision = 16;
        CHECK(odp_ttr_workspace_bytes(g, &t) == 0);
        odp_solve_opts o{};
        o.precision = 32;
        o.rk_order = 1;
        o.cfl = 0.8;
        odp_server *srv = nullptr;
        CHECK(odp_server_create(1 << 20, 0, &o, &srv) == ODP_EINVAL && !srv);
        odp_grid_destroy(g);
    }
    if (fails) {
        std::printf("%d checks failed\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
