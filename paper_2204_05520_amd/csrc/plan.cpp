// Plans: layout, host image, prologue (alpha^max + float64 schedules on the
// device), lockstep stepping and statistics for a list of solves.
//
// The host works out every solve's step count from the same float64 tables
// and operations as the device reduction and schedule (the maximum is exact
// and no contraction is allowed on either side), so enqueueing the steps
// needs no read-back: a call returns once its work is enqueued.  The device
// schedule stays the one the kernels read; it flags a schedule longer than
// the host's count.  Solves whose step comes from the costate box get it on
// the device, step by step; the host enqueues the all-inputs count, which
// bounds theirs (each box step is at least the all-inputs step).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <map>
#include <mutex>
#include <numeric>
#include <string>

namespace odp {

namespace {

// per-solve state: alpha^max[6] (0), nsteps (48), step (56), flags (64),
// dt min / max (72, 80)
constexpr size_t kStateBytes = 128;

int64_t step_capacity(const odp_grid *g, const odp_dynamics *dyn, const std::vector<double> &tau,
                      double cfl, double max_dt) {
    double ab[kMaxDim];
    alpha_bound(g, dyn, ab);
    double s = 0.0;
    for (int d = 0; d < g->ndim; ++d) s += ab[d] / g->dx[d];
    double dt_lo = s > 0.0 ? cfl / s : INFINITY;
    if (max_dt > 0.0) dt_lo = std::min(dt_lo, max_dt);
    const double span = tau.back() - tau.front();
    const double est = std::isfinite(dt_lo) ? std::ceil(span / dt_lo) : 0.0;
    // landing steps and a rounding slack per output interval
    return int64_t(std::min(est, 1e9)) + 2 * int64_t(tau.size()) + 8;
}

// Axis tables: coordinate, cos, sin per axis (float64, computed once on the
// host; the kernels read these values, never a transcendental).  Axes with
// the same node count, lower bound and spacing share their table (the many
// solves of a batch repeat a few axis shapes).
using AxisKey = std::tuple<int64_t, double, double>;
void make_tables(const odp_grid *g, std::vector<double> &tab, std::map<AxisKey, std::vector<double>> &cache) {
    tab.clear();
    for (int d = 0; d < g->ndim; ++d) {
        const int nd = int(g->n[d]);
        std::vector<double> &t = cache[AxisKey(g->n[d], g->lo[d], g->dx[d])];
        if (t.empty()) {
            t.resize(3 * size_t(nd));
            for (int k = 0; k < nd; ++k) {
                const double x = g->lo[d] + double(k) * g->dx[d];
                t[k] = x;
                t[nd + k] = std::cos(x);
                t[2 * nd + k] = std::sin(x);
            }
        }
        tab.insert(tab.end(), t.begin(), t.end());
    }
}

// alpha^max_d as the device reduction (alpha_kernel) computes it: the same
// float64 expression per node on the same table values, the largest over the
// nodes (taken over the axes each term depends on; the maximum is exact).
void host_alpha_max(const PlanItem &it, double *am) {
    const odp_grid *g = it.g;
    const double *p = it.dyn.p;
    const int N = g->ndim;
    const double *X[kMaxDim], *C[kMaxDim], *S[kMaxDim];
    size_t off = 0;
    for (int d = 0; d < N; ++d) {
        const size_t nd = size_t(g->n[d]);
        X[d] = it.tab.data() + off;
        C[d] = it.tab.data() + off + nd;
        S[d] = it.tab.data() + off + 2 * nd;
        off += 3 * nd;
    }
    for (int d = 0; d < kMaxDim; ++d) am[d] = 0.0;
    auto mx = [](double &a, double v) { a = std::fmax(a, v); };
    switch (it.dyn.id) {
    case ODP_DYN_SINGLE_INTEGRATOR:
        for (int d = 0; d < N; ++d) am[d] = std::fabs(p[1 + d]) + p[0];
        break;
    case ODP_DYN_DUBINS3D:
        for (int64_t k = 0; k < g->n[2]; ++k) {
            mx(am[0], std::fabs(p[0] * C[2][k]));
            mx(am[1], std::fabs(p[0] * S[2][k]));
        }
        am[2] = std::fabs(p[1]);
        break;
    case ODP_DYN_DYNCAR4D:
        for (int64_t j = 0; j < g->n[2]; ++j)
            for (int64_t k = 0; k < g->n[3]; ++k) {
                const double v = X[2][j];
                mx(am[0], std::fabs(v * C[3][k]));
                mx(am[1], std::fabs(v * S[3][k]));
            }
        am[2] = std::fabs(p[0]);
        am[3] = std::fabs(p[1]);
        break;
    case ODP_DYN_TWODUBINS6D:
        for (int64_t k = 0; k < g->n[2]; ++k) {
            mx(am[0], std::fabs(p[0] * C[2][k]));
            mx(am[1], std::fabs(p[0] * S[2][k]));
        }
        for (int64_t k = 0; k < g->n[5]; ++k) {
            mx(am[3], std::fabs(p[2] * C[5][k]));
            mx(am[4], std::fabs(p[2] * S[5][k]));
        }
        am[2] = std::fabs(p[1]);
        am[5] = std::fabs(p[3]);
        break;
    case ODP_DYN_PE3D:
        // all inputs admissible (the bound of the box alphas)
        for (int64_t k = 0; k < g->n[2]; ++k) {
            for (int64_t j = 0; j < g->n[1]; ++j)
                mx(am[0], std::fabs(-p[0] + p[1] * C[2][k]) + p[2] * std::fabs(X[1][j]));
            for (int64_t i = 0; i < g->n[0]; ++i)
                mx(am[1], std::fabs(p[1] * S[2][k]) + p[2] * std::fabs(X[0][i]));
        }
        am[2] = p[2] + p[3];
        break;
    }
}

// The float64 schedule as the device's sched_kernel computes it: the step
// count (-1 beyond max_steps) and the output index each step lands on.
int64_t host_schedule(const PlanItem &it, const odp_solve_opts &o, std::vector<int32_t> &land) {
    double sum = 0.0;
    for (int d = 0; d < it.g->ndim; ++d) sum += it.amax[d] / it.g->dx[d];
    double dtc = o.cfl / sum;
    if (o.max_dt > 0.0 && dtc > o.max_dt) dtc = o.max_dt;
    const std::vector<double> &tau = it.tau;
    double t = tau[0];
    size_t k = 1;
    int64_t n = 0;
    land.clear();
    while (k < tau.size()) {
        if (n >= it.max_steps) return -1;
        double tn;
        int32_t l = -1;
        if (dtc >= tau[k] - t) {
            tn = tau[k];
            l = int32_t(k);
        } else {
            tn = t + dtc;
        }
        land.push_back(l);
        ++n;
        t = tn;
        if (l >= 0) ++k;
    }
    return n;
}

}  // namespace

// Planes per block for a requested c: chunks of (nearly) equal length; for
// the default choice also a multiple of 4, the marching kernel's register
// cycle, except for chunks under 4 planes in up to four dimensions (there
// the march ends at the chunk end).
static int balanced_chunk(const odp_grid *g, int c, bool cycle4) {
    const int n0 = int(g->n[0]);
    c = std::max(1, std::min(c, n0));
    const int nchunks = (n0 + c - 1) / c;
    int b = (n0 + nchunks - 1) / nchunks;
    // up to four dimensions runs of fewer than 4 planes stay as they are
    // (small grids: more blocks, and the march ends at the chunk end)
    if (cycle4 && g->ndim >= 2 && (b >= 4 || g->ndim >= 5)) b = std::min((b + 3) / 4 * 4, (n0 + 3) / 4 * 4);
    return b;
}

// Tiles of one hyperplane (tile_group).  Six-dimensional solves of the
// vector kernels (first order; second order with two or more points per
// thread) whose cubes of axes 3..5 waste under 5% of the lanes in their
// ragged last tile take brick tiles when axes 1 and 2 split into squares:
// their axis-1..3 neighbour loads then hit the L2 of the XCD that marches
// them (36^6 float32 first order: 17.0 -> 15.9 ms per step).  First order
// with the LDS plane exchange, a row pitch of at most 32 vec (each wave
// loads its own halo rows) and even squares takes the quad layout, which
// also reads one axis-1 and one axis-2 neighbour per point from another
// wave's LDS tile (lds = 2).  Everything else takes row-major tiles.
static void choose_tiling(PlanItem &it, int space_order) {
    const int64_t span = int64_t(kBlock) * it.vec;
    it.brick = 0;
    it.cube = 0;
    it.cube_tiles = 0;
    it.quad = 0;
    it.nqb = uint32_t((it.qpad + span - 1) / span);
    const odp_grid *g = it.g;
    if (g->ndim != 6 || it.dyn.id == ODP_DYN_PE3D) return;
    // second order: the vector kernel only (the point-per-lane kernel keeps
    // its own row-major mapping)
    if (space_order == 2 && (it.vec < 2 || it.dyn.id == ODP_DYN_SINGLE_INTEGRATOR)) return;
    const int64_t cube = it.qpad / (g->n[1] * g->n[2]);
    auto fits = [&](int64_t k, int64_t sp) {
        const int64_t ct = (cube + sp - 1) / sp;
        return g->n[1] % k == 0 && g->n[2] % k == 0 && ct * sp * 20 <= cube * 21;
    };
    if (space_order == 1 && it.lds == 1 && it.pitch <= 32 * int64_t(it.vec)) {
        const int64_t ws = 64 * int64_t(it.vec);
        for (int64_t k : {6, 4, 2}) {
            if (!fits(k, ws)) continue;
            const int64_t ct = (cube + ws - 1) / ws;
            it.brick = uint32_t(k);
            it.quad = 1;
            it.lds = 2;
            it.cube = uint32_t(cube);
            it.cube_tiles = uint32_t(ct);
            it.nqb = uint32_t((g->n[1] / 2) * (g->n[2] / 2) * ct);
            return;
        }
    }
    if (!fits(3, span)) return;
    const int64_t ct = (cube + span - 1) / span;
    it.brick = 3;
    it.cube = uint32_t(cube);
    it.cube_tiles = uint32_t(ct);
    it.nqb = uint32_t(g->n[1] * g->n[2] * ct);
}

std::vector<int> plan_build(Plan &p, std::vector<PlanItem> items, const odp_solve_opts &opts,
                            int tile_chunk, bool round4) {
    p.opts = opts;
    p.xcd_group = opts.xcd_group > 0 ? opts.xcd_group
                                     : (items.size() == 1 ? default_xcd_group(items[0].g) : 0);
    p.error.clear();
    const int prec = opts.precision;
    const size_t eb = prec == 32 ? 4 : 8;
    const int n = int(items.size());
    int64_t total = 0;
    for (auto &it : items) {
        if (it.rk_order <= 0) it.rk_order = opts.rk_order;
        const int64_t nl = it.g->n[it.g->ndim - 1];
        if (it.pitch <= 0 || it.g->ndim < 2) it.pitch = int(nl);
        it.qpad = it.g->ndim < 2 ? 1 : (it.g->npts / it.g->n[0] / nl) * it.pitch;
        it.ppad = it.qpad * it.g->n[0];
        it.vec = choose_vec(it.g, prec, it.dyn.id, it.pitch);
        it.lds = uses_lds(it.g->ndim, it.pitch, it.vec);
        if (it.dyn.id == ODP_DYN_PE3D || (opts.space_order == 2 && it.pitch != nl)) {
            it.vec = 1;  // point-per-lane kernel (pursuit-evasion; ENO2 on padded rows)
            it.lds = 0;
        } else if (opts.space_order == 2) {
            // ENO2: VEC points per thread; the LDS exchange needs two rows
            // of halo on each side within a block's range, and pays in 3D
            // and 4D (measured: 4D 80^4 float32 -5%; 6D 36^6 +5%)
            it.lds = it.g->ndim >= 3 && it.g->ndim <= 4 && it.vec >= 2 &&
                     4 * int64_t(it.pitch) <= int64_t(kBlock) * it.vec;
        }
        it.box_cfl = it.dyn.id == ODP_DYN_PE3D && !opts.dissipation;
        choose_tiling(it, opts.space_order);
        total += it.ppad;
    }
    std::map<AxisKey, std::vector<double>> tables;
    for (auto &it : items) {
        int c = tile_chunk;
        if (c <= 0) {
            if (items.size() == 1) {
                // brick tiles: every block marches the whole axis (on the
                // 36^6 float32 grid 36 planes beat 8 and 12 by 7-12%)
                c = it.brick ? int(it.g->n[0]) : default_chunk(it.g, it.vec, prec, opts.space_order);
            } else {
                // many solves share every launch: about 8192 blocks in all
                c = int(std::max<int64_t>(1, total / (int64_t(kBlock) * it.vec * 8192)));
            }
        }
        const bool exact = tile_chunk <= 0 && items.size() == 1 && !it.brick &&
                           default_chunk_exact(it.g, it.vec, prec, opts.space_order);
        // (the default is the tuner's candidate 0: taken as it is, too)
        it.chunk = balanced_chunk(it.g, c, tile_chunk <= 0 ? !exact : round4);
        it.tiles = uint32_t(int64_t(it.nqb) * ((it.g->n[0] + it.chunk - 1) / it.chunk));
        it.max_steps = step_capacity(it.g, &it.dyn, it.tau, opts.cfl, opts.max_dt);
        it.tab_entries = 0;
        for (int d = 0; d < it.g->ndim; ++d) it.tab_entries += 3 * int(it.g->n[d]);
        // the schedule on the host (box_cfl: the all-inputs count, a bound)
        make_tables(it.g, it.tab, tables);
        host_alpha_max(it, it.amax);
        it.nsteps = host_schedule(it, opts, it.land);
        if (it.nsteps < 0 && p.error.empty()) p.error = "schedule overflow (internal step bound exceeded)";
        if (it.nsteps >= it.max_steps) it.max_steps = it.nsteps + 1;  // box_cfl sentinel above the count
        if (it.box_cfl) it.land.assign(it.land.size(), -1);         // landings decided on the device
    }
    // group by kernel instantiation
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    auto key = [&](int i) {
        return std::make_tuple(items[i].dyn.id, items[i].g->ndim, items[i].vec, items[i].rk_order, items[i].lds);
    };
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key(a) < key(b); });
    p.items.clear();
    p.items.reserve(items.size());
    for (int i : perm) p.items.push_back(std::move(items[i]));
    p.groups.clear();
    for (int i = 0; i < n; ++i) {
        const PlanItem &it = p.items[i];
        if (p.groups.empty() || p.groups.back().dyn != it.dyn.id || p.groups.back().ndim != it.g->ndim ||
            p.groups.back().vec != it.vec || p.groups.back().rk != it.rk_order || p.groups.back().lds != it.lds) {
            PlanGroup gr;
            gr.dyn = it.dyn.id;
            gr.ndim = it.g->ndim;
            gr.vec = it.vec;
            gr.rk = it.rk_order;
            gr.lds = it.lds;
            gr.first = i;
            p.groups.push_back(gr);
        }
        p.groups.back().count++;
        p.groups.back().box_parts = std::max(p.groups.back().box_parts, box_parts(it.g));
    }
    // Batches: every group of several solves splits in two halves of about
    // equal work (contiguous descriptor ranges), and the groups go to two
    // lanes (the caller's stream and a second one, forked and joined around
    // the stepping), the larger first onto the lighter lane: one lane's
    // launch ramps and tails overlap the other's body.
    if (n > 1) {
        auto work = [&](int i) {
            const PlanItem &it = p.items[size_t(i)];
            return double(it.tiles) * double(it.nsteps) * double(it.rk_order);
        };
        std::vector<PlanGroup> split;
        for (const PlanGroup &gr : p.groups) {
            if (gr.count < 2) {
                split.push_back(gr);
                continue;
            }
            double tot = 0.0, acc = 0.0;
            for (int i = gr.first; i < gr.first + gr.count; ++i) tot += work(i);
            int k = 0;
            while (k < gr.count - 1 && (k == 0 || acc + 0.5 * work(gr.first + k) <= 0.5 * tot)) acc += work(gr.first + k++);
            PlanGroup a = gr, b = gr;
            a.count = k;
            b.first = gr.first + k;
            b.count = gr.count - k;
            for (PlanGroup *h : {&a, &b}) {
                h->box_parts = 1;
                for (int i = h->first; i < h->first + h->count; ++i)
                    h->box_parts = std::max(h->box_parts, box_parts(p.items[size_t(i)].g));
            }
            split.push_back(a);
            split.push_back(b);
        }
        p.groups = std::move(split);
        std::vector<double> gw(p.groups.size(), 0.0);
        std::vector<size_t> go(p.groups.size());
        for (size_t g = 0; g < p.groups.size(); ++g) {
            go[g] = g;
            for (int i = p.groups[g].first; i < p.groups[g].first + p.groups[g].count; ++i) gw[g] += work(i);
        }
        std::stable_sort(go.begin(), go.end(), [&](size_t a, size_t b) { return gw[a] > gw[b]; });
        double lw[2] = {0.0, 0.0};
        for (size_t g : go) {
            const int l = lw[1] < lw[0] ? 1 : 0;
            p.groups[g].lane = l;
            lw[l] += gw[g];
        }
    }
    // members by step count, descending, so that the solves still running at
    // step k are a prefix of each group's tile table
    p.max_nsteps = 0;
    p.total_tiles = 0;
    for (PlanGroup &gr : p.groups) {
        gr.order.resize(size_t(gr.count));
        std::iota(gr.order.begin(), gr.order.end(), gr.first);
        std::stable_sort(gr.order.begin(), gr.order.end(),
                         [&](int a, int b) { return p.items[size_t(a)].nsteps > p.items[size_t(b)].nsteps; });
        gr.tile_base = p.total_tiles;
        gr.prefix.assign(1, 0);
        for (int i : gr.order) {
            gr.prefix.push_back(gr.prefix.back() + p.items[size_t(i)].tiles);
            p.max_nsteps = std::max(p.max_nsteps, p.items[size_t(i)].nsteps);
        }
        p.total_tiles += gr.prefix.back();
    }
    // layout
    size_t off = 0;
    p.desc_off = off;
    off += align256(size_t(n) * sizeof(SolveDesc));
    p.nsteps_off = off;
    off += align256(size_t(n) * 8);
    p.state_begin = off;
    for (auto &it : p.items) {
        it.state_off = off;
        off += kStateBytes;
    }
    off = align256(off);
    p.aux_begin = off;
    for (auto &it : p.items) {
        it.aux_off = off;
        off += align256(size_t(it.tab_entries) * 8) + align256(it.tau.size() * 8);
    }
    p.tt_off = off;
    off += n > 1 ? align256(p.total_tiles * 4) * 2 : 0;
    p.upload_bytes = off;
    p.sched_begin = off;
    for (auto &it : p.items) {
        it.sched_off = off;
        off += align256(size_t(it.max_steps) * 8);
        it.land_off = off;
        off += align256(size_t(it.max_steps) * 4);
        if (it.dyn.id == ODP_DYN_PE3D) {
            it.box_off = off;
            off += align256(size_t(2 * kBoxSlots * 6 + kBoxStepWords) * 8);
        }
        if (it.box_cfl) {
            it.tk_off = off;
            off += align256(size_t(it.max_steps) * 8) + align256(size_t(it.max_steps) * 4);
        }
    }
    p.arr_begin = off;
    for (auto &it : p.items) {
        const size_t arr = align256(size_t(it.ppad) * eb);
        it.B_off = off;
        off += arr;
        it.C_off = off;
        off += it.rk_order == 3 ? arr : 0;
        if (it.pad_io) {
            it.V0p_off = off;
            off += arr;
            it.Ap_off = off;
            off += arr;
        }
    }
    p.total = off;
    return perm;
}

void plan_image(const Plan &p, unsigned char *base, std::vector<unsigned char> &img) {
    img.assign(p.upload_bytes, 0);
    const odp_solve_opts &o = p.opts;
    for (size_t i = 0; i < p.items.size(); ++i) {
        const PlanItem &it = p.items[i];
        const odp_grid *g = it.g;
        SolveDesc s;
        std::memset(&s, 0, sizeof(s));
        s.ndim = g->ndim;
        s.n0 = int32_t(g->n[0]);
        s.Q = uint32_t(it.qpad);
        s.s0 = int64_t(s.Q);
        s.npts = g->npts;
        s.pitch = it.pitch;
        s.lds = it.lds;
        int64_t st = 1;
        for (int d = g->ndim - 1; d >= 0; --d) {
            // the last axis occupies `pitch` elements per row in memory
            const int64_t ext = (d == g->ndim - 1 && d > 0) ? it.pitch : g->n[d];
            s.n[d] = int32_t(g->n[d]);
            s.stride[d] = d > 0 ? int32_t(st) : 0;
            s.div[d] = make_fastdiv(uint32_t(ext));
            s.dx[d] = g->dx[d];
            s.inv2dx[d] = 1.0 / (2.0 * g->dx[d]);
            if (g->periodic[d]) s.periodic |= 1u << d;
            st *= ext;
        }
        s.chunk = it.chunk;
        s.vec = it.vec;
        s.nqb = it.nqb;
        s.brick = it.brick;
        s.cube = it.cube;
        s.cube_tiles = it.cube_tiles;
        s.quad = it.quad;
        s.tiles = it.tiles;
        s.rk_order = it.rk_order;
        s.dyn = it.dyn.id;
        s.u_mode = it.dyn.u_mode;
        s.d_mode = it.dyn.d_mode;
        s.global_alpha = o.dissipation;
        for (int k = 0; k < 16; ++k) s.p[k] = it.dyn.p[k];
        s.A = it.pad_io ? base + it.Ap_off : it.A;
        s.B = base + it.B_off;
        s.C = it.rk_order == 3 ? base + it.C_off : nullptr;
        s.V0 = it.pad_io ? base + it.V0p_off : it.V0;
        s.Vinit = it.pad_io ? base + it.V0p_off : (it.Vinit ? it.Vinit : it.V0);
        s.Vsrc_dense = it.pad_io ? it.V0 : nullptr;
        s.Adst_dense = it.pad_io ? it.A : nullptr;
        unsigned char *state = base + it.state_off;
        s.amax = (double *)state;
        s.nsteps = (int64_t *)(state + kMaxDim * 8);
        s.step = (int64_t *)(state + kMaxDim * 8 + 8);
        s.flags = (int32_t *)(state + kMaxDim * 8 + 16);
        s.dtmm = (double *)(state + kMaxDim * 8 + 24);
        s.box = it.dyn.id == ODP_DYN_PE3D ? (uint64_t *)(base + it.box_off) : nullptr;
        const size_t tab_off = it.aux_off;
        const size_t tau_off = tab_off + align256(size_t(it.tab_entries) * 8);
        s.tabd = (const double *)(base + tab_off);
        s.dt_sched = (double *)(base + it.sched_off);
        s.land = (int32_t *)(base + it.land_off);
        // computation method (an obstacle method alone takes the first
        // comparison, with the obstacle array as its reference)
        const int m = o.mode, om = o.obstacle_mode;
        if (m != ODP_BRS) {
            s.tclamp = 1;
            s.tmax = m % 2 == 0;
            s.tvn = m == ODP_MIN_VINIT || m == ODP_MAX_VINIT;
            // (the value-over-time methods take V^n from registers; their
            // tref is only a valid address for the kernel's unused load)
            s.tref = m <= ODP_MAX_V0 ? s.V0 : (m >= ODP_MIN_TARGET ? o.target_dev : s.A);
            if (om != ODP_OBSTACLE_NONE) {
                s.obst = 1;
                s.omax = om == ODP_MAX_OBSTACLE;
                s.oref = o.obstacle_dev;
            }
        } else if (om != ODP_OBSTACLE_NONE) {
            s.tclamp = 1;
            s.tmax = om == ODP_MAX_OBSTACLE;
            s.tref = o.obstacle_dev;
        }
        if (o.set_slices > 1) {
            const bool tsliced = m >= ODP_MIN_TARGET || (m == ODP_BRS && om != ODP_OBSTACLE_NONE);
            s.tstride = tsliced ? g->npts : 0;
            s.ostride = s.obst ? g->npts : 0;
        }
        s.tref0 = s.tref;
        s.oref0 = s.oref;
        s.ntau = int32_t(it.tau.size());
        s.tau = (const double *)(base + tau_off);
        s.cfl = o.cfl;
        s.max_dt = o.max_dt;
        s.max_steps = it.max_steps;
        s.expect_steps = it.nsteps;
        s.box_cfl = it.box_cfl ? 1 : 0;
        if (it.box_cfl) {
            s.t_after = (double *)(base + it.tk_off);
            s.k_after = (int32_t *)(base + it.tk_off + align256(size_t(it.max_steps) * 8));
            // extremes over the heading table of the heading terms of f_x, f_y
            const int nt = int(g->n[2]);
            const double *th = it.tab.data() + 3 * size_t(g->n[0]) + 3 * size_t(g->n[1]);
            s.pe_cmin = s.pe_smin = INFINITY;
            s.pe_cmax = s.pe_smax = -INFINITY;
            for (int k = 0; k < nt; ++k) {
                const double c = -it.dyn.p[0] + it.dyn.p[1] * th[nt + k];
                const double sn = it.dyn.p[1] * th[2 * nt + k];
                s.pe_cmin = std::fmin(s.pe_cmin, c);
                s.pe_cmax = std::fmax(s.pe_cmax, c);
                s.pe_smin = std::fmin(s.pe_smin, sn);
                s.pe_smax = std::fmax(s.pe_smax, sn);
            }
        }
        for (int d = 0; d < g->ndim; ++d) {
            int toff = 0;
            for (int e = 0; e < d; ++e) toff += 3 * int(g->n[e]);
            s.tab[d].off = toff;
            s.tab[d].n = int32_t(g->n[d]);
        }
        std::memcpy(img.data() + tab_off, it.tab.data(), it.tab.size() * 8);
        std::memcpy(img.data() + p.desc_off + i * sizeof(SolveDesc), &s, sizeof(s));
        std::memcpy(img.data() + tau_off, it.tau.data(), it.tau.size() * 8);
    }
    // tile tables of a plan of several solves: per group, members in
    // descending step count
    if (p.items.size() > 1) {
        uint32_t *ts = (uint32_t *)(img.data() + p.tt_off);
        uint32_t *tl = ts + align256(p.total_tiles * 4) / 4;
        size_t e = 0;
        for (const PlanGroup &gr : p.groups)
            for (int i : gr.order)
                for (uint32_t k = 0; k < p.items[size_t(i)].tiles; ++k, ++e) {
                    ts[e] = uint32_t(i);
                    tl[e] = k;
                }
    }
}

int plan_prologue(Plan &p, unsigned char *base, hipStream_t st, bool pageable) {
    int rc;
    if (!p.error.empty()) return set_error(ODP_EHIP, p.error);
    std::vector<unsigned char> img;
    plan_image(p, base, img);
    const int n = int(p.items.size());
    const SolveDesc *descs = (const SolveDesc *)(base + p.desc_off);
    int64_t *nsteps_dev = (int64_t *)(base + p.nsteps_off);
    // pageable: a plain copy from host memory (performed synchronously by
    // the runtime), for callers that must not allocate pinned staging
    if (pageable) {
        if ((rc = check_hip(hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, st), "upload")))
            return rc;
    } else if ((rc = upload_async(base, img.data(), img.size(), st))) {
        return rc;
    }
    if ((rc = check_hip(launch_init(descs, n, st), "init"))) return rc;
    for (const PlanGroup &gr : p.groups) {
        int64_t qmax = 1;
        for (int i = gr.first; i < gr.first + gr.count; ++i)
            qmax = std::max<int64_t>(qmax, p.items[i].g->npts / p.items[i].g->n[0]);
        const int bps = int(std::max<int64_t>(1, std::min<int64_t>((qmax + kBlock - 1) / kBlock, 2048)));
        if ((rc = check_hip(launch_alpha(gr.dyn, gr.ndim, descs + gr.first, gr.count, bps, st), "alpha")))
            return rc;
    }
    if ((rc = check_hip(launch_sched(descs, n, nsteps_dev, st), "schedule"))) return rc;
    return ODP_OK;
}

int plan_launch_step(const Plan &p, unsigned char *base, hipStream_t st0, int64_t k, hipStream_t st2) {
    int rc;
    const int prec = p.opts.precision;
    const int mk = method_kind(p.opts);
    const SolveDesc *descs = (const SolveDesc *)(base + p.desc_off);
    const bool single = p.items.size() == 1;
    const uint32_t *tsd = single ? nullptr : (const uint32_t *)(base + p.tt_off);
    const uint32_t *tld = single ? nullptr : tsd + align256(p.total_tiles * 4) / 4;
    for (const PlanGroup &gr : p.groups) {
        hipStream_t st = gr.lane && st2 ? st2 : st0;
        // members with more than k steps form a prefix of gr.order
        size_t m = 0;
        while (m < gr.order.size() && p.items[size_t(gr.order[m])].nsteps > k) ++m;
        const uint32_t nb = gr.prefix[m];
        if (nb == 0) continue;
        const uint32_t *ts = tsd ? tsd + gr.tile_base : nullptr;
        const uint32_t *tl = tld ? tld + gr.tile_base : nullptr;
        for (int j = 0; j < gr.rk; ++j) {
            const int kind = stage_kind(gr.rk, j, mk, gr.lds, p.opts.space_order == 2);
            if (gr.dyn == ODP_DYN_PE3D && !p.opts.dissipation) {
                // Algorithm 1's costate box of this stage's input, then (first
                // stage) the step from the box, then the update
                if ((rc = check_hip(launch_stage(prec, gr.dyn, gr.ndim, gr.vec, kind | 32, descs, ts, tl, nb, j, 0,
                                                 k, p.xcd_group, st),
                                    "box")))
                    return rc;
                if (j == 0 &&
                    (rc = check_hip(launch_box_dt(descs + gr.first, nullptr, gr.count, gr.box_parts, 0, k, st), "box step")))
                    return rc;
            }
            if ((rc = check_hip(launch_stage(prec, gr.dyn, gr.ndim, gr.vec, kind, descs,
                                             ts, tl, nb, j, 0, k, p.xcd_group, st),
                                "stage")))
                return rc;
        }
    }
    return ODP_OK;
}

namespace {

struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// The second lane of batches: one stream per host thread and device (so
// that graph captures on different threads never share it), created on
// first use at the default priority and kept until the process ends.
hipStream_t lane_stream() {
    thread_local std::vector<hipStream_t> per_device;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return nullptr;
    if (per_device.size() <= size_t(dev)) per_device.resize(size_t(dev) + 1, nullptr);
    if (!per_device[size_t(dev)] &&
        hipStreamCreateWithFlags(&per_device[size_t(dev)], hipStreamNonBlocking) != hipSuccess)
        per_device[size_t(dev)] = nullptr;
    return per_device[size_t(dev)];
}

int plan_enqueue(const Plan &p, unsigned char *base, hipStream_t st, void *V_all) {
    int rc;
    const odp_solve_opts &o = p.opts;
    const int prec = o.precision;
    const SolveDesc *descs = (const SolveDesc *)(base + p.desc_off);
    const bool single = p.items.size() == 1;
    const uint32_t *tsd = single ? nullptr : (const uint32_t *)(base + p.tt_off);
    const uint32_t *tld = single ? nullptr : tsd + align256(p.total_tiles * 4) / 4;
    for (const PlanGroup &gr : p.groups) {
        const uint32_t *ts = tsd ? tsd + gr.tile_base : nullptr;
        const uint32_t *tl = tld ? tld + gr.tile_base : nullptr;
        if ((rc = check_hip(launch_start_copy(prec, descs, ts, tl, gr.prefix.back(), st), "start copy"))) return rc;
    }
    const PlanItem &it0 = p.items[0];
    const size_t bytes = single ? size_t(it0.g->npts) * (prec == 32 ? 4 : 8) : 0;
    // batches with a lane-1 group: the second lane starts after the start
    // copies and rejoins the caller's stream before the finish copies
    hipStream_t st2 = nullptr;
    Events lane_ev;
    for (const PlanGroup &gr : p.groups)
        if (gr.lane) st2 = lane_stream();
    if (st2 && ((rc = check_hip(hipEventCreateWithFlags(&lane_ev.a, hipEventDisableTiming), "event")) ||
                (rc = check_hip(hipEventCreateWithFlags(&lane_ev.b, hipEventDisableTiming), "event")) ||
                (rc = check_hip(hipEventRecord(lane_ev.a, st), "record")) ||
                (rc = check_hip(hipStreamWaitEvent(st2, lane_ev.a, 0), "wait"))))
        return rc;
    // time-varying sets (single solves): the steps after landing on tau[j]
    // compare with slice j; a box_cfl solve learns its landings on the device
    const bool sliced = single && o.set_slices > 1;
    for (int64_t k = 0; k < p.max_nsteps; ++k) {
        if (sliced) {
            if (it0.box_cfl) {
                if (k > 0 && (rc = check_hip(launch_box_slice(prec, (SolveDesc *)descs, k, st), "slice"))) return rc;
            } else if (k > 0 && it0.land[size_t(k - 1)] >= 0 &&
                       (rc = check_hip(launch_set_slice(prec, (SolveDesc *)descs, it0.land[size_t(k - 1)], st),
                                       "slice"))) {
                return rc;
            }
        }
        if ((rc = plan_launch_step(p, base, st, k, st2))) return rc;
        if (single && V_all) {
            if (it0.box_cfl) {
                if ((rc = check_hip(launch_box_save(prec, descs, k, V_all, it0.g->npts, st), "save"))) return rc;
            } else if (it0.land[size_t(k)] >= 0) {
                const void *outb =
                    (it0.rk_order == 1 && ((k + it0.nsteps) & 1) == 0) ? base + it0.B_off : it0.A;
                unsigned char *dst = (unsigned char *)V_all + size_t(it0.land[size_t(k)]) * bytes;
                if ((rc = check_hip(hipMemcpyAsync(dst, outb, bytes, hipMemcpyDeviceToDevice, st), "save")))
                    return rc;
            }
        }
    }
    if (st2 && ((rc = check_hip(hipEventRecord(lane_ev.b, st2), "record")) ||
                (rc = check_hip(hipStreamWaitEvent(st, lane_ev.b, 0), "wait"))))
        return rc;
    for (const PlanGroup &gr : p.groups) {
        const uint32_t *ts = tsd ? tsd + gr.tile_base : nullptr;
        const uint32_t *tl = tld ? tld + gr.tile_base : nullptr;
        bool pad = false, box = false;
        for (int i = gr.first; i < gr.first + gr.count; ++i) {
            pad = pad || p.items[size_t(i)].pad_io;
            box = box || p.items[size_t(i)].box_cfl;
        }
        // box_cfl: an odd first-order step count's result to A, landing check
        if (box && (rc = check_hip(launch_box_finish(prec, descs, ts, tl, gr.prefix.back(), st), "box finish")))
            return rc;
        // padded members: the result back to the caller's dense array
        if (pad && (rc = check_hip(launch_finish_copy(prec, descs, ts, tl, gr.prefix.back(), st), "finish copy")))
            return rc;
    }
    return ODP_OK;
}

// Instantiated graphs of recent plans, keyed by everything that decides
// their launches (workspace address, step counts, tiling, options, V_all):
// a repeated solve of the same shape on the same workspace replays its graph
// without recording or instantiating it again.  The stepping reads every
// per-call value (V0, V_out, tables, tau) from the descriptors, which the
// prologue uploads before each replay.
struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // after its last launch (eviction waits for it)
};

std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;  // most recent first
constexpr size_t kGraphCache = 16;

std::vector<int64_t> plan_key(const Plan &p, unsigned char *base, void *V_all) {
    std::vector<int64_t> k;
    auto put = [&](int64_t v) { k.push_back(v); };
    int dev = 0;
    (void)hipGetDevice(&dev);
    put(dev);
    put(int64_t(uintptr_t(base)));
    put(int64_t(uintptr_t(V_all)));
    const odp_solve_opts &o = p.opts;
    put(o.precision);
    put(o.mode);
    put(o.obstacle_mode);
    put(o.space_order);
    put(o.dissipation);
    put(o.set_slices);
    put(p.xcd_group);
    put(int64_t(p.total_tiles));
    put(p.max_nsteps);
    put(int64_t(p.desc_off));
    put(int64_t(p.tt_off));
    for (const PlanItem &it : p.items) {
        put(it.dyn.id);
        put(it.g->ndim);
        put(it.rk_order);
        put(it.vec);
        put(it.lds);
        put(it.chunk);
        put(int64_t(it.tiles));
        put(it.nsteps);
        put(it.pad_io);
        put(it.box_cfl);
        for (size_t o : {it.aux_off, it.sched_off, it.land_off, it.box_off, it.tk_off, it.B_off, it.C_off,
                         it.V0p_off, it.Ap_off})
            put(int64_t(o));
        put(int64_t(uintptr_t(it.A)));
        put(it.g->npts);
        for (int32_t l : it.land) put(l);
    }
    for (const PlanGroup &gr : p.groups) {
        put(int64_t(gr.tile_base));
        for (int i : gr.order) put(i);
    }
    return k;
}

}  // namespace

int plan_stats(const Plan &p, unsigned char *base, double kernel_ms, odp_solve_stats *stats, hipStream_t st) {
    int rc;
    const odp_solve_opts &o = p.opts;
    // one copy: every solve's state (alpha^max, step count, flags, dt range)
    std::vector<unsigned char> aux(p.aux_begin - p.state_begin);
    if ((rc = check_hip(hipMemcpyAsync(aux.data(), base + p.state_begin, aux.size(), hipMemcpyDeviceToHost, st),
                        "read state")) ||
        (rc = check_hip(hipStreamSynchronize(st), "sync")))
        return rc;
    int worst = ODP_OK;
    std::string why;
    for (size_t i = 0; i < p.items.size(); ++i) {
        const PlanItem &it = p.items[i];
        const unsigned char *state = aux.data() + (it.state_off - p.state_begin);
        odp_solve_stats &sx = stats[i];
        std::memset(&sx, 0, sizeof(sx));
        int64_t nst;
        std::memcpy(&nst, state + kMaxDim * 8, 8);
        int32_t flags;
        std::memcpy(&flags, state + kMaxDim * 8 + 16, 4);
        if ((flags & kFlagStepsExceeded) || nst <= 0 || nst > it.nsteps) {
            worst = ODP_EHIP;
            why = "device schedule longer than the steps enqueued";
            nst = std::max<int64_t>(0, std::min(nst, it.nsteps));
        }
        sx.steps = nst;
        if (nst > 0) {
            std::memcpy(&sx.dt_min, state + kMaxDim * 8 + 24, 8);
            std::memcpy(&sx.dt_max, state + kMaxDim * 8 + 32, 8);
        }
        sx.t_final = it.tau.back();
        sx.kernel_ms = kernel_ms;
        sx.alg_bytes = alg_bytes_per_step(o.precision, it.rk_order,
                                           method_arrays(o) + box_reads(it.dyn.id, o, it.rk_order), it.g->npts) * double(nst);
        sx.alg_gbps = kernel_ms > 0 ? sx.alg_bytes / (kernel_ms * 1e6) : 0.0;
        sx.roofline_frac = sx.alg_gbps / 8000.0;
        std::memcpy(sx.alpha_max, state, sizeof(sx.alpha_max));
        sx.nonfinite = flags & kFlagNonFinite;
        if (sx.nonfinite && worst == ODP_OK) {
            worst = ODP_ENONFINITE;
            why = "NaN or Inf in the value function";
        }
    }
    if (worst != ODP_OK) return set_error(worst, why);
    return ODP_OK;
}

// Launch-bound plans (small grids, many steps) are recorded into one HIP
// graph and replayed with a single launch.
bool plan_wants_graph(const Plan &p) {
    if (p.opts.graph == 2 || p.opts.stream == nullptr) return false;
    if (p.opts.graph == 1) return true;
    int64_t pts = 0;
    for (const auto &it : p.items) pts = std::max<int64_t>(pts, it.ppad);
    return pts <= (int64_t(1) << 22) && p.max_nsteps * int64_t(p.groups.size()) >= 8;
}

int plan_steps(Plan &p, unsigned char *base, hipStream_t st, void *V_all) {
    if (!plan_wants_graph(p)) return plan_enqueue(p, base, st, V_all);
    int rc;
    std::vector<int64_t> key = plan_key(p, base, V_all);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto e = g_graphs.begin(); e != g_graphs.end(); ++e) {
        if (e->key != key) continue;
        g_graphs.splice(g_graphs.begin(), g_graphs, e);
        GraphEntry &g = g_graphs.front();
        if ((rc = check_hip(hipGraphLaunch(g.exec, st), "graph launch"))) return rc;
        return check_hip(hipEventRecord(g.done, st), "record");
    }
    hipGraph_t graph = nullptr;
    GraphEntry ne;
    ne.key = std::move(key);
    if ((rc = check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture")))
        return rc;
    const int erc = plan_enqueue(p, base, st, V_all);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (erc) {
        if (graph) (void)hipGraphDestroy(graph);
        return erc;
    }
    if ((rc = check_hip(ec, "end capture"))) return rc;
    rc = check_hip(hipGraphInstantiate(&ne.exec, graph, nullptr, nullptr, 0), "instantiate");
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
    if ((rc = check_hip(hipEventCreateWithFlags(&ne.done, hipEventDisableTiming), "event"))) {
        (void)hipGraphExecDestroy(ne.exec);
        return rc;
    }
    if ((rc = check_hip(hipGraphLaunch(ne.exec, st), "graph launch")) ||
        (rc = check_hip(hipEventRecord(ne.done, st), "record"))) {
        (void)hipStreamSynchronize(st);
        (void)hipGraphExecDestroy(ne.exec);
        (void)hipEventDestroy(ne.done);
        return rc;
    }
    g_graphs.push_front(std::move(ne));
    while (g_graphs.size() > kGraphCache) {
        GraphEntry &old = g_graphs.back();
        (void)hipEventSynchronize(old.done);  // its last replay has finished
        (void)hipGraphExecDestroy(old.exec);
        (void)hipEventDestroy(old.done);
        g_graphs.pop_back();
    }
    return ODP_OK;
}

}  // namespace odp
