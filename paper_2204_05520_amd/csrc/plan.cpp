// Plans: layout, host image, prologue (alpha^max + float64 schedules on the
// device), lockstep stepping and statistics for a list of solves.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>

namespace odp {

namespace {

constexpr size_t kStateBytes = 256;  // alpha^max[6], nsteps, step, flags

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

// Planes per block for a requested c: chunks of (nearly) equal length; for
// the default choice also a multiple of 4, the marching kernel's register
// cycle, except for chunks under 4 planes in up to four dimensions (there
// the march ends at the chunk end).
int balanced_chunk(const odp_grid *g, int c, bool cycle4) {
    const int n0 = int(g->n[0]);
    c = std::max(1, std::min(c, n0));
    const int nchunks = (n0 + c - 1) / c;
    int b = (n0 + nchunks - 1) / nchunks;
    // up to four dimensions runs of fewer than 4 planes stay as they are
    // (small grids: more blocks, and the march ends at the chunk end)
    if (cycle4 && g->ndim >= 2 && (b >= 4 || g->ndim >= 5)) b = std::min((b + 3) / 4 * 4, (n0 + 3) / 4 * 4);
    return b;
}

}  // namespace

std::vector<int> plan_build(Plan &p, std::vector<PlanItem> items, const odp_solve_opts &opts,
                            int tile_chunk, bool round4) {
    p.opts = opts;
    p.xcd_group = opts.xcd_group > 0 ? opts.xcd_group
                                     : (items.size() == 1 ? default_xcd_group(items[0].g) : 0);
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
        total += it.ppad;
    }
    for (auto &it : items) {
        int c = tile_chunk;
        if (c <= 0) {
            if (items.size() == 1) {
                c = default_chunk(it.g, it.vec, prec);
            } else {
                // many solves share every launch: about 8192 blocks in all
                c = int(std::max<int64_t>(1, total / (int64_t(kBlock) * it.vec * 8192)));
            }
        }
        it.chunk = balanced_chunk(it.g, c, tile_chunk <= 0 || round4);
        it.tiles = solve_tiles(it.g->n[0], it.qpad, it.chunk, it.vec);
        it.max_steps = step_capacity(it.g, &it.dyn, it.tau, opts.cfl, opts.max_dt);
        it.tab_entries = 0;
        for (int d = 0; d < it.g->ndim; ++d) it.tab_entries += 3 * int(it.g->n[d]);
    }
    // group by kernel instantiation
    std::vector<int> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    auto key = [&](int i) {
        return std::make_tuple(items[i].dyn.id, items[i].g->ndim, items[i].vec, items[i].rk_order, items[i].lds);
    };
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key(a) < key(b); });
    p.items.clear();
    for (int i : perm) p.items.push_back(items[i]);
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
    }
    // layout
    size_t off = 0;
    p.desc_off = off;
    off += align256(size_t(n) * sizeof(SolveDesc));
    p.nsteps_off = off;
    off += align256(size_t(n) * 8);
    p.aux_begin = off;
    for (auto &it : p.items) {
        it.aux_off = off;
        off += kStateBytes + align256(size_t(it.tab_entries) * 8) + align256(it.tau.size() * 8);
    }
    p.upload_bytes = off;
    p.total_tiles = 0;
    for (auto &it : p.items) p.total_tiles += it.tiles;
    p.tt_off = off;
    off += align256(p.total_tiles * 4) * 2;
    p.sched_begin = off;
    for (auto &it : p.items) {
        it.sched_off = off;
        off += align256(size_t(it.max_steps) * 8);
        it.land_off = off;
        off += align256(size_t(it.max_steps) * 4);
        if (it.dyn.id == ODP_DYN_PE3D) {
            it.box_off = off;
            off += align256(size_t(2 * kBoxSlots * 6) * 8);
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
        s.nqb = uint32_t((int64_t(s.Q) + int64_t(kBlock) * it.vec - 1) / (int64_t(kBlock) * it.vec));
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
        unsigned char *state = base + it.aux_off;
        s.amax = (double *)state;
        s.nsteps = (int64_t *)(state + kMaxDim * 8);
        s.step = (int64_t *)(state + kMaxDim * 8 + 8);
        s.flags = (int32_t *)(state + kMaxDim * 8 + 16);
        s.box = it.dyn.id == ODP_DYN_PE3D ? (uint64_t *)(base + it.box_off) : nullptr;
        const size_t tab_off = it.aux_off + kStateBytes;
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
        // axis tables: coordinate, cos, sin (float64, computed once on the host)
        double *tab = (double *)(img.data() + tab_off);
        int toff = 0;
        for (int d = 0; d < g->ndim; ++d) {
            const int nd = int(g->n[d]);
            s.tab[d].off = toff;
            s.tab[d].n = nd;
            for (int k = 0; k < nd; ++k) {
                const double x = g->lo[d] + double(k) * g->dx[d];
                tab[toff + k] = x;
                tab[toff + nd + k] = std::cos(x);
                tab[toff + 2 * nd + k] = std::sin(x);
            }
            toff += 3 * nd;
        }
        std::memcpy(img.data() + p.desc_off + i * sizeof(SolveDesc), &s, sizeof(s));
        std::memcpy(img.data() + tau_off, it.tau.data(), it.tau.size() * 8);
    }
}

int plan_prologue(Plan &p, unsigned char *base, hipStream_t st) {
    int rc;
    std::vector<unsigned char> img;
    plan_image(p, base, img);
    const int n = int(p.items.size());
    const SolveDesc *descs = (const SolveDesc *)(base + p.desc_off);
    int64_t *nsteps_dev = (int64_t *)(base + p.nsteps_off);
    if ((rc = check_hip(hipMemcpyAsync(base, img.data(), img.size(), hipMemcpyHostToDevice, st), "upload")))
        return rc;
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
    std::vector<int64_t> nst(size_t(n), 0);
    if ((rc = check_hip(hipMemcpyAsync(nst.data(), nsteps_dev, size_t(n) * 8, hipMemcpyDeviceToHost, st),
                        "read steps")))
        return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "sync"))) return rc;
    p.max_nsteps = 0;
    for (int i = 0; i < n; ++i) {
        if (nst[size_t(i)] <= 0) return set_error(ODP_EHIP, "schedule overflow (internal step bound exceeded)");
        p.items[size_t(i)].nsteps = nst[size_t(i)];
        p.max_nsteps = std::max(p.max_nsteps, nst[size_t(i)]);
    }
    // tile tables: per group, members by step count (descending), so that
    // the solves still running at step k are a prefix
    std::vector<uint32_t> ts, tl;
    ts.reserve(p.total_tiles);
    tl.reserve(p.total_tiles);
    for (PlanGroup &gr : p.groups) {
        gr.order.resize(size_t(gr.count));
        std::iota(gr.order.begin(), gr.order.end(), gr.first);
        std::stable_sort(gr.order.begin(), gr.order.end(),
                         [&](int a, int b) { return p.items[size_t(a)].nsteps > p.items[size_t(b)].nsteps; });
        gr.tile_base = ts.size();
        gr.prefix.assign(1, 0);
        for (int i : gr.order) {
            const uint32_t t = p.items[size_t(i)].tiles;
            for (uint32_t k = 0; k < t; ++k) {
                ts.push_back(uint32_t(i));
                tl.push_back(k);
            }
            gr.prefix.push_back(gr.prefix.back() + t);
        }
    }
    if (n > 1) {
        uint32_t *tsd = (uint32_t *)(base + p.tt_off);
        uint32_t *tld = tsd + align256(p.total_tiles * 4) / 4;
        if ((rc = check_hip(hipMemcpyAsync(tsd, ts.data(), ts.size() * 4, hipMemcpyHostToDevice, st), "tiles")) ||
            (rc = check_hip(hipMemcpyAsync(tld, tl.data(), tl.size() * 4, hipMemcpyHostToDevice, st), "tiles")))
            return rc;
        // the host vectors must outlive the copies
        if ((rc = check_hip(hipStreamSynchronize(st), "sync"))) return rc;
    }
    return ODP_OK;
}

int plan_launch_step(const Plan &p, unsigned char *base, hipStream_t st, int64_t k) {
    int rc;
    const int prec = p.opts.precision;
    const int mk = method_kind(p.opts);
    const SolveDesc *descs = (const SolveDesc *)(base + p.desc_off);
    const bool single = p.items.size() == 1;
    const uint32_t *tsd = single ? nullptr : (const uint32_t *)(base + p.tt_off);
    const uint32_t *tld = single ? nullptr : tsd + align256(p.total_tiles * 4) / 4;
    for (const PlanGroup &gr : p.groups) {
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
                // Algorithm 1's costate box of this stage's input, then the update
                if ((rc = check_hip(launch_stage(prec, gr.dyn, gr.ndim, gr.vec, kind | 32, descs, ts, tl, nb, j, 0,
                                                 k, p.xcd_group, st),
                                    "box")))
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

static int plan_enqueue(Plan &p, unsigned char *base, hipStream_t st, const std::vector<int32_t> *land,
                        void *V_all) {
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
    const size_t bytes = single ? size_t(p.items[0].g->npts) * (prec == 32 ? 4 : 8) : 0;
    // time-varying sets (single solves): the steps after landing on tau[j]
    // compare with slice j
    const bool sliced = single && o.set_slices > 1 && land;
    for (int64_t k = 0; k < p.max_nsteps; ++k) {
        if (sliced && k > 0 && (*land)[size_t(k - 1)] >= 0 &&
            (rc = check_hip(launch_set_slice(prec, (SolveDesc *)descs, (*land)[size_t(k - 1)], st), "slice")))
            return rc;
        if ((rc = plan_launch_step(p, base, st, k))) return rc;
        if (land && V_all && (*land)[size_t(k)] >= 0) {
            const PlanItem &it = p.items[0];
            const void *outb = (it.rk_order == 1 && ((k + it.nsteps) & 1) == 0) ? base + it.B_off : it.A;
            unsigned char *dst = (unsigned char *)V_all + size_t((*land)[size_t(k)]) * bytes;
            if ((rc = check_hip(hipMemcpyAsync(dst, outb, bytes, hipMemcpyDeviceToDevice, st), "save"))) return rc;
        }
    }
    // padded members: the result back to the caller's dense array
    for (const PlanGroup &gr : p.groups) {
        bool any = false;
        for (int i = gr.first; i < gr.first + gr.count; ++i) any = any || p.items[size_t(i)].pad_io;
        if (!any) continue;
        const uint32_t *ts = tsd ? tsd + gr.tile_base : nullptr;
        const uint32_t *tl = tld ? tld + gr.tile_base : nullptr;
        if ((rc = check_hip(launch_finish_copy(prec, descs, ts, tl, gr.prefix.back(), st), "finish copy")))
            return rc;
    }
    return ODP_OK;
}

int plan_stats(const Plan &p, unsigned char *base, double kernel_ms, odp_solve_stats *stats) {
    int rc;
    const odp_solve_opts &o = p.opts;
    // two bulk copies: every solve's state/tables/tau, every schedule
    std::vector<unsigned char> aux(p.upload_bytes - p.aux_begin), sched(p.arr_begin - p.sched_begin);
    if ((rc = check_hip(hipMemcpy(aux.data(), base + p.aux_begin, aux.size(), hipMemcpyDeviceToHost), "read state")) ||
        (rc = check_hip(hipMemcpy(sched.data(), base + p.sched_begin, sched.size(), hipMemcpyDeviceToHost),
                        "read schedules")))
        return rc;
    int worst = ODP_OK;
    for (size_t i = 0; i < p.items.size(); ++i) {
        const PlanItem &it = p.items[i];
        const unsigned char *state = aux.data() + (it.aux_off - p.aux_begin);
        const double *dts = (const double *)(sched.data() + (it.sched_off - p.sched_begin));
        odp_solve_stats &sx = stats[i];
        std::memset(&sx, 0, sizeof(sx));
        sx.steps = it.nsteps;
        sx.dt_min = *std::min_element(dts, dts + it.nsteps);
        sx.dt_max = *std::max_element(dts, dts + it.nsteps);
        sx.t_final = it.tau.back();
        sx.kernel_ms = kernel_ms;
        sx.alg_bytes = alg_bytes_per_step(o.precision, it.rk_order,
                                           method_arrays(o) + box_reads(it.dyn.id, o, it.rk_order), it.g->npts) * double(it.nsteps);
        sx.alg_gbps = kernel_ms > 0 ? sx.alg_bytes / (kernel_ms * 1e6) : 0.0;
        sx.roofline_frac = sx.alg_gbps / 8000.0;
        std::memcpy(sx.alpha_max, state, sizeof(sx.alpha_max));
        int32_t flags;
        std::memcpy(&flags, state + kMaxDim * 8 + 16, 4);
        sx.nonfinite = flags & 1;
        if (sx.nonfinite) worst = ODP_ENONFINITE;
    }
    if (worst != ODP_OK) return set_error(worst, "NaN or Inf in the value function");
    return ODP_OK;
}

}  // namespace odp

namespace odp {

// Launch-bound plans (small grids, many steps) are recorded into one HIP
// graph and replayed with a single launch; the call then waits for the
// graph to finish before it frees the executable graph.
bool plan_wants_graph(const Plan &p) {
    if (p.opts.graph == 2 || p.opts.stream == nullptr) return false;
    if (p.opts.graph == 1) return true;
    int64_t pts = 0;
    for (const auto &it : p.items) pts = std::max<int64_t>(pts, it.ppad);
    return pts <= (int64_t(1) << 22) && p.max_nsteps * int64_t(p.groups.size()) >= 8;
}

int plan_steps(Plan &p, unsigned char *base, hipStream_t st, const std::vector<int32_t> *land,
               void *V_all) {
    if (!plan_wants_graph(p)) return plan_enqueue(p, base, st, land, V_all);
    int rc;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if ((rc = check_hip(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "begin capture")))
        return rc;
    const int erc = plan_enqueue(p, base, st, land, V_all);
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (erc) {
        if (graph) (void)hipGraphDestroy(graph);
        return erc;
    }
    if ((rc = check_hip(ec, "end capture"))) return rc;
    rc = check_hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
    (void)hipGraphDestroy(graph);
    if (rc) return rc;
    rc = check_hip(hipGraphLaunch(exec, st), "graph launch");
    if (!rc) rc = check_hip(hipStreamSynchronize(st), "sync");
    (void)hipGraphExecDestroy(exec);
    return rc;
}

}  // namespace odp
