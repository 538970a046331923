// odp_hj_solve and odp_hj_batch: a plan of one solve, or of many solves
// stepped in lockstep (launch k covers every solve that still has a step k,
// so each solve's tiles spread over the whole GPU and launch boundaries
// order the steps).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "plan.h"
#include "tune.h"
#include "runtime.h"

using namespace odp;

namespace {

struct DeviceBuffer {
    void *ptr = nullptr;
    hipStream_t st = nullptr;
    bool owned = false;
    ~DeviceBuffer() {
        if (owned && ptr) (void)hipFreeAsync(ptr, st);
    }
};

int alloc_workspace(DeviceBuffer &buf, void *given, size_t given_bytes, size_t bytes, hipStream_t st) {
    buf.st = st;
    if (given) {
        if ((uintptr_t(given) & 255u) != 0) return set_error(ODP_EINVAL, "workspace must be 256-byte aligned");
        if (given_bytes < bytes)
            return set_error(ODP_ENOMEM, "workspace too small: " + std::to_string(bytes) + " bytes needed");
        buf.ptr = given;
        return ODP_OK;
    }
    hipError_t e = hipMallocAsync(&buf.ptr, bytes, st);
    if (e != hipSuccess) {
        buf.ptr = nullptr;
        return set_error(ODP_ENOMEM, std::string("device allocation failed: ") + hipGetErrorString(e));
    }
    buf.owned = true;
    return ODP_OK;
}

PlanItem make_item(const odp_grid *g, const odp_dynamics *dyn, const void *V0, const void *Vinit,
                   const double *tau, int ntau, void *A) {
    PlanItem it;
    it.g = g;
    it.dyn = *dyn;
    it.V0 = V0;
    it.Vinit = Vinit;
    it.A = A;
    it.tau.assign(tau, tau + ntau);
    return it;
}

struct Timer {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Timer() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    }
};

}  // namespace

extern "C" {

size_t odp_hj_workspace_bytes(const odp_grid *grid, const odp_dynamics *dyn, const double *tau,
                              int ntau, const odp_solve_opts *opts) {
    if (!grid || validate_opts(opts) != ODP_OK || validate_dyn(grid, dyn) != ODP_OK ||
        validate_tau(tau, ntau) != ODP_OK)
        return 0;
    Plan p;
    std::vector<PlanItem> items{make_item(grid, dyn, nullptr, nullptr, tau, ntau, nullptr)};
    if (opts->tile_chunk == ODP_TILE_AUTOTUNE) return tune_workspace_bytes(items, *opts);
    plan_build(p, std::move(items), *opts, opts->tile_chunk);
    return p.total;
}

int odp_hj_solve(const odp_grid *grid, const odp_dynamics *dyn, const void *V0_dev,
                 const void *V_init_dev, const double *tau, int ntau, const odp_solve_opts *opts,
                 void *workspace_dev, void *V_out_dev, void *V_all_dev, odp_solve_stats *stats) {
    if (!grid) return set_error(ODP_EINVAL, "grid is NULL");
    int rc;
    if ((rc = validate_opts(opts)) || (rc = validate_dyn(grid, dyn)) || (rc = validate_tau(tau, ntau)))
        return rc;
    if (!V0_dev || !V_out_dev) return set_error(ODP_EINVAL, "V0 and V_out are required");
    if (V_out_dev == V0_dev || V_out_dev == V_init_dev)
        return set_error(ODP_EINVAL, "V_out may not alias V0 or V_init");
    if (V_out_dev == opts->target_dev || V_out_dev == opts->obstacle_dev)
        return set_error(ODP_EINVAL, "V_out may not alias the target or obstacle array");
    if (opts->set_slices > 1 && opts->set_slices != ntau)
        return set_error(ODP_EINVAL, "set_slices must be 0, 1 or ntau");
    if (opts->save_all && !V_all_dev) return set_error(ODP_EINVAL, "save_all needs V_all");
    hipStream_t st = (hipStream_t)opts->stream;

    Plan p;
    std::vector<PlanItem> items{make_item(grid, dyn, V0_dev, V_init_dev, tau, ntau, V_out_dev)};
    DeviceBuffer ws;
    unsigned char *base = nullptr;
    int chunk = opts->tile_chunk;
    if (chunk == ODP_TILE_AUTOTUNE && tune_cached(items, *opts, &chunk)) {
        plan_build(p, std::move(items), *opts, chunk, true);
        if ((rc = alloc_workspace(ws, workspace_dev, SIZE_MAX, p.total, st))) return rc;
        base = (unsigned char *)ws.ptr;
    } else if (chunk == ODP_TILE_AUTOTUNE) {
        if ((rc = alloc_workspace(ws, workspace_dev, SIZE_MAX, tune_workspace_bytes(items, *opts), st))) return rc;
        base = (unsigned char *)ws.ptr;
        if ((rc = tune_tile_chunk(items, *opts, base, st, &chunk))) return rc;
        plan_build(p, std::move(items), *opts, chunk, true);
    } else {
        plan_build(p, std::move(items), *opts, chunk);
        if ((rc = alloc_workspace(ws, workspace_dev, SIZE_MAX, p.total, st))) return rc;
        base = (unsigned char *)ws.ptr;
    }
    if ((rc = plan_prologue(p, base, st))) return rc;

    if (opts->save_all) {
        const size_t bytes = size_t(grid->npts) * (opts->precision == 32 ? 4 : 8);
        const void *src = V_init_dev ? V_init_dev : V0_dev;
        if ((rc = check_hip(hipMemcpyAsync(V_all_dev, src, bytes, hipMemcpyDeviceToDevice, st), "save start")))
            return rc;
    }
    Timer tm;
    if (stats) {
        if ((rc = check_hip(hipEventCreate(&tm.e0), "event")) || (rc = check_hip(hipEventCreate(&tm.e1), "event")))
            return rc;
        (void)hipEventRecord(tm.e0, st);
    }
    if ((rc = plan_steps(p, base, st, opts->save_all ? V_all_dev : nullptr)))
        return rc;
    if (stats) {
        (void)hipEventRecord(tm.e1, st);
        if ((rc = check_hip(hipEventSynchronize(tm.e1), "sync"))) return rc;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        return plan_stats(p, base, ms, stats, st);
    }
    return ODP_OK;
}

static int batch_items(int nsolves, const odp_solve_desc *descs, const odp_solve_opts *common,
                       std::vector<PlanItem> &items) {
    int rc;
    if (nsolves < 1 || !descs) return set_error(ODP_EINVAL, "empty batch");
    if ((rc = validate_opts(common))) return rc;
    if (common->save_all) return set_error(ODP_EUNSUPPORTED, "save_all is not available for batches");
    if (common->target_dev || common->obstacle_dev)
        return set_error(ODP_EUNSUPPORTED, "target and obstacle arrays belong to one grid: use odp_hj_solve");
    items.clear();
    for (int i = 0; i < nsolves; ++i) {
        const odp_solve_desc &d = descs[i];
        if (!d.grid) return set_error(ODP_EINVAL, "batch entry " + std::to_string(i) + ": grid is NULL");
        if ((rc = validate_dyn(d.grid, &d.dyn)) || (rc = validate_tau(d.tau, d.ntau))) {
            const std::string why = odp_last_error();
            return set_error(rc, "batch entry " + std::to_string(i) + ": " + why);
        }
        if (!d.V0_dev || !d.V_out_dev || d.V0_dev == d.V_out_dev)
            return set_error(ODP_EINVAL, "batch entry " + std::to_string(i) + ": bad V0 / V_out");
        if (d.rk_order < 0 || d.rk_order > 3)
            return set_error(ODP_EINVAL, "batch entry " + std::to_string(i) + ": rk_order must be 0..3");
        items.push_back(make_item(d.grid, &d.dyn, d.V0_dev, nullptr, d.tau, d.ntau, d.V_out_dev));
        items.back().rk_order = d.rk_order;
        // rows that are not a whole number of 16-byte vectors: the plan works
        // on padded copies, so that every member runs the widest kernel
        const int64_t nl = d.grid->n[d.grid->ndim - 1];
        const int64_t w = common->precision == 32 ? 4 : 2;
        if (d.grid->ndim >= 2 && d.dyn.id != ODP_DYN_SINGLE_INTEGRATOR && nl % w != 0 &&
            common->space_order != 2) {
            items.back().pitch = int((nl + w - 1) / w * w);
            items.back().pad_io = true;
        }
    }
    return ODP_OK;
}

size_t odp_hj_batch_workspace_bytes(int nsolves, const odp_solve_desc *descs, const odp_solve_opts *common) {
    std::vector<PlanItem> items;
    if (batch_items(nsolves, descs, common, items) != ODP_OK) return 0;
    if (common->tile_chunk == ODP_TILE_AUTOTUNE) return tune_workspace_bytes(items, *common);
    Plan p;
    plan_build(p, std::move(items), *common, common->tile_chunk);
    return p.total;
}

int odp_hj_batch(int nsolves, const odp_solve_desc *descs, const odp_solve_opts *common,
                 void *workspace_dev, size_t workspace_bytes, odp_solve_stats *stats_per_solve) {
    int rc;
    std::vector<PlanItem> items;
    if ((rc = batch_items(nsolves, descs, common, items))) return rc;
    hipStream_t st = (hipStream_t)common->stream;
    Plan p;
    DeviceBuffer ws;
    unsigned char *base = nullptr;
    std::vector<int> perm;
    int chunk = common->tile_chunk;
    if (chunk == ODP_TILE_AUTOTUNE && tune_cached(items, *common, &chunk)) {
        perm = plan_build(p, std::move(items), *common, chunk, true);
        if ((rc = alloc_workspace(ws, workspace_dev, workspace_bytes, p.total, st))) return rc;
        base = (unsigned char *)ws.ptr;
    } else if (chunk == ODP_TILE_AUTOTUNE) {
        if ((rc = alloc_workspace(ws, workspace_dev, workspace_bytes, tune_workspace_bytes(items, *common), st)))
            return rc;
        base = (unsigned char *)ws.ptr;
        if ((rc = tune_tile_chunk(items, *common, base, st, &chunk))) return rc;
        perm = plan_build(p, std::move(items), *common, chunk, true);
    } else {
        perm = plan_build(p, std::move(items), *common, chunk);
        if ((rc = alloc_workspace(ws, workspace_dev, workspace_bytes, p.total, st))) return rc;
        base = (unsigned char *)ws.ptr;
    }
    if ((rc = plan_prologue(p, base, st))) return rc;
    Timer tm;
    if (stats_per_solve) {
        if ((rc = check_hip(hipEventCreate(&tm.e0), "event")) || (rc = check_hip(hipEventCreate(&tm.e1), "event")))
            return rc;
        (void)hipEventRecord(tm.e0, st);
    }
    if ((rc = plan_steps(p, base, st, nullptr))) return rc;
    if (stats_per_solve) {
        (void)hipEventRecord(tm.e1, st);
        if ((rc = check_hip(hipEventSynchronize(tm.e1), "sync"))) return rc;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        std::vector<odp_solve_stats> sorted(p.items.size());
        rc = plan_stats(p, base, ms, sorted.data(), st);
        for (size_t i = 0; i < perm.size(); ++i) stats_per_solve[perm[i]] = sorted[i];
        if (rc) return rc;
    }
    return ODP_OK;
}

size_t odp_ttr_workspace_bytes(const odp_grid *grid, const odp_ttr_opts *opts) {
    if (!grid || !opts || (opts->precision != 32 && opts->precision != 64)) return 0;
    size_t tab = 0;
    for (int d = 0; d < grid->ndim; ++d) tab += 3 * size_t(grid->n[d]);
    const size_t eb = opts->precision == 32 ? 4 : 8;
    const int K = opts->check_every > 0 ? opts->check_every : 32;
    return align256(sizeof(SolveDesc)) + align256(tab * 8) + align256(size_t(K) * kBoxSlots * 8) +
           align256(size_t(grid->npts) * eb);
}

int odp_ttr_solve(const odp_grid *grid, const odp_dynamics *dyn, const void *target_dev,
                  const odp_ttr_opts *opts, void *workspace_dev, size_t workspace_bytes,
                  void *phi_out_dev, odp_ttr_stats *stats) {
    int rc;
    if (!grid) return set_error(ODP_EINVAL, "grid is NULL");
    if (!opts) return set_error(ODP_EINVAL, "opts is NULL");
    if ((rc = validate_dyn(grid, dyn))) return rc;
    if (dyn->id == ODP_DYN_PE3D)
        return set_error(ODP_EUNSUPPORTED, "time to reach: the pursuit-evasion model is not available");
    if (opts->precision != 32 && opts->precision != 64) return set_error(ODP_EINVAL, "precision must be 32 or 64");
    if (!(opts->eps > 0.0) || !std::isfinite(opts->eps)) return set_error(ODP_EINVAL, "eps must be > 0");
    if (opts->max_iters < 1) return set_error(ODP_EINVAL, "max_iters must be >= 1");
    if (opts->check_every < 0) return set_error(ODP_EINVAL, "check_every must be >= 0");
    if (!(opts->big >= 0.0) || !std::isfinite(opts->big)) return set_error(ODP_EINVAL, "big must be >= 0");
    if (!target_dev || !phi_out_dev || target_dev == phi_out_dev)
        return set_error(ODP_EINVAL, "target and phi_out are required and may not alias");
    if (grid->n[0] > 65535) return set_error(ODP_EUNSUPPORTED, "axis 0 longer than 65535 nodes");
    hipStream_t st = (hipStream_t)opts->stream;
    const int prec = opts->precision;
    const size_t eb = prec == 32 ? 4 : 8;
    const int K = opts->check_every > 0 ? opts->check_every : 32;
    const double big = opts->big > 0.0 ? opts->big : 1e4;
    const int N = grid->ndim;
    const int64_t n0 = grid->n[0];
    const int64_t Q = grid->npts / n0;

    // descriptor: grid, tables and dynamics (what the kernel reads)
    SolveDesc s;
    std::memset(&s, 0, sizeof(s));
    s.ndim = N;
    s.n0 = int32_t(n0);
    s.Q = uint32_t(Q);
    s.s0 = Q;
    s.npts = grid->npts;
    s.pitch = int32_t(grid->n[N - 1]);
    int64_t stv = 1;
    for (int d = N - 1; d >= 0; --d) {
        s.n[d] = int32_t(grid->n[d]);
        s.stride[d] = d > 0 ? int32_t(stv) : 0;
        s.div[d] = make_fastdiv(uint32_t(grid->n[d]));
        s.dx[d] = grid->dx[d];
        s.inv2dx[d] = 1.0 / (2.0 * grid->dx[d]);
        if (grid->periodic[d]) s.periodic |= 1u << d;
        stv *= grid->n[d];
    }
    s.dyn = dyn->id;
    s.u_mode = dyn->u_mode;
    s.d_mode = dyn->d_mode;
    for (int k = 0; k < 16; ++k) s.p[k] = dyn->p[k];
    std::vector<double> tab;
    for (int d = 0; d < N; ++d) {
        const int nd = int(grid->n[d]);
        s.tab[d].off = int32_t(tab.size());
        s.tab[d].n = nd;
        for (int k = 0; k < nd; ++k) tab.push_back(grid->lo[d] + double(k) * grid->dx[d]);
        for (int k = 0; k < nd; ++k) tab.push_back(std::cos(grid->lo[d] + double(k) * grid->dx[d]));
        for (int k = 0; k < nd; ++k) tab.push_back(std::sin(grid->lo[d] + double(k) * grid->dx[d]));
    }

    const size_t need = odp_ttr_workspace_bytes(grid, opts);
    DeviceBuffer ws;
    if ((rc = alloc_workspace(ws, workspace_dev, workspace_bytes, need, st))) return rc;
    unsigned char *base = (unsigned char *)ws.ptr;
    const size_t tab_off = align256(sizeof(SolveDesc));
    const size_t ch_off = tab_off + align256(tab.size() * 8);
    const size_t buf_off = ch_off + align256(size_t(K) * kBoxSlots * 8);
    s.tabd = (const double *)(base + tab_off);
    SolveDesc *d_desc = (SolveDesc *)base;
    unsigned long long *d_ch = (unsigned long long *)(base + ch_off);
    void *bufB = base + buf_off;
    // the host images stay alive until the stream has copied them
    std::vector<unsigned long long> hch(size_t(K) * kBoxSlots, 0ull);
    if ((rc = check_hip(hipMemcpyAsync(d_desc, &s, sizeof(s), hipMemcpyHostToDevice, st), "ttr desc")) ||
        (rc = check_hip(hipMemcpyAsync(base + tab_off, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st),
                        "ttr tables")) ||
        (rc = check_hip(launch_ttr_init(prec, target_dev, phi_out_dev, grid->npts, big, st), "ttr init")))
        return rc;
    Timer tm;
    if ((rc = check_hip(hipEventCreate(&tm.e0), "event")) || (rc = check_hip(hipEventCreate(&tm.e1), "event")))
        return rc;
    (void)hipEventRecord(tm.e0, st);
    const uint32_t qblocks = uint32_t((Q + kBlock - 1) / kBlock);
    // axis-0 run per lane: about kTtrBlocks blocks in all (every CU a few),
    // so each lane amortises its per-column terms over several nodes
    constexpr int64_t kTtrBlocks = 1024;
    const int chunk = int(std::min<int64_t>(n0, std::max<int64_t>(1, (n0 * qblocks + kTtrBlocks - 1) / kTtrBlocks)));
    int64_t it = 0;
    double last = INFINITY;
    bool converged = false;
    void *cur = phi_out_dev, *nxt = bufB;
    while (it < opts->max_iters && !converged) {
        const int nb = int(std::min<int64_t>(K, opts->max_iters - it));
        if ((rc = check_hip(launch_ttr_zero(d_ch, nb * kBoxSlots, st), "ttr zero"))) return rc;
        for (int j = 0; j < nb; ++j) {
            if ((rc = check_hip(launch_ttr(prec, dyn->id, N, d_desc, qblocks, int(n0), chunk, cur, nxt, target_dev,
                                           d_ch + size_t(j) * kBoxSlots, st),
                                "ttr sweep")))
                return rc;
            std::swap(cur, nxt);
        }
        if ((rc = check_hip(hipMemcpyAsync(hch.data(), d_ch, size_t(nb) * kBoxSlots * 8, hipMemcpyDeviceToHost, st),
                            "ttr change")) ||
            (rc = check_hip(hipStreamSynchronize(st), "sync")))
            return rc;
        for (int j = 0; j < nb; ++j) {
            double c = 0.0;
            for (int k = 0; k < kBoxSlots; ++k) {
                double v;
                std::memcpy(&v, &hch[size_t(j) * kBoxSlots + size_t(k)], 8);
                c = std::max(c, v);
            }
            last = c;
            if (c < opts->eps) converged = true;
        }
        it += nb;
    }
    if (cur != phi_out_dev &&
        (rc = check_hip(hipMemcpyAsync(phi_out_dev, cur, size_t(grid->npts) * eb, hipMemcpyDeviceToDevice, st),
                        "ttr result")))
        return rc;
    (void)hipEventRecord(tm.e1, st);
    if ((rc = check_hip(hipEventSynchronize(tm.e1), "sync"))) return rc;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        stats->iters = it;
        stats->last_change = last;
        stats->converged = converged ? 1 : 0;
        stats->kernel_ms = ms;
        // each iteration reads the previous iterate and the target, writes the next
        stats->alg_bytes = 3.0 * double(eb) * double(grid->npts) * double(it);
        stats->alg_gbps = ms > 0 ? stats->alg_bytes / (double(ms) * 1e6) : 0.0;
        stats->roofline_frac = stats->alg_gbps / 8000.0;
    }
    return ODP_OK;
}

}  // extern "C"
