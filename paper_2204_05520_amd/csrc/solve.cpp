// odp_hj_solve and odp_hj_batch: a plan of one solve, or of many solves
// stepped in lockstep (launch k covers every solve that still has a step k,
// so each solve's tiles spread over the whole GPU and launch boundaries
// order the steps).
#include <hip/hip_runtime_api.h>

#include <algorithm>
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

    std::vector<int32_t> land;
    const bool want_land = opts->save_all || opts->set_slices > 1;
    if (want_land) {
        const PlanItem &it = p.items[0];
        land.resize(size_t(it.nsteps));
        if ((rc = check_hip(hipMemcpyAsync(land.data(), base + it.land_off, land.size() * 4,
                                           hipMemcpyDeviceToHost, st), "read landings")) ||
            (rc = check_hip(hipStreamSynchronize(st), "sync")))
            return rc;
    }
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
    if ((rc = plan_steps(p, base, st, want_land ? &land : nullptr, opts->save_all ? V_all_dev : nullptr)))
        return rc;
    if (stats) {
        (void)hipEventRecord(tm.e1, st);
        if ((rc = check_hip(hipEventSynchronize(tm.e1), "sync"))) return rc;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        return plan_stats(p, base, ms, stats);
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
    if ((rc = plan_steps(p, base, st, nullptr, nullptr))) return rc;
    if (stats_per_solve) {
        (void)hipEventRecord(tm.e1, st);
        if ((rc = check_hip(hipEventSynchronize(tm.e1), "sync"))) return rc;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, tm.e0, tm.e1);
        std::vector<odp_solve_stats> sorted(p.items.size());
        rc = plan_stats(p, base, ms, sorted.data());
        for (size_t i = 0; i < perm.size(); ++i) stats_per_solve[perm[i]] = sorted[i];
        if (rc) return rc;
    }
    return ODP_OK;
}

}  // extern "C"
