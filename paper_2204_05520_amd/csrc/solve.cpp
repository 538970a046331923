// Single-solve and batched drivers behind odp_hj_solve / odp_hj_batch.
//
// Per solve: upload the descriptor, axis tables and tau (one copy), zero
// the state, reduce alpha^max over the grid on the device, build the float64
// CFL schedule on the device, read back only the step count, then enqueue
// the stage launches of every step.  A batch runs the same per-solve
// prologue for all solves at once and then steps them in lockstep: launch k
// covers every solve that still has a step k, so each solve's tiles spread
// over the whole GPU and launch boundaries order the steps.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <numeric>
#include <vector>

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

int alloc_workspace(DeviceBuffer &buf, void *given, size_t bytes, hipStream_t st) {
    buf.st = st;
    if (given) {
        if ((uintptr_t(given) & 255u) != 0) return set_error(ODP_EINVAL, "workspace must be 256-byte aligned");
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

int chunk_for(const odp_grid *g, const odp_solve_opts *o, int vec) {
    int c = o->tile_chunk > 0 ? o->tile_chunk : default_chunk(g, vec, o->precision);
    return std::min<int>(c, int(g->n[0]));
}

int blocks_for_alpha(const odp_grid *g) {
    const int64_t Q = g->npts / g->n[0];
    return int(std::max<int64_t>(1, std::min<int64_t>((Q + kBlock - 1) / kBlock, 4096)));
}

}  // namespace

extern "C" {

size_t odp_hj_workspace_bytes(const odp_grid *grid, const odp_dynamics *dyn, const double *tau,
                              int ntau, const odp_solve_opts *opts) {
    if (!grid || validate_opts(opts) != ODP_OK || validate_dyn(grid, dyn) != ODP_OK ||
        validate_tau(tau, ntau) != ODP_OK)
        return 0;
    return solve_layout(grid, opts->precision, opts->rk_order, ntau, tau[ntau - 1] - tau[0], dyn,
                        opts->cfl, opts->max_dt)
        .total;
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
    if (opts->save_all && !V_all_dev) return set_error(ODP_EINVAL, "save_all needs V_all");
    hipStream_t st = (hipStream_t)opts->stream;
    const int prec = opts->precision;
    const size_t eb = prec == 32 ? 4 : 8;
    const size_t bytes = size_t(grid->npts) * eb;

    SolveLayout L = solve_layout(grid, prec, opts->rk_order, ntau, tau[ntau - 1] - tau[0], dyn,
                                 opts->cfl, opts->max_dt);
    DeviceBuffer ws;
    if ((rc = alloc_workspace(ws, workspace_dev, L.total, st))) return rc;
    unsigned char *base = (unsigned char *)ws.ptr;
    const int vec = choose_vec(grid, prec, dyn->id);
    const int chunk = chunk_for(grid, opts, vec);
    std::vector<unsigned char> img;
    build_solve_image(img, L, base, grid, dyn, opts, tau, ntau, V0_dev, V_out_dev, chunk, vec);
    const SolveDesc *d_desc = (const SolveDesc *)(base + L.desc);
    const uint32_t tiles = solve_tiles(grid, chunk, vec);

    if ((rc = check_hip(hipMemcpyAsync(base, img.data(), L.head, hipMemcpyHostToDevice, st), "upload")))
        return rc;
    if ((rc = check_hip(launch_init(d_desc, 1, st), "init"))) return rc;
    if ((rc = check_hip(launch_alpha(dyn->id, grid->ndim, d_desc, 1, blocks_for_alpha(grid), st), "alpha")))
        return rc;
    if ((rc = check_hip(launch_sched(d_desc, 1, st), "schedule"))) return rc;
    int64_t nsteps = 0;
    const unsigned char *state = base + L.state;
    if ((rc = check_hip(hipMemcpyAsync(&nsteps, state + kMaxDim * 8, 8, hipMemcpyDeviceToHost, st), "read steps")))
        return rc;
    if ((rc = check_hip(hipStreamSynchronize(st), "sync"))) return rc;
    if (nsteps <= 0) return set_error(ODP_EHIP, "schedule overflow (internal step bound exceeded)");

    std::vector<int32_t> land;
    if (opts->save_all) {
        land.resize(size_t(nsteps));
        if ((rc = check_hip(hipMemcpyAsync(land.data(), base + L.land, size_t(nsteps) * 4,
                                           hipMemcpyDeviceToHost, st), "read landings")))
            return rc;
        if ((rc = check_hip(hipStreamSynchronize(st), "sync"))) return rc;
    }

    // start value into the buffer the first step reads
    const void *src = V_init_dev ? V_init_dev : V0_dev;
    void *A = V_out_dev;
    void *B = base + L.B;
    void *start = (opts->rk_order == 1 && (nsteps & 1)) ? B : A;
    if ((rc = check_hip(hipMemcpyAsync(start, src, bytes, hipMemcpyDeviceToDevice, st), "start copy"))) return rc;
    if (opts->save_all &&
        (rc = check_hip(hipMemcpyAsync(V_all_dev, src, bytes, hipMemcpyDeviceToDevice, st), "save start")))
        return rc;

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        if ((rc = check_hip(hipEventCreate(&e0), "event")) || (rc = check_hip(hipEventCreate(&e1), "event")))
            return rc;
        (void)hipEventRecord(e0, st);
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        for (int j = 0; j < opts->rk_order; ++j) {
            if ((rc = check_hip(launch_stage(prec, dyn->id, grid->ndim, vec,
                                             stage_kind(opts->rk_order, j, opts->mode == ODP_BRT), d_desc,
                                             nullptr, nullptr, tiles,
                                             j, 0, k, st), "stage")))
                return rc;
        }
        if (opts->save_all && land[size_t(k)] >= 0) {
            const void *outb = (opts->rk_order == 1 && ((k + nsteps) & 1) == 0) ? B : A;
            unsigned char *dst = (unsigned char *)V_all_dev + size_t(land[size_t(k)]) * bytes;
            if ((rc = check_hip(hipMemcpyAsync(dst, outb, bytes, hipMemcpyDeviceToDevice, st), "save")))
                return rc;
        }
    }
    if (stats) {
        (void)hipEventRecord(e1, st);
        if ((rc = check_hip(hipEventSynchronize(e1), "sync"))) return rc;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        double amax[kMaxDim];
        int32_t flags = 0;
        std::vector<double> dts(static_cast<size_t>(nsteps));
        if ((rc = check_hip(hipMemcpy(amax, state, sizeof(amax), hipMemcpyDeviceToHost), "read alpha")) ||
            (rc = check_hip(hipMemcpy(&flags, state + kMaxDim * 8 + 16, 4, hipMemcpyDeviceToHost), "read flags")) ||
            (rc = check_hip(hipMemcpy(dts.data(), base + L.sched, size_t(nsteps) * 8, hipMemcpyDeviceToHost),
                            "read schedule")))
            return rc;
        std::memset(stats, 0, sizeof(*stats));
        stats->steps = nsteps;
        stats->dt_min = *std::min_element(dts.begin(), dts.end());
        stats->dt_max = *std::max_element(dts.begin(), dts.end());
        stats->t_final = tau[ntau - 1];
        stats->kernel_ms = ms;
        stats->alg_bytes = alg_bytes_per_step(prec, opts->rk_order, opts->mode == ODP_BRT, grid->npts) * double(nsteps);
        stats->alg_gbps = ms > 0 ? stats->alg_bytes / (ms * 1e6) : 0.0;
        stats->roofline_frac = stats->alg_gbps / 8000.0;
        for (int d = 0; d < kMaxDim; ++d) stats->alpha_max[d] = amax[d];
        stats->nonfinite = flags & 1;
        if (stats->nonfinite) return set_error(ODP_ENONFINITE, "NaN or Inf in the value function");
    }
    return ODP_OK;
}

}  // extern "C"
