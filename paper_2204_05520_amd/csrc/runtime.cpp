// Host side of libodp: errors, argument checks, grids, tiling choices.
#include "runtime.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

namespace odp {

static thread_local std::string g_last_error;

int set_error(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

int check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return ODP_OK;
    return set_error(ODP_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

namespace {

// Pinned staging blocks for upload_async, kept for the life of the process
// (a pinned allocation is a driver call; the blocks are recycled instead).
struct StageBlock {
    unsigned char *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;  // recorded after the block's last copy
    int device = -1;
};

std::mutex g_stage_mu;
std::vector<StageBlock> g_stage;

}  // namespace

int upload_async(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return ODP_OK;
    int dev = 0, rc;
    if ((rc = check_hip(hipGetDevice(&dev), "device"))) return rc;
    std::lock_guard<std::mutex> lk(g_stage_mu);
    StageBlock *b = nullptr;
    for (StageBlock &c : g_stage)
        if (c.device == dev && c.cap >= bytes && hipEventQuery(c.ev) == hipSuccess) {
            b = &c;
            break;
        }
    if (!b) {
        StageBlock n;
        n.device = dev;
        n.cap = std::max<size_t>(size_t(64) << 10, size_t(1) << size_t(std::ceil(std::log2(double(bytes)))));
        if ((rc = check_hip(hipHostMalloc((void **)&n.p, n.cap, hipHostMallocDefault), "pinned staging")))
            return rc;
        if ((rc = check_hip(hipEventCreateWithFlags(&n.ev, hipEventDisableTiming), "event"))) {
            (void)hipHostFree(n.p);
            return rc;
        }
        g_stage.push_back(n);
        b = &g_stage.back();
    }
    std::memcpy(b->p, src, bytes);
    if ((rc = check_hip(hipMemcpyAsync(dst, b->p, bytes, hipMemcpyHostToDevice, st), "upload"))) return rc;
    return check_hip(hipEventRecord(b->ev, st), "record");
}

static int dyn_ndim(int id) {
    switch (id) {
    case ODP_DYN_DUBINS3D: return 3;
    case ODP_DYN_DYNCAR4D: return 4;
    case ODP_DYN_TWODUBINS6D: return 6;
    case ODP_DYN_PE3D: return 3;
    default: return 0;
    }
}

int validate_dyn(const odp_grid *g, const odp_dynamics *dyn) {
    if (!dyn) return set_error(ODP_EINVAL, "dynamics is NULL");
    if (dyn->id < 0 || dyn->id > 4) return set_error(ODP_EINVAL, "unknown dynamics id");
    if (dyn->id != ODP_DYN_SINGLE_INTEGRATOR && dyn_ndim(dyn->id) != g->ndim)
        return set_error(ODP_EINVAL, "dynamics dimension does not match the grid");
    if ((dyn->u_mode != 0 && dyn->u_mode != 1) || (dyn->d_mode != 0 && dyn->d_mode != 1))
        return set_error(ODP_EINVAL, "u_mode / d_mode must be 0 or 1");
    for (int k = 0; k < 16; ++k)
        if (!std::isfinite(dyn->p[k])) return set_error(ODP_EINVAL, "non-finite dynamics parameter");
    switch (dyn->id) {
    case ODP_DYN_SINGLE_INTEGRATOR:
        if (dyn->p[0] < 0) return set_error(ODP_EINVAL, "u_max must be >= 0");
        break;
    case ODP_DYN_DUBINS3D:
        if (dyn->p[1] < 0) return set_error(ODP_EINVAL, "w_max must be >= 0");
        if (!g->periodic[2]) return set_error(ODP_EINVAL, "the heading axis must be periodic");
        break;
    case ODP_DYN_DYNCAR4D:
        if (dyn->p[0] < 0 || dyn->p[1] < 0) return set_error(ODP_EINVAL, "input bounds must be >= 0");
        if (!g->periodic[3]) return set_error(ODP_EINVAL, "the heading axis must be periodic");
        break;
    case ODP_DYN_TWODUBINS6D:
        if (dyn->p[1] < 0 || dyn->p[3] < 0) return set_error(ODP_EINVAL, "input bounds must be >= 0");
        if (!g->periodic[2] || !g->periodic[5])
            return set_error(ODP_EINVAL, "the heading axes must be periodic");
        break;
    case ODP_DYN_PE3D:
        if (dyn->p[2] < 0 || dyn->p[3] < 0) return set_error(ODP_EINVAL, "input bounds must be >= 0");
        if (!g->periodic[2]) return set_error(ODP_EINVAL, "the heading axis must be periodic");
        break;
    }
    return ODP_OK;
}

int validate_opts(const odp_solve_opts *o) {
    if (!o) return set_error(ODP_EINVAL, "opts is NULL");
    if (o->precision != 32 && o->precision != 64) return set_error(ODP_EINVAL, "precision must be 32 or 64");
    if (o->rk_order < 1 || o->rk_order > 3) return set_error(ODP_EINVAL, "rk_order must be 1, 2 or 3");
    if (!(o->cfl > 0.0 && o->cfl <= 1.0)) return set_error(ODP_EINVAL, "cfl must be in (0, 1]");
    if (o->mode < ODP_BRS || o->mode > ODP_MAX_TARGET) return set_error(ODP_EINVAL, "mode must be 0..6");
    if (o->obstacle_mode < ODP_OBSTACLE_NONE || o->obstacle_mode > ODP_MAX_OBSTACLE)
        return set_error(ODP_EINVAL, "obstacle_mode must be 0, 1 or 2");
    const bool wants_target = o->mode == ODP_MIN_TARGET || o->mode == ODP_MAX_TARGET;
    if (wants_target != (o->target_dev != nullptr))
        return set_error(ODP_EINVAL, wants_target ? "the target method needs target_dev"
                                                  : "target_dev is set but the method does not use it");
    if ((o->obstacle_mode != 0) != (o->obstacle_dev != nullptr))
        return set_error(ODP_EINVAL, o->obstacle_mode ? "the obstacle method needs obstacle_dev"
                                                      : "obstacle_dev is set but obstacle_mode is 0");
    if (o->space_order < 0 || o->space_order > 2) return set_error(ODP_EINVAL, "space_order must be 0, 1 or 2");
    if (o->set_slices < 0 || (o->set_slices > 1 && !o->target_dev && !o->obstacle_dev))
        return set_error(ODP_EINVAL, "set_slices needs a target or obstacle array");
    if (o->dissipation != 0 && o->dissipation != 1) return set_error(ODP_EINVAL, "dissipation must be 0 or 1");
    if (!(o->max_dt >= 0.0) || !std::isfinite(o->max_dt)) return set_error(ODP_EINVAL, "max_dt must be >= 0");
    if (o->save_all != 0 && o->save_all != 1) return set_error(ODP_EINVAL, "save_all must be 0 or 1");
    if (o->tile_chunk < 0 && o->tile_chunk != ODP_TILE_AUTOTUNE)
        return set_error(ODP_EINVAL, "tile_chunk must be >= 0 or ODP_TILE_AUTOTUNE");
    if (o->xcd_group < 0) return set_error(ODP_EINVAL, "xcd_group must be >= 0");
    if (o->graph < 0 || o->graph > 2) return set_error(ODP_EINVAL, "graph must be 0, 1 or 2");
    return ODP_OK;
}

int validate_tau(const double *tau, int ntau) {
    if (!tau || ntau < 2) return set_error(ODP_EINVAL, "tau needs at least two times");
    if (!(tau[0] >= 0.0) || !std::isfinite(tau[0])) return set_error(ODP_EINVAL, "tau[0] must be >= 0");
    for (int k = 1; k < ntau; ++k)
        if (!(tau[k] > tau[k - 1]) || !std::isfinite(tau[k]))
            return set_error(ODP_EINVAL, "tau must be finite and strictly increasing");
    return ODP_OK;
}

// Upper bound of max_i alpha_d(z_i) from the parameters and the domain
// (sizes the dt schedule; the schedule itself uses the device reduction).
void alpha_bound(const odp_grid *g, const odp_dynamics *dyn, double *ab) {
    for (int d = 0; d < kMaxDim; ++d) ab[d] = 0.0;
    const double *p = dyn->p;
    switch (dyn->id) {
    case ODP_DYN_SINGLE_INTEGRATOR:
        for (int d = 0; d < g->ndim; ++d) ab[d] = std::fabs(p[1 + d]) + p[0];
        break;
    case ODP_DYN_DUBINS3D:
        ab[0] = ab[1] = std::fabs(p[0]);
        ab[2] = p[1];
        break;
    case ODP_DYN_DYNCAR4D: {
        const double vm = std::max(std::fabs(g->lo[2]), std::fabs(g->hi[2]));
        ab[0] = ab[1] = vm;
        ab[2] = p[0];
        ab[3] = p[1];
        break;
    }
    case ODP_DYN_TWODUBINS6D:
        ab[0] = ab[1] = std::fabs(p[0]);
        ab[2] = p[1];
        ab[3] = ab[4] = std::fabs(p[2]);
        ab[5] = p[3];
        break;
    case ODP_DYN_PE3D: {
        const double xm = std::max(std::fabs(g->lo[0]), std::fabs(g->hi[0]));
        const double ym = std::max(std::fabs(g->lo[1]), std::fabs(g->hi[1]));
        ab[0] = std::fabs(p[0]) + std::fabs(p[1]) + p[2] * ym;
        ab[1] = std::fabs(p[1]) + p[2] * xm;
        ab[2] = p[2] + p[3];
        break;
    }
    }
}

int choose_vec(const odp_grid *g, int precision, int dyn, int64_t pitch) {
    if (g->ndim < 2 || dyn == ODP_DYN_SINGLE_INTEGRATOR) return 1;
    if (precision == 32 && pitch % 4 == 0) return 4;
    if (pitch % 2 == 0) return 2;
    return 1;
}

// Planes of axis 0 marched per block.  First order in four dimensions: the
// fewest chunks (of balanced lengths) whose tiles fill 65-100% of one round
// of resident blocks of the stage kernels (1024: 4 waves per SIMD in both
// precisions): a tile reads the two planes beyond its chunk
// and pays a start-up, so long chunks win as long as the GPU is full, and a
// second, partial round costs more than it saves (measured on 4D grids of
// 40-80 nodes per axis in both precisions: the choice matched or beat the
// autotuner, where about 2048 tiles per solve lost up to 20%; the ENO2
// kernel, whose waves wait longer on memory, lost 20% with it at 80^4).
// ENO2, grids with more whole-axis tiles than one round and other
// dimensions: about 2048 tiles per solve, at most a third of the axis from
// five dimensions on (measured on the 6D 36^6 grid: 12 planes beat 4, 8, 20
// and 36); the plan rounds these to whole 4-plane cycles.
namespace {
// blocks of the 4D first-order stage kernels resident at once (256 CUs, 4
// blocks of 4 waves each)
constexpr int64_t kResident4D = 1024;
}  // namespace

int default_chunk(const odp_grid *g, int vec, int precision, int space_order) {
    (void)precision;  // the same in both precisions (vec carries the width)
    const int64_t n0 = g->n[0];
    const int64_t Q = g->npts / n0;
    const int64_t nqb = (Q + int64_t(kBlock) * vec - 1) / (int64_t(kBlock) * vec);
    if (g->ndim == 4 && space_order == 1) {
        const int64_t round = kResident4D, fill = round * 13 / 20;
        int64_t most = 0, at = 0;
        for (int64_t nch = 1; nch <= n0; ++nch) {
            const int64_t b = (n0 + nch - 1) / nch;
            const int64_t tiles = nqb * ((n0 + b - 1) / b);
            if (tiles > round) break;  // tiles only grow with nch
            if (tiles >= fill) return int(b);
            if (tiles > most) {
                most = tiles;
                at = b;
            }
        }
        if (at > 0) return int(at);  // small grids: one round as full as it gets
    }
    int64_t c = (n0 * nqb + 2047) / 2048;
    if (g->ndim >= 5) c = std::min<int64_t>(c, (n0 + 2) / 3);
    return int(std::max<int64_t>(1, std::min<int64_t>(c, n0)));
}

// True when default_chunk's choice for this grid is taken as it is (not
// rounded to whole 4-plane cycles): the one-round choice in four dimensions.
bool default_chunk_exact(const odp_grid *g, int vec, int precision, int space_order) {
    (void)precision;
    if (g->ndim != 4 || space_order != 1) return false;
    const int64_t n0 = g->n[0];
    const int64_t nqb = (g->npts / n0 + int64_t(kBlock) * vec - 1) / (int64_t(kBlock) * vec);
    return nqb <= kResident4D;
}

// Tile runs per XCD: one contiguous run, except for grids whose arrays are
// far larger than the 256 MB Infinity Cache, where runs of 64 tiles dealt
// round robin keep the 8 XCDs on one shared working set.
int default_xcd_group(const odp_grid *g) { return g->npts >= (int64_t(1) << 28) ? 64 : 0; }

double alg_bytes_per_step(int precision, int rk_order, int narr, int64_t npts) {
    // each stage reads its stencil input once and writes its output once;
    // stages after the first also read V^n; the computation method reads
    // narr more arrays (V0 for the tube)
    const double b = precision == 32 ? 4.0 : 8.0;
    double per = 2.0 * rk_order + (rk_order - 1) + narr;
    return per * b * double(npts);
}

int method_arrays(const odp_solve_opts &o) {
    const int m = o.mode;
    return ((m == 1 || m == 2 || m == 5 || m == 6) ? 1 : 0) + (o.obstacle_mode != 0 ? 1 : 0);
}

int method_kind(const odp_solve_opts &o) {
    const bool t = o.mode != ODP_BRS, g = o.obstacle_mode != ODP_OBSTACLE_NONE;
    return (t || g ? 2 : 0) | (t && g ? 8 : 0);
}

}  // namespace odp

using namespace odp;

// ====================================================================== C ABI

extern "C" {

const char *odp_strerror(int code) {
    switch (code) {
    case ODP_OK: return "ok";
    case ODP_PENDING: return "pending";
    case ODP_EINVAL: return "invalid argument";
    case ODP_ENOMEM: return "out of memory or workspace too small";
    case ODP_EHIP: return "HIP runtime error";
    case ODP_EUNSUPPORTED: return "unsupported combination";
    case ODP_EAGAIN: return "queue full, try again";
    case ODP_ENONFINITE: return "non-finite value in the value function";
    case ODP_ECANCELED: return "request cancelled";
    default: return "unknown error code";
    }
}

const char *odp_last_error(void) { return g_last_error.c_str(); }

int odp_grid_create(int ndim, const int64_t *n, const double *lo, const double *hi,
                    const uint8_t *periodic, odp_grid **out) {
    if (!out) return set_error(ODP_EINVAL, "out is NULL");
    *out = nullptr;
    if (ndim < 1 || ndim > kMaxDim) return set_error(ODP_EINVAL, "ndim must be in [1, 6]");
    if (!n || !lo || !hi) return set_error(ODP_EINVAL, "n, lo and hi are required");
    std::unique_ptr<odp_grid> g(new odp_grid());
    g->ndim = ndim;
    g->npts = 1;
    for (int d = 0; d < ndim; ++d) {
        if (n[d] < 3 || n[d] > (int64_t(1) << 30))
            return set_error(ODP_EINVAL, "every axis needs between 3 and 2^30 nodes");
        if (!std::isfinite(lo[d]) || !std::isfinite(hi[d]) || !(hi[d] > lo[d]))
            return set_error(ODP_EINVAL, "bounds must be finite with lo < hi");
        g->n[d] = n[d];
        g->lo[d] = lo[d];
        g->hi[d] = hi[d];
        g->periodic[d] = periodic && periodic[d] ? 1 : 0;
        g->dx[d] = g->periodic[d] ? (hi[d] - lo[d]) / double(n[d]) : (hi[d] - lo[d]) / double(n[d] - 1);
        if (g->npts > (int64_t(1) << 40) / n[d]) return set_error(ODP_EINVAL, "grid too large");
        g->npts *= n[d];
    }
    if (g->npts / g->n[0] >= (int64_t(1) << 31))
        return set_error(ODP_EINVAL, "a hyperplane of axes 1..ndim-1 must hold < 2^31 points");
    *out = g.release();
    return ODP_OK;
}

void odp_grid_destroy(odp_grid *grid) { delete grid; }

int64_t odp_grid_points(const odp_grid *grid) { return grid ? grid->npts : 0; }

}  // extern "C"
