// Continuous-batching server: odp_server_create / odp_serve_submit /
// odp_serve_poll / odp_serve_cancel / odp_server_destroy.
//
// A scheduler thread owns a device slot table of solve descriptors.  Each
// iteration it
//   1. admits queued requests in arrival order while a slot is free and the
//      request's device footprint fits the HBM budget (allocation, V0 upload,
//      alpha^max and float64 schedule on the device, one synchronisation for
//      the step counts);
//   2. runs one tick: the active solves with the least remaining work (up to
//      a work budget) advance by up to kStepsPerTick steps, one batched
//      launch per RK stage and kernel group, each solve reading its own step
//      counter on the device;
//   3. retires finished solves (result copied to the host, memory freed).
// Requests that arrive while others run therefore join at the next tick and
// share every launch with them.  The per-point arithmetic is the same as in
// odp_hj_solve, so a served result equals the solve run alone, bit for bit.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <tuple>
#include <vector>

#include "plan.h"
#include "runtime.h"

using namespace odp;

namespace {

constexpr int kStepsPerTick = 8;
constexpr double kTickWork = 2.0e9;   // point-stage updates per tick (a few ms)
constexpr double kMaxWaitMs = 1500.0;
constexpr size_t kMaxQueue = 1 << 16;

enum { R_QUEUED = 0, R_RUNNING = 1, R_DONE = 2 };

using Clock = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    odp_grid grid{};
    odp_dynamics dyn{};
    std::vector<double> tau;
    int rk_order = 1;
    // Host copy of V0 in pinned memory (so that the scheduler's upload is an
    // asynchronous DMA); the same buffer later receives V(tau_last).
    unsigned char *host = nullptr;
    bool host_pinned = false;
    ~Req() {
        if (host_pinned) (void)hipHostFree(host);
        else delete[] host;
    }
    size_t bytes = 0;                   // one grid array (dense, host)
    size_t row = 0, row_pitch = 0, rows = 0;  // last-axis rows: bytes, device pitch, count
    size_t footprint = 0;               // device bytes while running
    int state = R_QUEUED;
    int rc = ODP_OK;
    bool cancel = false;
    odp_solve_stats stats{};
    Clock::time_point t_submit;
    // scheduler-owned while running
    unsigned char *dmem = nullptr;
    size_t off_v0 = 0, off_a = 0;
    int slot = -1;
    Plan plan;
    int64_t nsteps = 0, step = 0;
};

}  // namespace

struct odp_server {
    odp_solve_opts opts{};
    size_t budget = 0;
    int max_slots = 0;
    int device = 0;
    hipStream_t st = nullptr;
    SolveDesc *d_slots = nullptr;
    int64_t *d_nsteps = nullptr;
    uint32_t *d_tiles = nullptr;  // [cap] solve slot, [cap] local tile
    int32_t *d_list = nullptr;    // [max_slots] per-group member slots
    size_t tile_cap = 0;

    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Req>> queue;
    std::map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    int running = 0, done = 0;

    // scheduler thread only
    std::vector<std::shared_ptr<Req>> active;
    std::vector<int> free_slots;
    size_t used = 0;
    std::thread th;
};

namespace {

struct Group {
    int dyn, ndim, vec, rk;
    std::vector<int> slots;
    uint32_t tiles = 0;
    size_t tile_base = 0, list_base = 0;
};

// The server keeps its own copies of V0 and V on the device, so it stores
// last-axis rows with a pitch padded to the 16-byte vector width: every
// request then runs the widest vector kernel whatever its row length.
size_t request_layout(Req &r, const odp_solve_opts &o) {
    PlanItem it;
    it.g = &r.grid;
    it.dyn = r.dyn;
    it.tau = r.tau;
    it.rk_order = r.rk_order;
    const int64_t nl = r.grid.n[r.grid.ndim - 1];
    const int64_t w = o.precision == 32 ? 4 : 2;
    it.pitch = int((nl + w - 1) / w * w);
    // many requests share every launch: march at least 8 planes per block
    int chunk = o.tile_chunk;
    if (chunk <= 0) {
        int vec = choose_vec(&r.grid, o.precision, r.dyn.id, it.pitch);
        chunk = std::max(default_chunk(&r.grid, vec, o.precision), int(std::min<int64_t>(8, r.grid.n[0])));
    }
    std::vector<PlanItem> items{it};
    plan_build(r.plan, std::move(items), o, chunk);
    const PlanItem &pi = r.plan.items[0];
    r.row = size_t(nl) * (o.precision == 32 ? 4 : 8);
    r.row_pitch = size_t(pi.pitch) * (o.precision == 32 ? 4 : 8);
    r.rows = size_t(r.grid.npts / nl);
    const size_t padded = size_t(pi.ppad) * (o.precision == 32 ? 4 : 8);
    size_t off = r.plan.total;
    r.off_v0 = off;
    off += align256(padded);
    r.off_a = off;
    off += align256(padded);
    return off;
}

void finish(odp_server *s, const std::shared_ptr<Req> &r, int rc) {
    std::lock_guard<std::mutex> lk(s->mu);
    r->rc = rc;
    r->state = R_DONE;
    r->stats.latency_ms = std::chrono::duration<double, std::milli>(Clock::now() - r->t_submit).count();
    s->running--;
    s->done++;
}

void release(odp_server *s, const std::shared_ptr<Req> &r) {
    if (r->dmem) (void)hipFreeAsync(r->dmem, s->st);
    r->dmem = nullptr;
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    r->slot = -1;
    s->used -= r->footprint;
}

// Admit what fits; returns the admitted requests (already launched).
int admit(odp_server *s, std::vector<std::shared_ptr<Req>> &admitted) {
    std::vector<std::shared_ptr<Req>> take;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        size_t used = s->used;
        int slots = int(s->free_slots.size());
        while (!s->queue.empty() && slots > 0) {
            auto &r = s->queue.front();
            if (r->cancel) {
                r->rc = ODP_ECANCELED;
                r->state = R_DONE;
                s->done++;
                s->queue.pop_front();
                continue;
            }
            if (used + r->footprint > s->budget) break;  // arrival order: wait for memory
            used += r->footprint;
            slots--;
            r->state = R_RUNNING;
            s->running++;
            take.push_back(r);
            s->queue.pop_front();
        }
    }
    const odp_solve_opts &o = s->opts;
    std::vector<std::vector<unsigned char>> imgs;
    std::vector<std::shared_ptr<Req>> launched;
    for (auto &r : take) {
        void *mem = nullptr;
        if (hipMallocAsync(&mem, r->footprint, s->st) != hipSuccess) {
            finish(s, r, set_error(ODP_ENOMEM, "server: device allocation failed"));
            continue;
        }
        r->dmem = (unsigned char *)mem;
        r->slot = s->free_slots.back();
        s->free_slots.pop_back();
        s->used += r->footprint;
        PlanItem &it = r->plan.items[0];
        it.V0 = r->dmem + r->off_v0;
        it.A = r->dmem + r->off_a;
        imgs.emplace_back();
        plan_image(r->plan, r->dmem, imgs.back());
        SolveDesc *slot = s->d_slots + r->slot;
        int rc;
        if ((rc = check_hip(hipMemcpy2DAsync(r->dmem + r->off_v0, r->row_pitch, r->host, r->row, r->row, r->rows,
                                             hipMemcpyHostToDevice, s->st), "V0")) ||
            (rc = check_hip(hipMemcpyAsync(r->dmem, imgs.back().data(), imgs.back().size(), hipMemcpyHostToDevice, s->st), "image")) ||
            (rc = check_hip(hipMemcpyAsync(slot, imgs.back().data() + r->plan.desc_off, sizeof(SolveDesc),
                                           hipMemcpyHostToDevice, s->st), "slot")) ||
            (rc = check_hip(launch_init(slot, 1, s->st), "init")) ||
            (rc = check_hip(launch_alpha(r->dyn.id, r->grid.ndim, slot, 1,
                                         int(std::min<int64_t>(2048, (r->grid.npts / r->grid.n[0] + kBlock - 1) / kBlock)),
                                         s->st), "alpha")) ||
            (rc = check_hip(launch_sched(slot, 1, s->d_nsteps + r->slot, s->st), "schedule")) ||
            (rc = check_hip(launch_start_copy(o.precision, slot, nullptr, nullptr, it.tiles, s->st), "start copy"))) {
            release(s, r);
            finish(s, r, rc);
            continue;
        }
        launched.push_back(r);
    }
    if (launched.empty()) return ODP_OK;
    std::vector<int64_t> ns(size_t(s->max_slots));
    int rc;
    if ((rc = check_hip(hipMemcpyAsync(ns.data(), s->d_nsteps, ns.size() * 8, hipMemcpyDeviceToHost, s->st), "steps")) ||
        (rc = check_hip(hipStreamSynchronize(s->st), "sync")))
        return rc;
    for (auto &r : launched) {
        r->nsteps = ns[size_t(r->slot)];
        r->step = 0;
        if (r->nsteps <= 0) {
            release(s, r);
            finish(s, r, set_error(ODP_EHIP, "server: schedule overflow"));
            continue;
        }
        admitted.push_back(r);
    }
    return ODP_OK;
}

int build_groups(odp_server *s, const std::vector<std::shared_ptr<Req>> &sel, std::vector<Group> &groups) {
    groups.clear();
    std::map<std::tuple<int, int, int, int>, size_t> idx;
    for (auto &r : sel) {
        const PlanItem &it = r->plan.items[0];
        auto key = std::make_tuple(r->dyn.id, r->grid.ndim, it.vec, it.rk_order);
        auto f = idx.find(key);
        if (f == idx.end()) {
            idx[key] = groups.size();
            groups.push_back(Group{r->dyn.id, r->grid.ndim, it.vec, it.rk_order, {}, 0, 0, 0});
            f = idx.find(key);
        }
        groups[f->second].slots.push_back(r->slot);
    }
    std::vector<uint32_t> ts, tl;
    std::vector<int32_t> list;
    std::vector<const Req *> by_slot(size_t(s->max_slots), nullptr);
    for (auto &r : sel) by_slot[size_t(r->slot)] = r.get();
    for (Group &g : groups) {
        g.tile_base = ts.size();
        g.list_base = list.size();
        for (int sl : g.slots) {
            const uint32_t t = by_slot[size_t(sl)]->plan.items[0].tiles;
            for (uint32_t k = 0; k < t; ++k) {
                ts.push_back(uint32_t(sl));
                tl.push_back(k);
            }
            list.push_back(sl);
        }
        g.tiles = uint32_t(ts.size() - g.tile_base);
    }
    int rc;
    if (ts.size() > s->tile_cap) {
        if ((rc = check_hip(hipStreamSynchronize(s->st), "sync"))) return rc;
        if (s->d_tiles) (void)hipFree(s->d_tiles);
        s->tile_cap = std::max(ts.size(), 2 * s->tile_cap);
        if ((rc = check_hip(hipMalloc(&s->d_tiles, s->tile_cap * 8), "tile tables"))) {
            s->d_tiles = nullptr;
            s->tile_cap = 0;
            return rc;
        }
    }
    if (!ts.empty()) {
        if ((rc = check_hip(hipMemcpyAsync(s->d_tiles, ts.data(), ts.size() * 4, hipMemcpyHostToDevice, s->st), "tiles")) ||
            (rc = check_hip(hipMemcpyAsync(s->d_tiles + s->tile_cap, tl.data(), tl.size() * 4, hipMemcpyHostToDevice, s->st), "tiles")) ||
            (rc = check_hip(hipMemcpyAsync(s->d_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, s->st), "list")) ||
            (rc = check_hip(hipStreamSynchronize(s->st), "sync")))
            return rc;
    }
    return ODP_OK;
}

int tick(odp_server *s, const std::vector<Group> &groups) {
    const odp_solve_opts &o = s->opts;
    const int brt = o.mode == ODP_BRT;
    int rc;
    for (int m = 0; m < kStepsPerTick; ++m) {
        for (const Group &g : groups) {
            for (int j = 0; j < g.rk; ++j) {
                if ((rc = check_hip(launch_stage(o.precision, g.dyn, g.ndim, g.vec, stage_kind(g.rk, j, brt),
                                                 s->d_slots, s->d_tiles + g.tile_base,
                                                 s->d_tiles + s->tile_cap + g.tile_base, g.tiles, j, 1, 0,
                                                 s->opts.xcd_group, s->st),
                                    "stage")))
                    return rc;
            }
            if ((rc = check_hip(launch_advance(s->d_slots, s->d_list + g.list_base, int(g.slots.size()), s->st),
                                "advance")))
                return rc;
        }
    }
    return check_hip(hipStreamSynchronize(s->st), "sync");
}

// Copy the results of finished requests to their host buffers (one
// synchronisation for all of them), fill their statistics and free them.
int retire_done(odp_server *s, std::vector<std::shared_ptr<Req>> &fin) {
    if (fin.empty()) return ODP_OK;
    struct Back {
        unsigned char state[kMaxDim * 8 + 24];
        std::vector<double> dts;
    };
    std::vector<Back> back(fin.size());
    int rc = ODP_OK;
    for (size_t i = 0; i < fin.size() && rc == ODP_OK; ++i) {
        const auto &r = fin[i];
        const PlanItem &it = r->plan.items[0];
        back[i].dts.resize(static_cast<size_t>(r->nsteps));
        if ((rc = check_hip(hipMemcpy2DAsync(r->host, r->row, r->dmem + r->off_a, r->row_pitch, r->row, r->rows,
                                             hipMemcpyDeviceToHost, s->st), "result")) ||
            (rc = check_hip(hipMemcpyAsync(back[i].state, r->dmem + it.aux_off, sizeof(back[i].state),
                                           hipMemcpyDeviceToHost, s->st), "state")) ||
            (rc = check_hip(hipMemcpyAsync(back[i].dts.data(), r->dmem + it.sched_off, back[i].dts.size() * 8,
                                           hipMemcpyDeviceToHost, s->st), "schedule")))
            break;
    }
    if (rc == ODP_OK) rc = check_hip(hipStreamSynchronize(s->st), "sync");
    for (size_t i = 0; i < fin.size(); ++i) {
        const auto &r = fin[i];
        int rr = rc;
        if (rc == ODP_OK) {
            odp_solve_stats &sx = r->stats;
            const auto &dts = back[i].dts;
            sx.steps = r->nsteps;
            sx.dt_min = *std::min_element(dts.begin(), dts.end());
            sx.dt_max = *std::max_element(dts.begin(), dts.end());
            sx.t_final = r->tau.back();
            sx.alg_bytes = alg_bytes_per_step(s->opts.precision, r->rk_order, s->opts.mode == ODP_BRT,
                                              r->grid.npts) * double(r->nsteps);
            std::memcpy(sx.alpha_max, back[i].state, sizeof(sx.alpha_max));
            int32_t flags;
            std::memcpy(&flags, back[i].state + kMaxDim * 8 + 16, 4);
            sx.nonfinite = flags & 1;
            rr = sx.nonfinite ? ODP_ENONFINITE : ODP_OK;
        }
        release(s, r);
        finish(s, r, rr);
    }
    fin.clear();
    return rc;
}

int retire_cancelled(odp_server *s, const std::shared_ptr<Req> &r) {
    release(s, r);
    finish(s, r, ODP_ECANCELED);
    return ODP_OK;
}

void fail_all(odp_server *s, int rc) {
    for (auto &r : s->active) {
        release(s, r);
        finish(s, r, rc);
    }
    s->active.clear();
}

void scheduler(odp_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<Group> groups;
    std::vector<uint64_t> last_sel;
    bool dirty = true;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (s->stop) break;
            if (s->active.empty() && s->queue.empty()) {
                s->cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        std::vector<std::shared_ptr<Req>> admitted;
        if (admit(s, admitted) != ODP_OK) {
            fail_all(s, ODP_EHIP);
            dirty = true;
            continue;
        }
        if (!admitted.empty()) {
            for (auto &r : admitted) s->active.push_back(r);
            dirty = true;
        }
        // cancellations of running requests
        for (size_t i = 0; i < s->active.size();) {
            bool c;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                c = s->active[i]->cancel;
            }
            if (c) {
                retire_cancelled(s, s->active[i]);
                s->active.erase(s->active.begin() + long(i));
                dirty = true;
            } else {
                ++i;
            }
        }
        if (s->active.empty()) continue;
        // This tick advances the requests with the least remaining work
        // first, up to about kTickWork point-stage updates (at least one
        // request; any request waiting longer than kMaxWaitMs joins anyway),
        // so that small requests are not held behind large ones.
        std::vector<std::shared_ptr<Req>> order = s->active, sel;
        auto work = [](const std::shared_ptr<Req> &r, int64_t steps) {
            return double(steps) * double(r->plan.items[0].ppad) * double(r->plan.items[0].rk_order);
        };
        std::stable_sort(order.begin(), order.end(), [&](const std::shared_ptr<Req> &a, const std::shared_ptr<Req> &b) {
            return work(a, a->nsteps - a->step) < work(b, b->nsteps - b->step);
        });
        const auto now = Clock::now();
        double acc = 0.0;
        for (auto &r : order) {
            const double w = work(r, std::min<int64_t>(kStepsPerTick, r->nsteps - r->step));
            const double age = std::chrono::duration<double, std::milli>(now - r->t_submit).count();
            if (sel.empty() || acc + w <= kTickWork || age > kMaxWaitMs) {
                sel.push_back(r);
                acc += w;
            }
        }
        std::vector<uint64_t> sel_ids;
        for (auto &r : sel) sel_ids.push_back(r->ticket);
        if (sel_ids != last_sel) dirty = true;
        if (dirty) {
            if (build_groups(s, sel, groups) != ODP_OK) {
                fail_all(s, ODP_EHIP);
                continue;
            }
            last_sel = sel_ids;
            dirty = false;
        }
        if (tick(s, groups) != ODP_OK) {
            fail_all(s, ODP_EHIP);
            dirty = true;
            continue;
        }
        std::vector<std::shared_ptr<Req>> fin;
        for (auto &r : sel) r->step = std::min<int64_t>(r->step + kStepsPerTick, r->nsteps);
        for (size_t i = 0; i < s->active.size();) {
            auto &r = s->active[i];
            if (r->step >= r->nsteps) {
                fin.push_back(r);
                s->active.erase(s->active.begin() + long(i));
                dirty = true;
            } else {
                ++i;
            }
        }
        if (retire_done(s, fin) != ODP_OK) {
            fail_all(s, ODP_EHIP);
            dirty = true;
        }
    }
    // shutdown: cancel whatever is still running or queued
    for (auto &r : s->active) retire_cancelled(s, r);
    s->active.clear();
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &r : s->queue) {
        r->rc = ODP_ECANCELED;
        r->state = R_DONE;
    }
    s->queue.clear();
}

}  // namespace

extern "C" {

int odp_server_create(size_t hbm_budget_bytes, int max_slots, const odp_solve_opts *opts, odp_server **out) {
    if (!out) return set_error(ODP_EINVAL, "out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = validate_opts(opts))) return rc;
    if (opts->save_all) return set_error(ODP_EUNSUPPORTED, "save_all is not available when serving");
    if (max_slots < 1 || max_slots > 4096) return set_error(ODP_EINVAL, "max_slots must be in [1, 4096]");
    if (hbm_budget_bytes == 0) return set_error(ODP_EINVAL, "the HBM budget must be positive");
    std::unique_ptr<odp_server> s(new odp_server());
    s->opts = *opts;
    s->opts.stream = nullptr;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    if ((rc = check_hip(hipGetDevice(&s->device), "device")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking), "stream")))
        return rc;
    if ((rc = check_hip(hipMalloc(&s->d_slots, sizeof(SolveDesc) * size_t(max_slots)), "slots")) ||
        (rc = check_hip(hipMalloc(&s->d_nsteps, 8 * size_t(max_slots)), "slots")) ||
        (rc = check_hip(hipMalloc(&s->d_list, 4 * size_t(max_slots)), "slots"))) {
        if (s->d_slots) (void)hipFree(s->d_slots);
        if (s->d_nsteps) (void)hipFree(s->d_nsteps);
        (void)hipStreamDestroy(s->st);
        return rc;
    }
    for (int i = max_slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    odp_server *raw = s.release();
    raw->th = std::thread(scheduler, raw);
    *out = raw;
    return ODP_OK;
}

int odp_serve_submit(odp_server *srv, const odp_solve_desc *d, uint64_t *ticket) {
    if (!srv || !d || !ticket) return set_error(ODP_EINVAL, "NULL argument");
    if (!d->grid) return set_error(ODP_EINVAL, "grid is NULL");
    int rc;
    if ((rc = validate_dyn(d->grid, &d->dyn)) || (rc = validate_tau(d->tau, d->ntau))) return rc;
    if (!d->V0_dev) return set_error(ODP_EINVAL, "V0 (host) is NULL");
    if (d->rk_order < 0 || d->rk_order > 3) return set_error(ODP_EINVAL, "rk_order must be 0..3");
    auto r = std::make_shared<Req>();
    r->grid = *d->grid;
    r->dyn = d->dyn;
    r->tau.assign(d->tau, d->tau + d->ntau);
    r->rk_order = d->rk_order > 0 ? d->rk_order : srv->opts.rk_order;
    r->bytes = size_t(r->grid.npts) * (srv->opts.precision == 32 ? 4 : 8);
    r->footprint = request_layout(*r, srv->opts);
    if (r->footprint > srv->budget)
        return set_error(ODP_ENOMEM, "request needs " + std::to_string(r->footprint) + " device bytes, over the budget");
    if (hipHostMalloc((void **)&r->host, r->bytes, hipHostMallocDefault) == hipSuccess) {
        r->host_pinned = true;
    } else {
        (void)hipGetLastError();
        r->host = new (std::nothrow) unsigned char[r->bytes];
        if (!r->host) return set_error(ODP_ENOMEM, "server: host buffer allocation failed");
    }
    std::memcpy(r->host, d->V0_dev, r->bytes);
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return set_error(ODP_ECANCELED, "server is shutting down");
        if (srv->queue.size() >= kMaxQueue) return set_error(ODP_EAGAIN, "queue full");
        r->ticket = srv->next_ticket++;
        srv->queue.push_back(r);
        srv->all[r->ticket] = r;
        *ticket = r->ticket;
    }
    srv->cv.notify_one();
    return ODP_OK;
}

int odp_serve_poll(odp_server *srv, uint64_t ticket, void *V_out_host, size_t bytes, odp_solve_stats *stats) {
    if (!srv) return set_error(ODP_EINVAL, "server is NULL");
    std::shared_ptr<Req> r;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        auto f = srv->all.find(ticket);
        if (f == srv->all.end()) return set_error(ODP_EINVAL, "unknown ticket");
        if (f->second->state != R_DONE) return ODP_PENDING;
        r = f->second;
        if (r->rc == ODP_OK) {
            if (!V_out_host || bytes != r->bytes)
                return set_error(ODP_EINVAL, "V_out must hold exactly " + std::to_string(r->bytes) + " bytes");
        }
        srv->all.erase(f);
        srv->done--;
    }
    if (r->rc == ODP_OK) std::memcpy(V_out_host, r->host, r->bytes);
    if (stats) *stats = r->stats;
    if (r->rc != ODP_OK) return set_error(r->rc, std::string("request failed: ") + odp_strerror(r->rc));
    return ODP_OK;
}

int odp_serve_cancel(odp_server *srv, uint64_t ticket) {
    if (!srv) return set_error(ODP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto f = srv->all.find(ticket);
    if (f == srv->all.end()) return set_error(ODP_EINVAL, "unknown ticket");
    f->second->cancel = true;
    srv->cv.notify_one();
    return ODP_OK;
}

int odp_server_counts(odp_server *srv, int *queued, int *running, int *done) {
    if (!srv) return set_error(ODP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    if (queued) *queued = int(srv->queue.size());
    if (running) *running = srv->running;
    if (done) *done = srv->done;
    return ODP_OK;
}

void odp_server_destroy(odp_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv.notify_all();
    if (srv->th.joinable()) srv->th.join();
    (void)hipStreamSynchronize(srv->st);
    if (srv->d_tiles) (void)hipFree(srv->d_tiles);
    (void)hipFree(srv->d_slots);
    (void)hipFree(srv->d_nsteps);
    (void)hipFree(srv->d_list);
    (void)hipStreamDestroy(srv->st);
    delete srv;
}

}  // extern "C"
