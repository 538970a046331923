// Continuous-batching server: odp_server_create / odp_serve_submit /
// odp_serve_poll / odp_serve_cancel / odp_server_counts / odp_server_destroy.
//
// A scheduler thread owns a device slot table of solve descriptors and four
// streams, so that uploads, downloads and the per-request prologue overlap
// the time stepping of the requests already running:
//   admission (upload stream): in arrival order, while a slot is free and the
//     request's device footprint fits the HBM budget: allocation, V0 upload,
//     descriptor, alpha^max and the float64 schedule on the device, the start
//     copy and the step count read back; an event marks it ready;
//   tick (two compute streams, forked and joined per tick): the ready
//     requests in arrival order, up to a work budget, advance by
//     kStepsPerTick steps (small requests by up to kSmallStepsPerTick), one
//     batched launch per RK stage and kernel group per step of the tick,
//     the groups split over the two streams, each solve reading its own
//     step counter on the device; at most two
//     ticks are in flight, and while the scheduler waits for a tick slot it
//     keeps admitting arrivals and picking up finished admissions and
//     retirements;
//   retirement (download stream, after the tick that finished the request):
//     result, state and schedule to pinned host memory; an event marks it
//     done, then the device memory and the slot are released.
// The host mirrors every solve's step count, so it knows which tick finishes
// a request without reading the device.  Requests that arrive while others
// run join at a later tick and share every launch with them.  The per-point
// arithmetic is the same as in odp_hj_solve, so a served result equals the
// solve run alone, bit for bit.
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
constexpr int kSmallStepsPerTick = 16;
constexpr int kTicksInFlight = 2;
constexpr double kTickWork = 0.75e9;  // point-stage updates per tick (about 2 ms)
constexpr double kMaxWaitMs = 1500.0;
constexpr size_t kMaxQueue = 1 << 16;
constexpr size_t kStateBytes = kMaxDim * 8 + 40;  // alpha^max, step count, step, flags, dt range

enum { R_QUEUED = 0, R_RUNNING = 1, R_DONE = 2 };

using Clock = std::chrono::steady_clock;

// Pinned host buffers recycled by size class.  A pinned allocation is a
// driver call that costs far more than the small solves a server runs, and a
// pinned free waits for the whole device; the pool makes both rare: blocks of
// up to kSlabBlock bytes are carved from kSlab-byte slabs, larger ones are
// allocated one by one, and every block returns to its class's free list
// when its request is released.  Classes step by a quarter of a power of two
// (at most 25% over the request), and the pool keeps what it allocated until
// the server is destroyed, i.e. the peak of the buffers held at once.
class HostPool {
public:
    static constexpr size_t kMin = 256;
    static constexpr size_t kSlab = size_t(4) << 20;
    static constexpr size_t kSlabBlock = size_t(64) << 10;

    static size_t class_size(size_t bytes) {
        if (bytes <= kMin) return kMin;
        size_t base = kMin;
        while (base * 2 < bytes) base *= 2;  // base < bytes <= 2 base
        const size_t step = base / 4;
        return base + (bytes - base + step - 1) / step * step;
    }

    // A block of at least `bytes` bytes, or nullptr if pinned memory runs out.
    unsigned char *get(size_t bytes) {
        const size_t c = class_size(bytes);
        std::lock_guard<std::mutex> lk(mu_);
        std::vector<unsigned char *> &fl = free_[c];
        if (fl.empty()) {
            const size_t len = c <= kSlabBlock ? kSlab : c;
            unsigned char *p = nullptr;
            if (hipHostMalloc((void **)&p, len, hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            slabs_.push_back(p);
            for (size_t o = 0; o + c <= len; o += c) fl.push_back(p + o);
        }
        unsigned char *p = fl.back();
        fl.pop_back();
        return p;
    }

    void put(unsigned char *p, size_t bytes) {
        if (!p) return;
        std::lock_guard<std::mutex> lk(mu_);
        free_[class_size(bytes)].push_back(p);
    }

    ~HostPool() {
        for (unsigned char *p : slabs_) (void)hipHostFree(p);
    }

private:
    std::mutex mu_;
    std::map<size_t, std::vector<unsigned char *>> free_;
    std::vector<unsigned char *> slabs_;
};

struct Req {
    uint64_t ticket = 0;
    odp_grid grid{};
    odp_dynamics dyn{};
    std::vector<double> tau;
    int rk_order = 1;
    // Host copy of V0 in pinned memory from the server's pool (so that the
    // upload is an asynchronous DMA); the same buffer later receives
    // V(tau_last).
    unsigned char *host = nullptr;
    std::shared_ptr<HostPool> pool;  // owner of `host`; null: plain new[]
    size_t bytes = 0;                         // one grid array (dense, host)
    size_t row = 0, row_pitch = 0, rows = 0;  // last-axis rows: bytes, device pitch, count
    size_t footprint = 0;                     // device bytes while running
    int state = R_QUEUED;
    int rc = ODP_OK;
    bool cancel = false;
    odp_solve_stats stats{};
    Clock::time_point t_submit, t_admit, t_ready, t_ran;
    int tick_steps = 0;                       // steps of the tick being planned
    // scheduler-owned while running
    unsigned char *dmem = nullptr;
    size_t off_v0 = 0, off_a = 0;
    int slot = -1;
    Plan plan;
    int64_t nsteps = 0, step = 0;
    hipEvent_t ev = nullptr;  // admission, then retirement, done
    ~Req() {
        if (pool) pool->put(host, bytes);
        else delete[] host;
        if (ev) (void)hipEventDestroy(ev);
    }
};

// Pinned host staging whose last transfer is marked by an event.
struct Staging {
    unsigned char *p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
};

}  // namespace

struct odp_server {
    odp_solve_opts opts{};
    size_t budget = 0;
    int max_slots = 0;
    int device = 0;
    hipStream_t st = nullptr;   // ticks (lane 0)
    hipStream_t st2 = nullptr;  // ticks (lane 1), forked from and joined into st
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    hipStream_t ust = nullptr;  // admissions
    hipStream_t dst = nullptr;  // retirements
    SolveDesc *d_slots = nullptr;
    int64_t *d_nsteps = nullptr;
    int64_t *h_nsteps = nullptr;  // pinned, one per slot
    uint32_t *d_tiles = nullptr;  // [cap] solve slot, [cap] local tile
    int32_t *d_list = nullptr;    // [2 max_slots] per-group member slots, then each
                                  // member's steps in the tick (same order)
    size_t tile_cap = 0;
    Staging tab[2];               // tile tables on their way to the device
    int tab_next = 0;
    std::vector<Staging> up;      // per slot: descriptor image sent up
    std::vector<Staging> back;    // per slot: state and schedule read back
    std::shared_ptr<HostPool> pool = std::make_shared<HostPool>();  // request host buffers

    std::mutex mu;
    std::condition_variable cv;
    std::deque<std::shared_ptr<Req>> queue;
    std::map<uint64_t, std::shared_ptr<Req>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    int running = 0, done = 0;

    // scheduler thread only
    std::vector<std::shared_ptr<Req>> admitting, active, retiring;
    std::deque<hipEvent_t> ticks;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> free_slots;
    size_t used = 0;
    std::thread th;
};

namespace {

struct Group {
    int dyn, ndim, vec, rk, lds;
    int lane = 0;                  // 0: launched on st, 1: on st2
    std::vector<int> slots;        // members, by this tick's step count (descending)
    std::vector<int> steps;        // their step counts in this tick
    std::vector<uint32_t> prefix;  // prefix[m]: tiles of the first m members
    uint32_t tiles = 0;
    size_t tile_base = 0, list_base = 0;
    int box_parts = 1;             // blocks per member of the box CFL step (pursuit-evasion)
};

int get_event(odp_server *s, hipEvent_t *ev) {
    if (!s->ev_pool.empty()) {
        *ev = s->ev_pool.back();
        s->ev_pool.pop_back();
        return ODP_OK;
    }
    return check_hip(hipEventCreateWithFlags(ev, hipEventDisableTiming), "event");
}

void put_event(odp_server *s, hipEvent_t &ev) {
    if (ev) s->ev_pool.push_back(ev);
    ev = nullptr;
}

// Grow a pinned staging buffer after its last transfer has finished.
int stage_reserve(Staging &b, size_t need) {
    int rc;
    if (b.pending) {
        if ((rc = check_hip(hipEventSynchronize(b.ev), "staging"))) return rc;
        b.pending = false;
    }
    if (need <= b.cap) return ODP_OK;
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.cap = 0;
    const size_t cap = std::max<size_t>(need, 4096);
    if ((rc = check_hip(hipHostMalloc((void **)&b.p, cap, hipHostMallocDefault), "pinned staging"))) return rc;
    b.cap = cap;
    return ODP_OK;
}

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
    // many requests share every launch: blocks march 16 planes (each tile
    // reads two planes beyond its chunk, and a short chunk makes them a
    // large share: at 8 planes the 4D stage launches fetched 1.13-1.25x their
    // stencil input; measured at 200 requests/s, p99 with 8 / 12 / 16 / 20 /
    // 24 planes: 118-124 / 118 / 107-109 / 111 / 117 ms, half the axis 172
    // ms, the whole axis (too few tiles) 868 ms)
    int chunk = o.tile_chunk;
    if (chunk <= 0) chunk = int(std::min<int64_t>(16, r.grid.n[0]));
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
    const Clock::time_point now = Clock::now();
    auto ms = [](Clock::time_point a, Clock::time_point b) {
        return a.time_since_epoch().count() && b.time_since_epoch().count()
                   ? std::chrono::duration<double, std::milli>(b - a).count()
                   : 0.0;
    };
    r->stats.latency_ms = ms(r->t_submit, now);
    r->stats.queue_ms = ms(r->t_submit, r->t_admit);
    r->stats.admit_ms = ms(r->t_admit, r->t_ready);
    r->stats.run_ms = ms(r->t_ready, r->t_ran);
    r->stats.retire_ms = ms(r->t_ran, now);
    s->running--;
    s->done++;
}

// Release the request's device memory and slot.  Callers guarantee that no
// work still in flight on any stream touches either (the last use has
// completed, or every stream has been synchronised).
void release(odp_server *s, const std::shared_ptr<Req> &r) {
    if (r->dmem) (void)hipFreeAsync(r->dmem, s->ust);
    r->dmem = nullptr;
    if (r->slot >= 0) s->free_slots.push_back(r->slot);
    r->slot = -1;
    s->used -= r->footprint;
    put_event(s, r->ev);
}

// Enqueue the admission of every queued request that fits (upload stream).
void admit(odp_server *s) {
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
            r->t_admit = Clock::now();
            s->running++;
            take.push_back(r);
            s->queue.pop_front();
        }
    }
    const odp_solve_opts &o = s->opts;
    for (auto &r : take) {
        void *mem = nullptr;
        if (hipMallocAsync(&mem, r->footprint, s->ust) != hipSuccess) {
            (void)hipGetLastError();
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
        std::vector<unsigned char> img;
        plan_image(r->plan, r->dmem, img);
        SolveDesc *slot = s->d_slots + r->slot;
        // every source is pinned, so each copy is a DMA in stream order; the
        // slot's staging is reused only after this admission has finished
        Staging &up = s->up[size_t(r->slot)];
        int rc = stage_reserve(up, img.size());
        if (rc == ODP_OK) std::memcpy(up.p, img.data(), img.size());
        if (rc ||
            (rc = check_hip(hipMemcpy2DAsync(r->dmem + r->off_v0, r->row_pitch, r->host, r->row, r->row, r->rows,
                                             hipMemcpyHostToDevice, s->ust), "V0")) ||
            (rc = check_hip(hipMemcpyAsync(r->dmem, up.p, img.size(), hipMemcpyHostToDevice, s->ust), "image")) ||
            (rc = check_hip(hipMemcpyAsync(slot, up.p + r->plan.desc_off, sizeof(SolveDesc),
                                           hipMemcpyHostToDevice, s->ust), "slot")) ||
            (rc = check_hip(launch_init(slot, 1, s->ust), "init")) ||
            (rc = check_hip(launch_alpha(r->dyn.id, r->grid.ndim, slot, 1,
                                         int(std::min<int64_t>(2048, (it.qpad + kBlock - 1) / kBlock)), s->ust),
                            "alpha")) ||
            (rc = check_hip(launch_sched(slot, 1, s->d_nsteps + r->slot, s->ust), "schedule")) ||
            (rc = check_hip(launch_start_copy(o.precision, slot, nullptr, nullptr, it.tiles, s->ust), "start copy")) ||
            (rc = get_event(s, &r->ev)) || (rc = check_hip(hipEventRecord(r->ev, s->ust), "record"))) {
            (void)hipStreamSynchronize(s->ust);
            release(s, r);
            finish(s, r, rc);
            continue;
        }
        s->admitting.push_back(r);
    }
}

// Admissions whose prologue has finished join the active set.
bool poll_admissions(odp_server *s) {
    bool joined = false;
    for (size_t i = 0; i < s->admitting.size();) {
        auto r = s->admitting[i];
        if (hipEventQuery(r->ev) != hipSuccess) {
            ++i;
            continue;
        }
        put_event(s, r->ev);
        s->admitting.erase(s->admitting.begin() + long(i));
        bool cancel;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            cancel = r->cancel;
        }
        // the step count from the host's copy of the schedule (box_cfl: the
        // all-inputs count, a bound; finished solves' launches return early)
        r->nsteps = r->plan.items[0].nsteps;
        r->step = 0;
        if (cancel || r->nsteps <= 0) {
            release(s, r);
            finish(s, r, cancel ? ODP_ECANCELED : set_error(ODP_EHIP, "server: schedule overflow"));
            continue;
        }
        r->t_ready = Clock::now();
        s->active.push_back(r);
        joined = true;
    }
    return joined;
}

// Enqueue the read-back of a request that the tick marked by `after`
// finishes (download stream).
int start_retire(odp_server *s, const std::shared_ptr<Req> &r, hipEvent_t after) {
    const PlanItem &it = r->plan.items[0];
    Staging &b = s->back[size_t(r->slot)];
    int rc;
    if ((rc = stage_reserve(b, kStateBytes)) ||
        (rc = check_hip(hipStreamWaitEvent(s->dst, after, 0), "wait")) ||
        // a box_cfl first-order result after an odd step count is in B
        (it.box_cfl && (rc = check_hip(launch_box_finish(s->opts.precision, s->d_slots + r->slot, nullptr, nullptr,
                                                         it.tiles, s->dst), "box finish"))) ||
        (rc = check_hip(hipMemcpy2DAsync(r->host, r->row, r->dmem + r->off_a, r->row_pitch, r->row, r->rows,
                                         hipMemcpyDeviceToHost, s->dst), "result")) ||
        (rc = check_hip(hipMemcpyAsync(b.p, r->dmem + it.state_off, kStateBytes, hipMemcpyDeviceToHost, s->dst),
                        "state")) ||
        (rc = get_event(s, &r->ev)) || (rc = check_hip(hipEventRecord(r->ev, s->dst), "record")))
        return rc;
    r->t_ran = Clock::now();
    s->retiring.push_back(r);
    return ODP_OK;
}

// Retirements whose read-back has finished: statistics, release, done.
void poll_retirements(odp_server *s) {
    for (size_t i = 0; i < s->retiring.size();) {
        auto r = s->retiring[i];
        if (hipEventQuery(r->ev) != hipSuccess) {
            ++i;
            continue;
        }
        s->retiring.erase(s->retiring.begin() + long(i));
        const unsigned char *b = s->back[size_t(r->slot)].p;
        odp_solve_stats &sx = r->stats;
        int64_t nst;
        std::memcpy(&nst, b + kMaxDim * 8, 8);
        int32_t flags;
        std::memcpy(&flags, b + kMaxDim * 8 + 16, 4);
        const bool bad_steps = (flags & kFlagStepsExceeded) || nst <= 0 || nst > r->nsteps;
        if (bad_steps) nst = std::max<int64_t>(0, std::min(nst, r->nsteps));
        sx.steps = nst;
        if (nst > 0) {
            std::memcpy(&sx.dt_min, b + kMaxDim * 8 + 24, 8);
            std::memcpy(&sx.dt_max, b + kMaxDim * 8 + 32, 8);
        }
        sx.t_final = r->tau.back();
        sx.alg_bytes = alg_bytes_per_step(s->opts.precision, r->rk_order,
                                          method_arrays(s->opts) + box_reads(r->dyn.id, s->opts, r->rk_order),
                                          r->grid.npts) *
                       double(nst);
        std::memcpy(sx.alpha_max, b, sizeof(sx.alpha_max));
        sx.nonfinite = flags & kFlagNonFinite;
        release(s, r);
        finish(s, r, bad_steps ? ODP_EHIP : sx.nonfinite ? ODP_ENONFINITE : ODP_OK);
    }
}

// Kernel groups and tile tables of the selected requests; the tables go to
// the device on the compute stream, after the ticks already in flight.
// Within a group the members are ordered by their step count in this tick,
// largest first, so that the members still stepping at step m of the tick
// are a prefix of its tile table and of its member list.
int build_groups(odp_server *s, const std::vector<std::shared_ptr<Req>> &sel, std::vector<Group> &groups) {
    groups.clear();
    std::map<std::tuple<int, int, int, int, int>, size_t> idx;
    std::vector<const Req *> by_slot(size_t(s->max_slots), nullptr);
    for (auto &r : sel) {
        const PlanItem &it = r->plan.items[0];
        by_slot[size_t(r->slot)] = r.get();
        auto key = std::make_tuple(r->dyn.id, r->grid.ndim, it.vec, it.rk_order, it.lds);
        auto f = idx.find(key);
        if (f == idx.end()) {
            idx[key] = groups.size();
            Group g;
            g.dyn = r->dyn.id;
            g.ndim = r->grid.ndim;
            g.vec = it.vec;
            g.rk = it.rk_order;
            g.lds = it.lds;
            groups.push_back(g);
            f = idx.find(key);
        }
        groups[f->second].slots.push_back(r->slot);
    }
    for (Group &g : groups) {
        std::stable_sort(g.slots.begin(), g.slots.end(), [&](int a, int b) {
            return by_slot[size_t(a)]->tick_steps > by_slot[size_t(b)]->tick_steps;
        });
    }
    // Groups of 4D-and-up requests with two or more members split in two
    // halves of about equal tiles (each keeps the descending step order);
    // the groups then go to two lanes (streams) by their work in the tick,
    // the larger first onto the lighter lane.  Two lanes overlap one
    // launch's ramp and tail with the other's body: measured on batches of
    // the served 4D requests, 2 and 4 requests at 0.445 / 0.455 of the
    // roofline on one stream, 0.490 / 0.487 on two (four streams: no
    // better than one); 3D requests beside 4D ones on a stream of their
    // own hid half of their time.  3D groups stay whole: their launches
    // are short and launch-bound.
    const size_t ng = groups.size();
    for (size_t gi = 0; gi < ng; ++gi) {
        if (groups[gi].ndim < 4 || groups[gi].slots.size() < 2) continue;
        Group h = groups[gi];
        h.slots.clear();
        std::vector<int> keep;
        uint64_t ta = 0, tb = 0;
        for (int sl : groups[gi].slots) {
            const uint64_t t = by_slot[size_t(sl)]->plan.items[0].tiles;
            if (ta <= tb) {
                keep.push_back(sl);
                ta += t;
            } else {
                h.slots.push_back(sl);
                tb += t;
            }
        }
        groups[gi].slots = keep;
        groups.push_back(h);
    }
    std::vector<double> gw(groups.size(), 0.0);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group &g = groups[gi];
        g.steps.clear();
        g.box_parts = 1;
        for (int sl : g.slots) {
            const Req *r = by_slot[size_t(sl)];
            g.steps.push_back(r->tick_steps);
            g.box_parts = std::max(g.box_parts, box_parts(&r->grid));
            gw[gi] += double(r->tick_steps) * double(r->plan.items[0].ppad) * double(r->plan.items[0].rk_order);
        }
    }
    std::vector<size_t> gorder(groups.size());
    for (size_t gi = 0; gi < gorder.size(); ++gi) gorder[gi] = gi;
    std::stable_sort(gorder.begin(), gorder.end(), [&](size_t a, size_t b) { return gw[a] > gw[b]; });
    double lw[2] = {0.0, 0.0};
    for (size_t gi : gorder) {
        const int l = lw[1] < lw[0] ? 1 : 0;
        groups[gi].lane = l;
        lw[l] += gw[gi];
    }
    size_t ntiles = 0;
    for (auto &r : sel) ntiles += r->plan.items[0].tiles;
    int rc;
    if (ntiles > s->tile_cap) {
        // the old tables may still be read by a tick in flight
        if ((rc = check_hip(hipStreamSynchronize(s->st), "sync"))) return rc;
        const size_t cap = std::max(ntiles, 2 * s->tile_cap);
        if (s->d_tiles) (void)hipFree(s->d_tiles);
        s->d_tiles = nullptr;
        s->tile_cap = 0;
        if ((rc = check_hip(hipMalloc(&s->d_tiles, cap * 8), "tile tables"))) return rc;
        s->tile_cap = cap;
    }
    Staging &b = s->tab[s->tab_next];
    s->tab_next ^= 1;
    if ((rc = stage_reserve(b, ntiles * 8 + sel.size() * 8))) return rc;
    uint32_t *ts = (uint32_t *)b.p, *tl = ts + ntiles;
    int32_t *list = (int32_t *)(tl + ntiles);
    int32_t *inc = list + sel.size();
    size_t nt = 0, nl = 0;
    for (Group &g : groups) {
        g.tile_base = nt;
        g.list_base = nl;
        g.prefix.assign(1, 0);
        for (int sl : g.slots) {
            const uint32_t t = by_slot[size_t(sl)]->plan.items[0].tiles;
            for (uint32_t k = 0; k < t; ++k) {
                ts[nt] = uint32_t(sl);
                tl[nt++] = k;
            }
            inc[nl] = by_slot[size_t(sl)]->tick_steps;
            list[nl++] = sl;
            g.prefix.push_back(uint32_t(nt - g.tile_base));
        }
        g.tiles = uint32_t(nt - g.tile_base);
    }
    if (ntiles == 0) return ODP_OK;
    if ((rc = check_hip(hipMemcpyAsync(s->d_tiles, ts, ntiles * 4, hipMemcpyHostToDevice, s->st), "tiles")) ||
        (rc = check_hip(hipMemcpyAsync(s->d_tiles + s->tile_cap, tl, ntiles * 4, hipMemcpyHostToDevice, s->st),
                        "tiles")) ||
        (rc = check_hip(hipMemcpyAsync(s->d_list, list, nl * 4, hipMemcpyHostToDevice, s->st), "list")) ||
        (rc = check_hip(hipMemcpyAsync(s->d_list + s->max_slots, inc, nl * 4, hipMemcpyHostToDevice, s->st),
                        "tick steps")) ||
        (rc = check_hip(hipEventRecord(b.ev, s->st), "record")))
        return rc;
    b.pending = true;
    return ODP_OK;
}

int enqueue_tick(odp_server *s, const std::vector<Group> &groups, hipEvent_t *done) {
    const odp_solve_opts &o = s->opts;
    const int mk = method_kind(o);
    int rc;
    int most = 0;
    bool two = false;
    for (const Group &g : groups) {
        if (!g.steps.empty()) most = std::max(most, g.steps.front());
        two = two || (g.lane == 1 && !g.steps.empty());
    }
    // lane 1 starts after everything already on st (tables, earlier ticks)
    if (two && ((rc = check_hip(hipEventRecord(s->fork_ev, s->st), "record")) ||
                (rc = check_hip(hipStreamWaitEvent(s->st2, s->fork_ev, 0), "wait"))))
        return rc;
    for (int m = 0; m < most; ++m) {
        for (const Group &g : groups) {
            // members with more than m steps in this tick: a prefix
            int nm = 0;
            while (nm < int(g.steps.size()) && g.steps[size_t(nm)] > m) ++nm;
            if (nm == 0) continue;
            const uint32_t nt = g.prefix[size_t(nm)];
            const uint32_t *ts = s->d_tiles + g.tile_base, *tl = s->d_tiles + s->tile_cap + g.tile_base;
            hipStream_t q = g.lane ? s->st2 : s->st;
            for (int j = 0; j < g.rk; ++j) {
                const int kind = stage_kind(g.rk, j, mk, g.lds, o.space_order == 2);
                // pursuit-evasion: the costate box of each solve's stage input
                // first (each solve's own step counter picks its box buffer)
                // (step m of the tick: the solve's counter holds the tick's first step)
                if (g.dyn == ODP_DYN_PE3D && !o.dissipation &&
                    ((rc = check_hip(launch_stage(o.precision, g.dyn, g.ndim, g.vec, kind | 32, s->d_slots, ts, tl,
                                                  nt, j, 1, m, o.xcd_group, q),
                                     "box")) ||
                     // the step from the box of the first stage (Algorithm 1)
                     (j == 0 && (rc = check_hip(launch_box_dt(s->d_slots, s->d_list + g.list_base, nm, g.box_parts, 1, m, q),
                                                "box step")))))
                    return rc;
                if ((rc = check_hip(launch_stage(o.precision, g.dyn, g.ndim, g.vec, kind, s->d_slots, ts, tl, nt, j,
                                                 1, m, o.xcd_group, q),
                                    "stage")))
                    return rc;
            }
        }
    }
    // one advance per group: every member by its steps in the tick
    for (const Group &g : groups) {
        if (g.steps.empty()) continue;
        if ((rc = check_hip(launch_advance(s->d_slots, s->d_list + g.list_base, s->d_list + s->max_slots + g.list_base,
                                           int(g.steps.size()), g.lane ? s->st2 : s->st),
                            "advance")))
            return rc;
    }
    // the tick ends when both lanes have
    if (two && ((rc = check_hip(hipEventRecord(s->join_ev, s->st2), "record")) ||
                (rc = check_hip(hipStreamWaitEvent(s->st, s->join_ev, 0), "wait"))))
        return rc;
    if ((rc = get_event(s, done))) return rc;
    if ((rc = check_hip(hipEventRecord(*done, s->st), "record"))) put_event(s, *done);
    return rc;
}

void drain(odp_server *s) {
    (void)hipStreamSynchronize(s->st2);
    (void)hipStreamSynchronize(s->st);
    (void)hipStreamSynchronize(s->ust);
    (void)hipStreamSynchronize(s->dst);
    for (hipEvent_t &e : s->ticks) put_event(s, e);
    s->ticks.clear();
}

// Finish every request the scheduler holds with `rc` (after the device has
// drained; completed retirements keep their own result).
void fail_all(odp_server *s, int rc) {
    drain(s);
    poll_retirements(s);
    for (auto *v : {&s->admitting, &s->active, &s->retiring}) {
        for (auto &r : *v) {
            release(s, r);
            finish(s, r, rc);
        }
        v->clear();
    }
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
            if (s->active.empty() && s->queue.empty() && s->admitting.empty() && s->retiring.empty()) {
                s->cv.wait_for(lk, std::chrono::milliseconds(20));
                continue;
            }
        }
        poll_retirements(s);
        admit(s);
        if (poll_admissions(s)) dirty = true;
        // cancellations of running requests
        bool cancelled = false;
        for (auto &r : s->active) {
            std::lock_guard<std::mutex> lk(s->mu);
            cancelled |= r->cancel;
        }
        if (cancelled) {
            (void)hipStreamSynchronize(s->st);  // no tick may still read them
            for (hipEvent_t &e : s->ticks) put_event(s, e);
            s->ticks.clear();
            for (size_t i = 0; i < s->active.size();) {
                auto r = s->active[i];
                bool c;
                {
                    std::lock_guard<std::mutex> lk(s->mu);
                    c = r->cancel;
                }
                if (c) {
                    s->active.erase(s->active.begin() + long(i));
                    release(s, r);
                    finish(s, r, ODP_ECANCELED);
                } else {
                    ++i;
                }
            }
            dirty = true;
        }
        if (s->active.empty()) {
            if (!s->admitting.empty() || !s->retiring.empty())
                std::this_thread::sleep_for(std::chrono::microseconds(50));
            continue;
        }
        // wait for a tick slot without blocking: finished retirements and
        // admissions are picked up (and new arrivals admitted) meanwhile, so
        // their results and prologues are not held until the tick ends
        while (int(s->ticks.size()) >= kTicksInFlight) {
            if (hipEventQuery(s->ticks.front()) == hipSuccess) {
                put_event(s, s->ticks.front());
                s->ticks.pop_front();
                continue;
            }
            poll_retirements(s);
            admit(s);
            if (poll_admissions(s)) dirty = true;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
        }
        // This tick advances the requests in arrival order, up to about
        // kTickWork point-stage updates (at least one request; requests that
        // do not fit are passed over, so later small ones still join; any
        // request waiting longer than kMaxWaitMs joins anyway).  Measured at
        // 200 requests/s (p50 / p99 ms, two lanes, 8-plane chunks; 16-plane
        // chunks then took 0.75e9 to 14.1 / 109): least remaining work
        // first with a budget of 2e9, 17.5 / 140; arrival order with 2e9,
        // 17.7 / 145; with 1e9, 16.5 / 124; with 0.75e9, 14.4 / 119; with
        // 0.5e9, 12.1 / 148 (the launches get too small); least remaining
        // work with 1e9: 16.1 / 128, but the largest requests starve (max
        // 264 ms).  The p99 is set by the largest 4D requests, and the order
        // of arrival bounds their wait.
        std::vector<std::shared_ptr<Req>> order = s->active, sel;
        auto work = [](const std::shared_ptr<Req> &r, int64_t steps) {
            return double(steps) * double(r->plan.items[0].ppad) * double(r->plan.items[0].rk_order);
        };
        std::stable_sort(order.begin(), order.end(), [](const std::shared_ptr<Req> &a, const std::shared_ptr<Req> &b) {
            return a->t_submit < b->t_submit;
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
        // steps of each selected request in this tick: kStepsPerTick, or up
        // to kSmallStepsPerTick for a request whose extra steps cost under 2%
        // of the tick's work (small grids then finish in fewer ticks instead
        // of advancing at the large requests' pace; measured: p50 28.5 ->
        // 22.8 ms at the same p99); members with fewer steps drop out of the
        // tick's later launches
        double base = 0.0;
        for (auto &r : sel) base += work(r, std::min<int64_t>(kStepsPerTick, r->nsteps - r->step));
        std::vector<uint64_t> sel_ids;
        for (auto &r : sel) {
            const bool small = work(r, kSmallStepsPerTick - kStepsPerTick) <= 0.02 * base;
            r->tick_steps = int(std::min<int64_t>(small ? kSmallStepsPerTick : kStepsPerTick, r->nsteps - r->step));
            sel_ids.push_back(r->ticket);
            sel_ids.push_back(uint64_t(r->tick_steps));
        }
        if (sel_ids != last_sel) dirty = true;
        if (dirty) {
            if (build_groups(s, sel, groups) != ODP_OK) {
                fail_all(s, ODP_EHIP);
                last_sel.clear();
                continue;
            }
            last_sel = sel_ids;
            dirty = false;
        }
        hipEvent_t tick_done = nullptr;
        if (enqueue_tick(s, groups, &tick_done) != ODP_OK) {
            fail_all(s, ODP_EHIP);
            dirty = true;
            continue;
        }
        s->ticks.push_back(tick_done);
        for (auto &r : sel) r->step = std::min<int64_t>(r->step + r->tick_steps, r->nsteps);
        for (size_t i = 0; i < s->active.size();) {
            auto r = s->active[i];
            if (r->step >= r->nsteps) {
                s->active.erase(s->active.begin() + long(i));
                dirty = true;
                if (start_retire(s, r, tick_done) != ODP_OK) {
                    (void)hipStreamSynchronize(s->st);
                    (void)hipStreamSynchronize(s->dst);
                    release(s, r);
                    finish(s, r, ODP_EHIP);
                }
            } else {
                ++i;
            }
        }
    }
    // shutdown: let the device drain, keep finished results, cancel the rest
    drain(s);
    poll_retirements(s);
    for (auto *v : {&s->admitting, &s->active, &s->retiring}) {
        for (auto &r : *v) {
            release(s, r);
            finish(s, r, ODP_ECANCELED);
        }
        v->clear();
    }
    (void)hipStreamSynchronize(s->ust);
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto &r : s->queue) {
        r->rc = ODP_ECANCELED;
        r->state = R_DONE;
    }
    s->queue.clear();
}

void destroy_resources(odp_server *s) {
    if (s->d_tiles) (void)hipFree(s->d_tiles);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->d_nsteps) (void)hipFree(s->d_nsteps);
    if (s->d_list) (void)hipFree(s->d_list);
    if (s->h_nsteps) (void)hipHostFree(s->h_nsteps);
    for (Staging &b : s->tab) {
        if (b.p) (void)hipHostFree(b.p);
        if (b.ev) (void)hipEventDestroy(b.ev);
    }
    for (auto *v : {&s->up, &s->back})
        for (Staging &b : *v)
            if (b.p) (void)hipHostFree(b.p);
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    s->ev_pool.clear();
    for (hipEvent_t e : {s->fork_ev, s->join_ev})
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t *q : {&s->st, &s->st2, &s->ust, &s->dst})
        if (*q) (void)hipStreamDestroy(*q);
}

}  // namespace

extern "C" {

int odp_server_create(size_t hbm_budget_bytes, int max_slots, const odp_solve_opts *opts, odp_server **out) {
    if (!out) return set_error(ODP_EINVAL, "out is NULL");
    *out = nullptr;
    int rc;
    if ((rc = validate_opts(opts))) return rc;
    if (opts->save_all) return set_error(ODP_EUNSUPPORTED, "save_all is not available when serving");
    if (opts->target_dev || opts->obstacle_dev)
        return set_error(ODP_EUNSUPPORTED, "target and obstacle arrays belong to one grid: use odp_hj_solve");
    if (max_slots < 1 || max_slots > 4096) return set_error(ODP_EINVAL, "max_slots must be in [1, 4096]");
    if (hbm_budget_bytes == 0) return set_error(ODP_EINVAL, "the HBM budget must be positive");
    std::unique_ptr<odp_server> s(new odp_server());
    s->opts = *opts;
    s->opts.stream = nullptr;
    s->budget = hbm_budget_bytes;
    s->max_slots = max_slots;
    s->up.resize(size_t(max_slots));
    s->back.resize(size_t(max_slots));
    if ((rc = check_hip(hipGetDevice(&s->device), "device")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking), "stream")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&s->st2, hipStreamNonBlocking), "stream")) ||
        (rc = check_hip(hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming), "event")) ||
        (rc = check_hip(hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming), "event")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&s->ust, hipStreamNonBlocking), "stream")) ||
        (rc = check_hip(hipStreamCreateWithFlags(&s->dst, hipStreamNonBlocking), "stream")) ||
        (rc = check_hip(hipMalloc(&s->d_slots, sizeof(SolveDesc) * size_t(max_slots)), "slots")) ||
        (rc = check_hip(hipMalloc(&s->d_nsteps, 8 * size_t(max_slots)), "slots")) ||
        (rc = check_hip(hipMalloc(&s->d_list, 8 * size_t(max_slots)), "slots")) ||
        (rc = check_hip(hipHostMalloc((void **)&s->h_nsteps, 8 * size_t(max_slots), hipHostMallocDefault), "pinned")) ||
        (rc = check_hip(hipEventCreateWithFlags(&s->tab[0].ev, hipEventDisableTiming), "event")) ||
        (rc = check_hip(hipEventCreateWithFlags(&s->tab[1].ev, hipEventDisableTiming), "event"))) {
        destroy_resources(s.get());
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
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->queue.size() >= kMaxQueue) return set_error(ODP_EAGAIN, "queue full");
    }
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
    if ((r->host = srv->pool->get(r->bytes))) {
        r->pool = srv->pool;
    } else {
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
    drain(srv);
    destroy_resources(srv);
    // requests still held by clients keep their host buffers until released
    delete srv;
}

}  // extern "C"
