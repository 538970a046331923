// A plan: a list of solves laid out in one device workspace, stepped together.
//
// Workspace layout (byte offsets, 256-aligned regions):
//   descriptors   n x SolveDesc, contiguous (kernels index descs[i])
//   step counts   n x int64 (gathered by the schedule kernel)
//   aux           per solve: state (alpha^max, step counters, flags),
//                 axis tables, tau
//   --- everything above is uploaded from one host image ---
//   tile tables   2 x total tiles x uint32 (solve index, local tile), uploaded
//                 once the step counts are known (members sorted by steps)
//   schedules     per solve: dt of every step (float64) and landing index
//   arrays        per solve: B (and C for RK3)
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "runtime.h"

namespace odp {

struct PlanItem {
    const odp_grid *g = nullptr;
    odp_dynamics dyn{};
    const void *V0 = nullptr;
    const void *Vinit = nullptr;
    void *A = nullptr;
    std::vector<double> tau;
    int rk_order = 0;                   // 0: the plan options' order
    int pitch = 0;                      // last-axis row pitch in memory (0: dense)
    int64_t qpad = 0, ppad = 0;         // hyperplane / array elements with padding
    int vec = 1, chunk = 1;
    int lds = 0;                        // the stage kernel's LDS plane exchange (2: quad tiles)
    uint32_t brick = 0;                 // tile_group's brick side (0: row-major tiles)
    uint32_t cube = 0, cube_tiles = 0;  // brick > 0: the cubes of axes 3..5
    uint32_t quad = 0;                  // tile_group's quad layout (then lds == 2)
    uint32_t nqb = 0;                   // tiles per hyperplane
    // pad_io: the caller's V0 and A are dense while `pitch` pads the rows;
    // the plan keeps padded copies (V0p, Ap) and copies in and out itself
    bool pad_io = false;
    size_t V0p_off = 0, Ap_off = 0;
    uint32_t tiles = 0;
    int64_t max_steps = 0;
    int tab_entries = 0;
    size_t state_off = 0, aux_off = 0, sched_off = 0, land_off = 0, box_off = 0, tk_off = 0, B_off = 0, C_off = 0;
    // host side of the schedule: axis tables (x, cos x, sin x per axis, as
    // uploaded), alpha^max and the step count from the same float64
    // arithmetic as the device reduction and schedule, and the output index
    // each step lands on (-1: none)
    std::vector<double> tab;
    double amax[kMaxDim] = {0, 0, 0, 0, 0, 0};
    std::vector<int32_t> land;
    bool box_cfl = false;               // step from the costate box (device, per step)
    int64_t nsteps = 0;                 // steps enqueued (box_cfl: an upper bound)
};

struct PlanGroup {
    int dyn = 0, ndim = 0, vec = 1, rk = 1, lds = 0;
    int box_parts = 1;                  // blocks per member of the box CFL step
    int first = 0, count = 0;           // descriptor range
    std::vector<int> order;             // members sorted by step count, descending
    std::vector<uint32_t> prefix;       // prefix[m] = tiles of order[0..m)
    size_t tile_base = 0;               // first entry in the tile tables
    int lane = 0;                       // batches: 0 on the caller's stream, 1 on a second one
};

struct Plan {
    odp_solve_opts opts{};
    std::vector<PlanItem> items;        // descriptor order (grouped)
    std::vector<PlanGroup> groups;
    size_t desc_off = 0, nsteps_off = 0, state_begin = 0, aux_begin = 0, upload_bytes = 0;
    size_t tt_off = 0, total_tiles = 0, sched_begin = 0, arr_begin = 0, total = 0;
    int64_t max_nsteps = 0;
    int xcd_group = 0;                  // tile runs per XCD for the stage launches
    std::string error;                  // set by plan_build when a schedule overflows
};

// Order items by (dynamics, ndim, vector width, RK order), fill the layout.
// Returns the permutation applied (new index -> caller index).
// round4: round the chunk to whole 4-plane cycles (always for the default).
std::vector<int> plan_build(Plan &p, std::vector<PlanItem> items, const odp_solve_opts &opts,
                            int tile_chunk, bool round4 = false);
// The stage launches of step k for every group (the members that have a
// step k, as in the solve itself).
// Lane-1 groups go to st2 when it is given (else everything to st).
int plan_launch_step(const Plan &p, unsigned char *base, hipStream_t st, int64_t k, hipStream_t st2 = nullptr);
// Host image of [0, upload_bytes) for a workspace at device address base.
void plan_image(const Plan &p, unsigned char *base, std::vector<unsigned char> &img);
// Upload, alpha^max, schedules (stream-ordered: the step counts are known on
// the host from plan_build), member order and tile tables.
// pageable: upload from pageable host memory (no pinned staging).
int plan_prologue(Plan &p, unsigned char *base, hipStream_t st, bool pageable = false);
// Start copies and every step of every solve (stream-ordered, no sync).
// V_all: save_all of a single solve (slice k = V at tau[k]), else null.
int plan_steps(Plan &p, unsigned char *base, hipStream_t st, void *V_all);
// Whether the plan's stepping is recorded into a HIP graph.
bool plan_wants_graph(const Plan &p);
// Fill per-item stats after the stream has been synchronised.
int plan_stats(const Plan &p, unsigned char *base, double kernel_ms, odp_solve_stats *stats, hipStream_t st);


}  // namespace odp
