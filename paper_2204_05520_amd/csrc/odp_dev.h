// Shared host/device layout of libodp's solve descriptors.
//
// A solve is described once (SolveDesc, in device memory) and every stage
// launch covers a list of solves: a single solve is a list of one, a batch
// or a server tick is a list of many.  Blocks map to (solve, tile) through a
// tile table; a tile is a run of `chunk` planes of axis 0 times 256
// consecutive points of the hyperplane spanned by axes 1..ndim-1.
#pragma once

#include <stdint.h>

namespace odp {

constexpr int kMaxDim = 6;
constexpr int kBlock = 256;          // threads per stage block (4 wave64s)
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, blocks dealt round robin
constexpr int kBoxSlots = 64;        // costate box: partial boxes per buffer (blocks
                                     // spread their atomics over them)
// after the two box buffers: the box CFL step's largest box alpha per axis
// (order-preserving keys of non-negative doubles) and its block counter
constexpr int kBoxStepWords = 4;

// n / d for n < 2^31 as (mulhi(n, m) + n) >> s (round-up magic number).
struct FastDiv {
    uint32_t d, m, s, pad_;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t s = 0;
    while ((uint64_t(1) << s) < d) ++s;
    uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1;
    return FastDiv{d, uint32_t(m), s, 0};
}

// Per-axis tables in float64: coordinate x_k, cos x_k, sin x_k.
struct AxisTab {
    int32_t off;  // first entry of this axis in the table buffer (x at off,
                  // cos at off + n, sin at off + 2n)
    int32_t n;
};

struct SolveDesc {
    // ---- shape
    int32_t ndim;
    int32_t n0;              // nodes on axis 0 (the marched axis)
    uint32_t Q;              // elements per hyperplane of axes 1..ndim-1 (with padding)
    uint32_t periodic;       // bit d set: axis d periodic
    int32_t pitch;           // elements per last-axis row in memory (>= n[ndim-1];
                             // the elements beyond n[ndim-1] are padding)
    int32_t lds;             // 1: the marching kernel exchanges each plane of a
                             // block's range through LDS (ndim >= 3, pitch <= 128 vec)
    int64_t s0;              // stride of axis 0 (= Q)
    int64_t npts;
    int32_t n[kMaxDim];      // nodes per axis
    int32_t stride[kMaxDim]; // strides of axes 1..ndim-1 (entry 0 unused)
    FastDiv div[kMaxDim];    // divisors of the in-plane decomposition (pitch for the last axis)
    double inv2dx[kMaxDim];  // 1 / (2 dx_d)
    double dx[kMaxDim];
    AxisTab tab[kMaxDim];
    // ---- tiling
    int32_t chunk;           // planes of axis 0 per tile
    int32_t vec;             // consecutive last-axis points per thread
    uint32_t nqb;            // tiles per hyperplane (256 groups of vec elements each)
    uint32_t tiles;          // nqb * ceil(n0 / chunk)
    int32_t rk_order;
    uint32_t brick;          // 0: row-major tiles; k > 0 (six dimensions): tiles aligned
                             // to the cubes of axes 3..5, dealt in k x k squares of
                             // axes 1 and 2 (tile_group)
    uint32_t cube;           // brick > 0: elements per cube of axes 3..5
    uint32_t cube_tiles;     // brick > 0: tiles per cube, ceil(cube / span), span =
                             // 256 vec, or 64 vec with quad
    uint32_t quad;           // brick > 0 (even): a tile's four waves take the 2x2
                             // (axis 1, axis 2) pairs of a square at one cube offset
    uint32_t pad0_;
    // ---- dynamics
    int32_t dyn;
    int32_t u_mode, d_mode;
    int32_t global_alpha;
    double p[16];
    // ---- device memory (element type per launch)
    void *A;                 // V^n (caller's V_out)
    void *B;                 // stage 1 output / ping-pong partner
    void *C;                 // stage 2 output (RK3)
    const void *V0;
    const void *Vinit;       // start value (V0 unless restarting)
    const void *Vsrc_dense;  // caller's dense V0 when V0/A are padded copies (else null):
                             // the start copy fills V0 and the start buffer from it
    void *Adst_dense;        // caller's dense V_out when A is a padded copy (else null)
    const double *tabd;      // axis tables (float64)
    double *amax;            // alpha^max per axis (float64 bits, atomically maxed)
    double *dt_sched;        // dt of every step
    int32_t *land;           // tau index reached by each step, -1 if none
    int64_t *nsteps;         // device: step count of the schedule
    int64_t *step;           // device: next step to take (server ticks)
    int32_t *flags;          // kFlag* bits
    double *dtmm;            // smallest and largest step of the schedule
    uint64_t *box;           // costate box (pursuit-evasion only, else null): two
                             // buffers, used by alternate stages, of kBoxSlots
                             // partial boxes of 6 order-preserving keys each
                             // (D_min[3], then D_max[3]), then kBoxStepWords
                             // words for the box CFL step
    // ---- computation method: after every full step (the last stage) V is
    // compared with a reference point by point and replaced by the smaller
    // (or larger) of the two; then, optionally, again with an obstacle array
    int32_t tclamp;          // 1: the last stage compares (kind bit 1)
    int32_t tmax;            // 1: keep the larger value, 0: the smaller
    int32_t tvn;             // 1: the reference is V^n, the value before the step
                             // (then tref is any grid-sized array)
    int32_t obst;            // 1: a second comparison with oref follows (kind bit 3)
    int32_t omax;            // 1: keep the larger value, 0: the smaller
    int32_t ntau;
    const void *tref;        // reference array when tvn == 0 (V0, a target array,
                             // or the obstacle array of an obstacle-only method)
    const void *oref;        // obstacle array when obst == 1
    // time-varying sets: tref / oref point at the slice of the current tau
    // interval, set between steps from the slice-0 bases and the strides
    // (elements between slices; 0 for a reference that does not vary)
    const void *tref0;
    const void *oref0;
    int64_t tstride;
    int64_t ostride;
    const double *tau;       // output times (device copy)
    double cfl;
    double max_dt;
    int64_t max_steps;       // capacity of dt_sched / land
    int64_t expect_steps;    // steps the host enqueues: the step count of the
                             // schedule, worked out on the host with the same
                             // float64 arithmetic (the device checks it), or,
                             // with box_cfl, the all-inputs count, which
                             // bounds the box schedule's
    // ---- CFL step from the costate box (pursuit-evasion with per-point
    // dissipation, Algorithm 1): every step's dt comes from the largest box
    // alpha over the grid, reduced on the device after the first stage's box
    // pass; the step count is known once time lands on the last output time
    // (nsteps holds max_steps until then)
    int32_t box_cfl;
    int32_t pad1_;
    double *t_after;         // time after each step
    int32_t *k_after;        // output-time index each step's successor aims at
    double pe_cmin, pe_cmax; // min / max over the heading table of -v_a + v_b cos th
    double pe_smin, pe_smax; // min / max over the heading table of v_b sin th
};

// Tile qb of a hyperplane, thread t (0..kBlock-1): the element offset q0 of
// the tile's first group, the offset q of the thread's group of vec
// consecutive elements, and whether that group exists (a thread past the end
// takes the last group of its range, for loads only).
//   brick == 0: tiles of kBlock groups in row-major order.
//   brick == k: each cube of axes 3..5 (a fixed pair of axis-1 and axis-2
//   indices) is cut into cube_tiles tiles, the last one ragged; tiles are
//   numbered square by square of k x k (axis 1, axis 2) pairs, within a
//   square by tile of the cube, then by pair.  Consecutive tiles, which the
//   XCD-aware launch keeps on one XCD, are then each other's neighbours
//   along axes 1 and 2 (and, one tile of the cube further, axis 3), so those
//   neighbour loads hit that XCD's L2.
//   quad (k even): a tile is 4 waves of 64 groups; wave w takes the pair
//   (2 b1 + (w >> 1), 2 b2 + (w & 1)) of a 2x2 block (b1, b2) of the square,
//   all four at the same offset in their cubes, so each wave's neighbours
//   along axes 1 and 2 on one side are another wave's values; tiles are
//   numbered square by square, then by cube tile, then by 2x2 block.  q0 is
//   the start of the thread's wave's range.
struct TileGroup {
    uint32_t q0, q;
    bool active;
};

__host__ __device__ inline TileGroup tile_group(const SolveDesc &s, uint32_t qb, uint32_t t, uint32_t vec) {
    TileGroup r;
    const uint32_t span = uint32_t(kBlock) * vec;
    if (s.quad) {
        const uint32_t ws = 64u * vec;  // a wave's range
        const uint32_t hk = s.brick / 2u, nbq = hk * hk;
        const uint32_t per = nbq * s.cube_tiles;
        const uint32_t sq = qb / per, rem = qb - sq * per;
        const uint32_t j = rem / nbq, b = rem - j * nbq;
        const uint32_t b1 = b / hk, b2 = b - b1 * hk;
        const uint32_t nsq2 = uint32_t(s.n[2]) / s.brick;
        const uint32_t s1 = sq / nsq2, s2 = sq - s1 * nsq2;
        const uint32_t w = t >> 6, l = t & 63u;
        const uint32_t a1 = s1 * s.brick + 2u * b1 + (w >> 1), a2 = s2 * s.brick + 2u * b2 + (w & 1u);
        const uint32_t base = (a1 * uint32_t(s.n[2]) + a2) * s.cube;
        const uint32_t loc = j * ws + l * vec;
        r.q0 = base + j * ws;
        r.active = loc < s.cube;
        r.q = base + (r.active ? loc : s.cube - vec);
    } else if (s.brick) {
        const uint32_t k = s.brick, kk = k * k;
        const uint32_t per = kk * s.cube_tiles;
        const uint32_t sq = qb / per, rem = qb - sq * per;
        const uint32_t j = rem / kk, pr = rem - j * kk;
        const uint32_t r1 = pr / k, r2 = pr - r1 * k;
        const uint32_t nsq2 = uint32_t(s.n[2]) / k;
        const uint32_t s1 = sq / nsq2, s2 = sq - s1 * nsq2;
        const uint32_t base = ((s1 * k + r1) * uint32_t(s.n[2]) + s2 * k + r2) * s.cube;
        const uint32_t loc = j * span + t * vec;
        r.q0 = base + j * span;
        r.active = loc < s.cube;
        r.q = base + (r.active ? loc : s.cube - vec);
    } else {
        const uint32_t g = qb * uint32_t(kBlock) + t, Qg = s.Q / vec;
        r.q0 = qb * span;
        r.active = g < Qg;
        r.q = (r.active ? g : Qg - 1) * vec;
    }
    return r;
}

// flags bits (SolveDesc::flags)
constexpr int32_t kFlagNonFinite = 1;     // a NaN or Inf was produced
constexpr int32_t kFlagStepsExceeded = 2; // the device schedule needs more steps than were enqueued

}  // namespace odp
