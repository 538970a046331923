// Internal host-side interfaces of libodp (not part of the C ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "odp.h"
#include "odp_dev.h"

struct odp_grid {
    int ndim;
    int64_t n[odp::kMaxDim];
    double lo[odp::kMaxDim], hi[odp::kMaxDim];
    int periodic[odp::kMaxDim];
    double dx[odp::kMaxDim];
    int64_t npts;
};

namespace odp {

// kernels.hip
hipError_t launch_stage(int precision, int dyn, int ndim, int vec, int kind, const SolveDesc *d,
                        const uint32_t *ts, const uint32_t *tl, uint32_t nblocks, int stage,
                        int from_desc, int64_t step, int xgroup, hipStream_t st);
hipError_t launch_alpha(int dyn, int ndim, const SolveDesc *d, int nsolves, int blocks_per_solve,
                        hipStream_t st);
hipError_t launch_init(const SolveDesc *d, int nsolves, hipStream_t st);
hipError_t launch_sched(const SolveDesc *d, int nsolves, int64_t *nsteps_all, hipStream_t st);
hipError_t launch_advance(const SolveDesc *d, const int32_t *list, const int32_t *inc, int n, hipStream_t st);
// Time to reach: one Jacobi sweep (a lane per hyperplane point marching
// `chunk` axis-0 nodes, grid qblocks x ceil(n0 / chunk)), the start value,
// and zeroing of the change slots.
hipError_t launch_ttr(int precision, int dyn, int ndim, const SolveDesc *d, uint32_t qblocks, int n0, int chunk,
                      const void *src, void *dst, const void *target, unsigned long long *change,
                      hipStream_t st);
hipError_t launch_ttr_init(int precision, const void *target, void *phi, int64_t npts, double big,
                           hipStream_t st);
hipError_t launch_ttr_zero(unsigned long long *p, int n, hipStream_t st);
// Solves whose CFL step comes from the costate box (SolveDesc::box_cfl):
// the step of step k from the box of its first stage (one block per listed
// solve: list[j], or descriptor j when list is null; from_desc: each solve's
// own step counter), the final parity copy / landing check over the tiles,
// and the device-conditional save_all copy and set switch of solve 0.
// box CFL step: `parts` blocks per listed solve share its (x, y) nodes
// (box_parts), the last to finish takes the step
hipError_t launch_box_dt(const SolveDesc *d, const int32_t *list, int n, int parts, int from_desc, int64_t step,
                         hipStream_t st);
// Blocks per solve for the box CFL step: one node of (axis 0, axis 1) per thread, at most 1024 blocks.
inline int box_parts(const odp_grid *g) {
    const int64_t nodes = g->n[0] * g->n[1];
    const int64_t b = (nodes + kBlock - 1) / kBlock;
    return int(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}
hipError_t launch_box_finish(int precision, const SolveDesc *d, const uint32_t *ts, const uint32_t *tl,
                             uint32_t nblocks, hipStream_t st);
hipError_t launch_box_save(int precision, const SolveDesc *d, int64_t k, void *V_all, int64_t npts,
                           hipStream_t st);
hipError_t launch_box_slice(int precision, SolveDesc *d, int64_t k, hipStream_t st);
// Time-varying sets of a single solve: references of descs[0] to slice iv.
hipError_t launch_set_slice(int precision, SolveDesc *d, int iv, hipStream_t st);
// Padded members (SolveDesc::Adst_dense set): A to the caller's dense array.
hipError_t launch_finish_copy(int precision, const SolveDesc *d, const uint32_t *ts, const uint32_t *tl,
                              uint32_t nblocks, hipStream_t st);
hipError_t launch_start_copy(int precision, const SolveDesc *d, const uint32_t *ts,
                             const uint32_t *tl, uint32_t nblocks, hipStream_t st);

// runtime.cpp
int set_error(int code, const std::string &msg);
int check_hip(hipError_t e, const char *what);
int validate_dyn(const odp_grid *g, const odp_dynamics *dyn);
int validate_opts(const odp_solve_opts *o);
int validate_tau(const double *tau, int ntau);

// Host-to-device copy on stream st that does not wait: src is first copied
// into a pinned staging block (reused once the event after its last copy has
// completed), so the caller may free src on return.
int upload_async(void *dst, const void *src, size_t bytes, hipStream_t st);

// Upper bound of max_i alpha_d(z_i) from the parameters and the domain.
void alpha_bound(const odp_grid *g, const odp_dynamics *dyn, double *ab);
size_t align256(size_t x);

int default_chunk(const odp_grid *g, int vec, int precision, int space_order = 1);
bool default_chunk_exact(const odp_grid *g, int vec, int precision, int space_order = 1);
int default_xcd_group(const odp_grid *g);
// Points per thread along the last axis: the largest of 4 (float32 only), 2
// and 1 that divides the row pitch (1 for ndim 1 and the ball-input test
// dynamics).
int choose_vec(const odp_grid *g, int precision, int dyn, int64_t pitch);
// narr: grid-sized arrays the computation method reads per step besides the
// stencil input and V^n (method_arrays).
double alg_bytes_per_step(int precision, int rk_order, int narr, int64_t npts);
// Arrays the computation methods of o read per step: V0 or a target array
// for ODP_MIN/MAX_V0 and ODP_MIN/MAX_TARGET, plus the obstacle array.  The
// value-over-time methods compare with V^n, which the step reads anyway.
int method_arrays(const odp_solve_opts &o);
// Stencil-input reads per step of the costate-box passes (pursuit-evasion
// with per-point dissipation: one per Runge-Kutta stage).
inline int box_reads(int dyn, const odp_solve_opts &o, int rk_order) {
    return dyn == ODP_DYN_PE3D && !o.dissipation ? rk_order : 0;
}
// Kind bits of the last stage of a step for these options: bit 1 one
// comparison (a target method, or an obstacle method alone), bit 3 a
// second one (target and obstacle methods together).
int method_kind(const odp_solve_opts &o);
// Stage kind for launch_stage: bit 0 reads V^n, bits 1 and 3 the comparisons
// of the computation method (method_kind, last stage only), bit 2 the LDS
// plane exchange (every listed solve must have SolveDesc::lds set), bit 4
// second-order ENO differences (the point-per-lane kernel), bit 5 (added by
// the caller) the costate-box pass of the pursuit-evasion model.
// lds: 0 none, 1 the LDS plane exchange, 2 the exchange with quad tiles
// (kind bit 6: six dimensions, tile_group's quad layout).
inline int stage_kind(int rk_order, int stage, int mkind, int lds = 0, int eno2 = 0) {
    return (stage > 0 ? 1 : 0) | (stage == rk_order - 1 ? mkind : 0) | (lds ? 4 : 0) | (lds == 2 ? 64 : 0) |
           (eno2 ? 16 : 0);
}
// Whether a solve of this shape uses the LDS plane exchange.
inline int uses_lds(int ndim, int64_t pitch, int vec) { return ndim >= 3 && pitch <= 128 * int64_t(vec) ? 1 : 0; }

}  // namespace odp
