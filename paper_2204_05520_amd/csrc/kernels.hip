// gfx950 kernels of libodp besides the stage kernels: time to reach,
// alpha^max, the CFL schedule, start/finish copies, server step counters,
// and the dispatch of stage launches to the per-(precision, dynamics)
// slices compiled from stage_inst.hip.
#include <algorithm>

#include "kernels_dev.h"
#include "stage_inst.h"

namespace odp {

// ------------------------------------------------ time-to-reach (static)

// One Jacobi iteration of Lax-Friedrichs sweeping for the time to reach
// (the Time-independent HJ PDE subsection's Algorithm 2, with the parallel
// update in place of the serial sweep): from `src` to `dst`.  Off every
// non-periodic edge a node takes
//   min(src_i, [1 + H + sum_d sigma_d (src_{i+e_d} + src_{i-e_d}) / (2 dx_d)]
//              / sum_d sigma_d / dx_d)
// with H = pbar . f(z, u*, d*) at the centred costate and sigma_d the
// largest |f_d|; on a non-periodic edge of axis d it takes
// min(src_i, max(2 src_a - src_b, src_b)) (a, b the next two nodes inward;
// the smallest over its edge axes); target nodes (l <= 0) stay 0.  The
// largest |dst - src| of each block goes to one of kBoxSlots change slots
// (non-negative doubles order as their bits; the host takes the largest).
// Arithmetic in float64, stored as T.
//
// Each lane owns one point q of the hyperplane of axes 1..N-1 and marches
// `chunk` nodes along axis 0 (blockIdx.y selects the run).  No model here
// has dynamics that depend on axis 0, so f, sigma, the denominator and the
// in-plane edge tests are worked out once per lane; every node's own
// arithmetic is the same as with one node per lane.
template <typename T, int DYN, int N>
__global__ __launch_bounds__(kBlock) void ttr_kernel(const SolveDesc *__restrict__ sd, const T *__restrict__ src,
                                                     T *__restrict__ dst, const T *__restrict__ target,
                                                     unsigned long long *__restrict__ change, int chunk) {
    const SolveDesc &s = *sd;
    const uint32_t q = blockIdx.x * kBlock + threadIdx.x;
    const int i0b = int(blockIdx.y) * chunk;
    const int i0e = min(i0b + chunk, s.n0);
    double ch = 0.0;
    if (q < s.Q) {
        int ii[N];
        ii[0] = i0b;
        uint32_t rem = q;
#pragma unroll
        for (int d = N - 1; d >= 1; --d) {
            const uint32_t t = fdiv(rem, s.div[d]);
            ii[d] = int(rem - t * s.div[d].d);
            rem = t;
        }
        double f[N], sig[N];
        axis_terms<DYN, N>(s, ii, f);
        if constexpr (DYN == 0) {
            for (int d = 0; d < N; ++d) sig[d] = fabs(f[d]) + s.p[0];
        } else {
            for (int d = 0; d < N; ++d) sig[d] = fabs(f[d]);  // input axes: the bound
        }
        double den = 0.0;
        for (int d = 0; d < N; ++d) den += sig[d] * (2.0 * s.inv2dx[d]);
        // in-plane edges: the same for the whole run
        bool edge_in = false;
#pragma unroll
        for (int d = 1; d < N; ++d)
            if (!((s.periodic >> d) & 1u) && (ii[d] == 0 || ii[d] == s.n[d] - 1)) edge_in = true;
        const bool per0 = (s.periodic & 1u) != 0;
        for (int i0 = i0b; i0 < i0e; ++i0) {
            ii[0] = i0;
            const int64_t o = int64_t(i0) * s.s0 + q;
            const double old = double(src[o]);
            double nv = old;
            if (double(target[o]) <= 0.0) {
                nv = 0.0;
            } else if (edge_in || (!per0 && (i0 == 0 || i0 == s.n0 - 1))) {
                double eb = old;
#pragma unroll
                for (int d = 0; d < N; ++d) {
                    if ((s.periodic >> d) & 1u) continue;
                    const int64_t st = d == 0 ? s.s0 : int64_t(s.stride[d]);
                    const int nd = s.n[d];
                    if (ii[d] == 0 || ii[d] == nd - 1) {
                        const int64_t sg = ii[d] == 0 ? st : -st;
                        const double a = double(src[o + sg]), b = double(src[o + 2 * sg]);
                        double e = 2.0 * a - b;
                        if (b > e) e = b;
                        if (e < eb) eb = e;
                    }
                }
                nv = eb;
            } else {
                double pb[N], ns[N];
#pragma unroll
                for (int d = 0; d < N; ++d) {
                    const int64_t st = d == 0 ? s.s0 : int64_t(s.stride[d]);
                    const int nd = s.n[d];
                    const int64_t offr = ii[d] < nd - 1 ? st : -int64_t(nd - 1) * st;  // periodic wrap
                    const int64_t offl = ii[d] > 0 ? -st : int64_t(nd - 1) * st;
                    const double r = double(src[o + offr]), l = double(src[o + offl]);
                    pb[d] = (r - l) * s.inv2dx[d];
                    ns[d] = r + l;
                }
                double H = 0.0;
                if constexpr (DYN == 0) {
                    double n2 = 0.0;
                    for (int d = 0; d < N; ++d) n2 += pb[d] * pb[d];
                    const double nrm = sqrt(n2);
                    const double sg = s.u_mode ? 1.0 : -1.0;
                    for (int d = 0; d < N; ++d) {
                        const double u = nrm > 0.0 ? sg * s.p[0] * pb[d] / nrm : 0.0;
                        H += pb[d] * (f[d] + u);
                    }
                } else {
                    for (int d = 0; d < N; ++d) {
                        double fd = f[d];
                        if (axis_kind(DYN, d) == 1) {
                            const int mx = (DYN == 3 && d == 5) ? s.d_mode : s.u_mode;
                            fd = mx ? (pb[d] >= 0.0 ? f[d] : -f[d]) : (pb[d] >= 0.0 ? -f[d] : f[d]);
                        }
                        H += pb[d] * fd;
                    }
                }
                // reciprocal spacings instead of divisions (one division per node)
                double num = 1.0 + H;
                for (int d = 0; d < N; ++d) num += sig[d] * ns[d] * s.inv2dx[d];
                if (den > 0.0) {
                    const double cand = num / den;
                    if (cand < nv) nv = cand;
                }
            }
            const T out = T(nv);
            dst[o] = out;
            ch = fmax(ch, fabs(double(out) - old));
        }
    }
    // block maximum of the change, one atomic per block
    __shared__ double red[kBlock / 64];
    for (int off = 32; off >= 1; off >>= 1) ch = fmax(ch, __shfl_xor(ch, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ch;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kBlock / 64; ++w) m = fmax(m, red[w]);
        atomicMax(change + (blockIdx.x + blockIdx.y * gridDim.x) % kBoxSlots,
                  (unsigned long long)__double_as_longlong(m));
    }
}

// Start value of the time to reach: 0 on the target (l <= 0), big elsewhere.
template <typename T>
__global__ void ttr_init_kernel(const T *__restrict__ target, T *__restrict__ phi, int64_t npts, double big) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < npts) phi[i] = double(target[i]) <= 0.0 ? T(0) : T(big);
}

__global__ void ttr_zero_kernel(unsigned long long *__restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Zero alpha^max, the flags and the step counter of every listed solve.
__global__ void init_kernel(const SolveDesc *__restrict__ descs, int nsolves) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsolves) return;
    const SolveDesc &s = descs[i];
    for (int d = 0; d < kMaxDim; ++d) s.amax[d] = 0.0;
    *s.flags = 0;
    *s.step = 0;
    if (s.box) {  // costate box buffer of the first stage, the box CFL step's words
        for (int e = 0; e < 6 * kBoxSlots; ++e) s.box[e] = box_key(e % 6 < 3 ? INFINITY : -INFINITY);
        for (int e = 0; e < kBoxStepWords; ++e) s.box[12 * kBoxSlots + e] = 0;
    }
    *s.nsteps = 0;
}

// alpha^max_d = max over every grid point of alpha_d(z): per-thread maxima,
// wave64 butterfly, LDS across the waves, one atomic max per block and axis
// (float64 bit patterns of non-negative numbers order like the numbers).
template <int DYN, int N>
__global__ __launch_bounds__(kBlock) void alpha_kernel(const SolveDesc *__restrict__ descs) {
    const SolveDesc &s = descs[blockIdx.y];
    double m[N];
    for (int d = 0; d < N; ++d) m[d] = 0.0;
    for (uint32_t q = blockIdx.x * kBlock + threadIdx.x; q < s.Q; q += gridDim.x * kBlock) {
        int ii[N];
        uint32_t rem = q;
        for (int d = N - 1; d >= 1; --d) {
            const uint32_t t = fdiv(rem, s.div[d]);
            ii[d] = int(rem - t * s.div[d].d);
            rem = t;
        }
        if (N > 1 && ii[N - 1] >= s.n[N - 1]) continue;  // row padding
        for (int i0 = 0; i0 < s.n0; ++i0) {
            ii[0] = i0;
            double a[N];
            alpha_point<DYN, N>(s, ii, a);
            for (int d = 0; d < N; ++d) m[d] = fmax(m[d], a[d]);
        }
    }
    __shared__ double red[kBlock / 64][kMaxDim];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = 0; d < N; ++d) {
        double v = m[d];
        for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (lane == 0) red[wave][d] = v;
    }
    __syncthreads();
    if (threadIdx.x < N) {
        double v = red[0][threadIdx.x];
        for (int w = 1; w < kBlock / 64; ++w) v = fmax(v, red[w][threadIdx.x]);
        atomicMax((unsigned long long *)&s.amax[threadIdx.x], (unsigned long long)__double_as_longlong(v));
    }
}

// The float64 CFL schedule of every listed solve (one thread per solve):
// dt = cfl / sum_d alpha^max_d / dx_d, capped by max_dt, clipped so that the
// time lands exactly on every tau[k].  The host enqueued expect_steps steps,
// from the same arithmetic; a longer schedule (or an overflow) is flagged.
// Solves whose step comes from the costate box take it step by step
// (box_dt_kernel): their step count stays at max_steps until time lands on
// the last output time.
__global__ void sched_kernel(const SolveDesc *__restrict__ descs, int nsolves, int64_t *nsteps_all) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsolves) return;
    const SolveDesc &s = descs[i];
    if (s.box_cfl) {
        for (int d = 0; d < kMaxDim; ++d) s.amax[d] = 0.0;  // box alphas maxed in per step
        *s.nsteps = s.max_steps;
        if (nsteps_all) nsteps_all[i] = s.expect_steps;
        return;
    }
    double sum = 0.0;
    for (int d = 0; d < s.ndim; ++d) sum += s.amax[d] / s.dx[d];
    double dtc = s.cfl / sum;
    if (s.max_dt > 0.0 && dtc > s.max_dt) dtc = s.max_dt;
    double t = s.tau[0];
    int k = 1;
    int64_t n = 0;
    while (k < s.ntau) {
        if (n >= s.max_steps) { n = -1; break; }
        double dt, tn;
        int land = -1;
        if (dtc >= s.tau[k] - t) {
            dt = s.tau[k] - t;
            tn = s.tau[k];
            land = k;
        } else {
            dt = dtc;
            tn = t + dt;
        }
        s.dt_sched[n] = dt;
        s.land[n] = land;
        ++n;
        t = tn;
        if (land >= 0) ++k;
    }
    if (n < 0 || n > s.expect_steps) atomicOr(s.flags, kFlagStepsExceeded);
    double lo = INFINITY, hi = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        lo = fmin(lo, s.dt_sched[j]);
        hi = fmax(hi, s.dt_sched[j]);
    }
    s.dtmm[0] = lo;
    s.dtmm[1] = hi;
    *s.nsteps = n;
    if (nsteps_all) nsteps_all[i] = n;
}

// Largest pursuit-evasion box alpha over every heading of the grid at (x, y):
// the input pairs do not depend on the heading, and each |f_d| is the
// magnitude of a rounded sum that is monotone in its heading term
// (-v_a + v_b cos th for f_x, v_b sin th for f_y), so the largest over the
// headings is reached at the smallest or the largest of those terms: the
// same bits as taking the maximum of pe3d_alpha_box node by node.
__device__ __forceinline__ void pe3d_alpha_box_headings(const SolveDesc &s, double x, double y,
                                                        const double (&bmin)[3], const double (&bmax)[3],
                                                        double (&al)[3]) {
    al[0] = al[1] = al[2] = 0.0;
    double av[4], bv[4];
    const int n = pe3d_pairs(s, x, y, bmin, bmax, av, bv);
    for (int j = 0; j < n; ++j) {
        const double ay = av[j] * y, ax = av[j] * x;
        al[0] = fmax(al[0], fmax(fabs(s.pe_cmin + ay), fabs(s.pe_cmax + ay)));
        al[1] = fmax(al[1], fmax(fabs(s.pe_smin - ax), fabs(s.pe_smax - ax)));
        al[2] = fmax(al[2], fabs(bv[j] - av[j]));
    }
}

// The CFL step of step k for solves whose step comes from the costate box
// (Algorithm 1: alpha^max is the largest alpha_i of the step's dissipation
// loop, here over the box of the first stage's input, which the box pass of
// stage 0 has just reduced).  A row of gridDim.x blocks per listed solve
// (blockIdx.y): each takes the box from its 64 partial boxes (a lane each)
// and the largest box alpha over its share of the grid's (x, y) nodes (every heading at
// once), maxes it into the solve's step words with one atomic per axis, and
// counts itself in; the block that arrives last takes the float64 step,
// clipped to land on the next output time, records it as dt_sched[k], and
// clears the words for the next step.  Landing on the last output time fixes
// the step count at k + 1.  Every block of a row takes the same early exits
// (the step count only drops to k + 1 during the launch).
__global__ __launch_bounds__(kBlock) void box_dt_kernel(const SolveDesc *__restrict__ descs,
                                                        const int32_t *__restrict__ list, int from_desc,
                                                        int64_t fixed_step) {
    const SolveDesc &s = descs[list ? list[blockIdx.y] : int(blockIdx.y)];
    if (!s.box_cfl) return;
    const int64_t k = (from_desc ? *s.step : 0) + fixed_step;
    if (k >= *s.nsteps) return;
    const int box_buf = int((k * s.rk_order) & 1);
    const uint64_t *bx = s.box + 6 * kBoxSlots * box_buf;
    unsigned long long *words = (unsigned long long *)(s.box + 12 * kBoxSlots);
    // the box: lane j of every wave takes partial box j, then a butterfly
    static_assert(kBoxSlots == 64, "one partial box per lane");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double bmin[3], bmax[3];
    for (int d = 0; d < 3; ++d) {
        double a = box_val(bx[6 * lane + d]), b = box_val(bx[6 * lane + 3 + d]);
        for (int off = 32; off >= 1; off >>= 1) {
            a = fmin(a, __shfl_xor(a, off, 64));
            b = fmax(b, __shfl_xor(b, off, 64));
        }
        bmin[d] = a;
        bmax[d] = b;
    }
    double m[3] = {0.0, 0.0, 0.0};
    const int n0 = s.n[0], n1 = s.n[1];
    for (int p = int(blockIdx.x) * kBlock + int(threadIdx.x); p < n0 * n1; p += int(gridDim.x) * kBlock) {
        const int i0 = p / n1, i1 = p - i0 * n1;
        double al[3];
        pe3d_alpha_box_headings(s, tab_x(s, 0, i0), tab_x(s, 1, i1), bmin, bmax, al);
        for (int d = 0; d < 3; ++d) m[d] = fmax(m[d], al[d]);
    }
    __shared__ double red[kBlock / 64][3];
    __shared__ bool last;
    for (int d = 0; d < 3; ++d) {
        double v = m[d];
        for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (lane == 0) red[wave][d] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int d = 0; d < 3; ++d) {
            double v = red[0][d];
            for (int w = 1; w < kBlock / 64; ++w) v = fmax(v, red[w][d]);
            // alpha >= 0: its bits order as the values
            atomicMax(&words[d], (unsigned long long)__double_as_longlong(v));
        }
        __threadfence();
        last = atomicAdd(&words[3], 1ull) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x != 0) return;
    __threadfence();
    double amax[3];
    for (int d = 0; d < 3; ++d) {
        amax[d] = __longlong_as_double(
            (long long)__hip_atomic_load(&words[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        s.amax[d] = fmax(s.amax[d], amax[d]);
    }
    for (int e = 0; e < kBoxStepWords; ++e) words[e] = 0;
    double sum = 0.0;
    for (int d = 0; d < 3; ++d) sum += amax[d] / s.dx[d];
    double dtc = s.cfl / sum;
    if (s.max_dt > 0.0 && dtc > s.max_dt) dtc = s.max_dt;
    const double t = k > 0 ? s.t_after[k - 1] : s.tau[0];
    const int kt = k > 0 ? s.k_after[k - 1] : 1;
    double dt, tn;
    int land = -1;
    if (dtc >= s.tau[kt] - t) {
        dt = s.tau[kt] - t;
        tn = s.tau[kt];
        land = kt;
    } else {
        dt = dtc;
        tn = t + dt;
    }
    s.dt_sched[k] = dt;
    s.land[k] = land;
    s.dtmm[0] = k > 0 ? fmin(s.dtmm[0], dt) : dt;
    s.dtmm[1] = k > 0 ? fmax(s.dtmm[1], dt) : dt;
    s.t_after[k] = tn;
    s.k_after[k] = land >= 0 ? kt + 1 : kt;
    if (land == s.ntau - 1) *s.nsteps = k + 1;
}

// After the enqueued steps of box_cfl solves: a first-order solve whose
// step count turned out odd has its result in B (even steps read A), which
// moves to A; a schedule that had not landed on the last output time within
// the enqueued steps is flagged.
template <typename T>
__global__ __launch_bounds__(kBlock) void box_finish_kernel(const SolveDesc *__restrict__ descs,
                                                            const uint32_t *__restrict__ tile_solve,
                                                            const uint32_t *__restrict__ tile_local) {
    const uint32_t L = blockIdx.x;
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];
    if (!s.box_cfl) return;
    const int64_t nst = *s.nsteps;
    if (nst >= s.max_steps) {
        if (lt == 0 && threadIdx.x == 0) atomicOr(s.flags, kFlagStepsExceeded);
        return;
    }
    if (s.rk_order != 1 || (nst & 1) == 0) return;
    const uint32_t cid = lt / s.nqb;
    const uint32_t q = (lt - cid * s.nqb) * kBlock + threadIdx.x;
    if (q >= s.Q) return;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, s.n0);
    const T *src = (const T *)s.B;
    T *dst = (T *)s.A;
    for (int i0 = i0b; i0 < i0e; ++i0) dst[int64_t(i0) * s.s0 + q] = src[int64_t(i0) * s.s0 + q];
}

// save_all for a box_cfl solve (solve 0): if step k landed on an output
// time, copy its result (dense rows) into that slice of V_all.
template <typename T>
__global__ __launch_bounds__(kBlock) void box_save_kernel(const SolveDesc *__restrict__ descs, int64_t k,
                                                          T *__restrict__ V_all) {
    const SolveDesc &s = descs[0];
    if (k >= *s.nsteps) return;
    const int land = s.land[k];
    if (land < 0) return;
    const T *src = (s.rk_order == 1 && (k & 1) == 0) ? (const T *)s.B : (const T *)s.A;
    T *dst = V_all + int64_t(land) * s.npts;
    for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < s.npts; i += int64_t(gridDim.x) * kBlock)
        dst[i] = src[i];
}

// Time-varying sets for a box_cfl solve (solve 0): before step k, if step
// k - 1 landed on output time j, the references move to slice j.
template <typename T>
__global__ void box_slice_kernel(SolveDesc *__restrict__ descs, int64_t k) {
    if (threadIdx.x != 0) return;
    SolveDesc &s = descs[0];
    if (k == 0 || k >= *s.nsteps) return;
    const int iv = s.land[k - 1];
    if (iv < 0) return;
    s.tref = (const T *)s.tref0 + int64_t(iv) * s.tstride;
    s.oref = (const T *)s.oref0 + int64_t(iv) * s.ostride;
}

// Time-varying sets: point the comparison references of solve 0 at slice iv
// (the tau interval that the next steps lie in).
template <typename T>
__global__ void set_slice_kernel(SolveDesc *__restrict__ descs, int iv) {
    if (threadIdx.x != 0) return;
    SolveDesc &s = descs[0];
    s.tref = (const T *)s.tref0 + int64_t(iv) * s.tstride;
    s.oref = (const T *)s.oref0 + int64_t(iv) * s.ostride;
}

// End of a server tick: advance the step counter of every listed solve by
// its steps in the tick (inc[i]), capped at its step count.
__global__ void advance_kernel(const SolveDesc *__restrict__ descs, const int32_t *__restrict__ list,
                               const int32_t *__restrict__ inc, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const SolveDesc &s = descs[list[i]];
    const int64_t t = *s.step + inc[i];
    *s.step = t < *s.nsteps ? t : *s.nsteps;
}

// Copy the start value into the buffer the first step reads, for every
// listed solve.
template <typename T>
__global__ __launch_bounds__(kBlock) void start_copy_kernel(const SolveDesc *__restrict__ descs,
                                                            const uint32_t *__restrict__ tile_solve,
                                                            const uint32_t *__restrict__ tile_local) {
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, 0u);
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];
    const uint32_t cid = lt / s.nqb;
    const uint32_t g = (lt - cid * s.nqb) * kBlock + threadIdx.x;
    if (g >= s.Q / uint32_t(s.vec)) return;
    const uint32_t q = g * uint32_t(s.vec);
    T *dst = (s.rk_order == 1 && !s.box_cfl && ((*s.nsteps) & 1)) ? (T *)s.B : (T *)s.A;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, s.n0);
    if (s.Vsrc_dense) {
        // padded copies of the caller's dense V0: V0 and the start buffer
        // (padding elements set to zero)
        const int nd = s.ndim, nl = s.n[nd - 1];
        const uint32_t row = fdiv(q, s.div[nd - 1]);
        const int c0 = int(q - row * uint32_t(s.pitch));
        const int64_t dplane = int64_t(s.Q / uint32_t(s.pitch)) * nl;
        const T *src = (const T *)s.Vsrc_dense;
        T *v0 = (T *)s.V0;
        for (int i0 = i0b; i0 < i0e; ++i0) {
            const int64_t o = int64_t(i0) * s.s0 + q;
            const int64_t od = int64_t(i0) * dplane + int64_t(row) * nl + c0;
            for (int j = 0; j < s.vec; ++j) {
                const T v = c0 + j < nl ? src[od + j] : T(0);
                v0[o + j] = v;
                dst[o + j] = v;
            }
        }
        return;
    }
    const T *src = (const T *)s.Vinit;
    for (int i0 = i0b; i0 < i0e; ++i0) {
        const int64_t o = int64_t(i0) * s.s0 + q;
        for (int j = 0; j < s.vec; ++j) dst[o + j] = src[o + j];
    }
}

// Padded members: the final A to the caller's dense V_out.
template <typename T>
__global__ __launch_bounds__(kBlock) void finish_copy_kernel(const SolveDesc *__restrict__ descs,
                                                             const uint32_t *__restrict__ tile_solve,
                                                             const uint32_t *__restrict__ tile_local) {
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, 0u);
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];
    if (!s.Adst_dense) return;
    const uint32_t cid = lt / s.nqb;
    const uint32_t g = (lt - cid * s.nqb) * kBlock + threadIdx.x;
    if (g >= s.Q / uint32_t(s.vec)) return;
    const uint32_t q = g * uint32_t(s.vec);
    const int nd = s.ndim, nl = s.n[nd - 1];
    const uint32_t row = fdiv(q, s.div[nd - 1]);
    const int c0 = int(q - row * uint32_t(s.pitch));
    const int64_t dplane = int64_t(s.Q / uint32_t(s.pitch)) * nl;
    const T *a = (const T *)s.A;
    T *dst = (T *)s.Adst_dense;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, s.n0);
    for (int i0 = i0b; i0 < i0e; ++i0) {
        const int64_t o = int64_t(i0) * s.s0 + q;
        const int64_t od = int64_t(i0) * dplane + int64_t(row) * nl + c0;
        for (int j = 0; j < s.vec && c0 + j < nl; ++j) dst[od + j] = a[o + j];
    }
}

// --------------------------------------------------------- launchers

// kind: bit 0 the stage reads V^n (Runge-Kutta stages after the first),
// bit 1 the stage ends with the computation method's comparison, bit 3 a
// second one with the obstacle array (last stage of a step), bit 2 the LDS
// plane exchange; it must match what every listed solve does at this stage.
hipError_t launch_stage(int precision, int dyn, int ndim, int vec, int kind, const SolveDesc *d,
                        const uint32_t *ts, const uint32_t *tl, uint32_t nblocks, int stage,
                        int from_desc, int64_t step, int xgroup, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    using Slice = hipError_t (*)(ODP_STAGE_SLICE_ARGS);
    static const Slice f32[5] = {launch_stage_f32_d0, launch_stage_f32_d1, launch_stage_f32_d2,
                                 launch_stage_f32_d3, launch_stage_f32_d4};
    static const Slice f64[5] = {launch_stage_f64_d0, launch_stage_f64_d1, launch_stage_f64_d2,
                                 launch_stage_f64_d3, launch_stage_f64_d4};
    if (dyn < 0 || dyn > 4) return hipErrorInvalidValue;
    const Slice f = precision == 32 ? f32[dyn] : f64[dyn];
    return f(ndim, vec, kind, d, ts, tl, nblocks, stage, from_desc, step, xgroup, st);
}

template <int DYN, int N>
static hipError_t launch_alpha_t(const SolveDesc *d, int nsolves, int bps, hipStream_t st) {
    hipLaunchKernelGGL((alpha_kernel<DYN, N>), dim3(bps, nsolves), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_alpha(int dyn, int ndim, const SolveDesc *d, int nsolves, int blocks_per_solve,
                        hipStream_t st) {
    switch (dyn) {
    case 1: return launch_alpha_t<1, 3>(d, nsolves, blocks_per_solve, st);
    case 2: return launch_alpha_t<2, 4>(d, nsolves, blocks_per_solve, st);
    case 3: return launch_alpha_t<3, 6>(d, nsolves, blocks_per_solve, st);
    case 4: return launch_alpha_t<4, 3>(d, nsolves, blocks_per_solve, st);
    case 0:
        switch (ndim) {
        case 1: return launch_alpha_t<0, 1>(d, nsolves, blocks_per_solve, st);
        case 2: return launch_alpha_t<0, 2>(d, nsolves, blocks_per_solve, st);
        case 3: return launch_alpha_t<0, 3>(d, nsolves, blocks_per_solve, st);
        case 4: return launch_alpha_t<0, 4>(d, nsolves, blocks_per_solve, st);
        case 5: return launch_alpha_t<0, 5>(d, nsolves, blocks_per_solve, st);
        case 6: return launch_alpha_t<0, 6>(d, nsolves, blocks_per_solve, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(const SolveDesc *d, int nsolves, hipStream_t st) {
    hipLaunchKernelGGL(init_kernel, dim3((nsolves + 255) / 256), dim3(256), 0, st, d, nsolves);
    return hipGetLastError();
}

hipError_t launch_sched(const SolveDesc *d, int nsolves, int64_t *nsteps_all, hipStream_t st) {
    hipLaunchKernelGGL(sched_kernel, dim3((nsolves + 63) / 64), dim3(64), 0, st, d, nsolves, nsteps_all);
    return hipGetLastError();
}

hipError_t launch_start_copy(int precision, const SolveDesc *d, const uint32_t *ts,
                             const uint32_t *tl, uint32_t nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL(start_copy_kernel<float>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    else
        hipLaunchKernelGGL(start_copy_kernel<double>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    return hipGetLastError();
}

hipError_t launch_finish_copy(int precision, const SolveDesc *d, const uint32_t *ts,
                             const uint32_t *tl, uint32_t nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL(finish_copy_kernel<float>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    else
        hipLaunchKernelGGL(finish_copy_kernel<double>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    return hipGetLastError();
}

hipError_t launch_box_dt(const SolveDesc *d, const int32_t *list, int n, int parts, int from_desc, int64_t step,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(box_dt_kernel, dim3(parts > 0 ? parts : 1, n), dim3(kBlock), 0, st, d, list, from_desc,
                       step);
    return hipGetLastError();
}

hipError_t launch_box_finish(int precision, const SolveDesc *d, const uint32_t *ts, const uint32_t *tl,
                             uint32_t nblocks, hipStream_t st) {
    if (nblocks == 0) return hipSuccess;
    if (precision == 32)
        hipLaunchKernelGGL(box_finish_kernel<float>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    else
        hipLaunchKernelGGL(box_finish_kernel<double>, dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl);
    return hipGetLastError();
}

hipError_t launch_box_save(int precision, const SolveDesc *d, int64_t k, void *V_all, int64_t npts,
                           hipStream_t st) {
    const uint32_t nb = uint32_t(std::min<int64_t>((npts + kBlock - 1) / kBlock, 4096));
    if (precision == 32)
        hipLaunchKernelGGL(box_save_kernel<float>, dim3(nb), dim3(kBlock), 0, st, d, k, (float *)V_all);
    else
        hipLaunchKernelGGL(box_save_kernel<double>, dim3(nb), dim3(kBlock), 0, st, d, k, (double *)V_all);
    return hipGetLastError();
}

hipError_t launch_box_slice(int precision, SolveDesc *d, int64_t k, hipStream_t st) {
    if (precision == 32)
        hipLaunchKernelGGL(box_slice_kernel<float>, dim3(1), dim3(64), 0, st, d, k);
    else
        hipLaunchKernelGGL(box_slice_kernel<double>, dim3(1), dim3(64), 0, st, d, k);
    return hipGetLastError();
}

hipError_t launch_set_slice(int precision, SolveDesc *d, int iv, hipStream_t st) {
    if (precision == 32)
        hipLaunchKernelGGL(set_slice_kernel<float>, dim3(1), dim3(64), 0, st, d, iv);
    else
        hipLaunchKernelGGL(set_slice_kernel<double>, dim3(1), dim3(64), 0, st, d, iv);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_ttr_t(int dyn, int ndim, const SolveDesc *d, uint32_t qblocks, int n0, int chunk,
                               const void *src, void *dst, const void *target, unsigned long long *change,
                               hipStream_t st) {
    if (chunk < 1 || chunk > n0) return hipErrorInvalidValue;
    const dim3 grid(qblocks, uint32_t((n0 + chunk - 1) / chunk));
    const T *sp = (const T *)src, *tp = (const T *)target;
    T *dp = (T *)dst;
#define ODP_TTR(DY, NN) \
    hipLaunchKernelGGL((ttr_kernel<T, DY, NN>), grid, dim3(kBlock), 0, st, d, sp, dp, tp, change, chunk)
    switch (dyn) {
    case 1: ODP_TTR(1, 3); break;
    case 2: ODP_TTR(2, 4); break;
    case 3: ODP_TTR(3, 6); break;
    case 0:
        switch (ndim) {
        case 1: ODP_TTR(0, 1); break;
        case 2: ODP_TTR(0, 2); break;
        case 3: ODP_TTR(0, 3); break;
        case 4: ODP_TTR(0, 4); break;
        case 5: ODP_TTR(0, 5); break;
        case 6: ODP_TTR(0, 6); break;
        default: return hipErrorInvalidValue;
        }
        break;
    default: return hipErrorInvalidValue;
    }
#undef ODP_TTR
    return hipGetLastError();
}

hipError_t launch_ttr(int precision, int dyn, int ndim, const SolveDesc *d, uint32_t qblocks, int n0, int chunk,
                      const void *src, void *dst, const void *target, unsigned long long *change,
                      hipStream_t st) {
    if (precision == 32) return launch_ttr_t<float>(dyn, ndim, d, qblocks, n0, chunk, src, dst, target, change, st);
    return launch_ttr_t<double>(dyn, ndim, d, qblocks, n0, chunk, src, dst, target, change, st);
}

hipError_t launch_ttr_init(int precision, const void *target, void *phi, int64_t npts, double big,
                           hipStream_t st) {
    const dim3 grid(uint32_t((npts + 255) / 256));
    if (precision == 32)
        hipLaunchKernelGGL(ttr_init_kernel<float>, grid, dim3(256), 0, st, (const float *)target, (float *)phi, npts, big);
    else
        hipLaunchKernelGGL(ttr_init_kernel<double>, grid, dim3(256), 0, st, (const double *)target, (double *)phi, npts, big);
    return hipGetLastError();
}

hipError_t launch_ttr_zero(unsigned long long *p, int n, hipStream_t st) {
    hipLaunchKernelGGL(ttr_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_advance(const SolveDesc *d, const int32_t *list, const int32_t *inc, int n, hipStream_t st) {
    hipLaunchKernelGGL(advance_kernel, dim3((n + 255) / 256), dim3(256), 0, st, d, list, inc, n);
    return hipGetLastError();
}

}  // namespace odp
