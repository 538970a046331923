// Device code of libodp's stage kernels, shared by the kernel slices (one
// translation unit per precision and dynamics, stage_inst.hip) and the
// other kernels (kernels.hip).
// gfx950 kernels of libodp: the time-dependent HJ level-set step.
//
// Method (paper: Algorithm 1 and the HJ variational inequality): per grid
// point, one-sided differences along every axis, optimal bang-bang inputs
// for the central costate, the Hamiltonian, Lax-Friedrichs dissipation, a
// TVD Runge-Kutta stage and, for a tube, min with V0.  The Hamiltonian and
// the dissipation are folded per axis onto the raw differences:
//   drift axis d (f_d independent of the inputs, alpha_d >= |f_d|):
//     f pbar + alpha (p+ - p-)/2 = dr (f + alpha)/(2dx) + dl (f - alpha)/(2dx)
//   input axis d (box input of bound b, role sigma = +1 max / -1 min):
//     sigma b |pbar| + alpha (p+ - p-)/2 = sigma b |dr + dl|/(2dx)
//                                         + alpha (dr - dl)/(2dx)
// with dl = W_i - W_{i-e_d}, dr = W_{i+e_d} - W_i.  The per-axis
// coefficients depend only on the in-plane coordinates of a point (heading,
// speed), so each thread computes them once in float64 and then marches
// along axis 0, keeping the axis-0 neighbours in registers.
//
// Every floating-point contraction is written out (fma); the library is
// built with -ffp-contract=off so that all launch forms (single solve,
// batch, server tick) give the same bits for the same point.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "odp_dev.h"

namespace odp {

// ------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

// Blocks are dealt round robin to the 8 XCDs.  Renumber them so that each
// XCD works on runs of `group` consecutive tiles (neighbouring tiles then
// share that XCD's L2) while the 8 XCDs advance through the tile range
// together (one shared working set for the Infinity Cache).  group == 0: one
// contiguous run per XCD.
__device__ __forceinline__ uint32_t xcd_logical(uint32_t p, uint32_t nb, uint32_t group) {
    const uint32_t x = p % kNumXcd, k = p / kNumXcd;
    if (group == 0) {
        const uint32_t per = nb / kNumXcd, rem = nb % kNumXcd;
        return x * per + min(x, rem) + k;
    }
    const uint32_t span = kNumXcd * group;
    if (p >= (nb / span) * span) return p;  // the ragged tail keeps its order
    return ((k / group) * kNumXcd + x) * group + (k % group);
}

template <typename T>
__device__ __forceinline__ T ghost(T vb, T vin) {
    // ghost node beyond a non-periodic edge: extrapolated away from zero
    const T sg = T((vb > T(0)) - (vb < T(0)));
    return vb + sg * fabs(vb - vin);
}

// The same ghost from the difference vb - vin (computed by the caller with
// the same subtraction, so the result is the same bits).
template <typename T>
__device__ __forceinline__ T ghost_d(T vb, T diff) {
    const T sg = T((vb > T(0)) - (vb < T(0)));
    return vb + sg * fabs(diff);
}

// The second ghost node (second-order stencils): twice as far from the edge
// value, vb + 2 sgn(vb) |vb - vin|.
template <typename T>
__device__ __forceinline__ T ghost2(T vb, T vin) {
    const T sg = T((vb > T(0)) - (vb < T(0)));
    return vb + (T(2) * sg) * fabs(vb - vin);
}

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------- dynamics

// Axis kind per dynamics id: 0 drift, 1 box input.  Id 0 (single
// integrator, ball input) is handled separately.
__host__ __device__ constexpr int axis_kind(int dyn, int d) {
    return dyn == 1 ? (d == 2 ? 1 : 0)
         : dyn == 2 ? (d >= 2 ? 1 : 0)
         : dyn == 3 ? ((d == 2 || d == 5) ? 1 : 0)
         : 0;
}

__device__ __forceinline__ double tab_x(const SolveDesc &s, int d, int k) { return s.tabd[s.tab[d].off + k]; }
__device__ __forceinline__ double tab_cos(const SolveDesc &s, int d, int k) { return s.tabd[s.tab[d].off + s.tab[d].n + k]; }
__device__ __forceinline__ double tab_sin(const SolveDesc &s, int d, int k) { return s.tabd[s.tab[d].off + 2 * s.tab[d].n + k]; }

// f_d for drift axes and the bound for input axes at multi-index ii.
template <int DYN, int N>
__device__ __forceinline__ void axis_terms(const SolveDesc &s, const int (&ii)[N], double (&f)[N]) {
    if constexpr (DYN == 1) {          // x' = v cos th, y' = v sin th, th' = w
        f[0] = s.p[0] * tab_cos(s, 2, ii[2]);
        f[1] = s.p[0] * tab_sin(s, 2, ii[2]);
        f[2] = s.p[1];
    } else if constexpr (DYN == 2) {   // x' = v cos th, y' = v sin th, v' = a, th' = w
        const double v = tab_x(s, 2, ii[2]);
        f[0] = v * tab_cos(s, 3, ii[3]);
        f[1] = v * tab_sin(s, 3, ii[3]);
        f[2] = s.p[0];
        f[3] = s.p[1];
    } else if constexpr (DYN == 3) {   // evader (u on th_e), pursuer (d on th_p)
        f[0] = s.p[0] * tab_cos(s, 2, ii[2]);
        f[1] = s.p[0] * tab_sin(s, 2, ii[2]);
        f[2] = s.p[1];
        f[3] = s.p[2] * tab_cos(s, 5, ii[5]);
        f[4] = s.p[2] * tab_sin(s, 5, ii[5]);
        f[5] = s.p[3];
    } else {                           // z' = c + u: drift c_d
        for (int d = 0; d < N; ++d) f[d] = s.p[1 + d];
    }
}

// alpha_d(z): the largest |f_d| over the admissible inputs.
template <int DYN, int N>
__device__ __forceinline__ void alpha_point(const SolveDesc &s, const int (&ii)[N], double (&a)[N]) {
    if constexpr (DYN == 4) {
        // pursuit-evasion, all inputs admissible: |f_d| is largest at the
        // evader's bound of the sign that adds to the drift
        const double x = tab_x(s, 0, ii[0]), y = tab_x(s, 1, ii[1]);
        a[0] = fabs(-s.p[0] + s.p[1] * tab_cos(s, 2, ii[2])) + s.p[2] * fabs(y);
        a[1] = fabs(s.p[1] * tab_sin(s, 2, ii[2])) + s.p[2] * fabs(x);
        a[2] = s.p[2] + s.p[3];
        return;
    }
    double f[N];
    axis_terms<DYN, N>(s, ii, f);
    if constexpr (DYN == 0) {
        for (int d = 0; d < N; ++d) a[d] = fabs(f[d]) + s.p[0];
    } else {
        for (int d = 0; d < N; ++d) a[d] = fabs(f[d]);  // input axes: the bound
    }
}

// Per-point coefficients of the folded Hamiltonian + dissipation (float64,
// rounded once to T).
template <typename T, int DYN, int N>
struct Coef {
    T a[N], b[N];
    T h[DYN == 0 ? N : 1];  // ball input: 1 / (2 dx_d) for the costate norm
    T sig_umax;             // ball input: sigma u_max
};

template <typename T, int DYN, int N>
__device__ __forceinline__ Coef<T, DYN, N> make_coef(const SolveDesc &s, const int (&ii)[N]) {
    Coef<T, DYN, N> c;
    double f[N], al[N];
    axis_terms<DYN, N>(s, ii, f);
    if (s.global_alpha) {
        for (int d = 0; d < N; ++d) al[d] = s.amax[d];
    } else {
        alpha_point<DYN, N>(s, ii, al);
    }
    if constexpr (DYN == 0) {
        for (int d = 0; d < N; ++d) {
            c.a[d] = T(f[d] * s.inv2dx[d]);   // drift part of H, on (dr + dl)
            c.b[d] = T(al[d] * s.inv2dx[d]);  // dissipation, on (dr - dl)
            c.h[d] = T(s.inv2dx[d]);
        }
        c.sig_umax = T((s.u_mode ? 1.0 : -1.0) * s.p[0]);
    } else {
        for (int d = 0; d < N; ++d) {
            if (axis_kind(DYN, d) == 0) {
                c.a[d] = T((f[d] + al[d]) * s.inv2dx[d]);
                c.b[d] = T((f[d] - al[d]) * s.inv2dx[d]);
            } else {
                const int role = (DYN == 3 && d == 5) ? s.d_mode : s.u_mode;
                c.a[d] = T((role ? 1.0 : -1.0) * f[d] * s.inv2dx[d]);
                c.b[d] = T(al[d] * s.inv2dx[d]);
            }
        }
        c.h[0] = T(0);
        c.sig_umax = T(0);
    }
    return c;
}

// Running sum of the folded Lax-Friedrichs Hamiltonian.  Axes are always
// added in the order 0, 1, ..., N-1, whatever the kernel, so every launch
// form rounds identically.
template <typename T>
struct Acc {
    T L, n2;
};

template <typename T, int DYN, int N>
__device__ __forceinline__ void acc_axis(const Coef<T, DYN, N> &c, int d, T dl, T dr, Acc<T> &a) {
    if constexpr (DYN == 0) {
        const T sum = dr + dl;
        const T pb = sum * c.h[d];
        a.n2 = fma_t(pb, pb, a.n2);
        a.L = fma_t(c.a[d], sum, a.L);
        a.L = fma_t(c.b[d], dr - dl, a.L);
    } else {
        if (axis_kind(DYN, d) == 0) {
            a.L = fma_t(c.a[d], dr, a.L);
            a.L = fma_t(c.b[d], dl, a.L);
        } else {
            a.L = fma_t(c.a[d], fabs(dr + dl), a.L);
            a.L = fma_t(c.b[d], dr - dl, a.L);
        }
    }
}

template <typename T, int DYN, int N>
__device__ __forceinline__ T acc_finish(const Coef<T, DYN, N> &c, const Acc<T> &a) {
    if constexpr (DYN == 0) return fma_t(c.sig_umax, sqrt(a.n2), a.L);
    return a.L;
}

// TVD Runge-Kutta stage weights: out = a V^n + b (W + dt L).
__host__ __device__ inline void rk_weights(int order, int stage, double &a, double &b) {
    a = 0.0;
    b = 1.0;
    if (order == 2 && stage == 1) { a = 0.5; b = 0.5; }
    if (order == 3 && stage == 1) { a = 0.75; b = 0.25; }
    if (order == 3 && stage == 2) { a = 1.0 / 3.0; b = 2.0 / 3.0; }
}

// Buffers of stage `stage` of step k: stencil input W, pointwise V^n, output.
template <typename T>
__device__ __forceinline__ void stage_buffers(const SolveDesc &s, int stage, int64_t k, const T *&W,
                                              const T *&Vn, T *&out) {
    T *A = (T *)s.A, *B = (T *)s.B, *C = (T *)s.C;
    if (s.rk_order == 1) {
        // ping-pong; parity chosen so that the last step writes A (with the
        // step count not known ahead, box_cfl: even steps read A, and a
        // copy after the last step moves an odd count's result to A)
        const int64_t nst = *s.nsteps;
        const bool in_a = s.box_cfl ? (k & 1) == 0 : ((k + nst) & 1) == 0;
        W = in_a ? A : B;
        out = in_a ? B : A;
        Vn = W;
    } else if (s.rk_order == 2) {
        W = stage == 0 ? A : B;
        Vn = A;
        out = stage == 0 ? B : A;
    } else {
        W = stage == 0 ? A : (stage == 1 ? B : C);
        Vn = A;
        out = stage == 0 ? B : (stage == 1 ? C : A);
    }
}

// ------------------------------------------------------------ kernels

// Stage `stage` of step k for every listed solve: k = fixed_step, plus the
// solve's own step counter when step_from_desc != 0 (server ticks: the
// counter holds the step at the start of the tick, fixed_step the offset
// within it).
template <typename T, int DYN, int N>
__global__ __launch_bounds__(kBlock) void stage_kernel(const SolveDesc *__restrict__ descs,
                                                       const uint32_t *__restrict__ tile_solve,
                                                       const uint32_t *__restrict__ tile_local,
                                                       int stage, int step_from_desc,
                                                       int64_t fixed_step, int xgroup) {
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, uint32_t(xgroup));
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];

    const int64_t nsteps = *s.nsteps;
    const int64_t k = (step_from_desc ? *s.step : 0) + fixed_step;
    if (k >= nsteps || stage >= s.rk_order) return;

    const uint32_t cid = lt / s.nqb;
    const uint32_t qb = lt - cid * s.nqb;
    const uint32_t q = qb * kBlock + threadIdx.x;
    const bool active = q < s.Q;
    const uint32_t qq = active ? q : s.Q - 1;

    // in-plane multi-index and neighbour offsets (fixed for the march)
    int ii[N];
    ii[0] = 0;
    uint32_t rem = qq;
#pragma unroll
    for (int d = N - 1; d >= 1; --d) {
        const uint32_t t = fdiv(rem, s.div[d]);
        ii[d] = int(rem - t * s.div[d].d);
        rem = t;
    }
    int32_t offL[N], offR[N];
    uint32_t gl = 0, gr = 0;
#pragma unroll
    for (int d = 1; d < N; ++d) {
        const int32_t st = s.stride[d], nd = s.n[d];
        const bool per = (s.periodic >> d) & 1u;
        if (ii[d] > 0) offL[d] = -st;
        else if (per) offL[d] = (nd - 1) * st;
        else { offL[d] = 0; gl |= 1u << d; }
        if (ii[d] < nd - 1) offR[d] = st;
        else if (per) offR[d] = -(nd - 1) * st;
        else { offR[d] = 0; gr |= 1u << d; }
    }
    const Coef<T, DYN, N> cf = make_coef<T, DYN, N>(s, ii);

    const T *W, *Vn;
    T *out;
    stage_buffers<T>(s, stage, k, W, Vn, out);
    const T *Z = s.tvn ? Vn : (const T *)s.tref;
    const T *G = (const T *)s.oref;
    double wa, wb;
    rk_weights(s.rk_order, stage, wa, wb);
    const T ra = T(wa), rb = T(wb);
    const bool last = stage == s.rk_order - 1;
    const bool clamp = last && s.tclamp;
    const bool obst = last && s.obst;
    const bool tmax = s.tmax, omax = s.omax;
    const T dt = T(s.dt_sched[k]);

    const int64_t s0 = s.s0;
    const int n0 = s.n0;
    const bool per0 = s.periodic & 1u;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, n0);

    T wc = W[int64_t(i0b) * s0 + qq];
    T wm = i0b > 0 ? W[int64_t(i0b - 1) * s0 + qq] : (per0 ? W[int64_t(n0 - 1) * s0 + qq] : wc);
    int bad = 0;
    for (int i0 = i0b; i0 < i0e; ++i0) {
        const T *plane = W + int64_t(i0) * s0;
        const T wp = i0 + 1 < n0 ? plane[s0 + qq] : (per0 ? W[qq] : wc);
        Acc<T> acc{T(0), T(0)};
        {
            T l0 = wm, r0 = wp;
            if (!per0) {
                if (i0 == 0) l0 = ghost(wc, wp);
                if (i0 == n0 - 1) r0 = ghost(wc, wm);
            }
            acc_axis<T, DYN, N>(cf, 0, wc - l0, r0 - wc, acc);
        }
#pragma unroll
        for (int d = 1; d < N; ++d) {
            T wl = plane[qq + offL[d]];
            T wr = plane[qq + offR[d]];
            if (gl & (1u << d)) wl = ghost(wc, wr);
            if (gr & (1u << d)) wr = ghost(wc, wl);
            acc_axis<T, DYN, N>(cf, d, wc - wl, wr - wc, acc);
        }
        const T Lh = acc_finish<T, DYN, N>(cf, acc);
        const int64_t o = int64_t(i0) * s0 + qq;
        T v = fma_t(dt, Lh, wc);
        if (wa != 0.0) v = fma_t(ra, Vn[o], rb * v);
        if (clamp) {
            const T z = Z[o];
            if (tmax ? z > v : z < v) v = z;
        }
        if (obst) {
            const T g = G[o];
            if (omax ? g > v : g < v) v = g;
        }
        bad |= !isfinite(v);
        if (active) out[o] = v;
        wm = wc;
        wc = wp;
    }
    if (bad && active) atomicOr(s.flags, 1);
}

// Second-order ENO differences of one axis from the five nodes around the
// point (ghosts already substituted): the raw one-sided differences with half
// the smaller-magnitude second difference of the two stencils that contain
// each of them, dl = (W_i - W_{i-1}) + sel(S_{i-1}, S_i) / 2 and
// dr = (W_{i+1} - W_i) - sel(S_i, S_{i+1}) / 2 with S_j the second
// difference (W_{j+1} - W_j) - (W_j - W_{j-1}); a tie takes the first.
template <typename T>
__device__ __forceinline__ void eno2_diffs(T l2, T l1, T c, T r1, T r2, T &dl, T &dr) {
    const T dm = c - l1, dmm = l1 - l2, dp = r1 - c, dpp = r2 - r1;
    const T sm = dm - dmm, s0 = dp - dm, sp = dpp - dp;
    const T cm = fabs(sm) <= fabs(s0) ? sm : s0;
    const T cp = fabs(s0) <= fabs(sp) ? s0 : sp;
    dl = dm + T(0.5) * cm;
    dr = dp - T(0.5) * cp;
}

// Costate box keys: order-preserving unsigned images of doubles, so that
// integer atomic min / max order them as the doubles.
__device__ __forceinline__ uint64_t box_key(double v) {
    const uint64_t u = uint64_t(__double_as_longlong(v));
    return (u >> 63) ? ~u : (u | (1ull << 63));
}
__device__ __forceinline__ double box_val(uint64_t k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & ~(1ull << 63)) : ~k));
}

__device__ __forceinline__ double bang_d(double sw, double bound, int maximise) {
    return maximise ? (sw >= 0.0 ? bound : -bound) : (sw >= 0.0 ? -bound : bound);
}

// Input pairs of the pursuit-evasion game that some costate in the box
// [bmin, bmax] selects at (x, y): the pursuer's switching function is p_th,
// so each of its branches keeps the half of the p_th interval of its sign
// (closed at 0); the evader's is y p_x - x p_y - p_th, ranged over that half
// term by term.  The heading does not enter, so the pairs hold for every
// heading at (x, y).  Returns the number of pairs (evader a, pursuer b).
__device__ __forceinline__ int pe3d_pairs(const SolveDesc &s, double x, double y, const double (&bmin)[3],
                                          const double (&bmax)[3], double (&av)[4], double (&bv)[4]) {
    int n = 0;
    const double c0 = y, c1 = -x;
    const double m01 = fmin(c0 * bmin[0], c0 * bmax[0]) + fmin(c1 * bmin[1], c1 * bmax[1]);
    const double M01 = fmax(c0 * bmin[0], c0 * bmax[0]) + fmax(c1 * bmin[1], c1 * bmax[1]);
    for (int br = 1; br >= 0; --br) {
        double lo = bmin[2], hi = bmax[2];
        if (br) { if (lo < 0.0) lo = 0.0; }
        else    { if (hi > 0.0) hi = 0.0; }
        if (lo > hi || (!br && !(lo < 0.0))) continue;
        const double b = bang_d(br ? 1.0 : -1.0, s.p[3], s.d_mode);
        const double smin = m01 + fmin(-lo, -hi), smax = M01 + fmax(-lo, -hi);
        for (int ar = 1; ar >= 0; --ar) {
            if (ar ? !(smax >= 0.0) : !(smin < 0.0)) continue;
            av[n] = bang_d(ar ? 1.0 : -1.0, s.p[2], s.u_mode);
            bv[n] = b;
            ++n;
        }
    }
    return n;
}

// Pursuit-evasion dissipation over the costate box [bmin, bmax] at (x, y,
// th): the largest |f_d| over the input pairs some costate in the box selects.
__device__ __forceinline__ void pe3d_alpha_box(const SolveDesc &s, double x, double y, double cth,
                                               double sth, const double (&bmin)[3],
                                               const double (&bmax)[3], double (&al)[3]) {
    al[0] = al[1] = al[2] = 0.0;
    double av[4], bv[4];
    const int n = pe3d_pairs(s, x, y, bmin, bmax, av, bv);
    for (int j = 0; j < n; ++j) {
        const double f0 = -s.p[0] + s.p[1] * cth + av[j] * y;
        const double f1 = s.p[1] * sth - av[j] * x;
        const double f2 = bv[j] - av[j];
        al[0] = fmax(al[0], fabs(f0));
        al[1] = fmax(al[1], fabs(f1));
        al[2] = fmax(al[2], fabs(f2));
    }
}

// Stage of step k for the point-per-lane forms: second-order ENO
// differences (ORDER 2; the Spatial Derivatives subsection's ENO2, which the
// paper pairs with TVD-RK2) and the pursuit-evasion model (DYN 4, either
// order), whose evader input enters three axes.  One point per lane; axis-0
// neighbours ride in a register ring along the march, the in-plane
// neighbours are loaded per plane.  Beyond a non-periodic edge the m-th ghost
// node is vb + m sgn(vb)|vb - vin| (vb the edge node, vin its inner
// neighbour).  Rows may be padded (pitch > n_last): padding lanes store
// nothing.  PASS 1 (pursuit-evasion only) computes no update: it reduces the
// costate pbar of the stage input over the grid into the solve's box
// (Algorithm 1's D_min / D_max), which the update pass then reads.
template <typename T, int DYN, int N, int ORDER, int PASS>
__global__ __launch_bounds__(kBlock) void stage_point_kernel(const SolveDesc *__restrict__ descs,
                                                             const uint32_t *__restrict__ tile_solve,
                                                             const uint32_t *__restrict__ tile_local,
                                                             int stage, int step_from_desc,
                                                             int64_t fixed_step, int xgroup) {
    static_assert(DYN != 4 || N == 3, "pursuit-evasion is three-dimensional");
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, uint32_t(xgroup));
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];

    const int64_t nsteps = *s.nsteps;
    const int64_t k = (step_from_desc ? *s.step : 0) + fixed_step;
    if (k >= nsteps || stage >= s.rk_order) return;

    const uint32_t cid = lt / s.nqb;
    const uint32_t qb = lt - cid * s.nqb;
    const uint32_t q = qb * kBlock + threadIdx.x;
    uint32_t qq = q < s.Q ? q : s.Q - 1;

    int ii[N];
    ii[0] = 0;
    uint32_t rem = qq;
#pragma unroll
    for (int d = N - 1; d >= 1; --d) {
        const uint32_t t = fdiv(rem, s.div[d]);
        ii[d] = int(rem - t * s.div[d].d);
        rem = t;
    }
    const bool active = q < s.Q && (N == 1 || ii[N - 1] < s.n[N - 1]);
    if (N > 1 && ii[N - 1] >= s.n[N - 1]) {
        // padding lane: stand on the row's last node, so that every
        // neighbour offset below stays inside the row
        qq -= uint32_t(ii[N - 1] - (s.n[N - 1] - 1));
        ii[N - 1] = s.n[N - 1] - 1;
    }

    // in-plane offsets of the nodes at -2, -1, +1, +2 along axes 1..N-1
    // (relative to the point; periodic wrap applied).  A node beyond a
    // non-periodic edge is marked in gmask (bit 4d + j, j = 0..3 for -2, -1,
    // +1, +2) and replaced by a ghost after the loads (its offset is 0).
    int32_t off[N][4];
    uint32_t gmask = 0;
#pragma unroll
    for (int d = 1; d < N; ++d) {
        const int32_t st = s.stride[d], nd = s.n[d];
        const bool per = (s.periodic >> d) & 1u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int sh = j < 2 ? j - 2 : j - 1;
            const int kk = ii[d] + sh;
            if (kk >= 0 && kk < nd) off[d][j] = sh * st;
            else if (per) off[d][j] = ((kk + nd) % nd - ii[d]) * st;
            else { off[d][j] = 0; gmask |= 1u << (4 * d + j); }
        }
    }

    const T *W, *Vn;
    T *out;
    stage_buffers<T>(s, stage, k, W, Vn, out);
    const T dt = T(s.dt_sched[k]);
    const int64_t s0 = s.s0;
    const int n0 = s.n0;
    const bool per0 = s.periodic & 1u;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, n0);

    // costate box buffer of this stage: two, alternating with the global
    // stage index
    const int box_buf = int((k * s.rk_order + stage) & 1);
    // per-lane constants of the Hamiltonian
    Coef<T, DYN == 4 ? 0 : DYN, N> cf;
    if constexpr (DYN != 4 && PASS == 0) cf = make_coef<T, DYN, N>(s, ii);
    double pe_y = 0.0, pe_c = 0.0, pe_s = 0.0;
    double bmin[3] = {0.0, 0.0, 0.0}, bmax[3] = {0.0, 0.0, 0.0};
    T h[N];
#pragma unroll
    for (int d = 0; d < N; ++d) h[d] = T(s.inv2dx[d]);
    if constexpr (DYN == 4) {
        pe_y = tab_x(s, 1, ii[1]);
        pe_c = tab_cos(s, 2, ii[2]);
        pe_s = tab_sin(s, 2, ii[2]);
        if constexpr (PASS == 0) {
            if (!s.global_alpha) {
                // fold the partial boxes: lane l reads slot l, then a wave
                // butterfly leaves the box in every lane
                const uint64_t *bx = s.box + 6 * kBoxSlots * box_buf + 6 * (threadIdx.x & 63);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    double a = box_val(bx[d]), b = box_val(bx[3 + d]);
                    for (int o2 = 32; o2 >= 1; o2 >>= 1) {
                        a = fmin(a, __shfl_xor(a, o2, 64));
                        b = fmax(b, __shfl_xor(b, o2, 64));
                    }
                    bmin[d] = a;
                    bmax[d] = b;
                }
                // empty the other buffer for the next stage's box pass (the
                // passes of this stage read or wrote only this one)
                if (lt == 0) {
                    uint64_t *nx = s.box + 6 * kBoxSlots * (box_buf ^ 1);
                    for (int e = threadIdx.x; e < 6 * kBoxSlots; e += kBlock)
                        nx[e] = box_key(e % 6 < 3 ? INFINITY : -INFINITY);
                }
            }
        }
    }
    const T pe_cx = T(-s.p[0] + s.p[1] * pe_c), pe_sy = T(s.p[1] * pe_s);
    const T pe_yT = T(pe_y), pe_A = T(s.p[2]), pe_B = T(s.p[3]);

    const T *Z = s.tvn ? Vn : (const T *)s.tref;
    const T *G = (const T *)s.oref;
    double wa, wb;
    rk_weights(s.rk_order, stage, wa, wb);
    const T ra = T(wa), rb = T(wb);
    const bool last = stage == s.rk_order - 1;
    const bool clamp = last && s.tclamp;
    const bool obst = last && s.obst;
    const bool tmax = s.tmax, omax = s.omax;

    // axis-0 node j (-2 <= j <= n0 + 1) of this lane: wrapped, or a ghost
    auto ax0 = [&](int j) -> T {
        if (j >= 0 && j < n0) return W[int64_t(j) * s0 + qq];
        if (per0) return W[int64_t(j < 0 ? j + n0 : j - n0) * s0 + qq];
        const int b = j < 0 ? 0 : n0 - 1, in = j < 0 ? 1 : n0 - 2;
        const T vb = W[int64_t(b) * s0 + qq], vin = W[int64_t(in) * s0 + qq];
        return (j == -1 || j == n0) ? ghost(vb, vin) : ghost2(vb, vin);
    };
    T r0 = ORDER == 2 ? ax0(i0b - 2) : T(0), r1 = ax0(i0b - 1), r2 = ax0(i0b), r3 = ax0(i0b + 1), r4 = T(0);
    double mn[N], mx[N];
#pragma unroll
    for (int d = 0; d < N; ++d) { mn[d] = INFINITY; mx[d] = -INFINITY; }
    int bad = 0;
    for (int i0 = i0b; i0 < i0e; ++i0) {
        if constexpr (ORDER == 2) r4 = ax0(i0 + 2);
        const T wc = r2;
        const T *plane = W + int64_t(i0) * s0 + qq;
        T dl[N], dr[N];
        if constexpr (ORDER == 2) eno2_diffs(r0, r1, wc, r3, r4, dl[0], dr[0]);
        else { dl[0] = wc - r1; dr[0] = r3 - wc; }
#pragma unroll
        for (int d = 1; d < N; ++d) {
            T l2 = T(0), l1 = plane[off[d][1]], p1 = plane[off[d][2]], p2 = T(0);
            if constexpr (ORDER == 2) {
                l2 = plane[off[d][0]];
                p2 = plane[off[d][3]];
            }
            const uint32_t gm = (gmask >> (4 * d)) & 15u;
            if (gm) {
                // near a non-periodic edge: the edge node is the point or its
                // inner neighbour, both loaded above
                if (gm & 2u) { l1 = ghost(wc, p1); l2 = ghost2(wc, p1); }
                else if (gm & 1u) l2 = ghost(l1, wc);
                if (gm & 4u) { p1 = ghost(wc, l1); p2 = ghost2(wc, l1); }
                else if (gm & 8u) p2 = ghost(p1, wc);
            }
            if constexpr (ORDER == 2) eno2_diffs(l2, l1, wc, p1, p2, dl[d], dr[d]);
            else { dl[d] = wc - l1; dr[d] = p1 - wc; }
        }
        if constexpr (ORDER == 2) r0 = r1;
        r1 = r2;
        r2 = r3;
        r3 = ORDER == 2 ? r4 : ax0(i0 + 2);

        if constexpr (PASS == 1) {
            // costate box of this stage: pbar_d = (p+ + p-) / 2
            if (active) {
#pragma unroll
                for (int d = 0; d < N; ++d) {
                    const double pb = double((dl[d] + dr[d]) * h[d]);
                    mn[d] = fmin(mn[d], pb);
                    mx[d] = fmax(mx[d], pb);
                }
            }
            continue;
        }
        T Lh;
        if constexpr (DYN == 4) {
            const double xd = tab_x(s, 0, i0);
            const T x = T(xd);
            const T pbx = (dl[0] + dr[0]) * h[0], pby = (dl[1] + dr[1]) * h[1], pbt = (dl[2] + dr[2]) * h[2];
            const T sa = pbx * pe_yT - pby * x - pbt;
            const T a = s.u_mode ? (sa >= T(0) ? pe_A : -pe_A) : (sa >= T(0) ? -pe_A : pe_A);
            const T b = s.d_mode ? (pbt >= T(0) ? pe_B : -pe_B) : (pbt >= T(0) ? -pe_B : pe_B);
            const T f0 = pe_cx + a * pe_yT, f1 = pe_sy - a * x, f2 = b - a;
            T H = pbx * f0;
            H = fma_t(pby, f1, H);
            H = fma_t(pbt, f2, H);
            double al[3];
            if (s.global_alpha) {
                for (int d = 0; d < 3; ++d) al[d] = s.amax[d];
            } else {
                pe3d_alpha_box(s, xd, pe_y, pe_c, pe_s, bmin, bmax, al);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) H = fma_t(T(al[d]), (dr[d] - dl[d]) * h[d], H);
            Lh = H;
        } else {
            Acc<T> acc{T(0), T(0)};
#pragma unroll
            for (int d = 0; d < N; ++d) acc_axis<T, DYN, N>(cf, d, dl[d], dr[d], acc);
            Lh = acc_finish<T, DYN, N>(cf, acc);
        }
        const int64_t o = int64_t(i0) * s0 + qq;
        T v = fma_t(dt, Lh, wc);
        if (wa != 0.0) v = fma_t(ra, Vn[o], rb * v);
        if (clamp) {
            const T z = Z[o];
            if (tmax ? z > v : z < v) v = z;
        }
        if (obst) {
            const T g = G[o];
            if (omax ? g > v : g < v) v = g;
        }
        bad |= active && !isfinite(v);
        if (active) out[o] = v;
    }
    if constexpr (PASS == 1) {
        // wave reduction, then across the block's waves in LDS, then one
        // atomic per block and bound (the box has 2N addresses for the whole
        // grid: per-wave atomics would queue on them)
        __shared__ double red[kBlock / 64][2 * N];
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int d = 0; d < N; ++d) {
            double a = mn[d], b = mx[d];
            for (int o2 = 32; o2 >= 1; o2 >>= 1) {
                a = fmin(a, __shfl_xor(a, o2, 64));
                b = fmax(b, __shfl_xor(b, o2, 64));
            }
            if (lane == 0) {
                red[wave][d] = a;
                red[wave][N + d] = b;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * N) {
            const int e = threadIdx.x;
            double v = red[0][e];
            for (int w = 1; w < kBlock / 64; ++w) v = e < N ? fmin(v, red[w][e]) : fmax(v, red[w][e]);
            uint64_t *bx = s.box + 6 * kBoxSlots * box_buf + 6 * (blockIdx.x % kBoxSlots);
            if (e < N) atomicMin((unsigned long long *)&bx[e], (unsigned long long)box_key(v));
            else atomicMax((unsigned long long *)&bx[e], (unsigned long long)box_key(v));
        }
    } else {
        if (bad) atomicOr(s.flags, 1);
    }
}

// VEC consecutive points of the last axis per thread (16-byte loads and
// stores), for ndim >= 2 and n_last a multiple of VEC.  Each group of VEC
// points lies inside one row of the last axis, so the middle axes' neighbours
// of the whole group are one vector load each and share their ghost /
// periodic status; the last axis takes its two outer neighbours with scalar
// loads.  The next plane's centre values and pointwise operands are loaded
// one iteration ahead, after the current plane's neighbour loads, so that
// waiting for the neighbours does not wait for them.  KIND bit 0: the stage
// reads V^n; bit 1: the stage ends with the computation method's comparison
// (with V0, V^n, a target or an obstacle array: SolveDesc); bit 3: a second
// comparison, with the obstacle array, follows.
#define ODP_GLOBAL __attribute__((address_space(1)))

template <typename T, int VEC>
struct alignas(sizeof(T) * VEC) Pack {
    T v[VEC];
};

template <typename T, int VEC>
__device__ __forceinline__ Pack<T, VEC> ldp(const ODP_GLOBAL T *p) {
    Pack<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = *p;
    } else {
        typedef T ev __attribute__((ext_vector_type(VEC)));
        const ev x = *reinterpret_cast<const ODP_GLOBAL ev *>(p);
#pragma unroll
        for (int j = 0; j < VEC; ++j) r.v[j] = x[j];
    }
    return r;
}

// Streaming accesses (V^n, V0, the stage output) are non-temporal so that
// they do not push the stencil input's neighbour rows out of L2.
template <typename T, int VEC>
__device__ __forceinline__ Pack<T, VEC> ldp_nt(const ODP_GLOBAL T *p) {
    Pack<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = __builtin_nontemporal_load(p);
    } else {
        typedef T ev __attribute__((ext_vector_type(VEC)));
        const ev x = __builtin_nontemporal_load(reinterpret_cast<const ODP_GLOBAL ev *>(p));
#pragma unroll
        for (int j = 0; j < VEC; ++j) r.v[j] = x[j];
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void stp_lds(T *p, const Pack<T, VEC> &r) {
    if constexpr (VEC == 1) {
        *p = r.v[0];
    } else {
        typedef T ev __attribute__((ext_vector_type(VEC)));
        ev x;
#pragma unroll
        for (int j = 0; j < VEC; ++j) x[j] = r.v[j];
        *reinterpret_cast<ev *>(p) = x;
    }
}

template <typename T, int VEC>
__device__ __forceinline__ Pack<T, VEC> ldp_lds(const T *p) {
    Pack<T, VEC> r;
    if constexpr (VEC == 1) {
        r.v[0] = *p;
    } else {
        typedef T ev __attribute__((ext_vector_type(VEC)));
        const ev x = *reinterpret_cast<const ev *>(p);
#pragma unroll
        for (int j = 0; j < VEC; ++j) r.v[j] = x[j];
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void stp_nt(ODP_GLOBAL T *p, const Pack<T, VEC> &r) {
    if constexpr (VEC == 1) {
        __builtin_nontemporal_store(r.v[0], p);
    } else {
        typedef T ev __attribute__((ext_vector_type(VEC)));
        ev x;
#pragma unroll
        for (int j = 0; j < VEC; ++j) x[j] = r.v[j];
        __builtin_nontemporal_store(x, reinterpret_cast<ODP_GLOBAL ev *>(p));
    }
}

// Second-order ENO stage with VEC consecutive last-axis points per thread
// (rows without padding, n_last a multiple of VEC >= 2): the centre, the
// axis-0 ring (five planes) and the middle axes' neighbours at distance 1 and
// 2 are one 16-byte pack each for the whole group; along the last axis the
// group's own values and two scalars on each side give every element its
// five-node stencil.  Each point's arithmetic is the point-per-lane kernel's
// (same differences, same ghost substitutions, axes accumulated in the same
// order), so the two forms give the same bits.
// LDSX (ndim >= 3, 4 rows of the last axis within a block's range): each
// plane's values of the block's range, with two rows of halo on each side,
// go to a double-buffered LDS tile (one barrier per plane), from which the
// neighbours along axis N-2 (distance 1 and 2) and along the last axis are
// read; rows of axis N-2 wrapped across a periodic edge are loaded from
// memory (a wave-uniform branch).
template <typename T, int DYN, int N, int VEC, bool LDSX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(N == 4 && sizeof(T) == 8 ? 3 : 1))) void stage_eno2_vec_kernel(const SolveDesc *__restrict__ descs,
                                                                const uint32_t *__restrict__ tile_solve,
                                                                const uint32_t *__restrict__ tile_local,
                                                                int stage, int step_from_desc,
                                                                int64_t fixed_step, int xgroup) {
    static_assert(N >= 2 && VEC >= 2, "vector form: ndim >= 2, two or more points per thread");
    using P = Pack<T, VEC>;
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, uint32_t(xgroup));
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];

    const int64_t nsteps = *s.nsteps;
    const int64_t k = (step_from_desc ? *s.step : 0) + fixed_step;
    if (k >= nsteps || stage >= s.rk_order) return;

    const uint32_t cid = lt / s.nqb;
    const uint32_t qb = lt - cid * s.nqb;
    const TileGroup tg = tile_group(s, qb, threadIdx.x, VEC);  // row-major, or brick tiles (6D)
    const bool active = tg.active;
    const uint32_t q = tg.q;

    int ii[N];
    ii[0] = 0;
    uint32_t rem = q;
#pragma unroll
    for (int d = N - 1; d >= 1; --d) {
        const uint32_t t = fdiv(rem, s.div[d]);
        ii[d] = int(rem - t * s.div[d].d);
        rem = t;
    }
    // middle axes: offsets of the packs at -2, -1, +1, +2 (periodic wrap
    // applied); beyond a non-periodic edge: gmask bit 4d + j, offset 0
    int32_t off[N][4];
    uint32_t gmask = 0;
#pragma unroll
    for (int d = 1; d < N - 1; ++d) {
        const int32_t st = s.stride[d], nd = s.n[d];
        const bool per = (s.periodic >> d) & 1u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int sh = j < 2 ? j - 2 : j - 1;
            const int kk = ii[d] + sh;
            if (kk >= 0 && kk < nd) off[d][j] = sh * st;
            else if (per) off[d][j] = ((kk + nd) % nd - ii[d]) * st;
            else { off[d][j] = 0; gmask |= 1u << (4 * d + j); }
        }
    }
    // last axis: the two nodes before and after the group (il and n_last
    // are multiples of VEC >= 2, so only a group at a row end reaches past it)
    const int nl = s.n[N - 1], il = ii[N - 1];
    const bool perl = (s.periodic >> (N - 1)) & 1u;
    int32_t xo[4] = {-2, -1, VEC, VEC + 1};
    bool gxl = false, gxr = false;
    if (il == 0) {
        if (perl) { xo[0] = nl - 2; xo[1] = nl - 1; }
        else { xo[0] = xo[1] = 0; gxl = true; }
    }
    if (il + VEC == nl) {
        if (perl) { xo[2] = -il; xo[3] = 1 - il; }
        else { xo[2] = xo[3] = 0; gxr = true; }
    }

    Coef<T, DYN, N> cf[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        int jj[N];
#pragma unroll
        for (int d = 0; d < N; ++d) jj[d] = ii[d];
        jj[N - 1] = il + j;
        cf[j] = make_coef<T, DYN, N>(s, jj);
    }

    const T *Wg, *Vng;
    T *outg;
    stage_buffers<T>(s, stage, k, Wg, Vng, outg);
    const ODP_GLOBAL T *W = (const ODP_GLOBAL T *)Wg;
    const ODP_GLOBAL T *Vn = (const ODP_GLOBAL T *)Vng;
    ODP_GLOBAL T *out = (ODP_GLOBAL T *)outg;
    const ODP_GLOBAL T *Z = (const ODP_GLOBAL T *)(s.tvn ? (const void *)Vng : s.tref);
    const ODP_GLOBAL T *G = (const ODP_GLOBAL T *)s.oref;
    double wa, wb;
    rk_weights(s.rk_order, stage, wa, wb);
    const T ra = T(wa), rb = T(wb);
    const bool last = stage == s.rk_order - 1;
    const bool clamp = last && s.tclamp;
    const bool obst = last && s.obst;
    const bool tmax = s.tmax, omax = s.omax;
    const T dt = T(s.dt_sched[k]);

    const int64_t s0 = s.s0;
    const int n0 = s.n0;
    const bool per0 = s.periodic & 1u;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, n0);

    // LDS plane tile (LDSX): [2H halo | B block range | 2H halo], H the row
    // length; halo rows are loaded by 4H / VEC threads (rows outside the
    // hyperplane are clamped: such values are replaced by ghosts or wrapped
    // loads before use)
    constexpr int B = kBlock * VEC;
    constexpr int kTileX = LDSX ? 2 * B : 1;  // B + 4 H with 4 H <= B
    __shared__ __attribute__((aligned(16))) T xtile[2][kTileX];
    const int H = nl;
    const uint32_t q0 = tg.q0;
    const int me = int(q - q0) + 2 * H;
    const int nh = 2 * H / VEC;
    const int th = int(threadIdx.x);
    const bool hl = LDSX && th < 2 * nh;
    int hsrc = th < nh ? int(q0) - 2 * H + th * VEC : int(q0) + B + (th - nh) * VEC;
    hsrc = min(max(hsrc, 0), int(s.Q) - VEC);
    const int hdst = th < nh ? th * VEC : 2 * H + B + (th - nh) * VEC;
    // axis N-2 rows at -2, -1, +1, +2 that wrap across a periodic edge
    uint32_t wrapm = 0;
    if constexpr (LDSX) {
        if ((s.periodic >> (N - 2)) & 1u) {
            const int nd = s.n[N - 2];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int sh = j < 2 ? j - 2 : j - 1;
                const int kk = ii[N - 2] + sh;
                if (kk < 0 || kk >= nd) wrapm |= 1u << j;
            }
        }
    }
    const bool anywrap = __builtin_amdgcn_ballot_w64(wrapm != 0) != 0;
    // wave-level edge masks (computed once): bit d of wgm set when some lane
    // of the wave has a ghost node on middle axis d; the last axis' edges
    uint32_t wgm = 0;
#pragma unroll
    for (int d = 1; d < N - 1; ++d)
        if (__builtin_amdgcn_ballot_w64(((gmask >> (4 * d)) & 15u) != 0) != 0) wgm |= 1u << d;
    const bool wgxl = __builtin_amdgcn_ballot_w64(gxl) != 0, wgxr = __builtin_amdgcn_ballot_w64(gxr) != 0;

    // axis-0 plane j (-2 <= j <= n0 + 1) of this group: wrapped, or ghosts
    auto ax0 = [&](int j) -> P {
        if (j >= 0 && j < n0) return ldp<T, VEC>(W + int64_t(j) * s0 + q);
        if (per0) return ldp<T, VEC>(W + int64_t(j < 0 ? j + n0 : j - n0) * s0 + q);
        const int b = j < 0 ? 0 : n0 - 1, in = j < 0 ? 1 : n0 - 2;
        const P vb = ldp<T, VEC>(W + int64_t(b) * s0 + q), vin = ldp<T, VEC>(W + int64_t(in) * s0 + q);
        P g;
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            g.v[e] = (j == -1 || j == n0) ? ghost(vb.v[e], vin.v[e]) : ghost2(vb.v[e], vin.v[e]);
        return g;
    };
    // float64: the farthest axis-0 neighbour is loaded a plane ahead (4D
    // float64 230.5 -> 224.1 ms per solve, held at occupancy 3 with a few
    // values spilled; float32 with the same: 109.2 -> 116.2 ms, not used)
    constexpr bool kAx0Ahead = sizeof(T) == 8;
    P r0 = ax0(i0b - 2), r1 = ax0(i0b - 1), r2 = ax0(i0b), r3 = ax0(i0b + 1), r4, r5;
    if constexpr (kAx0Ahead) r4 = ax0(i0b + 2);
    // The next plane's middle-axis neighbours, halo rows and V^n are loaded
    // while this plane is computed (the barrier waits for LDS only), and are
    // copied into place after the compute, when they have landed.
    constexpr int NMG = LDSX ? N - 3 : N - 2;  // middle axes loaded from memory
    constexpr int NMA = NMG > 0 ? NMG : 1;
    // with two or more such axes the second set of packs would cost an
    // occupancy level: those load in their own plane's step
    constexpr bool kPref = NMG <= 1;
    P cu[NMA][4], nx[NMA][4];
    auto load_mid = [&](int i, P (&o)[NMA][4]) {
        const ODP_GLOBAL T *pl = W + int64_t(i) * s0 + q;
#pragma unroll
        for (int d = 1; d <= NMG; ++d)
#pragma unroll
            for (int j = 0; j < 4; ++j) o[d - 1][j] = ldp<T, VEC>(pl + off[d][j]);
    };
    if constexpr (NMG > 0 && kPref) load_mid(i0b, cu);
    P hq, vn, vnx;
    if (LDSX && hl) hq = ldp<T, VEC>(W + int64_t(i0b) * s0 + hsrc);
    if (kPref && wa != 0.0) vn = ldp_nt<T, VEC>(Vn + int64_t(i0b) * s0 + q);
    T nanacc = T(0);
    for (int i0 = i0b; i0 < i0e; ++i0) {
        if constexpr (kAx0Ahead) {
            if (i0 + 1 < i0e) r5 = ax0(i0 + 3);
        } else {
            r4 = ax0(i0 + 2);
        }
        const P wc = r2;
        const ODP_GLOBAL T *plane = W + int64_t(i0) * s0 + q;
        const int in = min(i0 + 1, i0e - 1);
        T *tl = xtile[i0 & 1];
        if constexpr (LDSX) {
            stp_lds<T, VEC>(tl + me, wc);
            if (hl) {
                stp_lds<T, VEC>(tl + hdst, hq);
                hq = ldp<T, VEC>(W + int64_t(in) * s0 + hsrc);
            }
        }
        if constexpr (NMG > 0 && kPref) load_mid(in, nx);
        if constexpr (NMG > 0 && !kPref) load_mid(i0, cu);
        if (kPref && wa != 0.0) vnx = ldp_nt<T, VEC>(Vn + int64_t(in) * s0 + q);
        if constexpr (LDSX) __syncthreads();
        Acc<T> acc[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            acc[j] = Acc<T>{T(0), T(0)};
            T dl, dr;
            eno2_diffs(r0.v[j], r1.v[j], wc.v[j], r3.v[j], r4.v[j], dl, dr);
            acc_axis<T, DYN, N>(cf[j], 0, dl, dr, acc[j]);
        }
#pragma unroll
        for (int d = 1; d < N - 1; ++d) {
            P l2, l1, p1, p2;
            if (LDSX && d == N - 2) {
                l2 = ldp_lds<T, VEC>(tl + me - 2 * H);
                l1 = ldp_lds<T, VEC>(tl + me - H);
                p1 = ldp_lds<T, VEC>(tl + me + H);
                p2 = ldp_lds<T, VEC>(tl + me + 2 * H);
                if (anywrap) {
                    if (wrapm & 1u) l2 = ldp<T, VEC>(plane + off[d][0]);
                    if (wrapm & 2u) l1 = ldp<T, VEC>(plane + off[d][1]);
                    if (wrapm & 4u) p1 = ldp<T, VEC>(plane + off[d][2]);
                    if (wrapm & 8u) p2 = ldp<T, VEC>(plane + off[d][3]);
                }
            } else {
                l2 = cu[d - 1][0];
                l1 = cu[d - 1][1];
                p1 = cu[d - 1][2];
                p2 = cu[d - 1][3];
            }
            // ghosts: one uniform branch, taken by the waves that hold a lane
            // next to a non-periodic face of axis d
            if (wgm & (1u << d)) {
                const uint32_t gm = (gmask >> (4 * d)) & 15u;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const T a1 = ghost(wc.v[e], p1.v[e]), a2 = ghost2(wc.v[e], p1.v[e]);
                    const T a3 = ghost(l1.v[e], wc.v[e]);
                    const T b1 = ghost(wc.v[e], l1.v[e]), b2 = ghost2(wc.v[e], l1.v[e]);
                    const T b3 = ghost(p1.v[e], wc.v[e]);
                    if (gm & 2u) { l1.v[e] = a1; l2.v[e] = a2; }
                    else if (gm & 1u) l2.v[e] = a3;
                    if (gm & 4u) { p1.v[e] = b1; p2.v[e] = b2; }
                    else if (gm & 8u) p2.v[e] = b3;
                }
            }
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                T dl, dr;
                eno2_diffs(l2.v[j], l1.v[j], wc.v[j], p1.v[j], p2.v[j], dl, dr);
                acc_axis<T, DYN, N>(cf[j], d, dl, dr, acc[j]);
            }
        }
        // last axis: e[0..VEC+3] = nodes il-2 .. il+VEC+1
        T e[VEC + 4];
        if constexpr (LDSX) {
            e[0] = tl[me + xo[0]];
            e[1] = tl[me + xo[1]];
            e[VEC + 2] = tl[me + xo[2]];
            e[VEC + 3] = tl[me + xo[3]];
        } else {
            e[0] = plane[xo[0]];
            e[1] = plane[xo[1]];
            e[VEC + 2] = plane[xo[2]];
            e[VEC + 3] = plane[xo[3]];
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) e[j + 2] = wc.v[j];
        if (wgxl) {
            const T g1 = ghost(wc.v[0], wc.v[1]), g2 = ghost2(wc.v[0], wc.v[1]);
            if (gxl) { e[1] = g1; e[0] = g2; }
        }
        if (wgxr) {
            const T g1 = ghost(wc.v[VEC - 1], wc.v[VEC - 2]), g2 = ghost2(wc.v[VEC - 1], wc.v[VEC - 2]);
            if (gxr) { e[VEC + 2] = g1; e[VEC + 3] = g2; }
        }
        const int64_t o = int64_t(i0) * s0 + q;
        if (!kPref && wa != 0.0) vn = ldp_nt<T, VEC>(Vn + o);
        P zr, gr;
        if (clamp) zr = ldp_nt<T, VEC>(Z + o);
        if (obst) gr = ldp_nt<T, VEC>(G + o);
        P res;
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            T dl, dr;
            eno2_diffs(e[j], e[j + 1], e[j + 2], e[j + 3], e[j + 4], dl, dr);
            acc_axis<T, DYN, N>(cf[j], N - 1, dl, dr, acc[j]);
            const T Lh = acc_finish<T, DYN, N>(cf[j], acc[j]);
            T v = fma_t(dt, Lh, wc.v[j]);
            if (wa != 0.0) v = fma_t(ra, vn.v[j], rb * v);
            if (clamp) {
                if (tmax ? zr.v[j] > v : zr.v[j] < v) v = zr.v[j];
            }
            if (obst) {
                if (omax ? gr.v[j] > v : gr.v[j] < v) v = gr.v[j];
            }
            nanacc = fma_t(v, T(0), nanacc);
            res.v[j] = v;
        }
        if (active) stp_nt<T, VEC>(out + o, res);
        r0 = r1;
        r1 = r2;
        r2 = r3;
        r3 = r4;
        if constexpr (kAx0Ahead) r4 = r5;
        if constexpr (NMG > 0 && kPref) {
#pragma unroll
            for (int d = 0; d < NMG; ++d)
#pragma unroll
                for (int j = 0; j < 4; ++j) cu[d][j] = nx[d][j];
        }
        if (kPref && wa != 0.0) vn = vnx;
    }
    if (nanacc != nanacc && active) atomicOr(s.flags, 1);
}

// The 4D float32 last stage (V^n, clamp and LDS exchange) is held to 128
// VGPRs (occupancy 4; two values spill): measured faster than occupancy 3.
// So are the 4D float64 stages with the LDS exchange (the last stage spills
// seven values): float64 64^4 and 80^4 1.5-3% faster, and every 4D
// first-order stage kernel then keeps 4 blocks per CU resident.
template <typename T, int DYN, int N, int VEC, int KIND>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(N == 4 && (KIND & 4) && (sizeof(T) == 8 || KIND == 7) ? 4 : 1))) void stage_vec_kernel(const SolveDesc *__restrict__ descs,
                                                           const uint32_t *__restrict__ tile_solve,
                                                           const uint32_t *__restrict__ tile_local,
                                                           int stage, int step_from_desc,
                                                           int64_t fixed_step, int xgroup) {
    static_assert(N >= 2, "the last axis must differ from the marched axis");
    constexpr bool kVn = KIND & 1;
    constexpr bool kClamp = KIND & 2;
    constexpr bool kLdsK = (KIND & 4) && N >= 3;
    constexpr bool kObst = (KIND & 8) && kClamp;
    // quad tiles (six dimensions): the four waves of a block are the 2x2
    // (axis 1, axis 2) pairs of a square at one offset in their cubes
    constexpr bool kQuad = (KIND & 64) && N == 6 && kLdsK;
    const uint32_t L = xcd_logical(blockIdx.x, gridDim.x, uint32_t(xgroup));
    const uint32_t si = tile_solve ? tile_solve[L] : 0u;
    const uint32_t lt = tile_solve ? tile_local[L] : L;
    const SolveDesc &s = descs[si];

    const int64_t nsteps = *s.nsteps;
    const int64_t k = (step_from_desc ? *s.step : 0) + fixed_step;
    if (k >= nsteps || stage >= s.rk_order) return;

    const uint32_t cid = lt / s.nqb;
    const uint32_t qb = lt - cid * s.nqb;
    const TileGroup tg = tile_group(s, qb, threadIdx.x, VEC);
    const bool active = tg.active;
    const uint32_t q = tg.q;

    int ii[N];
    ii[0] = 0;
    uint32_t rem = q;
#pragma unroll
    for (int d = N - 1; d >= 1; --d) {
        const uint32_t t = fdiv(rem, s.div[d]);
        ii[d] = int(rem - t * s.div[d].d);
        rem = t;
    }
    // middle axes 1..N-2: whole-group vector neighbours
    int32_t offL[N], offR[N];
    uint32_t gl = 0, gr = 0;
#pragma unroll
    for (int d = 1; d < N - 1; ++d) {
        const int32_t st = s.stride[d], nd = s.n[d];
        const bool per = (s.periodic >> d) & 1u;
        if (ii[d] > 0) offL[d] = -st;
        else if (per) offL[d] = (nd - 1) * st;
        else { offL[d] = 0; gl |= 1u << d; }
        if (ii[d] < nd - 1) offR[d] = st;
        else if (per) offR[d] = -(nd - 1) * st;
        else { offR[d] = 0; gr |= 1u << d; }
    }
    // last axis: a row holds nl points in a pitch of s.pitch elements (a
    // multiple of VEC); group elements past the row end (j > jend) are padding
    const int nl = s.n[N - 1];
    const int il = ii[N - 1];
    const int jend = nl - 1 - il;
    const bool perl = (s.periodic >> (N - 1)) & 1u;
    int32_t oxl, oxr;
    bool gxl = false, gxr = false;
    if (il > 0) oxl = -1;
    else if (perl) oxl = nl - 1;
    else { oxl = 0; gxl = true; }
    if (jend >= VEC) oxr = VEC;
    else if (perl) oxr = -il;
    else { oxr = 0; gxr = true; }

    Coef<T, DYN, N> cf[VEC];
#pragma unroll
    for (int j = 0; j < VEC; ++j) {
        int jj[N];
#pragma unroll
        for (int d = 0; d < N; ++d) jj[d] = ii[d];
        jj[N - 1] = il + j;
        cf[j] = make_coef<T, DYN, N>(s, jj);
    }

    const T *Wg, *Vng;
    T *outg;
    stage_buffers<T>(s, stage, k, Wg, Vng, outg);
    const ODP_GLOBAL T *W = (const ODP_GLOBAL T *)Wg;
    const ODP_GLOBAL T *Vn = (const ODP_GLOBAL T *)Vng;
    // reference of the comparison: an array, or (tvn) V^n, which is already
    // in registers (the stencil centre for RK1, vq after the first stage)
    const ODP_GLOBAL T *Zr = (const ODP_GLOBAL T *)s.tref;
    const ODP_GLOBAL T *Gr = (const ODP_GLOBAL T *)s.oref;
    const bool tmax = s.tmax, omax = s.omax, tvn = s.tvn;
    ODP_GLOBAL T *out = (ODP_GLOBAL T *)outg;
    double wa, wb;
    rk_weights(s.rk_order, stage, wa, wb);
    const T ra = T(wa), rb = T(wb);
    const T dt = T(s.dt_sched[k]);

    const int64_t s0 = s.s0;
    const int n0 = s.n0;
    const bool per0 = s.periodic & 1u;
    const int i0b = int(cid) * s.chunk;
    const int i0e = min(i0b + s.chunk, n0);
    // plane index of the axis-0 neighbour beyond j (wrapped when periodic,
    // clamped otherwise: the value is then replaced by a ghost or unused)
    auto plane_of = [&](int j) -> int64_t {
        if (j >= n0) j = per0 ? j - n0 : n0 - 1;
        if (j < 0) j = per0 ? j + n0 : 0;
        return int64_t(j) * s0;
    };

    // Every access is a uniform plane base plus this thread's 32-bit element
    // offset inside the plane (a plane holds fewer than 2^31 elements), so
    // the per-lane address arithmetic is done once, before the march.
    uint32_t qL[N], qR[N];
#pragma unroll
    for (int d = 1; d < N - 1; ++d) {
        qL[d] = uint32_t(int32_t(q) + offL[d]);
        qR[d] = uint32_t(int32_t(q) + offR[d]);
    }
    const uint32_t qxl = uint32_t(int32_t(q) + oxl), qxr = uint32_t(int32_t(q) + oxr);

    // Wave-uniform switches (almost every wave has none of them set): a lane
    // on a non-periodic face of a middle axis, of the last axis, or a group
    // that extends past the end of its row (padded rows).  The ghost and row
    // end logic sits in branches that such waves skip.
    const bool anyg = __builtin_amdgcn_ballot_w64((gl | gr) != 0) != 0;
    const bool rowx = __builtin_amdgcn_ballot_w64(gxl || gxr || jend < VEC - 1) != 0;
    // which faces any lane of the wave is on: bit d of wgl (wgr) set when
    // some lane is on the lower (upper) non-periodic face of middle axis d
    uint32_t wgl = 0, wgr = 0;
#pragma unroll
    for (int d = 1; d < N - 1; ++d) {
        if (__builtin_amdgcn_ballot_w64((gl >> d) & 1u) != 0) wgl |= 1u << d;
        if (__builtin_amdgcn_ballot_w64((gr >> d) & 1u) != 0) wgr |= 1u << d;
    }

    using P = Pack<T, VEC>;
    const int wlast = i0e, vlast = i0e - 1;
    T nanacc = T(0);

    // Block-level exchange through LDS (KIND bit 2, chosen by the host for
    // ndim >= 3 and a row pitch H <= 128 VEC): each plane's values of the
    // block's range [q0, q0 + B) of the hyperplane, with one row of H
    // elements beyond each end (loaded by 2 H / VEC threads one plane ahead),
    // are written to a double-buffered tile, from which every lane reads its
    // neighbours along axis N-2 (+-H) and along the last axis (same row,
    // wrapped when periodic).  Lanes on the first or last row of axis N-2
    // replace that value by a ghost, or, when the axis is periodic, by a
    // load of the wrapped row.
    // Quad tiles: each wave exchanges its own range of 64 VEC elements with a
    // row of halo on each side (loaded by its first 2 H / VEC lanes) in a
    // region of its own, and reads its neighbours along axis 1 (axis 2) on
    // the side of its partner wave w ^ 2 (w ^ 1) from the partner's region,
    // at the same offset; the other side is a memory load.
    constexpr int B = kBlock * VEC;
    // B + 2 H with H <= B / 2; quad: 4 (B / 4 + 2 H) with H <= B / 8
    constexpr int kTile = kLdsK ? 2 * B : 1;
    __shared__ __attribute__((aligned(16))) T tile[2][kTile];
    const int H = s.pitch;
    const uint32_t q0 = tg.q0;
    const int nh = H / VEC;
    const int th = int(threadIdx.x);
    int me, hsrc, hdst;
    bool hl;
    int dq1 = 0, dq2 = 0;       // kQuad: partner offsets in the tile
    bool up1 = false, up2 = false;  // kQuad: the wave is the upper pair member
    if constexpr (kQuad) {
        constexpr int WS = 64 * VEC;
        const int R = WS + 2 * H;
        const int w = th >> 6, l = th & 63;
        me = w * R + int(q - q0) + H;
        hl = l < 2 * nh;
        hsrc = l < nh ? int(q0) - H + l * VEC : int(q0) + WS + (l - nh) * VEC;
        hdst = w * R + (l < nh ? l * VEC : H + WS + (l - nh) * VEC);
        up1 = (w >> 1) & 1;
        up2 = w & 1;
        dq1 = ((w ^ 2) - w) * R;
        dq2 = ((w ^ 1) - w) * R;
    } else {
        me = int(q - q0) + H;
        hl = kLdsK && th < 2 * nh;
        hsrc = th < nh ? int(q0) - H + th * VEC : int(q0) + B + (th - nh) * VEC;
        hdst = th < nh ? th * VEC : H + B + (th - nh) * VEC;
    }
    hsrc = min(max(hsrc, 0), int(s.Q) - VEC);  // rows outside the hyperplane are never read
    bool lane_wrap = false;
    if constexpr (kLdsK)
        lane_wrap = ((s.periodic >> (N - 2)) & 1u) && (ii[N - 2] == 0 || ii[N - 2] == s.n[N - 2] - 1);
    const bool anywrap = __builtin_amdgcn_ballot_w64(lane_wrap) != 0;

    // The march is software pipelined: while plane i is computed, the loads
    // for plane i+1 (its in-plane neighbours, V^n, V0 and the halo rows) and
    // the stencil input of plane i+2 are in flight.  Registers have fixed
    // roles over a 4-plane cycle (unrolled by hand), so that no register
    // that a load in flight will write is ever copied (a copy would wait for
    // the load).  Indexes past the chunk end are clamped to its last plane
    // (L2 hits).  A difference shared by two points (W(i+1) - W(i) between
    // consecutive planes, W_{j+1} - W_j inside the group) is computed once:
    // it is the same subtraction, so the bits do not change.
    constexpr int NM = N > 2 ? N - 2 : 1;       // middle axes 1..N-2
    constexpr int NG = kLdsK ? N - 3 : N - 2;   // middle axes loaded from memory
    struct Nb {
        P l[NM], r[NM];
        T xl, xr;
    };
    // Live registers per thread: the stencil input of planes i, i+1 and the
    // one loading (plane i-1 survives only as the difference dm), the
    // in-plane neighbours of planes i and i+1, one pack each of V^n, V0 and
    // halo (reloaded once the previous plane's value has been used).
    P w[4];          // stencil-input ring (planes i-1, i, i+1, i+2)
    Nb nb[2];        // in-plane neighbours: plane i, plane i+1 (loading)
    P vq, zq;        // V^n and the comparison's reference of plane i
    P gq;            // obstacle of plane i (KIND bit 3)
    P hq;            // halo rows of plane i
    // kQuad: the memory side of axes 1 and 2
    uint32_t qg1 = 0, qg2 = 0;
    if constexpr (kQuad) {
        qg1 = up1 ? qR[1] : qL[1];
        qg2 = up2 ? qR[2] : qL[2];
    }
    auto load_nb = [&](int i, Nb &o) {
        const ODP_GLOBAL T *plane = W + int64_t(i) * s0;
        if constexpr (kQuad) {
            // axes 1 and 2: the memory side, held in l until the partner's
            // side is read from LDS
            o.l[0] = ldp<T, VEC>(plane + qg1);
            o.l[1] = ldp<T, VEC>(plane + qg2);
            o.l[2] = ldp<T, VEC>(plane + qL[3]);
            o.r[2] = ldp<T, VEC>(plane + qR[3]);
            return;
        }
#pragma unroll
        for (int d = 1; d <= NG; ++d) {
            o.l[d - 1] = ldp<T, VEC>(plane + qL[d]);
            o.r[d - 1] = ldp<T, VEC>(plane + qR[d]);
        }
        if constexpr (!kLdsK) {
            o.xl = plane[qxl];
            o.xr = plane[qxr];
        }
    };
    auto load_pw = [&](int i, P &ov, P &oz, P &og) {
        const int64_t o = int64_t(i) * s0 + q;
        if constexpr (kVn) ov = ldp_nt<T, VEC>(Vn + o);
        if constexpr (kClamp) oz = ldp_nt<T, VEC>(Zr + o);
        if constexpr (kObst) og = ldp_nt<T, VEC>(Gr + o);
    };
    w[0] = ldp<T, VEC>(W + plane_of(i0b - 1) + q);
    w[1] = ldp<T, VEC>(W + plane_of(i0b) + q);
    w[2] = ldp<T, VEC>(W + plane_of(i0b + 1) + q);
    // ndim >= 5: the outer-axis neighbours are loaded in their own plane's
    // step (three axes of pipelined neighbours would cost an occupancy level)
    constexpr bool kPipeNb = N <= 4;
    if constexpr (kPipeNb) load_nb(i0b, nb[0]);
    load_pw(i0b, vq, zq, gq);
    if (hl) hq = ldp<T, VEC>(W + int64_t(i0b) * s0 + hsrc);
    P dm;  // W(i) - W(i-1)
#pragma unroll
    for (int j = 0; j < VEC; ++j) dm.v[j] = w[1].v[j] - w[0].v[j];

    auto step = [&](auto kc, int i) {
        constexpr int K = decltype(kc)::value;
        const P &wc = w[(K + 1) % 4], &wp = w[(K + 2) % 4];
        Nb &cur = nb[K % 2];
        T *tb = &tile[K & 1][0];
        const int in = min(i + 1, vlast);
        if constexpr (kLdsK) {
            stp_lds<T, VEC>(tb + me, wc);
            if (hl) {
                stp_lds<T, VEC>(tb + hdst, hq);
                hq = ldp<T, VEC>(W + int64_t(in) * s0 + hsrc);
            }
        }
        // loads for the planes ahead
        if constexpr (kPipeNb) load_nb(in, nb[(K + 1) % 2]);
        else load_nb(min(i, vlast), cur);
        w[(K + 3) % 4] = ldp<T, VEC>(W + plane_of(min(i + 2, wlast)) + q);
        if constexpr (kLdsK) {
            __syncthreads();
            cur.l[N - 3] = ldp_lds<T, VEC>(tb + me - H);
            cur.r[N - 3] = ldp_lds<T, VEC>(tb + me + H);
            cur.xl = tb[me + oxl];
            cur.xr = tb[me + oxr];
            if constexpr (kQuad) {
                const P p1 = ldp_lds<T, VEC>(tb + me + dq1), p2 = ldp_lds<T, VEC>(tb + me + dq2);
                const P g1 = cur.l[0], g2 = cur.l[1];
                cur.l[0] = up1 ? p1 : g1;
                cur.r[0] = up1 ? g1 : p1;
                cur.l[1] = up2 ? p2 : g2;
                cur.r[1] = up2 ? g2 : p2;
            }
            if (anywrap && lane_wrap) {
                const ODP_GLOBAL T *plane = W + int64_t(min(i, vlast)) * s0;
                cur.l[N - 3] = ldp<T, VEC>(plane + qL[N - 2]);
                cur.r[N - 3] = ldp<T, VEC>(plane + qR[N - 2]);
            }
        }

        Acc<T> acc[VEC];
        P dp;  // W(i+1) - W(i)
        // The edge cases (ghost nodes) are substituted in one uniform branch
        // per kind and plane, taken only on the edge planes of axis 0 and by
        // the waves that hold a lane on a non-periodic face: the common path
        // is straight-line.  The values, and the order of the accumulation,
        // are the same either way.
        T dl0[VEC], dr0[VEC];
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            dp.v[j] = wp.v[j] - wc.v[j];
            dl0[j] = dm.v[j];
            dr0[j] = dp.v[j];
        }
        if (!per0 && (i == 0 || i == n0 - 1)) {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                if (i == 0) dl0[j] = wc.v[j] - ghost(wc.v[j], wp.v[j]);
                if (i == n0 - 1) dr0[j] = ghost_d(wc.v[j], dm.v[j]) - wc.v[j];
            }
        }
        T na[NM][VEC], nbv[NM][VEC];  // neighbour values of the middle axes
#pragma unroll
        for (int d = 1; d < N - 1; ++d)
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                na[d - 1][j] = cur.l[d - 1].v[j];
                nbv[d - 1][j] = cur.r[d - 1].v[j];
            }
        if (anyg) {
#pragma unroll
            for (int d = 1; d < N - 1; ++d) {
                if (wgl & (1u << d)) {
                    const bool on = (gl >> d) & 1u;
#pragma unroll
                    for (int j = 0; j < VEC; ++j) {
                        const T gv = ghost(wc.v[j], cur.r[d - 1].v[j]);
                        na[d - 1][j] = on ? gv : na[d - 1][j];
                    }
                }
                if (wgr & (1u << d)) {
                    const bool on = (gr >> d) & 1u;
#pragma unroll
                    for (int j = 0; j < VEC; ++j) {
                        const T gv = ghost(wc.v[j], cur.l[d - 1].v[j]);
                        nbv[d - 1][j] = on ? gv : nbv[d - 1][j];
                    }
                }
            }
        }
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            acc[j].L = T(0);
            acc[j].n2 = T(0);
            acc_axis<T, DYN, N>(cf[j], 0, dl0[j], dr0[j], acc[j]);
        }
#pragma unroll
        for (int d = 1; d < N - 1; ++d) {
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                acc_axis<T, DYN, N>(cf[j], d, wc.v[j] - na[d - 1][j], nbv[d - 1][j] - wc.v[j], acc[j]);
        }
        if (!rowx) {
            T dx[VEC + 1];
            dx[0] = wc.v[0] - cur.xl;
#pragma unroll
            for (int j = 1; j < VEC; ++j) dx[j] = wc.v[j] - wc.v[j - 1];
            dx[VEC] = cur.xr - wc.v[VEC - 1];
#pragma unroll
            for (int j = 0; j < VEC; ++j) acc_axis<T, DYN, N>(cf[j], N - 1, dx[j], dx[j + 1], acc[j]);
        } else {
#pragma unroll
            for (int j = 0; j < VEC; ++j) {
                T a = j > 0 ? wc.v[j > 0 ? j - 1 : 0] : cur.xl;
                T b = (j < jend && j < VEC - 1) ? wc.v[j < VEC - 1 ? j + 1 : j] : cur.xr;
                if (j == 0 && gxl) a = ghost(wc.v[0], b);
                if (j == jend && gxr) b = ghost(wc.v[j], a);
                acc_axis<T, DYN, N>(cf[j], N - 1, wc.v[j] - a, b - wc.v[j], acc[j]);
            }
        }
        P res;
        T nan_here = T(0);
#pragma unroll
        for (int j = 0; j < VEC; ++j) {
            const T Lh = acc_finish<T, DYN, N>(cf[j], acc[j]);
            T v = fma_t(dt, Lh, wc.v[j]);
            if constexpr (kVn) v = fma_t(ra, vq.v[j], rb * v);
            if constexpr (kClamp) {
                const T z = tvn ? (kVn ? vq.v[j] : wc.v[j]) : zq.v[j];
                if (tmax ? z > v : z < v) v = z;
            }
            if constexpr (kObst) {
                if (omax ? gq.v[j] > v : gq.v[j] < v) v = gq.v[j];
            }
            // v * 0 is NaN exactly when v is not finite (padding excluded)
            nan_here = fma_t(j > jend ? T(0) : v, T(0), nan_here);
            res.v[j] = v;
        }
        // V^n and V0 of the next plane: a step of compute hides their latency
        load_pw(in, vq, zq, gq);
        if (i < i0e) {
            nanacc += nan_here;
            if (active) stp_nt<T, VEC>(out + int64_t(i) * s0 + q, res);
        }
        dm = dp;
    };
    using K0 = std::integral_constant<int, 0>;
    using K1 = std::integral_constant<int, 1>;
    using K2 = std::integral_constant<int, 2>;
    using K3 = std::integral_constant<int, 3>;
    // 4-plane cycles.  Up to four dimensions the march stops at the chunk
    // end (the condition is the same for the whole block, so every barrier
    // is reached by all of its waves; loads already issued for the planes
    // beyond are clamped and never used): small grids take chunks shorter
    // than a cycle.  From five dimensions on chunks are whole cycles, and
    // planes past a shorter last chunk are computed from clamped loads and
    // neither stored nor checked (the exits cost the 6D kernel 2%).
    for (int i = i0b; i < i0e; i += 4) {
        step(K0{}, i);
        if constexpr (N <= 4)
            if (i + 1 >= i0e) break;
        step(K1{}, i + 1);
        if constexpr (N <= 4)
            if (i + 2 >= i0e) break;
        step(K2{}, i + 2);
        if constexpr (N <= 4)
            if (i + 3 >= i0e) break;
        step(K3{}, i + 3);
    }
    if (nanacc != nanacc && active) atomicOr(s.flags, 1);
}

// --------------------------------------------------------- launchers

template <typename T, int DYN, int N, int VEC>
static hipError_t launch_stage_t(int kind, const SolveDesc *d, const uint32_t *ts, const uint32_t *tl,
                                 uint32_t nblocks, int stage, int from_desc, int64_t step, int xg,
                                 hipStream_t st) {
    if constexpr (DYN == 4) {
        // pursuit-evasion: point per lane, first order or ENO2 (bit 4), the
        // costate-box pass (bit 5) or the update
        if (kind & 32) {
            if (kind & 16)
                hipLaunchKernelGGL((stage_point_kernel<T, DYN, N, 2, 1>), dim3(nblocks), dim3(kBlock), 0, st, d,
                                   ts, tl, stage, from_desc, step, xg);
            else
                hipLaunchKernelGGL((stage_point_kernel<T, DYN, N, 1, 1>), dim3(nblocks), dim3(kBlock), 0, st, d,
                                   ts, tl, stage, from_desc, step, xg);
        } else if (kind & 16) {
            hipLaunchKernelGGL((stage_point_kernel<T, DYN, N, 2, 0>), dim3(nblocks), dim3(kBlock), 0, st, d, ts,
                               tl, stage, from_desc, step, xg);
        } else {
            hipLaunchKernelGGL((stage_point_kernel<T, DYN, N, 1, 0>), dim3(nblocks), dim3(kBlock), 0, st, d, ts,
                               tl, stage, from_desc, step, xg);
        }
    } else if (kind & 16) {
        // second-order ENO (method flags at run time): VEC points per thread
        // where rows allow it, else point per lane
        if constexpr (VEC >= 2 && N >= 3 && DYN != 0) {
            if (kind & 4)
                hipLaunchKernelGGL((stage_eno2_vec_kernel<T, DYN, N, VEC, true>), dim3(nblocks), dim3(kBlock), 0,
                                   st, d, ts, tl, stage, from_desc, step, xg);
            else
                hipLaunchKernelGGL((stage_eno2_vec_kernel<T, DYN, N, VEC, false>), dim3(nblocks), dim3(kBlock), 0,
                                   st, d, ts, tl, stage, from_desc, step, xg);
        } else if constexpr (VEC >= 2 && N >= 2 && DYN != 0)
            hipLaunchKernelGGL((stage_eno2_vec_kernel<T, DYN, N, VEC, false>), dim3(nblocks), dim3(kBlock), 0, st,
                               d, ts, tl, stage, from_desc, step, xg);
        else
            hipLaunchKernelGGL((stage_point_kernel<T, DYN, N, 2, 0>), dim3(nblocks), dim3(kBlock), 0, st, d, ts,
                               tl, stage, from_desc, step, xg);
    } else if constexpr (N == 1) {
        hipLaunchKernelGGL((stage_kernel<T, DYN, N>), dim3(nblocks), dim3(kBlock), 0, st, d, ts, tl,
                           stage, from_desc, step, xg);
    } else {
#define ODP_STAGE_CASE(K)                                                                          \
    case K:                                                                                        \
        hipLaunchKernelGGL((stage_vec_kernel<T, DYN, N, VEC, K>), dim3(nblocks), dim3(kBlock), 0, st, \
                           d, ts, tl, stage, from_desc, step, xg);                                 \
        break;
        // bit 3 (a second comparison) only comes with bit 1; bit 2 (LDS)
        // only from three dimensions on; bit 6 (quad tiles) only in six
        switch (kind) {
            ODP_STAGE_CASE(0)
            ODP_STAGE_CASE(1)
            ODP_STAGE_CASE(2)
            ODP_STAGE_CASE(3)
            ODP_STAGE_CASE(10)
            ODP_STAGE_CASE(11)
        default:
            if constexpr (N >= 3) {
                switch (kind) {
                    ODP_STAGE_CASE(4)
                    ODP_STAGE_CASE(5)
                    ODP_STAGE_CASE(6)
                    ODP_STAGE_CASE(7)
                    ODP_STAGE_CASE(14)
                    ODP_STAGE_CASE(15)
                default:
                    if constexpr (N == 6) {
                        switch (kind) {
                            ODP_STAGE_CASE(68)
                            ODP_STAGE_CASE(69)
                            ODP_STAGE_CASE(70)
                            ODP_STAGE_CASE(71)
                            ODP_STAGE_CASE(78)
                            ODP_STAGE_CASE(79)
                        default: return hipErrorInvalidValue;
                        }
                    } else {
                        return hipErrorInvalidValue;
                    }
                }
            } else {
                return hipErrorInvalidValue;
            }
        }
#undef ODP_STAGE_CASE
    }
    return hipGetLastError();
}

template <typename T, int DYN, int N>
static hipError_t launch_stage_v(int vec, int kind, const SolveDesc *d, const uint32_t *ts,
                                 const uint32_t *tl, uint32_t nb, int stage, int fd, int64_t step,
                                 int xg, hipStream_t st) {
    if constexpr (N == 1 || DYN == 0 || DYN == 4) {
        return launch_stage_t<T, DYN, N, 1>(kind, d, ts, tl, nb, stage, fd, step, xg, st);
    } else {
        if constexpr (sizeof(T) == 4) {
            if (vec == 4) return launch_stage_t<T, DYN, N, 4>(kind, d, ts, tl, nb, stage, fd, step, xg, st);
        }
        if (vec == 2) return launch_stage_t<T, DYN, N, 2>(kind, d, ts, tl, nb, stage, fd, step, xg, st);
        return launch_stage_t<T, DYN, N, 1>(kind, d, ts, tl, nb, stage, fd, step, xg, st);
    }
}

}  // namespace odp
