/*
 * Oracle for the time-dependent Hamilton-Jacobi level-set solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, float64 CPU version of
 * the method, written to be checked by eye against the paper.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg load it; the
 * HIP library neither links nor calls it, and the two share no source.
 *
 * What it computes (paper: Algorithm 1 "solving HJ PDE", the HJ PDE and the
 * HJ variational inequality equations, the Grid / Time Integration / Spatial
 * Derivatives subsections, and the DubinsCapture example's input selection):
 *
 *   V(z, tau=tau_0) = V_init (V0 = l(z) unless a restart value is given)
 *   per time step, per Runge-Kutta stage, per grid point i (all independent):
 *     p-_d = (W_i - W_{i-e_d}) / dx_d,  p+_d = (W_{i+e_d} - W_i) / dx_d
 *       (first-order upwind; or second-order ENO, Spatial Derivatives: the
 *       one-sided difference corrected by half the smaller-magnitude second
 *       difference of the two candidate stencils, over dx_d)
 *     pbar = (p+ + p-) / 2
 *     (u*, d*) = argmin_d argmax_u pbar . f(z_i, u, d)
 *     H  = pbar . f(z_i, u*, d*)
 *     Hh = H + 1/2 sum_d alpha_d (p+_d - p-_d)         (Lax-Friedrichs)
 *     stage output = a * V^n + b * (W + dt * Hh)        (TVD Runge-Kutta)
 *   after the last stage of a step, the computation method (paper: the
 *   Computation Methods for Value Function table): a target-set operation
 *   V = min or max of V and V0, V^n (the value before the step) or a target
 *   array l, then an obstacle operation V = min or max of V and an obstacle
 *   array g (reach-avoid: min with l, then max with g); a tube (BRT) is
 *   min(V, V0)
 *   dt = CFL / sum_d (alpha^max_d / dx_d), clipped so that t lands exactly on
 *   every requested output time.
 *
 * Readings of the paper taken here (each one is listed in the design notes):
 *  - time runs forward in time-to-go tau = -s, so the step adds dt * Hh;
 *  - the dissipation enters with a plus sign in time-to-go, which makes the
 *    scheme the monotone (upwind-consistent) Lax-Friedrichs scheme; the
 *    printed minus sign, combined with the printed update, is downwind;
 *  - alpha_d(z) is the largest |f_d(z,u,d)| over the admissible inputs
 *    (equal to the costate-box maximum for bang-bang inputs, whose |f_d|
 *    does not depend on the costate);
 *  - dt carries the CFL number, which the printed step formula omits;
 *  - one dt per full step; the computation method after every full step,
 *    the target-set operation before the obstacle operation, the "value
 *    over time" reference being V^n, the value at the start of the step;
 *  - ghost value beyond a non-periodic edge: V_b + sgn(V_b) |V_b - V_in|,
 *    sgn(0) = 0, so the ghost has the boundary node's sign; the second
 *    ghost (second order) V_b + 2 sgn(V_b) |V_b - V_in|;
 *  - ENO2 ties (equal magnitudes) take the stencil nearer the upwind side
 *    (the first of the two candidates);
 *  - bang-bang tie at a zero switching function: a maximiser takes +max, a
 *    minimiser -max (the DubinsCapture listing's >= 0 branches);
 *  - third-order TVD-RK (Shu-Osher) added beside the paper's first and
 *    second order.
 *
 * Parity pinned by the non-GPU tests (closed forms, exact discrete identities,
 * invariants and reductions); absolute Dubins / 4D / 6D values beyond those
 * pins are "parity unpinned": the paper prints no value-function numbers.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OG_MAXD 6

/* ------------------------------------------------------------------ grid */

typedef struct {
    int ndim;
    long n[OG_MAXD];
    double lo[OG_MAXD], hi[OG_MAXD];
    int periodic[OG_MAXD];
    double dx[OG_MAXD];
    long stride[OG_MAXD];
    long npts;
} og_grid;

/* Grid section: node count, bounds and periodic flag per axis.  A periodic
 * axis excludes its upper bound, so its spacing is (hi - lo) / n. */
static int og_grid_init(og_grid *g, int ndim, const long *n, const double *lo,
                        const double *hi, const int *periodic)
{
    if (ndim < 1 || ndim > OG_MAXD) return -1;
    g->ndim = ndim;
    g->npts = 1;
    for (int d = 0; d < ndim; ++d) {
        if (n[d] < 3 || !(hi[d] > lo[d])) return -1;
        g->n[d] = n[d];
        g->lo[d] = lo[d];
        g->hi[d] = hi[d];
        g->periodic[d] = periodic[d] ? 1 : 0;
        g->dx[d] = g->periodic[d] ? (hi[d] - lo[d]) / (double)n[d]
                                  : (hi[d] - lo[d]) / (double)(n[d] - 1);
        g->npts *= n[d];
    }
    /* row-major, last axis fastest */
    long s = 1;
    for (int d = ndim - 1; d >= 0; --d) {
        g->stride[d] = s;
        s *= g->n[d];
    }
    return 0;
}

static void og_unravel(const og_grid *g, long idx, long *ii)
{
    for (int d = 0; d < g->ndim; ++d) {
        ii[d] = idx / g->stride[d];
        idx -= ii[d] * g->stride[d];
    }
}

static void og_state(const og_grid *g, const long *ii, double *z)
{
    for (int d = 0; d < g->ndim; ++d) z[d] = g->lo[d] + (double)ii[d] * g->dx[d];
}

/* ------------------------------------------------------------ dynamics */

enum { OG_SI = 0, OG_DUBINS3D = 1, OG_DYNCAR4D = 2, OG_TWODUBINS6D = 3, OG_PE3D = 4 };

typedef struct {
    int id;
    int u_mode; /* 1: the control maximises, 0: minimises */
    int d_mode; /* 1: the disturbance maximises, 0: minimises */
    double p[16];
} og_dyn;

static int og_dyn_ndim_ok(const og_dyn *dy, int ndim)
{
    switch (dy->id) {
    case OG_SI: return ndim >= 1 && ndim <= OG_MAXD;
    case OG_DUBINS3D: return ndim == 3;
    case OG_DYNCAR4D: return ndim == 4;
    case OG_TWODUBINS6D: return ndim == 6;
    case OG_PE3D: return ndim == 3;
    default: return 0;
    }
}

/* Bang-bang choice for a box input entering through switching function s:
 * the optimiser picks the bound whose product with s is largest (maximiser)
 * or smallest (minimiser); ties at s == 0 follow the DubinsCapture listing. */
static double og_bang(double s, double bound, int maximise)
{
    if (maximise) return s >= 0.0 ? bound : -bound;
    return s >= 0.0 ? -bound : bound;
}

/* Optimal control u* and disturbance d* for costate pbar (Algorithm 1,
 * "optimal control and disturbances"). */
static void og_opt_inputs(const og_dyn *dy, int ndim, const double *z, const double *pbar,
                          double *u, double *dd)
{
    (void)z;
    switch (dy->id) {
    case OG_SI: {
        /* ball |u| <= u_max: argmax p.u = u_max p/|p|, argmin = -u_max p/|p| */
        double nrm = 0.0;
        for (int d = 0; d < ndim; ++d) nrm += pbar[d] * pbar[d];
        nrm = sqrt(nrm);
        double sgn = dy->u_mode ? 1.0 : -1.0;
        for (int d = 0; d < ndim; ++d) u[d] = nrm > 0.0 ? sgn * dy->p[0] * pbar[d] / nrm : 0.0;
        break;
    }
    case OG_DUBINS3D: /* theta' = w: switching function p_theta */
        u[0] = og_bang(pbar[2], dy->p[1], dy->u_mode);
        break;
    case OG_DYNCAR4D: /* v' = a, theta' = w */
        u[0] = og_bang(pbar[2], dy->p[0], dy->u_mode);
        u[1] = og_bang(pbar[3], dy->p[1], dy->u_mode);
        break;
    case OG_TWODUBINS6D: /* evader turn on axis 2, pursuer turn on axis 5 */
        u[0] = og_bang(pbar[2], dy->p[1], dy->u_mode);
        dd[0] = og_bang(pbar[5], dy->p[3], dy->d_mode);
        break;
    case OG_PE3D: /* evader turn a: p_x y - p_y x - p_theta; pursuer turn b: p_theta */
        u[0] = og_bang(pbar[0] * z[1] - pbar[1] * z[0] - pbar[2], dy->p[2], dy->u_mode);
        dd[0] = og_bang(pbar[2], dy->p[3], dy->d_mode);
        break;
    }
}

/* f(z, u, d): the state derivative (appendix equations). */
static void og_dynamics(const og_dyn *dy, int ndim, const double *z, const double *u,
                        const double *dd, double *f)
{
    switch (dy->id) {
    case OG_SI: /* z' = c + u */
        for (int d = 0; d < ndim; ++d) f[d] = dy->p[1 + d] + u[d];
        break;
    case OG_DUBINS3D: /* x' = v cos th, y' = v sin th, th' = w */
        f[0] = dy->p[0] * cos(z[2]);
        f[1] = dy->p[0] * sin(z[2]);
        f[2] = u[0];
        break;
    case OG_DYNCAR4D: /* x' = v cos th, y' = v sin th, v' = a, th' = w */
        f[0] = z[2] * cos(z[3]);
        f[1] = z[2] * sin(z[3]);
        f[2] = u[0];
        f[3] = u[1];
        break;
    case OG_TWODUBINS6D: /* two Dubins cars: evader (u), pursuer (d) */
        f[0] = dy->p[0] * cos(z[2]);
        f[1] = dy->p[0] * sin(z[2]);
        f[2] = u[0];
        f[3] = dy->p[2] * cos(z[5]);
        f[4] = dy->p[2] * sin(z[5]);
        f[5] = dd[0];
        break;
    case OG_PE3D: /* relative pursuit-evasion: evader a, pursuer b, speeds v_a, v_b */
        f[0] = -dy->p[0] + dy->p[1] * cos(z[2]) + u[0] * z[1];
        f[1] = dy->p[1] * sin(z[2]) - u[0] * z[0];
        f[2] = dd[0] - u[0];
        break;
    }
}

/* alpha_d(z) = max over admissible (u, d) of |f_d(z, u, d)| (Algorithm 1's
 * dissipation coefficient, reading: the costate box covers both signs). */
static void og_alpha(const og_dyn *dy, int ndim, const double *z, double *alpha)
{
    if (dy->id == OG_SI) {
        /* max over the ball of |c_d + u_d| is reached at u = +-u_max e_d */
        for (int d = 0; d < ndim; ++d) alpha[d] = fabs(dy->p[1 + d]) + dy->p[0];
        return;
    }
    /* box inputs: |f_d| is affine in each input, so its maximum over the box
     * is at a vertex; enumerate every vertex. */
    double ub[4] = {0}, db[4] = {0};
    int nu = 0, nd = 0;
    switch (dy->id) {
    case OG_DUBINS3D: ub[0] = dy->p[1]; nu = 1; break;
    case OG_DYNCAR4D: ub[0] = dy->p[0]; ub[1] = dy->p[1]; nu = 2; break;
    case OG_TWODUBINS6D: ub[0] = dy->p[1]; db[0] = dy->p[3]; nu = 1; nd = 1; break;
    case OG_PE3D: ub[0] = dy->p[2]; db[0] = dy->p[3]; nu = 1; nd = 1; break;
    }
    for (int d = 0; d < ndim; ++d) alpha[d] = 0.0;
    int nv = 1 << (nu + nd);
    for (int v = 0; v < nv; ++v) {
        double u[4], dd[4], f[OG_MAXD];
        for (int a = 0; a < nu; ++a) u[a] = ((v >> a) & 1) ? ub[a] : -ub[a];
        for (int a = 0; a < nd; ++a) dd[a] = ((v >> (nu + a)) & 1) ? db[a] : -db[a];
        og_dynamics(dy, ndim, z, u, dd, f);
        for (int d = 0; d < ndim; ++d)
            if (fabs(f[d]) > alpha[d]) alpha[d] = fabs(f[d]);
    }
}

/* Switching functions of the box inputs (controls first, then
 * disturbances) at z: input j is bang-bang on the sign of c[j] . p.  coord[j]
 * is k when c[j] is the unit vector e_k, else -1.  Returns the input count. */
static int og_switching(const og_dyn *dy, int ndim, const double *z, double c[2][OG_MAXD],
                        int *coord, double *bound, int *maximise)
{
    for (int j = 0; j < 2; ++j)
        for (int d = 0; d < ndim; ++d) c[j][d] = 0.0;
    switch (dy->id) {
    case OG_DUBINS3D:
        c[0][2] = 1.0; coord[0] = 2; bound[0] = dy->p[1]; maximise[0] = dy->u_mode;
        return 1;
    case OG_DYNCAR4D:
        c[0][2] = 1.0; coord[0] = 2; bound[0] = dy->p[0]; maximise[0] = dy->u_mode;
        c[1][3] = 1.0; coord[1] = 3; bound[1] = dy->p[1]; maximise[1] = dy->u_mode;
        return 2;
    case OG_TWODUBINS6D:
        c[0][2] = 1.0; coord[0] = 2; bound[0] = dy->p[1]; maximise[0] = dy->u_mode;
        c[1][5] = 1.0; coord[1] = 5; bound[1] = dy->p[3]; maximise[1] = dy->d_mode;
        return 2;
    case OG_PE3D:
        c[0][0] = z[1]; c[0][1] = -z[0]; c[0][2] = -1.0; coord[0] = -1;
        bound[0] = dy->p[2]; maximise[0] = dy->u_mode;
        c[1][2] = 1.0; coord[1] = 2; bound[1] = dy->p[3]; maximise[1] = dy->d_mode;
        return 2;
    }
    return 0;
}

/* alpha_d(z) over the costate box (Algorithm 1's dissipation: the largest
 * |dH/dp_d| = |f_d(z, u*(p), d*(p))| for p in [dmin, dmax]).  Every input is
 * bang-bang on the sign of its switching function, so only the input
 * patterns (one sign per input) that some p in the box realises count.  A
 * pattern is tested by restricting the box: a switching function that is a
 * single coordinate p_k keeps p_k >= 0 (or p_k <= 0, closed at 0) of that
 * coordinate's interval; a general linear form (at most one per dynamics
 * here) is then ranged over the restricted box term by term, and its sign
 * condition holds if the range reaches it (>= 0: max >= 0; < 0: min < 0). */
static void og_alpha_box(const og_dyn *dy, int ndim, const double *z, const double *dmin,
                         const double *dmax, double *alpha)
{
    double c[2][OG_MAXD], bound[2];
    int coord[2], maximise[2];
    const int ni = og_switching(dy, ndim, z, c, coord, bound, maximise);
    const int nu = (dy->id == OG_TWODUBINS6D || dy->id == OG_PE3D) ? 1 : ni;
    for (int d = 0; d < ndim; ++d) alpha[d] = 0.0;
    for (int pat = 0; pat < (1 << ni); ++pat) {
        double lo[OG_MAXD], hi[OG_MAXD];
        for (int d = 0; d < ndim; ++d) { lo[d] = dmin[d]; hi[d] = dmax[d]; }
        int ok = 1;
        for (int j = 0; j < ni && ok; ++j) {
            if (coord[j] < 0) continue;
            const int k = coord[j];
            if ((pat >> j) & 1) { if (lo[k] < 0.0) lo[k] = 0.0; }
            else                { if (hi[k] > 0.0) hi[k] = 0.0; }
            if (lo[k] > hi[k] || (!((pat >> j) & 1) && !(lo[k] < 0.0))) ok = 0;
        }
        for (int j = 0; j < ni && ok; ++j) {
            if (coord[j] >= 0) continue;
            double smin = 0.0, smax = 0.0;
            for (int d = 0; d < ndim; ++d) {
                const double a = c[j][d] * lo[d], b = c[j][d] * hi[d];
                smin += a < b ? a : b;
                smax += a < b ? b : a;
            }
            if ((pat >> j) & 1) ok = smax >= 0.0;
            else ok = smin < 0.0;
        }
        if (!ok) continue;
        double u[4] = {0}, dd[4] = {0}, f[OG_MAXD];
        for (int j = 0; j < ni; ++j) {
            const double v = og_bang(((pat >> j) & 1) ? 1.0 : -1.0, bound[j], maximise[j]);
            if (j < nu) u[j] = v; else dd[j - nu] = v;
        }
        og_dynamics(dy, ndim, z, u, dd, f);
        for (int d = 0; d < ndim; ++d)
            if (fabs(f[d]) > alpha[d]) alpha[d] = fabs(f[d]);
    }
}

/* Dynamics whose dissipation is taken over the costate box: the relative
 * pursuit-evasion model, whose evader input enters three axes through a
 * switching function that mixes the costate with the state.  (For the other
 * box-input dynamics every input drives one axis with |f_d| equal to its
 * bound whatever its sign, so the box gives the all-inputs alpha; a pin
 * checks that equality.) */
static int og_box_dynamics(const og_dyn *dy) { return dy->id == OG_PE3D; }

/* --------------------------------------------------------------- fields */

/* A field is anything that can return W at a flat index: a plain array, or
 * a Runge-Kutta stage evaluated on demand (for sampled checks). */
typedef struct og_field og_field;
struct og_field {
    double (*get)(const og_field *self, long idx);
    const double *arr;
    const void *ctx;
    int level;
};

static double og_get_array(const og_field *f, long idx) { return f->arr[idx]; }

static double og_sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* W at the node s steps from point idx (multi-index ii) along axis d,
 * |s| <= 2 (the second-order stencil reaches two nodes). */
static double og_neighbor(const og_grid *g, const og_field *W, long idx, const long *ii,
                          int d, int s)
{
    long k = ii[d] + s;
    if (k >= 0 && k < g->n[d]) return W->get(W, idx + (long)s * g->stride[d]);
    if (g->periodic[d]) {
        long kw = (k + g->n[d]) % g->n[d];
        return W->get(W, idx + (kw - ii[d]) * g->stride[d]);
    }
    /* m-th ghost node beyond the edge node b (m = 1, 2): extrapolate away
     * from zero by m times the edge difference, so that every ghost keeps
     * the sign of the edge node */
    long b = k < 0 ? 0 : g->n[d] - 1;
    long in = k < 0 ? 1 : g->n[d] - 2;
    long m = k < 0 ? -k : k - b;
    double vb = W->get(W, idx + (b - ii[d]) * g->stride[d]);
    double vin = W->get(W, idx + (in - ii[d]) * g->stride[d]);
    return vb + (double)m * og_sgn(vb) * fabs(vb - vin);
}

/* ENO stencil choice: the second difference of smaller magnitude (the first
 * on a tie).  With f32 the magnitudes are compared as float32 values
 * computed in float32 from the float32-rounded stencil (the precision of a
 * float32 solve), which lets a single step be compared decision for
 * decision with a float32 implementation. */
static int og_eno_first(double x, double y)
{
    return fabs(x) <= fabs(y);
}

static int og_eno_first_f32(double w0, double w1, double w2, double w3)
{
    /* second differences (w2 - w1) - (w1 - w0) and (w3 - w2) - (w2 - w1) */
    float a0 = (float)w0, a1 = (float)w1, a2 = (float)w2, a3 = (float)w3;
    float d01 = a1 - a0, d12 = a2 - a1, d23 = a3 - a2;
    float x = d12 - d01, y = d23 - d12;
    return fabsf(x) <= fabsf(y);
}

/* One-sided derivatives p-, p+ and the costate pbar = (p+ + p-)/2 at point
 * idx (multi-index ii), first-order or ENO2 (order 2). */
static void og_costate(const og_grid *g, const og_field *W, long idx, const long *ii, int order,
                       int eno_f32, double *pm, double *pp, double *pbar)
{
    const int N = g->ndim;
    double wc = W->get(W, idx);
    for (int d = 0; d < N; ++d) {
        double wl = og_neighbor(g, W, idx, ii, d, -1);
        double wr = og_neighbor(g, W, idx, ii, d, +1);
        double dm = wc - wl, dp = wr - wc;
        if (order == 2) {
            /* second-order ENO (the level-set text's ENO2): one-sided
             * difference plus half of the smaller second difference of the
             * two stencils that contain it */
            double wll = og_neighbor(g, W, idx, ii, d, -2);
            double wrr = og_neighbor(g, W, idx, ii, d, +2);
            double sm = dm - (wl - wll);   /* second difference at i-1 */
            double s0 = dp - dm;           /* at i */
            double sp = (wrr - wr) - dp;   /* at i+1 */
            int fm = eno_f32 ? og_eno_first_f32(wll, wl, wc, wr) : og_eno_first(sm, s0);
            int fp = eno_f32 ? og_eno_first_f32(wl, wc, wr, wrr) : og_eno_first(s0, sp);
            dm = dm + 0.5 * (fm ? sm : s0);
            dp = dp - 0.5 * (fp ? s0 : sp);
        }
        pm[d] = dm / g->dx[d];
        pp[d] = dp / g->dx[d];
        pbar[d] = 0.5 * (pp[d] + pm[d]);
    }
}

/* Costate box of Algorithm 1: D_min, D_max = the smallest and largest pbar_d
 * over the grid, for field W (box[0..N) min, box[N..2N) max). */
static void og_costate_box(const og_grid *g, const og_field *W, int order, double *box)
{
    const int N = g->ndim;
    for (int d = 0; d < N; ++d) {
        box[d] = INFINITY;
        box[N + d] = -INFINITY;
    }
#pragma omp parallel
    {
        double part[2 * OG_MAXD];
        for (int d = 0; d < N; ++d) {
            part[d] = INFINITY;
            part[N + d] = -INFINITY;
        }
#pragma omp for schedule(static)
        for (long i = 0; i < g->npts; ++i) {
            long ii[OG_MAXD] = {0};
            double pm[OG_MAXD], pp[OG_MAXD], pbar[OG_MAXD];
            og_unravel(g, i, ii);
            og_costate(g, W, i, ii, order, 0, pm, pp, pbar);
            for (int d = 0; d < N; ++d) {
                if (pbar[d] < part[d]) part[d] = pbar[d];
                if (pbar[d] > part[N + d]) part[N + d] = pbar[d];
            }
        }
#pragma omp critical
        for (int d = 0; d < N; ++d) {
            if (part[d] < box[d]) box[d] = part[d];
            if (part[N + d] > box[N + d]) box[N + d] = part[N + d];
        }
    }
}

/* Lax-Friedrichs numerical Hamiltonian at point idx (one pass of the body
 * of Algorithm 1's grid loops for one point). alpha_glob != NULL selects the
 * global-alpha approximation; box != NULL (dynamics whose dissipation depends
 * on the costate) gives the costate box for alpha. */
static double og_hhat(const og_grid *g, const og_dyn *dy, const og_field *W, long idx,
                      const double *alpha_glob, int order, int eno_f32, const double *box)
{
    const int N = g->ndim;
    long ii[OG_MAXD] = {0};
    double z[OG_MAXD] = {0};
    og_unravel(g, idx, ii);
    og_state(g, ii, z);
    double pm[OG_MAXD], pp[OG_MAXD], pbar[OG_MAXD];
    og_costate(g, W, idx, ii, order, eno_f32, pm, pp, pbar);

    double u[OG_MAXD] = {0}, dd[OG_MAXD] = {0}, f[OG_MAXD];
    og_opt_inputs(dy, N, z, pbar, u, dd);
    og_dynamics(dy, N, z, u, dd, f);
    double H = 0.0;
    for (int d = 0; d < N; ++d) H += pbar[d] * f[d];

    double alpha[OG_MAXD];
    if (alpha_glob) {
        for (int d = 0; d < N; ++d) alpha[d] = alpha_glob[d];
    } else if (box) {
        og_alpha_box(dy, N, z, box, box + N, alpha);
    } else {
        og_alpha(dy, N, z, alpha);
    }
    double diss = 0.0;
    for (int d = 0; d < N; ++d) diss += 0.5 * alpha[d] * (pp[d] - pm[d]);
    return H + diss;
}

/* TVD Runge-Kutta stage weights: stage s output = a V^n + b (W + dt L(W)). */
static void og_rk_weights(int order, int stage, double *a, double *b)
{
    *a = 0.0;
    *b = 1.0;
    if (order == 2 && stage == 1) { *a = 0.5; *b = 0.5; }
    if (order == 3 && stage == 1) { *a = 0.75; *b = 0.25; }
    if (order == 3 && stage == 2) { *a = 1.0 / 3.0; *b = 2.0 / 3.0; }
}

static double og_combine(double a, double b, double vn, double w, double dt, double hh)
{
    if (a == 0.0) return w + dt * hh;
    return a * vn + b * (w + dt * hh);
}

/* alpha^max_d = max over all grid points of alpha_d(z_i). */
static void og_alpha_max(const og_grid *g, const og_dyn *dy, double *amax)
{
    for (int d = 0; d < g->ndim; ++d) amax[d] = 0.0;
    for (long i = 0; i < g->npts; ++i) {
        long ii[OG_MAXD];
        double z[OG_MAXD], a[OG_MAXD];
        og_unravel(g, i, ii);
        og_state(g, ii, z);
        og_alpha(dy, g->ndim, z, a);
        for (int d = 0; d < g->ndim; ++d)
            if (a[d] > amax[d]) amax[d] = a[d];
    }
}

/* alpha^max_d over the costate box: the largest alpha_i of Algorithm 1's
 * dissipation loop, each alpha_i taken over the box [box, box + N). */
static void og_alpha_box_max(const og_grid *g, const og_dyn *dy, const double *box, double *amax)
{
    for (int d = 0; d < g->ndim; ++d) amax[d] = 0.0;
#pragma omp parallel
    {
        double part[OG_MAXD] = {0};
#pragma omp for schedule(static)
        for (long i = 0; i < g->npts; ++i) {
            long ii[OG_MAXD];
            double z[OG_MAXD], a[OG_MAXD];
            og_unravel(g, i, ii);
            og_state(g, ii, z);
            og_alpha_box(dy, g->ndim, z, box, box + g->ndim, a);
            for (int d = 0; d < g->ndim; ++d)
                if (a[d] > part[d]) part[d] = a[d];
        }
#pragma omp critical
        for (int d = 0; d < g->ndim; ++d)
            if (part[d] > amax[d]) amax[d] = part[d];
    }
}

static double og_dt_cfl(const og_grid *g, const double *amax, double cfl, double max_dt)
{
    double s = 0.0;
    for (int d = 0; d < g->ndim; ++d) s += amax[d] / g->dx[d];
    double dt = cfl / s; /* +inf when nothing moves: the step then lands on tau */
    if (max_dt > 0.0 && dt > max_dt) dt = max_dt;
    return dt;
}

static int og_setup(og_grid *g, og_dyn *dy, int ndim, const long *n, const double *lo,
                    const double *hi, const int *periodic, int dyn_id, int u_mode, int d_mode,
                    const double *params)
{
    if (og_grid_init(g, ndim, n, lo, hi, periodic)) return -1;
    memset(dy, 0, sizeof(*dy));
    dy->id = dyn_id;
    dy->u_mode = u_mode;
    dy->d_mode = d_mode;
    for (int k = 0; k < 16; ++k) dy->p[k] = params[k];
    if (!og_dyn_ndim_ok(dy, ndim)) return -1;
    return 0;
}

/* ------------------------------------------------------------ solve */

/* Computation method after a full step (paper: Computation Methods for
 * Value Function table).  tmode: 0 none, 1 minVWithV0, 2 maxVWithV0,
 * 3 minVWithVInit, 4 maxVWithVInit (reference V^n, the value before the
 * step), 5 minVWithVTarget, 6 maxVWithVTarget (reference: target array);
 * omode: 0 none, 1 minVWithObstacle, 2 maxVWithObstacle.  The target-set
 * operation comes first (reach-avoid: max(min(V, l), g)). */
static double og_clamp(double v, long i, int tmode, int omode, const double *V0, const double *Vn,
                       const double *target, const double *obstacle)
{
    if (tmode) {
        const double ref = (tmode <= 2) ? V0[i] : (tmode <= 4) ? Vn[i] : target[i];
        if (tmode % 2 == 1) {
            if (ref < v) v = ref;
        } else {
            if (ref > v) v = ref;
        }
    }
    if (omode == 1 && obstacle[i] < v) v = obstacle[i];
    if (omode == 2 && obstacle[i] > v) v = obstacle[i];
    return v;
}

static int og_modes_ok(int tmode, int omode, const double *target, const double *obstacle)
{
    if (tmode < 0 || tmode > 6 || omode < 0 || omode > 2) return 0;
    if (tmode >= 5 && !target) return 0;
    if (omode && !obstacle) return 0;
    return 1;
}

/* Full solve from tau[0] to tau[ntau-1].  V_all (nullable) receives V at
 * every tau[k] (ntau slices, slice 0 = the start value).  set_slices 0 or 1:
 * target and obstacle are one grid array each, for the whole horizon;
 * set_slices = ntau: time-varying sets l(z, t), g(z, t) (the paper's
 * time-varying target and obstacle), slice k holds the set at tau[k] and the
 * steps from tau[k-1] to tau[k] compare with slice k-1, the set at the time
 * the interval starts (the table's index t-1).  Returns 0 or -1. */
int oracle_hj_solve(int ndim, const long *n, const double *lo, const double *hi,
                    const int *periodic, int dyn_id, int u_mode, int d_mode,
                    const double *params, const double *V0, const double *V_init,
                    const double *tau, int ntau, int rk_order, double cfl, int tmode, int omode,
                    const double *target, const double *obstacle, int set_slices,
                    int space_order, int global_alpha, double max_dt, double *V_out, double *V_all,
                    long *steps_out, double *dt_first, double *dt_min, double *dt_max)
{
    og_grid g;
    og_dyn dy;
    if (og_setup(&g, &dy, ndim, n, lo, hi, periodic, dyn_id, u_mode, d_mode, params)) return -1;
    if (rk_order < 1 || rk_order > 3 || ntau < 2 || !(cfl > 0.0)) return -1;
    if (space_order != 1 && space_order != 2) return -1;
    if (!og_modes_ok(tmode, omode, target, obstacle)) return -1;
    if (set_slices != 0 && set_slices != 1 && set_slices != ntau) return -1;
    for (int k = 1; k < ntau; ++k)
        if (!(tau[k] > tau[k - 1])) return -1;

    const long P = g.npts;
    double *Vn = V_out;
    double *S1 = (double *)malloc(sizeof(double) * (size_t)P);
    double *S2 = rk_order == 3 ? (double *)malloc(sizeof(double) * (size_t)P) : NULL;
    double *Nx = (double *)malloc(sizeof(double) * (size_t)P);
    if (!S1 || !Nx || (rk_order == 3 && !S2)) {
        free(S1); free(S2); free(Nx);
        return -1;
    }
    memcpy(Vn, V_init ? V_init : V0, sizeof(double) * (size_t)P);
    if (V_all) memcpy(V_all, Vn, sizeof(double) * (size_t)P);

    double t = tau[0];
    int k = 1;
    long steps = 0;
    double dtmin = INFINITY, dtmax = 0.0, dtfirst = 0.0;
    while (k < ntau) {
        /* alpha^max over the grid (recomputed every step) and the CFL step.
         * Dynamics whose dissipation depends on the costate take it, as in
         * Algorithm 1, from the alpha_i of the step's Hamiltonian evaluation:
         * over the costate box of V^n (the first stage's input); the
         * global-alpha approximation has no box and keeps the all-inputs
         * bound. */
        double amax[OG_MAXD];
        double box0[2 * OG_MAXD];
        const int box_cfl = og_box_dynamics(&dy) && !global_alpha;
        if (box_cfl) {
            og_field Vf = {og_get_array, Vn, NULL, 0};
            og_costate_box(&g, &Vf, space_order, box0);
            og_alpha_box_max(&g, &dy, box0, amax);
        } else {
            og_alpha_max(&g, &dy, amax);
        }
        double dt = og_dt_cfl(&g, amax, cfl, max_dt);
        double t_next;
        int land = 0;
        if (dt >= tau[k] - t) {
            dt = tau[k] - t;
            t_next = tau[k];
            land = 1;
        } else {
            t_next = t + dt;
        }
        const double *aglob = global_alpha ? amax : NULL;

        /* Runge-Kutta stages: stage s reads W (stencil) and V^n (pointwise) */
        double *stage_out[3] = {S1, S2, Nx};
        const double *W = Vn;
        for (int s = 0; s < rk_order; ++s) {
            double *out = (s == rk_order - 1) ? Nx : stage_out[s];
            double a, b;
            og_rk_weights(rk_order, s, &a, &b);
            og_field Wf = {og_get_array, W, NULL, 0};
            /* costate box of this Hamiltonian evaluation (dynamics whose
             * dissipation depends on it) */
            double box[2 * OG_MAXD];
            const int use_box = og_box_dynamics(&dy) && !aglob;
            if (use_box) {
                if (s == 0) memcpy(box, box0, sizeof(box));  /* the box of V^n, above */
                else og_costate_box(&g, &Wf, space_order, box);
            }
#pragma omp parallel for schedule(static)
            for (long i = 0; i < P; ++i) {
                double hh = og_hhat(&g, &dy, &Wf, i, aglob, space_order, 0, use_box ? box : NULL);
                out[i] = og_combine(a, b, Vn[i], W[i], dt, hh);
            }
            W = out;
        }
        /* computation method (a tube: V = min(V, V0), the HJ variational
         * inequality); Vn still holds the value before the step */
        if (tmode || omode) {
            const size_t off = set_slices > 1 ? (size_t)(k - 1) * (size_t)P : 0;
            const double *lk = target ? target + off : NULL;
            const double *gk = obstacle ? obstacle + off : NULL;
            for (long i = 0; i < P; ++i) Nx[i] = og_clamp(Nx[i], i, tmode, omode, V0, Vn, lk, gk);
        }
        memcpy(Vn, Nx, sizeof(double) * (size_t)P);

        if (steps == 0) dtfirst = dt;
        if (dt < dtmin) dtmin = dt;
        if (dt > dtmax) dtmax = dt;
        ++steps;
        t = t_next;
        if (land) {
            if (V_all) memcpy(V_all + (size_t)k * (size_t)P, Vn, sizeof(double) * (size_t)P);
            ++k;
        }
    }
    free(S1); free(S2); free(Nx);
    if (steps_out) *steps_out = steps;
    if (dt_first) *dt_first = dtfirst;
    if (dt_min) *dt_min = dtmin;
    if (dt_max) *dt_max = dtmax;
    return 0;
}

/* The CFL step and alpha^max alone (no time stepping). */
int oracle_cfl_dt(int ndim, const long *n, const double *lo, const double *hi,
                  const int *periodic, int dyn_id, int u_mode, int d_mode, const double *params,
                  double cfl, double *alpha_max_out, double *dt_out)
{
    og_grid g;
    og_dyn dy;
    if (og_setup(&g, &dy, ndim, n, lo, hi, periodic, dyn_id, u_mode, d_mode, params)) return -1;
    double amax[OG_MAXD];
    og_alpha_max(&g, &dy, amax);
    for (int d = 0; d < ndim; ++d) alpha_max_out[d] = amax[d];
    *dt_out = og_dt_cfl(&g, amax, cfl, 0.0);
    return 0;
}

/* ------------------------------------------- one step at sampled points */

typedef struct {
    const og_grid *g;
    const og_dyn *dy;
    const double *Vn;
    int rk_order;
    double dt;
    const double *aglob;
    int order;
    int eno_f32;
    const double *box;
} og_step_ctx;

/* Value of Runge-Kutta stage `level` (0 = V^n) at idx, evaluated on demand
 * from its own domain of dependence. */
static double og_stage_value(const og_field *self, long idx)
{
    const og_step_ctx *c = (const og_step_ctx *)self->ctx;
    if (self->level == 0) return c->Vn[idx];
    og_field prev = {og_stage_value, NULL, c, self->level - 1};
    double a, b;
    og_rk_weights(c->rk_order, self->level - 1, &a, &b);
    double hh = og_hhat(c->g, c->dy, &prev, idx, c->aglob, c->order, c->eno_f32, c->box);
    return og_combine(a, b, c->Vn[idx], og_stage_value(&prev, idx), c->dt, hh);
}

/* One full time step of size dt from V (whole grid, float64) evaluated only
 * at the flat indices idx[0..m): out[j] = V^{n+1}(idx[j]).  alpha_glob may be
 * NULL (per-point alpha). */
int oracle_step_at(int ndim, const long *n, const double *lo, const double *hi,
                   const int *periodic, int dyn_id, int u_mode, int d_mode,
                   const double *params, const double *V, const double *V0, double dt,
                   int rk_order, int tmode, int omode, const double *target, const double *obstacle,
                   const double *alpha_glob, int space_order, int eno_f32, long m, const long *idx,
                   double *out)
{
    og_grid g;
    og_dyn dy;
    if (og_setup(&g, &dy, ndim, n, lo, hi, periodic, dyn_id, u_mode, d_mode, params)) return -1;
    if (rk_order < 1 || rk_order > 3) return -1;
    if (space_order != 1 && space_order != 2) return -1;
    if (!og_modes_ok(tmode, omode, target, obstacle)) return -1;
    /* a costate box needs the whole stage input: one stage only (RK1) */
    double box[2 * OG_MAXD];
    const int use_box = og_box_dynamics(&dy) && !alpha_glob;
    if (use_box) {
        if (rk_order != 1) return -1;
        og_field Vf = {og_get_array, V, NULL, 0};
        og_costate_box(&g, &Vf, space_order, box);
    }
    og_step_ctx c = {&g, &dy, V, rk_order, dt, alpha_glob, space_order, eno_f32,
                     use_box ? box : NULL};
#pragma omp parallel for schedule(dynamic, 1)
    for (long j = 0; j < m; ++j) {
        og_field top = {og_stage_value, NULL, &c, rk_order};
        const double v = og_stage_value(&top, idx[j]);
        out[j] = og_clamp(v, idx[j], tmode, omode, V0, V, target, obstacle);
    }
    return 0;
}

/* ------------------------------------------ time-to-reach (static HJ) */

/* Time-to-reach by Lax-Friedrichs sweeping (the Time-independent HJ PDE
 * subsection and its Algorithm 2, after the cited sweeping method).  The TTR
 * phi solves  min_u max_d grad(phi) . f(z, u, d) = -1  outside the target,
 * phi = 0 on it.  Solving the Lax-Friedrichs numerical Hamiltonian of that
 * equation for phi_i gives the explicit point update
 *   phi_i <- min(phi_i, [1 + H + sum_d sigma_d (phi_{i+e_d} + phi_{i-e_d}) / (2 dx_d)]
 *                        / sum_d sigma_d / dx_d)
 * with H = pbar . f(z, u*, d*) at the centred costate pbar_d =
 * (phi_{i+e_d} - phi_{i-e_d}) / (2 dx_d) (u* minimising, d* maximising: the
 * caller passes those modes) and sigma_d = alpha_d(z), the largest |f_d|.
 * Readings: phi starts at 0 on the target (l(z) <= 0) and at `big`
 * elsewhere; target nodes stay 0; each iteration is one Gauss-Seidel sweep
 * over the nodes in row-major order, alternately forward and backward,
 * updating nodes off every non-periodic edge; then every node on a
 * non-periodic edge of axis d (axes in order) takes
 *   phi <- min(max(2 phi_a - phi_b, phi_b), phi)
 * with a, b the next two nodes inward along d; the iteration stops when the
 * largest change of an iteration is below eps (or after max_iters).  A node
 * with sum_d sigma_d = 0 keeps its value.
 * jacobi != 0: the parallel form instead of the sweep: every node of an
 * iteration reads the previous iterate only, and a node on the edges of
 * several axes takes the smallest of their extrapolations.  (The edge rule
 * keeps the smallest extrapolation an iteration ever produced, and the
 * extrapolation is not monotone in phi_b, so near non-periodic edges the
 * limit depends on the order of the updates.) */
int oracle_ttr_solve(int ndim, const long *n, const double *lo, const double *hi,
                     const int *periodic, int dyn_id, int u_mode, int d_mode,
                     const double *params, const double *target, double big, double eps,
                     long max_iters, int jacobi, double *phi, long *iters_out, double *change_out)
{
    og_grid g;
    og_dyn dy;
    if (og_setup(&g, &dy, ndim, n, lo, hi, periodic, dyn_id, u_mode, d_mode, params)) return -1;
    if (og_box_dynamics(&dy) || !(eps > 0.0) || max_iters < 1) return -1;
    const long P = g.npts;
    const int N = g.ndim;
    for (long i = 0; i < P; ++i) phi[i] = target[i] <= 0.0 ? 0.0 : big;
    double *old = (double *)malloc(sizeof(double) * (size_t)P);
    if (!old) return -1;
    long it = 0;
    double change = INFINITY;
    while (it < max_iters) {
        memcpy(old, phi, sizeof(double) * (size_t)P);
        const int backward = (int)(it & 1);
        for (long k = 0; k < P; ++k) {
            const long i = backward ? P - 1 - k : k;
            if (target[i] <= 0.0) continue;
            long ii[OG_MAXD] = {0};
            og_unravel(&g, i, ii);
            int edge = 0;
            for (int d = 0; d < N; ++d)
                if (!g.periodic[d] && (ii[d] == 0 || ii[d] == g.n[d] - 1)) edge = 1;
            if (edge) continue;
            double z[OG_MAXD] = {0}, pbar[OG_MAXD], nsum[OG_MAXD];
            og_state(&g, ii, z);
            og_field F = {og_get_array, jacobi ? old : phi, NULL, 0};
            for (int d = 0; d < N; ++d) {
                const double r = og_neighbor(&g, &F, i, ii, d, +1);
                const double l = og_neighbor(&g, &F, i, ii, d, -1);
                pbar[d] = (r - l) / (2.0 * g.dx[d]);
                nsum[d] = r + l;
            }
            double u[OG_MAXD] = {0}, dd[OG_MAXD] = {0}, f[OG_MAXD], sig[OG_MAXD];
            og_opt_inputs(&dy, N, z, pbar, u, dd);
            og_dynamics(&dy, N, z, u, dd, f);
            og_alpha(&dy, N, z, sig);
            double H = 0.0, num = 1.0, den = 0.0;
            for (int d = 0; d < N; ++d) H += pbar[d] * f[d];
            num += H;
            for (int d = 0; d < N; ++d) {
                num += sig[d] * nsum[d] / (2.0 * g.dx[d]);
                den += sig[d] / g.dx[d];
            }
            if (den > 0.0) {
                const double cand = num / den;
                if (cand < phi[i]) phi[i] = cand;
            }
        }
        /* edges of the non-periodic axes, axis by axis (Jacobi: from the
         * previous iterate, so the axes' extrapolations just combine by min) */
        const double *src = jacobi ? old : phi;
        for (int d = 0; d < N; ++d) {
            if (g.periodic[d]) continue;
            for (long i = 0; i < P; ++i) {
                if (target[i] <= 0.0) continue;
                long ii[OG_MAXD] = {0};
                og_unravel(&g, i, ii);
                const long s = g.stride[d];
                long a, b;
                if (ii[d] == 0) { a = i + s; b = i + 2 * s; }
                else if (ii[d] == g.n[d] - 1) { a = i - s; b = i - 2 * s; }
                else continue;
                double e = 2.0 * src[a] - src[b];
                if (src[b] > e) e = src[b];
                if (e < phi[i]) phi[i] = e;
            }
        }
        change = 0.0;
        for (long i = 0; i < P; ++i) {
            const double c = fabs(phi[i] - old[i]);
            if (c > change) change = c;
        }
        ++it;
        if (change < eps) break;
    }
    free(old);
    if (iters_out) *iters_out = it;
    if (change_out) *change_out = change;
    return 0;
}

/* alpha over a costate box and over all inputs at m states z (row-major,
 * m x ndim): test access to the dissipation coefficients. */
int oracle_alpha_box(int ndim, int dyn_id, int u_mode, int d_mode, const double *params, long m,
                     const double *z, const double *dmin, const double *dmax, double *alpha_box,
                     double *alpha_all)
{
    og_dyn dy;
    memset(&dy, 0, sizeof(dy));
    dy.id = dyn_id;
    dy.u_mode = u_mode;
    dy.d_mode = d_mode;
    for (int k = 0; k < 16; ++k) dy.p[k] = params[k];
    if (!og_dyn_ndim_ok(&dy, ndim) || dyn_id == OG_SI) return -1;
    for (long j = 0; j < m; ++j) {
        og_alpha_box(&dy, ndim, z + j * ndim, dmin, dmax, alpha_box + j * ndim);
        og_alpha(&dy, ndim, z + j * ndim, alpha_all + j * ndim);
    }
    return 0;
}

/* Algorithm 1's alpha^max for field V: the costate box of V, then the
 * largest box alpha over the grid (box_out: D_min[ndim], D_max[ndim]). */
int oracle_box_alpha_max(int ndim, const long *n, const double *lo, const double *hi,
                         const int *periodic, int dyn_id, int u_mode, int d_mode,
                         const double *params, const double *V, int space_order, double *box_out,
                         double *alpha_max_out)
{
    og_grid g;
    og_dyn dy;
    if (og_setup(&g, &dy, ndim, n, lo, hi, periodic, dyn_id, u_mode, d_mode, params)) return -1;
    if (dyn_id == OG_SI || (space_order != 1 && space_order != 2)) return -1;
    og_field Vf = {og_get_array, V, NULL, 0};
    og_costate_box(&g, &Vf, space_order, box_out);
    og_alpha_box_max(&g, &dy, box_out, alpha_max_out);
    return 0;
}

/* Hamiltonian p . f(z, u*, d*) with the optimal inputs for costate p at m
 * states (test access to the input choice). */
int oracle_hamiltonian(int ndim, int dyn_id, int u_mode, int d_mode, const double *params, long m,
                       const double *z, const double *p, double *H)
{
    og_dyn dy;
    memset(&dy, 0, sizeof(dy));
    dy.id = dyn_id;
    dy.u_mode = u_mode;
    dy.d_mode = d_mode;
    for (int k = 0; k < 16; ++k) dy.p[k] = params[k];
    if (!og_dyn_ndim_ok(&dy, ndim)) return -1;
    for (long j = 0; j < m; ++j) {
        double u[OG_MAXD] = {0}, dd[OG_MAXD] = {0}, f[OG_MAXD];
        og_opt_inputs(&dy, ndim, z + j * ndim, p + j * ndim, u, dd);
        og_dynamics(&dy, ndim, z + j * ndim, u, dd, f);
        H[j] = 0.0;
        for (int d = 0; d < ndim; ++d) H[j] += p[j * ndim + d] * f[d];
    }
    return 0;
}

/* Threads the OpenMP loops above use (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
