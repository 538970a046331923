/* CPU driver of the oracle for an AddressSanitizer / UndefinedBehaviorSanitizer
 * build: small solves of every dynamics, both spatial orders, every RK order,
 * the computation methods with time-varying sets and save_all, one-step
 * evaluation, the costate-box helpers and time to reach in both update
 * orders.  Prints "ok" on success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_hj_solve(int ndim, const long *n, const double *lo, const double *hi, const int *periodic, int dyn_id,
                    int u_mode, int d_mode, const double *params, const double *V0, const double *V_init,
                    const double *tau, int ntau, int rk_order, double cfl, int tmode, int omode,
                    const double *target, const double *obstacle, int set_slices, int space_order,
                    int global_alpha, double max_dt, double *V_out, double *V_all, long *steps_out,
                    double *dt_first, double *dt_min, double *dt_max);
int oracle_cfl_dt(int ndim, const long *n, const double *lo, const double *hi, const int *periodic, int dyn_id,
                  int u_mode, int d_mode, const double *params, double cfl, double *alpha_max_out, double *dt_out);
int oracle_step_at(int ndim, const long *n, const double *lo, const double *hi, const int *periodic, int dyn_id,
                   int u_mode, int d_mode, const double *params, const double *V, const double *V0, double dt,
                   int rk_order, int tmode, int omode, const double *target, const double *obstacle,
                   const double *alpha_glob, int space_order, int eno_f32, long m, const long *idx, double *out);
int oracle_ttr_solve(int ndim, const long *n, const double *lo, const double *hi, const int *periodic, int dyn_id,
                     int u_mode, int d_mode, const double *params, const double *target, double big, double eps,
                     long max_iters, int jacobi, double *phi, long *iters_out, double *change_out);
int oracle_alpha_box(int ndim, int dyn_id, int u_mode, int d_mode, const double *params, long m, const double *z,
                     const double *dmin, const double *dmax, double *alpha_box, double *alpha_all);
int oracle_hamiltonian(int ndim, int dyn_id, int u_mode, int d_mode, const double *params, long m,
                       const double *z, const double *p, double *H);
int oracle_box_alpha_max(int ndim, const long *n, const double *lo, const double *hi, const int *periodic,
                         int dyn_id, int u_mode, int d_mode, const double *params, const double *V,
                         int space_order, double *box_out, double *alpha_max_out);

static int fails = 0;
#define CHECK(c) do { if (!(c)) { printf("check failed line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static void grid_v0(int nd, const long *n, const double *lo, const double *hi, const int *per, double *V)
{
    long P = 1;
    for (int d = 0; d < nd; ++d) P *= n[d];
    for (long i = 0; i < P; ++i) {
        long r = i;
        double s = 0.0;
        for (int d = nd - 1; d >= 0; --d) {
            const long k = r % n[d];
            r /= n[d];
            const double dx = per[d] ? (hi[d] - lo[d]) / n[d] : (hi[d] - lo[d]) / (n[d] - 1);
            const double x = lo[d] + k * dx;
            if (d < 2) s += x * x;
        }
        V[i] = sqrt(s) - 1.0;
    }
}

int main(void)
{
    const int ids[5] = {0, 1, 2, 3, 4}, dims[5] = {2, 3, 4, 6, 3};
    const double prm[5][16] = {{1.0, 0.3, -0.2}, {1.0, 1.0}, {1.0, 1.0}, {1.0, 1.0, 1.0, 1.0}, {1.0, 1.0, 1.0, 1.0}};
    for (int k = 0; k < 5; ++k) {
        const int nd = dims[k];
        long n[6];
        double lo[6], hi[6];
        int per[6];
        long P = 1;
        for (int d = 0; d < nd; ++d) {
            n[d] = nd == 6 ? 5 + d % 2 : 7 + d;
            lo[d] = -4.0;
            hi[d] = 4.0;
            per[d] = 0;
            P *= n[d];
        }
        if (ids[k] == 1 || ids[k] == 4) per[2] = 1;
        if (ids[k] == 2) per[3] = 1;
        if (ids[k] == 3) per[2] = per[5] = 1;
        double *V0 = malloc(sizeof(double) * P), *V = malloc(sizeof(double) * P);
        double *all = malloc(sizeof(double) * 3 * P), *tg = malloc(sizeof(double) * 3 * P);
        grid_v0(nd, n, lo, hi, per, V0);
        for (long i = 0; i < 3 * P; ++i) tg[i] = V0[i % P] + 0.1 * (double)(i / P);
        const double tau[3] = {0.0, 0.05, 0.11};
        for (int order = 1; order <= 2; ++order)
            for (int rk = 1; rk <= 3; ++rk)
                for (int glob = 0; glob <= 1; ++glob) {
                    long steps = 0;
                    double a, b, c;
                    CHECK(oracle_hj_solve(nd, n, lo, hi, per, ids[k], 1, 0, prm[k], V0, NULL, tau, 3, rk, 0.8,
                                          5, 2, tg, tg, 3, order, glob, 0.0, V, all, &steps, &a, &b, &c) == 0);
                    CHECK(steps > 0 && isfinite(V[P - 1]));
                }
        double am[6], dt;
        CHECK(oracle_cfl_dt(nd, n, lo, hi, per, ids[k], 1, 0, prm[k], 0.8, am, &dt) == 0 && dt > 0);
        long idx[3] = {0, P / 2, P - 1};
        double out[3];
        CHECK(oracle_step_at(nd, n, lo, hi, per, ids[k], 1, 0, prm[k], V0, V0, 0.01, 1, 1, 0, NULL, NULL, NULL, 2,
                             1, 3, idx, out) == 0);
        if (ids[k] != 0) {
            double box[12], ab[6];
            const int rc = oracle_box_alpha_max(nd, n, lo, hi, per, ids[k], 1, 0, prm[k], V0, 2, box, ab);
            CHECK(rc == 0);
            double z[6] = {0.1, -0.2, 0.3, 0.4, 0.5, 0.6}, dmin[6], dmax[6], al[6], aa[6], p[6] = {1, -1, 1, -1, 1, -1};
            for (int d = 0; d < nd; ++d) { dmin[d] = -1.0; dmax[d] = 1.0; }
            CHECK(oracle_alpha_box(nd, ids[k], 1, 0, prm[k], 1, z, dmin, dmax, al, aa) == 0);
            double H;
            CHECK(oracle_hamiltonian(nd, ids[k], 1, 0, prm[k], 1, z, p, &H) == 0);
        }
        if (ids[k] != 4 && nd <= 4) {
            long it;
            double ch;
            for (int jac = 0; jac <= 1; ++jac)
                CHECK(oracle_ttr_solve(nd, n, lo, hi, per, ids[k], 0, 1, prm[k], V0, 1e4, 1e-9, 5000, jac, V, &it,
                                       &ch) == 0);
        }
        free(V0);
        free(V);
        free(all);
        free(tg);
    }
    if (fails) {
        printf("%d checks failed\n", fails);
        return 1;
    }
    printf("ok\n");
    return 0;
}
