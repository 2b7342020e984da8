/* Sanitizer driver of the FP64 oracle (test infrastructure): every entry
 * point on small grids, every boundary kind, with and without the free
 * surface, windowed point steps and the acoustic_iso forward.  Built with
 * -fsanitize=address,undefined by tests/test_host_sanitize.py; any invalid
 * access, leak or undefined behaviour aborts the run. */
#include "../../oracle/minimod_oracle.c"

#include <stdio.h>

static int fails = 0;
#define CHECK(x)                                                    \
    do {                                                            \
        if (!(x)) {                                                 \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
            fails++;                                                \
        }                                                           \
    } while (0)

static double* vel_of(int n, double v0) {
    double* v = (double*)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) v[i] = v0 + 7.0 * (i % 13);
    return v;
}

int main(void) {
    const int nx = 19, ny = 17, nz = 15, T = 9;
    const int N = nx * ny * nz;
    double* vel = vel_of(N, 1800.0);
    int src[6] = {9, 8, 7, 3, 2, 1};
    int rec[9] = {1, 1, 1, 18, 16, 14, 5, 9, 0};
    double wav[2 * 9], res[3 * 9], adj[2 * 9], tr[3 * 9], grad[19 * 17 * 15];
    for (int i = 0; i < 18; ++i) wav[i] = sin(0.3 * i);
    for (int i = 0; i < 27; ++i) res[i] = cos(0.7 * i);
    for (int bc = 0; bc <= 3; ++bc)
        for (int fs = 0; fs <= 1; ++fs) {
            if (bc == 3 && fs) continue;
            orc_grid g = {nx, ny, nz, 10.0, 11.0, 9.0, 0.0, bc, bc == 0 || bc == 3 ? 0 : 4, 0.05, 1e-3, 20.0, 0.0,
                          0, 0, 0, 0, 0, 0, fs};
            g.vmax = 1800.0 + 7.0 * 12;
            g.dt = 0.5 * orc_dt_stab(g.vmax, g.hx, g.hy, g.hz);
            double* pm = (double*)calloc(N, sizeof(double));
            double* pc = (double*)calloc(N, sizeof(double));
            double* mem = (double*)calloc(6 * (size_t)N, sizeof(double));
            CHECK(orc_forward(&g, vel, 2, src, wav, 3, rec, T, tr, pm, pc, mem) == ORC_OK);
            CHECK(orc_energy(&g, vel, pm, pc) == orc_energy(&g, vel, pm, pc));
            if (bc != 3) {
                CHECK(orc_adjoint(&g, vel, 3, rec, res, T, 2, src, adj) == ORC_OK);
                CHECK(orc_gradient(&g, vel, 2, src, wav, 3, rec, tr, T, 4, grad, NULL, NULL) == ORC_OK);
            }
            /* point step inside a window of the grid */
            int pts[6] = {3, 4, 5, 10, 9, 8};
            double out[2];
            orc_grid w = g;
            w.wx0 = 2; w.wy0 = 3; w.wz0 = 4; w.wnx = 10; w.wny = 9; w.wnz = 8;
            const int WN = 10 * 9 * 8;
            double* wv = vel_of(WN, 1800.0);
            double* wa = (double*)calloc(WN, sizeof(double));
            double* wb = (double*)calloc(WN, sizeof(double));
            double* wm = (double*)calloc(6 * (size_t)WN, sizeof(double));
            (void)orc_step_points(&w, wv, wa, wb, bc == 2 ? wm : NULL, 2, pts, NULL, out);
            free(wv); free(wa); free(wb); free(wm);
            free(pm); free(pc); free(mem);
            /* argument errors */
            int badp[3] = {nx, 0, 0};
            CHECK(orc_forward(&g, vel, 1, badp, wav, 0, rec, 1, NULL, NULL, NULL, NULL) == ORC_ERR_ARG);
        }
    /* acoustic_iso: none and sponge, with and without the free surface */
    double* rho = vel_of(N, 1000.0);
    for (int bc = 0; bc <= 1; ++bc)
        for (int fs = 0; fs <= 1; ++fs) {
            orc_grid g = {nx, ny, nz, 10.0, 10.0, 10.0, 0.0, bc, bc ? 4 : 0, 0.05, 1e-3, 20.0, 0.0,
                          0, 0, 0, 0, 0, 0, fs};
            g.dt = 0.5 * orc_iso_dt_stab(1800.0 + 7.0 * 12, 10.0, 10.0, 10.0);
            double* st = (double*)calloc(4 * (size_t)N, sizeof(double));
            CHECK(orc_iso_forward(&g, vel, rho, 2, src, wav, 3, rec, T, tr, st) == ORC_OK);
            double e = orc_iso_energy(&g, vel, rho, st, st, st + N);
            CHECK(e == e);
            double* d = (double*)malloc(sizeof(double) * N);
            orc_iso_dplus(&g, st, 2, d);
            free(d);
            free(st);
        }
    double rk[16];
    orc_ricker(15.0, 0.1, 1e-3, 16, rk);
    free(rho);
    free(vel);
    if (fails) return 1;
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
