/*
 * Minimod acoustic_iso_cd oracle: a plain, slow, FP64 CPU implementation of
 * the time-stepping method, written from the paper (Meng, Atle, Calandra,
 * Araya-Polo, "Minimod: A Finite Difference solver for Seismic Modeling",
 * arXiv 2007.06048).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * GPU library.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it.  It shares no code, header, table or helper
 * with the HIP path; both sides receive the same seeded inputs and nothing
 * else.
 *
 * What is computed (section "Finite Differences", Eq. (acoustic_iso_cd) and
 * the semi-discretised Eq. (minimod-semidisc), 25-point stencil formula):
 *
 *   p^{n+1} - Q p^n + p^{n-1} = dt^2 v^2 f^n,   Q = 2 + dt^2 v^2 Lap,
 *   Lap p ~ sum_m c_xm [p(i+m)+p(i-m)-2p] + c_ym[...] + c_zm[...],  m=1..4,
 *
 * with the 8th-order Taylor coefficients c_m = a_m / h^2,
 * a = (8/5, -1/5, 8/315, -1/560) (the paper names the order but prints no
 * values; these are the unique order-8 central weights).  Algorithm 1
 * ("Minimod high-level description") fixes p^0 = 0 and the loop over time
 * steps; Algorithm 2 splits the domain into an inner region and damping
 * slabs at the six faces, which the section "Minimod Description" says use
 * a PML/CPML boundary.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *  - source:  f^n at the source cell is w(n dt)/(hx hy hz) and enters
 *             p^{n+1} through dt^2 v^2 (Eq. (minimod-semidisc) right side);
 *  - ghosts:  values outside the domain are zero (bc none, sponge, CPML);
 *             bc periodic wraps (a test mode);
 *  - sponge:  p^{n+1} = G (2 p^n - G p^{n-1} + D (Lap p^n + s^n)),
 *             G = gx gy gz,  g(k) = exp(-(sigma d_k)^2), d_k = nb - k cells
 *             inside the layer, 1 elsewhere;
 *  - CPML:    recursive-convolution CPML for the second-order equation with
 *             kappa = 1: per damped axis i, psi_i <- b psi_i + a D1_i p^n,
 *             zeta_i <- b zeta_i + a (D2_i p^n + D1_i psi_i), and the
 *             Laplacian gains D1_i psi_i + zeta_i inside the layer.
 *             d(q) = d0 q^2, d0 = -3 vmax ln R / (2 nb h), alpha = pi f0 (1-q),
 *             b = exp(-(d+alpha) dt), a = d (b-1)/(d+alpha),
 *             q = (nb-k)/nb in the layer, 0 inside;
 *  - dt:      dt = cfl * 2 / (vmax sqrt(S (hx^-2+hy^-2+hz^-2))),
 *             S = 4 (a1 + a3), the symbol maximum of the 1D operator;
 *  - wavelet: Ricker, w(t) = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
 *             tau = t - t0;
 *  - traces:  traces[n][r] = p^{n+1}(x_r), n = 0..T-1.
 *
 * Adjoint and gradient (the inverse problem the paper names as motivation
 * in "Seismic Modeling"): the exact discrete adjoint of the forward
 * recursion, written in the scaled variable eta = D G mu, which obeys the
 * forward recursion run backward in time:
 *   eta^m = G (2 eta^{m+1} - G eta^{m+2} + D (Lap eta^{m+1} + C + R^T r^m)),
 * where C = 0 except for CPML, whose memory recursions are transposed too
 * (adj_cpml below),
 * and the gradient with respect to squared slowness m = 1/v^2:
 *   dJ/dm = -(1/(dt^2 G)) sum_n eta^{n+1} (p^{n+1} - 2 G p^n + G^2 p^{n-1}).
 *
 * The CPML damping profile is pinned by PML reflection theory (the layer sum
 * of d h reproduces ln R up to its quadrature error) and alpha by the
 * standard CFS profile.  The sponge profile is read back from the forward
 * step itself (one step from a unit impulse with and without the sponge;
 * their ratio is G) and checked for the Cerjan form: exactly nb damped
 * cells per end, depth 1 at the innermost, G(d) = G(1)^(d^2) and
 * -ln G(1) = sigma^2.
 *
 * Layout of every 3D array: index (k*ny + j)*nx + i, x fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MEM 2
#define ORC_ERR_UNSUPPORTED 3

enum { BC_NONE = 0, BC_SPONGE = 1, BC_CPML = 2, BC_PERIODIC = 3 };

typedef struct {
    int nx, ny, nz;
    double hx, hy, hz;
    double dt;
    int bc;
    int nb;          /* damping width in cells (sponge and CPML) */
    double sigma;    /* sponge strength */
    double R;        /* CPML nominal reflection coefficient */
    double f0;       /* CPML alpha_max = pi * f0 */
    double vmax;     /* CPML d0 uses the model maximum velocity */
    /* Optional storage window (orc_step_points only): when wnx > 0 every
     * array holds just the box [wx0, wx0+wnx) x [wy0, wy0+wny) x
     * [wz0, wz0+wnz) of the grid, indexed like a full array of that box.
     * Indices stay global: the domain edges, layers and sources are those
     * of the nx x ny x nz grid. */
    int wx0, wy0, wz0, wnx, wny, wnz;
    /* Free surface on the top face (section "Minimod Description" names it
     * as the option at the surface): p = 0 on the plane k = 0 at every time
     * level, cells above it hold the odd mirror p(i,j,-k) = -p(i,j,k), and
     * the top face has no damping layer.  Not with bc periodic. */
    int fs;
} orc_grid;

static int g_window_miss;  /* set when a windowed access falls outside the window */

/* Order-8 central second-derivative weights a_m and first-derivative
 * weights beta_m, m = 1..4 (index 0 unused). */
static const double A2[5] = {0.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
static const double B1[5] = {0.0, 4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};

static size_t npts(const orc_grid* g) { return (size_t)g->nx * g->ny * g->nz; }

/* points stored per array: the window if there is one, else the grid */
static size_t nstore(const orc_grid* g) {
    return g->wnx > 0 ? (size_t)g->wnx * g->wny * g->wnz : npts(g);
}

static size_t lin(const orc_grid* g, int i, int j, int k) {
    if (g->wnx > 0) {
        i -= g->wx0;
        j -= g->wy0;
        k -= g->wz0;
        if (i < 0 || j < 0 || k < 0 || i >= g->wnx || j >= g->wny || k >= g->wnz) {
            g_window_miss = 1;
            return 0;
        }
        return ((size_t)k * g->wny + j) * g->wnx + i;
    }
    return ((size_t)k * g->ny + j) * g->nx + i;
}

static int wrap(int i, int n) {
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* Value of field f at (i,j,k); zero outside the domain unless periodic;
 * with a free surface, the odd mirror image above the plane k = 0. */
static double at(const orc_grid* g, const double* f, int i, int j, int k) {
    if (g->bc == BC_PERIODIC) {
        return f[lin(g, wrap(i, g->nx), wrap(j, g->ny), wrap(k, g->nz))];
    }
    if (g->fs && k < 0) return -at(g, f, i, j, -k);
    if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return 0.0;
    return f[lin(g, i, j, k)];
}

/* ---------------------------------------------------------------- scalars */

/* Largest stable dt of the leapfrog scheme with this stencil: the checkerboard
 * mode has symbol 4 (a1 + a3) per axis, and the recursion stays bounded while
 * dt^2 v^2 * sum_axes S/h^2 <= 4. */
double orc_dt_stab(double vmax, double hx, double hy, double hz) {
    double S = 4.0 * (A2[1] + A2[3]);
    double sum = 1.0 / (hx * hx) + 1.0 / (hy * hy) + 1.0 / (hz * hz);
    return 2.0 / (vmax * sqrt(S * sum));
}

void orc_ricker(double f0, double t0, double dt, int n, double* out) {
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < n; ++i) {
        double tau = i * dt - t0;
        double x = pi * pi * f0 * f0 * tau * tau;
        out[i] = (1.0 - 2.0 * x) * exp(-x);
    }
}

/* ------------------------------------------------------- stencil operators */

/* Discrete Laplacian in the paper's form:
 *   sum_m c_xm [p(i+m)+p(i-m)-2p] + c_ym [...] + c_zm [...]. */
static double lap_at(const orc_grid* g, const double* p, int i, int j, int k) {
    double c = at(g, p, i, j, k);
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int m = 1; m <= 4; ++m) {
        sx += (A2[m] / (g->hx * g->hx)) * (at(g, p, i + m, j, k) + at(g, p, i - m, j, k) - 2.0 * c);
        sy += (A2[m] / (g->hy * g->hy)) * (at(g, p, i, j + m, k) + at(g, p, i, j - m, k) - 2.0 * c);
        sz += (A2[m] / (g->hz * g->hz)) * (at(g, p, i, j, k + m) + at(g, p, i, j, k - m) - 2.0 * c);
    }
    return sx + sy + sz;
}

/* One axis of the Laplacian (D2 along axis ax = 0,1,2). */
static double d2_axis(const orc_grid* g, const double* p, int i, int j, int k, int ax) {
    int di = ax == 0, dj = ax == 1, dk = ax == 2;
    double h = ax == 0 ? g->hx : (ax == 1 ? g->hy : g->hz);
    double c = at(g, p, i, j, k);
    double s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += (A2[m] / (h * h)) *
             (at(g, p, i + m * di, j + m * dj, k + m * dk) + at(g, p, i - m * di, j - m * dj, k - m * dk) - 2.0 * c);
    return s;
}

/* Centred first derivative along axis ax. */
static double d1_axis(const orc_grid* g, const double* p, int i, int j, int k, int ax) {
    int di = ax == 0, dj = ax == 1, dk = ax == 2;
    double h = ax == 0 ? g->hx : (ax == 1 ? g->hy : g->hz);
    double s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += (B1[m] / h) * (at(g, p, i + m * di, j + m * dj, k + m * dk) - at(g, p, i - m * di, j - m * dj, k - m * dk));
    return s;
}

void orc_laplacian(const orc_grid* g, const double* p, double* out) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) out[lin(g, i, j, k)] = lap_at(g, p, i, j, k);
}

/* ---------------------------------------------------- boundary profiles */

/* Depth of index k inside the damping layer of an axis of n cells, counted
 * so that the outermost cell has depth nb and the first inner cell 0:
 * returns nb - k on the low side, nb - (n-1-k) on the high side, 0 inside. */
static int layer_depth(int k, int n, int nb) {
    int dl = nb - k;
    int dh = nb - (n - 1 - k);
    int d = dl > dh ? dl : dh;
    return d > 0 ? d : 0;
}

/* Depth inside the damping layer of axis ax (0 x, 1 y, 2 z) at index k;
 * a free surface removes the layer at the top (k < nb on the z axis). */
static int axis_depth(const orc_grid* g, int ax, int k) {
    int n = ax == 0 ? g->nx : (ax == 1 ? g->ny : g->nz);
    if (g->fs && ax == 2 && k < g->nb) return 0;
    return layer_depth(k, n, g->nb);
}

/* Sponge factor of axis ax at index k. */
static double sponge_g(const orc_grid* g, int ax, int k) {
    int d = axis_depth(g, ax, k);
    if (d == 0) return 1.0;
    double x = g->sigma * d;
    return exp(-x * x);
}

double orc_sponge_G(const orc_grid* g, int i, int j, int k) {
    if (g->bc != BC_SPONGE) return 1.0;
    return sponge_g(g, 0, i) * sponge_g(g, 1, j) * sponge_g(g, 2, k);
}

/* CPML coefficients (a, b) of axis ax at index k along that axis.  Returns 0
 * if k is outside the layer of that axis (then a = 0 and psi stays zero). */
static int cpml_ab(const orc_grid* g, int ax, int k, double* a, double* b) {
    double h = ax == 0 ? g->hx : (ax == 1 ? g->hy : g->hz);
    int d = axis_depth(g, ax, k);
    if (d == 0) {
        *a = 0.0;
        *b = 1.0;
        return 0;
    }
    const double pi = 3.14159265358979323846;
    double q = (double)d / g->nb;
    double d0 = -3.0 * g->vmax * log(g->R) / (2.0 * g->nb * h);
    double dq = d0 * q * q;
    double al = pi * g->f0 * (1.0 - q);
    double bb = exp(-(dq + al) * g->dt);
    *b = bb;
    *a = (dq + al) > 0.0 ? dq * (bb - 1.0) / (dq + al) : 0.0;
    return 1;
}

void orc_cpml_coeffs(const orc_grid* g, int ax, int k, double* a, double* b) { cpml_ab(g, ax, k, a, b); }

/* CPML memory: 6 full-grid arrays, psi_x psi_y psi_z zeta_x zeta_y zeta_z. */
static void cpml_update(const orc_grid* g, const double* p, double* mem, double* Lp, double* scratch) {
    size_t N = npts(g);
    for (int ax = 0; ax < 3; ++ax) {
        double* psi = mem + (size_t)ax * N;
        double* zeta = mem + (size_t)(3 + ax) * N;
        /* psi_i <- b psi_i + a D1_i p^n, inside the layer of axis i */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    int kk = ax == 0 ? i : (ax == 1 ? j : k);
                    double a, b;
                    size_t id = lin(g, i, j, k);
                    if (cpml_ab(g, ax, kk, &a, &b))
                        scratch[id] = b * psi[id] + a * d1_axis(g, p, i, j, k, ax);
                    else
                        scratch[id] = 0.0;
                }
        memcpy(psi, scratch, N * sizeof(double));
        /* zeta_i <- b zeta_i + a (D2_i p^n + D1_i psi_i); Lap += D1_i psi_i + zeta_i */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    int kk = ax == 0 ? i : (ax == 1 ? j : k);
                    double a, b;
                    size_t id = lin(g, i, j, k);
                    if (!cpml_ab(g, ax, kk, &a, &b)) continue;
                    double dpsi = d1_axis(g, psi, i, j, k, ax);
                    zeta[id] = b * zeta[id] + a * (d2_axis(g, p, i, j, k, ax) + dpsi);
                    Lp[id] += dpsi + zeta[id];
                }
    }
}

/* ------------------------------------------------------------- forward */

static int check_grid(const orc_grid* g) {
    if (!g || g->nx < 1 || g->ny < 1 || g->nz < 1) return ORC_ERR_ARG;
    if (g->wnx < 0 || g->wny < 0 || g->wnz < 0) return ORC_ERR_ARG;
    if (g->hx <= 0 || g->hy <= 0 || g->hz <= 0 || g->dt <= 0) return ORC_ERR_ARG;
    if (g->bc < 0 || g->bc > 3) return ORC_ERR_ARG;
    if ((g->bc == BC_SPONGE || g->bc == BC_CPML) && g->nb < 1) return ORC_ERR_ARG;
    if (g->fs && g->bc == BC_PERIODIC) return ORC_ERR_ARG;
    return ORC_OK;
}

static int check_pts(const orc_grid* g, int n, const int* ijk) {
    for (int s = 0; s < n; ++s) {
        int i = ijk[3 * s], j = ijk[3 * s + 1], k = ijk[3 * s + 2];
        if (i < 0 || j < 0 || k < 0 || i >= g->nx || j >= g->ny || k >= g->nz) return ORC_ERR_ARG;
    }
    return ORC_OK;
}

/* One leapfrog step.  Reads p_prev = p^{n-1}, p_cur = p^n, writes p_next.
 * src_term holds s^n on the grid (zero except at sources).  If Lp_out is
 * given it receives the (CPML-corrected) Laplacian. */
static void step(const orc_grid* g, const double* D, const double* p_prev, const double* p_cur,
                 const double* src_term, double* mem, double* Lp, double* scratch, double* p_next) {
    orc_laplacian(g, p_cur, Lp);
    if (g->bc == BC_CPML) cpml_update(g, p_cur, mem, Lp, scratch);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = lin(g, i, j, k);
                double G = orc_sponge_G(g, i, j, k);
                double s = src_term ? src_term[id] : 0.0;
                p_next[id] = G * (2.0 * p_cur[id] - G * p_prev[id] + D[id] * (Lp[id] + s));
                if (g->fs && k == 0) p_next[id] = 0.0;
            }
}

static double* alloc_d(size_t n) { return (double*)calloc(n ? n : 1, sizeof(double)); }

static void fill_D(const orc_grid* g, const double* vel, double* D) {
    size_t N = npts(g);
    for (size_t id = 0; id < N; ++id) {
        double v = vel[id];
        D[id] = g->dt * g->dt * v * v;
    }
}

/* Forward modeling for T steps from the state (p_prev, p_cur) = (p^{-1}, p^0)
 * given on entry (zero for Algorithm 1); on return they hold (p^{T-1}, p^T).
 * wav is [T][nsrc] raw wavelet samples w(t_n); traces [T][nrec] receives
 * p^{n+1} at the receivers (may be NULL).  cpml_mem, if not NULL, is the
 * 6*N CPML memory in/out (psi_x,y,z then zeta_x,y,z); otherwise it starts
 * at zero. */
int orc_forward(const orc_grid* g, const double* vel, int nsrc, const int* src, const double* wav, int nrec,
                const int* rec, int T, double* traces, double* p_prev, double* p_cur, double* cpml_mem) {
    if (g && g->wnx > 0) return ORC_ERR_ARG;
    if (check_grid(g) || T < 0 || nsrc < 0 || nrec < 0) return ORC_ERR_ARG;
    if (check_pts(g, nsrc, src) || check_pts(g, nrec, rec)) return ORC_ERR_ARG;
    size_t N = npts(g);
    double* D = alloc_d(N);
    double* Lp = alloc_d(N);
    double* scratch = alloc_d(N);
    double* nxt = alloc_d(N);
    double* S = alloc_d(N);
    double* mem = NULL;
    int own_mem = 0;
    if (g->bc == BC_CPML) {
        if (cpml_mem) mem = cpml_mem;
        else {
            mem = alloc_d(6 * N);
            own_mem = 1;
        }
    }
    if (!D || !Lp || !scratch || !nxt || !S || (g->bc == BC_CPML && !mem)) {
        free(D); free(Lp); free(scratch); free(nxt); free(S);
        if (own_mem) free(mem);
        return ORC_ERR_MEM;
    }
    fill_D(g, vel, D);
    double inv_vol = 1.0 / (g->hx * g->hy * g->hz);
    for (int n = 0; n < T; ++n) {
        memset(S, 0, N * sizeof(double));
        for (int s = 0; s < nsrc; ++s)
            S[lin(g, src[3 * s], src[3 * s + 1], src[3 * s + 2])] += wav[(size_t)n * nsrc + s] * inv_vol;
        step(g, D, p_prev, p_cur, S, mem, Lp, scratch, nxt);
        if (traces)
            for (int r = 0; r < nrec; ++r)
                traces[(size_t)n * nrec + r] = nxt[lin(g, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])];
        memcpy(p_prev, p_cur, N * sizeof(double));
        memcpy(p_cur, nxt, N * sizeof(double));
    }
    free(D); free(Lp); free(scratch); free(nxt); free(S);
    if (own_mem) free(mem);
    return ORC_OK;
}

/* p^{n+1} at a list of points from a given state: the same step as
 * orc_forward, evaluated point by point (for sampled checks on grids too
 * large to step whole; with a storage window the arrays cover only a box
 * around the points, at least 8 cells wide on every side for CPML).  cpml_mem (6*N, may be NULL when bc != CPML) holds
 * psi and zeta of step n-1 and is not modified.  src_term_at[q] is s^n at
 * point q (the caller adds w/(hx hy hz) where a source sits). */
int orc_step_points(const orc_grid* g, const double* vel, const double* p_prev, const double* p_cur,
                    const double* cpml_mem, int npt, const int* ijk, const double* src_term_at, double* out) {
    if (check_grid(g) || check_pts(g, npt, ijk)) return ORC_ERR_ARG;
    if (g->bc == BC_CPML && !cpml_mem) return ORC_ERR_ARG;
    size_t N = nstore(g);
    g_window_miss = 0;
    for (int q = 0; q < npt; ++q) {
        int i = ijk[3 * q], j = ijk[3 * q + 1], k = ijk[3 * q + 2];
        size_t id = lin(g, i, j, k);
        double L = lap_at(g, p_cur, i, j, k);
        if (g->bc == BC_CPML) {
            for (int ax = 0; ax < 3; ++ax) {
                int pos[3] = {i, j, k};
                int n_ax = ax == 0 ? g->nx : (ax == 1 ? g->ny : g->nz);
                double a, b;
                if (!cpml_ab(g, ax, pos[ax], &a, &b)) continue;
                const double* psi = cpml_mem + (size_t)ax * N;
                const double* zeta = cpml_mem + (size_t)(3 + ax) * N;
                /* new psi along the axis at offsets -4..4 */
                double pn[9];
                for (int m = -4; m <= 4; ++m) {
                    int p2[3] = {i, j, k};
                    p2[ax] += m;
                    double aa, bb;
                    if (p2[ax] < 0 || p2[ax] >= n_ax || !cpml_ab(g, ax, p2[ax], &aa, &bb)) {
                        pn[m + 4] = 0.0;
                        continue;
                    }
                    size_t id2 = lin(g, p2[0], p2[1], p2[2]);
                    pn[m + 4] = bb * psi[id2] + aa * d1_axis(g, p_cur, p2[0], p2[1], p2[2], ax);
                }
                double h = ax == 0 ? g->hx : (ax == 1 ? g->hy : g->hz);
                double dpsi = 0.0;
                for (int m = 1; m <= 4; ++m) dpsi += (B1[m] / h) * (pn[4 + m] - pn[4 - m]);
                double zn = b * zeta[id] + a * (d2_axis(g, p_cur, i, j, k, ax) + dpsi);
                L += dpsi + zn;
            }
        }
        double G = orc_sponge_G(g, i, j, k);
        double v = vel[id];
        double D = g->dt * g->dt * v * v;
        double s = src_term_at ? src_term_at[q] : 0.0;
        out[q] = (g->fs && k == 0) ? 0.0 : G * (2.0 * p_cur[id] - G * p_prev[id] + D * (L + s));
    }
    return g_window_miss ? ORC_ERR_ARG : ORC_OK;
}

/* Discrete energy between consecutive states p^n and p^{n+1}:
 *   E^{n+1/2} = sum (p^{n+1}-p^n)^2 / (v^2 dt^2) - sum p^{n+1} Lap p^n. */
double orc_energy(const orc_grid* g, const double* vel, const double* pn, const double* pn1) {
    size_t N = npts(g);
    double* Lp = alloc_d(N);
    if (!Lp) return NAN;
    orc_laplacian(g, pn, Lp);
    double kin = 0.0, pot = 0.0;
    for (size_t id = 0; id < N; ++id) {
        double v = vel[id];
        double d = pn1[id] - pn[id];
        kin += d * d / (v * v * g->dt * g->dt);
        pot += pn1[id] * Lp[id];
    }
    free(Lp);
    return kin - pot;
}

/* ------------------------------------------------------------- adjoint */

/* Adjoint of the CPML recursions, for one backward step.  The forward step n
 * is, per damped axis i with layer mask M_i (all operators with zero ghosts):
 *   psi^{n+1}  = M (b psi^n + a D1 p^n),
 *   zeta^{n+1} = M (b zeta^n + a (D2 p^n + D1 psi^{n+1})),
 *   p^{n+1}    = 2 p^n - p^{n-1} + D (Lap p^n + M (D1 psi^{n+1} + zeta^{n+1}) + s^n).
 * With mu the adjoint of p, eta = D mu, and Zb, Pb the adjoints of zeta and
 * psi, transposing each line (D1^T = -D1, D2^T = D2 on the zero-ghost grid):
 *   Zb^{m+1} = M (eta^{m+1} + b Zb^{m+2}),
 *   Pb^{m+1} = M (-D1 (M eta^{m+1} + a Zb^{m+1}) + b Pb^{m+2}),
 * and the adjoint of p^m gains  C = sum_i (-D1 (a Pb^{m+1}) + D2 (a Zb^{m+1})),
 * which reaches 4 cells past the layer.  amem holds Pb_x,y,z then Zb_x,y,z
 * (6 full-grid arrays): on entry the values of level m+2, on return m+1.
 * C (full grid) is overwritten. */
static void adj_cpml(const orc_grid* g, const double* e1, double* amem, double* C, double* u, double* az,
                     double* ap) {
    size_t N = npts(g);
    memset(C, 0, N * sizeof(double));
    for (int ax = 0; ax < 3; ++ax) {
        double* Pb = amem + (size_t)ax * N;
        double* Zb = amem + (size_t)(3 + ax) * N;
        /* Zb <- M (eta + b Zb);  u = M eta + a Zb;  az = a Zb */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    int kk = ax == 0 ? i : (ax == 1 ? j : k);
                    double a, b;
                    size_t id = lin(g, i, j, k);
                    if (cpml_ab(g, ax, kk, &a, &b)) {
                        Zb[id] = e1[id] + b * Zb[id];
                        u[id] = e1[id] + a * Zb[id];
                        az[id] = a * Zb[id];
                    } else {
                        Zb[id] = 0.0;
                        u[id] = 0.0;
                        az[id] = 0.0;
                    }
                }
        /* Pb <- M (-D1 u + b Pb);  ap = a Pb */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    int kk = ax == 0 ? i : (ax == 1 ? j : k);
                    double a, b;
                    size_t id = lin(g, i, j, k);
                    if (cpml_ab(g, ax, kk, &a, &b)) {
                        Pb[id] = -d1_axis(g, u, i, j, k, ax) + b * Pb[id];
                        ap[id] = a * Pb[id];
                    } else {
                        Pb[id] = 0.0;
                        ap[id] = 0.0;
                    }
                }
        /* C += -D1 (a Pb) + D2 (a Zb), on every cell */
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t id = lin(g, i, j, k);
                    C[id] += -d1_axis(g, ap, i, j, k, ax) + d2_axis(g, az, i, j, k, ax);
                }
    }
}

/* Work arrays of the CPML adjoint: memory (6N) and C, u, az, ap (N each). */
typedef struct {
    double* amem;
    double *C, *u, *az, *ap;
} adj_work;

static int adj_work_alloc(const orc_grid* g, adj_work* w) {
    memset(w, 0, sizeof(*w));
    if (g->bc != BC_CPML) return ORC_OK;
    size_t N = npts(g);
    w->amem = alloc_d(6 * N);
    w->C = alloc_d(N);
    w->u = alloc_d(N);
    w->az = alloc_d(N);
    w->ap = alloc_d(N);
    return (w->amem && w->C && w->u && w->az && w->ap) ? ORC_OK : ORC_ERR_MEM;
}

static void adj_work_free(adj_work* w) {
    free(w->amem); free(w->C); free(w->u); free(w->az); free(w->ap);
}

/* One backward step of the scaled adjoint: eta^m from eta^{m+1}, eta^{m+2},
 * the receiver residual r^m and (CPML) the adjoint memory.  Without CPML it
 * is the forward step with the residual as a source of unit scale at the
 * receivers. */
static void adj_step(const orc_grid* g, const double* D, const double* e2, const double* e1, const double* rt,
                     double* Lp, adj_work* w, double* out) {
    orc_laplacian(g, e1, Lp);
    if (g->bc == BC_CPML) adj_cpml(g, e1, w->amem, w->C, w->u, w->az, w->ap);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = lin(g, i, j, k);
                double G = orc_sponge_G(g, i, j, k);
                double c = g->bc == BC_CPML ? w->C[id] : 0.0;
                out[id] = G * (2.0 * e1[id] - G * e2[id] + D[id] * (Lp[id] + c + rt[id]));
                if (g->fs && k == 0) out[id] = 0.0;
            }
}

/* Adjoint run for T steps with residual resid [T][nrec] (resid[n] pairs with
 * the trace of p^{n+1}).  adj_src [T][nsrc] receives eta^{n+1} at the source
 * points.  With zero initial adjoint state this is the transpose of the map
 * (sources s^n) -> (traces), in the sense
 *   sum_n <R p^{n+1}, r^n> = sum_n <s^n, eta^{n+1}(src)>. */
int orc_adjoint(const orc_grid* g, const double* vel, int nrec, const int* rec, const double* resid, int T, int nsrc,
                const int* src, double* adj_src) {
    if (g && g->wnx > 0) return ORC_ERR_ARG;
    if (check_grid(g) || T < 0) return ORC_ERR_ARG;
    if (check_pts(g, nsrc, src) || check_pts(g, nrec, rec)) return ORC_ERR_ARG;
    size_t N = npts(g);
    double *D = alloc_d(N), *Lp = alloc_d(N), *e2 = alloc_d(N), *e1 = alloc_d(N), *en = alloc_d(N),
           *rt = alloc_d(N);
    adj_work w;
    int rc = adj_work_alloc(g, &w);
    if (!D || !Lp || !e2 || !e1 || !en || !rt || rc) {
        free(D); free(Lp); free(e2); free(e1); free(en); free(rt);
        adj_work_free(&w);
        return ORC_ERR_MEM;
    }
    fill_D(g, vel, D);
    for (int m = T; m >= 1; --m) {
        memset(rt, 0, N * sizeof(double));
        for (int r = 0; r < nrec; ++r)
            rt[lin(g, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])] += resid[(size_t)(m - 1) * nrec + r];
        adj_step(g, D, e2, e1, rt, Lp, &w, en);
        if (adj_src)
            for (int s = 0; s < nsrc; ++s)
                adj_src[(size_t)(m - 1) * nsrc + s] = en[lin(g, src[3 * s], src[3 * s + 1], src[3 * s + 2])];
        memcpy(e2, e1, N * sizeof(double));
        memcpy(e1, en, N * sizeof(double));
    }
    free(D); free(Lp); free(e2); free(e1); free(en); free(rt);
    adj_work_free(&w);
    return ORC_OK;
}

/* FWI gradient of J = 1/2 sum_n sum_r (d^n_r - dobs^n_r)^2 with respect to
 * m = 1/v^2, for a forward run from zero state.  The forward wavefields are
 * regenerated segment by segment from FP64 checkpoints taken every ckpt
 * steps (ckpt >= T keeps one segment); a checkpoint holds (p^{cK-1}, p^{cK})
 * and, for CPML, the six memory arrays.  FP64 replay is exact, so ckpt does
 * not change the result.  traces [T][nrec] and loss may be NULL. */
int orc_gradient(const orc_grid* g, const double* vel, int nsrc, const int* src, const double* wav, int nrec,
                 const int* rec, const double* d_obs, int T, int ckpt, double* grad, double* traces, double* loss) {
    if (g && g->wnx > 0) return ORC_ERR_ARG;
    if (check_grid(g) || T < 1 || ckpt < 1) return ORC_ERR_ARG;
    if (check_pts(g, nsrc, src) || check_pts(g, nrec, rec)) return ORC_ERR_ARG;
    size_t N = npts(g);
    const int cpml = g->bc == BC_CPML;
    size_t M6 = cpml ? 6 * N : 0;  /* CPML memory per state */
    size_t CK = 2 * N + M6;         /* one checkpoint */
    int nseg = (T + ckpt - 1) / ckpt;
    double* D = alloc_d(N);
    double* Lp = alloc_d(N);
    double* S = alloc_d(N);
    double* a = alloc_d(N);
    double* b = alloc_d(N);
    double* c = alloc_d(N);
    double* mem = alloc_d(M6);
    double* scratch = alloc_d(N);
    double* ck = alloc_d((size_t)nseg * CK);
    double* tr = alloc_d((size_t)T * nrec);
    double* res = alloc_d((size_t)T * nrec);
    double* seg = alloc_d((size_t)(ckpt + 2) * N);
    double *e2 = alloc_d(N), *e1 = alloc_d(N), *en = alloc_d(N), *rt = alloc_d(N);
    adj_work w;
    int rc = adj_work_alloc(g, &w);
    if (!D || !Lp || !S || !a || !b || !c || !mem || !scratch || !ck || !tr || !res || !seg || !e2 || !e1 || !en ||
        !rt || rc) {
        rc = ORC_ERR_MEM;
        goto done;
    }
    fill_D(g, vel, D);
    double inv_vol = 1.0 / (g->hx * g->hy * g->hz);
    /* forward: a = p^{n-1}, b = p^n, checkpoint (p^{cK-1}, p^{cK}, memory) */
    for (int n = 0; n < T; ++n) {
        if (n % ckpt == 0) {
            double* cp = ck + (size_t)(n / ckpt) * CK;
            memcpy(cp, a, N * sizeof(double));
            memcpy(cp + N, b, N * sizeof(double));
            if (cpml) memcpy(cp + 2 * N, mem, M6 * sizeof(double));
        }
        memset(S, 0, N * sizeof(double));
        for (int s = 0; s < nsrc; ++s)
            S[lin(g, src[3 * s], src[3 * s + 1], src[3 * s + 2])] += wav[(size_t)n * nsrc + s] * inv_vol;
        step(g, D, a, b, S, cpml ? mem : NULL, Lp, scratch, c);
        for (int r = 0; r < nrec; ++r) tr[(size_t)n * nrec + r] = c[lin(g, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])];
        double* t = a; a = b; b = c; c = t;
    }
    double J = 0.0;
    for (size_t q = 0; q < (size_t)T * nrec; ++q) {
        res[q] = tr[q] - d_obs[q];
        J += 0.5 * res[q] * res[q];
    }
    if (traces) memcpy(traces, tr, (size_t)T * nrec * sizeof(double));
    if (loss) *loss = J;
    memset(grad, 0, N * sizeof(double));
    /* backward over segments, last first */
    for (int cseg = nseg - 1; cseg >= 0; --cseg) {
        int n0 = cseg * ckpt;
        int n1 = n0 + ckpt < T ? n0 + ckpt : T;
        /* seg[t - n0 + 1] = p^t for t = n0-1 .. n1 */
        const double* cp = ck + (size_t)cseg * CK;
        memcpy(seg, cp, 2 * N * sizeof(double));
        if (cpml) memcpy(mem, cp + 2 * N, M6 * sizeof(double));
        for (int n = n0; n < n1; ++n) {
            memset(S, 0, N * sizeof(double));
            for (int s = 0; s < nsrc; ++s)
                S[lin(g, src[3 * s], src[3 * s + 1], src[3 * s + 2])] += wav[(size_t)n * nsrc + s] * inv_vol;
            step(g, D, seg + (size_t)(n - n0) * N, seg + (size_t)(n - n0 + 1) * N, S, cpml ? mem : NULL, Lp, scratch,
                 seg + (size_t)(n - n0 + 2) * N);
        }
        for (int m = n1; m >= n0 + 1; --m) {
            memset(rt, 0, N * sizeof(double));
            for (int r = 0; r < nrec; ++r)
                rt[lin(g, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])] += res[(size_t)(m - 1) * nrec + r];
            adj_step(g, D, e2, e1, rt, Lp, &w, en);
            const double* pm = seg + (size_t)(m - n0 + 1) * N;
            const double* pm1 = seg + (size_t)(m - n0) * N;
            const double* pm2 = seg + (size_t)(m - n0 - 1) * N;
#pragma omp parallel for schedule(static)
            for (int k = 0; k < g->nz; ++k)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i) {
                        size_t id = lin(g, i, j, k);
                        double G = orc_sponge_G(g, i, j, k);
                        double d2p = pm[id] - 2.0 * G * pm1[id] + G * G * pm2[id];
                        grad[id] -= en[id] * d2p / (g->dt * g->dt * G);
                    }
            double* t = e2; e2 = e1; e1 = en; en = t;
        }
    }
done:
    free(D); free(Lp); free(S); free(a); free(b); free(c); free(mem); free(scratch); free(ck); free(tr); free(res);
    free(seg); free(e2); free(e1); free(en); free(rt);
    adj_work_free(&w);
    return rc;
}

/* Number of threads the OpenMP runtime will use (for reporting). */
int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following parallel loops (timing at a chosen core count). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ========================================================= acoustic_iso */
/*
 * The paper's second propagator, Eq. (acoustic_iso_vd): the first-order
 * variable-density system
 *   (1/(rho v^2)) dp/dt - div u = f,   rho du/dt - grad p = 0,
 * on a staggered (Yee) grid, section "Finite Differences": p at the cell
 * centres, u_x at the faces (i+1/2, j, k), u_y at (i, j+1/2, k), u_z at
 * (i, j, k+1/2); array index (i,j,k) of u_x holds the face i+1/2.  Readings:
 *  - staggered order-8 first differences, weights c = (1225/1024,
 *    -245/3072, 49/5120, -5/7168):
 *      D+ p (face i+1/2) = sum_m c_m (p(i+m) - p(i+1-m)) / h,
 *      D- u (cell i)     = sum_m c_m (u(i+m-1) - u(i-m)) / h,
 *    zero outside the grid (or periodic), so D- = -(D+)^T;
 *  - leapfrog staggered in time, u at half steps:
 *      u^{n+1/2} = G (u^{n-1/2} + dt b D+ p^n),
 *      p^{n+1}   = G (p^n + dt K (D- . u^{n+1/2} + s^n)),
 *    K = rho v^2, b = the face buoyancy: 1 over the mean density of the two
 *    cells beside the face, 2 / (rho_0 + rho_1) (1/rho of the inner cell on
 *    the last face of an axis).  Averaging rho, not 1/rho, is what makes a
 *    long wave crossing layers one cell thick travel at the homogenised
 *    speed 1/sqrt(<rho> <1/K>) of the continuous system;
 *    s^n = w(t_n)/(hx hy hz) at the source cell; G = the sponge factor of
 *    the cell (for u, the cell whose right face it is);
 *  - dt = cfl / (C vmax sqrt(hx^-2 + hy^-2 + hz^-2)), C = c1 - c2 + c3 - c4,
 *    the largest symbol of the staggered derivative (checkerboard mode);
 *  - traces[n][r] = p^{n+1} at the receivers; initial state zero;
 *  - free surface (as for acoustic_iso_cd): p = 0 on the plane k = 0, p odd
 *    about it above (so the p-derivative faces see -p(-k)), u_z even about
 *    it, no damping layer on the top face; sources and receivers on the
 *    plane inject and record nothing;
 *  - CPML (section "Finite Differences": every propagator has CPML
 *    boundaries): the first-order convolutional PML with kappa = 1.  Inside
 *    the layers each first derivative gains a memory variable updated by
 *    the recursive convolution psi <- b psi + a (that derivative):
 *      u_a^{n+1/2} = u_a^{n-1/2} + dt b (D+_a p^n + psi_pa),
 *        psi_pa <- bf psi_pa + af D+_a p^n          (at the faces),
 *      p^{n+1} = p^n + dt K (sum_a (D-_a u_a^{n+1/2} + psi_ua) + s^n),
 *        psi_ua <- bc psi_ua + ac D-_a u_a^{n+1/2}  (at the cells),
 *    with d, alpha, b = exp(-(d + alpha) dt), a = d (b - 1)/(d + alpha) as
 *    for acoustic_iso_cd, evaluated at the position of the quantity: a cell
 *    at depth nb - k inside the low layer (k - (n - 1 - nb) inside the high
 *    one), a face i + 1/2 at depth nb - i - 1/2 (i + 1/2 - (n - 1 - nb)),
 *    q = depth / nb clamped to 1 (the face beyond the last cell).
 */
static const double C8[5] = {0.0, 1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0};

double orc_iso_dt_stab(double vmax, double hx, double hy, double hz) {
    double C = C8[1] - C8[2] + C8[3] - C8[4];
    double sum = 1.0 / (hx * hx) + 1.0 / (hy * hy) + 1.0 / (hz * hz);
    return 1.0 / (C * vmax * sqrt(sum));
}

static double axis_h(const orc_grid* g, int ax) { return ax == 0 ? g->hx : (ax == 1 ? g->hy : g->hz); }

/* D+ of cell field p along axis ax, at the face (i,j,k) + 1/2 e_ax. */
static double dplus(const orc_grid* g, const double* p, int i, int j, int k, int ax) {
    int di = ax == 0, dj = ax == 1, dk = ax == 2;
    double h = axis_h(g, ax), s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += (C8[m] / h) * (at(g, p, i + m * di, j + m * dj, k + m * dk) -
                            at(g, p, i - (m - 1) * di, j - (m - 1) * dj, k - (m - 1) * dk));
    return s;
}

/* u_z above a free surface: p is odd about the surface plane k = 0, so its
 * z derivative, and u_z, are even about it: the face -1/2 - m holds u_z of
 * the face m + 1/2 (index -1 - m mirrors index m). */
static double at_uz(const orc_grid* g, const double* u, int i, int j, int k) {
    if (g->fs && k < 0) return at(g, u, i, j, -1 - k);
    return at(g, u, i, j, k);
}

/* D- of face field u (index i holds face i+1/2) along axis ax, at cell (i,j,k). */
static double dminus(const orc_grid* g, const double* u, int i, int j, int k, int ax) {
    int di = ax == 0, dj = ax == 1, dk = ax == 2;
    double h = axis_h(g, ax), s = 0.0;
    for (int m = 1; m <= 4; ++m)
        s += (C8[m] / h) * (at_uz(g, u, i + (m - 1) * di, j + (m - 1) * dj, k + (m - 1) * dk) -
                            at_uz(g, u, i - m * di, j - m * dj, k - m * dk));
    return s;
}

/* Buoyancy at the face (i,j,k) + 1/2 e_ax: 1 / (arithmetic mean of rho of
 * the two cells beside it). */
static double face_b(const orc_grid* g, const double* rho, int i, int j, int k, int ax) {
    int n = ax == 0 ? g->nx : (ax == 1 ? g->ny : g->nz);
    int pos = ax == 0 ? i : (ax == 1 ? j : k);
    double b0 = 1.0 / rho[lin(g, i, j, k)];
    int q = pos + 1;
    if (q >= n) {
        if (g->bc != BC_PERIODIC) return b0;
        q = 0;
    }
    int i1 = ax == 0 ? q : i, j1 = ax == 1 ? q : j, k1 = ax == 2 ? q : k;
    return 2.0 / (rho[lin(g, i, j, k)] + rho[lin(g, i1, j1, k1)]);
}

/* D+ along axis ax of a whole cell field (test access to the operator). */
void orc_iso_dplus(const orc_grid* g, const double* p, int ax, double* out) {
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) out[lin(g, i, j, k)] = dplus(g, p, i, j, k, ax);
}

static int iso_check(const orc_grid* g) {
    if (check_grid(g) || g->wnx > 0) return ORC_ERR_ARG;
    if (g->fs && g->bc == BC_PERIODIC) return ORC_ERR_UNSUPPORTED;
    return ORC_OK;
}

/* CPML coefficients at a position of the given depth (in cells) inside the
 * layer of axis ax; depth 0: outside (a = 0, b = 1). */
static int cpml_ab_depth(const orc_grid* g, int ax, double depth, double* a, double* b) {
    if (depth <= 0.0) {
        *a = 0.0;
        *b = 1.0;
        return 0;
    }
    const double pi = 3.14159265358979323846;
    double h = axis_h(g, ax);
    double q = depth / g->nb;
    if (q > 1.0) q = 1.0;
    double d0 = -3.0 * g->vmax * log(g->R) / (2.0 * g->nb * h);
    double dq = d0 * q * q;
    double al = pi * g->f0 * (1.0 - q);
    double bb = exp(-(dq + al) * g->dt);
    *b = bb;
    *a = (dq + al) > 0.0 ? dq * (bb - 1.0) / (dq + al) : 0.0;
    return 1;
}

/* Depth of the face i + 1/2 of axis ax inside its damping layers (0 outside);
 * no layer on the top face under a free surface. */
static double face_depth(const orc_grid* g, int ax, int i) {
    int n = ax == 0 ? g->nx : (ax == 1 ? g->ny : g->nz);
    double lo = g->nb - i - 0.5;
    if (g->fs && ax == 2) lo = 0.0;
    double hi = i + 0.5 - (n - 1 - g->nb);
    double d = lo > hi ? lo : hi;
    return d > 0.0 ? d : 0.0;
}

/* acoustic_iso CPML coefficients of axis ax at index k: cell (face = 0) or
 * face k + 1/2 (face = 1) (test access to the profiles). */
void orc_iso_cpml_coeffs(const orc_grid* g, int ax, int k, int face, double* a, double* b) {
    double depth = face ? face_depth(g, ax, k) : (double)axis_depth(g, ax, k);
    cpml_ab_depth(g, ax, depth, a, b);
}

/* acoustic_iso forward run for T steps.  state (p^n, u_x, u_y, u_z at
 * n-1/2, then with CPML psi_px, psi_py, psi_pz at the faces and psi_ux,
 * psi_uy, psi_uz at the cells: 4N, or 10N with CPML) is the start state and
 * receives the end state; NULL starts from zero.  wav [T][nsrc], traces
 * [T][nrec] (may be NULL). */
int orc_iso_forward(const orc_grid* g, const double* vel, const double* rho, int nsrc, const int* src,
                    const double* wav, int nrec, const int* rec, int T, double* traces, double* state) {
    int rc = iso_check(g);
    if (rc) return rc;
    if (T < 0 || nsrc < 0 || nrec < 0 || check_pts(g, nsrc, src) || check_pts(g, nrec, rec)) return ORC_ERR_ARG;
    size_t N = npts(g);
    const int cpml = g->bc == BC_CPML;
    double* st = state ? state : alloc_d((cpml ? 10 : 4) * N);
    double* pn = alloc_d(N);
    double* S = alloc_d(N);
    if (!st || !pn || !S) {
        if (!state) free(st);
        free(pn); free(S);
        return ORC_ERR_MEM;
    }
    double* p = st;
    double* u[3] = {st + N, st + 2 * N, st + 3 * N};
    double* psi_p[3] = {st + 4 * N, st + 5 * N, st + 6 * N};  /* CPML only */
    double* psi_u[3] = {st + 7 * N, st + 8 * N, st + 9 * N};
    double inv_vol = 1.0 / (g->hx * g->hy * g->hz);
    for (int n = 0; n < T; ++n) {
        /* u^{n+1/2} from p^n */
        for (int ax = 0; ax < 3; ++ax) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < g->nz; ++k)
                for (int j = 0; j < g->ny; ++j)
                    for (int i = 0; i < g->nx; ++i) {
                        size_t id = lin(g, i, j, k);
                        double G = orc_sponge_G(g, i, j, k);
                        double dp = dplus(g, p, i, j, k, ax);
                        if (cpml) {
                            double a, b;
                            int pos = ax == 0 ? i : (ax == 1 ? j : k);
                            if (cpml_ab_depth(g, ax, face_depth(g, ax, pos), &a, &b)) {
                                psi_p[ax][id] = b * psi_p[ax][id] + a * dp;
                                dp += psi_p[ax][id];
                            }
                        }
                        u[ax][id] = G * (u[ax][id] + g->dt * face_b(g, rho, i, j, k, ax) * dp);
                    }
        }
        /* p^{n+1} from p^n, u^{n+1/2} and s^n */
        memset(S, 0, N * sizeof(double));
        for (int s = 0; s < nsrc; ++s)
            S[lin(g, src[3 * s], src[3 * s + 1], src[3 * s + 2])] += wav[(size_t)n * nsrc + s] * inv_vol;
#pragma omp parallel for schedule(static)
        for (int k = 0; k < g->nz; ++k)
            for (int j = 0; j < g->ny; ++j)
                for (int i = 0; i < g->nx; ++i) {
                    size_t id = lin(g, i, j, k);
                    double G = orc_sponge_G(g, i, j, k);
                    double K = rho[id] * vel[id] * vel[id];
                    double du[3];
                    for (int ax = 0; ax < 3; ++ax) {
                        du[ax] = dminus(g, u[ax], i, j, k, ax);
                        if (cpml) {
                            double a, b;
                            int pos = ax == 0 ? i : (ax == 1 ? j : k);
                            if (cpml_ab_depth(g, ax, (double)axis_depth(g, ax, pos), &a, &b)) {
                                psi_u[ax][id] = b * psi_u[ax][id] + a * du[ax];
                                du[ax] += psi_u[ax][id];
                            }
                        }
                    }
                    double div = du[0] + du[1] + du[2];
                    pn[id] = G * (p[id] + g->dt * K * (div + S[id]));
                    if (g->fs && k == 0) pn[id] = 0.0; /* pressure release: p = 0 on the surface plane */
                }
        memcpy(p, pn, N * sizeof(double));
        if (traces)
            for (int r = 0; r < nrec; ++r)
                traces[(size_t)n * nrec + r] = p[lin(g, rec[3 * r], rec[3 * r + 1], rec[3 * r + 2])];
    }
    if (!state) free(st);
    free(pn); free(S);
    return ORC_OK;
}

/* Discrete energy between p^n (p_n) and p^{n+1} (p_n1) with u^{n+1/2}
 * (u_half, 3N): E = sum over faces |u|^2 / b + sum over cells p^n p^{n+1} / K,
 * which the scheme keeps constant without sponge and source. */
double orc_iso_energy(const orc_grid* g, const double* vel, const double* rho, const double* p_n, const double* p_n1,
                      const double* u_half) {
    size_t N = npts(g);
    double e = 0.0;
    for (int k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t id = lin(g, i, j, k);
                for (int ax = 0; ax < 3; ++ax) {
                    double w = u_half[(size_t)ax * N + id];
                    e += w * w / face_b(g, rho, i, j, k, ax);
                }
                e += p_n[id] * p_n1[id] / (rho[id] * vel[id] * vel[id]);
            }
    return e;
}
