/*
 * minimod.h - C ABI of the MI355X (gfx950) acoustic_iso_cd propagator.
 *
 * Method (Meng, Atle, Calandra, Araya-Polo, "Minimod: A Finite Difference
 * solver for Seismic Modeling", arXiv 2007.06048):
 *  - Eq. (acoustic_iso_cd): (1/v^2) p_tt - Lap p = f, constant density;
 *  - Eq. (minimod-semidisc): p^{n+1} - Q p^n + p^{n-1} = dt^2 v^2 f^n,
 *    Q = 2 + dt^2 v^2 Lap (second-order leapfrog in time);
 *  - the 25-point stencil of section "Finite Differences": radius 4 per axis,
 *    8th-order Taylor coefficients c_m = a_m/h^2,
 *    a = (8/5, -1/5, 8/315, -1/560);
 *  - Algorithm 1 (time loop from p^0 = 0, source added every step) and
 *    Algorithm 2 (inner region plus damping slabs on the six faces, PML/CPML
 *    boundary per section "Minimod Description").
 * Where the paper is silent this library implements the readings below
 * (they are also the readings of the test oracle):
 *  - source term: s^n = w(t_n) / (dx dy dz) at the source cell, entering
 *    p^{n+1} as dt^2 v^2 s^n (a discrete point source);
 *  - cells outside the grid are zero (radius-4 ghost zone);
 *  - MM_BC_SPONGE: p^{n+1} = G (2 p^n - G p^{n-1} + D (Lap p^n + s^n)),
 *    D = (dt v)^2, G = g(i) g(j) g(k), g = exp(-(sigma d)^2) at depth d =
 *    nb - k cells inside a layer of nb cells, 1 elsewhere;
 *  - MM_BC_CPML: kappa = 1 recursive-convolution CPML of the second-order
 *    equation: per damped axis psi <- b psi + a D1 p^n,
 *    zeta <- b zeta + a (D2 p^n + D1 psi), Lap gains D1 psi + zeta in the
 *    layer; d = d0 q^2, d0 = -3 vmax ln(R) / (2 nb h), alpha = pi f0 (1 - q),
 *    b = exp(-(d + alpha) dt), a = d (b - 1)/(d + alpha), q = depth/nb;
 *  - dt = cfl * 2 / (vmax sqrt(S (dx^-2 + dy^-2 + dz^-2))), S = 4 (a1 + a3):
 *    cfl is the fraction of the leapfrog stability limit;
 *  - receivers: traces[n][r] = p^{n+1} at the receiver cell.
 *
 * Conventions.
 *  - All 3D arrays handed to the library are float32, C order [nz][ny][nx]
 *    (x fastest), in device memory.  Point lists are host int32 triples
 *    (i, j, k) = (x, y, z), 0-based.
 *  - Every device buffer belongs to the caller: velocities, wavelets,
 *    traces, gradients and the workspace.  The library never allocates
 *    device memory; it owns only small host tables and HIP graph objects,
 *    released by mm_destroy.
 *  - All work is enqueued on the stream given to mm_init (NULL = the null
 *    stream).  Functions return when the work is enqueued, except where
 *    noted (mm_gradient reads the loss back and synchronises).
 *  - Time: after k steps the context holds (p^{k-1}, p^k).
 *    mm_forward_steps(n) produces p^{k+1} .. p^{k+n}; wavelet row j is
 *    w(t_{k+j}) and enters p^{k+j+1}; traces row j is p^{k+j+1} at the
 *    receivers.
 *  - Errors: every function returns an mm_status and mm_last_error()
 *    describes a failure.  Argument, state, stability and workspace errors
 *    are found before anything is enqueued, so the context is unchanged.
 *    MM_ERR_DEVICE (a HIP call failed) can come after part of a run was
 *    enqueued: the context then refuses further steps with MM_ERR_STATE
 *    until mm_reset.  A context is not thread-safe; use one per stream.
 *  - Batches: a context holds one or more shots, each on its own grid
 *    (sub-volume) with its own sources and receivers; all shots share
 *    spacing, dt, boundary kind and width.  Wavelet and trace rows
 *    concatenate the shots' sources / receivers in shot order.  One launch
 *    per kernel per time step covers every shot.
 */
#ifndef MINIMOD_H
#define MINIMOD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mm_ctx mm_ctx;

typedef enum {
    MM_OK = 0,
    MM_ERR_ARG = 1,         /* invalid size, spacing, point, pointer or option */
    MM_ERR_UNSTABLE = 2,    /* cfl > 1 or dt above the stability limit */
    MM_ERR_WORKSPACE = 3,   /* workspace too small or misaligned */
    MM_ERR_DEVICE = 4,      /* a HIP call failed */
    MM_ERR_STATE = 5,       /* call not valid in the context's current state */
    MM_ERR_NONFINITE = 6,   /* NaN/Inf or non-positive velocity */
    MM_ERR_UNSUPPORTED = 7  /* valid request the library does not implement */
} mm_status;

typedef enum { MM_BC_NONE = 0, MM_BC_SPONGE = 1, MM_BC_CPML = 2 } mm_bc;

/* Propagators of section "Minimod Description".
 *  - MM_MODEL_ISO_CD: acoustic_iso_cd, Eq. (acoustic_iso_cd), the second-order
 *    constant-density equation described above (every feature of this ABI);
 *  - MM_MODEL_ISO: acoustic_iso, Eq. (acoustic_iso_vd), the first-order
 *    variable-density system (1/(rho v^2)) dp/dt - div u = f, rho du/dt -
 *    grad p = 0 on the staggered (Yee) grid: p at cell centres, u_x at the
 *    faces (i+1/2, j, k) (array index i), u_y at (i, j+1/2, k), u_z at
 *    (i, j, k+1/2); order-8 staggered differences c = (1225/1024, -245/3072,
 *    49/5120, -5/7168); staggered leapfrog
 *      u^{n+1/2} = G (u^{n-1/2} + dt b D+ p^n),
 *      p^{n+1}   = G (p^n + dt rho v^2 (D- . u^{n+1/2} + s^n)),
 *    b the face buoyancy 2 / (rho_0 + rho_1), one over the mean density of
 *    the two cells beside the face (1/rho of the inner cell on the last
 *    face), G the cell's sponge factor;
 *    dt = cfl / (C vmax sqrt(dx^-2 + dy^-2 + dz^-2)), C = 2161/1680.
 *    Forward modelling only, bc none, sponge or CPML, with or without the
 *    free surface (p = 0 on the top plane and odd above it, u_z even about
 *    it).  CPML (section "Finite Differences"): inside the layers D+ p (at
 *    the faces) and D- u (at the cells) each gain a memory psi <- b psi + a
 *    (that derivative), with the coefficients of the constant-density CPML
 *    evaluated at the face's or cell's own depth in the layer. */
typedef enum { MM_MODEL_ISO_CD = 0, MM_MODEL_ISO = 1 } mm_model;

/* Forward CPML strategy of acoustic_iso_cd (mm_params.cpml_kernel).  Both
 * compute the same update (section "Finite Differences", CPML); they differ
 * in the kernels and in the order the layer terms are summed, so results
 * agree to rounding. */
typedef enum {
    MM_CPML_AUTO = 0,  /* tuned with the tile variant when tile == -1, else the layer pass when 30 % or
                          more of the cells lie in a damping layer */
    MM_CPML_LAYER = 1, /* a layer kernel updates the memory of every layer cell and writes a
                          correction that the stencil kernel over the whole grid adds (best when the
                          layers hold a large share of the cells) */
    MM_CPML_FUSED = 2  /* the stencil kernel runs the interior, a fused kernel the cells near the faces
                          with their memory update in the same pass (no correction array) */
} mm_cpml_kernel;

/* Snapshot storage of the gradient's checkpoints. */
typedef enum {
    MM_SNAP_FP32 = 0, /* lossless */
    MM_SNAP_BF16 = 1  /* p^k and the increment p^k - p^{k-1} in bfloat16, each scaled per block of
                         4096 cells by its largest magnitude; see mm_snap_encode.  The replay's
                         per-step d2p fields (the imaging condition's second time difference of
                         the forward field) are kept in bfloat16 too, rounded to nearest even
                         (no scale: bfloat16 has the exponent range of float) */
} mm_snap;

typedef struct {
    int32_t nx, ny, nz;      /* grid points per axis (single-shot contexts) */
    double dx, dy, dz;       /* spacing, metres */
    double dt;               /* time step, s; 0 => cfl * stability limit */
    double cfl;              /* fraction of the stability limit, (0, 1]; used when dt == 0 */
    double vmax;             /* velocity for dt and CPML d0; 0 => max of the model(s) */
    int32_t bc;              /* mm_bc */
    int32_t nb;              /* damping layer width in cells; each axis needs n >= 2 nb + 1 (sponge),
                                2 nb + 4 (CPML, nb <= 128), 2 nb + 8 (CPML with ckpt_every > 0, nb <= 64) */
    double sponge_sigma;     /* sponge strength (0.015 typical) */
    double cpml_R;           /* CPML nominal reflection coefficient, (0, 1]; 1 disables damping */
    double cpml_f0;          /* CPML frequency: alpha_max = pi * cpml_f0, >= 0 */
    int32_t ckpt_every;      /* gradient checkpoint interval in steps; 0 => no gradient support */
    int32_t snap;            /* mm_snap for the checkpointed wavefields (CPML memory is kept in FP32) */
    int32_t nsteps_max;      /* longest gradient / adjoint run the workspace must hold */
    int32_t tile;            /* stencil tile variant; 0 => library default, -1 => autotune at init */
    int32_t group_kb;        /* batches: consecutive shots run in groups whose working set (fields,
                                CPML memory) is at most this many KiB, each group's time steps back to
                                back, so a group stays resident in the 256 MB last-level cache; a shot
                                larger than the budget is a group of its own; 0 => 262144 (256 MiB),
                                -1 => one group: all shots advance together */
    int32_t free_surface;    /* 1: free surface on the top face (section "Minimod Description": the
                                option at the surface): p = 0 on the plane z = 0, the cells above it
                                mirror p with odd symmetry, and the top face has no damping layer;
                                sources and receivers on that plane inject and record nothing */
    int32_t model;           /* mm_model; 0 => acoustic_iso_cd */
    int32_t cache_hints;     /* loads of data a step reads once (p^{n-1}, (dt v)^2, CPML memory and
                                corrections; acoustic_iso: p^n and dt rho v^2 in the pressure kernel)
                                with the non-temporal hint: 0 auto (when the working set of every
                                shot of a launch exceeds the 256 MiB Infinity Cache), 1 never,
                                2 always.  Results are bitwise the same either way; only the speed
                                differs. */
    int32_t watch_every;     /* > 0: after every watch_every-th forward step (counted from step 0)
                                the new wavefield of every shot is scanned for NaN or Inf on the
                                device (one extra read of the field, no synchronisation); the first
                                such step is kept and reported by mm_watch (and by mm_gradient) as
                                MM_ERR_NONFINITE.  0 => off */
    int32_t cpml_kernel;     /* mm_cpml_kernel; 0 => MM_CPML_AUTO */
} mm_params;

/* One shot of a batched context. */
typedef struct {
    int32_t nx, ny, nz;            /* grid of this shot */
    const float* vel;              /* device [nz][ny][nx] velocity, m/s (read only during init) */
    const int32_t* src_ijk;        /* host [nsrc][3] */
    int32_t nsrc;
    const int32_t* rec_ijk;        /* host [nrec][3] */
    int32_t nrec;
    const float* rho;              /* device [nz][ny][nx] density, kg/m^3 (acoustic_iso only, read only
                                      during init; ignored by acoustic_iso_cd) */
} mm_shot;

/* Fill *p with defaults (sponge 0.015, CPML R = 1e-3, cfl 0.5, ...). */
void mm_default_params(mm_params* p);

/* Stable time step for params p and maximum velocity vmax (host only).
 * Returns MM_ERR_UNSTABLE if p->dt > 0 exceeds the limit or p->cfl > 1. */
mm_status mm_dt(const mm_params* p, double vmax, double* dt_out);

/* Ricker wavelet w_i = (1 - 2 pi^2 f0^2 tau^2) exp(-pi^2 f0^2 tau^2),
 * tau = i dt - t0, i = 0..n-1, computed in FP64 and rounded to float
 * (host only; the source signature is a reading, the paper gives fmax). */
mm_status mm_ricker(double f0, double t0, double dt, int32_t n, float* host_out);

/* Device workspace needed by a context with these shots (bytes, multiple
 * of 256).  Nothing is launched. */
mm_status mm_workspace_size(const mm_params* p, int32_t nshots, const mm_shot* shots, size_t* bytes);

/* Create a context: validates, derives dt, computes (dt v)^2 and the
 * boundary tables on the device, zeroes the state (step 0).  workspace is a
 * caller-owned device buffer of at least mm_workspace_size bytes, 256-byte
 * aligned, that must outlive the context.  hip_stream is a hipStream_t (or
 * NULL).  If p->vmax == 0 the models are reduced on the device and read
 * back (a synchronisation). */
mm_status mm_init_batch(mm_ctx** out, const mm_params* p, int32_t nshots, const mm_shot* shots,
                        void* workspace, size_t ws_bytes, void* hip_stream);

/* Single-shot form: the grid is p->nx * p->ny * p->nz, velocity vel_dev. */
mm_status mm_init(mm_ctx** out, const mm_params* p, const float* vel_dev, const int32_t* src_ijk_host,
                  int32_t nsrc, const int32_t* rec_ijk_host, int32_t nrec, void* workspace, size_t ws_bytes,
                  void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * as mm_init, with the context's device memory taken from a fixed array of
 * 64 MiB that the library holds on every GPU it runs on until the process
 * ends, instead of a caller workspace.  Calls no hipMalloc, hipFree or other
 * allocating routine and runs no autotuning (p->tile == -1 runs the default
 * tile variant).  The array is per GPU (the current device) and shared by
 * every call on that GPU: a later mm_init_static on the same GPU takes it
 * over, after which the earlier context fails every call except
 * mm_destroy with MM_ERR_STATE; calls that overlap on one GPU (two threads,
 * or work of the earlier context still in flight on its stream) race.
 * Everything the run needs at zero is cleared by this call.  Errors as
 * mm_init, and MM_ERR_WORKSPACE with the sizes in mm_last_error(NULL) when
 * mm_workspace_size of the problem exceeds 64 MiB. */
mm_status mm_init_static(mm_ctx** out, const mm_params* p, const float* vel_dev, const int32_t* src_ijk_host,
                         int32_t nsrc, const int32_t* rec_ijk_host, int32_t nrec, void* hip_stream);

/* Advance nsteps steps.  wavelet: device [nsteps][nsrc_total] raw samples
 * (may be NULL only if nsrc_total == 0).  traces: device
 * [nsteps][nrec_total] or NULL.  If the context was made with
 * ckpt_every > 0 and the run starts at step 0, checkpoints are stored and
 * the wavelet is kept for the gradient's replay (nsteps <= nsteps_max). */
mm_status mm_forward_steps(mm_ctx* ctx, int32_t nsteps, const float* wavelet, float* traces);

/* Same result as mm_forward_steps, with the whole step loop captured once
 * into a HIP graph and launched as one graph (re-used while nsteps and the
 * pointers are unchanged).  Bitwise identical to mm_forward_steps. */
mm_status mm_forward_steps_graph(mm_ctx* ctx, int32_t nsteps, const float* wavelet, float* traces);

/* Adjoint (reverse-time) steps: the exact transpose of the forward steps
 * (the inverse problem motivating the method, section "Seismic Modeling").
 * The scaled adjoint eta obeys the forward recursion run backward with the
 * residual injected at the receivers with unit scale:
 *   eta^m = G (2 eta^{m+1} - G eta^{m+2} + D (Lap eta^{m+1} + C + R^T r^m)),
 * C = 0 except for CPML, where the transposed memory recursions
 *   Zb <- eta^{m+1} + b Zb,  Pb <- b Pb - D1 (eta^{m+1} + a Zb)  (layer cells)
 * give C = sum over damped axes of D2 (a Zb) - D1 (a Pb).
 * The first call starts from eta = 0 at time m = T (the forward step count)
 * and each call continues downward.  resid: device [nsteps][nrec_total] in
 * forward time order (row j pairs with the trace of p^{m0+j}, where
 * m0 = current adjoint time - nsteps + 1).  adj_at_src (device
 * [nsteps][nsrc_total] or NULL) receives eta^{m} at the sources, same row
 * order.  grad_m (device [nz][ny][nx] of a single-shot context, or NULL) is
 * accumulated with -(1/(dt^2 G)) eta^m (p^m - 2 G p^{m-1} + G^2 p^{m-2}),
 * the imaging condition of the gradient w.r.t. m = 1/v^2; it needs the
 * checkpoints of a forward run made from step 0 with ckpt_every > 0, and
 * clobbers the forward state (call mm_reset before a new forward run). */
mm_status mm_adjoint_steps(mm_ctx* ctx, int32_t nsteps, const float* resid, float* adj_at_src, float* grad_m);

/* FWI gradient of J = 1/2 sum_n sum_r (d^n_r - d_obs^n_r)^2 w.r.t.
 * m = 1/v^2 for a single-shot context: reset, forward nsteps with
 * checkpoints, residual, adjoint with imaging.  grad_m is overwritten;
 * traces (device [nsteps][nrec], may be NULL) receives the modelled data;
 * loss_host (may be NULL) receives J (this synchronises the stream). */
mm_status mm_gradient(mm_ctx* ctx, int32_t nsteps, const float* wavelet, const float* d_obs, float* grad_m,
                      float* traces, double* loss_host);

/* Zero the forward and adjoint state and the CPML memory; step = 0. */
mm_status mm_reset(mm_ctx* ctx);

/* BF16 snapshot codec of the gradient's checkpoints (MM_SNAP_BF16): the
 * state (p^{k-1}, p^k) of the leapfrog of Eq. (minimod-semidisc) as
 *   c0[i] = bf16(p^k[i] / s0[b]),   c1[i] = bf16((p^k[i] - p^{k-1}[i]) / s1[b]),
 * b = i / 4096, with s0[b] (s1[b]) the largest magnitude of p^k (of the
 * increment) over cells 4096 b .. 4096 b + 4095 (1 if all are zero); float
 * division and subtraction rounded to nearest, bf16 = round to nearest even
 * of the float.  Decoding writes p^k[i] = f(c0[i]) * s0[b] and
 * p^{k-1}[i] = p^k[i] - f(c1[i]) * s1[b], f the exact bf16 -> float
 * widening, each product and the difference rounded once.
 * Arguments: prev, cur: device float [n]; c0, c1: device uint16 [n];
 * s0, s1: device float [mm_snap_blocks(n)]; all caller-owned, not
 * overlapping; enqueued on `stream` (hipStream_t, NULL = default stream).
 * Errors: MM_ERR_ARG for n < 0 or a NULL array with n > 0, MM_ERR_DEVICE
 * for a failed launch. */
int64_t mm_snap_blocks(int64_t n);
mm_status mm_snap_encode(const float* prev_dev, const float* cur_dev, int64_t n, uint16_t* c0_dev,
                         uint16_t* c1_dev, float* s0_dev, float* s1_dev, void* stream);
mm_status mm_snap_decode(const uint16_t* c0_dev, const uint16_t* c1_dev, const float* s0_dev, const float* s1_dev,
                         int64_t n, float* prev_dev, float* cur_dev, void* stream);

/* Result of the watchdog (mm_params.watch_every): synchronises the context's
 * stream and returns MM_ERR_NONFINITE if a scanned wavefield held NaN or Inf
 * (*bad_step, if not NULL, receives the first such step: the state after it),
 * else MM_OK with *bad_step = -1.  The finding stays until mm_reset or
 * mm_set_state.  MM_ERR_STATE if the context was made with watch_every = 0. */
mm_status mm_watch(mm_ctx* ctx, int32_t* bad_step);

/* Size of the state blob of mm_get_state / mm_set_state, in bytes. */
mm_status mm_state_size(const mm_ctx* ctx, size_t* bytes);

/* Copy the state to / from a caller device buffer.  Layout per shot, in
 * shot order (acoustic_iso: p^k, u_x, u_y, u_z at k - 1/2, each
 * [nz][ny][nx]); acoustic_iso_cd: p^{k-1} [nz][ny][nx], p^k [nz][ny][nx] (float32), then for
 * CPML psi_x, psi_y, psi_z, zeta_x, zeta_y, zeta_z in slab layout:
 * x-slabs [nz][ny][2nb], y-slabs [nz][2nb][nx], z-slabs [2nb][ny][nx],
 * where slab index s < nb is grid index s and s >= nb is grid index
 * n - 2nb + s.  mm_set_state also sets the step counter; with a free surface
 * it leaves p = 0 on the surface plane. */
mm_status mm_get_state(mm_ctx* ctx, void* dst_dev);
mm_status mm_set_state(mm_ctx* ctx, const void* src_dev, int32_t step);

/* Time step, step counter, tile variant and number of shot groups in use.
 * Any output pointer may be NULL. */
mm_status mm_get_info(const mm_ctx* ctx, double* dt, int32_t* step, int32_t* tile, int32_t* ngroups);

/* The forward CPML strategy in use (MM_CPML_LAYER or MM_CPML_FUSED; MM_CPML_AUTO
 * for other boundaries and for acoustic_iso). */
mm_status mm_get_cpml_kernel(const mm_ctx* ctx, int32_t* kernel);

/* Pick the stencil tile variant by timing each candidate on this context
 * (state is zeroed afterwards; synchronises).  steps_per_trial (>= 1) is a
 * minimum: it is raised so that one trial lasts about 2 ms (at most 200
 * steps); every variant is timed once and the four fastest twice more,
 * interleaved, keeping each one's best time; with MM_CPML_AUTO the four
 * are also timed in the other forward CPML strategy, which is kept if it
 * wins by 3% or more.  Results are cached per (grid, boundary, model, grouping) for the
 * life of the process.  *tile_out may be NULL. */
mm_status mm_autotune(mm_ctx* ctx, int32_t steps_per_trial, int32_t* tile_out);

/* Force a tile variant (0 = default).  Returns MM_ERR_ARG if unknown. */
mm_status mm_set_tile(mm_ctx* ctx, int32_t tile);

/* Number of tile variants and a description of variant t (static string). */
int32_t mm_num_tiles(void);
const char* mm_tile_name(int32_t t);

/* Step timing on the context's stream: while stride > 0, every stride-th
 * time step (of one shot group) records the start of its first kernel and
 * the end of its last kernel into a pair of HIP events, stamped by the
 * launches themselves (hipExtLaunchKernel, no extra stream packets).  A
 * step is the kernels that advance the wavefields by one time level (with
 * CPML the layer kernel and the stencil kernel); point injection by a
 * separate kernel (more than 4 sources per shot) is not included.
 * mm_profile_read synchronises the stream, returns the summed
 * milliseconds and the number of timed steps, and clears the record.
 * stride 0 stops timing.  Graph launches are not timed. */
mm_status mm_profile(mm_ctx* ctx, int32_t stride);
mm_status mm_profile_read(mm_ctx* ctx, double* ms, int32_t* launches);

void mm_destroy(mm_ctx* ctx);
const char* mm_status_str(mm_status s);
/* Message of the last failed call on ctx (or of the last failed call that
 * had no context, if ctx is NULL).  Never NULL. */
const char* mm_last_error(const mm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* MINIMOD_H */
