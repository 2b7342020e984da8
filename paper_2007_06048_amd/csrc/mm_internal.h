// Internal types shared by the host runtime (mm_api.cpp) and the gfx950
// kernels (mm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace mm {

// Per-shot device descriptor.  All 3D arrays are [nz][ny][nx], x fastest.
struct ShotDev {
    float* buf[2];        // wavefields: after k steps p^k is buf[k&1], p^{k-1} is buf[(k+1)&1]
    float* vdt2;          // (dt v)^2
    const float* prof;    // sponge: g_x[nx] g_y[ny] g_z[nz]; CPML: a_x b_x [nx], a_y b_y [ny], a_z b_z [nz]
    float* psi[3];        // CPML memory, slab layouts (see minimod.h); adjoint fields: its adjoint
    float* psi2[3];       // forward fields, fused CPML kernel: the second buffer of psi (psi^k in psi at even k,
                          // in psi2 at odd k; the layer pass keeps psi in place in psi)
    float* zeta[3];
    // the correction added to the Laplacian this step by the stencil kernel (bc 2), slabs of cw
    // cells per end, written by the layer pass of the step (forward) or the adjoint CPML kernel
    float* corr[3];
    int nx, ny, nz, nb;
    int cw;               // width of the correction slabs: nb (forward), nb + 4 (adjoint)
    int fs;               // free surface on plane z = 0 (p = 0 there, odd mirror above)
    int nsrc_in;          // sources added inside the stencil kernel (0..4)
    int src_col[4];       // their columns in the wavelet row
    long long src_off[4]; // their cells
    // acoustic_iso (staggered grid): vdt2 holds dt rho v^2, rdt rho / dt; u[a]
    // the particle velocity on the faces (index i of u_x is the face i+1/2)
    float* u[3];
    float* rdt;
};

enum { MAX_INLINE_SRC = 4 };

// One z-marching tile of one shot: the kernel stages the xy rectangle of
// its launch's tile shape at (x0, y0) and writes the cells [x0, x1) x
// [y0, y1) x [z0, z1) (x1, y1 clip the rectangle to the tile's region).
struct TileEnt {
    int shot, x0, y0, z0, z1, flags, x1, y1;
};

// TileEnt::flags: the tile meets the x / y / z damping layer (CPML), or
// holds a source added inside the stencil kernel.
enum { TF_LX = 1, TF_LY = 2, TF_LZ = 4, TF_SRC = 8 };

// Stencil weights a_m / h^2 per axis (m = 1..4) and first-derivative weights
// beta_m / h (CPML).
struct Coefs {
    float cx[4], cy[4], cz[4];
    float bx[4], by[4], bz[4];
    float sx[4], sy[4], sz[4];  // staggered first-difference weights c_m / h (acoustic_iso)
};

// Point injection table in CSR form: unique cells, each with the list of
// columns of the value row that land on it.
struct InjTab {
    const int* cell_shot;
    const long long* cell_off;
    const int* start;     // [ncell + 1]
    const int* col;       // column in the value row
    const float* cell_g;  // sponge factor G at the cell (1 if no sponge)
    int ncell;
    float scale;          // 1/(dx dy dz) for sources, 1 for adjoint residuals
};

// Point gather table.
struct GatherTab {
    const int* shot;
    const long long* off;
    int n;
};

// Extra per-step operands.
//  mode 1: d2p[x] = G (dt v)^2 Lap p^n + the source term (= p^{n+1} - 2G p^n
//          + G^2 p^{n-1}; single shot)
//  mode 2: grad[x] += neg_inv_dt2 / G * p^{n+1}[x] * d2p[x]  (imaging)
//  inline sources: lap += src_scale * wrow[col] at a shot's source cells
//  folded record: the first gather_blocks blocks copy p^n (the previous
//  step's output) at the receivers into gather_out
struct StepAux {
    void* d2p_out;
    const void* d2p_in;
    int d2p_bf16;  // the d2p segment holds bfloat16 (round to nearest even) instead of float
    float* grad;
    float neg_inv_dt2;
    float src_scale;
    const float* wrow;
    const int* g_shot;
    const long long* g_off;
    int g_n;
    int gather_blocks;  // multiple of 8 (keeps the XCD pattern of the tile blocks)
    float* gather_out;
    // 1: in forward steps p^{n-1} and (dt v)^2, read once per step, are
    // loaded with the non-temporal hint (set when the step's working set
    // exceeds the Infinity Cache, so they do not evict the reused p^n)
    int stream_loads;
};

enum { MODE_PLAIN = 0, MODE_D2P = 1, MODE_IMAGE = 2 };

// Tile variants of the stencil kernel.
struct TileShape {
    int tx;     // tile width in x (threads per row)
    int ry;     // rows per thread
    int nt;     // threads per block (256, 512 or 1024): nt / tx thread rows
    int target; // desired number of blocks (z-chunking)
    int pd;     // planes of loads in flight ahead of the current plane (1 or 2)
    const char* name;
};
int num_tile_variants();
const TileShape& tile_variant(int t);
int tile_rows(int t);  // TY of variant t

// bc: 0 none, 1 sponge, 2 CPML (launch_cpml_forward or launch_cpml_adjoint
// must have written the layer corrections of the same step first)
// With ev0 / ev1 the launch records its own start and end time stamps into
// them (hipExtLaunchKernel), for per-launch timing without extra packets.
hipError_t launch_step(int variant, int bc, int mode, const TileEnt* tiles, int ntiles,
                       const ShotDev* shots, int parity, const Coefs& cf, const StepAux& aux,
                       hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
// Forward CPML step of the tiles that meet a layer, memory update included.
// kind: CS_FRAME, the tiles of the middle z range (flagged TF_LX / TF_LY);
// CS_ZLAYER, the tiles of the z-layer chunks [0, nb) and [nz - nb, nz) that
// meet no x or y layer; CS_ZCORNER, those that do; CS_ALL, any mix of the
// three in one launch (z-layer tiles flagged TF_LZ, frame tiles not; all of
// the corner shape).  mode MODE_PLAIN or MODE_D2P.  The tiles of each kind
// are cstep_tile_w(kind) x cstep_tile_h(kind).
enum { CS_FRAME = 0, CS_ZLAYER = 1, CS_ZCORNER = 2, CS_ALL = 3 };
hipError_t launch_cpml_step(int kind, int mode, const TileEnt* tiles, int ntiles, const ShotDev* shots, int parity,
                            const Coefs& cf, const StepAux& aux, hipStream_t s, hipEvent_t ev0 = nullptr,
                            hipEvent_t ev1 = nullptr);
int cstep_tile_w(int kind);
int cstep_tile_h(int kind);
// Forward CPML layer pass of the shots [0, nshots) of `shots` for this step,
// before the stencil kernel with bc 2: psi^{n+1} and zeta^{n+1} (in place in
// ShotDev::psi and zeta) and the correction D1 psi^{n+1} + zeta^{n+1} of
// every layer cell (slabs of nb cells per end, nb <= 128).  The block table
// (cpml_block_table with width nb) and ev0 as for launch_cpml_adjoint;
// stream: non-temporal loads of psi and zeta.
hipError_t launch_cpml_forward(const ShotDev* shots, int nshots, int nb, bool stream, const int* block_off_dev,
                               const int* block_off_host, int parity, const Coefs& cf, hipStream_t s,
                               hipEvent_t ev0 = nullptr);
// Adjoint CPML memory update and corrections of every shot for this step,
// before the adjoint stencil kernel: the transposed memory recursions and a
// correction reaching 4 cells past the layer (nb <= 64).  The block table
// (3 (nshots + 1) ints, made by cpml_block_table with width nb + 4) is passed
// both as the device copy the kernel reads and as the host copy that sizes
// the grid.  ev0 (may be null) receives the kernel's start time stamp.
void cpml_block_table(const int* nx, const int* ny, const int* nz, int nshots, int width, int* off);
hipError_t launch_cpml_adjoint(const ShotDev* shots, int nshots, int nb, const int* block_off_dev,
                               const int* block_off_host, int parity, const Coefs& cf, hipStream_t s,
                               hipEvent_t ev0 = nullptr);
// acoustic_iso: one step is launch_iso_u (u^{n+1/2} from p^n = buf[parity])
// then launch_iso_p (p^{n+1} into buf[parity ^ 1]), over the same tile
// table as the stencil kernel; bc 0 none, 1 sponge.  Sources are added by
// launch_inject (vdt2 = dt rho v^2).  stream: the working set exceeds the
// Infinity Cache (non-temporal loads of data read for the last time).  ev0 /
// ev1 (may be null) receive the start of the first and the end of the second
// kernel.
hipError_t launch_iso_step(int variant, int bc, bool stream, const TileEnt* tiles, int ntiles, const ShotDev* shots,
                           int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
bool iso_variant_ok(int variant);
// dt rho v^2 and rho / dt of one shot (n cells)
hipError_t launch_iso_setup(const float* vel, const float* rho, long long n, double dt, float* kdt, float* rdt,
                            hipStream_t s);
hipError_t launch_inject(const InjTab& tab, const ShotDev* shots, int parity, const float* vals, int ncols,
                         int mode, const StepAux& aux, hipStream_t s);
hipError_t launch_gather(const GatherTab& tab, const ShotDev* shots, int parity, float* out, hipStream_t s);
hipError_t launch_vdt2(const float* vel, float* vdt2, long long n, double dt, hipStream_t s);
hipError_t launch_vcheck(const float* vel, long long n, unsigned* result2, hipStream_t s);
hipError_t launch_fill(float* p, long long n, float v, hipStream_t s);
// Watchdog: w[0] |= 1 and w[1] = min(w[1], step) if p[0 .. n) holds NaN or
// Inf; launch_watch_reset sets w = {0, 0xFFFFFFFF}.
hipError_t launch_watch(const float* p, long long n, int step, unsigned* w, hipStream_t s);
hipError_t launch_watch_reset(unsigned* w, hipStream_t s);
hipError_t launch_copy(float* dst, const float* src, long long n, hipStream_t s);
// BF16 snapshot codec of a checkpoint (p^{k-1}, p^k): c0 = bf16(p^k / s0),
// c1 = bf16((p^k - p^{k-1}) / s1), scales per block of SNAP_BLOCK cells
// (snap_blocks(n) of each); decode writes both fields back.
constexpr int SNAP_BLOCK = 4096;
long long snap_blocks(long long n);
hipError_t launch_snap_encode(const float* prev, const float* cur, long long n, uint16_t* c0, uint16_t* c1, float* s0,
                              float* s1, hipStream_t s);
hipError_t launch_snap_decode(const uint16_t* c0, const uint16_t* c1, const float* s0, const float* s1, long long n,
                              float* prev, float* cur, hipStream_t s);
hipError_t launch_residual_loss(const float* traces, const float* dobs, float* resid, long long n,
                                double* partial, int nparts, double* loss, hipStream_t s);

// Device address of this GPU's static workspace (mm_init_static) and its size.
hipError_t static_workspace(void** out);
size_t static_workspace_bytes();

}  // namespace mm
