// gfx950 kernels of the acoustic_iso_cd propagator.
//
// Time step (Eq. (minimod-semidisc) of the paper, second-order leapfrog)
//   p^{n+1} = G (p^n + ((p^n - G p^{n-1}) + D Lap p^n)),   D = (dt v)^2,
// with the 25-point radius-4 Laplacian of section "Finite Differences"
// evaluated in the paper's own form
//   Lap p = sum_m c_xm [(p(i+m)-p) + (p(i-m)-p)] + (same in y and z),
// which keeps FP32 rounding about ten times smaller than folding the -2p
// terms into one centre weight.  G is the sponge factor (1 without sponge).
//
// Memory plan (HBM-bound: ~16 algorithmic bytes and ~50 flops per point):
//  - one block owns an xy tile of TX x TY points and marches along z over a
//    chunk of planes; each p^n value is read from HBM once, its z
//    neighbours live in a 9-deep register queue per thread, its x/y
//    neighbours come from a double-buffered LDS copy of the current plane
//    with radius-4 halos (halos are L2 / infinity-cache hits: the
//    neighbouring tiles read them as their own interior);
//  - the next plane's loads (queue head, halos, p^{n-1}, D) are issued one
//    iteration ahead so they overlap the current plane's arithmetic;
//  - p^{n+1} overwrites p^{n-1} in place (each point is read and written by
//    the same thread), so two wavefield buffers suffice;
//  - blocks are remapped so that consecutive tiles run on the same XCD
//    (hardware deals blocks round-robin over the 8 XCDs), which keeps the
//    halo exchange between neighbouring tiles inside one XCD's L2.
// A free surface on plane z = 0 costs nothing in the loop: the host sets
// (dt v)^2 = 0 on that plane and keeps the state there at 0, so the update
// leaves p = 0 exactly, and the z queue of the first chunk starts with the
// odd mirror -p(1..4) of the planes below.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mm_internal.h"

namespace mm {

// Global-memory views: loads through a buffer resource (scalar base, 32-bit
// per-lane byte offset, hardware range check returning 0 past the end, so
// ghost cells need no branch), stores through address-space-1 pointers.
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) uint16_t gu16;
constexpr unsigned OOB = 0xFFFFFFFFu;  // byte offset that is always out of range

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf_rne(float f) {
    const unsigned u = __float_as_uint(f);
    const unsigned lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// A step's outputs (p^{n+1}, and psi^{n+1} and zeta^{n+1} in the fused CPML
// kernel) with STREAM (a working set beyond the Infinity Cache): stored with
// the non-temporal hint, so the written lines leave L2 early and the p^n lines
// that the tiles' halos and the next z-chunk's prologue re-read stay
// (1024^2 x 512 with CPML: 2392 -> 2300 us per step, the stencil 1375 ->
// 1303-1321 us).  Inside the cache the plain store is kept: there the next
// launch reads the fields back from the Infinity Cache.
template <bool NT>
__device__ __forceinline__ void put(gfloat* p, float v) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// The replay's d2p segment holds float or (BF, StepAux::d2p_bf16) bfloat16
// elements.  It is written once in the replay and read once in the imaging:
// non-temporal both ways, so it does not push the wavefields out of the caches.
template <bool BF>
__device__ __forceinline__ void d2p_put(void* seg, long long o, float v) {
    if constexpr (BF) __builtin_nontemporal_store(f2bf_rne(v), &((gu16*)seg)[o]);
    else __builtin_nontemporal_store(v, &((gfloat*)seg)[o]);
}
template <bool BF>
__device__ __forceinline__ float d2p_get(const void* seg, long long o) {
    if constexpr (BF) return __uint_as_float((unsigned)__builtin_nontemporal_load(&((const gu16*)seg)[o]) << 16);
    else return __builtin_nontemporal_load(&((const gfloat*)seg)[o]);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, int z, long long plane) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(base + (long long)z * plane), (short)0, (int)(plane * 4),
                                             0x00020000);
}

__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0));
}
// the same with the non-temporal hint (aux bit 1): for data read once per step
__device__ __forceinline__ float bload_nt(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    return __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 2));
}

// shapes (TX, RY) x z-chunking targets (total blocks over all shots; chunks
// are at least 4 planes) with one plane of prefetch, plus a few two-plane
// prefetch variants of the large tiles; entry 0 is the default
static const TileShape kTiles[] = {
    {64, 4, 256, 2048, 1, "64x16/2048/p1"},   {64, 4, 256, 1024, 1, "64x16/1024/p1"},
    {64, 4, 256, 4096, 1, "64x16/4096/p1"},   {64, 4, 256, 16384, 1, "64x16/16k/p1"},
    {64, 4, 256, 65536, 1, "64x16/64k/p1"},   {64, 2, 256, 2048, 1, "64x8/2048/p1"},
    {64, 2, 256, 1024, 1, "64x8/1024/p1"},    {64, 2, 256, 4096, 1, "64x8/4096/p1"},
    {64, 2, 256, 16384, 1, "64x8/16k/p1"},    {64, 2, 256, 65536, 1, "64x8/64k/p1"},
    {64, 8, 256, 2048, 1, "64x32/2048/p1"},   {64, 8, 256, 1024, 1, "64x32/1024/p1"},
    {64, 8, 256, 4096, 1, "64x32/4096/p1"},   {64, 8, 256, 16384, 1, "64x32/16k/p1"},
    {64, 8, 256, 65536, 1, "64x32/64k/p1"},   {32, 2, 256, 2048, 1, "32x16/2048/p1"},
    {32, 2, 256, 1024, 1, "32x16/1024/p1"},   {32, 2, 256, 4096, 1, "32x16/4096/p1"},
    {32, 2, 256, 16384, 1, "32x16/16k/p1"},   {32, 2, 256, 65536, 1, "32x16/64k/p1"},
    {32, 4, 256, 2048, 1, "32x32/2048/p1"},   {32, 4, 256, 1024, 1, "32x32/1024/p1"},
    {32, 4, 256, 4096, 1, "32x32/4096/p1"},   {32, 4, 256, 16384, 1, "32x32/16k/p1"},
    {32, 4, 256, 65536, 1, "32x32/64k/p1"},   {32, 1, 256, 2048, 1, "32x8/2048/p1"},
    {32, 1, 256, 1024, 1, "32x8/1024/p1"},    {32, 1, 256, 4096, 1, "32x8/4096/p1"},
    {32, 1, 256, 16384, 1, "32x8/16k/p1"},    {32, 1, 256, 65536, 1, "32x8/64k/p1"},
    {64, 4, 256, 1024, 2, "64x16/1024/p2"},   {64, 4, 256, 4096, 2, "64x16/4096/p2"},
    {64, 8, 256, 1024, 2, "64x32/1024/p2"},   {64, 8, 256, 2048, 2, "64x32/2048/p2"},
    {32, 2, 256, 4096, 2, "32x16/4096/p2"},   {32, 1, 256, 4096, 2, "32x8/4096/p2"},
    // larger blocks: taller tiles (fewer halo rows per point) at one or two rows per thread
    {64, 1, 1024, 1024, 1, "64x16t1024/1024"}, {64, 1, 1024, 4096, 1, "64x16t1024/4096"},
    {64, 2, 1024, 512, 1, "64x32t1024/512"},   {64, 2, 1024, 2048, 1, "64x32t1024/2048"},
    {32, 1, 1024, 1024, 1, "32x32t1024/1024"}, {32, 1, 1024, 4096, 1, "32x32t1024/4096"},
    {64, 2, 512, 1024, 1, "64x16t512/1024"},   {64, 2, 512, 4096, 1, "64x16t512/4096"},
    {32, 2, 512, 1024, 1, "32x32t512/1024"},   {32, 2, 512, 4096, 1, "32x32t512/4096"},
    {64, 4, 512, 1024, 1, "64x32t512/1024"},   {64, 4, 512, 4096, 1, "64x32t512/4096"},
};

int num_tile_variants() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileShape& tile_variant(int t) { return kTiles[t]; }
int tile_rows(int t) { return (kTiles[t].nt / kTiles[t].tx) * kTiles[t].ry; }

// ------------------------------------------------------------- stencil step

// The small-tile, one-plane-prefetch shapes are held to 72 VGPRs (7 waves per
// SIMD instead of 6 for the CPML adjoint and the imaging instantiations);
// they fit without spilling, the larger shapes and the CPML imaging mode
// would not.  BC == 2 adds the CPML corrections of the step's layer pass
// (launch_cpml_forward, or launch_cpml_adjoint for the adjoint fields); the
// other forward CPML strategy runs the interior with BC == 0 and the cells
// near the faces in k_cstep.
template <int TX, int RY, int PD, int BC, int MODE, int NT, bool STREAM, bool BF>
__global__ __launch_bounds__(NT)
__attribute__((amdgpu_waves_per_eu((PD == 1 && RY <= 2 && !(BC == 2 && MODE != MODE_PLAIN)) ? 7 : 1)))
void k_step(const TileEnt* __restrict__ tiles, int ntiles, int per_xcd, const ShotDev* __restrict__ shots,
            int parity, Coefs cf, StepAux aux) {
    constexpr int BY = NT / TX;  // thread rows
    constexpr int TY = BY * RY;
    constexpr int LW = TX + 8;
    // y halo: with BY <= 8 every thread row loads 8 / BY of the 8 halo rows,
    // with more thread rows the first 8 load one each
    constexpr bool YSPLIT = BY <= 8;
    constexpr int YH = YSPLIT ? 8 / BY : 1;
    constexpr bool SPONGE = BC == 1;
    constexpr bool CPML = BC == 2;
    static_assert(!YSPLIT || 8 % BY == 0, "y halo split");
    __shared__ float lds[2][TY + 8][LW];

    if ((int)blockIdx.x < aux.gather_blocks) {
        // record of the previous step: its output is this step's p^n (256 receivers per block)
        const int tid = threadIdx.y * TX + threadIdx.x;
        const int r = blockIdx.x * 256 + tid;
        if (tid < 256 && r < aux.g_n) aux.gather_out[r] = shots[aux.g_shot[r]].buf[parity][aux.g_off[r]];
        return;
    }
    // consecutive tiles on one XCD: block b runs on XCD b % 8
    const int b = blockIdx.x - aux.gather_blocks;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    const TileEnt te = tiles[t];
    const ShotDev& sd = shots[te.shot];
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const float* __restrict__ pc = sd.buf[parity];
    float* __restrict__ pn = sd.buf[parity ^ 1];
    const float* __restrict__ vd = sd.vdt2;
    const long long plane = (long long)nx * ny;

    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x = te.x0 + tx;
    const bool xin = x < nx;

    int row[RY];
    bool in[RY], own[RY];  // in the grid (staged in LDS) / written by this tile
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = te.y0 + ty + r * BY;
        in[r] = xin && row[r] < ny;
        own[r] = x < te.x1 && row[r] < te.y1;
    }
    // x halo: lanes 0..7 of every thread row carry the 4 left and 4 right columns
    const int hcol = tx < 4 ? te.x0 - 4 + tx : te.x0 + TX + (tx - 4);
    const bool hx_lane = tx < 8 && hcol >= 0 && hcol < nx;
    // y halo: thread row ty loads halo rows ty, ty + BY, ... of the 8
    const bool hy_row = YSPLIT || ty < 8;  // wave-uniform (a wave spans 1 or 2 thread rows)
    int hrow[YH];
    bool hy_ok[YH];
#pragma unroll
    for (int h = 0; h < YH; ++h) {
        const int hr = ty + h * BY;
        hrow[h] = hr < 4 ? te.y0 - 4 + hr : te.y0 + TY + (hr - 4);
        hy_ok[h] = hy_row && xin && hrow[h] >= 0 && hrow[h] < ny;
    }

    // per-lane byte offsets inside a plane (OOB where the cell is outside the grid)
    unsigned voc[RY], vox[RY], voy[YH];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        voc[r] = in[r] ? (unsigned)(row[r] * nx + x) * 4u : OOB;
        vox[r] = (hx_lane && row[r] < ny) ? (unsigned)(row[r] * nx + hcol) * 4u : OOB;
    }
#pragma unroll
    for (int h = 0; h < YH; ++h) voy[h] = hy_ok[h] ? (unsigned)(hrow[h] * nx + x) * 4u : OOB;
    // CPML corrections (slab arrays of cw cells per end; OOB where the cell is not in them)
    const int cw = sd.cw, cw2 = 2 * cw;
    const bool tile_layer = CPML && (te.flags & (TF_LX | TF_LY | TF_LZ));
    // (the z slab [2cw][ny][nx] is indexed like a plane of the grid: offset voc)
    unsigned vcx[CPML ? RY : 1], vcy[CPML ? RY : 1];
    if (CPML) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = row[r];
            const bool lxr = in[r] && (x < cw || x >= nx - cw);
            const bool lyr = in[r] && (y < cw || y >= ny - cw);
            // x slab of plane z: rows (z * ny + y) of 2cw cells -> offset (y * 2cw + s) inside plane z's block
            vcx[r] = lxr ? (unsigned)(y * cw2 + (x < cw ? x : x - (nx - cw2))) * 4u : OOB;
            // y slab of plane z: [2cw][nx] per plane
            vcy[r] = lyr ? (unsigned)((y < cw ? y : y - (ny - cw2)) * nx + x) * 4u : OOB;
        }
    }

    float gx = 1.0f, gyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) gyv[r] = 1.0f;
    if (SPONGE) {
        gx = xin ? sd.prof[x] : 1.0f;
#pragma unroll
        for (int r = 0; r < RY; ++r) gyv[r] = in[r] ? sd.prof[nx + row[r]] : 1.0f;
    }

    const int z0 = te.z0, z1 = te.z1;
    // z queue: planes z0-4 .. z0+3
    float q[RY][9];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int z = z0 - 4 + m;
        const bool zin = z >= 0 && z < nz;  // block-uniform
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(pc, zin ? z : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][m] = zin ? bload(rp, voc[r]) : 0.0f;
    }
    if (z0 == 0 && sd.fs) {
        // above a free surface on plane 0: the odd mirror, planes -1..-4 = -p(1..4)
        const __amdgpu_buffer_rsrc_t r4 = plane_rsrc(pc, 4 < nz ? 4 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][3] = -q[r][5];
            q[r][2] = -q[r][6];
            q[r][1] = -q[r][7];
            q[r][0] = 4 < nz ? -bload(r4, voc[r]) : 0.0f;
        }
    }

    // prefetch stages: stage k holds the loads for plane z + k (queue head p^n(z+k+4),
    // p^{n-1}(z+k), (dt v)^2(z+k), the x / y halos of plane z+k)
    float nq[PD][RY], npp[PD][RY], nvd[PD][RY], nxh[PD][RY], nyh[PD][YH];
    constexpr bool stream = STREAM;  // working set beyond the Infinity Cache: p^{n-1}, (dt v)^2 non-temporal
    constexpr int RC = CPML ? RY : 1;
    float ncr[PD][RC];  // sum of the CPML corrections of the cell (0 outside the layers)
    auto fetch = [&](int k, int zn) {
        const bool hin = zn + 4 < nz;
        const __amdgpu_buffer_rsrc_t rh = plane_rsrc(pc, hin ? zn + 4 : 0, plane);
        const __amdgpu_buffer_rsrc_t rc = plane_rsrc(pc, zn, plane);
        const __amdgpu_buffer_rsrc_t rm = plane_rsrc(pn, zn, plane);
        const __amdgpu_buffer_rsrc_t rv = plane_rsrc(vd, zn, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            nq[k][r] = hin ? bload(rh, voc[r]) : 0.0f;
            npp[k][r] = stream ? bload_nt(rm, voc[r]) : bload(rm, voc[r]);
            nvd[k][r] = stream ? bload_nt(rv, voc[r]) : bload(rv, voc[r]);
            nxh[k][r] = bload(rc, vox[r]);
        }
        if (hy_row) {
#pragma unroll
            for (int h = 0; h < YH; ++h) nyh[k][h] = bload(rc, voy[h]);
        } else {
#pragma unroll
            for (int h = 0; h < YH; ++h) nyh[k][h] = 0.0f;
        }
        if (CPML) {
#pragma unroll
            for (int r = 0; r < RC; ++r) ncr[k][r] = 0.0f;
            if (tile_layer) {
                // each axis only where the tile meets its layers (block-uniform tests)
                float a[RC], b[RC], c[RC];
#pragma unroll
                for (int r = 0; r < RC; ++r) a[r] = b[r] = c[r] = 0.0f;
                if (te.flags & TF_LX) {
                    const long long pxs = (long long)ny * cw2;
                    const __amdgpu_buffer_rsrc_t cx = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(sd.corr[0] + zn * pxs), (short)0, (int)(pxs * 4), 0x00020000);
#pragma unroll
                    for (int r = 0; r < RC; ++r) a[r] = stream ? bload_nt(cx, vcx[r]) : bload(cx, vcx[r]);
                }
                if (te.flags & TF_LY) {
                    const long long pys = (long long)cw2 * nx;
                    const __amdgpu_buffer_rsrc_t cy = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(sd.corr[1] + zn * pys), (short)0, (int)(pys * 4), 0x00020000);
#pragma unroll
                    for (int r = 0; r < RC; ++r) b[r] = stream ? bload_nt(cy, vcy[r]) : bload(cy, vcy[r]);
                }
                if ((te.flags & TF_LZ) && (zn < cw || zn >= nz - cw)) {
                    const int zs = zn < cw ? zn : zn - (nz - cw2);
                    const __amdgpu_buffer_rsrc_t cz = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(sd.corr[2] + (long long)zs * plane), (short)0, (int)(plane * 4), 0x00020000);
#pragma unroll
                    for (int r = 0; r < RC; ++r) c[r] = stream ? bload_nt(cz, voc[r]) : bload(cz, voc[r]);
                }
#pragma unroll
                for (int r = 0; r < RC; ++r) ncr[k][r] = (a[r] + b[r]) + c[r];
            }
        }
    };
#pragma unroll
    for (int k = 0; k < PD; ++k)
        if (z0 + k < z1) fetch(k, z0 + k);

    const int xx = 4 + tx;
    gfloat* __restrict__ pn_g = (gfloat*)pn;
    for (int z = z0; z < z1; ++z) {
        float cpp[RY], cvd[RY], cxh[RY], cyh[YH], ccr[RC];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][8] = nq[0][r];
            cpp[r] = npp[0][r];
            cvd[r] = nvd[0][r];
            cxh[r] = nxh[0][r];
        }
        if (CPML) {
#pragma unroll
            for (int r = 0; r < RC; ++r) ccr[r] = ncr[0][r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) cyh[h] = nyh[0][h];
#pragma unroll
        for (int k = 0; k + 1 < PD; ++k) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                nq[k][r] = nq[k + 1][r];
                npp[k][r] = npp[k + 1][r];
                nvd[k][r] = nvd[k + 1][r];
                nxh[k][r] = nxh[k + 1][r];
            }
#pragma unroll
            for (int h = 0; h < YH; ++h) nyh[k][h] = nyh[k + 1][h];
            if (CPML) {
#pragma unroll
                for (int r = 0; r < RC; ++r) ncr[k][r] = ncr[k + 1][r];
            }
        }
        if (z + PD < z1) fetch(PD - 1, z + PD);

        float(*L)[LW] = lds[z & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            L[4 + ty + r * BY][xx] = q[r][4];
            if (tx < 8) L[4 + ty + r * BY][tx < 4 ? tx : TX + tx] = cxh[r];
        }
        if (hy_row) {
#pragma unroll
            for (int h = 0; h < YH; ++h) {
                const int hr = ty + h * BY;
                L[hr < 4 ? hr : TY + hr][xx] = cyh[h];
            }
        }
        __syncthreads();

        const float gz = SPONGE ? sd.prof[nx + ny + z] : 1.0f;
        const long long zoff = (long long)z * plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yy = 4 + ty + r * BY;
            const float c = q[r][4];
            float lx = 0.0f, ly = 0.0f, lzv = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                lx = fmaf(cf.cx[m - 1], (L[yy][xx + m] - c) + (L[yy][xx - m] - c), lx);
                ly = fmaf(cf.cy[m - 1], (L[yy + m][xx] - c) + (L[yy - m][xx] - c), ly);
                lzv = fmaf(cf.cz[m - 1], (q[r][4 + m] - c) + (q[r][4 - m] - c), lzv);
            }
            float lap = (lx + ly) + lzv;
            if (CPML) lap += ccr[CPML ? r : 0];
            if (own[r]) {
                const long long o = zoff + (row[r] * nx + x);
                if ((te.flags & TF_SRC) && aux.wrow) {
#pragma unroll
                    for (int k = 0; k < MAX_INLINE_SRC; ++k)
                        if (k < sd.nsrc_in && o == sd.src_off[k]) lap = fmaf(aux.src_scale, aux.wrow[sd.src_col[k]], lap);
                }
                float out, G = 1.0f;
                if (SPONGE) {
                    G = gx * gyv[r] * gz;
                    out = G * (c + fmaf(cvd[r], lap, c - G * cpp[r]));
                } else {
                    out = c + fmaf(cvd[r], lap, c - cpp[r]);
                }
                put<STREAM>(&pn_g[o], out);
                if (MODE == MODE_D2P) d2p_put<BF>(aux.d2p_out, o, G * (cvd[r] * lap));
                if (MODE == MODE_IMAGE) {
                    gfloat* gr = (gfloat*)aux.grad;
                    gr[o] = fmaf(aux.neg_inv_dt2 / G * out, d2p_get<BF>(aux.d2p_in, o), gr[o]);
                }
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int m = 0; m < 8; ++m) q[r][m] = q[r][m + 1];
    }
}

template <int TX, int RY, int PD, int BC, int MODE, int NT, bool STREAM = false, bool BF = false>
static void launch_step_k(dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd, const ShotDev* shots, int parity,
                          const Coefs& cf, const StepAux& aux, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 block(TX, NT / TX);
    if (ev0 || ev1)  // either stamp alone is allowed (a CPML launch may have taken the start)
        hipExtLaunchKernelGGL(k_step<TX, RY, PD, BC, MODE, NT, STREAM, BF>, grid, block, 0, s, ev0, ev1, 0, tiles,
                              ntiles, per_xcd, shots, parity, cf, aux);
    else
        k_step<TX, RY, PD, BC, MODE, NT, STREAM, BF><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity,
                                                                         cf, aux);
}

template <int TX, int RY, int PD, int BC, int NT>
static hipError_t launch_step_bc(int mode, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd,
                                 const ShotDev* shots, int parity, const Coefs& cf, const StepAux& aux,
                                 hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (mode == MODE_PLAIN && aux.stream_loads)
        launch_step_k<TX, RY, PD, BC, MODE_PLAIN, NT, true>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s,
                                                            ev0, ev1);
    else if (mode == MODE_PLAIN)
        launch_step_k<TX, RY, PD, BC, MODE_PLAIN, NT>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0,
                                                      ev1);
    else if (mode == MODE_D2P && aux.d2p_bf16)
        launch_step_k<TX, RY, PD, BC, MODE_D2P, NT, false, true>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux,
                                                                 s, ev0, ev1);
    else if (mode == MODE_D2P)
        launch_step_k<TX, RY, PD, BC, MODE_D2P, NT>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else if (aux.d2p_bf16)
        launch_step_k<TX, RY, PD, BC, MODE_IMAGE, NT, false, true>(grid, tiles, ntiles, per_xcd, shots, parity, cf,
                                                                   aux, s, ev0, ev1);
    else
        launch_step_k<TX, RY, PD, BC, MODE_IMAGE, NT>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0,
                                                      ev1);
    return hipGetLastError();
}

template <int TX, int RY, int NT>
static hipError_t launch_step_t(int pd, int bc, int mode, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd,
                                const ShotDev* shots, int parity, const Coefs& cf, const StepAux& aux,
                                hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    // CPML: launch_cpml has written the layer corrections of this step
#define MM_BC(PD_, BC_) \
    return launch_step_bc<TX, RY, PD_, BC_, NT>(mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1)
    if constexpr (NT == 256) {
        if (pd == 2) {
            if (bc == 1) MM_BC(2, 1);
            if (bc == 2) MM_BC(2, 2);
            MM_BC(2, 0);
        }
    }
    if (pd != 1) return hipErrorInvalidValue;
    if (bc == 1) MM_BC(1, 1);
    if (bc == 2) MM_BC(1, 2);
    MM_BC(1, 0);
#undef MM_BC
}

hipError_t launch_step(int variant, int bc, int mode, const TileEnt* tiles, int ntiles, const ShotDev* shots,
                       int parity, const Coefs& cf, const StepAux& aux, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ntiles <= 0) return hipSuccess;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grid(8 * per_xcd + aux.gather_blocks);
    const TileShape& ts = kTiles[variant];
#define MM_T(TX_, RY_, NT_) \
    return launch_step_t<TX_, RY_, NT_>(ts.pd, bc, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, \
                                        ev1)
    if (ts.nt == 1024) {
        if (ts.tx == 64) {
            if (ts.ry == 1) MM_T(64, 1, 1024);
            if (ts.ry == 2) MM_T(64, 2, 1024);
        } else if (ts.ry == 1) {
            MM_T(32, 1, 1024);
        }
        return hipErrorInvalidValue;
    }
    if (ts.nt == 512) {
        if (ts.tx == 64) {
            if (ts.ry == 2) MM_T(64, 2, 512);
            if (ts.ry == 4) MM_T(64, 4, 512);
        } else if (ts.ry == 2) {
            MM_T(32, 2, 512);
        }
        return hipErrorInvalidValue;
    }
    if (ts.tx == 64) {
        if (ts.ry == 2) MM_T(64, 2, 256);
        if (ts.ry == 4) MM_T(64, 4, 256);
        MM_T(64, 8, 256);
    }
    if (ts.ry == 1) MM_T(32, 1, 256);
    if (ts.ry == 2) MM_T(32, 2, 256);
    MM_T(32, 4, 256);
#undef MM_T
}

// ------------------------------------------------------ CPML, fused step
//
// Time step of the tiles that meet a CPML layer, with the memory update of
// every damped axis done in the same pass (no correction arrays written and
// read back).  Per damped axis a and layer cell,
//   psi_a^{n+1} = b_a psi_a^n + a_a D1_a p^n,
//   zeta_a^{n+1} = b_a zeta_a^n + a_a (D2_a p^n + D1_a psi_a^{n+1}),
// and the cell's Laplacian gains D1_a psi_a^{n+1} + zeta_a^{n+1}.  D1 of
// psi^{n+1} reaches 8 cells of p^n, so:
//  - x and y: the staged plane carries 8-cell halos (tiles flagged TF_LX /
//    TF_LY), psi^{n+1} is formed over the tile and 4 cells around it into
//    LDS (the outer ring redundantly with the neighbouring tile, from the
//    same p^n and psi^n), and D1 psi is taken from there after a barrier;
//  - z (tiles flagged TF_LZ in LZ launches, whose z-chunks are exactly the
//    layers [0, nb) and [nz - nb, nz)): the register queue holds planes
//    z-4 .. z+8, psi_z^{n+1} of plane z+4 is formed as soon as plane z+8
//    arrives and kept in a second queue of planes z-4 .. z+4 (zero outside
//    the chunk, which is outside the layer).  Other tiles of an LZ launch
//    (the frame, when one launch takes every kind) use the same deeper
//    queue without the z memory.
// psi is double-buffered by step parity (current in ShotDev::psi at even
// steps and in ShotDev::psi2 at odd ones, the next in the other), so the
// ring of a tile reads psi^n while its owner writes psi^{n+1}; zeta is
// updated in place by the owner only.  Cells owned by the tile are
// [x0, x1) x [y0, y1) x [z0, z1); the plane is staged over the full TX x TY
// so the ring around the owned cells holds real p^n values.
template <int TX, int RY, int NT, int PD, bool XY, bool LZ, int MODE, bool STREAM, bool BF>
__global__ __launch_bounds__(NT) void k_cstep(const TileEnt* __restrict__ tiles, int ntiles, int per_xcd,
                                              const ShotDev* __restrict__ shots, int parity, Coefs cf,
                                              StepAux aux) {
    constexpr int BY = NT / TX;  // thread rows
    constexpr int TY = BY * RY;
    constexpr int H = 8;  // halo of the staged plane
    constexpr int LW = TX + 2 * H;
    constexpr int QD = LZ ? 13 : 9;             // z queue: planes z-4 .. z+QD-5
    constexpr int YH = BY >= 16 ? 1 : 16 / BY;  // plane halo rows per thread row (16 in all)
    constexpr int PH = BY >= 8 ? 1 : 8 / BY;    // psi_y ring rows per thread row (8 in all)
    static_assert(TX >= 16 && (BY >= 16 || 16 % BY == 0), "halo split");
    __shared__ float lds[2][TY + 2 * H][LW];
    __shared__ float psx[TY][TX + 8];  // psi_x^{n+1}: tile rows, columns x0-4 .. x0+TX+3
    __shared__ float psy[TY + 8][TX];  // psi_y^{n+1}: tile columns, rows y0-4 .. y0+TY+3

    if ((int)blockIdx.x < aux.gather_blocks) {
        // record of the previous step: its output is this step's p^n (256 receivers per block)
        const int tid = threadIdx.y * TX + threadIdx.x;
        const int r = blockIdx.x * 256 + tid;
        if (tid < 256 && r < aux.g_n) aux.gather_out[r] = shots[aux.g_shot[r]].buf[parity][aux.g_off[r]];
        return;
    }
    const int b = blockIdx.x - aux.gather_blocks;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    const TileEnt te = tiles[t];
    const ShotDev& sd = shots[te.shot];
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb;
    const long long plane = (long long)nx * ny;
    const float* __restrict__ pc = sd.buf[parity];
    float* __restrict__ pn = sd.buf[parity ^ 1];
    const float* __restrict__ vd = sd.vdt2;
    const float* __restrict__ prof = sd.prof;  // a_x b_x [nx], a_y b_y [ny], a_z b_z [nz]
    const float* __restrict__ rpx = parity ? sd.psi2[0] : sd.psi[0];
    const float* __restrict__ rpy = parity ? sd.psi2[1] : sd.psi[1];
    const float* __restrict__ rpz = parity ? sd.psi2[2] : sd.psi[2];
    float* __restrict__ wpx = parity ? sd.psi[0] : sd.psi2[0];
    float* __restrict__ wpy = parity ? sd.psi[1] : sd.psi2[1];
    float* __restrict__ wpz = parity ? sd.psi[2] : sd.psi2[2];
    const long long pxs = (long long)ny * nb2, pys = (long long)nb2 * nx;  // slab planes of x and y

    // x / y layers only in the XY instantiations (the z-layer tiles away from the x and y faces
    // run without that machinery, and its registers), the z layer only in the LZ ones; within an
    // instantiation the tile's flags decide (a launch may mix frame and z-layer tiles)
    const bool tlx = XY && (te.flags & TF_LX) != 0, tly = XY && (te.flags & TF_LY) != 0;
    const bool lz = LZ && (te.flags & TF_LZ) != 0;
    const bool wide = tlx || tly;  // block-uniform
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x = te.x0 + tx;
    const bool xin = x < nx;
    int row[RY];
    bool in[RY], own[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = te.y0 + ty + r * BY;
        in[r] = xin && row[r] < ny;
        own[r] = x < te.x1 && row[r] < te.y1;
    }
    // plane halo: lanes 0..15 carry columns x0-8 .. x0-1 and x0+TX .. x0+TX+7, thread rows the
    // 16 rows y0-8 .. y0-1 and y0+TY .. y0+TY+7 (the outer 4 of each side only on wide tiles)
    const int hcol = tx < 8 ? te.x0 - 8 + tx : te.x0 + TX + (tx - 8);
    const bool hx_lane = tx < 16 && (wide || (tx >= 4 && tx < 12)) && hcol >= 0 && hcol < nx;
    const bool hy_row = BY <= 16 || ty < 16;  // wave-uniform
    unsigned voc[RY], vox[RY], voy[YH];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        voc[r] = in[r] ? (unsigned)(row[r] * nx + x) * 4u : OOB;
        vox[r] = (hx_lane && row[r] < ny) ? (unsigned)(row[r] * nx + hcol) * 4u : OOB;
    }
#pragma unroll
    for (int h = 0; h < YH; ++h) {
        const int hr = ty + h * BY;
        const int y = hr < 8 ? te.y0 - 8 + hr : te.y0 + TY + (hr - 8);
        const bool ok = hy_row && hr < 16 && (wide || (hr >= 4 && hr < 12)) && xin && y >= 0 && y < ny;
        voy[h] = ok ? (unsigned)(y * nx + x) * 4u : OOB;
    }
    // x layer: this thread's column, and (lanes 0..7) the psi_x ring columns x0-4 .. x0-1, x0+TX .. x0+TX+3
    const bool xl = tlx && xin && (x < nb || x >= nx - nb);
    const float axc = xl ? prof[x] : 0.0f, bxc = xl ? prof[nx + x] : 0.0f;
    const int pcol = tx < 4 ? te.x0 - 4 + tx : te.x0 + TX + (tx - 4);
    const bool pxl = tlx && tx < 8 && pcol >= 0 && pcol < nx && (pcol < nb || pcol >= nx - nb);
    const float apx = pxl ? prof[pcol] : 0.0f, bpx = pxl ? prof[nx + pcol] : 0.0f;
    unsigned vsx[RY], vpx[RY], vsy[RY];
    bool yl[RY];
    float ayc[RY], byc[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        const int y = row[r];
        vsx[r] = (xl && y < ny) ? (unsigned)(y * nb2 + (x < nb ? x : x - (nx - nb2))) * 4u : OOB;
        vpx[r] = (pxl && y < ny) ? (unsigned)(y * nb2 + (pcol < nb ? pcol : pcol - (nx - nb2))) * 4u : OOB;
        yl[r] = tly && in[r] && (y < nb || y >= ny - nb);
        vsy[r] = yl[r] ? (unsigned)((y < nb ? y : y - (ny - nb2)) * nx + x) * 4u : OOB;
        ayc[r] = yl[r] ? prof[2 * nx + y] : 0.0f;
        byc[r] = yl[r] ? prof[2 * nx + ny + y] : 0.0f;
    }
    // y layer: the psi_y ring rows y0-4 .. y0-1 and y0+TY .. y0+TY+3 (thread row ty takes ty, ty + BY, ... < 8)
    unsigned vpy[PH];
    float apy[PH], bpy[PH];
#pragma unroll
    for (int h = 0; h < PH; ++h) {
        const int hr = ty + h * BY;
        const int y = hr < 4 ? te.y0 - 4 + hr : te.y0 + TY + (hr - 4);
        const bool ok = tly && hr < 8 && xin && y >= 0 && y < ny && (y < nb || y >= ny - nb);
        vpy[h] = ok ? (unsigned)((y < nb ? y : y - (ny - nb2)) * nx + x) * 4u : OOB;
        apy[h] = ok ? prof[2 * nx + y] : 0.0f;
        bpy[h] = ok ? prof[2 * nx + ny + y] : 0.0f;
    }
    const float* __restrict__ zprof = prof + 2 * nx + 2 * ny;  // a_z [nz], b_z [nz]

    const int z0 = te.z0, z1 = te.z1;
    float q[RY][QD];
#pragma unroll
    for (int m = 0; m < QD - 1; ++m) {
        const int z = z0 - 4 + m;
        const bool zin = z >= 0 && z < nz;  // block-uniform
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(pc, zin ? z : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][m] = zin ? bload(rp, voc[r]) : 0.0f;
    }
    if (!lz && z0 == 0 && sd.fs) {
        // above a free surface on plane 0: the odd mirror, planes -1..-4 = -p(1..4)
        const __amdgpu_buffer_rsrc_t r4 = plane_rsrc(pc, 4 < nz ? 4 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][3] = -q[r][5];
            q[r][2] = -q[r][6];
            q[r][1] = -q[r][7];
            q[r][0] = 4 < nz ? -bload(r4, voc[r]) : 0.0f;
        }
    }
    auto zslab = [&](int z) { return z < nb ? z : z - (nz - nb2); };
    // psi_z^{n+1} of planes z-4 .. z+4 (LZ): the planes before the chunk are outside the layer
    float ps[LZ ? RY : 1][9];
    if (lz) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int m = 0; m < 9; ++m) ps[r][m] = 0.0f;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int zz = z0 + j;
            if (zz < z1) {
                const __amdgpu_buffer_rsrc_t ro = plane_rsrc(rpz, zslab(zz), plane);
                const float az = zprof[zz], bz = zprof[nz + zz];
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    float d1 = 0.0f;
#pragma unroll
                    for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bz[m - 1], q[r][4 + j + m] - q[r][4 + j - m], d1);
                    const float v = fmaf(bz, bload(ro, voc[r]), az * d1);
                    ps[r][4 + j] = v;
                    if (own[r]) put<STREAM>(&((gfloat*)wpz)[(long long)zslab(zz) * plane + (row[r] * nx + x)], v);
                }
            }
        }
    }

    // prefetch stage for plane zn (PD planes in flight): queue head p^n(zn+QD-5), p^{n-1},
    // (dt v)^2, the plane halos, psi^n and zeta^n of the cell (x, y: plane zn; z: psi of plane
    // zn+4, zeta of zn), psi^n of the rings
    struct Stage {
        float q[RY], pp[RY], vd[RY], xh[RY], yh[YH];
        float sx[RY], zx[RY], hx[RY], sy[RY], zy[RY], hy[PH], sz[RY], zz[RY];
    };
    auto fetch = [&](Stage& f, int zn) {
        const int zq = zn + QD - 5;
        const bool hin = zq < nz;
        const __amdgpu_buffer_rsrc_t rh = plane_rsrc(pc, hin ? zq : 0, plane);
        const __amdgpu_buffer_rsrc_t rc = plane_rsrc(pc, zn, plane);
        const __amdgpu_buffer_rsrc_t rm = plane_rsrc(pn, zn, plane);
        const __amdgpu_buffer_rsrc_t rv = plane_rsrc(vd, zn, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            f.q[r] = hin ? bload(rh, voc[r]) : 0.0f;
            f.pp[r] = STREAM ? bload_nt(rm, voc[r]) : bload(rm, voc[r]);
            f.vd[r] = STREAM ? bload_nt(rv, voc[r]) : bload(rv, voc[r]);
            f.xh[r] = bload(rc, vox[r]);
            f.sx[r] = f.zx[r] = f.hx[r] = f.sy[r] = f.zy[r] = f.sz[r] = f.zz[r] = 0.0f;
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) f.yh[h] = bload(rc, voy[h]);
#pragma unroll
        for (int h = 0; h < PH; ++h) f.hy[h] = 0.0f;
        if (tlx) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(rpx, zn, pxs);
            const __amdgpu_buffer_rsrc_t rz = plane_rsrc(sd.zeta[0], zn, pxs);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                f.sx[r] = STREAM ? bload_nt(rs, vsx[r]) : bload(rs, vsx[r]);
                f.zx[r] = STREAM ? bload_nt(rz, vsx[r]) : bload(rz, vsx[r]);
                f.hx[r] = bload(rs, vpx[r]);
            }
        }
        if (tly) {
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(rpy, zn, pys);
            const __amdgpu_buffer_rsrc_t rz = plane_rsrc(sd.zeta[1], zn, pys);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                f.sy[r] = STREAM ? bload_nt(rs, vsy[r]) : bload(rs, vsy[r]);
                f.zy[r] = STREAM ? bload_nt(rz, vsy[r]) : bload(rz, vsy[r]);
            }
#pragma unroll
            for (int h = 0; h < PH; ++h) f.hy[h] = bload(rs, vpy[h]);
        }
        if (lz) {
            const bool pin = zn + 4 < z1;  // the chunk is the whole layer
            const __amdgpu_buffer_rsrc_t rs = plane_rsrc(rpz, pin ? zslab(zn + 4) : 0, plane);
            const __amdgpu_buffer_rsrc_t rz = plane_rsrc(sd.zeta[2], zslab(zn), plane);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                f.sz[r] = pin ? (STREAM ? bload_nt(rs, voc[r]) : bload(rs, voc[r])) : 0.0f;
                f.zz[r] = STREAM ? bload_nt(rz, voc[r]) : bload(rz, voc[r]);
            }
        }
    };
    Stage stg[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k)
        if (z0 + k < z1) fetch(stg[k], z0 + k);

    const int xx = H + tx;
    gfloat* __restrict__ pn_g = (gfloat*)pn;
    for (int z = z0; z < z1; ++z) {
        const Stage cur = stg[0];
#pragma unroll
        for (int k = 0; k + 1 < PD; ++k) stg[k] = stg[k + 1];
        if (z + PD < z1) fetch(stg[PD - 1], z + PD);
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][QD - 1] = cur.q[r];
        const float *cpp = cur.pp, *cvd = cur.vd, *cxh = cur.xh, *cyh = cur.yh, *csx = cur.sx, *czx = cur.zx,
                    *chx = cur.hx, *csy = cur.sy, *czy = cur.zy, *chy = cur.hy, *csz = cur.sz, *czz = cur.zz;

        if (lz) {
            // psi_z^{n+1} of plane z+4: its D1 needs planes z .. z+8, now all in the queue
            const int zp = z + 4;
            if (zp < z1) {
                const float az = zprof[zp], bz = zprof[nz + zp];
                const long long so = (long long)zslab(zp) * plane;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    float d1 = 0.0f;
#pragma unroll
                    for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bz[m - 1], q[r][8 + m] - q[r][8 - m], d1);
                    const float v = fmaf(bz, csz[r], az * d1);
                    ps[r][8] = v;
                    if (own[r]) put<STREAM>(&((gfloat*)wpz)[so + (row[r] * nx + x)], v);
                }
            } else {
#pragma unroll
                for (int r = 0; r < RY; ++r) ps[r][8] = 0.0f;
            }
        }

        float(*L)[LW] = lds[z & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            L[H + ty + r * BY][xx] = q[r][4];
            if (tx < 16) L[H + ty + r * BY][tx < 8 ? tx : TX + tx] = cxh[r];
        }
        if (hy_row) {
#pragma unroll
            for (int h = 0; h < YH; ++h) {
                const int hr = ty + h * BY;
                if (hr < 16) L[hr < 8 ? hr : TY + hr][xx] = cyh[h];
            }
        }
        __syncthreads();

        if (wide) {
            if (tlx) {
                const long long so = (long long)z * pxs;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int yy = H + ty + r * BY;
                    float v = 0.0f;
                    if (xl && in[r]) {
                        float d1 = 0.0f;
#pragma unroll
                        for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bx[m - 1], L[yy][xx + m] - L[yy][xx - m], d1);
                        v = fmaf(bxc, csx[r], axc * d1);
                        if (own[r]) put<STREAM>(&((gfloat*)wpx)[so + (vsx[r] >> 2)], v);
                    }
                    psx[ty + r * BY][4 + tx] = v;
                    if (tx < 8) {
                        float w = 0.0f;
                        if (pxl && row[r] < ny) {
                            const int cc = tx < 4 ? H - 4 + tx : H + TX + (tx - 4);
                            float d1 = 0.0f;
#pragma unroll
                            for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bx[m - 1], L[yy][cc + m] - L[yy][cc - m], d1);
                            w = fmaf(bpx, chx[r], apx * d1);
                        }
                        psx[ty + r * BY][tx < 4 ? tx : TX + tx] = w;
                    }
                }
            }
            if (tly) {
                const long long so = (long long)z * pys;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int yy = H + ty + r * BY;
                    float v = 0.0f;
                    if (yl[r]) {
                        float d1 = 0.0f;
#pragma unroll
                        for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.by[m - 1], L[yy + m][xx] - L[yy - m][xx], d1);
                        v = fmaf(byc[r], csy[r], ayc[r] * d1);
                        if (own[r]) put<STREAM>(&((gfloat*)wpy)[so + (vsy[r] >> 2)], v);
                    }
                    psy[4 + ty + r * BY][tx] = v;
                }
#pragma unroll
                for (int h = 0; h < PH; ++h) {
                    const int hr = ty + h * BY;
                    if (hr < 8) {
                        float w = 0.0f;
                        if (vpy[h] != OOB) {
                            const int lr = hr < 4 ? H - 4 + hr : H + TY + (hr - 4);
                            float d1 = 0.0f;
#pragma unroll
                            for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.by[m - 1], L[lr + m][xx] - L[lr - m][xx], d1);
                            w = fmaf(bpy[h], chy[h], apy[h] * d1);
                        }
                        psy[hr < 4 ? hr : TY + hr][tx] = w;
                    }
                }
            }
            __syncthreads();
        }

        const long long zoff = (long long)z * plane;
        const float az = lz ? zprof[z] : 0.0f, bz = lz ? zprof[nz + z] : 0.0f;
        const long long zso = lz ? (long long)zslab(z) * plane : 0;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yy = H + ty + r * BY;
            const float c = q[r][4];
            float lx = 0.0f, ly = 0.0f, lzv = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                lx = fmaf(cf.cx[m - 1], (L[yy][xx + m] - c) + (L[yy][xx - m] - c), lx);
                ly = fmaf(cf.cy[m - 1], (L[yy + m][xx] - c) + (L[yy - m][xx] - c), ly);
                lzv = fmaf(cf.cz[m - 1], (q[r][4 + m] - c) + (q[r][4 - m] - c), lzv);
            }
            float lap = (lx + ly) + lzv;
            float cx = 0.0f, cy = 0.0f, cz = 0.0f;
            bool layer = false;
            if (tlx && xl && in[r]) {
                const int pr = ty + r * BY;
                float d1 = 0.0f;
#pragma unroll
                for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bx[m - 1], psx[pr][4 + tx + m] - psx[pr][4 + tx - m], d1);
                const float zn = fmaf(bxc, czx[r], axc * (lx + d1));
                if (own[r]) put<STREAM>(&((gfloat*)sd.zeta[0])[(long long)z * pxs + (vsx[r] >> 2)], zn);
                cx = d1 + zn;
                layer = true;
            }
            if (tly && yl[r]) {
                const int pr = 4 + ty + r * BY;
                float d1 = 0.0f;
#pragma unroll
                for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.by[m - 1], psy[pr + m][tx] - psy[pr - m][tx], d1);
                const float zn = fmaf(byc[r], czy[r], ayc[r] * (ly + d1));
                if (own[r]) put<STREAM>(&((gfloat*)sd.zeta[1])[(long long)z * pys + (vsy[r] >> 2)], zn);
                cy = d1 + zn;
                layer = true;
            }
            if (lz && in[r]) {
                float d1 = 0.0f;
#pragma unroll
                for (int m = 1; m <= 4; ++m) d1 = fmaf(cf.bz[m - 1], ps[r][4 + m] - ps[r][4 - m], d1);
                const float zn = fmaf(bz, czz[r], az * (lzv + d1));
                if (own[r]) put<STREAM>(&((gfloat*)sd.zeta[2])[zso + (row[r] * nx + x)], zn);
                cz = d1 + zn;
                layer = true;
            }
            if (layer) lap += (cx + cy) + cz;
            if (own[r]) {
                const long long o = zoff + (row[r] * nx + x);
                if ((te.flags & TF_SRC) && aux.wrow) {
#pragma unroll
                    for (int k = 0; k < MAX_INLINE_SRC; ++k)
                        if (k < sd.nsrc_in && o == sd.src_off[k]) lap = fmaf(aux.src_scale, aux.wrow[sd.src_col[k]], lap);
                }
                const float out = c + fmaf(cvd[r], lap, c - cpp[r]);
                put<STREAM>(&pn_g[o], out);
                if (MODE == MODE_D2P) d2p_put<BF>(aux.d2p_out, o, cvd[r] * lap);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
#pragma unroll
            for (int m = 0; m < QD - 1; ++m) q[r][m] = q[r][m + 1];
            if (lz) {
#pragma unroll
                for (int m = 0; m < 8; ++m) ps[r][m] = ps[r][m + 1];
            }
        }
    }
}

// shape of the fused CPML kernel: 512 threads, loads two planes ahead; 32-wide tiles of one row
// per thread where the x / y machinery runs (its 8-cell halos and rings), 64 x 16 tiles for the
// z-layer chunks away from the x / y faces (their 4-cell halos cost half as much of a row:
// 461 against 490 us per step at 1024^2 x 512)
constexpr int CS_NT = 512, CS_PD = 2;
constexpr int CS_TX = 32, CS_RY = 1;        // frame and corners (and CS_ALL)
constexpr int CS_ZL_TX = 64, CS_ZL_RY = 2;  // z-layer chunks (CS_ZLAYER)
template <bool XY, bool LZ>
constexpr int cs_tx() { return (LZ && !XY) ? CS_ZL_TX : CS_TX; }
template <bool XY, bool LZ>
constexpr int cs_ry() { return (LZ && !XY) ? CS_ZL_RY : CS_RY; }
int cstep_tile_w(int kind) { return kind == CS_ZLAYER ? CS_ZL_TX : CS_TX; }
int cstep_tile_h(int kind) { return kind == CS_ZLAYER ? (CS_NT / CS_ZL_TX) * CS_ZL_RY : (CS_NT / CS_TX) * CS_RY; }

template <bool XY, bool LZ, int MODE, bool STREAM, bool BF = false>
static void launch_cstep_k(dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd, const ShotDev* shots, int parity,
                           const Coefs& cf, const StepAux& aux, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int TX = cs_tx<XY, LZ>(), RY = cs_ry<XY, LZ>();
    const dim3 block(TX, CS_NT / TX);
    hipExtLaunchKernelGGL(k_cstep<TX, RY, CS_NT, CS_PD, XY, LZ, MODE, STREAM, BF>, grid, block, 0, s, ev0, ev1, 0,
                          tiles, ntiles, per_xcd, shots, parity, cf, aux);
}

template <bool XY, bool LZ>
static void launch_cstep_m(int mode, bool st, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd,
                           const ShotDev* shots, int parity, const Coefs& cf, const StepAux& aux, hipStream_t s,
                           hipEvent_t ev0, hipEvent_t ev1) {
    if (mode == MODE_D2P && aux.d2p_bf16)
        launch_cstep_k<XY, LZ, MODE_D2P, false, true>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0,
                                                      ev1);
    else if (mode == MODE_D2P)
        launch_cstep_k<XY, LZ, MODE_D2P, false>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else if (st)
        launch_cstep_k<XY, LZ, MODE_PLAIN, true>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else
        launch_cstep_k<XY, LZ, MODE_PLAIN, false>(grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
}

hipError_t launch_cpml_step(int kind, int mode, const TileEnt* tiles, int ntiles, const ShotDev* shots, int parity,
                            const Coefs& cf, const StepAux& aux, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ntiles <= 0) return hipSuccess;
    if (mode != MODE_PLAIN && mode != MODE_D2P) return hipErrorInvalidValue;
    const int per_xcd = (ntiles + 7) / 8;
    const dim3 grid(8 * per_xcd + aux.gather_blocks);
    const bool st = aux.stream_loads != 0 && mode == MODE_PLAIN;
    if (kind == CS_FRAME)
        launch_cstep_m<true, false>(mode, st, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else if (kind == CS_ZLAYER)
        launch_cstep_m<false, true>(mode, st, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else if (kind == CS_ZCORNER || kind == CS_ALL)
        launch_cstep_m<true, true>(mode, st, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s, ev0, ev1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------ acoustic_iso
//
// The first-order variable-density system (paper, Eq. (acoustic_iso_vd)) on
// the staggered grid, two z-marching kernels per step over the stencil
// kernel's tile table:
//   k_iso_u:  u_a^{n+1/2} = G (u_a^{n-1/2} + (dt b_a) D+_a p^n),  a = x, y, z,
//   k_iso_p:  p^{n+1} = G (p^n + (dt rho v^2) (D-_x u_x + D-_y u_y + D-_z u_z)),
// with the order-8 staggered differences D+ p (face i+1/2) = sum_m c_m
// (p(i+m) - p(i+1-m)) / h and D- u (cell i) = sum_m c_m (u(i+m-1) - u(i-m)) / h
// (index i of u_x is the face i+1/2), zero outside the grid.  p^n lives in
// LDS (x / y neighbours) and a register queue (z); in k_iso_p, u_x and u_y
// are staged in LDS with their x / y halos and u_z in a register queue.
// Sources are added to p^{n+1} by k_inject (dt rho v^2 s).  The face
// buoyancy is formed on the fly from rho / dt of the two cells beside the
// face: dt b = 2 / (rho_0 / dt + rho_1 / dt), one over their mean density
// (the inner cell's dt / rho on the last face of an axis).

// acoustic_iso CPML memory of one thread's cells (FACE = 0: psi_u of D- u at the
// cells, in ShotDev::zeta) or faces (FACE = 1: psi_p of D+ p at the faces,
// in ShotDev::psi): slab arrays of W = nb + 1 cells per end (x [nz][ny][2W],
// y [nz][2W][nx], z [2W][ny][nx], slab index s < W is grid index s, else
// n - 2W + s); (a, b) per axis from the shot's tables (cells first, then
// faces: 2 (nx + ny + nz) floats each).  Outside the layers a = 0, b = 1, so
// the memory of the slab cells next to a layer stays zero.
template <int RY, bool FACE>
struct IsoPml {
    bool xl, yl[RY];
    float ax, bx, ay[RY], by[RY];
    unsigned vx[RY], vy[RY];
    const float* tab;  // the z columns of the tables: a_z [nz], b_z [nz]
    int W;
    __device__ void init(const ShotDev& sd, const TileEnt& te, int x, const int* row, const bool* in) {
        const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
        W = sd.nb + 1;
        const int W2 = 2 * W;
        const float* t0 = sd.prof + (FACE ? 2 * (nx + ny + nz) : 0);
        tab = t0 + 2 * nx + 2 * ny;
        xl = (te.flags & TF_LX) && x < nx && (x < W || x >= nx - W);
        ax = xl ? t0[x] : 0.0f;
        bx = xl ? t0[nx + x] : 1.0f;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int y = row[r];
            vx[r] = (xl && in[r]) ? (unsigned)(y * W2 + (x < W ? x : x - (nx - W2))) * 4u : OOB;
            yl[r] = (te.flags & TF_LY) && in[r] && (y < W || y >= ny - W);
            vy[r] = yl[r] ? (unsigned)((y < W ? y : y - (ny - W2)) * nx + x) * 4u : OOB;
            ay[r] = yl[r] ? t0[2 * nx + y] : 0.0f;
            by[r] = yl[r] ? t0[2 * nx + ny + y] : 1.0f;
        }
        (void)nz;
    }
    // plane z of the z-axis memory holds layer cells (block-uniform)
    __device__ bool zl(const ShotDev& sd, const TileEnt& te, int z) const {
        return (te.flags & TF_LZ) && (z < W || z >= sd.nz - W);
    }
    __device__ int zs(const ShotDev& sd, int z) const { return z < W ? z : z - (sd.nz - 2 * W); }
};

template <int TX, int RY>
struct IsoTile {
    static constexpr int BY = 256 / TX, TY = BY * RY, YH = 8 / BY;
};

template <int TX, int RY, int BC>
__global__ __launch_bounds__(256) void k_iso_u(const TileEnt* __restrict__ tiles, int ntiles, int per_xcd,
                                               const ShotDev* __restrict__ shots, int parity, Coefs cf) {
    constexpr int BY = IsoTile<TX, RY>::BY, TY = IsoTile<TX, RY>::TY, YH = IsoTile<TX, RY>::YH;
    constexpr int LW = TX + 8;
    constexpr bool SPONGE = BC == 1;
    constexpr bool CPML = BC == 2;
    __shared__ float lds[2][TY + 8][LW];  // p^n of the plane with halos
    __shared__ float ldb[2][TY + 8][LW];  // rho / dt of the plane with halos (face buoyancy)
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    const TileEnt te = tiles[t];
    const ShotDev& sd = shots[te.shot];
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const long long plane = (long long)nx * ny;
    const float* __restrict__ pc = sd.buf[parity];
    const float* __restrict__ bd = sd.rdt;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x = te.x0 + tx;
    const bool xin = x < nx;
    const bool xlast = x + 1 >= nx;  // the last x face takes the inner cell's buoyancy
    int row[RY];
    bool in[RY];
    unsigned voc[RY], vox[RY], voy[YH];
    const int hcol = tx < 4 ? te.x0 - 4 + tx : te.x0 + TX + (tx - 4);
    const bool hx_lane = tx < 8 && hcol >= 0 && hcol < nx;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = te.y0 + ty + r * BY;
        in[r] = xin && row[r] < ny;
        voc[r] = in[r] ? (unsigned)(row[r] * nx + x) * 4u : OOB;
        vox[r] = (hx_lane && row[r] < ny) ? (unsigned)(row[r] * nx + hcol) * 4u : OOB;
    }
#pragma unroll
    for (int h = 0; h < YH; ++h) {
        const int hr = ty + h * BY;
        const int y = hr < 4 ? te.y0 - 4 + hr : te.y0 + TY + (hr - 4);
        voy[h] = (xin && y >= 0 && y < ny) ? (unsigned)(y * nx + x) * 4u : OOB;
    }
    float gx = 1.0f, gyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) gyv[r] = 1.0f;
    if (SPONGE) {
        gx = xin ? sd.prof[x] : 1.0f;
#pragma unroll
        for (int r = 0; r < RY; ++r) gyv[r] = in[r] ? sd.prof[nx + row[r]] : 1.0f;
    }
    IsoPml<RY, true> pm;  // CPML: memory of D+ p at this thread's faces
    if (CPML) pm.init(sd, te, x, row, in);
    const long long pxs = CPML ? (long long)ny * 2 * pm.W : 0, pys = CPML ? (long long)2 * pm.W * nx : 0;
    const int z0 = te.z0, z1 = te.z1;
    // p queue: planes z-4 .. z+4 (D+ at the face z+1/2 uses z-3 .. z+4); buoyancy of planes z, z+1
    float q[RY][9], b0[RY], b1[RY];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int z = z0 - 4 + m;
        const bool zin = z >= 0 && z < nz;
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(pc, zin ? z : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) q[r][m] = zin ? bload(rp, voc[r]) : 0.0f;
    }
    {
        const __amdgpu_buffer_rsrc_t rb = plane_rsrc(bd, z0 < nz ? z0 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) b1[r] = bload(rb, voc[r]);
    }
    if (z0 == 0 && sd.fs) {
        // free surface: p is odd about the plane z = 0 (p(0) = 0), so planes -4 .. -1 hold
        // -p(4) .. -p(1) (block-uniform branch)
        const __amdgpu_buffer_rsrc_t r4 = plane_rsrc(pc, 4 < nz ? 4 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][3] = -q[r][5];
            q[r][2] = -q[r][6];
            q[r][1] = -q[r][7];
            q[r][0] = 4 < nz ? -bload(r4, voc[r]) : 0.0f;
        }
    }
    // stage for plane zn: p^n(zn+4), halos of p and rho/dt at zn, rho/dt(zn+1), u at zn
    float nq[RY], nxh[RY], nyh[YH], nbh[RY], nbx[RY], nby[YH], nu[3][RY];
    float nm[CPML ? 3 : 1][RY];  // CPML memory of the three face derivatives at plane zn
    auto fetch = [&](int zn) {
        if (CPML) {
            const __amdgpu_buffer_rsrc_t mx = plane_rsrc(sd.psi[0], zn, pxs);
            const __amdgpu_buffer_rsrc_t my = plane_rsrc(sd.psi[1], zn, pys);
            const bool zl = pm.zl(sd, te, zn);
            const __amdgpu_buffer_rsrc_t mz = plane_rsrc(sd.psi[2], zl ? pm.zs(sd, zn) : 0, plane);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                nm[0][r] = bload(mx, pm.vx[r]);
                nm[CPML ? 1 : 0][r] = bload(my, pm.vy[r]);
                nm[CPML ? 2 : 0][r] = zl ? bload(mz, voc[r]) : 0.0f;
            }
        }
        const bool hin = zn + 4 < nz, bin = zn + 1 < nz;
        const __amdgpu_buffer_rsrc_t rh = plane_rsrc(pc, hin ? zn + 4 : 0, plane);
        const __amdgpu_buffer_rsrc_t rc = plane_rsrc(pc, zn, plane);
        const __amdgpu_buffer_rsrc_t rbc = plane_rsrc(bd, zn, plane);
        const __amdgpu_buffer_rsrc_t rbn = plane_rsrc(bd, bin ? zn + 1 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            nq[r] = hin ? bload(rh, voc[r]) : 0.0f;
            nxh[r] = bload(rc, vox[r]);
            nbx[r] = bload(rbc, vox[r]);
            nbh[r] = bin ? bload(rbn, voc[r]) : 0.0f;
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            nyh[h] = bload(rc, voy[h]);
            nby[h] = bload(rbc, voy[h]);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const __amdgpu_buffer_rsrc_t ru = plane_rsrc(sd.u[a], zn, plane);
#pragma unroll
            for (int r = 0; r < RY; ++r) nu[a][r] = bload(ru, voc[r]);
        }
    };
    if (z0 < z1) fetch(z0);
    const int xx = 4 + tx;
    for (int z = z0; z < z1; ++z) {
        float cu[3][RY], cxh[RY], cyh[YH], cbx[RY], cby[YH], cm[CPML ? 3 : 1][RY];
        if (CPML) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int r = 0; r < RY; ++r) cm[CPML ? a : 0][r] = nm[CPML ? a : 0][r];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][8] = nq[r];
            cxh[r] = nxh[r];
            cbx[r] = nbx[r];
            b0[r] = b1[r];
            b1[r] = nbh[r];
#pragma unroll
            for (int a = 0; a < 3; ++a) cu[a][r] = nu[a][r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            cyh[h] = nyh[h];
            cby[h] = nby[h];
        }
        if (z + 1 < z1) fetch(z + 1);
        float(*L)[LW] = lds[z & 1];
        float(*B)[LW] = ldb[z & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            L[4 + ty + r * BY][xx] = q[r][4];
            B[4 + ty + r * BY][xx] = b0[r];
            if (tx < 8) {
                L[4 + ty + r * BY][tx < 4 ? tx : TX + tx] = cxh[r];
                B[4 + ty + r * BY][tx < 4 ? tx : TX + tx] = cbx[r];
            }
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int hr = ty + h * BY;
            L[hr < 4 ? hr : TY + hr][xx] = cyh[h];
            B[hr < 4 ? hr : TY + hr][xx] = cby[h];
        }
        __syncthreads();
        const float gz = SPONGE ? sd.prof[nx + ny + z] : 1.0f;
        const bool zlast = z + 1 >= nz;
        const long long zoff = (long long)z * plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yy = 4 + ty + r * BY;
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                dx = fmaf(cf.sx[m - 1], L[yy][xx + m] - L[yy][xx + 1 - m], dx);
                dy = fmaf(cf.sy[m - 1], L[yy + m][xx] - L[yy + 1 - m][xx], dy);
                dz = fmaf(cf.sz[m - 1], q[r][4 + m] - q[r][5 - m], dz);
            }
            if (in[r]) {
                const long long o = zoff + (row[r] * nx + x);
                const float G = SPONGE ? gx * gyv[r] * gz : 1.0f;
                // dt times the face buoyancy: 2 / (rho_0 / dt + rho_1 / dt), the inner cell's
                // dt / rho_0 on the last face of an axis
                const float rc = b0[r];
                const float fx = 2.0f / (rc + (xlast ? rc : B[yy][xx + 1]));
                const float fy = 2.0f / (rc + (row[r] + 1 >= ny ? rc : B[yy + 1][xx]));
                const float fz = 2.0f / (rc + (zlast ? rc : b1[r]));
                if (CPML) {
                    // psi <- b psi + a D+ p, and D+ p gains psi (faces inside the layers)
                    if (pm.xl) {
                        const float v = fmaf(pm.bx, cm[0][r], pm.ax * dx);
                        ((gfloat*)sd.psi[0])[(long long)z * pxs + (pm.vx[r] >> 2)] = v;
                        dx += v;
                    }
                    if (pm.yl[r]) {
                        const float v = fmaf(pm.by[r], cm[CPML ? 1 : 0][r], pm.ay[r] * dy);
                        ((gfloat*)sd.psi[1])[(long long)z * pys + (pm.vy[r] >> 2)] = v;
                        dy += v;
                    }
                    if (pm.zl(sd, te, z)) {
                        const float v = fmaf(pm.tab[nz + z], cm[CPML ? 2 : 0][r], pm.tab[z] * dz);
                        ((gfloat*)sd.psi[2])[(long long)pm.zs(sd, z) * plane + (row[r] * nx + x)] = v;
                        dz += v;
                    }
                }
                ((gfloat*)sd.u[0])[o] = G * fmaf(fx, dx, cu[0][r]);
                ((gfloat*)sd.u[1])[o] = G * fmaf(fy, dy, cu[1][r]);
                ((gfloat*)sd.u[2])[o] = G * fmaf(fz, dz, cu[2][r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int m = 0; m < 8; ++m) q[r][m] = q[r][m + 1];
    }
}

// STREAM: the working set exceeds the Infinity Cache, so p^n (its last read
// of the step) and dt rho v^2 (read once) are loaded with the non-temporal hint
template <int TX, int RY, int BC, bool STREAM>
__global__ __launch_bounds__(256) void k_iso_p(const TileEnt* __restrict__ tiles, int ntiles, int per_xcd,
                                               const ShotDev* __restrict__ shots, int parity, Coefs cf) {
    constexpr int BY = IsoTile<TX, RY>::BY, TY = IsoTile<TX, RY>::TY, YH = IsoTile<TX, RY>::YH;
    constexpr int LW = TX + 8;
    constexpr bool SPONGE = BC == 1;
    constexpr bool CPML = BC == 2;
    __shared__ float lx[2][TY][LW];      // u_x of the plane with its x halo
    __shared__ float ly[2][TY + 8][TX];  // u_y of the plane with its y halo
    const int b = blockIdx.x;
    const int t = (b & 7) * per_xcd + (b >> 3);
    if (t >= ntiles) return;
    const TileEnt te = tiles[t];
    const ShotDev& sd = shots[te.shot];
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz;
    const long long plane = (long long)nx * ny;
    const float* __restrict__ pc = sd.buf[parity];
    gfloat* __restrict__ pn = (gfloat*)sd.buf[parity ^ 1];
    const float* __restrict__ kd = sd.vdt2;
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int x = te.x0 + tx;
    const bool xin = x < nx;
    int row[RY];
    bool in[RY];
    unsigned voc[RY], vox[RY], voy[YH];
    const int hcol = tx < 4 ? te.x0 - 4 + tx : te.x0 + TX + (tx - 4);
    const bool hx_lane = tx < 8 && hcol >= 0 && hcol < nx;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = te.y0 + ty + r * BY;
        in[r] = xin && row[r] < ny;
        voc[r] = in[r] ? (unsigned)(row[r] * nx + x) * 4u : OOB;
        vox[r] = (hx_lane && row[r] < ny) ? (unsigned)(row[r] * nx + hcol) * 4u : OOB;
    }
#pragma unroll
    for (int h = 0; h < YH; ++h) {
        const int hr = ty + h * BY;
        const int y = hr < 4 ? te.y0 - 4 + hr : te.y0 + TY + (hr - 4);
        voy[h] = (xin && y >= 0 && y < ny) ? (unsigned)(y * nx + x) * 4u : OOB;
    }
    float gx = 1.0f, gyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) gyv[r] = 1.0f;
    if (SPONGE) {
        gx = xin ? sd.prof[x] : 1.0f;
#pragma unroll
        for (int r = 0; r < RY; ++r) gyv[r] = in[r] ? sd.prof[nx + row[r]] : 1.0f;
    }
    IsoPml<RY, false> pm;  // CPML: memory of D- u at this thread's cells
    if (CPML) pm.init(sd, te, x, row, in);
    const long long pxs = CPML ? (long long)ny * 2 * pm.W : 0, pys = CPML ? (long long)2 * pm.W * nx : 0;
    const int z0 = te.z0, z1 = te.z1;
    // u_z queue: planes z-4 .. z+3 (D- at cell z uses them all)
    float w[RY][8];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const int z = z0 - 4 + m;
        const bool zin = z >= 0 && z < nz;
        const __amdgpu_buffer_rsrc_t rp = plane_rsrc(sd.u[2], zin ? z : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) w[r][m] = zin ? bload(rp, voc[r]) : 0.0f;
    }
    if (z0 == 0 && sd.fs) {
        // free surface: u_z is even about the plane z = 0, the face -1/2 - m holding u_z of
        // the face m + 1/2 (index -1 - m mirrors index m; block-uniform branch)
        const __amdgpu_buffer_rsrc_t r3 = plane_rsrc(sd.u[2], 3 < nz ? 3 : 0, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            w[r][3] = w[r][4];
            w[r][2] = w[r][5];
            w[r][1] = w[r][6];
            w[r][0] = 3 < nz ? bload(r3, voc[r]) : 0.0f;
        }
    }
    float nw[RY], nux[RY], nuxh[RY], nuy[RY], nuyh[YH], np_[RY], nk[RY];
    float nm[CPML ? 3 : 1][RY];  // CPML memory of the three cell derivatives at plane zn
    auto fetch = [&](int zn) {
        if (CPML) {
            const __amdgpu_buffer_rsrc_t mx = plane_rsrc(sd.zeta[0], zn, pxs);
            const __amdgpu_buffer_rsrc_t my = plane_rsrc(sd.zeta[1], zn, pys);
            const bool zl = pm.zl(sd, te, zn);
            const __amdgpu_buffer_rsrc_t mz = plane_rsrc(sd.zeta[2], zl ? pm.zs(sd, zn) : 0, plane);
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                nm[0][r] = bload(mx, pm.vx[r]);
                nm[CPML ? 1 : 0][r] = bload(my, pm.vy[r]);
                nm[CPML ? 2 : 0][r] = zl ? bload(mz, voc[r]) : 0.0f;
            }
        }
        const bool hin = zn + 3 < nz;
        const __amdgpu_buffer_rsrc_t rw = plane_rsrc(sd.u[2], hin ? zn + 3 : 0, plane);
        const __amdgpu_buffer_rsrc_t rx = plane_rsrc(sd.u[0], zn, plane);
        const __amdgpu_buffer_rsrc_t ry = plane_rsrc(sd.u[1], zn, plane);
        const __amdgpu_buffer_rsrc_t rpc = plane_rsrc(pc, zn, plane);
        const __amdgpu_buffer_rsrc_t rk = plane_rsrc(kd, zn, plane);
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            nw[r] = hin ? bload(rw, voc[r]) : 0.0f;
            nux[r] = bload(rx, voc[r]);
            nuxh[r] = bload(rx, vox[r]);
            nuy[r] = bload(ry, voc[r]);
            np_[r] = STREAM ? bload_nt(rpc, voc[r]) : bload(rpc, voc[r]);
            nk[r] = STREAM ? bload_nt(rk, voc[r]) : bload(rk, voc[r]);
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) nuyh[h] = bload(ry, voy[h]);
    };
    if (z0 < z1) fetch(z0);
    const int xx = 4 + tx;
    for (int z = z0; z < z1; ++z) {
        float cux[RY], cuxh[RY], cuy[RY], cuyh[YH], cp[RY], ck[RY], cm[CPML ? 3 : 1][RY];
        if (CPML) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int r = 0; r < RY; ++r) cm[CPML ? a : 0][r] = nm[CPML ? a : 0][r];
        }
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            w[r][7] = nw[r];
            cux[r] = nux[r];
            cuxh[r] = nuxh[r];
            cuy[r] = nuy[r];
            cp[r] = np_[r];
            ck[r] = nk[r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) cuyh[h] = nuyh[h];
        if (z + 1 < z1) fetch(z + 1);
        float(*X)[LW] = lx[z & 1];
        float(*Y)[TX] = ly[z & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            X[ty + r * BY][xx] = cux[r];
            if (tx < 8) X[ty + r * BY][tx < 4 ? tx : TX + tx] = cuxh[r];
            Y[4 + ty + r * BY][tx] = cuy[r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int hr = ty + h * BY;
            Y[hr < 4 ? hr : TY + hr][tx] = cuyh[h];
        }
        __syncthreads();
        const float gz = SPONGE ? sd.prof[nx + ny + z] : 1.0f;
        const long long zoff = (long long)z * plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yr = ty + r * BY;
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                dx = fmaf(cf.sx[m - 1], X[yr][xx + m - 1] - X[yr][xx - m], dx);
                dy = fmaf(cf.sy[m - 1], Y[4 + yr + m - 1][tx] - Y[4 + yr - m][tx], dy);
                dz = fmaf(cf.sz[m - 1], w[r][3 + m] - w[r][4 - m], dz);
            }
            if (in[r]) {
                const long long o = zoff + (row[r] * nx + x);
                const float G = SPONGE ? gx * gyv[r] * gz : 1.0f;
                if (CPML) {
                    // psi <- b psi + a D- u, and D- u gains psi (cells inside the layers)
                    if (pm.xl) {
                        const float v = fmaf(pm.bx, cm[0][r], pm.ax * dx);
                        ((gfloat*)sd.zeta[0])[(long long)z * pxs + (pm.vx[r] >> 2)] = v;
                        dx += v;
                    }
                    if (pm.yl[r]) {
                        const float v = fmaf(pm.by[r], cm[CPML ? 1 : 0][r], pm.ay[r] * dy);
                        ((gfloat*)sd.zeta[1])[(long long)z * pys + (pm.vy[r] >> 2)] = v;
                        dy += v;
                    }
                    if (pm.zl(sd, te, z)) {
                        const float v = fmaf(pm.tab[nz + z], cm[CPML ? 2 : 0][r], pm.tab[z] * dz);
                        ((gfloat*)sd.zeta[2])[(long long)pm.zs(sd, z) * plane + (row[r] * nx + x)] = v;
                        dz += v;
                    }
                }
                pn[o] = G * fmaf(ck[r], (dx + dy) + dz, cp[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int m = 0; m < 7; ++m) w[r][m] = w[r][m + 1];
    }
}

template <int TX, int RY, int BC>
static void launch_iso_bc(bool stream, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd, const ShotDev* shots,
                          int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const dim3 block(TX, 256 / TX);
    hipExtLaunchKernelGGL(k_iso_u<TX, RY, BC>, grid, block, 0, s, ev0, nullptr, 0, tiles, ntiles, per_xcd, shots,
                          parity, cf);
    if (stream)
        hipExtLaunchKernelGGL(k_iso_p<TX, RY, BC, true>, grid, block, 0, s, nullptr, ev1, 0, tiles, ntiles, per_xcd,
                              shots, parity, cf);
    else
        hipExtLaunchKernelGGL(k_iso_p<TX, RY, BC, false>, grid, block, 0, s, nullptr, ev1, 0, tiles, ntiles, per_xcd,
                              shots, parity, cf);
}

template <int TX, int RY>
static hipError_t launch_iso_t(int bc, bool stream, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd,
                               const ShotDev* shots, int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0,
                               hipEvent_t ev1) {
    if (bc == 1)
        launch_iso_bc<TX, RY, 1>(stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    else if (bc == 2)
        launch_iso_bc<TX, RY, 2>(stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    else
        launch_iso_bc<TX, RY, 0>(stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    return hipGetLastError();
}

bool iso_variant_ok(int variant) { return variant >= 0 && variant < num_tile_variants() && kTiles[variant].nt == 256; }

hipError_t launch_iso_step(int variant, int bc, bool stream, const TileEnt* tiles, int ntiles, const ShotDev* shots,
                           int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (ntiles <= 0) return hipSuccess;
    if (!iso_variant_ok(variant) || bc < 0 || bc > 2) return hipErrorInvalidValue;
    const int per_xcd = (ntiles + 7) / 8;
    const dim3 grid(8 * per_xcd);
    const TileShape& ts = kTiles[variant];
    if (ts.tx == 64) {
        if (ts.ry == 2) return launch_iso_t<64, 2>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
        if (ts.ry == 4) return launch_iso_t<64, 4>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
        return launch_iso_t<64, 8>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    }
    if (ts.ry == 1) return launch_iso_t<32, 1>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    if (ts.ry == 2) return launch_iso_t<32, 2>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
    return launch_iso_t<32, 4>(bc, stream, grid, tiles, ntiles, per_xcd, shots, parity, cf, s, ev0, ev1);
}

__global__ __launch_bounds__(256) void k_iso_setup(const float* __restrict__ vel, const float* __restrict__ rho,
                                                   long long n, double dt, float* __restrict__ kdt,
                                                   float* __restrict__ rdt) {
    for (long long o = blockIdx.x * 256LL + threadIdx.x; o < n; o += (long long)gridDim.x * 256) {
        const double r0 = rho[o], v = vel[o];
        kdt[o] = (float)(dt * r0 * v * v);
        rdt[o] = (float)(r0 / dt);
    }
}

hipError_t launch_iso_setup(const float* vel, const float* rho, long long n, double dt, float* kdt, float* rdt,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long blocks = std::min<long long>((n + 255) / 256, 65536);
    k_iso_setup<<<dim3((unsigned)blocks), 256, 0, s>>>(vel, rho, n, dt, kdt, rdt);
    return hipGetLastError();
}

// ------------------------------------------------------------ CPML adjoint
//
// The adjoint fields' CPML runs as one launch per step before their stencil
// kernel, one thread per cell of the damping layers of every axis (nb + 4
// cells at each end), writing a correction that the stencil kernel adds to
// the Laplacian of those cells.  The axes write disjoint arrays, so they
// share one launch: the grid is the x-layer blocks (whole 2 (nb + 4)-cell
// rows, lanes along x), then the y-layer and z-layer blocks (64 x-columns by
// the cells of one end).
//
// Slab arrays: memory x [nz][ny][2nb], y [nz][2nb][nx], z [2nb][ny][nx]
// (slab index s < nb is grid index s, s >= nb is grid index n - 2nb + s);
// corrections the same with nb + 4 cells per end.

// Compact block enumeration over the shots: part x has, per shot, one block
// per CPML_XG * rows_per_block rows; parts y and z have 2 ends x 64-column
// blocks x the planes (nz for y, ny for z).  off[3 * (nshots + 1)] holds the
// exclusive prefix sums of the block counts of each part.
constexpr int CPML_XG = 8;  // row groups per x-layer block

struct CpmlGrid {
    const int* off;  // [3][nshots + 1]
    int nshots;
    int rows_per_block;
};

__device__ __forceinline__ int find_shot(const int* off, int nshots, int b) {
    int lo = 0, hi = nshots - 1;  // largest s with off[s] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Adjoint of the CPML step, run on the adjoint fields before their stencil
// kernel.  With eta the current adjoint field and Zb, Pb the adjoints of
// zeta and psi (held in the adjoint fields' psi / zeta slabs), transposing
// the forward recursions gives, per damped axis,
//   Zb <- eta + b Zb,   Pb <- b Pb - D1 (eta + a Zb)   (layer cells),
// and the adjoint stencil adds  C = D2 (a Zb) - D1 (a Pb),  which reaches 4
// cells past the layer, so its slabs (corr) are cw = nb + 4 cells per end.
// D1 is antisymmetric and D2 symmetric on the zero-ghost grid, hence the
// signs.  Three phases, each reading the previous one's values along the
// axis from LDS (zero outside the layer).
__device__ void cpml_x_block_adj(const ShotDev& sd, int parity, const Coefs& cf, int blk, int rpb, float* lds) {
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb, W = sd.cw, W2 = 2 * W;
    const int e = threadIdx.x;
    const int r = e / W2, sl = e - r * W2;
    const int x = sl < W ? sl : nx - W2 + sl;
    const int lo = sl < W ? 0 : W, hi = lo + W;  // this end of the row
    const bool layer = x < nb || x >= nx - nb;
    const int ms = x < nb ? x : x - (nx - nb2);  // memory slab index (layer cells)
    const float* __restrict__ eta = sd.buf[parity];
    float* __restrict__ Pb = sd.psi[0];
    float* __restrict__ Zb = sd.zeta[0];
    float* __restrict__ co = sd.corr[0];
    float* lu = lds;
    float* laz = lds + 256;
    float* lap = lds + 512;
    const float a = sd.prof[x], b = sd.prof[nx + x];
    for (int g = 0; g < CPML_XG; ++g) {
        const int row = (blk * CPML_XG + g) * rpb + r;
        const bool active = r < rpb && row < ny * nz;
        const long long o = (long long)row * nx + x;  // row = z * ny + y
        const long long mi = (long long)row * nb2 + ms;
        float u = 0.0f, az = 0.0f;
        if (active && layer) {
            const float ev = eta[o];
            const float zb = fmaf(b, Zb[mi], ev);
            Zb[mi] = zb;
            u = fmaf(a, zb, ev);
            az = a * zb;
        }
        lu[e] = u;
        laz[e] = az;
        __syncthreads();
        float ap = 0.0f;
        if (active && layer) {
            float d1u = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const float vp = sl + m < hi ? lu[e + m] : 0.0f;
                const float vm = sl - m >= lo ? lu[e - m] : 0.0f;
                d1u = fmaf(cf.bx[m - 1], vp - vm, d1u);
            }
            const float pb = fmaf(b, Pb[mi], -d1u);
            Pb[mi] = pb;
            ap = a * pb;
        }
        lap[e] = ap;
        __syncthreads();
        if (active) {
            float d1 = 0.0f, d2 = 0.0f;
            const float c = laz[e];
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const bool okp = sl + m < hi, okm = sl - m >= lo;
                const float pp = okp ? lap[e + m] : 0.0f, pm = okm ? lap[e - m] : 0.0f;
                const float zp = okp ? laz[e + m] : 0.0f, zm = okm ? laz[e - m] : 0.0f;
                d1 = fmaf(cf.bx[m - 1], pp - pm, d1);
                d2 = fmaf(cf.cx[m - 1], (zp - c) + (zm - c), d2);
            }
            co[(long long)row * W2 + sl] = d2 - d1;
        }
        __syncthreads();  // lds is rewritten by the next row group
    }
}

template <int AX>
__device__ void cpml_yz_block_adj(const ShotDev& sd, int parity, const Coefs& cf, int xblk, int w, int side,
                                  float* lds) {
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb, W = sd.cw, W2 = 2 * W;
    if (w >= (AX == 2 ? ny : nz)) return;  // whole block
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x = xblk * 64 + tx;
    const bool active = x < nx;
    const long long plane = (long long)nx * ny;
    const int n = AX == 2 ? nz : ny;
    const long long stride = AX == 2 ? plane : (long long)nx;
    const long long base = AX == 2 ? (long long)w * nx + x : (long long)w * plane + x;
    // memory slabs (2 nb cells) and correction slabs (2 W cells) along the axis
    const long long mbase = AX == 2 ? (long long)w * nx + x : (long long)w * nb2 * nx + x;
    const long long cbase = AX == 2 ? (long long)w * nx + x : (long long)w * W2 * nx + x;
    const long long sstride = AX == 2 ? plane : (long long)nx;
    const float* prof = AX == 2 ? sd.prof + 2 * nx + 2 * ny : sd.prof + 2 * nx;
    const int s0 = side ? n - W : 0;  // first grid index of this end's W cells
    const int l0 = side ? W - nb : 0;  // its layer cells are [l0, l0 + nb)
    float* lu = lds;                   // [W][64] each
    float* laz = lds + W * 64;
    float* lap = lds + 2 * W * 64;
    const float* __restrict__ eta = sd.buf[parity];
    float* __restrict__ Pb = sd.psi[AX];
    float* __restrict__ Zb = sd.zeta[AX];
    float* __restrict__ co = sd.corr[AX];
    const float bc1 = AX == 2 ? cf.bz[0] : cf.by[0], bc2 = AX == 2 ? cf.bz[1] : cf.by[1];
    const float bc3 = AX == 2 ? cf.bz[2] : cf.by[2], bc4 = AX == 2 ? cf.bz[3] : cf.by[3];
    const float bcoef[4] = {bc1, bc2, bc3, bc4};
    for (int s = ty; s < W; s += 4) {
        float u = 0.0f, az = 0.0f;
        if (active && s >= l0 && s < l0 + nb) {
            const int z = s0 + s;
            const long long mi = mbase + (long long)((side ? nb : 0) + s - l0) * sstride;
            const float ev = eta[base + z * stride];
            const float zb = fmaf(prof[n + z], Zb[mi], ev);
            Zb[mi] = zb;
            u = fmaf(prof[z], zb, ev);
            az = prof[z] * zb;
        }
        lu[s * 64 + tx] = u;
        laz[s * 64 + tx] = az;
    }
    __syncthreads();
    for (int s = ty; s < W; s += 4) {
        float ap = 0.0f;
        if (active && s >= l0 && s < l0 + nb) {
            const int z = s0 + s;
            const long long mi = mbase + (long long)((side ? nb : 0) + s - l0) * sstride;
            float d1u = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const float vp = s + m < W ? lu[(s + m) * 64 + tx] : 0.0f;
                const float vm = s - m >= 0 ? lu[(s - m) * 64 + tx] : 0.0f;
                d1u = fmaf(bcoef[m - 1], vp - vm, d1u);
            }
            const float pb = fmaf(prof[n + z], Pb[mi], -d1u);
            Pb[mi] = pb;
            ap = prof[z] * pb;
        }
        lap[s * 64 + tx] = ap;
    }
    __syncthreads();
    if (!active) return;
    for (int s = ty; s < W; s += 4) {
        float d1 = 0.0f, d2 = 0.0f;
        const float c = laz[s * 64 + tx];
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
            const bool okp = s + m < W, okm = s - m >= 0;
            const float pp = okp ? lap[(s + m) * 64 + tx] : 0.0f, pm = okm ? lap[(s - m) * 64 + tx] : 0.0f;
            const float zp = okp ? laz[(s + m) * 64 + tx] : 0.0f, zm = okm ? laz[(s - m) * 64 + tx] : 0.0f;
            d1 = fmaf(bcoef[m - 1], pp - pm, d1);
            d2 = fmaf(AX == 2 ? cf.cz[m - 1] : cf.cy[m - 1], (zp - c) + (zm - c), d2);
        }
        co[cbase + (long long)((side ? W : 0) + s) * sstride] = d2 - d1;
    }
}

__global__ __launch_bounds__(256) void k_cpml_adj(const ShotDev* __restrict__ shots, int parity, Coefs cf,
                                                  CpmlGrid g) {
    extern __shared__ float lds[];
    const int S = g.nshots;
    const int* ox = g.off;
    const int* oy = g.off + (S + 1);
    const int* oz = g.off + 2 * (S + 1);
    int b = blockIdx.x;
    if (b < ox[S]) {
        const int s = find_shot(ox, S, b);
        cpml_x_block_adj(shots[s], parity, cf, b - ox[s], g.rows_per_block, lds);
        return;
    }
    b -= ox[S];
    const bool ypart = b < oy[S];
    if (!ypart) b -= oy[S];
    const int* o = ypart ? oy : oz;
    const int s = find_shot(o, S, b);
    const ShotDev& sd = shots[s];
    const int local = b - o[s];
    const int xb = (sd.nx + 63) / 64;
    const int W = ypart ? sd.nz : sd.ny;
    const int xblk = local % xb, rest = local / xb;
    const int w = rest % W, side = rest / W;
    if (ypart) cpml_yz_block_adj<1>(sd, parity, cf, xblk, w, side, lds);
    else cpml_yz_block_adj<2>(sd, parity, cf, xblk, w, side, lds);
}

// ------------------------------------------------------ CPML, layer pass
//
// The other forward CPML strategy (for grids whose layers hold a large share
// of the cells, where the fused kernel's z-marching strips leave the chip
// idle): one launch per step before the stencil kernel (BC == 2), one thread
// per layer cell of every axis, in the block enumeration of the adjoint with
// nb cells per end.  Per damped axis and layer cell
//   psi^{n+1} = b psi^n + a D1 p^n,   zeta^{n+1} = b zeta^n + a (D2 p^n + D1 psi^{n+1}),
// and the correction D1 psi^{n+1} + zeta^{n+1} goes to the slabs (corr) that
// the stencil kernel adds to the Laplacian.  psi is zero outside its layer
// and the two layers of an axis are at least 4 cells apart, so a block that
// holds a whole layer segment along the axis has every psi^{n+1} it needs in
// LDS, and psi and zeta are updated in place (ShotDev::psi; the second psi
// buffer of k_cstep stays untouched, which keeps the step's working set at
// that of the three slab arrays).

// NT: psi and zeta (read once per step) are loaded with the non-temporal hint
template <bool NT>
__device__ __forceinline__ float once(const float* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT>
__device__ void cpml_x_block_fwd(const ShotDev& sd, int parity, const Coefs& cf, int blk, int rpb, float* lds) {
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb;
    const int e = threadIdx.x;
    const int r = e / nb2, sl = e - r * nb2;
    const int x = sl < nb ? sl : nx - nb2 + sl;
    const int lo = sl < nb ? 0 : nb, hi = lo + nb;  // this end of the row (the other is >= 4 cells away)
    const float* __restrict__ p = sd.buf[parity];
    float* __restrict__ ps = sd.psi[0];
    float* __restrict__ ze = sd.zeta[0];
    float* __restrict__ co = sd.corr[0];
    const float a = sd.prof[x], b = sd.prof[nx + x];
    for (int g = 0; g < CPML_XG; ++g) {
        const int row = (blk * CPML_XG + g) * rpb + r;
        const bool active = r < rpb && row < ny * nz;
        const long long o = (long long)row * nx + x;  // row = z * ny + y
        const long long si = (long long)row * nb2 + sl;
        float d2 = 0.0f;
        if (active) {
            const float c = p[o];
            float d1 = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const float fp = x + m < nx ? p[o + m] : 0.0f;
                const float fm = x - m >= 0 ? p[o - m] : 0.0f;
                d1 = fmaf(cf.bx[m - 1], fp - fm, d1);
                d2 = fmaf(cf.cx[m - 1], (fp - c) + (fm - c), d2);
            }
            const float pv = fmaf(b, once<NT>(ps + si), a * d1);
            ps[si] = pv;
            lds[e] = pv;
        }
        __syncthreads();
        if (active) {
            float dpsi = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const float vp = sl + m < hi ? lds[e + m] : 0.0f;
                const float vm = sl - m >= lo ? lds[e - m] : 0.0f;
                dpsi = fmaf(cf.bx[m - 1], vp - vm, dpsi);
            }
            const float zn = fmaf(b, once<NT>(ze + si), a * (d2 + dpsi));
            ze[si] = zn;
            co[si] = dpsi + zn;
        }
        __syncthreads();  // lds is rewritten by the next row group
    }
}

// y (AX = 1) or z (AX = 2) layers of one end: block = 64 x-columns, thread row
// ty takes cells ty, ty + 4, ... of the nb cells; w is z (AX = 1) or y (AX = 2).
template <int AX, bool NT>
__device__ void cpml_yz_block_fwd(const ShotDev& sd, int parity, const Coefs& cf, int xblk, int w, int side,
                                  float* lds) {
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb;
    if (w >= (AX == 2 ? ny : nz)) return;  // whole block
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int x = xblk * 64 + tx;
    const bool active = x < nx;
    const long long plane = (long long)nx * ny;
    const int n = AX == 2 ? nz : ny;
    const long long stride = AX == 2 ? plane : (long long)nx;
    const long long base = AX == 2 ? (long long)w * nx + x : (long long)w * plane + x;
    const long long sbase = AX == 2 ? (long long)w * nx + x : (long long)w * nb2 * nx + x;
    const long long sstride = AX == 2 ? plane : (long long)nx;
    const float* prof = AX == 2 ? sd.prof + 2 * nx + 2 * ny : sd.prof + 2 * nx;
    const int s0 = side ? n - nb : 0;
    const int soff = side ? nb : 0;  // slab index of the first cell of this end
    float* psl = lds;                // [nb][64]: psi^{n+1}
    float* d2l = lds + nb * 64;      // [nb][64]: D2 p^n
    const float* __restrict__ p = sd.buf[parity];
    float* __restrict__ psi = sd.psi[AX];
    if (active) {
        for (int s = ty; s < nb; s += 4) {
            const int z = s0 + s;
            const long long o = base + z * stride;
            const float c = p[o];
            float d1 = 0.0f, d2 = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                const float fp = z + m < n ? p[o + m * stride] : 0.0f;
                const float fm = z - m >= 0 ? p[o - m * stride] : 0.0f;
                d1 = fmaf(AX == 2 ? cf.bz[m - 1] : cf.by[m - 1], fp - fm, d1);
                d2 = fmaf(AX == 2 ? cf.cz[m - 1] : cf.cy[m - 1], (fp - c) + (fm - c), d2);
            }
            const long long si = sbase + (long long)(soff + s) * sstride;
            const float ps = fmaf(prof[n + z], once<NT>(psi + si), prof[z] * d1);
            psi[si] = ps;
            psl[s * 64 + tx] = ps;
            d2l[s * 64 + tx] = d2;
        }
    }
    __syncthreads();
    if (!active) return;
    float* __restrict__ ze = sd.zeta[AX];
    float* __restrict__ co = sd.corr[AX];
    for (int s = ty; s < nb; s += 4) {
        const int z = s0 + s;
        float dpsi = 0.0f;
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
            const float vp = s + m < nb ? psl[(s + m) * 64 + tx] : 0.0f;
            const float vm = s - m >= 0 ? psl[(s - m) * 64 + tx] : 0.0f;
            dpsi = fmaf(AX == 2 ? cf.bz[m - 1] : cf.by[m - 1], vp - vm, dpsi);
        }
        const long long si = sbase + (long long)(soff + s) * sstride;
        const float zn = fmaf(prof[n + z], once<NT>(ze + si), prof[z] * (d2l[s * 64 + tx] + dpsi));
        ze[si] = zn;
        co[si] = dpsi + zn;
    }
}

template <bool NT>
__global__ __launch_bounds__(256) void k_cpml_fwd(const ShotDev* __restrict__ shots, int parity, Coefs cf,
                                                  CpmlGrid g) {
    extern __shared__ float lds[];
    const int S = g.nshots;
    const int* ox = g.off;
    const int* oy = g.off + (S + 1);
    const int* oz = g.off + 2 * (S + 1);
    int b = blockIdx.x;
    if (b < ox[S]) {
        const int s = find_shot(ox, S, b);
        cpml_x_block_fwd<NT>(shots[s], parity, cf, b - ox[s], g.rows_per_block, lds);
        return;
    }
    b -= ox[S];
    const bool ypart = b < oy[S];
    if (!ypart) b -= oy[S];
    const int* o = ypart ? oy : oz;
    const int s = find_shot(o, S, b);
    const ShotDev& sd = shots[s];
    const int local = b - o[s];
    const int xb = (sd.nx + 63) / 64;
    const int W = ypart ? sd.nz : sd.ny;
    const int xblk = local % xb, rest = local / xb;
    const int w = rest % W, side = rest / W;
    if (ypart) cpml_yz_block_fwd<1, NT>(sd, parity, cf, xblk, w, side, lds);
    else cpml_yz_block_fwd<2, NT>(sd, parity, cf, xblk, w, side, lds);
}

int cpml_rows_per_block(int width) { return 256 / (2 * width); }

void cpml_block_table(const int* nx, const int* ny, const int* nz, int nshots, int width, int* off) {
    const int rpb = cpml_rows_per_block(width);
    int* ox = off;
    int* oy = off + (nshots + 1);
    int* oz = off + 2 * (nshots + 1);
    ox[0] = oy[0] = oz[0] = 0;
    for (int i = 0; i < nshots; ++i) {
        const long long rows = (long long)ny[i] * nz[i];
        const int xb = (nx[i] + 63) / 64;
        ox[i + 1] = ox[i] + (int)((rows + (long long)rpb * CPML_XG - 1) / ((long long)rpb * CPML_XG));
        oy[i + 1] = oy[i] + 2 * xb * nz[i];
        oz[i + 1] = oz[i] + 2 * xb * ny[i];
    }
}

hipError_t launch_cpml_forward(const ShotDev* shots, int nshots, int nb, bool stream, const int* block_off_dev,
                               const int* block_off_host, int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0) {
    if (nshots <= 0) return hipSuccess;
    if (nb < 1 || nb > 128) return hipErrorInvalidValue;
    CpmlGrid g;
    g.off = block_off_dev;
    g.nshots = nshots;
    g.rows_per_block = cpml_rows_per_block(nb);
    const int S = nshots;
    const long long blocks =
        (long long)block_off_host[S] + block_off_host[(S + 1) + S] + block_off_host[2 * (S + 1) + S];
    // psi and D2 p of one end, [nb][64] each (x part: 256)
    const size_t fl = std::max((size_t)2 * nb * 64, (size_t)256);
    const dim3 grid((unsigned)blocks), block(256);
    const unsigned lds = (unsigned)(sizeof(float) * fl);
    if (stream)
        hipExtLaunchKernelGGL(k_cpml_fwd<true>, grid, block, lds, s, ev0, nullptr, 0, shots, parity, cf, g);
    else
        hipExtLaunchKernelGGL(k_cpml_fwd<false>, grid, block, lds, s, ev0, nullptr, 0, shots, parity, cf, g);
    return hipGetLastError();
}

hipError_t launch_cpml_adjoint(const ShotDev* shots, int nshots, int nb, const int* block_off_dev,
                               const int* block_off_host, int parity, const Coefs& cf, hipStream_t s, hipEvent_t ev0) {
    if (nshots <= 0) return hipSuccess;
    if (nb < 1 || nb > 64) return hipErrorInvalidValue;
    const int width = nb + 4;
    CpmlGrid g;
    g.off = block_off_dev;
    g.nshots = nshots;
    g.rows_per_block = cpml_rows_per_block(width);
    const int S = nshots;
    const long long blocks =
        (long long)block_off_host[S] + block_off_host[(S + 1) + S] + block_off_host[2 * (S + 1) + S];
    // three [W][64] arrays (x part: 3 x 256)
    const size_t fl = 3 * (size_t)std::max(width * 64, 256);
    const dim3 grid((unsigned)blocks), block(256);
    hipExtLaunchKernelGGL(k_cpml_adj, grid, block, (unsigned)(sizeof(float) * fl), s, ev0, nullptr, 0, shots,
                          parity, cf, g);
    return hipGetLastError();
}

// ------------------------------------------------------- inject and gather

template <int MODE, bool BF>
__global__ __launch_bounds__(256) void k_inject(InjTab tab, const ShotDev* __restrict__ shots, int parity,
                                                const float* __restrict__ vals, StepAux aux) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= tab.ncell) return;
    const float g = tab.cell_g[u];
    if (g == 0.0f) return;  // a cell on a free surface: nothing enters
    float acc = 0.0f;
    for (int q = tab.start[u]; q < tab.start[u + 1]; ++q) acc += vals[tab.col[q]];
    const ShotDev& sd = shots[tab.cell_shot[u]];
    const long long o = tab.cell_off[u];
    const float term = g * (sd.vdt2[o] * (tab.scale * acc));
    float* pn = sd.buf[parity ^ 1];
    pn[o] += term;
    if (MODE == MODE_D2P) d2p_put<BF>(aux.d2p_out, o, d2p_get<BF>(aux.d2p_out, o) + term);
    if (MODE == MODE_IMAGE) aux.grad[o] = fmaf(aux.neg_inv_dt2 / g * term, d2p_get<BF>(aux.d2p_in, o), aux.grad[o]);
}

hipError_t launch_inject(const InjTab& tab, const ShotDev* shots, int parity, const float* vals, int ncols, int mode,
                         const StepAux& aux, hipStream_t s) {
    (void)ncols;
    if (tab.ncell <= 0) return hipSuccess;
    dim3 grid((tab.ncell + 255) / 256);
    const bool h = aux.d2p_bf16 != 0;
    if (mode == MODE_PLAIN)
        k_inject<MODE_PLAIN, false><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else if (mode == MODE_D2P && h)
        k_inject<MODE_D2P, true><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else if (mode == MODE_D2P)
        k_inject<MODE_D2P, false><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else if (h)
        k_inject<MODE_IMAGE, true><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else
        k_inject<MODE_IMAGE, false><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_gather(GatherTab tab, const ShotDev* __restrict__ shots, int parity,
                                                float* __restrict__ out) {
    const int r = blockIdx.x * 256 + threadIdx.x;
    if (r >= tab.n) return;
    out[r] = shots[tab.shot[r]].buf[parity ^ 1][tab.off[r]];
}

hipError_t launch_gather(const GatherTab& tab, const ShotDev* shots, int parity, float* out, hipStream_t s) {
    if (tab.n <= 0) return hipSuccess;
    k_gather<<<(tab.n + 255) / 256, 256, 0, s>>>(tab, shots, parity, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- set-up

static dim3 stride_grid(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

__global__ __launch_bounds__(256) void k_vdt2(const float* __restrict__ vel, float* __restrict__ vdt2, long long n,
                                              double dt) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const double v = dt * (double)vel[i];
        vdt2[i] = (float)(v * v);
    }
}

hipError_t launch_vdt2(const float* vel, float* vdt2, long long n, double dt, hipStream_t s) {
    k_vdt2<<<stride_grid(n), 256, 0, s>>>(vel, vdt2, n, dt);
    return hipGetLastError();
}

// result2[0] = max over the model of the float bits (positive floats order as
// unsigned), result2[1] |= 1 if any value is NaN, Inf or <= 0.
__global__ __launch_bounds__(256) void k_vcheck(const float* __restrict__ vel, long long n, unsigned* result2) {
    __shared__ unsigned smax[256], sbad[256];
    unsigned mx = 0, bad = 0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float v = vel[i];
        if (!(v > 0.0f) || !isfinite(v)) bad = 1;
        else mx = max(mx, __float_as_uint(v));
    }
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            smax[threadIdx.x] = max(smax[threadIdx.x], smax[threadIdx.x + w]);
            sbad[threadIdx.x] |= sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&result2[0], smax[0]);
        if (sbad[0]) atomicOr(&result2[1], 1u);
    }
}

hipError_t launch_vcheck(const float* vel, long long n, unsigned* result2, hipStream_t s) {
    k_vcheck<<<stride_grid(n), 256, 0, s>>>(vel, n, result2);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill(float* __restrict__ p, long long n, float v) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) p[i] = v;
}

hipError_t launch_fill(float* p, long long n, float v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill<<<stride_grid(n), 256, 0, s>>>(p, n, v);
    return hipGetLastError();
}

// Watchdog scan: one vector atomic per wave that saw a non-finite value.
__global__ __launch_bounds__(256) void k_watch(const float* __restrict__ p, long long n, int step,
                                               unsigned* __restrict__ w) {
    bool bad = false;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        bad = bad || !isfinite(p[i]);
    if (__ballot(bad) && (threadIdx.x & 63) == __ffsll((long long)__ballot(bad)) - 1) {
        atomicOr(&w[0], 1u);
        atomicMin(&w[1], (unsigned)step);
    }
}

__global__ void k_watch_reset(unsigned* __restrict__ w) {
    if (threadIdx.x == 0) {
        w[0] = 0u;
        w[1] = 0xFFFFFFFFu;
    }
}

hipError_t launch_watch(const float* p, long long n, int step, unsigned* w, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_watch<<<stride_grid(n), 256, 0, s>>>(p, n, step, w);
    return hipGetLastError();
}

hipError_t launch_watch_reset(unsigned* w, hipStream_t s) {
    k_watch_reset<<<1, 64, 0, s>>>(w);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(float* __restrict__ d, const float* __restrict__ src, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) d[i] = src[i];
}

hipError_t launch_copy(float* dst, const float* src, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_copy<<<stride_grid(n), 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

// ------------------------------------------------------- snapshot codec
//
// A checkpoint (p^{k-1}, p^k) is stored as two bfloat16 arrays: c0 = bf16(p^k / s0)
// and c1 = bf16((p^k - p^{k-1}) / s1), each scaled per block of SNAP_BLOCK cells
// by the block's largest magnitude (1 for an all-zero block), rounded to nearest
// even.  Keeping the increment instead of p^{k-1} itself stores the part of the
// state the leapfrog amplifies most (the difference of two nearly equal fields)
// with its own 8-bit relative precision.  Decoding gives p^k = f(c0) s0 and
// p^{k-1} = p^k - f(c1) s1, each product and difference rounded once.
// One pass each way: read 8 B and write 4 B per cell, or the reverse.

__device__ __forceinline__ float block_absmax256(float m, float* sm) {
    // wave reduction, then the 4 waves of the block through LDS
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    return fmaxf(fmaxf(sm[0], sm[1]), fmaxf(sm[2], sm[3]));
}

constexpr int SNAP_PER_THREAD = SNAP_BLOCK / 256;

__global__ __launch_bounds__(256) void k_snap_encode(const float* __restrict__ prev, const float* __restrict__ cur,
                                                     long long n, uint16_t* __restrict__ c0,
                                                     uint16_t* __restrict__ c1, float* __restrict__ s0,
                                                     float* __restrict__ s1) {
    __shared__ float sm[2][4];
    const long long base = (long long)blockIdx.x * SNAP_BLOCK;
    float v[SNAP_PER_THREAD], d[SNAP_PER_THREAD];
    float m0 = 0.0f, m1 = 0.0f;
#pragma unroll
    for (int k = 0; k < SNAP_PER_THREAD; ++k) {
        const long long i = base + k * 256 + threadIdx.x;
        const bool ok = i < n;
        const float c = ok ? __builtin_nontemporal_load(cur + i) : 0.0f;
        const float p = ok ? __builtin_nontemporal_load(prev + i) : 0.0f;
        v[k] = c;
        d[k] = c - p;
        m0 = fmaxf(m0, fabsf(v[k]));
        m1 = fmaxf(m1, fabsf(d[k]));
    }
    m0 = block_absmax256(m0, sm[0]);
    m1 = block_absmax256(m1, sm[1]);
    const float a0 = m0 > 0.0f ? m0 : 1.0f, a1 = m1 > 0.0f ? m1 : 1.0f;
    if (threadIdx.x == 0) {
        s0[blockIdx.x] = a0;
        s1[blockIdx.x] = a1;
    }
#pragma unroll
    for (int k = 0; k < SNAP_PER_THREAD; ++k) {
        const long long i = base + k * 256 + threadIdx.x;
        if (i < n) {
            c0[i] = f2bf_rne(v[k] / a0);
            c1[i] = f2bf_rne(d[k] / a1);
        }
    }
}

__global__ __launch_bounds__(256) void k_snap_decode(const uint16_t* __restrict__ c0, const uint16_t* __restrict__ c1,
                                                     const float* __restrict__ s0, const float* __restrict__ s1,
                                                     long long n, float* __restrict__ prev, float* __restrict__ cur) {
#pragma clang fp contract(off)  // the product and the difference are rounded separately
    const long long base = (long long)blockIdx.x * SNAP_BLOCK;
    const float a0 = s0[blockIdx.x], a1 = s1[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SNAP_PER_THREAD; ++k) {
        const long long i = base + k * 256 + threadIdx.x;
        if (i < n) {
            const float v = __uint_as_float((unsigned)c0[i] << 16) * a0;
            const float d = __uint_as_float((unsigned)c1[i] << 16) * a1;
            cur[i] = v;
            prev[i] = v - d;
        }
    }
}

long long snap_blocks(long long n) { return (n + SNAP_BLOCK - 1) / SNAP_BLOCK; }

hipError_t launch_snap_encode(const float* prev, const float* cur, long long n, uint16_t* c0, uint16_t* c1, float* s0,
                              float* s1, hipStream_t s) {
    const long long nb = snap_blocks(n);
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    k_snap_encode<<<dim3((unsigned)nb), 256, 0, s>>>(prev, cur, n, c0, c1, s0, s1);
    return hipGetLastError();
}

hipError_t launch_snap_decode(const uint16_t* c0, const uint16_t* c1, const float* s0, const float* s1, long long n,
                              float* prev, float* cur, hipStream_t s) {
    const long long nb = snap_blocks(n);
    if (nb <= 0) return hipSuccess;
    if (nb > 0x7FFFFFFFLL) return hipErrorInvalidValue;
    k_snap_decode<<<dim3((unsigned)nb), 256, 0, s>>>(c0, c1, s0, s1, n, prev, cur);
    return hipGetLastError();
}

// --------------------------------------------------------- residual, loss

__global__ __launch_bounds__(256) void k_resid_part(const float* __restrict__ tr, const float* __restrict__ dobs,
                                                    float* __restrict__ resid, long long n,
                                                    double* __restrict__ part) {
    __shared__ double sm[256];
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const float r = tr[i] - dobs[i];
        resid[i] = r;
        acc += (double)r * (double)r;
    }
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_sum_final(const double* __restrict__ part, int nparts,
                                                   double* __restrict__ out) {
    __shared__ double sm[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    sm[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0.5 * sm[0];
}

hipError_t launch_residual_loss(const float* traces, const float* dobs, float* resid, long long n, double* partial,
                                int nparts, double* loss, hipStream_t s) {
    dim3 g = stride_grid(n);
    if ((int)g.x > nparts) g.x = nparts;
    k_resid_part<<<g, 256, 0, s>>>(traces, dobs, resid, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_final<<<1, 256, 0, s>>>(partial, (int)g.x, loss);
    return hipGetLastError();
}



// --------------------------------------------------------- static workspace
//
// Device memory of the contexts made by mm_init_static, for callers that
// cannot allocate: one array per GPU, which that GPU holds until the process
// ends.  Host code must not use the array's name as an address (on the host
// it is a stand-in symbol); static_workspace looks up its device address
// once per device, with that device current, and keeps it.
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticWorkspaceBytes];

size_t static_workspace_bytes() { return kStaticWorkspaceBytes; }

hipError_t static_workspace(void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    *out = nullptr;
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return e;
    if (d < 0 || d >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[d]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[d] = p;
    }
    *out = addr[d];
    return hipSuccess;
}

}  // namespace mm
