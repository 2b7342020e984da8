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
#include <hip/hip_runtime.h>

#include "mm_internal.h"

namespace mm {

static const TileShape kTiles[] = {
    {64, 4, 2048, "64x16/2048"}, {64, 4, 1024, "64x16/1024"}, {64, 4, 4096, "64x16/4096"},
    {64, 2, 2048, "64x8/2048"},  {64, 2, 1024, "64x8/1024"},  {64, 2, 4096, "64x8/4096"},
    {64, 8, 2048, "64x32/2048"}, {64, 8, 1024, "64x32/1024"}, {64, 8, 4096, "64x32/4096"},
    {32, 2, 2048, "32x16/2048"}, {32, 2, 1024, "32x16/1024"}, {32, 2, 4096, "32x16/4096"},
    {32, 4, 2048, "32x32/2048"}, {32, 4, 1024, "32x32/1024"}, {32, 4, 4096, "32x32/4096"},
    {32, 1, 2048, "32x8/2048"},  {32, 1, 1024, "32x8/1024"},  {32, 1, 4096, "32x8/4096"},
};

int num_tile_variants() { return (int)(sizeof(kTiles) / sizeof(kTiles[0])); }
const TileShape& tile_variant(int t) { return kTiles[t]; }
int tile_rows(int t) { return (256 / kTiles[t].tx) * kTiles[t].ry; }

// ------------------------------------------------------------- stencil step

template <int TX, int RY, bool SPONGE, int MODE>
__global__ __launch_bounds__(256) void k_step(const TileEnt* __restrict__ tiles, int ntiles, int per_xcd,
                                              const ShotDev* __restrict__ shots, int parity, Coefs cf,
                                              StepAux aux) {
    constexpr int BY = 256 / TX;
    constexpr int TY = BY * RY;
    constexpr int LW = TX + 8;
    constexpr int YH = 8 / BY;
    static_assert(BY <= 8 && 8 % BY == 0, "y halo split");
    __shared__ float lds[2][TY + 8][LW];

    // consecutive tiles on one XCD: block b runs on XCD b % 8
    const int b = blockIdx.x;
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
    bool in[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        row[r] = te.y0 + ty + r * BY;
        in[r] = xin && row[r] < ny;
    }
    // x halo: lanes 0..7 of every thread row carry the 4 left and 4 right columns
    const int hcol = tx < 4 ? te.x0 - 4 + tx : te.x0 + TX + (tx - 4);
    const bool hx_lane = tx < 8 && hcol >= 0 && hcol < nx;
    // y halo: thread row ty loads halo rows ty, ty + BY, ... of the 8
    int hrow[YH];
    bool hy_ok[YH];
#pragma unroll
    for (int h = 0; h < YH; ++h) {
        const int hr = ty + h * BY;
        hrow[h] = hr < 4 ? te.y0 - 4 + hr : te.y0 + TY + (hr - 4);
        hy_ok[h] = xin && hrow[h] >= 0 && hrow[h] < ny;
    }

    auto ld = [&](const float* __restrict__ base, bool ok, int yy, int xx, int z) -> float {
        return (ok && z >= 0 && z < nz) ? base[(long long)z * plane + (long long)yy * nx + xx] : 0.0f;
    };

    float gx = 1.0f, gyv[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) gyv[r] = 1.0f;
    if (SPONGE) {
        gx = xin ? sd.prof[x] : 1.0f;
#pragma unroll
        for (int r = 0; r < RY; ++r) gyv[r] = in[r] ? sd.prof[nx + row[r]] : 1.0f;
    }

    const int z0 = te.z0, z1 = te.z1;
    float q[RY][9];
#pragma unroll
    for (int r = 0; r < RY; ++r)
#pragma unroll
        for (int m = 0; m < 8; ++m) q[r][m] = ld(pc, in[r], row[r], x, z0 - 4 + m);

    float nq[RY], npp[RY], nvd[RY], nxh[RY], nyh[YH];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
        nq[r] = ld(pc, in[r], row[r], x, z0 + 4);
        npp[r] = ld(pn, in[r], row[r], x, z0);
        nvd[r] = ld(vd, in[r], row[r], x, z0);
        nxh[r] = ld(pc, hx_lane && row[r] < ny, row[r], hcol, z0);
    }
#pragma unroll
    for (int h = 0; h < YH; ++h) nyh[h] = ld(pc, hy_ok[h], hrow[h], x, z0);

    const int xx = 4 + tx;
    for (int z = z0; z < z1; ++z) {
        float cpp[RY], cvd[RY], cxh[RY], cyh[YH];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            q[r][8] = nq[r];
            cpp[r] = npp[r];
            cvd[r] = nvd[r];
            cxh[r] = nxh[r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) cyh[h] = nyh[h];
        if (z + 1 < z1) {
#pragma unroll
            for (int r = 0; r < RY; ++r) {
                nq[r] = ld(pc, in[r], row[r], x, z + 5);
                npp[r] = ld(pn, in[r], row[r], x, z + 1);
                nvd[r] = ld(vd, in[r], row[r], x, z + 1);
                nxh[r] = ld(pc, hx_lane && row[r] < ny, row[r], hcol, z + 1);
            }
#pragma unroll
            for (int h = 0; h < YH; ++h) nyh[h] = ld(pc, hy_ok[h], hrow[h], x, z + 1);
        }

        float(*L)[LW] = lds[z & 1];
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            L[4 + ty + r * BY][xx] = q[r][4];
            if (tx < 8) L[4 + ty + r * BY][tx < 4 ? tx : TX + tx] = cxh[r];
        }
#pragma unroll
        for (int h = 0; h < YH; ++h) {
            const int hr = ty + h * BY;
            L[hr < 4 ? hr : TY + hr][xx] = cyh[h];
        }
        __syncthreads();

        const float gz = SPONGE ? sd.prof[nx + ny + z] : 1.0f;
        const long long zoff = (long long)z * plane;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int yy = 4 + ty + r * BY;
            const float c = q[r][4];
            float lap = 0.0f;
#pragma unroll
            for (int m = 1; m <= 4; ++m) {
                lap = fmaf(cf.cx[m - 1], (L[yy][xx + m] - c) + (L[yy][xx - m] - c), lap);
                lap = fmaf(cf.cy[m - 1], (L[yy + m][xx] - c) + (L[yy - m][xx] - c), lap);
                lap = fmaf(cf.cz[m - 1], (q[r][4 + m] - c) + (q[r][4 - m] - c), lap);
            }
            if (in[r]) {
                const long long o = zoff + (long long)row[r] * nx + x;
                float out, G = 1.0f;
                if (SPONGE) {
                    G = gx * gyv[r] * gz;
                    out = G * (c + fmaf(cvd[r], lap, c - G * cpp[r]));
                } else {
                    out = c + fmaf(cvd[r], lap, c - cpp[r]);
                }
                pn[o] = out;
                if (MODE == MODE_D2P) aux.d2p_out[o] = G * (cvd[r] * lap);
                if (MODE == MODE_IMAGE) aux.grad[o] = fmaf(aux.neg_inv_dt2 / G * out, aux.d2p_in[o], aux.grad[o]);
            }
        }
#pragma unroll
        for (int r = 0; r < RY; ++r)
#pragma unroll
            for (int m = 0; m < 8; ++m) q[r][m] = q[r][m + 1];
    }
}

template <int TX, int RY>
static hipError_t launch_step_t(bool sponge, int mode, dim3 grid, const TileEnt* tiles, int ntiles, int per_xcd,
                                const ShotDev* shots, int parity, const Coefs& cf, const StepAux& aux,
                                hipStream_t s) {
    dim3 block(TX, 256 / TX);
    if (sponge) {
        if (mode == MODE_PLAIN)
            k_step<TX, RY, true, MODE_PLAIN><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf, aux);
        else if (mode == MODE_D2P)
            k_step<TX, RY, true, MODE_D2P><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf, aux);
        else
            k_step<TX, RY, true, MODE_IMAGE><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf, aux);
    } else {
        if (mode == MODE_PLAIN)
            k_step<TX, RY, false, MODE_PLAIN><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf, aux);
        else if (mode == MODE_D2P)
            k_step<TX, RY, false, MODE_D2P><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf, aux);
        else
            k_step<TX, RY, false, MODE_IMAGE><<<grid, block, 0, s>>>(tiles, ntiles, per_xcd, shots, parity, cf,
                                                                       aux);
    }
    return hipGetLastError();
}

hipError_t launch_step(int variant, bool sponge, int mode, const TileEnt* tiles, int ntiles, const ShotDev* shots,
                       int parity, const Coefs& cf, const StepAux& aux, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const int per_xcd = (ntiles + 7) / 8;
    dim3 grid(8 * per_xcd);
    const TileShape& ts = kTiles[variant];
    if (ts.tx == 64) {
        if (ts.ry == 2) return launch_step_t<64, 2>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
        if (ts.ry == 4) return launch_step_t<64, 4>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
        return launch_step_t<64, 8>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
    }
    if (ts.ry == 1) return launch_step_t<32, 1>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
    if (ts.ry == 2) return launch_step_t<32, 2>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
    return launch_step_t<32, 4>(sponge, mode, grid, tiles, ntiles, per_xcd, shots, parity, cf, aux, s);
}

// -------------------------------------------------------------------- CPML
//
// The damping layers are the union of six slabs.  They are enumerated as
// three disjoint regions: the two z slabs (whole planes), the two y slabs
// of the remaining planes, the two x slabs of the remaining rows.  Each
// point updates the memory of every axis whose layer it lies in.

__device__ __forceinline__ bool in_layer(int i, int n, int nb) { return i < nb || i >= n - nb; }

__device__ __forceinline__ int slab_index(int i, int n, int nb) { return i < nb ? i : i - (n - 2 * nb); }

__device__ __forceinline__ long long slab_count(const ShotDev& sd) {
    const long long nb2 = 2LL * sd.nb;
    return nb2 * sd.ny * sd.nx + (sd.nz - nb2) * nb2 * sd.nx + (sd.nz - nb2) * (sd.ny - nb2) * nb2;
}

__device__ __forceinline__ bool slab_point(const ShotDev& sd, long long i, int& x, int& y, int& z) {
    const int nx = sd.nx, ny = sd.ny, nz = sd.nz, nb = sd.nb, nb2 = 2 * nb;
    const long long r0 = (long long)nb2 * ny * nx;
    if (i < r0) {
        const int s = (int)(i / ((long long)ny * nx));
        const long long rem = i - (long long)s * ny * nx;
        z = s < nb ? s : nz - nb2 + s;
        y = (int)(rem / nx);
        x = (int)(rem - (long long)y * nx);
        return true;
    }
    i -= r0;
    const long long r1 = (long long)(nz - nb2) * nb2 * nx;
    if (i < r1) {
        const long long per = (long long)nb2 * nx;
        z = nb + (int)(i / per);
        const long long rem = i - (long long)(z - nb) * per;
        const int s = (int)(rem / nx);
        y = s < nb ? s : ny - nb2 + s;
        x = (int)(rem - (long long)s * nx);
        return true;
    }
    i -= r1;
    const long long r2 = (long long)(nz - nb2) * (ny - nb2) * nb2;
    if (i < r2) {
        const long long per = (long long)(ny - nb2) * nb2;
        z = nb + (int)(i / per);
        const long long rem = i - (long long)(z - nb) * per;
        y = nb + (int)(rem / nb2);
        const int s = (int)(rem - (long long)(y - nb) * nb2);
        x = s < nb ? s : nx - nb2 + s;
        return true;
    }
    return false;
}

// linear index of (x, y, z) in the slab array of axis ax
__device__ __forceinline__ long long slab_lin(const ShotDev& sd, int ax, int x, int y, int z) {
    const int nb2 = 2 * sd.nb;
    if (ax == 0) return ((long long)z * sd.ny + y) * nb2 + slab_index(x, sd.nx, sd.nb);
    if (ax == 1) return ((long long)z * nb2 + slab_index(y, sd.ny, sd.nb)) * sd.nx + x;
    return ((long long)slab_index(z, sd.nz, sd.nb) * sd.ny + y) * sd.nx + x;
}

__device__ __forceinline__ const float* prof_a(const ShotDev& sd, int ax) {
    return ax == 0 ? sd.prof : (ax == 1 ? sd.prof + 2 * sd.nx : sd.prof + 2 * sd.nx + 2 * sd.ny);
}

// psi_ax <- b psi_ax + a D1_ax p^n in the layer of each axis
__global__ __launch_bounds__(256) void k_cpml_psi(const ShotDev* __restrict__ shots, int parity, Coefs cf) {
    const ShotDev& sd = shots[blockIdx.y];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= slab_count(sd)) return;
    int x, y, z;
    if (!slab_point(sd, i, x, y, z)) return;
    const float* __restrict__ p = sd.buf[parity];
    const int pos[3] = {x, y, z};
    const int n[3] = {sd.nx, sd.ny, sd.nz};
    const long long stride[3] = {1, sd.nx, (long long)sd.nx * sd.ny};
    const long long o = (long long)z * stride[2] + (long long)y * sd.nx + x;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (!in_layer(pos[ax], n[ax], sd.nb)) continue;
        float d1 = 0.0f;
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
            const float bw = ax == 0 ? cf.bx[m - 1] : (ax == 1 ? cf.by[m - 1] : cf.bz[m - 1]);
            const float fp = pos[ax] + m < n[ax] ? p[o + m * stride[ax]] : 0.0f;
            const float fm = pos[ax] - m >= 0 ? p[o - m * stride[ax]] : 0.0f;
            d1 = fmaf(bw, fp - fm, d1);
        }
        const float* pa = prof_a(sd, ax);
        const float a = pa[pos[ax]], bb = pa[n[ax] + pos[ax]];
        float* psi = sd.psi[ax];
        const long long s = slab_lin(sd, ax, x, y, z);
        psi[s] = fmaf(bb, psi[s], a * d1);
    }
}

// zeta_ax <- b zeta_ax + a (D2_ax p^n + D1_ax psi_ax); p^{n+1} += D sum (D1 psi + zeta)
__global__ __launch_bounds__(256) void k_cpml_corr(const ShotDev* __restrict__ shots, int parity, Coefs cf) {
    const ShotDev& sd = shots[blockIdx.y];
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= slab_count(sd)) return;
    int x, y, z;
    if (!slab_point(sd, i, x, y, z)) return;
    const float* __restrict__ p = sd.buf[parity];
    float* __restrict__ pn = sd.buf[parity ^ 1];
    const int pos[3] = {x, y, z};
    const int n[3] = {sd.nx, sd.ny, sd.nz};
    const long long stride[3] = {1, sd.nx, (long long)sd.nx * sd.ny};
    const long long o = (long long)z * stride[2] + (long long)y * sd.nx + x;
    const float c = p[o];
    float corr = 0.0f;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        if (!in_layer(pos[ax], n[ax], sd.nb)) continue;
        const float* psi = sd.psi[ax];
        float d2 = 0.0f, dpsi = 0.0f;
#pragma unroll
        for (int m = 1; m <= 4; ++m) {
            const int ip = pos[ax] + m, im = pos[ax] - m;
            const float fp = ip < n[ax] ? p[o + m * stride[ax]] : 0.0f;
            const float fm = im >= 0 ? p[o - m * stride[ax]] : 0.0f;
            const float cw = ax == 0 ? cf.cx[m - 1] : (ax == 1 ? cf.cy[m - 1] : cf.cz[m - 1]);
            const float bw = ax == 0 ? cf.bx[m - 1] : (ax == 1 ? cf.by[m - 1] : cf.bz[m - 1]);
            d2 = fmaf(cw, (fp - c) + (fm - c), d2);
            int pp[3] = {x, y, z}, pm[3] = {x, y, z};
            pp[ax] = ip;
            pm[ax] = im;
            const float sp = (ip < n[ax] && in_layer(ip, n[ax], sd.nb)) ? psi[slab_lin(sd, ax, pp[0], pp[1], pp[2])] : 0.0f;
            const float sm = (im >= 0 && in_layer(im, n[ax], sd.nb)) ? psi[slab_lin(sd, ax, pm[0], pm[1], pm[2])] : 0.0f;
            dpsi = fmaf(bw, sp - sm, dpsi);
        }
        const float* pa = prof_a(sd, ax);
        const float a = pa[pos[ax]], bb = pa[n[ax] + pos[ax]];
        float* zeta = sd.zeta[ax];
        const long long s = slab_lin(sd, ax, x, y, z);
        const float zn = fmaf(bb, zeta[s], a * (d2 + dpsi));
        zeta[s] = zn;
        corr += dpsi + zn;
    }
    pn[o] = fmaf(sd.vdt2[o], corr, pn[o]);
}

hipError_t launch_cpml(const ShotDev* shots, int nshots, int max_slab_pts, int parity, const Coefs& cf,
                       hipStream_t s) {
    if (nshots <= 0 || max_slab_pts <= 0) return hipSuccess;
    dim3 grid((max_slab_pts + 255) / 256, nshots);
    k_cpml_psi<<<grid, 256, 0, s>>>(shots, parity, cf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_cpml_corr<<<grid, 256, 0, s>>>(shots, parity, cf);
    return hipGetLastError();
}

// ------------------------------------------------------- inject and gather

template <int MODE>
__global__ __launch_bounds__(256) void k_inject(InjTab tab, const ShotDev* __restrict__ shots, int parity,
                                                const float* __restrict__ vals, StepAux aux) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= tab.ncell) return;
    float acc = 0.0f;
    for (int q = tab.start[u]; q < tab.start[u + 1]; ++q) acc += vals[tab.col[q]];
    const ShotDev& sd = shots[tab.cell_shot[u]];
    const long long o = tab.cell_off[u];
    const float g = tab.cell_g[u];
    const float term = g * (sd.vdt2[o] * (tab.scale * acc));
    float* pn = sd.buf[parity ^ 1];
    pn[o] += term;
    if (MODE == MODE_D2P) aux.d2p_out[o] += term;
    if (MODE == MODE_IMAGE) aux.grad[o] = fmaf(aux.neg_inv_dt2 / g * term, aux.d2p_in[o], aux.grad[o]);
}

hipError_t launch_inject(const InjTab& tab, const ShotDev* shots, int parity, const float* vals, int ncols, int mode,
                         const StepAux& aux, hipStream_t s) {
    (void)ncols;
    if (tab.ncell <= 0) return hipSuccess;
    dim3 grid((tab.ncell + 255) / 256);
    if (mode == MODE_PLAIN)
        k_inject<MODE_PLAIN><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else if (mode == MODE_D2P)
        k_inject<MODE_D2P><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
    else
        k_inject<MODE_IMAGE><<<grid, 256, 0, s>>>(tab, shots, parity, vals, aux);
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

__global__ __launch_bounds__(256) void k_copy(float* __restrict__ d, const float* __restrict__ src, long long n) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) d[i] = src[i];
}

hipError_t launch_copy(float* dst, const float* src, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_copy<<<stride_grid(n), 256, 0, s>>>(dst, src, n);
    return hipGetLastError();
}

// ------------------------------------------------------- snapshot codec

__global__ __launch_bounds__(256) void k_absmax_part(const float* __restrict__ x, long long n,
                                                     float* __restrict__ part) {
    __shared__ float sm[256];
    float m = 0.0f;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        m = fmaxf(m, fabsf(x[i]));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ __launch_bounds__(256) void k_absmax_final(const float* __restrict__ part, int nparts,
                                                      float* __restrict__ result) {
    __shared__ float sm[256];
    float m = 0.0f;
    for (int i = threadIdx.x; i < nparts; i += 256) m = fmaxf(m, part[i]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) result[0] = sm[0] > 0.0f ? sm[0] : 1.0f;
}

hipError_t launch_absmax(const float* x, long long n, float* partial, int nparts, float* result, hipStream_t s) {
    dim3 g = stride_grid(n);
    if ((int)g.x > nparts) g.x = nparts;
    k_absmax_part<<<g, 256, 0, s>>>(x, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_absmax_final<<<1, 256, 0, s>>>(partial, (int)g.x, result);
    return hipGetLastError();
}

// float -> bfloat16, round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf_rne(float f) {
    const unsigned u = __float_as_uint(f);
    const unsigned lsb = (u >> 16) & 1u;
    return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__global__ __launch_bounds__(256) void k_pack_bf16(const float* __restrict__ x, long long n,
                                                   const float* __restrict__ scale, uint16_t* __restrict__ out) {
    const float s = scale[0];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        out[i] = f2bf_rne(x[i] / s);
}

__global__ __launch_bounds__(256) void k_unpack_bf16(const uint16_t* __restrict__ in, long long n,
                                                     const float* __restrict__ scale, float* __restrict__ x) {
    const float s = scale[0];
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        x[i] = __uint_as_float((unsigned)in[i] << 16) * s;
}

hipError_t launch_pack_bf16(const float* x, long long n, const float* scale, uint16_t* out, hipStream_t s) {
    k_pack_bf16<<<stride_grid(n), 256, 0, s>>>(x, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_unpack_bf16(const uint16_t* in, long long n, const float* scale, float* x, hipStream_t s) {
    k_unpack_bf16<<<stride_grid(n), 256, 0, s>>>(in, n, scale, x);
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

}  // namespace mm
