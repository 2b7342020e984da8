// Host runtime of the acoustic_iso_cd library: argument checks, time step,
// workspace carving, boundary and point tables, the time loop, the
// adjoint/gradient with checkpoints, HIP graph capture and the tile
// autotuner.  Every array operation runs in the kernels of mm_kernels.hip;
// this file only computes scalars and small 1D tables and enqueues work.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/minimod.h"
#include "mm_internal.h"

using namespace mm;

namespace {

// Order-8 central weights: second derivative a_m, first derivative beta_m.
const double kA2[4] = {8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};
const double kB1[4] = {4.0 / 5.0, -1.0 / 5.0, 4.0 / 105.0, -1.0 / 280.0};
// staggered order-8 first difference (acoustic_iso)
const double kS1[4] = {1225.0 / 1024.0, -245.0 / 3072.0, 49.0 / 5120.0, -5.0 / 7168.0};
const double kPi = 3.14159265358979323846;

thread_local std::string g_err;  // last error without a context

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct ShotGeom {
    int nx, ny, nz;
    long long n() const { return (long long)nx * ny * nz; }
};

// Cells per end of the CPML memory slabs: the layer width, and one more for
// acoustic_iso, whose high end has a layer face beyond the last cell.
int mem_width(const mm_params& p) { return p.model == MM_MODEL_ISO ? p.nb + 1 : p.nb; }

// Bytes one forward step of a shot touches: three fields, and for CPML the
// memory (psi, zeta) and correction slabs; acoustic_iso: two pressure fields,
// three face velocities, dt rho v^2 and rho / dt.
double shot_set_bytes(const mm_params& p, const ShotGeom& q) {
    double b = p.model == MM_MODEL_ISO ? 28.0 * q.n() : 12.0 * q.n();
    if (p.bc == MM_BC_CPML) {
        const double nb2 = 2.0 * mem_width(p);
        b += 12.0 * ((double)q.nz * q.ny * nb2 + (double)q.nz * nb2 * q.nx + nb2 * q.ny * q.nx);
    }
    return b;
}

// Infinity Cache (memory-side last-level cache) of one MI355X
constexpr double kInfinityCacheBytes = 256.0 * 1024.0 * 1024.0;

// Shot groups of a batch: consecutive shots whose working set (three
// fields, CPML memory and corrections) fits the budget; every shot alone if
// it is larger.  One group holds all shots when the budget is negative.
std::vector<std::pair<int, int>> make_groups(const mm_params& p, const std::vector<ShotGeom>& shots) {
    std::vector<std::pair<int, int>> g;
    const double budget = p.group_kb < 0 ? 1e300 : (p.group_kb == 0 ? 262144.0 : (double)p.group_kb) * 1024.0;
    int s0 = 0;
    double acc = 0.0;
    for (int s = 0; s < (int)shots.size(); ++s) {
        const double b = shot_set_bytes(p, shots[s]);
        if (s > s0 && acc + b > budget) {
            g.push_back({s0, s});
            s0 = s;
            acc = 0.0;
        }
        acc += b;
    }
    g.push_back({s0, (int)shots.size()});
    return g;
}

// Tiles of one variant over shots [s0, s1), in shot-major, z-chunk, y, x
// order; the z-chunk count aims at the variant's block target over the range.
void build_tiles_range(int variant, const std::vector<ShotGeom>& shots, int s0, int s1, std::vector<TileEnt>& out) {
    const TileShape& ts = tile_variant(variant);
    const int TX = ts.tx, TY = tile_rows(variant);
    long long xy = 0;
    for (int s = s0; s < s1; ++s) xy += (long long)((shots[s].nx + TX - 1) / TX) * ((shots[s].ny + TY - 1) / TY);
    long long nch = xy > 0 ? (ts.target + xy - 1) / xy : 1;
    if (nch < 1) nch = 1;
    for (int s = s0; s < s1; ++s) {
        const auto& g = shots[s];
        int zlen = (int)((g.nz + nch - 1) / nch);
        if (zlen < 4) zlen = 4;
        for (int z0 = 0; z0 < g.nz; z0 += zlen) {
            const int z1 = std::min(g.nz, z0 + zlen);
            for (int y0 = 0; y0 < g.ny; y0 += TY)
                for (int x0 = 0; x0 < g.nx; x0 += TX)
                    out.push_back(TileEnt{s, x0, y0, z0, z1, 0, std::min(g.nx, x0 + TX), std::min(g.ny, y0 + TY)});
        }
    }
}

// The box [bx0, bx1) x [by0, by1) x [z0, z1) of shot s cut into tw x th
// rectangles (the last ones clipped to the box) and z chunks of zlen planes.
void tile_box(int s, int bx0, int bx1, int by0, int by1, int z0, int z1, int zlen, int tw, int th,
              std::vector<TileEnt>& out) {
    if (bx1 <= bx0 || by1 <= by0 || z1 <= z0) return;
    for (int za = z0; za < z1; za += zlen) {
        const int zb = std::min(z1, za + zlen);
        for (int y = by0; y < by1; y += th)
            for (int x = bx0; x < bx1; x += tw)
                out.push_back(TileEnt{s, x, y, za, zb, 0, std::min(bx1, x + tw), std::min(by1, y + th)});
    }
}

// Forward CPML regions of a shot: the interior box [bx0, bx1) x [by0, by1) x
// [zlo, zhi) holds no layer cell (its last tiles are clipped to it; bx0 is nb
// rounded up to 32 cells, which keeps every row of its tiles on 128-byte
// lines: the stencil fetches 16.5 B per point with the box at x = 32 and
// 20.8 with it at x = 16); the frame around it in the middle z range
// [zlo, zhi) and the z-layer chunks [0, nb) (none under a free surface) and
// [nz - nb, nz) belong to the fused CPML kernel.
struct CpmlRegions {
    int bx0, bx1, by0, by1, zlo, zhi;
};

CpmlRegions cpml_regions(const ShotGeom& g, int nb, bool fs) {
    CpmlRegions r;
    r.bx0 = std::min(g.nx, (nb + 31) / 32 * 32);
    r.bx1 = std::max(r.bx0, g.nx - nb);
    r.by0 = std::min(g.ny, nb);
    r.by1 = std::max(r.by0, g.ny - nb);
    r.zlo = fs ? 0 : nb;
    r.zhi = g.nz - nb;
    return r;
}

// blocks of a group's frame launch (z-chunking of the strips, at least 16 planes each): 8192 at
// 1024^2 x 512 gives 16-plane chunks and 437 us per step, against 457 us at 2048 (50 planes) and
// 479 at 1024 (90); the frame kernel is latency-bound, so more, shorter chains beat the prologues
constexpr int kStripTarget = 8192;
// Below this many fused-kernel tiles in a group, its frame, z-layer and corner tiles go in one
// launch: each kind alone leaves most of the chip idle while its blocks march through z, and
// one launch lets the three overlap.
constexpr int kMergeTiles = 4096;

// Where the tile lists of one shot group sit in the tile table.
struct GroupTiles {
    int full_off = 0, nfull = 0;  // variant tiles over the whole grid: every step without forward CPML
    int in_off = 0, nin = 0;      // forward CPML: variant tiles of the interior boxes
    int st_off = 0, nst = 0;      // forward CPML: fused tiles of the frames (middle z range)
    int zl_off = 0, nzl = 0;      // forward CPML: fused tiles of the z-layer chunks that meet no x / y layer
    int zc_off = 0, nzc = 0;      // forward CPML: fused tiles of the z-layer chunks that meet one
    // the frame, z-layer and corner lists (consecutive) run as one launch: fewer than kMergeTiles
    // tiles, all in the corner shape
    bool one = false;
    bool merged() const { return one; }
};

// Every tile list: the full lists of all groups first (so that one launch
// over [0, sum of nfull) covers every shot), then for forward CPML the
// interior, frame and z-layer lists of each group.
void build_tiles(int variant, const mm_params& p, const std::vector<ShotGeom>& shots,
                 const std::vector<std::pair<int, int>>& groups, std::vector<TileEnt>& out,
                 std::vector<GroupTiles>& gt) {
    out.clear();
    gt.assign(groups.size(), GroupTiles());
    for (size_t k = 0; k < groups.size(); ++k) {
        gt[k].full_off = (int)out.size();
        build_tiles_range(variant, shots, groups[k].first, groups[k].second, out);
        gt[k].nfull = (int)out.size() - gt[k].full_off;
    }
    if (p.bc != MM_BC_CPML || p.model != MM_MODEL_ISO_CD) return;
    const int TX = tile_variant(variant).tx, TY = tile_rows(variant);
    const int CW = cstep_tile_w(CS_FRAME), CH = cstep_tile_h(CS_FRAME), nb = p.nb;
    const int ZW = cstep_tile_w(CS_ZLAYER), ZH = cstep_tile_h(CS_ZLAYER);
    const int CZW = cstep_tile_w(CS_ZCORNER), CZH = cstep_tile_h(CS_ZCORNER);
    const bool fs = p.free_surface != 0;
    for (size_t k = 0; k < groups.size(); ++k) {
        const int s0 = groups[k].first, s1 = groups[k].second;
        // interior boxes, z-chunked towards the variant's block target
        long long xy = 0, sxy = 0;
        for (int s = s0; s < s1; ++s) {
            const CpmlRegions r = cpml_regions(shots[s], nb, fs);
            xy += (long long)((r.bx1 - r.bx0 + TX - 1) / TX) * ((r.by1 - r.by0 + TY - 1) / TY);
            const int nx = shots[s].nx, ny = shots[s].ny;
            sxy += (long long)((r.bx0 + CW - 1) / CW + (nx - r.bx1 + CW - 1) / CW) * ((ny + CH - 1) / CH) +
                   (long long)((r.bx1 - r.bx0 + CW - 1) / CW) * ((r.by0 + CH - 1) / CH + (ny - r.by1 + CH - 1) / CH);
        }
        const long long nch = std::max(1LL, xy > 0 ? (tile_variant(variant).target + xy - 1) / xy : 1);
        const long long sch = std::max(1LL, sxy > 0 ? (kStripTarget + sxy - 1) / sxy : 1);
        gt[k].in_off = (int)out.size();
        for (int s = s0; s < s1; ++s) {
            const CpmlRegions r = cpml_regions(shots[s], nb, fs);
            const int zlen = std::max(4, (int)((r.zhi - r.zlo + nch - 1) / nch));
            tile_box(s, r.bx0, r.bx1, r.by0, r.by1, r.zlo, r.zhi, zlen, TX, TY, out);
        }
        gt[k].nin = (int)out.size() - gt[k].in_off;
        gt[k].st_off = (int)out.size();
        for (int s = s0; s < s1; ++s) {
            const CpmlRegions r = cpml_regions(shots[s], nb, fs);
            const int nx = shots[s].nx, ny = shots[s].ny;
            const int zlen = std::max(16, (int)((r.zhi - r.zlo + sch - 1) / sch));
            tile_box(s, 0, r.bx0, 0, ny, r.zlo, r.zhi, zlen, CW, CH, out);         // low x
            tile_box(s, r.bx1, nx, 0, ny, r.zlo, r.zhi, zlen, CW, CH, out);        // high x
            tile_box(s, r.bx0, r.bx1, 0, r.by0, r.zlo, r.zhi, zlen, CW, CH, out);  // low y
            tile_box(s, r.bx0, r.bx1, r.by1, ny, r.zlo, r.zhi, zlen, CW, CH, out); // high y
        }
        gt[k].nst = (int)out.size() - gt[k].st_off;
        // z-layer chunks: the box away from the x / y layers (the interior box's xy range) in
        // tiles of the z-layer kind, the frame around it in corner tiles; a group with few fused
        // tiles runs all of them in one launch of the corner instantiation, so then its z-layer
        // box takes the corner shape too
        auto zlayer = [&](int w, int h) {
            gt[k].zl_off = (int)out.size();
            for (int s = s0; s < s1; ++s) {
                const ShotGeom& g = shots[s];
                const CpmlRegions r = cpml_regions(g, nb, fs);
                if (!fs) tile_box(s, r.bx0, r.bx1, r.by0, r.by1, 0, nb, nb, w, h, out);
                tile_box(s, r.bx0, r.bx1, r.by0, r.by1, g.nz - nb, g.nz, nb, w, h, out);
            }
            gt[k].nzl = (int)out.size() - gt[k].zl_off;
            gt[k].zc_off = (int)out.size();
            for (int s = s0; s < s1; ++s) {
                const ShotGeom& g = shots[s];
                const CpmlRegions r = cpml_regions(g, nb, fs);
                for (int c = 0; c < 2; ++c) {
                    if (c == 0 && fs) continue;
                    const int za = c == 0 ? 0 : g.nz - nb, zb = c == 0 ? nb : g.nz;
                    tile_box(s, 0, r.bx0, 0, g.ny, za, zb, nb, CZW, CZH, out);         // low x
                    tile_box(s, r.bx1, g.nx, 0, g.ny, za, zb, nb, CZW, CZH, out);      // high x
                    tile_box(s, r.bx0, r.bx1, 0, r.by0, za, zb, nb, CZW, CZH, out);    // low y
                    tile_box(s, r.bx0, r.bx1, r.by1, g.ny, za, zb, nb, CZW, CZH, out); // high y
                }
            }
            gt[k].nzc = (int)out.size() - gt[k].zc_off;
        };
        zlayer(CZW, CZH);
        gt[k].one = gt[k].nst + gt[k].nzl + gt[k].nzc < kMergeTiles && CW == CZW && CH == CZH;
        if (!gt[k].one && (ZW != CZW || ZH != CZH)) {
            out.resize(gt[k].zl_off);
            zlayer(ZW, ZH);
        }
    }
}

struct Layout {
    size_t total = 0;
    size_t shots_dev = 0, shots_adj = 0, tiles = 0, scratch = 0;
    int max_tiles = 0;
    std::vector<size_t> buf0, buf1, vdt2, prof, ebuf0, ebuf1;
    std::vector<size_t> psi[3], psi2[3], zeta[3], corr[3];
    std::vector<size_t> apsi[3], azeta[3], acorr[3];  // CPML adjoint memory and corrections
    std::vector<size_t> iso_u[3], iso_b;              // acoustic_iso face velocities, rho / dt
    size_t src_shot = 0, src_off = 0, src_start = 0, src_col = 0, src_g = 0;
    size_t rin_shot = 0, rin_off = 0, rin_start = 0, rin_col = 0, rin_g = 0;
    size_t rg_shot = 0, rg_off = 0, sg_shot = 0, sg_off = 0;
    size_t cpml_off = 0;  // CPML block tables: per group (forward), then all shots (adjoint)
    bool adjoint = false, grad = false;
    int nseg = 0;
    size_t seg = 0, ckpt = 0, ckpt_scale = 0, ckpt_scale_n = 0, wav_store = 0, tr_store = 0, resid_store = 0;
    size_t ckpt_field_bytes = 0;
    size_t ckpt_mem = 0, ckpt_mem_bytes = 0;  // CPML memory of each checkpoint (FP32)
};

const int kPartials = 2048;  // reduction partial slots

size_t take(Layout& L, size_t bytes) {
    const size_t off = L.total;
    L.total += align256(bytes ? bytes : 1);
    return off;
}

void compute_layout(const mm_params& p, const std::vector<ShotGeom>& shots, int nsrc, int nrec, Layout& L) {
    L = Layout();
    const int S = (int)shots.size();
    L.shots_dev = take(L, sizeof(ShotDev) * S);
    L.shots_adj = take(L, sizeof(ShotDev) * S);
    int mt = 0;
    std::vector<TileEnt> tmp;
    std::vector<GroupTiles> gt;
    const auto groups = make_groups(p, shots);
    for (int v = 0; v < num_tile_variants(); ++v) {
        build_tiles(v, p, shots, groups, tmp, gt);
        mt = std::max(mt, (int)tmp.size());
    }
    L.max_tiles = mt;
    L.tiles = take(L, sizeof(TileEnt) * mt);
    // scratch: vcheck (2 u32), loss partials + loss
    L.scratch = take(L, 64 + sizeof(double) * (kPartials + 2));
    L.adjoint = p.ckpt_every > 0;
    L.grad = L.adjoint && S == 1;
    for (int s = 0; s < S; ++s) {
        const auto& g = shots[s];
        const size_t fb = sizeof(float) * (size_t)g.n();
        L.buf0.push_back(take(L, fb));
        L.buf1.push_back(take(L, fb));
        L.vdt2.push_back(take(L, fb));
        const int np = (p.bc == MM_BC_CPML ? (p.model == MM_MODEL_ISO ? 4 : 2) : 1) * (g.nx + g.ny + g.nz);
        L.prof.push_back(take(L, sizeof(float) * np));
        const size_t nb2 = 2 * (size_t)std::max(mem_width(p), 0);
        const size_t sl[3] = {(size_t)g.nz * g.ny * nb2, (size_t)g.nz * nb2 * g.nx, nb2 * g.ny * g.nx};
        const size_t w2 = 2 * (size_t)std::max(p.nb, 0) + 8;  // adjoint corrections: nb + 4 cells per end
        const size_t wl[3] = {(size_t)g.nz * g.ny * w2, (size_t)g.nz * w2 * g.nx, w2 * g.ny * g.nx};
        const bool c = p.bc == MM_BC_CPML, ca = c && L.adjoint;
        for (int a = 0; a < 3; ++a) {
            L.psi[a].push_back(c ? take(L, sizeof(float) * sl[a]) : 0);
            L.zeta[a].push_back(c ? take(L, sizeof(float) * sl[a]) : 0);
            // the second psi buffer of the forward CPML step and the layer pass's corrections
            // (acoustic_iso updates its memory in place and needs neither)
            L.psi2[a].push_back(c && p.model != MM_MODEL_ISO ? take(L, sizeof(float) * sl[a]) : 0);
            L.corr[a].push_back(c && p.model != MM_MODEL_ISO ? take(L, sizeof(float) * sl[a]) : 0);
            L.apsi[a].push_back(ca ? take(L, sizeof(float) * sl[a]) : 0);
            L.azeta[a].push_back(ca ? take(L, sizeof(float) * sl[a]) : 0);
            L.acorr[a].push_back(ca ? take(L, sizeof(float) * wl[a]) : 0);
        }
        L.ebuf0.push_back(L.adjoint ? take(L, fb) : 0);
        L.ebuf1.push_back(L.adjoint ? take(L, fb) : 0);
        const bool iso = p.model == MM_MODEL_ISO;
        for (int a = 0; a < 3; ++a) L.iso_u[a].push_back(iso ? take(L, fb) : 0);
        L.iso_b.push_back(iso ? take(L, fb) : 0);
    }
    L.src_shot = take(L, sizeof(int) * nsrc);
    L.src_off = take(L, sizeof(long long) * nsrc);
    L.src_start = take(L, sizeof(int) * (nsrc + 1));
    L.src_col = take(L, sizeof(int) * nsrc);
    L.src_g = take(L, sizeof(float) * nsrc);
    L.rin_shot = take(L, sizeof(int) * nrec);
    L.rin_off = take(L, sizeof(long long) * nrec);
    L.rin_start = take(L, sizeof(int) * (nrec + 1));
    L.rin_col = take(L, sizeof(int) * nrec);
    L.rin_g = take(L, sizeof(float) * nrec);
    L.rg_shot = take(L, sizeof(int) * nrec);
    L.rg_off = take(L, sizeof(long long) * nrec);
    L.sg_shot = take(L, sizeof(int) * nsrc);
    L.sg_off = take(L, sizeof(long long) * nsrc);
    // block tables of the CPML layer kernels: the adjoint's (every shot), then one per group (forward)
    L.cpml_off = take(L, sizeof(int) * 3 * (2 * S + 1 + (int)groups.size()));
    if (L.grad) {
        const long long N = shots[0].n();
        const int K = p.ckpt_every;
        L.nseg = (p.nsteps_max + K - 1) / K;
        // the replay's d2p fields: bfloat16 with BF16 snapshots, float otherwise
        L.seg = take(L, (p.snap == MM_SNAP_BF16 ? 2 : 4) * (size_t)K * N);
        L.ckpt_field_bytes = align256((p.snap == MM_SNAP_BF16 ? 2 : 4) * (size_t)N);
        L.ckpt = take(L, (size_t)L.nseg * 2 * L.ckpt_field_bytes);
        // BF16: two scales per block of SNAP_BLOCK cells per checkpoint
        L.ckpt_scale_n = p.snap == MM_SNAP_BF16 ? (size_t)snap_blocks(N) : 0;
        L.ckpt_scale = take(L, sizeof(float) * 2 * L.ckpt_scale_n * L.nseg);
        if (p.bc == MM_BC_CPML) {
            const auto& g = shots[0];
            const size_t nb2 = 2 * (size_t)p.nb;
            L.ckpt_mem_bytes = 2 * sizeof(float) * ((size_t)g.nz * g.ny * nb2 + (size_t)g.nz * nb2 * g.nx + nb2 * g.ny * g.nx);
            L.ckpt_mem = take(L, (size_t)L.nseg * L.ckpt_mem_bytes);
        }
        L.wav_store = take(L, sizeof(float) * (size_t)p.nsteps_max * nsrc);
        L.tr_store = take(L, sizeof(float) * (size_t)p.nsteps_max * nrec);
        L.resid_store = take(L, sizeof(float) * (size_t)p.nsteps_max * nrec);
    }
}

// Depth of index k inside a layer of nb cells at either end of n cells:
// nb at the outermost cell, 1 at the innermost layer cell, 0 inside.
int layer_depth(int k, int n, int nb) {
    const int d = std::max(nb - k, nb - (n - 1 - k));
    return d > 0 ? d : 0;
}

void sponge_table(int n, int nb, double sigma, float* out) {
    for (int k = 0; k < n; ++k) {
        const int d = layer_depth(k, n, nb);
        const double x = sigma * d;
        out[k] = d > 0 ? (float)std::exp(-x * x) : 1.0f;
    }
}

void cpml_table(int n, int nb, double h, double dt, double vmax, double R, double f0, float* a, float* b) {
    const double d0 = -3.0 * vmax * std::log(R) / (2.0 * nb * h);
    for (int k = 0; k < n; ++k) {
        const int dep = layer_depth(k, n, nb);
        if (dep == 0) {
            a[k] = 0.0f;
            b[k] = 1.0f;
            continue;
        }
        const double q = (double)dep / nb;
        const double d = d0 * q * q;
        const double al = kPi * f0 * (1.0 - q);
        const double bb = std::exp(-(d + al) * dt);
        b[k] = (float)bb;
        a[k] = (d + al) > 0.0 ? (float)(d * (bb - 1.0) / (d + al)) : 0.0f;
    }
}

// The same at the faces i + 1/2 of a staggered axis (acoustic_iso): depth
// nb - i - 1/2 in the low layer, i + 1/2 - (n - 1 - nb) in the high one, q
// clamped to 1 (the face beyond the last cell).
void cpml_face_table(int n, int nb, double h, double dt, double vmax, double R, double f0, float* a, float* b) {
    const double d0 = -3.0 * vmax * std::log(R) / (2.0 * nb * h);
    for (int k = 0; k < n; ++k) {
        const double dep = std::max(nb - k - 0.5, k + 0.5 - (n - 1 - nb));
        if (dep <= 0.0) {
            a[k] = 0.0f;
            b[k] = 1.0f;
            continue;
        }
        const double q = std::min(1.0, dep / nb);
        const double d = d0 * q * q;
        const double al = kPi * f0 * (1.0 - q);
        const double bb = std::exp(-(d + al) * dt);
        b[k] = (float)bb;
        a[k] = (d + al) > 0.0 ? (float)(d * (bb - 1.0) / (d + al)) : 0.0f;
    }
}

double dt_stab(const mm_params& p, double vmax) {
    const double sum = 1.0 / (p.dx * p.dx) + 1.0 / (p.dy * p.dy) + 1.0 / (p.dz * p.dz);
    if (p.model == MM_MODEL_ISO) {
        // staggered leapfrog: the checkerboard symbol of D+ is 2 C / h, C = c1 - c2 + c3 - c4
        const double C = kS1[0] - kS1[1] + kS1[2] - kS1[3];
        return 1.0 / (C * vmax * std::sqrt(sum));
    }
    const double S = 4.0 * (kA2[0] + kA2[2]);
    return 2.0 / (vmax * std::sqrt(S * sum));
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

struct GraphKey {
    int nsteps = -1;
    const float* wav = nullptr;
    float* tr = nullptr;
    int step = -1;
    int variant = -1;
    bool ckpt = false;  // the captured steps store checkpoints (and the wavelet for the replay)
    bool operator==(const GraphKey& o) const {
        return nsteps == o.nsteps && wav == o.wav && tr == o.tr && step == o.step && variant == o.variant &&
               ckpt == o.ckpt;
    }
};

struct mm_ctx {
    mm_params p{};
    hipStream_t stream = nullptr;
    double dt = 0.0, vmax = 0.0;
    std::vector<ShotGeom> geom;
    std::vector<ShotDev> shots_h, shots_adj_h;
    Layout L;
    char* ws = nullptr;
    ShotDev* d_shots = nullptr;
    ShotDev* d_shots_adj = nullptr;
    TileEnt* d_tiles = nullptr;
    std::vector<TileEnt> tiles_h;
    int nfull = 0, variant = 0;  // nfull: tiles of the full lists of all groups (the table's head)
    InjTab src_inj{}, rec_inj{};
    GatherTab rec_gather{}, src_gather{};
    int nsrc = 0, nrec = 0;
    struct Group {
        int s0, s1;            // shots [s0, s1)
        GroupTiles t;          // its slices of the tile table
        int rec0, rec1;        // receivers (columns of a trace row)
        int cell0, cell1;      // source cells of the injection table
        bool stream = false;   // working set beyond the Infinity Cache (StepAux::stream_loads)
        std::vector<int> cpml_h;   // block table of the layer pass over the group's shots (host copy)
        const int* cpml_d = nullptr;
    };
    std::vector<Group> groups;
    // forward CPML strategy (acoustic_iso_cd): the layer pass, then the stencil over the whole
    // grid adding its corrections (true); or the interior stencil and the fused kernel over the
    // cells near the faces (false)
    bool layer_pass = false;
    bool stream_all = false;      // the same for all shots together (adjoint steps)
    std::vector<int> cpml_adj_h;  // CPML block table of the adjoint (all shots, width nb + 4)
    const int* cpml_adj_d = nullptr;
    bool inline_src = false;
    std::vector<std::vector<long long>> src_cells;  // per shot, for tile flags
    Coefs cf{};
    bool sponge = false, cpml = false;
    bool iso = false;  // acoustic_iso (staggered first-order system)
    // time state
    int step = 0;
    bool fwd_valid = true;
    // gradient / adjoint
    bool ckpt_active = false;
    bool adj_started = false;
    bool adj_grad = false;
    int adj_T = 0, adj_j = 0, seg_loaded = -1;
    // scratch pointers
    unsigned* vcheck = nullptr;
    unsigned* watch = nullptr;  // watchdog flag and first bad step (scratch words 4, 5)
    double* loss_part = nullptr;
    double* loss_dev = nullptr;
    // graph
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    GraphKey gkey;
    std::string err;
    // host tables kept alive until their uploads complete
    std::vector<char> host_tables;
    // mm_init_static: the device whose static workspace holds the context, and the
    // take-over count of that workspace when the context was made (0: caller's workspace)
    int static_dev = -1;
    unsigned long long static_gen = 0;
    // stencil timing
    int prof_stride = 0;
    long long prof_count = 0;
    std::vector<hipEvent_t> prof_ev;
    size_t prof_used = 0;
};

namespace {

mm_status fail(mm_ctx* c, mm_status s, const std::string& msg) {
    if (c) c->err = msg;
    g_err = msg;
    return s;
}

mm_status dev(mm_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return MM_OK;
    return fail(c, MM_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Take-overs of each GPU's static workspace: a context made by mm_init_static
// stays usable until the next mm_init_static on the same GPU.
std::mutex g_static_mu;
unsigned long long g_static_gen[64] = {};

mm_status live(mm_ctx* c) {
    if (!c || c->static_dev < 0) return MM_OK;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_gen[c->static_dev] != c->static_gen)
        return fail(c, MM_ERR_STATE, "the static workspace of this GPU was taken over by a later mm_init_static");
    return MM_OK;
}

#define MM_TRY(expr)                 \
    do {                             \
        mm_status _s = (expr);       \
        if (_s != MM_OK) return _s;  \
    } while (0)

template <class T>
T* at(char* ws, size_t off) {
    return reinterpret_cast<T*>(ws + off);
}

mm_status check_params(const mm_params* p, mm_ctx* c) {
    if (!p) return fail(c, MM_ERR_ARG, "params is NULL");
    if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz))
        return fail(c, MM_ERR_ARG, "grid spacing must be finite and > 0");
    if (p->bc < MM_BC_NONE || p->bc > MM_BC_CPML) return fail(c, MM_ERR_ARG, "unknown boundary kind");
    if (p->bc != MM_BC_NONE && p->nb < 1) return fail(c, MM_ERR_ARG, "damping width nb must be >= 1");
    if (p->nb < 0 || p->nb > 4096) return fail(c, MM_ERR_ARG, "damping width nb out of range");
    if (p->bc == MM_BC_CPML && p->nb > 128) return fail(c, MM_ERR_ARG, "CPML width nb must be <= 128");
    if (p->bc == MM_BC_CPML && p->ckpt_every > 0 && p->nb > 64)
        return fail(c, MM_ERR_ARG, "CPML width nb must be <= 64 with adjoint storage (ckpt_every > 0)");
    if (p->bc == MM_BC_SPONGE && !(std::isfinite(p->sponge_sigma) && p->sponge_sigma >= 0.0))
        return fail(c, MM_ERR_ARG, "sponge_sigma must be finite and >= 0");
    if (p->bc == MM_BC_CPML && !(std::isfinite(p->cpml_R) && p->cpml_R > 0.0 && p->cpml_R <= 1.0))
        return fail(c, MM_ERR_ARG, "cpml_R must be in (0, 1]");
    if (p->bc == MM_BC_CPML && !(std::isfinite(p->cpml_f0) && p->cpml_f0 >= 0.0))
        return fail(c, MM_ERR_ARG, "cpml_f0 must be finite and >= 0");
    if (!(std::isfinite(p->dt) && p->dt >= 0.0)) return fail(c, MM_ERR_ARG, "dt must be finite and >= 0");
    if (p->dt == 0.0 && !(std::isfinite(p->cfl) && p->cfl > 0.0)) return fail(c, MM_ERR_ARG, "cfl must be > 0");
    if (!(std::isfinite(p->vmax) && p->vmax >= 0.0)) return fail(c, MM_ERR_ARG, "vmax must be finite and >= 0");
    if (p->ckpt_every < 0) return fail(c, MM_ERR_ARG, "ckpt_every must be >= 0");
    if (p->ckpt_every > 0 && p->nsteps_max < 1) return fail(c, MM_ERR_ARG, "nsteps_max must be >= 1");
    if (p->snap != MM_SNAP_FP32 && p->snap != MM_SNAP_BF16) return fail(c, MM_ERR_ARG, "unknown snapshot kind");
    if (p->tile < -1 || p->tile >= num_tile_variants()) return fail(c, MM_ERR_ARG, "unknown tile variant");
    if (p->group_kb < -1) return fail(c, MM_ERR_ARG, "group_kb must be >= -1");
    if (p->free_surface != 0 && p->free_surface != 1) return fail(c, MM_ERR_ARG, "free_surface must be 0 or 1");
    if (p->model != MM_MODEL_ISO_CD && p->model != MM_MODEL_ISO) return fail(c, MM_ERR_ARG, "unknown model");
    if (p->cache_hints < 0 || p->cache_hints > 2) return fail(c, MM_ERR_ARG, "cache_hints must be 0, 1 or 2");
    if (p->watch_every < 0) return fail(c, MM_ERR_ARG, "watch_every must be >= 0");
    if (p->cpml_kernel < 0 || p->cpml_kernel > 2) return fail(c, MM_ERR_ARG, "cpml_kernel must be 0, 1 or 2");
    if (p->model == MM_MODEL_ISO) {
        if (p->ckpt_every > 0) return fail(c, MM_ERR_UNSUPPORTED, "acoustic_iso has no adjoint (ckpt_every must be 0)");
        if (p->tile > 0 && !iso_variant_ok(p->tile))
            return fail(c, MM_ERR_ARG, "acoustic_iso runs the 256-thread tile variants only");
    }
    return MM_OK;
}

mm_status check_shot(const mm_params* p, const mm_shot& s, int idx, bool need_vel, mm_ctx* c) {
    char buf[160];
    const int n[3] = {s.nx, s.ny, s.nz};
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1 || n[a] > (1 << 20)) {
            snprintf(buf, sizeof buf, "shot %d: grid size %d out of range", idx, n[a]);
            return fail(c, MM_ERR_ARG, buf);
        }
        // the two layers of an axis must not overlap; CPML also keeps them a stencil radius apart,
        // and its adjoint (whose correction reaches 4 cells past each layer) two radii
        const bool cadj = p->bc == MM_BC_CPML && p->ckpt_every > 0;
        const int nmin = p->bc == MM_BC_CPML ? 2 * p->nb + (cadj ? 8 : 4) : 2 * p->nb + 1;
        if (p->bc != MM_BC_NONE && n[a] < nmin) {
            snprintf(buf, sizeof buf, "shot %d: grid size %d < %s = %d", idx, n[a],
                     p->bc == MM_BC_CPML ? (cadj ? "2*nb+8 (CPML with adjoint storage)" : "2*nb+4") : "2*nb+1",
                     nmin);
            return fail(c, MM_ERR_ARG, buf);
        }
    }
    if ((long long)s.nx * s.ny * s.nz > (1LL << 34)) return fail(c, MM_ERR_ARG, "grid too large");
    if ((long long)s.nx * s.ny >= (1LL << 30)) return fail(c, MM_ERR_ARG, "grid plane nx*ny must be < 2^30");
    if (p->bc == MM_BC_CPML && (s.ny > 65535 || s.nz > 65535 || (long long)s.ny * s.nz > (1LL << 30)))
        return fail(c, MM_ERR_ARG, "CPML grids need ny, nz <= 65535");
    if (need_vel && !s.vel) return fail(c, MM_ERR_ARG, "velocity pointer is NULL");
    if (need_vel && p->model == MM_MODEL_ISO && !s.rho) return fail(c, MM_ERR_ARG, "acoustic_iso needs a density model");
    if (s.nsrc < 0 || s.nrec < 0) return fail(c, MM_ERR_ARG, "negative source/receiver count");
    if ((s.nsrc > 0 && !s.src_ijk) || (s.nrec > 0 && !s.rec_ijk))
        return fail(c, MM_ERR_ARG, "source/receiver list is NULL");
    for (int q = 0; q < s.nsrc + s.nrec; ++q) {
        const int32_t* t = q < s.nsrc ? s.src_ijk + 3 * q : s.rec_ijk + 3 * (q - s.nsrc);
        if (t[0] < 0 || t[1] < 0 || t[2] < 0 || t[0] >= s.nx || t[1] >= s.ny || t[2] >= s.nz) {
            snprintf(buf, sizeof buf, "shot %d: %s %d at (%d,%d,%d) outside the %dx%dx%d grid", idx,
                     q < s.nsrc ? "source" : "receiver", q < s.nsrc ? q : q - s.nsrc, t[0], t[1], t[2], s.nx, s.ny,
                     s.nz);
            return fail(c, MM_ERR_ARG, buf);
        }
    }
    return MM_OK;
}

mm_status totals(const mm_params* p, int32_t nshots, const mm_shot* shots, bool need_vel, std::vector<ShotGeom>& g,
                 int& nsrc, int& nrec, mm_ctx* c) {
    if (nshots < 1 || !shots) return fail(c, MM_ERR_ARG, "need at least one shot");
    g.clear();
    long long ns = 0, nr = 0;
    for (int s = 0; s < nshots; ++s) {
        MM_TRY(check_shot(p, shots[s], s, need_vel, c));
        g.push_back(ShotGeom{shots[s].nx, shots[s].ny, shots[s].nz});
        ns += shots[s].nsrc;
        nr += shots[s].nrec;
    }
    if (ns > (1 << 28) || nr > (1 << 28)) return fail(c, MM_ERR_ARG, "too many sources or receivers");
    nsrc = (int)ns;
    nrec = (int)nr;
    return MM_OK;
}

// CSR of unique cells for point injection.
struct Csr {
    std::vector<int> shot, start, col;
    std::vector<long long> off;
    std::vector<float> g;
};

void build_csr(const std::vector<int>& shot, const std::vector<long long>& off, const std::vector<float>& gval,
               Csr& out) {
    const int n = (int)shot.size();
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
        return shot[a] != shot[b] ? shot[a] < shot[b] : off[a] < off[b];
    });
    out = Csr();
    for (int q = 0; q < n; ++q) {
        const int i = idx[q];
        if (q == 0 || shot[i] != out.shot.back() || off[i] != out.off.back()) {
            out.shot.push_back(shot[i]);
            out.off.push_back(off[i]);
            out.g.push_back(gval[i]);
            out.start.push_back(q);
        }
        out.col.push_back(i);
    }
    out.start.push_back(n);
}

mm_status upload(mm_ctx* c, void* dst, const void* src, size_t bytes) {
    if (bytes == 0) return MM_OK;
    return dev(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream), "upload");
}

// Flags of the tiles [a, b) of the table: the cells a tile writes meet the
// damping layers of width w of an axis (CPML), or hold an inline source.
// zflag: TF_LZ (every tile of the list is a z-layer chunk), 0 (from the
// tile's z range) or -1 (never: the frame and interior lists).
void tile_flags(mm_ctx* c, int a, int b, int w, int zflag) {
    auto meets = [w](int a0, int a1, int n) { return a0 < w || a1 > n - w; };  // [a0, a1) vs the layers
    for (int i = a; i < b; ++i) {
        TileEnt& t = c->tiles_h[i];
        const ShotGeom& g = c->geom[t.shot];
        int f = zflag > 0 ? zflag : 0;
        if (c->cpml) {
            if (meets(t.x0, t.x1, g.nx)) f |= TF_LX;
            if (meets(t.y0, t.y1, g.ny)) f |= TF_LY;
            if (zflag == 0 && meets(t.z0, t.z1, g.nz)) f |= TF_LZ;
        }
        if (c->inline_src)
            for (long long o : c->src_cells[t.shot]) {
                const int z = (int)(o / ((long long)g.nx * g.ny));
                const int y = (int)((o / g.nx) % g.ny), x = (int)(o % g.nx);
                if (x >= t.x0 && x < t.x1 && y >= t.y0 && y < t.y1 && z >= t.z0 && z < t.z1) f |= TF_SRC;
            }
        t.flags = f;
    }
}

mm_status set_variant(mm_ctx* c, int v) {
    std::vector<std::pair<int, int>> gr;
    for (const auto& g : c->groups) gr.push_back({g.s0, g.s1});
    std::vector<GroupTiles> gt;
    build_tiles(v, c->p, c->geom, gr, c->tiles_h, gt);
    c->nfull = 0;
    for (size_t i = 0; i < c->groups.size(); ++i) {
        const GroupTiles& t = gt[i];
        c->groups[i].t = t;
        c->nfull += t.nfull;
        // full lists: the adjoint's correction slabs reach nb + 4 cells per end
        // (acoustic_iso: its memory slabs, one cell wider than the layer)
        tile_flags(c, t.full_off, t.full_off + t.nfull, c->iso ? mem_width(c->p) : c->p.nb + (c->L.adjoint ? 4 : 0),
                   0);
        tile_flags(c, t.in_off, t.in_off + t.nin, c->p.nb, -1);
        tile_flags(c, t.st_off, t.st_off + t.nst, c->p.nb, -1);
        tile_flags(c, t.zl_off, t.zl_off + t.nzl, c->p.nb, TF_LZ);
        tile_flags(c, t.zc_off, t.zc_off + t.nzc, c->p.nb, TF_LZ);
    }
    if ((int)c->tiles_h.size() > c->L.max_tiles) return fail(c, MM_ERR_WORKSPACE, "tile table overflow");
    MM_TRY(dev(c, hipStreamSynchronize(c->stream), "sync"));
    MM_TRY(upload(c, c->d_tiles, c->tiles_h.data(), sizeof(TileEnt) * c->tiles_h.size()));
    MM_TRY(dev(c, hipStreamSynchronize(c->stream), "sync"));
    c->variant = v;
    return MM_OK;
}

void drop_graph(mm_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->gexec = nullptr;
    c->graph = nullptr;
    c->gkey = GraphKey();
}

mm_status zero_state(mm_ctx* c, hipStream_t s) {
    MM_TRY(dev(c, launch_watch_reset(c->watch, s), "watch reset"));
    for (size_t i = 0; i < c->geom.size(); ++i) {
        const long long n = c->geom[i].n();
        const ShotDev& sd = c->shots_h[i];
        if (c->iso)
            for (int a = 0; a < 3; ++a) MM_TRY(dev(c, launch_fill(sd.u[a], n, 0.0f, s), "fill"));
        MM_TRY(dev(c, launch_fill(sd.buf[0], n, 0.0f, s), "fill"));
        MM_TRY(dev(c, launch_fill(sd.buf[1], n, 0.0f, s), "fill"));
        if (c->cpml) {
            const long long nb2 = 2LL * mem_width(c->p);
            const long long sl[3] = {(long long)c->geom[i].nz * c->geom[i].ny * nb2,
                                     (long long)c->geom[i].nz * nb2 * c->geom[i].nx,
                                     nb2 * c->geom[i].ny * c->geom[i].nx};
            for (int a = 0; a < 3; ++a) {
                MM_TRY(dev(c, launch_fill(sd.psi[a], sl[a], 0.0f, s), "fill"));
                if (!c->iso) MM_TRY(dev(c, launch_fill(sd.psi2[a], sl[a], 0.0f, s), "fill"));
                MM_TRY(dev(c, launch_fill(sd.zeta[a], sl[a], 0.0f, s), "fill"));
            }
        }
    }
    return MM_OK;
}

mm_status zero_adjoint(mm_ctx* c, hipStream_t s) {
    for (size_t i = 0; i < c->geom.size(); ++i) {
        const long long n = c->geom[i].n();
        MM_TRY(dev(c, launch_fill(c->shots_adj_h[i].buf[0], n, 0.0f, s), "fill"));
        MM_TRY(dev(c, launch_fill(c->shots_adj_h[i].buf[1], n, 0.0f, s), "fill"));
        if (c->cpml) {
            const long long nb2 = 2LL * c->p.nb;
            const auto& g = c->geom[i];
            const long long sl[3] = {(long long)g.nz * g.ny * nb2, (long long)g.nz * nb2 * g.nx, nb2 * g.ny * g.nx};
            for (int a = 0; a < 3; ++a) {
                MM_TRY(dev(c, launch_fill(c->shots_adj_h[i].psi[a], sl[a], 0.0f, s), "fill"));
                MM_TRY(dev(c, launch_fill(c->shots_adj_h[i].zeta[a], sl[a], 0.0f, s), "fill"));
            }
        }
    }
    return MM_OK;
}

// Watchdog schedule: the state after `steps_done` forward steps is scanned
// when watch_every divides it.
bool watch_due(int steps_done, int watch_every) { return watch_every > 0 && steps_done > 0 && steps_done % watch_every == 0; }

// Watchdog result from its two device words {flag, first bad step}.
mm_status watch_result(const unsigned w[2], int32_t* bad_step, std::string* msg) {
    if (!(w[0] & 1u)) {
        if (bad_step) *bad_step = -1;
        return MM_OK;
    }
    const int32_t b = w[1] > 0x7FFFFFFFu ? -1 : (int32_t)w[1];
    if (bad_step) *bad_step = b;
    if (msg) *msg = "non-finite wavefield (NaN or Inf) first seen in the state after step " + std::to_string(b);
    return MM_ERR_NONFINITE;
}

// One leapfrog step of the forward (or adjoint) field set, for the shots of
// group g (nullptr: every shot in one launch; forward CPML needs a group).
mm_status enqueue_step(mm_ctx* c, const ShotDev* shots, int parity, int mode, const StepAux& aux, hipStream_t s,
                       const mm_ctx::Group* g) {
    const bool timed = c->prof_stride > 0 && s == c->stream && (c->prof_count++ % c->prof_stride) == 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (timed) {
        // the step's first kernel stamps its start into ev0, the last its end into ev1
        while (c->prof_ev.size() < c->prof_used + 2) {
            hipEvent_t e;
            MM_TRY(dev(c, hipEventCreate(&e), "event"));
            c->prof_ev.push_back(e);
        }
        ev0 = c->prof_ev[c->prof_used];
        ev1 = c->prof_ev[c->prof_used + 1];
        c->prof_used += 2;
    }
    if (c->cpml && !c->iso && shots == c->d_shots && c->layer_pass) {
        // forward CPML, layer pass: psi^{n+1}, zeta^{n+1} and the corrections of the group's
        // layer cells, then the stencil over the group's whole grids adds the corrections
        if (!g) return fail(c, MM_ERR_STATE, "forward CPML step without a shot group");
        MM_TRY(dev(c, launch_cpml_forward(shots + g->s0, g->s1 - g->s0, c->p.nb, g->stream, g->cpml_d,
                                          g->cpml_h.data(), parity, c->cf, s, ev0),
                   "cpml layer launch"));
        StepAux a = aux;
        a.stream_loads = g->stream ? 1 : 0;
        MM_TRY(dev(c, launch_step(c->variant, MM_BC_CPML, mode, c->d_tiles + g->t.full_off, g->t.nfull, shots,
                                  parity, c->cf, a, s, nullptr, ev1),
                   "stencil launch"));
        return MM_OK;
    }
    if (c->cpml && !c->iso && shots == c->d_shots) {
        // forward CPML: the interior boxes (plain stencil), then the frames, the z-layer tiles
        // and the z-layer corner tiles (fused CPML kernel; one launch for the three when the
        // group has few of them); the launches write disjoint cells and read only p^n of the
        // step, so their order is free; the receivers ride in the first launch that runs
        if (!g) return fail(c, MM_ERR_STATE, "forward CPML step without a shot group");
        const GroupTiles& t = g->t;
        const bool one = t.merged();
        const int off[4] = {t.in_off, t.st_off, t.zl_off, t.zc_off};
        const int cnt[4] = {t.nin, one ? t.nst + t.nzl + t.nzc : t.nst, one ? 0 : t.nzl, one ? 0 : t.nzc};
        const int kind[4] = {-1, one ? CS_ALL : CS_FRAME, CS_ZLAYER, CS_ZCORNER};
        int first = -1, last = -1;
        for (int k = 0; k < 4; ++k)
            if (cnt[k] > 0) {
                if (first < 0) first = k;
                last = k;
            }
        StepAux a = aux;
        a.stream_loads = g->stream ? 1 : 0;
        for (int k = 0; k < 4; ++k) {
            if (cnt[k] <= 0) continue;
            StepAux ak = a;
            if (k != first) ak.gather_blocks = 0;
            hipEvent_t e0 = k == first ? ev0 : nullptr, e1 = k == last ? ev1 : nullptr;
            const TileEnt* tl = c->d_tiles + off[k];
            if (k == 0)
                MM_TRY(dev(c, launch_step(c->variant, MM_BC_NONE, mode, tl, cnt[k], shots, parity, c->cf, ak, s, e0, e1),
                           "stencil launch"));
            else
                MM_TRY(dev(c, launch_cpml_step(kind[k], mode, tl, cnt[k], shots, parity, c->cf, ak, s, e0, e1),
                           "cpml step launch"));
        }
        return MM_OK;
    }
    if (c->cpml && !c->iso) {
        MM_TRY(dev(c, launch_cpml_adjoint(shots, (int)c->geom.size(), c->p.nb, c->cpml_adj_d, c->cpml_adj_h.data(),
                                          parity, c->cf, s, ev0),
                   "adjoint cpml launch"));
        ev0 = nullptr;  // stamped by the CPML kernel
    }
    const TileEnt* tiles = c->d_tiles + (g ? g->t.full_off : 0);
    const int nt = g ? g->t.nfull : c->nfull;
    if (c->iso) {
        MM_TRY(dev(c, launch_iso_step(c->variant, c->p.bc, g ? g->stream : c->stream_all, tiles, nt, shots, parity,
                                      c->cf, s, ev0, ev1),
                   "acoustic_iso launch"));
        return MM_OK;
    }
    StepAux a = aux;
    a.stream_loads = (g ? g->stream : c->stream_all) ? 1 : 0;
    MM_TRY(dev(c, launch_step(c->variant, c->p.bc, mode, tiles, nt, shots, parity, c->cf, a, s, ev0, ev1),
               "stencil launch"));
    return MM_OK;
}

InjTab group_cells(const InjTab& t, const mm_ctx::Group& g) {
    InjTab r = t;
    r.cell_shot += g.cell0;
    r.cell_off += g.cell0;
    r.start += g.cell0;
    r.cell_g += g.cell0;
    r.ncell = g.cell1 - g.cell0;
    return r;
}

GatherTab group_recs(const GatherTab& t, const mm_ctx::Group& g) {
    GatherTab r = t;
    r.shot += g.rec0;
    r.off += g.rec0;
    r.n = g.rec1 - g.rec0;
    return r;
}

float* ckpt_field(mm_ctx* c, int seg, int which) {
    return reinterpret_cast<float*>(c->ws + c->L.ckpt + ((size_t)seg * 2 + which) * c->L.ckpt_field_bytes);
}

// The buffer that holds psi^k of a forward shot after k steps (parity k & 1):
// with the fused kernel the step of parity q reads psi from psi (q = 0) or psi2
// (q = 1) and writes the other; the layer pass keeps it in psi.
float* psi_now(const mm_ctx* c, const ShotDev& sd, int a, int parity) {
    return parity && !c->layer_pass ? sd.psi2[a] : sd.psi[a];
}

// CPML memory (psi_x,y,z, zeta_x,y,z) of checkpoint seg, kept in FP32
mm_status ckpt_memory(mm_ctx* c, int seg, bool save, int parity, hipStream_t s) {
    if (!c->cpml) return MM_OK;
    const auto& g = c->geom[0];
    const size_t nb2 = 2 * (size_t)c->p.nb;
    const size_t sl[3] = {(size_t)g.nz * g.ny * nb2, (size_t)g.nz * nb2 * g.nx, nb2 * g.ny * g.nx};
    char* base = c->ws + c->L.ckpt_mem + (size_t)seg * c->L.ckpt_mem_bytes;
    size_t o = 0;
    for (int k = 0; k < 6; ++k) {
        float* f = k < 3 ? psi_now(c, c->shots_h[0], k, parity) : c->shots_h[0].zeta[k - 3];
        const size_t bytes = sizeof(float) * sl[k % 3];
        float* dst = save ? reinterpret_cast<float*>(base + o) : f;
        const float* src = save ? f : reinterpret_cast<const float*>(base + o);
        MM_TRY(dev(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "checkpoint copy"));
        o += bytes;
    }
    return MM_OK;
}

mm_status save_ckpt(mm_ctx* c, int seg, int parity, hipStream_t s) {
    const long long N = c->geom[0].n();
    const ShotDev& sd = c->shots_h[0];
    const float* prev = sd.buf[parity ^ 1];  // p^{k-1}
    const float* cur = sd.buf[parity];       // p^k
    if (c->p.snap == MM_SNAP_FP32) {
        MM_TRY(dev(c, hipMemcpyAsync(ckpt_field(c, seg, 0), prev, sizeof(float) * N, hipMemcpyDeviceToDevice, s),
                   "checkpoint copy"));
        MM_TRY(dev(c, hipMemcpyAsync(ckpt_field(c, seg, 1), cur, sizeof(float) * N, hipMemcpyDeviceToDevice, s),
                   "checkpoint copy"));
    } else {
        float* sc = at<float>(c->ws, c->L.ckpt_scale) + 2 * c->L.ckpt_scale_n * seg;
        MM_TRY(dev(c, launch_snap_encode(prev, cur, N, reinterpret_cast<uint16_t*>(ckpt_field(c, seg, 0)),
                                         reinterpret_cast<uint16_t*>(ckpt_field(c, seg, 1)), sc,
                                         sc + c->L.ckpt_scale_n, s),
                   "snapshot encode"));
    }
    return ckpt_memory(c, seg, true, parity, s);
}

mm_status restore_ckpt(mm_ctx* c, int seg, int parity, hipStream_t s) {
    const long long N = c->geom[0].n();
    const ShotDev& sd = c->shots_h[0];
    float* prev = sd.buf[parity ^ 1];
    float* cur = sd.buf[parity];
    if (c->p.snap == MM_SNAP_FP32) {
        MM_TRY(dev(c, hipMemcpyAsync(prev, ckpt_field(c, seg, 0), sizeof(float) * N, hipMemcpyDeviceToDevice, s),
                   "checkpoint copy"));
        MM_TRY(dev(c, hipMemcpyAsync(cur, ckpt_field(c, seg, 1), sizeof(float) * N, hipMemcpyDeviceToDevice, s),
                   "checkpoint copy"));
    } else {
        const float* sc = at<float>(c->ws, c->L.ckpt_scale) + 2 * c->L.ckpt_scale_n * seg;
        MM_TRY(dev(c, launch_snap_decode(reinterpret_cast<const uint16_t*>(ckpt_field(c, seg, 0)),
                                         reinterpret_cast<const uint16_t*>(ckpt_field(c, seg, 1)), sc,
                                         sc + c->L.ckpt_scale_n, N, prev, cur, s),
                   "snapshot decode"));
    }
    return ckpt_memory(c, seg, false, parity, s);
}

// Forward steps: each group of shots runs all nsteps steps before the next
// group starts (shots are independent, so this is the same result as
// advancing every shot together).
mm_status enqueue_forward(mm_ctx* c, int nsteps, const float* wav, float* traces, hipStream_t s) {
    const StepAux none{};
    const bool ck = c->ckpt_active;  // single-shot contexts only: one group
    if (ck && c->nsrc > 0)
        MM_TRY(dev(c, hipMemcpyAsync(at<float>(c->ws, c->L.wav_store) + (size_t)c->step * c->nsrc, wav,
                                     sizeof(float) * (size_t)nsteps * c->nsrc, hipMemcpyDeviceToDevice, s),
                   "wavelet copy"));
    for (const auto& g : c->groups) {
        const GatherTab rg = group_recs(c->rec_gather, g);
        const InjTab inj = group_cells(c->src_inj, g);
        for (int j = 0; j < nsteps; ++j) {
            const int k = c->step + j;
            const int parity = k & 1;
            if (ck && k % c->p.ckpt_every == 0) MM_TRY(save_ckpt(c, k / c->p.ckpt_every, parity, s));
            StepAux aux = none;
            aux.src_scale = c->src_inj.scale;
            aux.wrow = c->nsrc > 0 ? wav + (size_t)j * c->nsrc : nullptr;
            if (j > 0 && traces && rg.n > 0 && !c->iso) {
                // the stencil launch also records the previous step's receivers
                aux.g_shot = rg.shot;
                aux.g_off = rg.off;
                aux.g_n = rg.n;
                aux.gather_blocks = ((rg.n + 255) / 256 + 7) / 8 * 8;
                aux.gather_out = traces + (size_t)(j - 1) * c->nrec + g.rec0;
            }
            MM_TRY(enqueue_step(c, c->d_shots, parity, MODE_PLAIN, aux, s, &g));
            if (inj.ncell > 0 && !c->inline_src)
                MM_TRY(dev(c, launch_inject(inj, c->d_shots, parity, aux.wrow, c->nsrc, MODE_PLAIN, none, s), "inject"));
            if (c->iso && traces && rg.n > 0 && j + 1 < nsteps)
                MM_TRY(dev(c, launch_gather(rg, c->d_shots, parity, traces + (size_t)j * c->nrec + g.rec0, s),
                           "record"));
            if (watch_due(k + 1, c->p.watch_every))
                for (int i = g.s0; i < g.s1; ++i)
                    MM_TRY(dev(c, launch_watch(c->shots_h[i].buf[parity ^ 1], c->geom[i].n(), k + 1, c->watch, s),
                               "watch"));
        }
        if (nsteps > 0 && traces && rg.n > 0)
            MM_TRY(dev(c, launch_gather(rg, c->d_shots, (c->step + nsteps - 1) & 1,
                                        traces + (size_t)(nsteps - 1) * c->nrec + g.rec0, s),
                       "record"));
    }
    return MM_OK;
}

mm_status check_forward(mm_ctx* c, int nsteps, const float* wav) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    if (nsteps < 0) return fail(c, MM_ERR_ARG, "nsteps must be >= 0");
    if (c->nsrc > 0 && nsteps > 0 && !wav) return fail(c, MM_ERR_ARG, "wavelet is NULL");
    if (!c->fwd_valid)
        return fail(c, MM_ERR_STATE, "forward state was consumed by a gradient replay or a failed launch; call mm_reset");
    if ((long long)c->step + nsteps > (1LL << 30)) return fail(c, MM_ERR_ARG, "step counter overflow");
    return MM_OK;
}

void begin_forward(mm_ctx* c, int nsteps) {
    if (c->L.grad) {
        if (c->step == 0) c->ckpt_active = true;
        if (c->ckpt_active && c->step + nsteps > c->p.nsteps_max) c->ckpt_active = false;
    }
    c->adj_started = false;
}

// Replay segment sg from its checkpoint, keeping d2p of every step.
mm_status replay_segment(mm_ctx* c, int sg, hipStream_t s) {
    const int K = c->p.ckpt_every;
    const int n0 = sg * K, n1 = std::min(n0 + K, c->adj_T);
    const long long N = c->geom[0].n();
    MM_TRY(restore_ckpt(c, sg, n0 & 1, s));
    char* seg = c->ws + c->L.seg;
    const size_t esz = c->p.snap == MM_SNAP_BF16 ? 2 : 4;
    const float* wav = at<float>(c->ws, c->L.wav_store);
    for (int n = n0; n < n1; ++n) {
        StepAux aux{};
        aux.d2p_out = seg + (size_t)(n - n0) * N * esz;
        aux.d2p_bf16 = c->p.snap == MM_SNAP_BF16;
        aux.src_scale = c->src_inj.scale;
        aux.wrow = c->nsrc > 0 ? wav + (size_t)n * c->nsrc : nullptr;
        MM_TRY(enqueue_step(c, c->d_shots, n & 1, MODE_D2P, aux, s, &c->groups[0]));
        if (c->nsrc > 0 && !c->inline_src)
            MM_TRY(dev(c, launch_inject(c->src_inj, c->d_shots, n & 1, aux.wrow, c->nsrc, MODE_D2P, aux, s),
                       "inject"));
    }
    c->seg_loaded = sg;
    c->fwd_valid = false;
    return MM_OK;
}

mm_status enqueue_adjoint(mm_ctx* c, int nsteps, const float* resid, float* adj_src, float* grad, hipStream_t s) {
    const int mcur = c->adj_T - c->adj_j;
    const int m0 = mcur - nsteps + 1;
    const long long N = c->geom[0].n();
    for (int j = 0; j < nsteps; ++j) {
        const int jj = c->adj_j + j;
        const int m = c->adj_T - jj;
        const int parity = jj & 1;
        StepAux aux{};
        int mode = MODE_PLAIN;
        if (grad) {
            const int K = c->p.ckpt_every;
            const int sg = (m - 1) / K;
            if (c->seg_loaded != sg) MM_TRY(replay_segment(c, sg, s));
            aux.d2p_in = c->ws + c->L.seg + (size_t)((m - 1) - sg * K) * N * (c->p.snap == MM_SNAP_BF16 ? 2 : 4);
            aux.d2p_bf16 = c->p.snap == MM_SNAP_BF16;
            aux.grad = grad;
            aux.neg_inv_dt2 = (float)(-1.0 / (c->dt * c->dt));
            mode = MODE_IMAGE;
        }
        MM_TRY(enqueue_step(c, c->d_shots_adj, parity, mode, aux, s, nullptr));
        const int row = m - m0;
        if (c->nrec > 0)
            MM_TRY(dev(c, launch_inject(c->rec_inj, c->d_shots_adj, parity, resid + (size_t)row * c->nrec, c->nrec,
                                        mode, aux, s),
                       "adjoint inject"));
        if (adj_src && c->nsrc > 0)
            MM_TRY(dev(c, launch_gather(c->src_gather, c->d_shots_adj, parity, adj_src + (size_t)row * c->nsrc, s),
                       "adjoint record"));
    }
    return MM_OK;
}

std::string tune_key(const mm_ctx* c) {
    std::string k = std::to_string(c->p.model) + "/" + std::to_string(c->p.bc) + "/" + std::to_string(c->p.nb) + "/" +
                    std::to_string(c->p.cache_hints) + "/" + std::to_string(c->p.cpml_kernel) + "/" +
                    std::to_string(c->p.free_surface);
    for (const auto& g : c->groups) k += "/" + std::to_string(g.s1 - g.s0);
    for (const auto& g : c->geom) k += ":" + std::to_string(g.nx) + "x" + std::to_string(g.ny) + "x" + std::to_string(g.nz);
    return k;
}

// tuned (tile variant, forward CPML layer pass) per problem
std::mutex g_tune_mu;
std::map<std::string, std::pair<int, bool>> g_tune_cache;

// The forward CPML strategy (acoustic_iso_cd) before or without tuning: the
// layer pass when the cells outside the interior boxes are 30 % or more of
// the context's cells.  The fused kernel's z-marching strips then hold too
// few blocks to fill the chip (measured per step: 79 against 142 us at 240^3
// with 20-cell layers; 2.82 against 2.42 ms the other way at 1024^2 x 512
// with 32-cell layers).
bool layer_pass_default(const mm_params& p, const std::vector<ShotGeom>& shots) {
    if (p.cpml_kernel == MM_CPML_LAYER) return true;
    if (p.cpml_kernel == MM_CPML_FUSED) return false;
    double all = 0.0, inner = 0.0;
    const int zl = p.free_surface ? 1 : 2;
    for (const auto& g : shots) {
        all += (double)g.n();
        inner += (double)std::max(0, g.nx - 2 * p.nb) * std::max(0, g.ny - 2 * p.nb) * std::max(0, g.nz - zl * p.nb);
    }
    return inner < 0.7 * all;
}

}  // namespace

// ====================================================================== ABI

extern "C" {

void mm_default_params(mm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->dx = p->dy = p->dz = 10.0;
    p->cfl = 0.5;
    p->bc = MM_BC_SPONGE;
    p->nb = 12;
    p->sponge_sigma = 0.015;
    p->cpml_R = 1e-3;
    p->cpml_f0 = 15.0;
    p->snap = MM_SNAP_FP32;
}

const char* mm_status_str(mm_status s) {
    switch (s) {
        case MM_OK: return "ok";
        case MM_ERR_ARG: return "invalid argument";
        case MM_ERR_UNSTABLE: return "unstable time step";
        case MM_ERR_WORKSPACE: return "workspace too small or misaligned";
        case MM_ERR_DEVICE: return "device error";
        case MM_ERR_STATE: return "invalid state for this call";
        case MM_ERR_NONFINITE: return "non-finite or non-positive value";
        case MM_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* mm_last_error(const mm_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

mm_status mm_dt(const mm_params* p, double vmax, double* dt_out) {
    MM_TRY(check_params(p, nullptr));
    if (!finite_pos(vmax)) return fail(nullptr, MM_ERR_ARG, "vmax must be finite and > 0");
    if (!dt_out) return fail(nullptr, MM_ERR_ARG, "dt_out is NULL");
    const double lim = dt_stab(*p, vmax);
    if (p->dt > 0.0) {
        if (p->dt > lim) return fail(nullptr, MM_ERR_UNSTABLE, "dt exceeds the stability limit");
        *dt_out = p->dt;
        return MM_OK;
    }
    if (p->cfl > 1.0) return fail(nullptr, MM_ERR_UNSTABLE, "cfl > 1 is unstable");
    *dt_out = p->cfl * lim;
    return MM_OK;
}

mm_status mm_ricker(double f0, double t0, double dt, int32_t n, float* out) {
    if (!(std::isfinite(f0) && f0 > 0) || !std::isfinite(t0) || !finite_pos(dt) || n < 0 || (n > 0 && !out))
        return fail(nullptr, MM_ERR_ARG, "bad Ricker arguments");
    for (int i = 0; i < n; ++i) {
        const double tau = i * dt - t0;
        const double x = (kPi * f0 * tau) * (kPi * f0 * tau);
        out[i] = (float)((1.0 - 2.0 * x) * std::exp(-x));
    }
    return MM_OK;
}

mm_status mm_workspace_size(const mm_params* p, int32_t nshots, const mm_shot* shots, size_t* bytes) {
    MM_TRY(check_params(p, nullptr));
    if (!bytes) return fail(nullptr, MM_ERR_ARG, "bytes is NULL");
    std::vector<ShotGeom> g;
    int ns, nr;
    MM_TRY(totals(p, nshots, shots, false, g, ns, nr, nullptr));
    Layout L;
    compute_layout(*p, g, ns, nr, L);
    *bytes = L.total;
    return MM_OK;
}

mm_status mm_init_batch(mm_ctx** out, const mm_params* p, int32_t nshots, const mm_shot* shots, void* workspace,
                        size_t ws_bytes, void* hip_stream) {
    if (!out) return fail(nullptr, MM_ERR_ARG, "out is NULL");
    *out = nullptr;
    MM_TRY(check_params(p, nullptr));
    std::vector<ShotGeom> geom;
    int nsrc, nrec;
    MM_TRY(totals(p, nshots, shots, true, geom, nsrc, nrec, nullptr));
    if (p->dt == 0.0 && p->cfl > 1.0) return fail(nullptr, MM_ERR_UNSTABLE, "cfl > 1 is unstable");
    Layout L;
    compute_layout(*p, geom, nsrc, nrec, L);
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
        return fail(nullptr, MM_ERR_WORKSPACE, "workspace must be a non-NULL 256-byte aligned device pointer");
    if (ws_bytes < L.total) {
        char buf[128];
        snprintf(buf, sizeof buf, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
        return fail(nullptr, MM_ERR_WORKSPACE, buf);
    }

    mm_ctx* c = new mm_ctx();
    c->p = *p;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    c->geom = geom;
    c->L = L;
    c->ws = reinterpret_cast<char*>(workspace);
    c->nsrc = nsrc;
    c->nrec = nrec;
    c->sponge = p->bc == MM_BC_SPONGE;
    c->cpml = p->bc == MM_BC_CPML;
    c->iso = p->model == MM_MODEL_ISO;
    hipStream_t s = c->stream;
    auto bail = [&](mm_status st) {
        g_err = c->err;
        delete c;
        return st;
    };

    char* scr = c->ws + L.scratch;
    c->vcheck = reinterpret_cast<unsigned*>(scr);
    c->watch = c->vcheck + 4;
    c->loss_part = reinterpret_cast<double*>(scr + 64);
    c->loss_dev = c->loss_part + kPartials;

    // velocity check and maximum (one synchronisation)
    mm_status st = dev(c, launch_fill(reinterpret_cast<float*>(c->vcheck), 2, 0.0f, s), "fill");
    if (st) return bail(st);
    for (int i = 0; i < nshots; ++i) {
        st = dev(c, launch_vcheck(shots[i].vel, geom[i].n(), c->vcheck, s), "velocity check");
        if (st) return bail(st);
    }
    if (c->iso) {
        // the density must be finite and positive too (its maximum goes to a second slot)
        unsigned* dchk = c->vcheck + 2;
        st = dev(c, launch_fill(reinterpret_cast<float*>(dchk), 2, 0.0f, s), "fill");
        for (int i = 0; i < nshots && !st; ++i)
            st = dev(c, launch_vcheck(shots[i].rho, geom[i].n(), dchk, s), "density check");
        unsigned dres[2] = {0, 0};
        if (!st) st = dev(c, hipMemcpyAsync(dres, dchk, sizeof dres, hipMemcpyDeviceToHost, s), "readback");
        if (!st) st = dev(c, hipStreamSynchronize(s), "sync");
        if (st) return bail(st);
        if (dres[1]) return bail(fail(c, MM_ERR_NONFINITE, "density has NaN, Inf or non-positive values"));
    }
    unsigned vres[2] = {0, 0};
    st = dev(c, hipMemcpyAsync(vres, c->vcheck, sizeof vres, hipMemcpyDeviceToHost, s), "readback");
    if (!st) st = dev(c, hipStreamSynchronize(s), "sync");
    if (st) return bail(st);
    if (vres[1]) return bail(fail(c, MM_ERR_NONFINITE, "velocity has NaN, Inf or non-positive values"));
    float vmf;
    std::memcpy(&vmf, &vres[0], sizeof vmf);
    c->vmax = p->vmax > 0.0 ? p->vmax : (double)vmf;
    if (p->vmax > 0.0 && p->vmax < (double)vmf) return bail(fail(c, MM_ERR_ARG, "vmax is below the model maximum"));
    const double lim = dt_stab(*p, c->vmax);
    if (p->dt > 0.0) {
        if (p->dt > lim) return bail(fail(c, MM_ERR_UNSTABLE, "dt exceeds the stability limit"));
        c->dt = p->dt;
    } else {
        c->dt = p->cfl * lim;
    }

    // coefficients
    const double h[3] = {p->dx, p->dy, p->dz};
    for (int m = 0; m < 4; ++m) {
        c->cf.cx[m] = (float)(kA2[m] / (h[0] * h[0]));
        c->cf.cy[m] = (float)(kA2[m] / (h[1] * h[1]));
        c->cf.cz[m] = (float)(kA2[m] / (h[2] * h[2]));
        c->cf.bx[m] = (float)(kB1[m] / h[0]);
        c->cf.by[m] = (float)(kB1[m] / h[1]);
        c->cf.bz[m] = (float)(kB1[m] / h[2]);
        c->cf.sx[m] = (float)(kS1[m] / h[0]);
        c->cf.sy[m] = (float)(kS1[m] / h[1]);
        c->cf.sz[m] = (float)(kS1[m] / h[2]);
    }

    // shot descriptors and 1D boundary tables
    std::vector<std::vector<float>> prof(nshots);
    for (int i = 0; i < nshots; ++i) {
        const ShotGeom& g = geom[i];
        ShotDev sd{};
        sd.buf[0] = at<float>(c->ws, L.buf0[i]);
        sd.buf[1] = at<float>(c->ws, L.buf1[i]);
        sd.vdt2 = at<float>(c->ws, L.vdt2[i]);
        sd.prof = at<float>(c->ws, L.prof[i]);
        for (int a = 0; a < 3; ++a) {
            sd.psi[a] = c->cpml ? at<float>(c->ws, L.psi[a][i]) : nullptr;
            sd.zeta[a] = c->cpml ? at<float>(c->ws, L.zeta[a][i]) : nullptr;
            sd.psi2[a] = c->cpml && !c->iso ? at<float>(c->ws, L.psi2[a][i]) : nullptr;
            sd.corr[a] = c->cpml && !c->iso ? at<float>(c->ws, L.corr[a][i]) : nullptr;
        }
        sd.nx = g.nx;
        sd.ny = g.ny;
        sd.nz = g.nz;
        sd.nb = p->nb;
        sd.cw = p->nb;
        sd.fs = p->free_surface;
        for (int a = 0; a < 3; ++a) sd.u[a] = c->iso ? at<float>(c->ws, L.iso_u[a][i]) : nullptr;
        sd.rdt = c->iso ? at<float>(c->ws, L.iso_b[i]) : nullptr;
        c->shots_h.push_back(sd);
        ShotDev sa = sd;
        sa.nsrc_in = 0;
        sa.buf[0] = L.adjoint ? at<float>(c->ws, L.ebuf0[i]) : nullptr;
        sa.buf[1] = L.adjoint ? at<float>(c->ws, L.ebuf1[i]) : nullptr;
        for (int a = 0; a < 3; ++a) {
            const bool ca = c->cpml && L.adjoint;
            sa.psi[a] = ca ? at<float>(c->ws, L.apsi[a][i]) : nullptr;
            sa.zeta[a] = ca ? at<float>(c->ws, L.azeta[a][i]) : nullptr;
            sa.psi2[a] = nullptr;
            sa.corr[a] = ca ? at<float>(c->ws, L.acorr[a][i]) : nullptr;
        }
        sa.cw = p->nb + 4;
        c->shots_adj_h.push_back(sa);
        const int n[3] = {g.nx, g.ny, g.nz};
        std::vector<float>& pr = prof[i];
        // a free surface removes the damping of the top face (z < nb): no sponge, and CPML
        // coefficients a = b = 0 there, so the layer memory stays 0 and adds nothing
        const bool fs = p->free_surface != 0;
        if (c->cpml) {
            // (a, b) per axis at the cells; acoustic_iso appends the same at its faces i + 1/2
            pr.resize((c->iso ? 4 : 2) * (g.nx + g.ny + g.nz));
            float* q = pr.data();
            for (int face = 0; face <= (c->iso ? 1 : 0); ++face)
                for (int a = 0; a < 3; ++a) {
                    if (face)
                        cpml_face_table(n[a], p->nb, h[a], c->dt, c->vmax, p->cpml_R, p->cpml_f0, q, q + n[a]);
                    else
                        cpml_table(n[a], p->nb, h[a], c->dt, c->vmax, p->cpml_R, p->cpml_f0, q, q + n[a]);
                    if (fs && a == 2) {
                        std::fill(q, q + p->nb, 0.0f);
                        std::fill(q + n[a], q + n[a] + p->nb, 0.0f);
                    }
                    q += 2 * n[a];
                }
        } else {
            pr.resize(g.nx + g.ny + g.nz);
            float* q = pr.data();
            for (int a = 0; a < 3; ++a) {
                if (c->sponge) sponge_table(n[a], p->nb, p->sponge_sigma, q);
                else std::fill(q, q + n[a], 1.0f);
                if (fs && a == 2 && c->sponge) std::fill(q, q + p->nb, 1.0f);
                q += n[a];
            }
        }
    }
    c->d_shots = at<ShotDev>(c->ws, L.shots_dev);
    c->d_shots_adj = at<ShotDev>(c->ws, L.shots_adj);
    c->d_tiles = at<TileEnt>(c->ws, L.tiles);

    // point tables
    std::vector<int> s_shot, r_shot;
    std::vector<long long> s_off, r_off;
    std::vector<float> s_g, r_g;
    for (int i = 0; i < nshots; ++i) {
        const ShotGeom& g = geom[i];
        auto lin = [&](const int32_t* t) { return ((long long)t[2] * g.ny + t[1]) * g.nx + t[0]; };
        auto gval = [&](const int32_t* t) {
            if (p->free_surface && t[2] == 0) return 0.0f;  // the surface plane stays 0
            if (!c->sponge) return 1.0f;
            const float* q = prof[i].data();
            return q[t[0]] * q[g.nx + t[1]] * q[g.nx + g.ny + t[2]];
        };
        for (int k = 0; k < shots[i].nsrc; ++k) {
            s_shot.push_back(i);
            s_off.push_back(lin(shots[i].src_ijk + 3 * k));
            s_g.push_back(gval(shots[i].src_ijk + 3 * k));
        }
        for (int k = 0; k < shots[i].nrec; ++k) {
            r_shot.push_back(i);
            r_off.push_back(lin(shots[i].rec_ijk + 3 * k));
            r_g.push_back(gval(shots[i].rec_ijk + 3 * k));
        }
    }
    Csr cs, cr;
    build_csr(s_shot, s_off, s_g, cs);
    build_csr(r_shot, r_off, r_g, cr);
    // sources are added inside the stencil kernel when no shot has more than MAX_INLINE_SRC
    c->inline_src = !c->iso;  // acoustic_iso adds every source with the injection kernel
    for (int i = 0; i < nshots; ++i) c->inline_src = c->inline_src && shots[i].nsrc <= MAX_INLINE_SRC;
    c->src_cells.assign(nshots, {});
    {
        int col = 0;
        for (int i = 0; i < nshots; ++i)
            for (int k = 0; k < shots[i].nsrc; ++k, ++col) {
                if (!c->inline_src) continue;
                ShotDev& sd = c->shots_h[i];
                sd.src_col[sd.nsrc_in] = col;
                sd.src_off[sd.nsrc_in] = s_off[col];
                sd.nsrc_in++;
                c->src_cells[i].push_back(s_off[col]);
            }
    }

    // stage every host table in one buffer kept alive in the context
    size_t hb = 0;
    auto reserve = [&](size_t bytes) { size_t o = hb; hb += align256(bytes); return o; };
    const size_t o_shots = reserve(sizeof(ShotDev) * nshots), o_adj = reserve(sizeof(ShotDev) * nshots);
    std::vector<size_t> o_prof;
    for (int i = 0; i < nshots; ++i) o_prof.push_back(reserve(sizeof(float) * prof[i].size()));
    c->host_tables.assign(hb, 0);
    char* H = c->host_tables.data();
    std::memcpy(H + o_shots, c->shots_h.data(), sizeof(ShotDev) * nshots);
    std::memcpy(H + o_adj, c->shots_adj_h.data(), sizeof(ShotDev) * nshots);
    for (int i = 0; i < nshots; ++i) std::memcpy(H + o_prof[i], prof[i].data(), sizeof(float) * prof[i].size());

    st = upload(c, c->d_shots, H + o_shots, sizeof(ShotDev) * nshots);
    if (!st) st = upload(c, c->d_shots_adj, H + o_adj, sizeof(ShotDev) * nshots);
    for (int i = 0; i < nshots && !st; ++i)
        st = upload(c, const_cast<float*>(c->shots_h[i].prof), H + o_prof[i], sizeof(float) * prof[i].size());
    // point tables: uploaded from vectors that live until the synchronisation below
    auto up = [&](size_t off, const void* src, size_t bytes) {
        if (!st) st = upload(c, c->ws + off, src, bytes);
    };
    up(L.src_shot, cs.shot.data(), sizeof(int) * cs.shot.size());
    up(L.src_off, cs.off.data(), sizeof(long long) * cs.off.size());
    up(L.src_start, cs.start.data(), sizeof(int) * cs.start.size());
    up(L.src_col, cs.col.data(), sizeof(int) * cs.col.size());
    up(L.src_g, cs.g.data(), sizeof(float) * cs.g.size());
    up(L.rin_shot, cr.shot.data(), sizeof(int) * cr.shot.size());
    up(L.rin_off, cr.off.data(), sizeof(long long) * cr.off.size());
    up(L.rin_start, cr.start.data(), sizeof(int) * cr.start.size());
    up(L.rin_col, cr.col.data(), sizeof(int) * cr.col.size());
    up(L.rin_g, cr.g.data(), sizeof(float) * cr.g.size());
    up(L.rg_shot, r_shot.data(), sizeof(int) * r_shot.size());
    up(L.rg_off, r_off.data(), sizeof(long long) * r_off.size());
    up(L.sg_shot, s_shot.data(), sizeof(int) * s_shot.size());
    up(L.sg_off, s_off.data(), sizeof(long long) * s_off.size());
    {
        // shot groups: receivers and source cells of each; the adjoint CPML block table
        std::vector<int> rec_start(nshots + 1, 0);
        for (int i = 0; i < nshots; ++i) rec_start[i + 1] = rec_start[i] + shots[i].nrec;
        // auto: non-temporal hints only when every shot of a launch alone overflows the cache (a
        // large shot re-reads its own p^n planes; many small shots that together exceed it do not
        // gain, measured 1.72 vs 2.05 ms per step for 32 shots in one group)
        auto hinted = [&](int s0, int s1) {
            double smallest = 1e300;
            for (int i = s0; i < s1; ++i) smallest = std::min(smallest, shot_set_bytes(*p, geom[i]));
            return p->cache_hints == 2 || (p->cache_hints == 0 && smallest > kInfinityCacheBytes);
        };
        c->stream_all = hinted(0, nshots);
        for (const auto& gr : make_groups(*p, geom)) {
            mm_ctx::Group g;
            g.s0 = gr.first;
            g.s1 = gr.second;
            g.stream = hinted(g.s0, g.s1);
            g.rec0 = rec_start[g.s0];
            g.rec1 = rec_start[g.s1];
            g.cell0 = (int)(std::lower_bound(cs.shot.begin(), cs.shot.end(), g.s0) - cs.shot.begin());
            g.cell1 = (int)(std::lower_bound(cs.shot.begin(), cs.shot.end(), g.s1) - cs.shot.begin());
            c->groups.push_back(std::move(g));
        }
        size_t cpml_pos = 3 * (size_t)(nshots + 1);  // after the adjoint's table
        if (c->cpml && !c->iso)
            for (auto& g : c->groups) {
                std::vector<int> gx, gy, gz;
                for (int i = g.s0; i < g.s1; ++i) {
                    gx.push_back(geom[i].nx);
                    gy.push_back(geom[i].ny);
                    gz.push_back(geom[i].nz);
                }
                const int ng = g.s1 - g.s0;
                g.cpml_h.assign(3 * (ng + 1), 0);
                cpml_block_table(gx.data(), gy.data(), gz.data(), ng, p->nb, g.cpml_h.data());
                g.cpml_d = at<int>(c->ws, L.cpml_off) + cpml_pos;
                up(L.cpml_off + sizeof(int) * cpml_pos, g.cpml_h.data(), sizeof(int) * g.cpml_h.size());
                cpml_pos += g.cpml_h.size();
            }
        if (c->cpml && L.adjoint) {
            std::vector<int> gx, gy, gz;
            for (const auto& q : geom) {
                gx.push_back(q.nx);
                gy.push_back(q.ny);
                gz.push_back(q.nz);
            }
            c->cpml_adj_h.assign(3 * (nshots + 1), 0);
            cpml_block_table(gx.data(), gy.data(), gz.data(), nshots, p->nb + 4, c->cpml_adj_h.data());
            c->cpml_adj_d = at<int>(c->ws, L.cpml_off);
            up(L.cpml_off, c->cpml_adj_h.data(), sizeof(int) * c->cpml_adj_h.size());
        }
    }
    for (int i = 0; i < nshots && !st; ++i) {
        if (c->iso) {
            const ShotDev& q = c->shots_h[i];
            st = dev(c, launch_iso_setup(shots[i].vel, shots[i].rho, geom[i].n(), c->dt, q.vdt2, q.rdt, s),
                     "coefficients");
        } else {
            st = dev(c, launch_vdt2(shots[i].vel, c->shots_h[i].vdt2, geom[i].n(), c->dt, s), "vdt2");
        }
        // free surface: (dt v)^2 (acoustic_iso: dt rho v^2) = 0 on plane z = 0 keeps p = 0 there
        // (the state starts at 0)
        if (!st && p->free_surface)
            st = dev(c, launch_fill(c->shots_h[i].vdt2, (long long)geom[i].nx * geom[i].ny, 0.0f, s), "fill");
    }
    if (!st) st = dev(c, hipStreamSynchronize(s), "sync");
    if (st) return bail(st);

    c->src_inj = InjTab{at<int>(c->ws, L.src_shot), at<long long>(c->ws, L.src_off), at<int>(c->ws, L.src_start),
                        at<int>(c->ws, L.src_col), at<float>(c->ws, L.src_g), (int)cs.shot.size(),
                        (float)(1.0 / (p->dx * p->dy * p->dz))};
    c->rec_inj = InjTab{at<int>(c->ws, L.rin_shot), at<long long>(c->ws, L.rin_off), at<int>(c->ws, L.rin_start),
                        at<int>(c->ws, L.rin_col), at<float>(c->ws, L.rin_g), (int)cr.shot.size(), 1.0f};
    c->rec_gather = GatherTab{at<int>(c->ws, L.rg_shot), at<long long>(c->ws, L.rg_off), nrec};
    c->src_gather = GatherTab{at<int>(c->ws, L.sg_shot), at<long long>(c->ws, L.sg_off), nsrc};

    st = zero_state(c, s);
    if (!st && L.adjoint) st = zero_adjoint(c, s);
    if (st) return bail(st);

    int v = p->tile > 0 ? p->tile : 0;
    c->layer_pass = c->cpml && !c->iso && layer_pass_default(*p, geom);
    if (p->tile == -1) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(c));
        if (it != g_tune_cache.end()) {
            v = it->second.first;
            c->layer_pass = it->second.second;
        }
    }
    st = set_variant(c, v);
    if (st) return bail(st);
    if (p->tile == -1 && v == 0) {
        st = mm_autotune(c, 3, nullptr);
        if (st) return bail(st);
    }
    *out = c;
    return MM_OK;
}

mm_status mm_init(mm_ctx** out, const mm_params* p, const float* vel_dev, const int32_t* src, int32_t nsrc,
                  const int32_t* rec, int32_t nrec, void* workspace, size_t ws_bytes, void* hip_stream) {
    if (!p) return fail(nullptr, MM_ERR_ARG, "params is NULL");
    mm_shot s{p->nx, p->ny, p->nz, vel_dev, src, nsrc, rec, nrec, nullptr};
    return mm_init_batch(out, p, 1, &s, workspace, ws_bytes, hip_stream);
}

mm_status mm_init_static(mm_ctx** out, const mm_params* p, const float* vel_dev, const int32_t* src, int32_t nsrc,
                         const int32_t* rec, int32_t nrec, void* hip_stream) {
    if (!out) return fail(nullptr, MM_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, MM_ERR_ARG, "params is NULL");
    mm_shot shot{p->nx, p->ny, p->nz, vel_dev, src, nsrc, rec, nrec, nullptr};
    size_t need = 0;
    MM_TRY(mm_workspace_size(p, 1, &shot, &need));
    const size_t have = static_workspace_bytes();
    if (need > have) {
        char buf[160];
        snprintf(buf, sizeof buf, "the problem needs %zu bytes of device memory; the static workspace holds %zu", need,
                 have);
        return fail(nullptr, MM_ERR_WORKSPACE, buf);
    }
    int d = -1;
    hipError_t e = hipGetDevice(&d);
    if (e != hipSuccess) return fail(nullptr, MM_ERR_DEVICE, std::string("device: ") + hipGetErrorString(e));
    if (d < 0 || d >= 64) return fail(nullptr, MM_ERR_DEVICE, "device index out of range");
    void* ws = nullptr;
    e = static_workspace(&ws);
    if (e != hipSuccess) return fail(nullptr, MM_ERR_DEVICE, std::string("static workspace: ") + hipGetErrorString(e));
    // no autotuning (its trials create HIP events): tile -1 runs the default variant
    mm_params q = *p;
    if (q.tile == -1) q.tile = 0;
    unsigned long long gen;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        gen = ++g_static_gen[d];  // earlier static contexts on this GPU stop here
    }
    mm_ctx* c = nullptr;
    MM_TRY(mm_init_batch(&c, &q, 1, &shot, ws, have, hip_stream));
    c->static_dev = d;
    c->static_gen = gen;
    *out = c;
    return MM_OK;
}

mm_status mm_forward_steps(mm_ctx* c, int32_t nsteps, const float* wav, float* traces) {
    MM_TRY(check_forward(c, nsteps, wav));
    begin_forward(c, nsteps);
    const mm_status st = enqueue_forward(c, nsteps, wav, traces, c->stream);
    if (st) {
        // a launch failed after earlier steps were enqueued: the state is no
        // longer that of a whole number of steps
        c->fwd_valid = false;
        return st;
    }
    c->step += nsteps;
    return MM_OK;
}

mm_status mm_forward_steps_graph(mm_ctx* c, int32_t nsteps, const float* wav, float* traces) {
    MM_TRY(check_forward(c, nsteps, wav));
    if (nsteps == 0) return MM_OK;
    begin_forward(c, nsteps);
    GraphKey key;
    key.nsteps = nsteps;
    key.wav = wav;
    key.tr = traces;
    key.step = c->ckpt_active ? c->step : (c->step & 1);
    key.variant = c->variant;
    key.ckpt = c->ckpt_active;
    if (!(c->gexec && c->gkey == key)) {
        drop_graph(c);
        if (!c->cap_stream) MM_TRY(dev(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "stream"));
        MM_TRY(dev(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture"));
        mm_status st = enqueue_forward(c, nsteps, wav, traces, c->cap_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
        if (st) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        MM_TRY(dev(c, e, "end capture"));
        c->graph = g;
        MM_TRY(dev(c, hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0), "graph instantiate"));
        c->gkey = key;
    }
    MM_TRY(dev(c, hipGraphLaunch(c->gexec, c->stream), "graph launch"));
    c->step += nsteps;
    return MM_OK;
}

mm_status mm_adjoint_steps(mm_ctx* c, int32_t nsteps, const float* resid, float* adj_src, float* grad) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    if (!c->L.adjoint) return fail(c, MM_ERR_STATE, "context was created with ckpt_every = 0 (no adjoint storage)");
    if (nsteps < 0) return fail(c, MM_ERR_ARG, "nsteps must be >= 0");
    if (c->nrec > 0 && nsteps > 0 && !resid) return fail(c, MM_ERR_ARG, "residual is NULL");
    if (grad && !c->L.grad) return fail(c, MM_ERR_UNSUPPORTED, "gradients need a single-shot context");
    const int T = c->adj_started ? c->adj_T : c->step;
    const int done = c->adj_started ? c->adj_j : 0;
    if (done + nsteps > T) return fail(c, MM_ERR_STATE, "adjoint would run past time 0");
    if (grad && !(c->ckpt_active && T <= c->p.nsteps_max))
        return fail(c, MM_ERR_STATE, "gradient needs a checkpointed forward run from step 0 (<= nsteps_max steps)");
    if (grad && c->adj_started && !c->adj_grad)
        return fail(c, MM_ERR_STATE, "adjoint was started without a gradient; reset and rerun the forward");
    if (!c->adj_started) {
        MM_TRY(zero_adjoint(c, c->stream));
        c->adj_started = true;
        c->adj_T = c->step;
        c->adj_j = 0;
        c->adj_grad = grad != nullptr;
        c->seg_loaded = -1;
    }
    MM_TRY(enqueue_adjoint(c, nsteps, resid, adj_src, grad, c->stream));
    c->adj_j += nsteps;
    return MM_OK;
}

mm_status mm_reset(mm_ctx* c) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    MM_TRY(zero_state(c, c->stream));
    if (c->L.adjoint) MM_TRY(zero_adjoint(c, c->stream));
    c->step = 0;
    c->fwd_valid = true;
    c->ckpt_active = false;
    c->adj_started = false;
    c->seg_loaded = -1;
    return MM_OK;
}

mm_status mm_gradient(mm_ctx* c, int32_t nsteps, const float* wav, const float* d_obs, float* grad, float* traces,
                      double* loss_host) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    if (!c->L.grad) return fail(c, MM_ERR_STATE, "gradients need a single-shot context with ckpt_every > 0");
    if (nsteps < 1 || nsteps > c->p.nsteps_max) return fail(c, MM_ERR_ARG, "nsteps must be in [1, nsteps_max]");
    if (!grad || (c->nrec > 0 && !d_obs) || (c->nsrc > 0 && !wav)) return fail(c, MM_ERR_ARG, "NULL operand");
    hipStream_t s = c->stream;
    MM_TRY(mm_reset(c));
    float* tr = traces ? traces : at<float>(c->ws, c->L.tr_store);
    begin_forward(c, nsteps);
    MM_TRY(enqueue_forward(c, nsteps, wav, tr, s));
    c->step = nsteps;
    float* resid = at<float>(c->ws, c->L.resid_store);
    const long long nr = (long long)nsteps * c->nrec;
    if (nr > 0) MM_TRY(dev(c, launch_residual_loss(tr, d_obs, resid, nr, c->loss_part, kPartials, c->loss_dev, s), "loss"));
    MM_TRY(dev(c, launch_fill(grad, c->geom[0].n(), 0.0f, s), "fill"));
    MM_TRY(mm_adjoint_steps(c, nsteps, resid, nullptr, grad));
    if (loss_host) {
        if (nr > 0) {
            MM_TRY(dev(c, hipMemcpyAsync(loss_host, c->loss_dev, sizeof(double), hipMemcpyDeviceToHost, s), "readback"));
            MM_TRY(dev(c, hipStreamSynchronize(s), "sync"));
        } else {
            *loss_host = 0.0;
        }
    }
    if (c->p.watch_every > 0) return mm_watch(c, nullptr);
    return MM_OK;
}

mm_status mm_watch(mm_ctx* c, int32_t* bad_step) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    if (c->p.watch_every <= 0) return fail(c, MM_ERR_STATE, "the context was made with watch_every = 0");
    unsigned w[2] = {0u, 0u};
    MM_TRY(dev(c, hipMemcpyAsync(w, c->watch, sizeof w, hipMemcpyDeviceToHost, c->stream), "readback"));
    MM_TRY(dev(c, hipStreamSynchronize(c->stream), "sync"));
    std::string msg;
    const mm_status st = watch_result(w, bad_step, &msg);
    if (st != MM_OK) return fail(c, st, msg);
    return MM_OK;
}

int64_t mm_snap_blocks(int64_t n) { return n > 0 ? (int64_t)snap_blocks(n) : 0; }

mm_status mm_snap_encode(const float* prev, const float* cur, int64_t n, uint16_t* c0, uint16_t* c1, float* s0,
                         float* s1, void* stream) {
    if (n < 0) return fail(nullptr, MM_ERR_ARG, "n must be >= 0");
    if (n > 0 && (!prev || !cur || !c0 || !c1 || !s0 || !s1)) return fail(nullptr, MM_ERR_ARG, "NULL array");
    const hipError_t e = launch_snap_encode(prev, cur, n, c0, c1, s0, s1, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, MM_ERR_DEVICE, std::string("snapshot encode: ") + hipGetErrorString(e));
    return MM_OK;
}

mm_status mm_snap_decode(const uint16_t* c0, const uint16_t* c1, const float* s0, const float* s1, int64_t n,
                         float* prev, float* cur, void* stream) {
    if (n < 0) return fail(nullptr, MM_ERR_ARG, "n must be >= 0");
    if (n > 0 && (!prev || !cur || !c0 || !c1 || !s0 || !s1)) return fail(nullptr, MM_ERR_ARG, "NULL array");
    const hipError_t e = launch_snap_decode(c0, c1, s0, s1, n, prev, cur, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, MM_ERR_DEVICE, std::string("snapshot decode: ") + hipGetErrorString(e));
    return MM_OK;
}

mm_status mm_state_size(const mm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return fail(nullptr, MM_ERR_ARG, "NULL argument");
    size_t b = 0;
    for (const auto& g : c->geom) {
        b += (c->iso ? 4 : 2) * sizeof(float) * (size_t)g.n();
        if (c->cpml) {
            const size_t nb2 = 2 * (size_t)mem_width(c->p);
            b += 2 * sizeof(float) * ((size_t)g.nz * g.ny * nb2 + (size_t)g.nz * nb2 * g.nx + nb2 * g.ny * g.nx);
        }
    }
    *bytes = b;
    return MM_OK;
}

static mm_status state_copy(mm_ctx* c, char* ext, bool to_ext) {
    size_t o = 0;
    const int par = c->step & 1;
    auto cp = [&](void* field, size_t bytes) -> mm_status {
        void* d = to_ext ? (void*)(ext + o) : field;
        const void* s = to_ext ? (const void*)field : (const void*)(ext + o);
        o += bytes;
        return dev(c, hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, c->stream), "state copy");
    };
    for (size_t i = 0; i < c->geom.size(); ++i) {
        const auto& g = c->geom[i];
        const size_t fb = sizeof(float) * (size_t)g.n();
        if (c->iso) {
            // acoustic_iso: p^k, then u_x, u_y, u_z at k - 1/2, then with CPML the memory of
            // the face derivatives (psi) and of the cell derivatives (zeta)
            MM_TRY(cp(c->shots_h[i].buf[par], fb));
            for (int a = 0; a < 3; ++a) MM_TRY(cp(c->shots_h[i].u[a], fb));
            if (c->cpml) {
                const size_t w2 = 2 * (size_t)mem_width(c->p);
                const size_t sl[3] = {(size_t)g.nz * g.ny * w2, (size_t)g.nz * w2 * g.nx, w2 * g.ny * g.nx};
                for (int a = 0; a < 3; ++a) MM_TRY(cp(c->shots_h[i].psi[a], sizeof(float) * sl[a]));
                for (int a = 0; a < 3; ++a) MM_TRY(cp(c->shots_h[i].zeta[a], sizeof(float) * sl[a]));
            }
            continue;
        }
        MM_TRY(cp(c->shots_h[i].buf[par ^ 1], fb));
        MM_TRY(cp(c->shots_h[i].buf[par], fb));
        if (c->cpml) {
            const size_t nb2 = 2 * (size_t)c->p.nb;
            const size_t sl[3] = {(size_t)g.nz * g.ny * nb2, (size_t)g.nz * nb2 * g.nx, nb2 * g.ny * g.nx};
            for (int a = 0; a < 3; ++a) MM_TRY(cp(psi_now(c, c->shots_h[i], a, par), sizeof(float) * sl[a]));
            for (int a = 0; a < 3; ++a) MM_TRY(cp(c->shots_h[i].zeta[a], sizeof(float) * sl[a]));
        }
    }
    return MM_OK;
}

mm_status mm_get_state(mm_ctx* c, void* dst) {
    if (!c || !dst) return fail(c, MM_ERR_ARG, "NULL argument");
    MM_TRY(live(c));
    if (!c->fwd_valid) return fail(c, MM_ERR_STATE, "forward state was consumed by a gradient replay");
    return state_copy(c, reinterpret_cast<char*>(dst), true);
}

mm_status mm_set_state(mm_ctx* c, const void* src, int32_t step) {
    if (!c || !src) return fail(c, MM_ERR_ARG, "NULL argument");
    MM_TRY(live(c));
    if (step < 0) return fail(c, MM_ERR_ARG, "step must be >= 0");
    c->step = step;
    c->fwd_valid = true;
    c->ckpt_active = false;
    c->adj_started = false;
    MM_TRY(state_copy(c, const_cast<char*>(reinterpret_cast<const char*>(src)), false));
    MM_TRY(dev(c, launch_watch_reset(c->watch, c->stream), "watch reset"));
    if (c->p.free_surface) {
        // the surface plane holds p = 0 at every time level
        for (size_t i = 0; i < c->geom.size(); ++i)
            for (int w = 0; w < 2; ++w)
                MM_TRY(dev(c, launch_fill(c->shots_h[i].buf[w], (long long)c->geom[i].nx * c->geom[i].ny, 0.0f,
                                          c->stream),
                           "fill"));
    }
    return MM_OK;
}

mm_status mm_get_info(const mm_ctx* c, double* dt, int32_t* step, int32_t* tile, int32_t* ngroups) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    if (dt) *dt = c->dt;
    if (step) *step = c->step;
    if (tile) *tile = c->variant;
    if (ngroups) *ngroups = (int32_t)c->groups.size();
    return MM_OK;
}

mm_status mm_get_cpml_kernel(const mm_ctx* c, int32_t* kernel) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    if (kernel) *kernel = !c->cpml || c->iso ? MM_CPML_AUTO : (c->layer_pass ? MM_CPML_LAYER : MM_CPML_FUSED);
    return MM_OK;
}

int32_t mm_num_tiles(void) { return num_tile_variants(); }

const char* mm_tile_name(int32_t t) { return (t >= 0 && t < num_tile_variants()) ? tile_variant(t).name : "?"; }

mm_status mm_set_tile(mm_ctx* c, int32_t t) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    if (t < 0 || t >= num_tile_variants()) return fail(c, MM_ERR_ARG, "unknown tile variant");
    if (c->iso && !iso_variant_ok(t)) return fail(c, MM_ERR_ARG, "acoustic_iso runs the 256-thread tile variants only");
    drop_graph(c);
    return set_variant(c, t);
}

mm_status mm_autotune(mm_ctx* c, int32_t steps, int32_t* tile_out) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(live(c));
    if (steps < 1) return fail(c, MM_ERR_ARG, "steps_per_trial must be >= 1");
    hipEvent_t e0, e1;
    MM_TRY(dev(c, hipEventCreate(&e0), "event"));
    MM_TRY(dev(c, hipEventCreate(&e1), "event"));
    const StepAux none{};  // trial steps inject nothing (no wavelet row)
    // one trial: 2 untimed steps, then `steps` steps timed with HIP events
    // (raised after the first trial so that a trial lasts about 2 ms)
    // the forward CPML strategy is tuned too unless the parameters fix it
    const bool both = c->cpml && !c->iso && c->p.cpml_kernel == MM_CPML_AUTO;
    auto trial = [&](int v, bool lp, float* ms) -> mm_status {
        c->layer_pass = lp;
        MM_TRY(set_variant(c, v));
        for (const auto& g : c->groups)
            for (int j = 0; j < 2; ++j) MM_TRY(enqueue_step(c, c->d_shots, j & 1, MODE_PLAIN, none, c->stream, &g));
        MM_TRY(dev(c, hipEventRecord(e0, c->stream), "event"));
        for (const auto& g : c->groups)
            for (int j = 0; j < steps; ++j) MM_TRY(enqueue_step(c, c->d_shots, j & 1, MODE_PLAIN, none, c->stream, &g));
        MM_TRY(dev(c, hipEventRecord(e1, c->stream), "event"));
        MM_TRY(dev(c, hipEventSynchronize(e1), "event"));
        return dev(c, hipEventElapsedTime(ms, e0, e1), "event");
    };
    // every variant once (in the default CPML strategy), then the fastest few
    // twice more, interleaved, in each strategy, each keeping its best time
    // (near-ties are otherwise decided by run-to-run noise)
    const bool lp0 = c->layer_pass;
    const int v_in = c->variant;
    std::vector<std::pair<float, int>> res;
    mm_status st = MM_OK;
    for (int v = 0; v < num_tile_variants() && !st; ++v) {
        if (c->iso && !iso_variant_ok(v)) continue;
        float ms = 0.0f;
        st = trial(v, lp0, &ms);
        if (st) break;
        if (res.empty() && ms > 0.0f && ms < 2.0f) {
            steps = std::min(200, std::max(steps, (int)std::ceil(2.0f * steps / ms)));
            st = trial(v, lp0, &ms);
        }
        if (!st) res.push_back({ms, v});
    }
    std::sort(res.begin(), res.end());
    const size_t top = std::min<size_t>(res.size(), 4);
    struct Cand {
        float ms;
        int v;
        bool lp;
    };
    std::vector<Cand> cand;
    for (size_t k = 0; k < top; ++k) {
        cand.push_back({res[k].first, res[k].second, lp0});
        if (both) cand.push_back({1e30f, res[k].second, !lp0});
    }
    for (int round = 0; round < 2 && !st; ++round)
        for (size_t k = 0; k < cand.size() && !st; ++k) {
            float ms = 0.0f;
            st = trial(cand[k].v, cand[k].lp, &ms);
            if (!st) cand[k].ms = std::min(cand[k].ms, ms);
        }
    int best = c->variant;
    bool best_lp = lp0;
    if (!st && !cand.empty()) {
        // the fastest pair; the other CPML strategy only if it wins by 3% or more (trials of a few
        // milliseconds differ by about that much from run to run)
        auto fastest = [&](bool lp) {
            const Cand* b = nullptr;
            for (const Cand& x : cand)
                if (x.lp == lp && (!b || x.ms < b->ms)) b = &x;
            return b;
        };
        const Cand* a = fastest(lp0);
        const Cand* o = fastest(!lp0);
        const Cand* b = (o && o->ms < 0.97f * a->ms) ? o : a;
        best = b->v;
        best_lp = b->lp;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) {
        // a failed trial: back to the tile variant and strategy the context had (its state, which
        // the trials overwrote, needs mm_reset or mm_set_state as after any failed launch)
        const std::string err = c->err;
        c->layer_pass = lp0;
        (void)set_variant(c, v_in);
        c->fwd_valid = false;
        c->err = err;
        return st;
    }
    drop_graph(c);
    c->layer_pass = best_lp;
    MM_TRY(set_variant(c, best));
    MM_TRY(mm_reset(c));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(c)] = {best, best_lp};
    }
    if (tile_out) *tile_out = best;
    return MM_OK;
}

mm_status mm_profile(mm_ctx* c, int32_t stride) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    if (stride < 0) return fail(c, MM_ERR_ARG, "stride must be >= 0");
    c->prof_stride = stride;
    c->prof_count = 0;
    return MM_OK;
}

mm_status mm_profile_read(mm_ctx* c, double* ms, int32_t* launches) {
    if (!c) return fail(nullptr, MM_ERR_ARG, "context is NULL");
    MM_TRY(dev(c, hipStreamSynchronize(c->stream), "sync"));
    double tot = 0.0;
    for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
        float m = 0.0f;
        MM_TRY(dev(c, hipEventElapsedTime(&m, c->prof_ev[i], c->prof_ev[i + 1]), "event"));
        tot += m;
    }
    if (ms) *ms = tot;
    if (launches) *launches = (int32_t)(c->prof_used / 2);
    c->prof_used = 0;
    c->prof_count = 0;
    return MM_OK;
}

void mm_destroy(mm_ctx* c) {
    if (!c) return;
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
    drop_graph(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

}  // extern "C"
