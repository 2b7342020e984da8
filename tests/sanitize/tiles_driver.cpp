// CPU check of the tile plans the host runtime builds (compiled together
// with mm_api.cpp, linked with the kernel object for the tile table): for
// every tile variant, boundary kind with free surface or not, and a set of
// grid shapes (ragged, minimal, one GPU's production share), each cell of a
// shot is written by exactly one tile of the full list and exactly one tile
// of the forward CPML lists; interior tiles hold no layer cell, frame tiles
// no z-layer cell, z-layer tiles are exactly the layers (split into those
// that may meet an x or y layer and those that do not); no tile is larger
// than its launch's shape or leaves the grid.  Run by
// tests/test_host_sanitize.py (optimised, without the sanitizers: it visits
// every cell of every plan).
#include "../../paper_2007_06048_amd/csrc/mm_api.cpp"

#include <array>

int main() {
    long bad = 0;
    int cases = 0;
    auto err = [&](const char* what, int a, int b, int c) {
        if (++bad <= 10) std::printf("%s (%d %d %d)\n", what, a, b, c);
    };
    // nx of the production share (1024, nb 32) on thin y and z; ragged, minimal and mixed shapes
    const std::vector<std::array<int, 4>> dims = {{1024, 40, 68, 32}, {120, 130, 70, 20}, {64, 64, 64, 12},
                                                  {37, 29, 23, 5},    {28, 28, 28, 12},   {100, 33, 41, 8},
                                                  {257, 75, 70, 33},  {16, 16, 16, 6},    {129, 65, 40, 16},
                                                  {45, 300, 30, 10}};
    const int CW = cstep_tile_w(CS_FRAME), CH = cstep_tile_h(CS_FRAME);
    const int ZW = cstep_tile_w(CS_ZLAYER), ZH = cstep_tile_h(CS_ZLAYER);
    for (const auto& d : dims)
        for (int fs = 0; fs < 2; ++fs)
            for (int v = 0; v < num_tile_variants(); ++v) {
                mm_params p{};
                mm_default_params(&p);
                p.bc = MM_BC_CPML;
                p.nb = d[3];
                p.free_surface = fs;
                std::vector<ShotGeom> shots = {{d[0], d[1], d[2]}, {d[1], d[2] + 3, std::max(d[0] / 2, 2 * d[3] + 4)}};
                const std::vector<std::pair<int, int>> groups = {{0, 1}, {1, 2}};
                std::vector<TileEnt> out;
                std::vector<GroupTiles> gt;
                build_tiles(v, p, shots, groups, out, gt);
                const int TX = tile_variant(v).tx, TY = tile_rows(v);
                for (size_t gi = 0; gi < groups.size(); ++gi) {
                    const int si = groups[gi].first;
                    const ShotGeom& g = shots[si];
                    std::vector<unsigned char> full(g.n(), 0), fwd(g.n(), 0);
                    // kind 0 full, 1 interior, 2 frame, 3 z layers
                    auto mark = [&](std::vector<unsigned char>& m, int off, int n, int kind) {
                        for (int i = off; i < off + n; ++i) {
                            const TileEnt& t = out[i];
                            if (t.shot != si) err("wrong shot", i, t.shot, si);
                            if (t.x0 < 0 || t.y0 < 0 || t.z0 < 0 || t.x1 > g.nx || t.y1 > g.ny || t.z1 > g.nz ||
                                t.x1 <= t.x0 || t.y1 <= t.y0 || t.z1 <= t.z0)
                                err("tile outside the grid", t.x0, t.y0, t.z0);
                            const bool var = kind <= 1;
                            const int tw = var ? TX : std::max(CW, ZW), th = var ? TY : std::max(CH, ZH);
                            if (t.x1 - t.x0 > tw || t.y1 - t.y0 > th)
                                err("tile larger than its shape", t.x1 - t.x0, t.y1 - t.y0, kind);
                            if (kind == 3 && !((t.z0 == 0 && t.z1 == p.nb && !fs) || (t.z0 == g.nz - p.nb && t.z1 == g.nz)))
                                err("z-layer chunk", t.z0, t.z1, fs);
                            for (int z = t.z0; z < t.z1; ++z)
                                for (int y = t.y0; y < t.y1; ++y)
                                    for (int x = t.x0; x < t.x1; ++x) {
                                        m[((size_t)z * g.ny + y) * g.nx + x]++;
                                        const bool zl = (!fs && z < p.nb) || z >= g.nz - p.nb;
                                        const bool lay = zl || x < p.nb || x >= g.nx - p.nb || y < p.nb ||
                                                         y >= g.ny - p.nb;
                                        if (kind == 1 && lay) err("layer cell in the interior", x, y, z);
                                        if (kind == 2 && zl) err("z-layer cell in the frame", x, y, z);
                                    }
                        }
                    };
                    // the fused lists are consecutive (one launch may take all three), and a group
                    // run as one launch has all of them in the corner shape
                    if (gt[gi].st_off + gt[gi].nst != gt[gi].zl_off || gt[gi].zl_off + gt[gi].nzl != gt[gi].zc_off)
                        err("fused lists not consecutive", gt[gi].st_off, gt[gi].zl_off, gt[gi].zc_off);
                    if (gt[gi].merged())
                        for (int i = gt[gi].st_off; i < gt[gi].zc_off + gt[gi].nzc; ++i)
                            if (out[i].x1 - out[i].x0 > cstep_tile_w(CS_ZCORNER) ||
                                out[i].y1 - out[i].y0 > cstep_tile_h(CS_ZCORNER))
                                err("tile of a one-launch group larger than the corner shape", i, out[i].x0, out[i].y0);
                    mark(full, gt[gi].full_off, gt[gi].nfull, 0);
                    mark(fwd, gt[gi].in_off, gt[gi].nin, 1);
                    mark(fwd, gt[gi].st_off, gt[gi].nst, 2);
                    mark(fwd, gt[gi].zl_off, gt[gi].nzl, 3);
                    mark(fwd, gt[gi].zc_off, gt[gi].nzc, 3);
                    // z-layer tiles of the plain list (no x / y memory code) meet no x / y layer
                    for (int i = 0; i < gt[gi].nzl; ++i) {
                        const TileEnt& t = out[gt[gi].zl_off + i];
                        if (t.x0 < p.nb || t.x1 > g.nx - p.nb || t.y0 < p.nb || t.y1 > g.ny - p.nb)
                            err("z-layer tile with x / y layer cells in the plain list", t.x0, t.y0, t.z0);
                    }
                    for (size_t i = 0; i < full.size(); ++i)
                        if (full[i] != 1 || fwd[i] != 1) err("cell not written once", (int)i, full[i], fwd[i]);
                    ++cases;
                }
            }
    if (bad) {
        std::printf("tile plans: %ld failures\n", bad);
        return 1;
    }
    std::printf("tile plans: %d cases ok\n", cases);
    return 0;
}
