// Sanitizer driver of the host runtime (mm_api.cpp, built with
// -fsanitize=address,undefined by tests/test_host_sanitize.py): the entry
// points that run without a GPU, over many parameter sets, so the layout,
// tile-plan and table code runs under the sanitizers; mm_init_batch with an
// aligned fake workspace stops at its first device call (no GPU here) and
// must free what it built.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/minimod.h"

static int fails = 0;
#define CHECK(x)                                                             \
    do {                                                                     \
        if (!(x)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

int main() {
    mm_params p;
    mm_default_params(&p);
    double dt = 0.0;
    CHECK(mm_dt(&p, 4500.0, &dt) == MM_OK && dt > 0.0);
    CHECK(mm_dt(nullptr, 4500.0, &dt) == MM_ERR_ARG);
    std::vector<float> w(257);
    CHECK(mm_ricker(15.0, 0.1, 1e-3, 257, w.data()) == MM_OK);
    CHECK(mm_ricker(15.0, 0.1, 1e-3, -1, w.data()) == MM_ERR_ARG);
    for (int s = 0; s <= 7; ++s) CHECK(mm_status_str((mm_status)s) != nullptr);
    CHECK(mm_num_tiles() > 0 && mm_tile_name(0) != nullptr && mm_tile_name(-3) != nullptr);
    int32_t src[6] = {5, 6, 7, 1, 2, 3}, rec[9] = {0, 0, 0, 4, 4, 4, 9, 9, 9};
    const int dims[][3] = {{40, 36, 32}, {37, 29, 23}, {64, 64, 64}, {130, 70, 41}, {28, 28, 28}};
    for (const auto& d : dims)
        for (int bc = 0; bc <= 2; ++bc)
            for (int model = 0; model <= 1; ++model)
                for (int fs = 0; fs <= 1; ++fs)
                    for (int ck = 0; ck <= 1; ++ck)
                        for (int nshots = 1; nshots <= 3; nshots += 2) {
                            mm_default_params(&p);
                            p.nx = d[0];
                            p.ny = d[1];
                            p.nz = d[2];
                            p.dx = p.dy = p.dz = 10.0;
                            p.bc = bc;
                            p.nb = bc == 2 ? 6 : (bc == 1 ? 5 : 0);
                            p.model = model;
                            p.free_surface = fs;
                            p.ckpt_every = ck ? 8 : 0;
                            p.snap = ck ? (d[0] & 1) : 0;
                            p.nsteps_max = 40;
                            p.group_kb = nshots > 1 ? 64 : 0;
                            std::vector<mm_shot> shots;
                            for (int i = 0; i < nshots; ++i)
                                shots.push_back(mm_shot{d[0] - i, d[1], d[2] + i, nullptr, src, 2, rec, 3, nullptr});
                            size_t bytes = 0;
                            const mm_status st = mm_workspace_size(&p, nshots, shots.data(), &bytes);
                            // acoustic_iso has no adjoint: rejected
                            if (model == 1 && ck) {
                                CHECK(st != MM_OK);
                                continue;
                            }
                            CHECK(st == MM_OK && bytes > 0);
                            // a context on a fake (aligned, never dereferenced on the host) workspace: the
                            // run stops at the first device call and frees what it built
                            for (auto& s : shots) s.vel = reinterpret_cast<const float*>(0x10000);
                            if (model == 1)
                                for (auto& s : shots) s.rho = reinterpret_cast<const float*>(0x20000);
                            mm_ctx* ctx = nullptr;
                            const mm_status si = mm_init_batch(&ctx, &p, nshots, shots.data(),
                                                               reinterpret_cast<void*>(0x100000), bytes, nullptr);
                            CHECK(si != MM_OK && ctx == nullptr);
                            CHECK(mm_last_error(nullptr) != nullptr);
                        }
    // argument errors
    mm_default_params(&p);
    p.nx = p.ny = p.nz = 10;
    p.bc = 2;
    p.nb = 8;  // too wide for 10 cells
    mm_shot one{10, 10, 10, nullptr, src, 1, rec, 1, nullptr};
    size_t b = 0;
    CHECK(mm_workspace_size(&p, 1, &one, &b) == MM_ERR_ARG);
    mm_ctx* ctx = nullptr;
    CHECK(mm_init_batch(&ctx, &p, 1, &one, nullptr, 0, nullptr) != MM_OK);
    CHECK(mm_init_batch(nullptr, &p, 1, &one, nullptr, 0, nullptr) == MM_ERR_ARG);
    CHECK(mm_snap_blocks(4097) == 2 && mm_snap_blocks(0) == 0);
    CHECK(mm_snap_encode(nullptr, nullptr, -1, nullptr, nullptr, nullptr, nullptr, nullptr) == MM_ERR_ARG);
    mm_destroy(nullptr);
    if (fails) return 1;
    std::printf("host sanitizer driver: ok\n");
    return 0;
}
