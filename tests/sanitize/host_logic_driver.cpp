// Host-side logic of the runtime that needs no GPU, compiled together with
// mm_api.cpp (run by tests/test_host_sanitize.py under the sanitizers): the
// watchdog's schedule and its decoding of the device words, the CPML
// memory width per model, and the default forward CPML strategy.
#include "../../paper_2007_06048_amd/csrc/mm_api.cpp"

static int fails = 0;
#define CHECK(x)                                                             \
    do {                                                                     \
        if (!(x)) {                                                          \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #x); \
            ++fails;                                                         \
        }                                                                    \
    } while (0)

int main() {
    // scanned after steps K, 2K, ...; never when off
    CHECK(!watch_due(0, 5) && !watch_due(4, 5) && watch_due(5, 5) && !watch_due(6, 5) && watch_due(10, 5));
    CHECK(watch_due(1, 1) && watch_due(7, 1));
    for (int s = 0; s < 50; ++s) CHECK(!watch_due(s, 0));
    // device words {flag, first step}
    int32_t bad = 7;
    std::string msg;
    const unsigned clean[2] = {0u, 0xFFFFFFFFu};
    CHECK(watch_result(clean, &bad, &msg) == MM_OK && bad == -1 && msg.empty());
    const unsigned hit[2] = {1u, 40u};
    CHECK(watch_result(hit, &bad, &msg) == MM_ERR_NONFINITE && bad == 40);
    CHECK(msg.find("step 40") != std::string::npos);
    CHECK(watch_result(hit, nullptr, nullptr) == MM_ERR_NONFINITE);
    // parameter check
    mm_params p;
    mm_default_params(&p);
    CHECK(p.watch_every == 0);
    p.watch_every = -1;
    CHECK(check_params(&p, nullptr) == MM_ERR_ARG);
    p.watch_every = 3;
    CHECK(check_params(&p, nullptr) == MM_OK);
    // CPML memory slabs: nb cells per end, one more for acoustic_iso (its last face)
    p.nb = 9;
    p.model = MM_MODEL_ISO_CD;
    CHECK(mem_width(p) == 9);
    p.model = MM_MODEL_ISO;
    CHECK(mem_width(p) == 10);
    // forward CPML strategy without tuning: the layer pass when 30 % or more of the cells lie in a
    // layer (240^3 with 20 cells: 42 %; 1024^2 x 512 with 32 cells: 23 %), or as forced
    p.model = MM_MODEL_ISO_CD;
    p.bc = MM_BC_CPML;
    p.nb = 20;
    p.cpml_kernel = MM_CPML_AUTO;
    CHECK(layer_pass_default(p, {{240, 240, 240}}));
    p.nb = 32;
    CHECK(!layer_pass_default(p, {{1024, 1024, 512}}));
    CHECK(layer_pass_default(p, {{1024, 1024, 512}, {128, 128, 128}}) == false);
    CHECK(layer_pass_default(p, {{128, 128, 128}}));
    p.cpml_kernel = MM_CPML_LAYER;
    CHECK(layer_pass_default(p, {{1024, 1024, 512}}));
    p.cpml_kernel = MM_CPML_FUSED;
    CHECK(!layer_pass_default(p, {{240, 240, 240}}));
    p.cpml_kernel = 3;
    CHECK(check_params(&p, nullptr) == MM_ERR_ARG);
    if (fails) return 1;
    std::printf("host logic: ok\n");
    return 0;
}
