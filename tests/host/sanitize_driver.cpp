// Host-side paths of libsp2 under AddressSanitizer and UBSan: every call
// below returns before its first HIP call (argument checks, workspace
// sizes, status strings, the learned model's create / coefficients / save /
// load / destroy and its text parser on malformed files).  Built against a
// host-only, sanitizer-instrumented build of the library by
// tests/test_host_sanitizers.py; exits non-zero on the first mismatch.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "sp2.h"

static int fails = 0;
#define CHECK(cond)                                                      \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++fails;                                                     \
        }                                                                \
    } while (0)

static void write_file(const std::string& path, const char* text) {
    FILE* f = std::fopen(path.c_str(), "w");
    if (!f) std::exit(3);
    std::fputs(text, f);
    std::fclose(f);
}

int main(int argc, char** argv) {
    const std::string dir = argc > 1 ? argv[1] : ".";
    CHECK(sp2_version() >= 100);
    for (int s = -8; s <= 4; ++s) CHECK(std::strlen(sp2_status_str(s)) > 0);
    // workspace sizes
    for (int n : {1, 2, 63, 64, 65, 1000, 2048, 2049, 4096, 32768}) {
        for (int c = 0; c <= 5; ++c) {
            const size_t b = sp2_workspace_size(n, SP2_F32, (sp2_compute)c);
            CHECK(c == SP2_C_F32 ? b == 0 : b > 0);   // FP32 compute is reserved, not built
        }
        CHECK(sp2_sparse_workspace_size(n) > 0);
        CHECK(sp2_cheb_workspace_size(n, 4) > 0);
    }
    CHECK(sp2_workspace_size(0, SP2_F64, SP2_C_F64) == 0);
    CHECK(sp2_workspace_size(70000, SP2_F64, SP2_C_F64) == 0);
    CHECK(sp2_sparse_workspace_size(70000) == 0);
    CHECK(sp2_cheb_workspace_size(100, 0) == 0);
    // argument checks before any HIP call
    sp2_info info;
    void* H = (void*)(uintptr_t)(1 << 20);
    void* D = (void*)(uintptr_t)(1 << 24);
    void* W = (void*)(uintptr_t)(1 << 28);
    CHECK(sp2_density(H, D, 0, 4, 2, 1e-10, 50, SP2_F64, SP2_C_F64, -1, W, 1 << 30, nullptr, &info) == SP2_E_INVALID);
    CHECK(info.status == SP2_E_INVALID);
    CHECK(sp2_density(H, D, 4, 4, 2, NAN, 50, SP2_F64, SP2_C_F64, -1, W, 1 << 30, nullptr, &info) == SP2_E_INVALID);
    CHECK(sp2_density(H, D, 4, 4, 2, 1e-10, 50, SP2_F64, SP2_C_F64, -1, nullptr, 0, nullptr, &info) ==
          SP2_E_WORKSPACE);
    CHECK(sp2_density_sparse(H, D, 4, 4, 2, 1e-10, 50, SP2_F64, -1.0, W, 1 << 30, nullptr, &info) ==
          SP2_E_INVALID);
    CHECK(sp2_cheb_density(H, D, 64, 64, SP2_F64, 0.0, 1.0, 1, 9, nullptr, 0, nullptr, &info) == SP2_E_INVALID);
    CHECK(sp2_density_noalloc(H, D, 0, 4, 2, 1e-10, 50, SP2_F64, SP2_C_F64, -1, nullptr, &info) == SP2_E_INVALID);
    sp2_plan* plan = nullptr;
    int ns[2] = {64, 4096}, no[2] = {32, 32};
    CHECK(sp2_plan_create(&plan, 2, ns, no, SP2_F64, SP2_C_F64, 1e-10, 50, nullptr) == SP2_E_INVALID);
    CHECK(plan == nullptr);
    sp2_graph* g = nullptr;
    CHECK(sp2_graph_create(&g, H, 32, 32, SP2_F64, -1.0, 4, 1e-10, 50, nullptr) == SP2_E_INVALID);
    CHECK(sp2_graph_create(&g, H, 32, 32, SP2_F64, 0.1, 33, 1e-10, 50, nullptr) == SP2_E_INVALID);
    CHECK(g == nullptr);
    CHECK(sp2_graph_destroy(nullptr) == SP2_E_INVALID);
    // learned model host calls: create, coefficients, save, load, parser errors
    double coef[9] = {1.0, 0.0, 0.0, 1.1, -0.1, 1e-3, 0.7, 0.3, -2.5e-4};
    sp2_learned* m = nullptr;
    CHECK(sp2_learned_create(&m, 3, coef) == SP2_OK && m);
    double back[9] = {0};
    double loss = -1.0;
    CHECK(sp2_learned_coefficients(m, back, 9, &loss) == 3);
    CHECK(sp2_learned_coefficients(m, back, 2, nullptr) == 3);   // short capacity copies nothing past it
    for (int i = 0; i < 9; ++i) CHECK(back[i] == (double)(float)coef[i]);
    const std::string path = dir + "/model.txt";
    CHECK(sp2_learned_save(m, path.c_str()) == SP2_OK);
    sp2_learned* m2 = nullptr;
    CHECK(sp2_learned_load(&m2, path.c_str()) == SP2_OK && m2);
    double back2[9] = {0};
    CHECK(sp2_learned_coefficients(m2, back2, 9, nullptr) == 3);
    for (int i = 0; i < 9; ++i) CHECK(back2[i] == back[i]);
    CHECK(sp2_learned_destroy(m2) == SP2_OK);
    CHECK(sp2_learned_destroy(m) == SP2_OK);
    const char* bad[] = {
        "",
        "not a model\n",
        "sp2_learned 1\n",
        "sp2_learned 1\nlayers -3\nfit_loss 0x0p+0\n",
        "sp2_learned 1\nlayers 100000000\nfit_loss 0x0p+0\n",
        "sp2_learned 1\nlayers 2\nfit_loss 0x0p+0\n0x1p+0 0x0p+0 0x0p+0\n",
        "sp2_learned 1\nlayers 1\nfit_loss 0x0p+0\nnan 0 0\n",
        "sp2_learned 2\nlayers 1\nfit_loss 0x0p+0\n0x1p+0 0x0p+0 0x0p+0\n",
    };
    for (const char* text : bad) {
        const std::string p = dir + "/bad.txt";
        write_file(p, text);
        sp2_learned* mb = nullptr;
        CHECK(sp2_learned_load(&mb, p.c_str()) != SP2_OK);
        CHECK(mb == nullptr);
    }
    CHECK(sp2_learned_load(&m2, (dir + "/missing.txt").c_str()) != SP2_OK);
    double nanc[3] = {1.0, NAN, 0.0};
    CHECK(sp2_learned_create(&m, 1, nanc) != SP2_OK);
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("sanitized host checks passed\n");
    return 0;
}
