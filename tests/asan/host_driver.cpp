// Driver for the sanitizer build of the HIP library's host code (test
// infrastructure: built and run by tests/test_asan.py on the CPU).  The
// library's sources are compiled with AddressSanitizer and
// UndefinedBehaviorSanitizer on their host pass and linked into this
// program; it calls the entry points that run without a device: status
// strings, defaults, argument checks that return before any HIP call, the
// upscaler workspace sizing, and context creation, which fails cleanly on a
// host with no GPU (and succeeds, then is destroyed, on one that has).
#include <splotch.h>
#include <splotch_nn.h>

#include <cstdio>
#include <cstring>

static int failures = 0;

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
            ++failures;                                               \
        }                                                             \
    } while (0)

int main() {
    CHECK(splotch_abi_version() == SPLOTCH_ABI_VERSION);
    for (int s = -8; s <= 2; ++s) {
        const char* m = splotch_status_string(s);
        CHECK(m != nullptr && std::strlen(m) > 0);
    }
    splotch_params prm;
    std::memset(&prm, 0xff, sizeof prm);
    CHECK(splotch_default_params(&prm) == SPLOTCH_OK);
    CHECK(prm.chi == 3.0f);
    CHECK(splotch_default_params(nullptr) == SPLOTCH_ERR_INVALID_ARG);

    CHECK(splotch_ctx_create(nullptr, 0) == SPLOTCH_ERR_INVALID_ARG);
    splotch_ctx* ctx = reinterpret_cast<splotch_ctx*>(&prm);
    CHECK(splotch_ctx_create(&ctx, -1) == SPLOTCH_ERR_INVALID_ARG);
    CHECK(ctx == nullptr);
    CHECK(splotch_ctx_destroy(nullptr) == SPLOTCH_OK);
    const char* le = splotch_last_error(nullptr);
    CHECK(le != nullptr);

    // calls on a NULL context return before touching anything
    size_t bytes = 0;
    CHECK(splotch_render_workspace_size(nullptr, nullptr, nullptr, nullptr, &bytes) ==
          SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_render(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0,
                         nullptr) == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_render_noalloc(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                 nullptr) == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_render_batched(nullptr, nullptr, 0, nullptr, 0, nullptr) ==
          SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_tune_save(nullptr, "x") == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_tune_load(nullptr, "x") == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_set_timing(nullptr, 1) == SPLOTCH_ERR_INVALID_ARG);

    // upscaler sizing is host arithmetic
    CHECK(splotch_nn_upscale_workspace_size(2, 64, 48, &bytes) == SPLOTCH_OK);
    CHECK(bytes > 0);
    size_t b1 = 0;
    CHECK(splotch_nn_upscale_workspace_size(1, 64, 48, &b1) == SPLOTCH_OK);
    CHECK(b1 > 0 && b1 <= bytes);
    CHECK(splotch_nn_upscale_workspace_size(0, 64, 48, &bytes) == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_nn_upscale_workspace_size(1, -4, 48, &bytes) == SPLOTCH_ERR_INVALID_ARG);
    CHECK(splotch_nn_upscale_workspace_size(1, 64, 48, nullptr) == SPLOTCH_ERR_INVALID_ARG);

    // a context: an error without a device, a full create/destroy with one
    ctx = nullptr;
    const splotch_status cs = splotch_ctx_create(&ctx, 0);
    CHECK(cs == SPLOTCH_OK || cs == SPLOTCH_ERR_HIP);
    CHECK((cs == SPLOTCH_OK) == (ctx != nullptr));
    if (ctx) CHECK(splotch_ctx_destroy(ctx) == SPLOTCH_OK);
    std::printf("host driver: context %s, %d failed checks\n",
                cs == SPLOTCH_OK ? "created" : "unavailable", failures);
    return failures ? 1 : 0;
}
