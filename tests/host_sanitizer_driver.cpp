// Host-only paths of the C ABI for the AddressSanitizer / UndefinedBehavior-
// Sanitizer build of the runtime (tests/test_host_sanitizers.py): workspace
// sizing over a range of grids and options, every argument check that runs
// before a HIP call, status strings, error text and NULL handles. Needs no
// GPU. Exits non-zero on the first unexpected result.
#include <cstdio>
#include <cstring>

#include "helmg.h"

static int failures = 0;

#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            std::fprintf(stderr, "line %d: expected %s\n", __LINE__, #cond); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

int main() {
    // status strings for every code, and one outside the range
    for (int s = -8; s <= 2; ++s) EXPECT(mg_status_string(static_cast<mg_status>(s)) != nullptr);
    EXPECT(std::strcmp(mg_status_string(MG_E_DIVERGED), "MG_E_DIVERGED") == 0);

    // workspace sizes: valid grids grow with n and with FP32 copies and batch size;
    // grids that do not halve to the coarsest size, too many levels or a coarsest
    // grid too large for the direct solve give 0
    mg_setup_opts o{};
    o.precision = MG_FP64;
    o.max_batch = 1;
    o.coarsest_n = 4;
    size_t prev = 0;
    for (int n = 8; n <= 1024; n *= 2) {
        const size_t w = mg_workspace_bytes(n, 0, MG_TRANSFER_BEZIER, &o);
        EXPECT(w > prev);
        prev = w;
    }
    EXPECT(mg_workspace_bytes(63, 0, MG_TRANSFER_BEZIER, &o) == 0);
    EXPECT(mg_workspace_bytes(64, 9, MG_TRANSFER_BEZIER, &o) == 0);
    EXPECT(mg_workspace_bytes(4096, 3, MG_TRANSFER_BEZIER, &o) == 0);
    EXPECT(mg_workspace_bytes(-64, 0, MG_TRANSFER_BEZIER, &o) == 0);
    mg_setup_opts big = o;
    big.precision = MG_FP32_REFINED;
    big.max_batch = 4;
    EXPECT(mg_workspace_bytes(64, 0, MG_TRANSFER_LINEAR, &big) > mg_workspace_bytes(64, 0, MG_TRANSFER_LINEAR, &o));
    EXPECT(mg_workspace_bytes(64, 0, MG_TRANSFER_BEZIER, nullptr) > 0);  // NULL opts: the defaults
    o.coarsest_n = 6;
    EXPECT(mg_workspace_bytes(96, 0, MG_TRANSFER_BEZIER, &o) > 0);
    o.coarsest_n = 4;

    // setup: each argument check fails before any HIP call (pointers are never
    // dereferenced), with its reason in the thread's last error
    void* fake = reinterpret_cast<void*>(static_cast<size_t>(1) << 20);
    const double* k2 = static_cast<const double*>(fake);
    mg_handle h = nullptr;
    const size_t ws = static_cast<size_t>(1) << 30;
    EXPECT(mg_setup(k2, 64, -1.0, 0.1, 0, MG_TRANSFER_BEZIER, &o, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(std::strstr(mg_last_error(nullptr), "h must be") != nullptr);
    EXPECT(mg_setup(k2, 64, 1.0 / 64, -0.5, 0, MG_TRANSFER_BEZIER, &o, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(mg_setup(k2, 63, 1.0 / 63, 0.1, 0, MG_TRANSFER_BEZIER, &o, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, 7, &o, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(mg_setup(nullptr, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &o, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &o, nullptr, ws, nullptr, &h) == MG_E_WORKSPACE);
    EXPECT(std::strstr(mg_last_error(nullptr), "workspace") != nullptr);
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &o, fake, ws, nullptr, nullptr) == MG_E_ARG);
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &o, fake, 16, nullptr, &h) == MG_E_WORKSPACE);
    mg_setup_opts bad = o;
    bad.max_batch = 0;
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &bad, fake, ws, nullptr, &h) == MG_E_ARG);
    bad = o;
    bad.precision = 9;
    EXPECT(mg_setup(k2, 64, 1.0 / 64, 0.1, 0, MG_TRANSFER_BEZIER, &bad, fake, ws, nullptr, &h) == MG_E_ARG);
    EXPECT(h == nullptr);
    EXPECT(std::strlen(mg_last_error(nullptr)) > 0);

    // entry points that take a handle reject NULL; destroying NULL does nothing
    EXPECT(mg_update_k2(nullptr, k2, nullptr) == MG_E_ARG);
    EXPECT(mg_solve(nullptr, fake, fake, 1, 1e-6, MG_V, MG_GMRES3, nullptr, nullptr, nullptr) == MG_E_ARG);
    EXPECT(mg_destroy(nullptr) == MG_OK);
    return failures == 0 ? 0 : 1;
}
