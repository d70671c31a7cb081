// Host-side argument checks of the C ABI under AddressSanitizer and
// UndefinedBehaviorSanitizer.  Linked against a host-only build of the
// library (no device code), so it runs without a GPU: every call below is
// rejected by the host code before any HIP call.  Prints "abi ok" when
// every status and message is as documented; any sanitizer report aborts.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "feasm.h"

static int failures = 0;

static void expect(int got, int want, const char* what, const char* msg_part) {
    const char* msg = last_error();
    const bool msg_ok = msg_part == nullptr || (msg && std::strstr(msg, msg_part));
    if (got != want || !msg_ok) {
        std::printf("FAIL %s: status %d (want %d), message \"%s\"\n", what, got, want,
                    msg ? msg : "(null)");
        ++failures;
    }
}

static void* fake_alloc(size_t, hipStream_t, void*) { return nullptr; }
static void fake_release(void*, hipStream_t, void*) {}

int main() {
    // never dereferenced: validation fails before any use
    const int32_t* conn = reinterpret_cast<const int32_t*>(0x1000);
    double* dptr = reinterpret_cast<double*>(0x2000);
    feasm_pattern* h = reinterpret_cast<feasm_pattern*>(0x3000);

    feasm_pattern* out = h;
    expect(pattern_build(nullptr, 4, 4, 1, 9, FEASM_BUILD_CSR, nullptr, &out), FEASM_EINVAL,
           "pattern_build null conn", "pattern_build");
    if (out != nullptr) {
        std::printf("FAIL pattern_build left a handle on failure\n");
        ++failures;
    }
    expect(pattern_build(conn, 0, 4, 1, 9, FEASM_BUILD_CSR, nullptr, &out), FEASM_EINVAL,
           "pattern_build n_elem 0", nullptr);
    expect(pattern_build(conn, 4, 4, 1, 9, 0, nullptr, &out), FEASM_EINVAL,
           "pattern_build no format", nullptr);
    expect(pattern_build(conn, 4, 4, 1, 9, 64, nullptr, &out), FEASM_EINVAL,
           "pattern_build unknown flag", nullptr);
    expect(pattern_build(conn, int64_t(1) << 30, 4, 1, 9, FEASM_BUILD_CSR, nullptr, &out),
           FEASM_EOVERFLOW, "pattern_build too many entries", nullptr);
    expect(pattern_build(conn, 4, 100, 50, 9, FEASM_BUILD_CSR, nullptr, &out), FEASM_ELIMIT,
           "pattern_build element too large", nullptr);
    expect(pattern_build(conn, 4, 4, 1, 9, FEASM_BUILD_CSR, nullptr, nullptr), FEASM_EINVAL,
           "pattern_build null out", nullptr);

    expect(assemble_csr(nullptr, dptr, dptr, 0, nullptr), FEASM_EINVAL, "assemble_csr",
           "null handle");
    expect(assemble_crac(nullptr, dptr, dptr, 0, nullptr), FEASM_EINVAL, "assemble_crac",
           "null handle");
    expect(reassemble_values(nullptr, 0, dptr, dptr, 0, nullptr), FEASM_EINVAL,
           "reassemble_values", "null handle");
    expect(pattern_info(nullptr, nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL, "pattern_info",
           nullptr);
    expect(pattern_arrays(nullptr, nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL,
           "pattern_arrays", nullptr);
    expect(pattern_colouring(nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL,
           "pattern_colouring", nullptr);
    expect(pattern_tune(nullptr, 1, 0), FEASM_EINVAL, "pattern_tune", nullptr);
    expect(spmv_csr(nullptr, dptr, dptr, dptr, nullptr), FEASM_EINVAL, "spmv_csr", "null handle");
    expect(spmv_crac(nullptr, dptr, dptr, dptr, nullptr), FEASM_EINVAL, "spmv_crac", "null handle");
    expect(hex8_element_matrices(nullptr, dptr, dptr, dptr, nullptr), FEASM_EINVAL,
           "hex8_element_matrices", nullptr);
    expect(assemble_hex8(nullptr, 1, dptr, dptr, dptr, 0, nullptr), FEASM_EINVAL, "assemble_hex8",
           "null handle");
    int64_t count = 0;
    expect(spin_aborts(nullptr, &count), FEASM_EINVAL, "spin_aborts", nullptr);
    expect(assemble_spin_noalloc(nullptr, FEASM_FMT_CSR, dptr, dptr, nullptr, 0, nullptr),
           FEASM_EINVAL, "assemble_spin_noalloc", "null handle");

    expect(generate_ke(0, 4, 4, 1, 0, nullptr, nullptr), FEASM_EINVAL, "generate_ke null", nullptr);
    expect(generate_ke(2, 4, 4, 1, 0, dptr, nullptr), FEASM_EINVAL, "generate_ke recipe", nullptr);
    expect(generate_ke(1, 4, 91, 1, 0, dptr, nullptr), FEASM_ELIMIT, "generate_ke size", nullptr);
    expect(generate_ke(1, 0, 24, 1, 0, dptr, nullptr), FEASM_OK, "generate_ke empty", nullptr);

    feasm_batch* b = nullptr;
    expect(batch_create(nullptr, 1, 0, 0, &b), FEASM_EINVAL, "batch_create null", nullptr);
    expect(batch_create(&h, 0, 0, 0, &b), FEASM_EINVAL, "batch_create empty", nullptr);
    expect(assemble_batch(nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL, "assemble_batch",
           nullptr);
    expect(batch_info(nullptr, nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL, "batch_info",
           nullptr);
    expect(serve_run(nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, nullptr), FEASM_EINVAL,
           "serve_run", nullptr);
    {
        feasm_serve_mesh mesh{};
        mesh.conn = conn;
        mesh.n_elem = 4;
        mesh.nodes_per_elem = 4;
        mesh.dofs_per_node = 1;
        mesh.n_nodes = 9;
        feasm_serve_config cfg{};
        cfg.fmt = FEASM_FMT_CRAC;
        cfg.slots = 0;
        expect(serve_run(&mesh, 1, nullptr, 0, &cfg, nullptr, nullptr, nullptr), FEASM_EINVAL,
               "serve_run slots", "slots");
        cfg.slots = 2;
        mesh.recipe = 5;
        expect(serve_run(&mesh, 1, nullptr, 0, &cfg, nullptr, nullptr, nullptr), FEASM_EINVAL,
               "serve_run recipe", "recipe");
        mesh.recipe = 0;
        mesh.conn = nullptr;
        expect(serve_run(&mesh, 1, nullptr, 0, &cfg, nullptr, nullptr, nullptr), FEASM_EINVAL,
               "serve_run no mesh", "connectivity");
    }

    expect(set_allocator(fake_alloc, nullptr, nullptr), FEASM_EINVAL, "set_allocator half",
           "both");
    expect(set_allocator(nullptr, fake_release, nullptr), FEASM_EINVAL, "set_allocator half",
           "both");
    expect(set_allocator(nullptr, nullptr, nullptr), FEASM_OK, "set_allocator default", nullptr);

    pattern_free(nullptr);
    batch_free(nullptr);
    if (failures == 0) std::printf("abi ok\n");
    return failures == 0 ? 0 : 1;
}
