// Driver for a sanitizer build of the library's host runtime (test
// infrastructure, host code only).
//
// tests/test_sanitizers.py builds liblbm355 with AddressSanitizer and
// UndefinedBehaviorSanitizer on its host code (-Xarch_host) and links this
// driver against it.  The driver goes through the C ABI's argument checks and
// handle checks, which run before any HIP call, plus creation on whatever
// device is present: with no GPU, creation fails with LB_EHIP and a message;
// with one, a small lattice, batch and D2Q9 lattice are created, stepped and
// destroyed.  Prints "sanitize_host_abi ok" and exits 0, else exits 1.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lb.h"

static int failures = 0;

static void expect(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAIL %s (last error: %s)\n", what, lb_last_error());
        ++failures;
    }
}

static bool err_has(const char *needle) { return std::strstr(lb_last_error(), needle) != nullptr; }

int main()
{
    // rejected arguments: no handle, a message naming the argument
    expect(lb_create(0, 8, 8, 0.8, nullptr) == nullptr && err_has("extents"), "zero extent");
    expect(lb_create(8, 8, 8, 0.5, nullptr) == nullptr && err_has("tau"), "tau = 0.5");
    expect(lb_create(8, 8, 8, std::nan(""), nullptr) == nullptr && err_has("tau"), "tau = NaN");
    expect(lb_create(1 << 12, 1 << 12, 1 << 8, 0.8, nullptr) == nullptr && err_has("2^31"), "too many sites");
    std::vector<uint8_t> flags(4 * 3 * 2, 0);
    flags[7] = 2;
    expect(lb_create(4, 3, 2, 0.8, flags.data()) == nullptr && err_has("flag value 2"), "bad flag value");
    expect(lb_create_ex(4, 3, 2, 0.8, nullptr, 7, nullptr) == nullptr && err_has("codec"), "bad codec");

    // dead or null handles
    lb_destroy(nullptr);
    lb_batch_destroy(nullptr);
    lb2d_destroy(nullptr);
    double sums[8];
    expect(lb_step(nullptr, 1) == LB_ESTATE, "lb_step(NULL)");
    expect(lb_step_noalloc(nullptr, 1) == LB_ESTATE, "lb_step_noalloc(NULL)");
    expect(lb_sums(nullptr, sums, 1) == LB_ESTATE, "lb_sums(NULL)");
    expect(lb_macros(nullptr, nullptr, nullptr) == LB_ESTATE, "lb_macros(NULL)");
    expect(lb_batch_step(nullptr, 1) == LB_ESTATE, "lb_batch_step(NULL)");
    expect(lb2d_step(nullptr, 1) == LB_ESTATE, "lb2d_step(NULL)");

    // batches and D2Q9 lattices with bad arguments
    const int dims[6] = {8, 8, 8, 0, 4, 4};
    const double taus[2] = {0.8, 0.8};
    expect(lb_batch_create(2, dims, taus, nullptr, LB_F32, nullptr, 0) == nullptr, "batch with a zero extent");
    expect(lb_batch_create(0, dims, taus, nullptr, LB_F32, nullptr, 0) == nullptr, "empty batch");
    expect(lb2d_create(0, 8, 0.8, nullptr, 0.0, 0.0, nullptr) == nullptr && err_has("extents"), "2d zero extent");

    // creation on the device that is present (none: LB_EHIP with a message)
    lb_lattice *lat = lb_create_ex(16, 6, 4, 0.7, nullptr, LB_F16S, nullptr);
    if (!lat) {
        expect(std::strlen(lb_last_error()) > 0, "a creation failure carries a message");
    } else {
        expect(lb_set_force(lat, 1e-5, 0.0, 0.0) == LB_OK, "set_force");
        expect(lb_init_eq(lat, nullptr, nullptr) == LB_OK, "init_eq");
        expect(lb_step(lat, 70) == LB_OK, "step");
        expect(lb_step_noalloc(lat, 3) == LB_OK, "step_noalloc");
        expect(lb_sums(lat, sums, 2) == LB_OK, "sums");
        lb_destroy(lat);
        const int bd[6] = {8, 6, 4, 12, 5, 3};
        lb_batch *b = lb_batch_create(2, bd, taus, nullptr, LB_F32, nullptr, 0);
        expect(b != nullptr, "batch create");
        if (b) {
            expect(lb_batch_step(b, 66) == LB_OK, "batch step");
            expect(lb_batch_sync(b) == LB_OK, "batch sync");
            lb_batch_destroy(b);
        }
        lb2d_lattice *l2 = lb2d_create(12, 10, 0.6, nullptr, 0.05, 0.0, nullptr);
        expect(l2 != nullptr, "2d create");
        if (l2) {
            expect(lb2d_init_eq(l2, nullptr, nullptr) == LB_OK && lb2d_step(l2, 5) == LB_OK, "2d step");
            lb2d_destroy(l2);
        }
    }
    if (failures) {
        std::printf("sanitize_host_abi: %d failure(s)\n", failures);
        return 1;
    }
    std::printf("sanitize_host_abi ok\n");
    return 0;
}
