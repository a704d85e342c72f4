// Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the
// library's host code (FP64 plan generator, C ABI validation and host tables),
// run without a GPU by tests/test_sanitize_host.py.  Exits non-zero when a call
// returns an unexpected status; the sanitizers abort on a memory or UB error.
#include <cstdio>
#include <vector>

#include "dsbt.h"

static int failures = 0;
static void expect(const char* what, dsbt_status got, dsbt_status want) {
    if (got != want) {
        std::printf("FAIL %s: status %d, expected %d (%s)\n", what, got, want, dsbt_last_error());
        ++failures;
    }
}

int main() {
    // FP64 moment tables over the tile sizes and l the plans use
    const int cases[][3] = {{16, 0, 16}, {64, 1, 32}, {256, 2, 32}, {512, 31, 32}, {2048, 63, 32},
                            {1024, 64, 64}, {8192, 127, 64}, {1024, 255, 128}};
    for (const auto& c : cases) {
        int64_t need = 0;
        expect("ftb size", dsbt_host_ftb_tables(c[0], c[1], c[2], nullptr, 0, &need), DSBT_OK);
        std::vector<double> out((size_t)need);
        expect("ftb tables", dsbt_host_ftb_tables(c[0], c[1], c[2], out.data(), need, &need), DSBT_OK);
        double s = 0.0;
        for (double v : out) s += v * v;
        if (!(s > 0.0)) ++failures;
    }
    int64_t need = 0;
    expect("ftb bad N", dsbt_host_ftb_tables(100, 3, 4, nullptr, 0, &need), DSBT_ERR_UNSUPPORTED);
    expect("ftb bad l", dsbt_host_ftb_tables(64, 127, 64, nullptr, 0, &need), DSBT_ERR_UNSUPPORTED);
    expect("ftb bad tile", dsbt_host_ftb_tables(64, 31, 8, nullptr, 0, &need), DSBT_ERR_UNSUPPORTED);

    // kinetic momenta, plain and from the roots of eq. kcorr
    for (int ell : {0, 1, 2, 7, 31, 64, 127}) {
        std::vector<double> k(1024);
        expect("momenta plain", dsbt_kinetic_momenta(1024, ell, 102.4, DSBT_K_PLAIN, k.data()), DSBT_OK);
        expect("momenta corrected", dsbt_kinetic_momenta(1024, ell, 102.4, DSBT_K_CORRECTED, k.data()), DSBT_OK);
    }
    expect("momenta NULL", dsbt_kinetic_momenta(64, 1, 1.0, DSBT_K_PLAIN, nullptr), DSBT_ERR_INVALID_ARG);

    // monomial tables (binary128 expansion)
    for (int ell : {2, 9, 24}) {
        int64_t sz[3];
        expect("monomial sizes", dsbt_host_monomial_tables(256, ell, nullptr, nullptr, nullptr, sz), DSBT_OK);
        std::vector<double> xi(sz[0] + 1), al(sz[1] + 1), cp(sz[2] + 1);
        expect("monomial", dsbt_host_monomial_tables(256, ell, xi.data(), al.data(), cp.data(), sz), DSBT_OK);
    }

    // angular grid and Legendre blocks
    const int ang[][2] = {{1, 1}, {16, 1}, {17, 5}, {64, 63}};
    for (const auto& a : ang) {
        std::vector<double> eta(a[0]), w(a[0]), phi(a[1]), P((size_t)a[1] * a[0] * a[0]);
        expect("sht grid", dsbt_sht_grid(a[0], a[1], eta.data(), w.data(), phi.data()), DSBT_OK);
        expect("sht tables", dsbt_sht_host_tables(a[0], a[1], P.data()), DSBT_OK);
    }
    expect("sht grid even", dsbt_sht_grid(8, 4, nullptr, nullptr, nullptr), DSBT_ERR_UNSUPPORTED);

    // plan creation: argument checks, then no device
    dsbt_plan h = nullptr;
    dsbt_channel ch[2] = {{64, 3, 6.4, 0}, {64, 2, 6.4, 64}};
    dsbt_plan_opts o;
    dsbt_plan_opts_default(&o);
    expect("create NULL out", dsbt_plan_create(nullptr, ch, 2, &o, nullptr), DSBT_ERR_INVALID_ARG);
    o.precision = 9;
    expect("create precision", dsbt_plan_create(&h, ch, 2, &o, nullptr), DSBT_ERR_INVALID_ARG);
    dsbt_plan_opts_default(&o);
    o.check_finite = 3;
    expect("create check_finite", dsbt_plan_create(&h, ch, 2, &o, nullptr), DSBT_ERR_INVALID_ARG);
    dsbt_plan_opts_default(&o);
    const dsbt_status st = dsbt_plan_create(&h, ch, 2, &o, nullptr);
    if (st != DSBT_ERR_NO_DEVICE && st != DSBT_OK) ++failures;
    if (st == DSBT_OK) dsbt_plan_destroy(h);
    const int32_t ells[3] = {0, -1, 2};
    expect("uniform negative l", dsbt_plan_create_uniform(&h, 64, 6.4, ells, 3, 1, nullptr, nullptr),
           DSBT_ERR_UNSUPPORTED);
    expect("forward NULL", dsbt_forward(nullptr, nullptr, nullptr, nullptr), DSBT_ERR_INVALID_ARG);
    expect("inverse NULL", dsbt_inverse(nullptr, nullptr, nullptr, nullptr), DSBT_ERR_INVALID_ARG);
    expect("step NULL", dsbt_kinetic_step(nullptr, nullptr, 1, nullptr, 0, nullptr), DSBT_ERR_INVALID_ARG);
    expect("potential NULL", dsbt_set_potential(nullptr, nullptr, 0.1), DSBT_ERR_INVALID_ARG);
    expect("autotune NULL", dsbt_autotune(nullptr, 0, nullptr, 1, nullptr, nullptr, nullptr, nullptr),
           DSBT_ERR_INVALID_ARG);
    expect("destroy NULL", dsbt_plan_destroy(nullptr), DSBT_OK);
    for (int s = -7; s <= 0; ++s)
        if (!dsbt_status_string(s)) ++failures;
    std::printf("host sanitize driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
