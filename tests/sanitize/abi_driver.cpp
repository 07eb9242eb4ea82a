// Calls every entry point of include/spaimg.h with arguments the host must
// reject before any device work (bad sizes, dimensions, coefficients, batch,
// option values, null pointers and handles), so that a host build with
// -fsanitize=address,undefined checks the argument paths of mg_api.cpp
// (tests/test_sanitize.py).  No call reaches the GPU.  Exit status 0 when
// every call returned MG_EINVAL with a message.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "spaimg.h"

static int failures = 0;

static void expect_einval(int rc, const char* what) {
    if (rc != MG_EINVAL || std::strlen(mg_last_error()) == 0) {
        std::fprintf(stderr, "%s: rc %d, message '%s'\n", what, rc, mg_last_error());
        ++failures;
    }
}

int main() {
    const double c2[3] = {0.2, 0.0, 0.0};
    const double bad[3] = {0.2, std::numeric_limits<double>::quiet_NaN(), 0.0};
    mg_handle_t h = reinterpret_cast<mg_handle_t>(1);
    expect_einval(mg_setup(64, 1, c2, 3, &h), "setup d=1");
    expect_einval(mg_setup(48, 2, c2, 3, &h), "setup N=48");
    expect_einval(mg_setup(2, 2, c2, 3, &h), "setup N=2");
    expect_einval(mg_setup(1 << 17, 2, c2, 3, &h), "setup N too large");
    expect_einval(mg_setup(4096, 3, c2, 2, &h), "setup 3D too large");
    expect_einval(mg_setup(64, 2, c2, 2, &h), "setup coefficient count");
    expect_einval(mg_setup(64, 2, bad, 3, &h), "setup NaN coefficient");
    expect_einval(mg_setup(64, 2, nullptr, 3, &h), "setup null coefficients");
    expect_einval(mg_setup(64, 2, c2, 3, nullptr), "setup null out");
    if (h != nullptr) {
        std::fprintf(stderr, "mg_setup left a handle after failing\n");
        ++failures;
    }
    void* p = reinterpret_cast<void*>(1);  // never dereferenced
    const double* pr = static_cast<const double*>(p);
    double* pw = static_cast<double*>(p);
    expect_einval(mg_vcycle_noalloc(64, 2, c2, 3, 0, pr, pw, nullptr), "noalloc batch 0");
    expect_einval(mg_vcycle_noalloc(2048, 2, c2, 3, 1, pr, pw, nullptr), "noalloc workspace");
    expect_einval(mg_vcycle_noalloc(64, 2, c2, 3, 1, nullptr, pw, nullptr), "noalloc null b");
    expect_einval(mg_vcycle_noalloc(64, 2, bad, 3, 1, pr, pw, nullptr), "noalloc NaN");
    mg_handle_t z = nullptr;
    double d = 0.0;
    int n = 0;
    double cb[3] = {0, 0, 0};
    expect_einval(mg_set_option(z, MG_OPT_BATCH, 2.0), "set_option");
    expect_einval(mg_set_option(z, MG_OPT_BATCH, std::nan("")), "set_option NaN");
    expect_einval(mg_set_coeffs(z, c2, 3), "set_coeffs");
    expect_einval(mg_vcycle(z, pr, pw, nullptr),
                  "vcycle");
    expect_einval(mg_solve(z, pr, pw, 1e-10,
                           nullptr, nullptr), "solve");
    expect_einval(mg_checkpoint(z, pw, p, MG_CKPT_FP32, nullptr),
                  "checkpoint");
    expect_einval(mg_vcycle_adjoint(z, pr, p, MG_CKPT_FP64,
                                    pr, pw,
                                    pw, cb, nullptr), "adjoint");
    expect_einval(mg_sweep(z, MG_OP_SMOOTH, 0, MG_PREC_FP64, p, p, p, nullptr), "sweep");
    expect_einval(mg_sweep_zero_restrict(z, 0, MG_PREC_FP64, p, p, p, nullptr), "zsr");
    expect_einval(mg_sweep_smooth_restrict(z, 0, MG_PREC_FP64, p, p, p, p, nullptr), "sr");
    expect_einval(mg_sweep_post_pre_restrict(z, 0, MG_PREC_FP64, p, p, p, p, p, p, nullptr),
                  "psr");
    expect_einval(mg_sweep_correct(z, 0, MG_PREC_FP64, p, p, p, p, nullptr), "correct");
    expect_einval(mg_coarse_cycle(z, 0, MG_PREC_FP64, p, p, nullptr), "coarse_cycle");
    expect_einval(mg_residual_norm(z, pr,
                                   pr, &d, nullptr), "norm");
    expect_einval(mg_get_timing(z, 0, 0, &d, &n), "get_timing");
    expect_einval(mg_reset_timing(z), "reset_timing");
    expect_einval(mg_num_levels(z), "num_levels");
    mg_destroy(nullptr);
    return failures == 0 ? 0 : 1;
}
