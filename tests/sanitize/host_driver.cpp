// Exercises the host layer of the library (no device work: descriptors are validated and laid
// out on the host, and every call that would need a prepared problem must refuse) for a build
// whose host code carries AddressSanitizer and UndefinedBehaviorSanitizer.  Exit 0 = all checks
// held.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "cs.h"

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            std::printf("check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                             \
        }                                                         \
    } while (0)

int main() {
    const int F = 15, P = 1000, B = 6;
    std::vector<double> freqs(F), ninv(2 * F, 0.25);
    for (int f = 0; f < F; ++f) freqs[f] = 40.0 * std::pow(10.0, f / 14.0);
    std::vector<int32_t> ncl(3 * B);
    for (int b = 0; b < B; ++b) {
        ncl[3 * b] = 10 + b;
        ncl[3 * b + 1] = 3;
        ncl[3 * b + 2] = 1 + b;
    }
    cs_problem_desc d{};
    d.nfreq = F;
    d.npix = P;
    d.nitems = B;
    d.freqs_ghz = freqs.data();
    d.nu0_dust_ghz = 353.0;
    d.nu0_sync_ghz = 23.0;
    d.tcmb_k = 2.7255;
    d.precision = CS_FP32_BULK;
    d.d_dtype = CS_DTYPE_F64;
    d.d = (const void *)0x100000;  // never dereferenced before cs_problem_prepare
    d.d_item_stride = 2 * F * P;
    d.ninv_mode = CS_NINV_BAND;
    d.ninv_band = ninv.data();
    d.labels = (const int32_t *)0x200000;
    d.labels_item_stride = 3 * P;
    d.nclusters = ncl.data();

    cs_problem *p = nullptr;
    CHECK(cs_problem_create(&d, &p) == CS_OK && p);
    std::vector<int64_t> off(B + 1);
    CHECK(cs_problem_param_offsets(p, off.data()) == CS_OK && off[1] == 10 + 3 + 1);
    size_t ws = 0;
    CHECK(cs_problem_workspace_bytes(p, &ws) == CS_OK && ws > (size_t)2 * F * P * 4 * B);
    size_t ows = 0;
    CHECK(cs_optimizer_workspace_bytes(p, 10, &ows) == CS_OK && ows > 0);
    CHECK(cs_optimizer_workspace_bytes(p, 33, &ows) == CS_E_INVALID);
    cs_schedule s{2, 0, 1, 1};
    CHECK(cs_problem_set_schedule(p, &s) == CS_OK);
    s.shared_segments = 3;
    CHECK(cs_problem_set_schedule(p, &s) == CS_E_INVALID);
    cs_schedule g{};
    CHECK(cs_problem_get_schedule(p, &g) == CS_OK && g.shared_segments == 1 && g.waves_per_block == 2);
    double *fake = (double *)0x300000;
    CHECK(cs_likelihood(p, fake, fake, nullptr, nullptr) == CS_E_STATE);
    CHECK(cs_likelihood_grad(p, fake, fake, fake, nullptr, nullptr, nullptr) == CS_E_STATE);
    CHECK(cs_component_maps(p, fake, fake, 0, nullptr, nullptr, nullptr) == CS_E_STATE);
    CHECK(cs_problem_autotune(p, fake, fake, fake, 1, nullptr, nullptr) == CS_E_STATE);
    cs_optim_opts o{};
    CHECK(cs_optim_default_opts(&o) == CS_OK && o.m == 10 && o.switch_rel == 1e-4);
    int32_t st = 0, it = 0, running = -1;
    CHECK(cs_optimize_batch_run(p, &o, fake, fake, fake, fake, &it, &st, nullptr, (void *)0x400000, ows, 0, 0, &running,
                                nullptr) == CS_E_STATE && running == 0);
    o.switch_rel = 1.5;
    CHECK(cs_optimize_batch(p, &o, fake, fake, fake, fake, &it, &st, nullptr, (void *)0x400000, ows, nullptr) ==
          CS_E_INVALID);
    int64_t ni = 0, ns = 0;
    CHECK(cs_problem_item_info(p, 0, &ni, &ns) == CS_E_STATE);
    // contiguous chunks tile the items
    int32_t prev = 0;
    for (int k = 0; k < 4; ++k) {
        int32_t b = -1, e = -1;
        CHECK(cs_item_range(k, 4, B, &b, &e) == CS_OK && b == prev && e == (k + 1) * B / 4);
        cs_problem_desc sub{};
        if (e > b) {
            CHECK(cs_problem_desc_slice(&d, b, e, &sub) == CS_OK && sub.nitems == e - b);
            cs_problem *q = nullptr;
            CHECK(cs_problem_create(&sub, &q) == CS_OK);
            std::vector<int64_t> qo(e - b + 1);
            CHECK(cs_problem_param_offsets(q, qo.data()) == CS_OK && qo[e - b] == off[e] - off[b]);
            cs_problem_destroy(q);
        }
        prev = e;
    }
    CHECK(prev == B);
    cs_problem_desc bad = d;
    bad.nfreq = 33;
    cs_problem *q = nullptr;
    CHECK(cs_problem_create(&bad, &q) == CS_E_UNSUPPORTED && !q && std::strlen(cs_last_error()) > 0);
    bad = d;
    bad.labels_item_stride = 5;
    CHECK(cs_problem_create(&bad, &q) == CS_E_INVALID);
    for (int c = 0; c <= 6; ++c) CHECK(std::strlen(cs_status_str((cs_status)c)) > 0);
    cs_problem_destroy(p);
    cs_problem_destroy(nullptr);
    std::printf("host driver: all checks held\n");
    return 0;
}
