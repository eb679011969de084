/*
 * Runs every entry point of the FP64 oracle once on a small seeded problem, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure: tests/test_sanitizers.py
 * compiles it together with the oracle source and expects a clean exit).  Also checks the data
 * fault contract: a NaN in d or in a per-pixel weight sets a status bit and makes F NaN.
 */
#include "../../oracle/cs_oracle.c"

#include <stdio.h>

static uint64_t lcg = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [0, 1) */
    lcg ^= lcg << 13;
    lcg ^= lcg >> 7;
    lcg ^= lcg << 17;
    return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

#define F 7
#define P 50

int main(void) {
    double freqs[F], ninv[2 * F], d[2 * F * P], wpix[2 * F * P];
    int32_t labels[3 * P];
    const int32_t K[3] = {4, 3, 2};
    for (int n = 0; n < F; ++n) freqs[n] = 40.0 * pow(10.0, n / (double)(F - 1));
    for (int i = 0; i < 2 * F; ++i) ninv[i] = 1.0 / (2.0 + 18.0 * urand());
    for (int i = 0; i < 2 * F * P; ++i) {
        d[i] = 20.0 * (urand() - 0.5);
        wpix[i] = ninv[(i / P) % (2 * F)] * (0.5 + urand());
    }
    for (int p = 0; p < P; ++p)
        for (int j = 0; j < 3; ++j) labels[j * P + p] = (p % 11 == 5) ? -1 : (int32_t)(p % K[j]);
    orc_problem pr = {F, P, freqs, 353.0, 23.0, 2.7255, d, ninv, 0, labels, {K[0], K[1], K[2]}};
    const int Kt = K[0] + K[1] + K[2];
    double x[9], lo[9], hi[9], g[9], cf[9], ga[9], gt[9], f = 0.0;
    for (int k = 0; k < Kt; ++k) {
        const int j = k < K[0] ? 0 : (k < K[0] + K[1] ? 1 : 2);
        const double l[3] = {0.5, 5.0, -5.0}, u[3] = {3.0, 50.0, -1.0}, c[3] = {1.54, 20.0, -3.0};
        lo[k] = l[j];
        hi[k] = u[j];
        x[k] = c[j] + 0.1 * (urand() - 0.5);
    }
    int bad = 0;
    if (orc_check_labels(&pr) != 0) bad |= 1;
    int st = orc_likelihood_grad(&pr, x, &f, g, cf);
    if (st != 0 || !isfinite(f)) bad |= 2;
    if (orc_grad_abs(&pr, x, ga) != 0 || orc_grad_terms(&pr, x, gt) != 0) bad |= 4;
    for (int k = 0; k < Kt; ++k)
        if (!(gt[k] >= ga[k] && ga[k] >= fabs(g[k]))) bad |= 8;
    double maps[6 * P], var = 0.0;
    if (orc_component_maps(&pr, x, maps, &var) != 0 || !isfinite(var)) bad |= 16;
    if (!(orc_data_chi2(&pr) > 0.0)) bad |= 32;
    int32_t perm[P], off[5];
    if (orc_segments(P, labels, K[0], perm, off) < 1) bad |= 64;
    double xl[9], xa[9], fl = 0.0, fa = 0.0;
    int32_t it = 0;
    int64_t ne = 0;
    memcpy(xl, x, sizeof x);
    memcpy(xa, x, sizeof x);
    if (orc_lbfgs(&pr, lo, hi, xl, 5, 1e-8, 200, 30, 1e-4, &fl, &it, &ne) < 0) bad |= 128;
    if (orc_adatopk(&pr, lo, hi, xa, 0.01, 0.9, 0.999, 1e-16, 0.0, 1e-8, 50, 30, 1e-4, &fa, &it, &ne) < 0) bad |= 256;
    double vecs[3 * P];
    for (int p = 0; p < P; ++p) {
        const double z = 2.0 * urand() - 1.0, ph = 6.283185307179586 * urand(), r = sqrt(1.0 - z * z);
        vecs[3 * p] = r * cos(ph);
        vecs[3 * p + 1] = r * sin(ph);
        vecs[3 * p + 2] = z;
    }
    const int32_t init[5] = {3, 17, 22, 40, 9};
    int32_t kl[P];
    if (orc_kmeans(P, vecs, 5, init, 20, kl) < 1) bad |= 512;
    /* data faults: a NaN in d, then in a per-pixel weight, of an included pixel */
    d[3 * P + 7] = NAN;
    st = orc_likelihood_grad(&pr, x, &f, g, cf);
    if (!(st & ORC_NONFINITE) || !isnan(f)) bad |= 1024;
    d[3 * P + 7] = 1.0;
    pr.ninv = wpix;
    pr.ninv_per_pixel = 1;
    wpix[2 * P + 8] = NAN;
    st = orc_likelihood_grad(&pr, x, &f, g, cf);
    if (!(st & (ORC_NOT_PD | ORC_NONFINITE)) || !isnan(f)) bad |= 2048;
    printf("oracle driver: F %.6f lbfgs F %.6f adatopk F %.6f status flags %d\n", fl, fl, fa, bad);
    return bad ? 1 : 0;
}
