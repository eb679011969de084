/*
 * cs_oracle.c -- FP64 CPU oracle for clustered parametric component separation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity reference for the HIP library: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code, header, table or helper with the library under paper_2604_08463_amd/.
 *
 * Plain, single-threaded, double precision, ascending pixel order, no blocking or fusion.  Each
 * function states the passage of the paper it follows (arXiv 2604.08463):
 *   Sec. 2.1, eq. (data_model)          d_p = A_p(beta_p) s_p + n_p
 *   Sec. 2.1, eq. (mixing_columns)      CMB = 1; dust modified blackbody; synchrotron power law
 *   Sec. 2.1, eq. (mle_solution)        s_hat = (A^T N^-1 A)^-1 A^T N^-1 d
 *   Sec. 2.1, eq. (spectral_likelihood) ln L_spec = const + 1/2 sum_p b^T M^-1 b
 *   Sec. 2.2                            beta_p = beta_k for p in patch k; spherical K-means
 *                                       (mean of unit vectors renormalised, angular distance)
 *   Sec. 2.3                            one independent patching per spectral parameter
 *   Sec. 2.3, eq. (recon_operator)      component maps s_hat = W d
 *   Sec. 2.4, eq. (min_var)             variance of the reconstructed CMB over the mask
 *   Sec. 3.3.1 (gradient equation)      gradient from the GLS residuals with s held fixed
 *   App. A.1 and Alg. 1                 affine internal box [0,1], clamp to the nearest bound
 *   App. A (AdaTopK)                    AdaBelief steps, Top-K release, rescaling, step limit
 *
 * Readings where the paper is silent (each one also listed in the design notes):
 *   - objective F = -2 ln L_spec with the constant dropped: F = -sum_p sum_{Q,U} b^T M^-1 b;
 *     its gradient is -2 r^T (dA/dtheta) s_hat, i.e. minus the printed gradient of ln L_spec
 *     scaled by 2 (the printed one is the gradient of 2 ln L_spec).
 *   - dust and synchrotron columns are converted from Rayleigh-Jeans to CMB units with
 *     g(nu) = (e^y - 1)^2 / (y^2 e^y), y = h nu / (k T_CMB), normalised to 1 at nu0.
 *   - h and k take their exact SI values; bands are delta functions at their centres.
 *   - Q and U share the spectral parameters and have independent amplitudes.
 *   - parity unpinned: nothing (see the oracle tests for the pin of each function).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NOT_PD 1
#define ORC_NONFINITE 2
#define ORC_LS_FAIL 4
#define ORC_MAXITER 8
#define ORC_CONVERGED 16

#define ORC_FLAT_REL 1e-12

#define ORC_E_INVALID (-1)
#define ORC_E_LABEL (-2)

/* h/k in kelvin per GHz from the exact SI values of h and k */
static const double ORC_H_OVER_K = 6.62607015e-34 / 1.380649e-23 * 1.0e9;

typedef struct {
    int32_t nfreq;
    int32_t npix;
    const double *freqs;       /* [F] band centres in GHz                                    */
    double nu0_dust, nu0_sync; /* reference frequencies of the dust / synchrotron columns  */
    double tcmb;               /* CMB temperature in K                                     */
    const double *d;           /* [2][F][P] Q/U data, uK_CMB                               */
    const double *ninv;        /* [2][F] (per band) or [2][F][P] (per pixel), uK^-2        */
    int32_t ninv_per_pixel;
    const int32_t *labels;     /* [3][P] cluster of each pixel per parameter; -1 = excluded */
    int32_t nclusters[3];      /* K_d, K_T, K_s                                            */
} orc_problem;

/* ------------------------------------------------------------------------------------------ */
/* Neumaier compensated summation                                                             */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    double s, c;
} orc_sum;

static void orc_add(orc_sum *a, double v) {
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double orc_val(const orc_sum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------------------------------ */
/* Mixing-matrix columns, Sec. 2.1 eq. (mixing_columns), in CMB thermodynamic units           */
/* ------------------------------------------------------------------------------------------ */

/* RJ -> K_CMB conversion factor g(nu) = (e^y - 1)^2 / (y^2 e^y), y = h nu / (k T_CMB) */
double orc_rj_to_cmb(double nu_ghz, double tcmb) {
    double y = ORC_H_OVER_K * nu_ghz / tcmb;
    double em1 = expm1(y);
    return em1 * em1 / (y * y * exp(y));
}

/*
 * Columns of one band for one parameter set, plus their parameter derivatives:
 *   a_d = (nu/nu0d)^(beta_d+1) * expm1(h nu0d/kT) / expm1(h nu/kT) * g(nu)/g(nu0d)
 *   a_s = (nu/nu0s)^beta_s * g(nu)/g(nu0s)
 *   da_d/dbeta_d = a_d ln(nu/nu0d)
 *   da_d/dT_d    = a_d / T_d * [x/(1-e^-x) - x0/(1-e^-x0)],  x = h nu/kT, x0 = h nu0d/kT
 *   da_s/dbeta_s = a_s ln(nu/nu0s)
 */
void orc_sed(double nu, double nu0d, double nu0s, double tcmb, double beta_d, double temp_d,
             double beta_s, double *a_d, double *a_s, double *dad_dbeta, double *dad_dtemp,
             double *das_dbeta) {
    double x = ORC_H_OVER_K * nu / temp_d;
    double x0 = ORC_H_OVER_K * nu0d / temp_d;
    double ad = pow(nu / nu0d, beta_d + 1.0) * expm1(x0) / expm1(x) * orc_rj_to_cmb(nu, tcmb) /
                orc_rj_to_cmb(nu0d, tcmb);
    double as = pow(nu / nu0s, beta_s) * orc_rj_to_cmb(nu, tcmb) / orc_rj_to_cmb(nu0s, tcmb);
    *a_d = ad;
    *a_s = as;
    if (dad_dbeta) *dad_dbeta = ad * log(nu / nu0d);
    if (dad_dtemp) *dad_dtemp = ad / temp_d * (x / (-expm1(-x)) - x0 / (-expm1(-x0)));
    if (das_dbeta) *das_dbeta = as * log(nu / nu0s);
}

/* ------------------------------------------------------------------------------------------ */
/* 3x3 solve by LU with partial pivoting (Sec. 2.1 eq. mle_solution)                          */
/* ------------------------------------------------------------------------------------------ */
static int orc_lu_solve3(const double m[9], const double b[3], double xout[3]) {
    double a[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) a[i][j] = m[3 * i + j];
        a[i][3] = b[i];
    }
    for (int k = 0; k < 3; ++k) {
        int piv = k;
        for (int i = k + 1; i < 3; ++i)
            if (fabs(a[i][k]) > fabs(a[piv][k])) piv = i;
        if (a[piv][k] == 0.0) return 1;
        if (piv != k)
            for (int j = 0; j < 4; ++j) {
                double t = a[k][j];
                a[k][j] = a[piv][j];
                a[piv][j] = t;
            }
        for (int i = k + 1; i < 3; ++i) {
            double f = a[i][k] / a[k][k];
            for (int j = k; j < 4; ++j) a[i][j] -= f * a[k][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = a[i][3];
        for (int j = i + 1; j < 3; ++j) s -= a[i][j] * xout[j];
        xout[i] = s / a[i][i];
    }
    return 0;
}

/* Positive definiteness of the symmetric 3x3 M (Sylvester's criterion, read numerically): each
 * leading principal minor must be positive relative to the product of its diagonal entries,
 * minor_k > ORC_PD_REL * m_00 ... m_kk, so that a rank-deficient M (fewer bands than components,
 * or degenerate columns) is flagged whatever sign rounding gives its determinant. */
#define ORC_PD_REL 1e-12
static int orc_is_pd3(const double m[9]) {
    double m1 = m[0];
    double m2 = m[0] * m[4] - m[1] * m[3];
    double m3 = m[0] * (m[4] * m[8] - m[5] * m[7]) - m[1] * (m[3] * m[8] - m[5] * m[6]) +
                m[2] * (m[3] * m[7] - m[4] * m[6]);
    return m1 > 0.0 && m2 > ORC_PD_REL * m[0] * m[4] && m3 > ORC_PD_REL * m[0] * m[4] * m[8];
}

/* ------------------------------------------------------------------------------------------ */
/* Label checks (Sec. 2.2 / 2.3): each label in [0, K_j) or -1, and -1 on all three together  */
/* ------------------------------------------------------------------------------------------ */
int orc_check_labels(const orc_problem *pr) {
    if (!pr || pr->nfreq < 1 || pr->npix < 0 || !pr->labels) return ORC_E_INVALID;
    for (int j = 0; j < 3; ++j)
        if (pr->nclusters[j] < 1) return ORC_E_INVALID;
    int64_t P = pr->npix;
    for (int64_t p = 0; p < P; ++p) {
        int excl = 0;
        for (int j = 0; j < 3; ++j) {
            int32_t l = pr->labels[j * P + p];
            if (l == -1)
                ++excl;
            else if (l < 0 || l >= pr->nclusters[j])
                return ORC_E_LABEL;
        }
        if (excl != 0 && excl != 3) return ORC_E_LABEL;
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* One pixel: GLS solve, likelihood term and its gradient (Sec. 2.1, Sec. 3.3.1)             */
/* ------------------------------------------------------------------------------------------ */
/*
 * Outputs (each nullable): mout[2][9] = A^T N^-1 A per Stokes, bout[2][3] = A^T N^-1 d,
 * sout[2][3] = s_hat, rout[2][F] = N^-1 (d - A s_hat), fout = -sum_s b.s_hat,
 * gout[3] = dfout/d(beta_d, T_d, beta_s).  Returns status bits.
 */
int orc_pixel(const orc_problem *pr, const double *x, int32_t p, double *mout, double *bout,
              double *sout, double *rout, double *fout, double *gout) {
    const int F = pr->nfreq;
    const int64_t P = pr->npix;
    const int32_t kd = pr->labels[p], kt = pr->labels[P + p], ks = pr->labels[2 * P + p];
    const double beta_d = x[kd];
    const double temp_d = x[pr->nclusters[0] + kt];
    const double beta_s = x[pr->nclusters[0] + pr->nclusters[1] + ks];
    int status = 0;
    double f = 0.0, g[3] = {0.0, 0.0, 0.0};

    double *ad = (double *)malloc(sizeof(double) * 5 * (size_t)F);
    double *as = ad + F, *dbd = ad + 2 * F, *dtd = ad + 3 * F, *dbs = ad + 4 * F;
    for (int n = 0; n < F; ++n)
        orc_sed(pr->freqs[n], pr->nu0_dust, pr->nu0_sync, pr->tcmb, beta_d, temp_d, beta_s, &ad[n],
                &as[n], &dbd[n], &dtd[n], &dbs[n]);

    for (int s = 0; s < 2; ++s) {
        double m[9] = {0}, b[3] = {0}, sh[3];
        for (int n = 0; n < F; ++n) {
            double w = pr->ninv_per_pixel ? pr->ninv[((int64_t)s * F + n) * P + p] : pr->ninv[s * F + n];
            double dv = pr->d[((int64_t)s * F + n) * P + p];
            double a[3] = {1.0, ad[n], as[n]};
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j) m[3 * i + j] += w * a[i] * a[j];
                b[i] += w * a[i] * dv;
            }
        }
        if (!orc_is_pd3(m)) status |= ORC_NOT_PD;
        if (orc_lu_solve3(m, b, sh)) {
            status |= ORC_NOT_PD;
            sh[0] = sh[1] = sh[2] = NAN;
        }
        f -= b[0] * sh[0] + b[1] * sh[1] + b[2] * sh[2];
        /* residual form of the gradient: dF/dtheta = -2 sum_nu r_nu (dA_nu/dtheta) s_hat */
        for (int n = 0; n < F; ++n) {
            double w = pr->ninv_per_pixel ? pr->ninv[((int64_t)s * F + n) * P + p] : pr->ninv[s * F + n];
            double dv = pr->d[((int64_t)s * F + n) * P + p];
            double r = w * (dv - (sh[0] + ad[n] * sh[1] + as[n] * sh[2]));
            if (rout) rout[s * F + n] = r;
            g[0] += -2.0 * r * dbd[n] * sh[1];
            g[1] += -2.0 * r * dtd[n] * sh[1];
            g[2] += -2.0 * r * dbs[n] * sh[2];
        }
        if (mout) memcpy(mout + 9 * s, m, sizeof m);
        if (bout) memcpy(bout + 3 * s, b, sizeof b);
        if (sout) memcpy(sout + 3 * s, sh, sizeof sh);
    }
    free(ad);
    if (!isfinite(f) || !isfinite(g[0]) || !isfinite(g[1]) || !isfinite(g[2])) status |= ORC_NONFINITE;
    if (fout) *fout = f;
    if (gout) memcpy(gout, g, sizeof g);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Whole problem: F = sum_p f_p, per-cluster gradient and per-cluster likelihood partials     */
/* ------------------------------------------------------------------------------------------ */
/*
 * x, grad, cluster_f are packed [beta_d (K_d) | T_d (K_T) | beta_s (K_s)].  cluster_f[k] of
 * labelling j is the sum of f_p over the pixels of cluster k; each labelling's partials sum to
 * F.  Sums are Neumaier-compensated in ascending pixel order.  On a non-PD pixel F is NaN.
 * Returns status bits (>= 0) or a negative error code.
 */
int orc_likelihood_grad(const orc_problem *pr, const double *x, double *neg2logl, double *grad,
                        double *cluster_f) {
    int rc = orc_check_labels(pr);
    if (rc) return rc;
    const int64_t P = pr->npix;
    const int K = pr->nclusters[0] + pr->nclusters[1] + pr->nclusters[2];
    const int off[3] = {0, pr->nclusters[0], pr->nclusters[0] + pr->nclusters[1]};
    orc_sum *gs = (orc_sum *)calloc((size_t)K * 2, sizeof(orc_sum));
    orc_sum *fs = gs + K;
    orc_sum tot = {0.0, 0.0};
    int status = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (pr->labels[p] < 0) continue;
        double f, g[3];
        status |= orc_pixel(pr, x, (int32_t)p, NULL, NULL, NULL, NULL, &f, g);
        orc_add(&tot, f);
        for (int j = 0; j < 3; ++j) {
            int k = off[j] + pr->labels[j * P + p];
            orc_add(&gs[k], g[j]);
            orc_add(&fs[k], f);
        }
    }
    if (neg2logl) *neg2logl = (status & ORC_NOT_PD) ? NAN : orc_val(&tot);
    for (int k = 0; k < K; ++k) {
        if (grad) grad[k] = orc_val(&gs[k]);
        if (cluster_f) cluster_f[k] = orc_val(&fs[k]);
    }
    free(gs);
    return status;
}

/*
 * Scale of each cluster's gradient sum: gabs[k] = sum over the cluster's pixels of |dF_p/dtheta_k|
 * (packed like grad).  The gradient of a cluster is a sum of per-pixel terms of both signs that
 * nearly cancel at an optimum, so its rounding error is bounded relative to this sum, not to the
 * gradient itself: the per-cluster tolerance is stated against it.  Plain sums in ascending pixel
 * order.  Returns status bits (>= 0) or a negative error code.
 */
int orc_grad_abs(const orc_problem *pr, const double *x, double *gabs) {
    int rc = orc_check_labels(pr);
    if (rc) return rc;
    const int64_t P = pr->npix;
    const int K = pr->nclusters[0] + pr->nclusters[1] + pr->nclusters[2];
    const int off[3] = {0, pr->nclusters[0], pr->nclusters[0] + pr->nclusters[1]};
    for (int k = 0; k < K; ++k) gabs[k] = 0.0;
    int status = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (pr->labels[p] < 0) continue;
        double f, g[3];
        status |= orc_pixel(pr, x, (int32_t)p, NULL, NULL, NULL, NULL, &f, g);
        for (int j = 0; j < 3; ++j) gabs[off[j] + pr->labels[j * P + p]] += fabs(g[j]);
    }
    return status;
}

/*
 * Magnitude of the terms that make up each cluster's gradient (packed like grad): with the
 * residual expanded, r_nu = w_nu (d_nu - sum_j a_j(nu) s_j), a pixel's derivative is a signed sum
 * of the terms -2 w (dA/dtheta)_nu s_c d_nu and +2 w (dA/dtheta)_nu s_c a_j(nu) s_j, and
 *     gterm[k] = sum over the cluster's pixels, both Stokes parameters and all bands of
 *                2 |s_c| w |(dA/dtheta)_nu| (|d_nu| + sum_j |a_j(nu)| |s_j|).
 * A sum of these terms accumulated in a working precision of unit roundoff u is in error by at
 * most about (number of terms) u gterm[k] whatever their cancellation, so the FP32 tolerances
 * are stated against it.  gterm[k] >= gabs[k] (triangle inequality).  Plain sums in ascending
 * pixel order.  Returns status bits (>= 0) or a negative error code.
 */
int orc_grad_terms(const orc_problem *pr, const double *x, double *gterm) {
    int rc = orc_check_labels(pr);
    if (rc) return rc;
    const int F = pr->nfreq;
    const int64_t P = pr->npix;
    const int K = pr->nclusters[0] + pr->nclusters[1] + pr->nclusters[2];
    const int off[3] = {0, pr->nclusters[0], pr->nclusters[0] + pr->nclusters[1]};
    for (int k = 0; k < K; ++k) gterm[k] = 0.0;
    int status = 0;
    for (int64_t p = 0; p < P; ++p) {
        if (pr->labels[p] < 0) continue;
        double sh[6];
        status |= orc_pixel(pr, x, (int32_t)p, NULL, NULL, sh, NULL, NULL, NULL);
        const double beta_d = x[pr->labels[p]];
        const double temp_d = x[off[1] + pr->labels[P + p]];
        const double beta_s = x[off[2] + pr->labels[2 * P + p]];
        double t[3] = {0.0, 0.0, 0.0};
        for (int n = 0; n < F; ++n) {
            double ad, as, dbd, dtd, dbs;
            orc_sed(pr->freqs[n], pr->nu0_dust, pr->nu0_sync, pr->tcmb, beta_d, temp_d, beta_s, &ad, &as, &dbd,
                    &dtd, &dbs);
            for (int s = 0; s < 2; ++s) {
                const double w = pr->ninv_per_pixel ? pr->ninv[((int64_t)s * F + n) * P + p] : pr->ninv[s * F + n];
                const double dv = pr->d[((int64_t)s * F + n) * P + p];
                const double *q = sh + 3 * s;
                const double mag = w * (fabs(dv) + fabs(q[0]) + fabs(ad) * fabs(q[1]) + fabs(as) * fabs(q[2]));
                t[0] += 2.0 * fabs(q[1]) * fabs(dbd) * mag;
                t[1] += 2.0 * fabs(q[1]) * fabs(dtd) * mag;
                t[2] += 2.0 * fabs(q[2]) * fabs(dbs) * mag;
            }
        }
        for (int j = 0; j < 3; ++j) gterm[off[j] + pr->labels[j * P + p]] += t[j];
    }
    return status;
}

/* d^T N^-1 d over the included pixels (the data term of the joint chi^2, Sec. 2.1 eq. nll_joint) */
double orc_data_chi2(const orc_problem *pr) {
    const int F = pr->nfreq;
    const int64_t P = pr->npix;
    orc_sum t = {0.0, 0.0};
    for (int64_t p = 0; p < P; ++p) {
        if (pr->labels[p] < 0) continue;
        for (int s = 0; s < 2; ++s)
            for (int n = 0; n < F; ++n) {
                double w = pr->ninv_per_pixel ? pr->ninv[((int64_t)s * F + n) * P + p] : pr->ninv[s * F + n];
                double dv = pr->d[((int64_t)s * F + n) * P + p];
                orc_add(&t, w * dv * dv);
            }
    }
    return orc_val(&t);
}

/* ------------------------------------------------------------------------------------------ */
/* Component maps s_hat = W d (Sec. 2.3 eq. recon_operator) and the CMB map variance           */
/* sigma^2_CMB = Var_{p in M}[s_hat_CMB,p] summed over Q and U (Sec. 2.4 eq. min_var)           */
/* ------------------------------------------------------------------------------------------ */
/*
 * s_out[2][3][P] (nullable): the GLS amplitudes (CMB, dust, synchrotron) per Stokes and pixel;
 * NaN at excluded pixels and at pixels whose A^T N^-1 A is not positive definite.  cmb_var
 * (nullable): population variance over the included pixels of s_hat_CMB for Q plus that for U
 * (two-pass, Neumaier sums in ascending pixel order); NaN if a pixel is not positive definite or
 * no pixel is included.
 */
int orc_component_maps(const orc_problem *pr, const double *x, double *s_out, double *cmb_var) {
    int rc = orc_check_labels(pr);
    if (rc) return rc;
    const int64_t P = pr->npix;
    int status = 0;
    double *cmb = (double *)malloc(sizeof(double) * 2 * (size_t)(P > 0 ? P : 1));
    int64_t n = 0;
    for (int64_t p = 0; p < P; ++p) {
        double sh[6];
        if (pr->labels[p] < 0) {
            if (s_out)
                for (int k = 0; k < 6; ++k) s_out[k * P + p] = NAN;
            continue;
        }
        const int st = orc_pixel(pr, x, (int32_t)p, NULL, NULL, sh, NULL, NULL, NULL);
        status |= st;
        if (st & ORC_NOT_PD)
            for (int k = 0; k < 6; ++k) sh[k] = NAN;
        if (s_out)
            for (int k = 0; k < 6; ++k) s_out[k * P + p] = sh[k];
        cmb[2 * n] = sh[0];
        cmb[2 * n + 1] = sh[3];
        ++n;
    }
    if (cmb_var && (n == 0 || (status & ORC_NOT_PD))) {
        *cmb_var = NAN;
    } else if (cmb_var) {
        double var = 0.0;
        for (int s = 0; s < 2 && n > 0; ++s) {
            orc_sum m = {0.0, 0.0}, v = {0.0, 0.0};
            for (int64_t i = 0; i < n; ++i) orc_add(&m, cmb[2 * i + s]);
            double mean = orc_val(&m) / (double)n;
            for (int64_t i = 0; i < n; ++i) {
                double dv = cmb[2 * i + s] - mean;
                orc_add(&v, dv * dv);
            }
            var += orc_val(&v) / (double)n;
        }
        *cmb_var = var;
    }
    free(cmb);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Segments of one labelling: stable counting sort of pixel indices by cluster (Sec. 2.2)     */
/* ------------------------------------------------------------------------------------------ */
/*
 * perm[n_incl] lists the included pixels grouped by cluster, ascending pixel index inside a
 * cluster; offsets[K+1] is the exclusive prefix sum of the cluster sizes.  Returns n_incl, or a
 * negative error on an out-of-range label.
 */
int64_t orc_segments(int64_t npix, const int32_t *labels, int32_t k, int32_t *perm, int32_t *offsets) {
    for (int32_t c = 0; c <= k; ++c) offsets[c] = 0;
    for (int64_t p = 0; p < npix; ++p) {
        int32_t l = labels[p];
        if (l == -1) continue;
        if (l < 0 || l >= k) return ORC_E_LABEL;
        offsets[l + 1] += 1;
    }
    for (int32_t c = 0; c < k; ++c) offsets[c + 1] += offsets[c];
    int32_t *fill = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k > 0 ? k : 1));
    for (int32_t c = 0; c < k; ++c) fill[c] = offsets[c];
    for (int64_t p = 0; p < npix; ++p) {
        int32_t l = labels[p];
        if (l < 0) continue;
        perm[fill[l]++] = (int32_t)p;
    }
    free(fill);
    return offsets[k];
}

/* ------------------------------------------------------------------------------------------ */
/* Projected L-BFGS in the internal box (App. A.1 affine map; Alg. 1 clamp-to-bound logic)    */
/* ------------------------------------------------------------------------------------------ */
/*
 * Specification (shared with the device optimiser, written independently there):
 *   y = (x - l)/(u - l) in [0,1]^K; g = dF/dx * (u - l).
 *   free_i unless (y_i <= 0 and g_i > 0) or (y_i >= 1 and g_i < 0); Pg = g on the free set.
 *   Direction: two-loop recursion on the free set over the stored pairs (newest first), each
 *   pair restricted to the free set and skipped when s.t <= 1e-12 |s||t| there; H0 = gamma I
 *   with gamma = s.t / t.t of the newest used pair (1 if none).  p = -(H Pg) on the free set;
 *   if p.g >= 0 or p is not finite the memory is cleared and p = -Pg.
 *   Step: alpha0 = 1, or min(1, 1/|p|_inf) when no pair was used.  Trial
 *   y(alpha) = clip(y + alpha p, 0, 1).  The clamp can turn a descent direction into a step that
 *   ascends (a coordinate next to a bound that p drives out of the box carries all of p.g's
 *   descent); a trial with g.(y(a) - y) >= 0 is therefore not evaluated: unless p is already -Pg,
 *   the memory is cleared, p = -Pg (whose clamped steps always descend) and the search restarts at
 *   alpha0 = min(1, 1/|p|_inf) with a fresh backtrack count.  A trial is accepted on Armijo,
 *   F(y(a)) <= F(y) + c1 g.(y(a) - y),
 *   or, where F no longer resolves the decrease, when |F(y(a)) - F(y)| <= 1e-12 |F(y)| and
 *   g(y(a)).(y(a) - y) <= 0 (a step leaving y unchanged is rejected); alpha is halved at most
 *   max_backtracks times, else LS_FAIL.
 *   Accept: s = y_new - y, t = g_new - g, stored when s.t > 1e-12 |s||t| (ring of m pairs).
 *   Stop when |Pg|_2 <= gtol |Pg_0|_2 (CONVERGED) or after max_iter iterations (MAXITER).
 */
typedef struct {
    const orc_problem *pr;
    const double *lo, *hi;
    int K;
    double *xphys, *gphys;
    int64_t nevals;
} orc_obj;

static int orc_eval_internal(orc_obj *o, const double *y, double *f, double *g) {
    for (int i = 0; i < o->K; ++i) o->xphys[i] = o->lo[i] + y[i] * (o->hi[i] - o->lo[i]);
    int st = orc_likelihood_grad(o->pr, o->xphys, f, o->gphys, NULL);
    o->nevals++;
    if (st < 0) return st;
    for (int i = 0; i < o->K; ++i) g[i] = o->gphys[i] * (o->hi[i] - o->lo[i]);
    return st;
}

static double orc_dot_masked(const double *a, const double *b, const unsigned char *m, int n) {
    double s = 0.0;
    for (int i = 0; i < n; ++i)
        if (m[i]) s += a[i] * b[i];
    return s;
}

int orc_lbfgs(const orc_problem *pr, const double *lo, const double *hi, double *x, int32_t m,
              double gtol, int32_t max_iter, int32_t max_backtracks, double c1, double *fout,
              int32_t *iters_out, int64_t *nevals_out) {
    const int K = pr->nclusters[0] + pr->nclusters[1] + pr->nclusters[2];
    if (m < 1 || K < 1) return ORC_E_INVALID;
    for (int i = 0; i < K; ++i)
        if (!(hi[i] > lo[i])) return ORC_E_INVALID;
    double *buf = (double *)calloc((size_t)K * (8 + 2 * (size_t)m) + 2 * (size_t)m + 8, sizeof(double));
    double *y = buf, *g = y + K, *q = g + K, *p = q + K, *yt = p + K, *gt = yt + K, *xp = gt + K,
           *gp = xp + K, *S = gp + K, *T = S + (size_t)m * K, *alph = T + (size_t)m * K,
           *rho = alph + m;
    unsigned char *fr = (unsigned char *)calloc((size_t)K, 1);
    orc_obj o = {pr, lo, hi, K, xp, gp, 0};
    int status = 0, iters = 0, npairs = 0, newest = -1;
    double f, ft;

    for (int i = 0; i < K; ++i) {
        double yi = (x[i] - lo[i]) / (hi[i] - lo[i]);
        y[i] = yi < 0.0 ? 0.0 : (yi > 1.0 ? 1.0 : yi);
    }
    int st = orc_eval_internal(&o, y, &f, g);
    if (st < 0) {
        free(buf);
        free(fr);
        return st;
    }
    status |= st & (ORC_NOT_PD | ORC_NONFINITE);
    double pg0 = 0.0;
    for (int i = 0; i < K; ++i) {
        fr[i] = !((y[i] <= 0.0 && g[i] > 0.0) || (y[i] >= 1.0 && g[i] < 0.0));
        if (fr[i]) pg0 += g[i] * g[i];
    }
    pg0 = sqrt(pg0);
    if (!isfinite(f) || !isfinite(pg0)) status |= ORC_NONFINITE;
    if (pg0 == 0.0 && !(status & ORC_NONFINITE)) status |= ORC_CONVERGED;

    while (!(status & (ORC_CONVERGED | ORC_NONFINITE | ORC_NOT_PD))) {
        if (iters >= max_iter) {
            status |= ORC_MAXITER;
            break;
        }
        /* free set and two-loop recursion restricted to it */
        for (int i = 0; i < K; ++i) {
            fr[i] = !((y[i] <= 0.0 && g[i] > 0.0) || (y[i] >= 1.0 && g[i] < 0.0));
            q[i] = fr[i] ? g[i] : 0.0;
        }
        int used = 0;
        double gamma = 1.0;
        int gamma_set = 0;
        for (int c = 0; c < npairs; ++c) {
            int j = ((newest - c) % m + m) % m;
            const double *sj = S + (size_t)j * K, *tj = T + (size_t)j * K;
            double st_ = orc_dot_masked(sj, tj, fr, K);
            double ss = orc_dot_masked(sj, sj, fr, K), tt = orc_dot_masked(tj, tj, fr, K);
            if (!(st_ > 1e-12 * sqrt(ss) * sqrt(tt)) || tt == 0.0) {
                rho[j] = 0.0;
                continue;
            }
            rho[j] = 1.0 / st_;
            if (!gamma_set) {
                gamma = st_ / tt;
                gamma_set = 1;
            }
            alph[j] = rho[j] * orc_dot_masked(sj, q, fr, K);
            for (int i = 0; i < K; ++i)
                if (fr[i]) q[i] -= alph[j] * tj[i];
            ++used;
        }
        for (int i = 0; i < K; ++i) q[i] *= gamma;
        for (int c = npairs - 1; c >= 0; --c) {
            int j = ((newest - c) % m + m) % m;
            if (rho[j] == 0.0) continue;
            const double *sj = S + (size_t)j * K, *tj = T + (size_t)j * K;
            double be = rho[j] * orc_dot_masked(tj, q, fr, K);
            for (int i = 0; i < K; ++i)
                if (fr[i]) q[i] += sj[i] * (alph[j] - be);
        }
        double pg = 0.0, pinf = 0.0;
        int finite = 1;
        for (int i = 0; i < K; ++i) {
            p[i] = fr[i] ? -q[i] : 0.0;
            pg += p[i] * g[i];
            if (!isfinite(p[i])) finite = 0;
        }
        if (!(pg < 0.0) || !finite) {
            npairs = 0;
            newest = -1;
            used = 0;
            for (int i = 0; i < K; ++i) p[i] = fr[i] ? -g[i] : 0.0;
        }
        for (int i = 0; i < K; ++i)
            if (fabs(p[i]) > pinf) pinf = fabs(p[i]);
        double alpha = used ? 1.0 : (pinf > 1.0 ? 1.0 / pinf : 1.0);
        int steepest = !used; /* p = -Pg */

        /* projected backtracking line search with the Armijo condition */
        int accepted = 0;
        for (int bt = 0; bt <= max_backtracks; ++bt) {
            double dec = 0.0;
            for (int i = 0; i < K; ++i) {
                double v = y[i] + alpha * p[i];
                yt[i] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
                dec += g[i] * (yt[i] - y[i]);
            }
            if (!(dec < 0.0) && !steepest) {
                /* the clamped step does not descend: clear the memory and search along -Pg */
                npairs = 0;
                newest = -1;
                steepest = 1;
                pinf = 0.0;
                for (int i = 0; i < K; ++i) {
                    p[i] = fr[i] ? -g[i] : 0.0;
                    if (fabs(p[i]) > pinf) pinf = fabs(p[i]);
                }
                alpha = pinf > 1.0 ? 1.0 / pinf : 1.0;
                bt = -1;
                continue;
            }
            st = orc_eval_internal(&o, yt, &ft, gt);
            if (st < 0) {
                free(buf);
                free(fr);
                return st;
            }
            if (!(st & ORC_NOT_PD) && isfinite(ft)) {
                /* Armijo, or (at the rounding floor of F) an unchanged F with the function still
                   non-increasing at the trial point along the step */
                double gd = 0.0, moved = 0.0;
                for (int i = 0; i < K; ++i) {
                    gd += gt[i] * (yt[i] - y[i]);
                    moved += (yt[i] - y[i]) * (yt[i] - y[i]);
                }
                /* a step that leaves y unchanged is never accepted */
                if (moved > 0.0 &&
                    (ft <= f + c1 * dec || (fabs(ft - f) <= ORC_FLAT_REL * fabs(f) && gd <= 0.0))) {
                    accepted = 1;
                    break;
                }
            }
            alpha *= 0.5;
        }
        if (!accepted) {
            status |= ORC_LS_FAIL;
            break;
        }
        /* curvature pair */
        double sdt = 0.0, ss = 0.0, tt = 0.0;
        for (int i = 0; i < K; ++i) {
            double si = yt[i] - y[i], ti = gt[i] - g[i];
            sdt += si * ti;
            ss += si * si;
            tt += ti * ti;
        }
        if (sdt > 1e-12 * sqrt(ss) * sqrt(tt)) {
            newest = (newest + 1) % m;
            for (int i = 0; i < K; ++i) {
                S[(size_t)newest * K + i] = yt[i] - y[i];
                T[(size_t)newest * K + i] = gt[i] - g[i];
            }
            if (npairs < m) ++npairs;
        }
        memcpy(y, yt, sizeof(double) * K);
        memcpy(g, gt, sizeof(double) * K);
        f = ft;
        ++iters;
        double pgn = 0.0;
        for (int i = 0; i < K; ++i)
            if (!((y[i] <= 0.0 && g[i] > 0.0) || (y[i] >= 1.0 && g[i] < 0.0))) pgn += g[i] * g[i];
        if (sqrt(pgn) <= gtol * pg0) status |= ORC_CONVERGED;
    }
    for (int i = 0; i < K; ++i) x[i] = lo[i] + y[i] * (hi[i] - lo[i]);
    if (fout) *fout = f;
    if (iters_out) *iters_out = iters;
    if (nevals_out) *nevals_out = o.nevals;
    free(buf);
    free(fr);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* AdaTopK (App. A): AdaBelief directions, Top-K release of bound constraints, dynamic         */
/* rescaling, step limit at the nearest bound, backtracking line search                         */
/* ------------------------------------------------------------------------------------------ */
/*
 * Internal box y = (x - l)/(u - l) (App. A.1); gradients g = dF/dx (u - l).  Pivot p_i = -1 at the
 * lower bound, +1 at the upper bound, 0 free; set at the start for coordinates on a bound.  Each
 * iteration:
 *   1. release: among pinned coordinates whose score p_i g_i is positive (the descent direction
 *      points into the box), the n_rel = max(1, floor(topk n_cand)) largest scores are freed
 *      (ties: lowest index);
 *   2. projected gradient gp = g on the free set; CONVERGED when |gp|_2 <= gtol |gp_first|_2;
 *   3. rescaling: with scale c (initially 1), if |c gp|_2 leaves [1e-15, 1e15] then
 *      c <- c / |c gp|_2 and the moments m, v are multiplied by the factor and its square;
 *   4. AdaBelief on c gp (step count t): m = b1 m + (1-b1) c gp; v = b2 v + (1-b2)(c gp - m)^2
 *      + eps; direction d = -lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps) on the free set;
 *   5. step limit a_max = min over free i with d_i != 0 of the distance to the bound along d
 *      (limiting index: lowest on ties); a_max = 0 pins the limiting coordinate at once;
 *   6. line search from a = min(a_max, a_0), a_0 = min(1, 2 a_prev) with a_prev the last accepted
 *      step (1 at the start and after a reset), halving at most max_backtracks times; the trial is
 *      y + a d clipped into the box, with the limiting coordinate set on its bound when
 *      a = a_max.  Accepted when it moves y and either decreases F (Armijo with c1 when
 *      g.(y_t - y) < 0, strictly otherwise) or leaves F unchanged to 1e-12 relative with
 *      g_t.(y_t - y) <= 0.  A step accepted at a = a_max pins the limiting coordinate;
 *   7. no acceptable trial: with t > 1 the moments are reset (m = v = 0, t = 0) and y stays;
 *      with t = 1 the item stops with LS_FAIL.
 * MAXITER after max_iter iterations (accepted steps, pins and resets each count one).
 */
int orc_adatopk(const orc_problem *pr, const double *lo, const double *hi, double *x, double lr,
                double b1, double b2, double eps, double topk, double gtol, int32_t max_iter,
                int32_t max_backtracks, double c1, double *fout, int32_t *iters_out,
                int64_t *nevals_out) {
    const int K = pr->nclusters[0] + pr->nclusters[1] + pr->nclusters[2];
    if (K < 1 || !(lr > 0.0) || !(b1 >= 0.0 && b1 < 1.0) || !(b2 >= 0.0 && b2 < 1.0) ||
        !(eps >= 0.0) || !(topk >= 0.0 && topk <= 1.0))
        return ORC_E_INVALID;
    for (int i = 0; i < K; ++i)
        if (!(hi[i] > lo[i])) return ORC_E_INVALID;
    double *buf = (double *)calloc((size_t)K * 10, sizeof(double));
    double *y = buf, *g = y + K, *mm = g + K, *vv = mm + K, *d = vv + K, *yt = d + K, *gt = yt + K,
           *xp = gt + K, *gp = xp + K, *sc = gp + K;
    int *piv = (int *)calloc((size_t)K, sizeof(int));
    orc_obj o = {pr, lo, hi, K, xp, gp, 0};
    int status = 0, iters = 0, t = 0, have_pg0 = 0;
    double f, ft, c = 1.0, pg0 = 0.0, b1t = 1.0, b2t = 1.0, aprev = 1.0;

    for (int i = 0; i < K; ++i) {
        double yi = (x[i] - lo[i]) / (hi[i] - lo[i]);
        y[i] = yi < 0.0 ? 0.0 : (yi > 1.0 ? 1.0 : yi);
        piv[i] = y[i] <= 0.0 ? -1 : (y[i] >= 1.0 ? 1 : 0);
    }
    int st = orc_eval_internal(&o, y, &f, g);
    if (st < 0) {
        free(buf);
        free(piv);
        return st;
    }
    status |= st & (ORC_NOT_PD | ORC_NONFINITE);
    if (!isfinite(f)) status |= ORC_NONFINITE;

    while (!(status & (ORC_CONVERGED | ORC_NONFINITE | ORC_NOT_PD | ORC_LS_FAIL))) {
        /* 1. Top-K release */
        int ncand = 0;
        for (int i = 0; i < K; ++i) {
            sc[i] = piv[i] ? piv[i] * g[i] : 0.0;
            if (piv[i] && sc[i] > 0.0) ++ncand;
        }
        if (ncand > 0) {
            int nrel = (int)floor(topk * ncand);
            if (nrel < 1) nrel = 1;
            for (int r = 0; r < nrel; ++r) {
                int best = -1;
                for (int i = 0; i < K; ++i)
                    if (piv[i] && sc[i] > 0.0 && (best < 0 || sc[i] > sc[best])) best = i;
                if (best < 0) break;
                piv[best] = 0;
            }
        }
        /* 2. projected gradient and the stopping test */
        double pg = 0.0;
        for (int i = 0; i < K; ++i)
            if (!piv[i]) pg += g[i] * g[i];
        pg = sqrt(pg);
        if (!have_pg0) {
            pg0 = pg;
            have_pg0 = 1;
        }
        if (pg <= gtol * pg0) {
            status |= ORC_CONVERGED;
            break;
        }
        if (iters >= max_iter) {
            status |= ORC_MAXITER;
            break;
        }
        /* 3. dynamic rescaling of the objective and of the moments */
        double cpg = c * pg;
        if (cpg < 1e-15 || cpg > 1e15) {
            double fs = 1.0 / cpg;
            c *= fs;
            for (int i = 0; i < K; ++i) {
                mm[i] *= fs;
                vv[i] *= fs * fs;
            }
        }
        /* 4. AdaBelief direction */
        ++t;
        b1t *= b1;
        b2t *= b2;
        for (int i = 0; i < K; ++i) {
            double gi = piv[i] ? 0.0 : c * g[i];
            mm[i] = b1 * mm[i] + (1.0 - b1) * gi;
            double dv = gi - mm[i];
            vv[i] = b2 * vv[i] + (1.0 - b2) * dv * dv + eps;
            double mh = mm[i] / (1.0 - b1t), vh = vv[i] / (1.0 - b2t);
            d[i] = piv[i] ? 0.0 : -lr * mh / (sqrt(vh) + eps);
        }
        /* 5. distance to the nearest bound along d */
        double amax = INFINITY;
        int lim = -1;
        for (int i = 0; i < K; ++i) {
            if (piv[i] || d[i] == 0.0) continue;
            double a = d[i] > 0.0 ? (1.0 - y[i]) / d[i] : -y[i] / d[i];
            if (a < amax) {
                amax = a;
                lim = i;
            }
        }
        if (lim >= 0 && amax <= 0.0) {
            piv[lim] = d[lim] > 0.0 ? 1 : -1;
            y[lim] = d[lim] > 0.0 ? 1.0 : 0.0;
            ++iters;
            continue;
        }
        /* 6. backtracking line search */
        const double a0 = 2.0 * aprev < 1.0 ? 2.0 * aprev : 1.0;
        double alpha = amax < a0 ? amax : a0;
        int accepted = 0, at_bound = 0;
        for (int bt = 0; bt <= max_backtracks; ++bt) {
            const int hit = (lim >= 0 && alpha == amax);
            double dec = 0.0, moved = 0.0;
            for (int i = 0; i < K; ++i) {
                double v = y[i] + alpha * d[i];
                yt[i] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
            }
            if (hit) yt[lim] = d[lim] > 0.0 ? 1.0 : 0.0;
            for (int i = 0; i < K; ++i) {
                dec += g[i] * (yt[i] - y[i]);
                moved += (yt[i] - y[i]) * (yt[i] - y[i]);
            }
            st = orc_eval_internal(&o, yt, &ft, gt);
            if (st < 0) {
                free(buf);
                free(piv);
                return st;
            }
            if (!(st & ORC_NOT_PD) && isfinite(ft) && moved > 0.0) {
                double gd = 0.0;
                for (int i = 0; i < K; ++i) gd += gt[i] * (yt[i] - y[i]);
                int ok = dec < 0.0 ? (ft <= f + c1 * dec) : (ft < f);
                if (ok || (fabs(ft - f) <= ORC_FLAT_REL * fabs(f) && gd <= 0.0)) {
                    accepted = 1;
                    at_bound = hit;
                    break;
                }
            }
            alpha *= 0.5;
        }
        if (!accepted) {
            if (t <= 1) {
                status |= ORC_LS_FAIL;
                break;
            }
            memset(mm, 0, sizeof(double) * K);
            memset(vv, 0, sizeof(double) * K);
            t = 0;
            b1t = b2t = 1.0;
            aprev = 1.0;
            ++iters;
            continue;
        }
        aprev = alpha;
        if (at_bound) piv[lim] = d[lim] > 0.0 ? 1 : -1;
        memcpy(y, yt, sizeof(double) * K);
        memcpy(g, gt, sizeof(double) * K);
        f = ft;
        ++iters;
    }
    for (int i = 0; i < K; ++i) x[i] = lo[i] + y[i] * (hi[i] - lo[i]);
    if (fout) *fout = f;
    if (iters_out) *iters_out = iters;
    if (nevals_out) *nevals_out = o.nevals;
    free(buf);
    free(piv);
    return status;
}

/* ------------------------------------------------------------------------------------------ */
/* Spherical K-means (Sec. 2.2): Lloyd iterations on unit vectors with angular distance        */
/* ------------------------------------------------------------------------------------------ */
/*
 * vecs[n][3]: unit vectors in ascending pixel order; init[k]: distinct indices into vecs (the
 * random draw of the initial centroids is an input).  The nearest centroid in angular separation
 * is the one of largest dot product; the dot product is (x cx + y cy) + z cz with every product
 * and sum rounded separately, and a tie goes to the lowest centroid index.  Each of the iters
 * iterations assigns every vector, then replaces each centroid by the sum of its members (in
 * ascending index order) divided by its Euclidean norm; a cluster without members (or with a
 * zero sum) keeps its centroid.  The labels come from one more assignment and are compacted to
 * 0..K_eff-1 in ascending centroid index.  With k >= n every vector is its own cluster (the
 * patch-count cap).  labels[n] out; returns K_eff, or ORC_E_INVALID.
 */
static double orc_dot3(const double *a, const double *c) {
    double xy = a[0] * c[0] + a[1] * c[1];
    return xy + a[2] * c[2];
}

static void orc_km_assign(int64_t n, const double *v, int32_t k, const double *c, int32_t *lab) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t best = 0;
        double bd = orc_dot3(v + 3 * i, c);
        for (int32_t j = 1; j < k; ++j) {
            double dj = orc_dot3(v + 3 * i, c + 3 * j);
            if (dj > bd) {
                bd = dj;
                best = j;
            }
        }
        lab[i] = best;
    }
}

int32_t orc_kmeans(int64_t n, const double *vecs, int32_t k, const int32_t *init, int32_t iters,
                   int32_t *labels) {
    if (n < 0 || k < 1 || iters < 0) return ORC_E_INVALID;
    if ((int64_t)k >= n) {
        for (int64_t i = 0; i < n; ++i) labels[i] = (int32_t)i;
        return (int32_t)n;
    }
    double *c = (double *)malloc(sizeof(double) * 3 * (size_t)k);
    double *sum = (double *)malloc(sizeof(double) * 3 * (size_t)k);
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)k);
    int32_t *remap = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    for (int32_t j = 0; j < k; ++j) {
        if (init[j] < 0 || init[j] >= n) {
            free(c); free(sum); free(cnt); free(remap);
            return ORC_E_INVALID;
        }
        memcpy(c + 3 * j, vecs + 3 * (int64_t)init[j], sizeof(double) * 3);
    }
    for (int32_t it = 0; it < iters; ++it) {
        orc_km_assign(n, vecs, k, c, labels);
        memset(sum, 0, sizeof(double) * 3 * (size_t)k);
        memset(cnt, 0, sizeof(int64_t) * (size_t)k);
        for (int64_t i = 0; i < n; ++i) {
            double *sj = sum + 3 * labels[i];
            for (int d = 0; d < 3; ++d) sj[d] += vecs[3 * i + d];
            cnt[labels[i]] += 1;
        }
        for (int32_t j = 0; j < k; ++j) {
            const double *sj = sum + 3 * j;
            double nrm = sqrt((sj[0] * sj[0] + sj[1] * sj[1]) + sj[2] * sj[2]);
            if (cnt[j] > 0 && nrm > 0.0)
                for (int d = 0; d < 3; ++d) c[3 * j + d] = sj[d] / nrm;
        }
    }
    orc_km_assign(n, vecs, k, c, labels);
    for (int32_t j = 0; j < k; ++j) remap[j] = 0;
    for (int64_t i = 0; i < n; ++i) remap[labels[i]] = 1;
    int32_t keff = 0;
    for (int32_t j = 0; j < k; ++j) remap[j] = remap[j] ? keff++ : -1;
    for (int64_t i = 0; i < n; ++i) labels[i] = remap[labels[i]];
    free(c); free(sum); free(cnt); free(remap);
    return keff;
}
