"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (CPU only).

Every check here compares the oracle with something that is not the oracle: 50-digit mpmath
evaluations of the physical definitions, closed forms of small systems, a textbook least-squares
routine, complex-step derivatives of an independent complex implementation, invariants of the
spectral likelihood, brute force on tiny inputs and SciPy's L-BFGS-B.
"""

import math

import mpmath as mp
import numpy as np
import pytest
import scipy.optimize

import skygen
from oracle import oracle as O

mp.mp.dps = 50
H = mp.mpf("6.62607015e-34")
KB = mp.mpf("1.380649e-23")
CL = mp.mpf(299792458)
TCMB = mp.mpf("2.7255")
GHZ = mp.mpf(10) ** 9


# --------------------------------------------------------------------------------------------
# 50-digit physical definitions (intensity route, independent of the oracle's expm1 algebra)
# --------------------------------------------------------------------------------------------

def mp_planck(nu_ghz, temp):
    nu = mp.mpf(nu_ghz) * GHZ
    return 2 * H * nu ** 3 / CL ** 2 / (mp.exp(H * nu / (KB * temp)) - 1)


def mp_dbdt_cmb(nu_ghz):
    return mp.diff(lambda t: mp_planck(nu_ghz, t), TCMB)


def mp_dust(nu, beta, temp, nu0=353.0):
    num = (mp.mpf(nu) / nu0) ** beta * mp_planck(nu, temp) / mp_dbdt_cmb(nu)
    return num / (mp_planck(nu0, temp) / mp_dbdt_cmb(nu0))


def mp_sync(nu, beta, nu0=23.0):
    def rj(n):
        n = mp.mpf(n) * GHZ
        return 2 * KB * n ** 2 / CL ** 2

    return (mp.mpf(nu) / nu0) ** beta * rj(nu) / mp_dbdt_cmb(nu) / (rj(nu0) / mp_dbdt_cmb(nu0))


def one_pixel(freqs, d, w, x, nu0d=353.0, nu0s=23.0):
    """Oracle problem holding a single pixel with one cluster per parameter."""
    F = len(freqs)
    dd = np.asarray(d, dtype=np.float64).reshape(2, F, 1)
    ww = np.asarray(w, dtype=np.float64).reshape(2, F)
    lab = np.zeros((3, 1), dtype=np.int32)
    return O.Problem(np.asarray(freqs, dtype=np.float64), dd, ww, lab, (1, 1, 1), nu0d, nu0s)


# --------------------------------------------------------------------------------------------
# mixing-matrix columns
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("nu", [23.0, 40.0, 100.0, 353.0, 402.0, 448.0])
@pytest.mark.parametrize("beta_d,temp_d,beta_s", [(1.54, 20.0, -3.0), (0.5, 5.0, -5.0), (3.0, 50.0, -1.0)])
def test_sed_matches_planck_definition(nu, beta_d, temp_d, beta_s):
    ad, as_, dbd, dtd, dbs = O.sed(nu, beta_d, temp_d, beta_s)
    ref_d = mp_dust(nu, beta_d, temp_d)
    ref_s = mp_sync(nu, beta_s)
    assert abs(ad - float(ref_d)) <= 1e-13 * abs(float(ref_d))
    assert abs(as_ - float(ref_s)) <= 1e-13 * abs(float(ref_s))
    # parameter derivatives against 50-digit numerical differentiation of the definitions
    r_dbd = mp.diff(lambda b: mp_dust(nu, b, temp_d), beta_d)
    r_dtd = mp.diff(lambda t: mp_dust(nu, beta_d, t), temp_d)
    r_dbs = mp.diff(lambda b: mp_sync(nu, b), beta_s)
    for got, ref in ((dbd, r_dbd), (dtd, r_dtd), (dbs, r_dbs)):
        ref = float(ref)
        assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300) + 1e-300


def test_sed_normalised_at_reference():
    ad, as_, _, _, _ = O.sed(353.0, 1.7, 17.0, -2.8)
    assert abs(ad - 1.0) < 1e-15
    _, as0, _, _, _ = O.sed(23.0, 1.7, 17.0, -2.8)
    assert abs(as0 - 1.0) < 1e-15


@pytest.mark.parametrize("nu", [23.0, 40.0, 353.0, 402.0])
def test_rj_to_cmb_factor_is_planck_derivative(nu):
    # g(nu) converts RJ temperature to CMB temperature: (2 k nu^2 / c^2) / (dB/dT at T_CMB)
    n = mp.mpf(nu) * GHZ
    ref = 2 * KB * n ** 2 / CL ** 2 / mp_dbdt_cmb(nu)
    assert abs(O.rj_to_cmb(nu) - float(ref)) <= 1e-14 * float(ref)


# --------------------------------------------------------------------------------------------
# one-pixel closed forms
# --------------------------------------------------------------------------------------------

def _pixel_draw(seed, F):
    g = np.random.default_rng(seed)
    freqs = np.sort(g.uniform(30.0, 420.0, F))
    w = np.tile(1.0 / g.uniform(2.0, 20.0, F) ** 2, (2, 1))
    d = g.normal(0.0, 30.0, (2, F))
    x = np.array([g.uniform(1.2, 1.9), g.uniform(12.0, 30.0), g.uniform(-3.4, -2.6)])
    return freqs, d, w, x


@pytest.mark.parametrize("seed", range(4))
def test_three_bands_square_system(seed):
    # A is square: the GLS fit is exact, F = -d^T W d and the gradient vanishes for every beta
    freqs, d, w, x = _pixel_draw(seed, 3)
    pr = one_pixel(freqs, d, w, x)
    f, g, _, st = pr.likelihood_grad(x)
    ref = -float(np.sum(w * d * d))
    assert st == 0
    assert abs(f - ref) <= 1e-11 * abs(ref)
    scale = np.abs(d).max() ** 2 * w.max() * 10
    assert np.all(np.abs(g) <= 1e-9 * scale)


@pytest.mark.parametrize("seed", range(4))
def test_four_bands_cross_product_form(seed):
    # F = -d^T W d + (u.d)^2 / (u^T W^-1 u), u = generalised cross product of A's columns
    freqs, d, w, x = _pixel_draw(seed, 4)
    pr = one_pixel(freqs, d, w, x)
    f, _, _, _ = pr.likelihood_grad(x)
    A = mp.matrix(4, 3)
    for i, nu in enumerate(freqs):
        A[i, 0] = 1
        A[i, 1] = mp_dust(nu, x[0], x[1])
        A[i, 2] = mp_sync(nu, x[2])
    u = [(-1) ** i * mp.det(mp.matrix([[A[r, c] for c in range(3)] for r in range(4) if r != i])) for i in range(4)]
    ref = mp.mpf(0)
    for s in range(2):
        dw = sum(mp.mpf(w[s, i]) * mp.mpf(d[s, i]) ** 2 for i in range(4))
        ud = sum(u[i] * mp.mpf(d[s, i]) for i in range(4))
        uwu = sum(u[i] ** 2 / mp.mpf(w[s, i]) for i in range(4))
        ref += -dw + ud ** 2 / uwu
    assert abs(f - float(ref)) <= 1e-12 * abs(float(ref))


@pytest.mark.parametrize("F", [5, 15, 22])
def test_adjugate_form_50_digits(F):
    freqs, d, w, x = _pixel_draw(F, F)
    pr = one_pixel(freqs, d, w, x)
    f, _, _, _ = pr.likelihood_grad(x)
    ref = mp.mpf(0)
    for s in range(2):
        M = mp.matrix(3, 3)
        b = mp.matrix(3, 1)
        for i, nu in enumerate(freqs):
            a = [mp.mpf(1), mp_dust(nu, x[0], x[1]), mp_sync(nu, x[2])]
            for r in range(3):
                b[r] += mp.mpf(w[s, i]) * a[r] * mp.mpf(d[s, i])
                for c in range(3):
                    M[r, c] += mp.mpf(w[s, i]) * a[r] * a[c]
        adj = mp.matrix(3, 3)
        for r in range(3):
            for c in range(3):
                minor = mp.matrix([[M[i, j] for j in range(3) if j != r] for i in range(3) if i != c])
                adj[r, c] = (-1) ** (r + c) * mp.det(minor)
        ref -= (b.T * adj * b)[0, 0] / mp.det(M)
    assert abs(f - float(ref)) <= 1e-11 * abs(float(ref))


# --------------------------------------------------------------------------------------------
# textbook least squares and the chi^2 identity
# --------------------------------------------------------------------------------------------

def test_matches_lstsq_reduction():
    sky = skygen.make_tiny(40, 15, (2, 2, 2), seed=3)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    f, _, _, _ = pr.likelihood_grad(x)
    lab = sky.item_labels(0)
    d = sky.item_d(0)
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1]]
    ref = 0.0
    for p in range(sky.npix):
        bd, td, bs = x[off[0] + lab[0, p]], x[off[1] + lab[1, p]], x[off[2] + lab[2, p]]
        A = np.stack([np.ones(sky.nfreq), skygen.sky_sed_dust(sky.freqs, bd, td), skygen.sky_sed_sync(sky.freqs, bs)], 1)
        for s in range(2):
            sw = np.sqrt(sky.ninv[s])
            sol = np.linalg.lstsq(sw[:, None] * A, sw * d[s, :, p], rcond=None)[0]
            res = sw * (d[s, :, p] - A @ sol)
            ref -= np.sum((sw * d[s, :, p]) ** 2) - np.sum(res ** 2)
    assert abs(f - ref) <= 1e-10 * abs(ref)


def test_chi2_nonnegative_and_invariant_under_model_signal():
    sky = skygen.make_tiny(30, 15, (2, 1, 2), seed=4)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    f, _, _, _ = pr.likelihood_grad(x)
    chi2 = pr.data_chi2() + f
    assert chi2 >= 0.0
    # add a sky built with the model's own SEDs at x: chi^2 at x is unchanged
    lab = sky.item_labels(0)
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1]]
    g = np.random.default_rng(9)
    d2 = sky.item_d(0).copy()
    for p in range(sky.npix):
        bd, td, bs = x[off[0] + lab[0, p]], x[off[1] + lab[1, p]], x[off[2] + lab[2, p]]
        A = np.stack([np.ones(sky.nfreq), skygen.sky_sed_dust(sky.freqs, bd, td), skygen.sky_sed_sync(sky.freqs, bs)], 1)
        for s in range(2):
            d2[s, :, p] += A @ g.normal(0, 50.0, 3)
    pr2 = O.Problem.from_sky(sky, d=d2)
    f2, _, _, _ = pr2.likelihood_grad(x)
    chi2b = pr2.data_chi2() + f2
    assert abs(chi2b - chi2) <= 1e-9 * pr2.data_chi2()


# --------------------------------------------------------------------------------------------
# gradient: complex step of an independent complex implementation, and central differences
# --------------------------------------------------------------------------------------------

_HK = 6.62607015e-34 / 1.380649e-23 * 1e9


def _complex_F(sky, item, x):
    """F(x) for complex x through the intensity route; analytic in x (no conjugation)."""
    lab = sky.item_labels(item)
    d = sky.item_d(item)
    K = sky.nclusters[item]
    off = [0, K[0], K[0] + K[1]]
    nu = sky.freqs[:, None]
    bd = x[off[0] + lab[0]][None]
    td = x[off[1] + lab[1]][None]
    bs = x[off[2] + lab[2]][None]

    def planck(n, t):
        return n ** 3 / (np.exp(_HK * n / t) - 1.0)

    def dbdt(n):
        y = _HK * n / 2.7255
        return n ** 4 * np.exp(y) / (np.exp(y) - 1.0) ** 2

    ad = np.exp(bd * np.log(nu / 353.0)) * planck(nu, td) / dbdt(nu) / (planck(353.0, td) / dbdt(353.0))
    as_ = np.exp(bs * np.log(nu / 23.0)) * nu ** 2 / dbdt(nu) / (23.0 ** 2 / dbdt(23.0))
    A = np.stack([np.ones_like(ad), ad, as_], axis=-1).transpose(1, 0, 2)  # [P, F, 3]
    tot = 0.0
    for s in range(2):
        w = sky.ninv[s][None, :, None]
        M = np.einsum("pfi,pfj->pij", A * w, A)
        b = np.einsum("pfi,pf->pi", A * w, d[s].T)
        sol = np.linalg.solve(M, b[..., None])[..., 0]
        tot = tot - np.sum(b * sol)
    return tot


@pytest.mark.parametrize("k", [(1, 1, 1), (3, 2, 4)])
def test_gradient_matches_complex_step(k):
    sky = skygen.make_tiny(48, 15, k, seed=5)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    _, g, _, _ = pr.likelihood_grad(x)
    h = 1e-30
    cs = np.array([_complex_F(sky, 0, x + 1j * h * np.eye(x.size)[i]).imag / h for i in range(x.size)])
    assert np.max(np.abs(g - cs)) <= 1e-9 * np.max(np.abs(cs))


def test_gradient_central_differences():
    sky = skygen.make_tiny(64, 15, (3, 2, 2), seed=1)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    _, g, _, _ = pr.likelihood_grad(x)
    h = 1e-6
    for i in range(x.size):
        e = np.zeros_like(x)
        e[i] = h
        fd = (pr.likelihood_grad(x + e)[0] - pr.likelihood_grad(x - e)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-5 * max(abs(g[i]), 1e-2 * np.max(np.abs(g)))


def test_gradient_abs_scale_of_clusters():
    # the per-cluster scale sum_p |dF_p/dtheta| of the condition-aware gradient tolerance: it is
    # the sum of the per-pixel gradients' magnitudes (per-pixel gradients summed, signed, give the
    # complex-step-pinned gradient), bounds |grad| from above, and equals it for one-pixel clusters
    sky = skygen.make_tiny(40, 15, (3, 2, 40), seed=8)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    _, g, _, _ = pr.likelihood_grad(x)
    ga = pr.grad_abs(x)
    lab = sky.item_labels(0)
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1]]
    brute = np.zeros_like(ga)
    signed = np.zeros_like(ga)
    for p in range(sky.npix):
        gp = pr.pixel(x, p)["g"]
        for j in range(3):
            brute[off[j] + lab[j, p]] += abs(gp[j])
            signed[off[j] + lab[j, p]] += gp[j]
    assert np.allclose(signed, g, rtol=1e-12, atol=0)
    assert np.allclose(ga, brute, rtol=1e-14, atol=0)
    assert np.all(np.abs(g) <= ga * (1 + 1e-14))
    single = off[2] + np.arange(K[2])  # 40 beta_s clusters of one pixel each
    assert np.array_equal(np.bincount(lab[2], minlength=K[2]), np.ones(K[2], dtype=int))
    assert np.allclose(ga[single], np.abs(g[single]), rtol=1e-15, atol=0)


def test_gradient_term_magnitudes():
    # the FP32 tolerance scale: every signed term of a cluster's gradient enumerated one by one
    # (pixel, Stokes, band; the data term and the three model terms of the expanded residual).
    # Their signed sum must give the complex-step-pinned gradient -- so the enumeration is
    # complete -- and the sum of their magnitudes is gterm; it bounds gabs and |grad| from above
    sky = skygen.make_tiny(6, 5, (2, 2, 3), seed=12)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    _, g, _, _ = pr.likelihood_grad(x)
    gt = pr.grad_terms(x)
    ga = pr.grad_abs(x)
    lab = sky.item_labels(0)
    d = sky.item_d(0)
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1]]
    signed = np.zeros_like(g)
    mags = np.zeros_like(g)
    for p in range(sky.npix):
        bd, td, bs = x[lab[0, p]], x[off[1] + lab[1, p]], x[off[2] + lab[2, p]]
        sh = pr.pixel(x, p)["s"]
        for n, nu in enumerate(sky.freqs):
            ad, as_, dbd, dtd, dbs = O.sed(nu, bd, td, bs)
            a = (1.0, ad, as_)
            for s in range(2):
                w = sky.ninv[s, n]
                for j, (der, col) in enumerate(((dbd, 1), (dtd, 1), (dbs, 2))):
                    k = off[j] + lab[j, p]
                    terms = [-2.0 * w * der * sh[s, col] * d[s, n, p]]
                    terms += [2.0 * w * der * sh[s, col] * a[i] * sh[s, i] for i in range(3)]
                    signed[k] += sum(terms)
                    mags[k] += sum(abs(t) for t in terms)
    assert np.allclose(signed, g, rtol=1e-10, atol=1e-12 * np.max(np.abs(g)))
    assert np.allclose(gt, mags, rtol=1e-13, atol=0)
    assert np.all(gt >= ga * (1 - 1e-14)) and np.all(ga >= np.abs(g) * (1 - 1e-14))


# --------------------------------------------------------------------------------------------
# invariants of the spectral likelihood
# --------------------------------------------------------------------------------------------

def test_reference_frequency_invariance():
    # b^T M^-1 b depends only on span(A): rescaling a column (nu0, g(nu0)) changes nothing
    sky = skygen.make_tiny(40, 15, (2, 3, 2), seed=6)
    x = sky.x[0]
    f1, g1, _, _ = O.Problem.from_sky(sky).likelihood_grad(x)
    pr2 = O.Problem(sky.freqs, sky.item_d(0), sky.ninv, sky.item_labels(0), sky.nclusters[0], 217.0, 30.0)
    f2, g2, _, _ = pr2.likelihood_grad(x)
    assert abs(f1 - f2) <= 1e-12 * abs(f1)
    assert np.max(np.abs(g1 - g2)) <= 1e-10 * np.max(np.abs(g1))


def test_pixel_normal_equations_symmetry_and_cmb_response():
    sky = skygen.make_tiny(12, 15, (1, 1, 1), seed=7)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    d = sky.item_d(0)
    for p in range(sky.npix):
        det = pr.pixel(x, p)
        for s in range(2):
            M = det["M"][s]
            assert np.array_equal(M, M.T)
            assert np.all(np.linalg.eigvalsh(M) > 0)
            A = np.stack([np.ones(sky.nfreq), *[np.array([O.sed(nu, x[0], x[1], x[2])[j] for nu in sky.freqs]) for j in (0, 1)]], 1)
            atr = A.T @ det["r"][s]
            scale = np.abs(A).T @ np.abs(sky.ninv[s] * d[s, :, p])
            assert np.all(np.abs(atr) <= 1e-12 * scale)
    # CMB unit response: adding c to every band shifts s_cmb by c and leaves the others
    d2 = d.copy() + 3.25
    pr2 = O.Problem.from_sky(sky, d=d2)
    for p in range(sky.npix):
        s1 = pr.pixel(x, p)["s"]
        s2 = pr2.pixel(x, p)["s"]
        assert np.allclose(s2[:, 0] - s1[:, 0], 3.25, rtol=0, atol=1e-9)
        assert np.allclose(s2[:, 1:], s1[:, 1:], rtol=0, atol=1e-9 * np.abs(s1).max())


def test_pixel_permutation_invariance():
    sky = skygen.make_tiny(50, 15, (4, 2, 3), seed=8)
    x = sky.x[0]
    f1, g1, c1, _ = O.Problem.from_sky(sky).likelihood_grad(x)
    perm = np.random.default_rng(1).permutation(sky.npix)
    pr2 = O.Problem(sky.freqs, sky.item_d(0)[:, :, perm], sky.ninv, sky.item_labels(0)[:, perm], sky.nclusters[0])
    f2, g2, c2, _ = pr2.likelihood_grad(x)
    assert abs(f1 - f2) <= 1e-14 * abs(f1)
    assert np.max(np.abs(g1 - g2)) <= 1e-13 * np.max(np.abs(g1))


def test_cluster_partials_sum_and_empty_clusters():
    sky = skygen.make_tiny(60, 15, (5, 3, 4), seed=9)
    lab = sky.item_labels(0).copy()
    lab[0][lab[0] == 4] = 3  # beta_d cluster 4 becomes empty
    pr = O.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, sky.nclusters[0])
    f, g, cf, st = pr.likelihood_grad(sky.x[0])
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1], K.sum()]
    for j in range(3):
        assert abs(cf[off[j]:off[j + 1]].sum() - f) <= 1e-13 * abs(f)
    assert g[4] == 0.0 and cf[4] == 0.0


def test_model_consistent_noiseless_optimum():
    sky = skygen.make_tiny(40, 15, (3, 2, 2), seed=10, noiseless=True, model_consistent=True)
    pr = O.Problem.from_sky(sky)
    xt = sky.meta["x_true"]
    f, g, _, _ = pr.likelihood_grad(xt)
    assert abs(f + pr.data_chi2()) <= 1e-12 * pr.data_chi2()
    # gradient scale: the gradient at a perturbed point
    _, gp, _, _ = pr.likelihood_grad(xt + 0.05)
    assert np.max(np.abs(g)) <= 1e-10 * np.max(np.abs(gp))


# --------------------------------------------------------------------------------------------
# labels and segments
# --------------------------------------------------------------------------------------------

def test_segments_bit_exact_against_brute_force():
    g = np.random.default_rng(11)
    for k in (1, 3, 17):
        lab = g.integers(-1, k, 200).astype(np.int32)
        perm, off = O.segments(lab, k)
        ref_perm = [p for c in range(k) for p in range(lab.size) if lab[p] == c]
        ref_off = [0]
        for c in range(k):
            ref_off.append(ref_off[-1] + int(np.sum(lab == c)))
        assert perm.tolist() == ref_perm
        assert off.tolist() == ref_off


def test_label_errors():
    sky = skygen.make_tiny(10, 15, (2, 2, 2), seed=12)
    lab = sky.item_labels(0).copy()
    lab[1, 3] = 2  # out of range
    assert O.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, (2, 2, 2)).check_labels() == O.E_LABEL
    lab = sky.item_labels(0).copy()
    lab[0, 5] = -1  # excluded for one parameter only
    assert O.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, (2, 2, 2)).check_labels() == O.E_LABEL
    lab = sky.item_labels(0).copy()
    lab[:, 5] = -1  # excluded pixel
    assert O.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, (2, 2, 2)).check_labels() == 0


def test_not_pd_when_weights_vanish():
    sky = skygen.make_tiny(6, 15, (1, 1, 1), seed=13)
    w = np.zeros((2, 15, 6))
    w[:, :, :] = sky.ninv[:, :, None]
    w[:, :, 2] = 0.0  # pixel 2 carries no information: M = 0
    pr = O.Problem(sky.freqs, sky.item_d(0), w, sky.item_labels(0), (1, 1, 1))
    f, _, _, st = pr.likelihood_grad(sky.x[0])
    assert st & O.NOT_PD and math.isnan(f)


def test_excluded_pixels_do_not_contribute():
    sky = skygen.make_tiny(30, 15, (2, 2, 2), seed=14, mask_frac=0.3)
    lab = sky.item_labels(0)
    keep = lab[0] >= 0
    f1, g1, _, _ = O.Problem.from_sky(sky).likelihood_grad(sky.x[0])
    pr2 = O.Problem(sky.freqs, sky.item_d(0)[:, :, keep], sky.ninv, lab[:, keep], sky.nclusters[0])
    f2, g2, _, _ = pr2.likelihood_grad(sky.x[0])
    assert f1 == f2 and np.array_equal(g1, g2)


# --------------------------------------------------------------------------------------------
# projected L-BFGS
# --------------------------------------------------------------------------------------------

def _grid_min(pr, lo, hi, n):
    axes = [np.linspace(lo[i], hi[i], n) for i in range(3)]
    best = (np.inf, None)
    for a in axes[0]:
        for b in axes[1]:
            for c in axes[2]:
                x = np.array([a, b, c])
                f = pr.likelihood_grad(x)[0]
                if f < best[0]:
                    best = (f, x)
    return best, [ax[1] - ax[0] for ax in axes]


def test_lbfgs_beats_brute_force_grid():
    sky = skygen.make_tiny(16, 15, (1, 1, 1), seed=15, model_consistent=True)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0], sky.upper[0]
    (fg, xg), cell = _grid_min(pr, lo, hi, 41)
    x, f, it, ne, st = pr.lbfgs(np.array(skygen.X0), lo, hi)
    assert st & O.CONVERGED
    assert f <= fg + 1e-12 * abs(fg)
    assert np.all(np.abs(x - xg) <= np.array(cell) * 1.0 + 1e-12)


def test_lbfgs_two_dust_clusters_matches_scipy():
    sky = skygen.make_tiny(16, 15, (2, 1, 1), seed=16, model_consistent=True)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0], sky.upper[0]
    x0 = np.array([1.54, 1.54, 20.0, -3.0])
    x, f, it, ne, st = pr.lbfgs(x0, lo, hi)
    assert st & O.CONVERGED
    res = scipy.optimize.minimize(lambda z: pr.likelihood_grad(z)[0], x0, jac=lambda z: pr.likelihood_grad(z)[1],
                                  method="L-BFGS-B", bounds=list(zip(lo, hi)),
                                  options=dict(ftol=1e-16, gtol=1e-12, maxiter=5000))
    assert f <= res.fun + 1e-12 * abs(res.fun)
    assert np.all(np.abs(x - res.x) <= 1e-4 * np.maximum(1.0, np.abs(res.x)))


def test_lbfgs_kkt_at_result():
    sky = skygen.make_tiny(64, 15, (3, 2, 2), seed=17)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0], sky.upper[0]
    x0 = np.concatenate([np.full(3, 1.54), np.full(2, 20.0), np.full(2, -3.0)])
    x, f, it, ne, st = pr.lbfgs(x0, lo, hi)
    _, g0, _, _ = pr.likelihood_grad(x0)
    _, g, _, _ = pr.likelihood_grad(x)
    gi = g * (hi - lo)
    y = (x - lo) / (hi - lo)
    free = ~(((y <= 0) & (gi > 0)) | ((y >= 1) & (gi < 0)))
    y0 = (x0 - lo) / (hi - lo)
    g0i = g0 * (hi - lo)
    free0 = ~(((y0 <= 0) & (g0i > 0)) | ((y0 >= 1) & (g0i < 0)))
    assert st & O.CONVERGED
    assert np.linalg.norm(gi[free]) <= 1e-8 * np.linalg.norm(g0i[free0])
    assert np.all((x >= lo) & (x <= hi))


def test_oracle_regression_fixture():
    # values written by tests/golden/make_golden.py (oracle only); guards against silent changes
    import json
    import os
    fx = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_workload1.json")))
    sky = skygen.make_config(1)
    pr = O.Problem.from_sky(sky, 0)
    for pt in fx["points"]:
        f, g, _, st = pr.likelihood_grad(np.array(pt["x"]))
        assert abs(f - pt["neg2logL"]) <= 1e-13 * abs(pt["neg2logL"])
        assert np.allclose(g, pt["grad"], rtol=1e-11, atol=1e-11 * np.max(np.abs(pt["grad"])))


def test_component_maps_match_lstsq_and_numpy_variance():
    # s_hat = W d (Sec. 2.3 eq. recon_operator) against numpy lstsq on the intensity-route A;
    # sigma^2_CMB (Sec. 2.4 eq. min_var) against numpy's population variance, Q plus U
    sky = skygen.make_tiny(60, 15, (3, 2, 2), seed=18, mask_frac=0.2)
    pr = O.Problem.from_sky(sky)
    x = sky.x[0]
    s, var, st = pr.component_maps(x)
    lab = sky.item_labels(0)
    d = sky.item_d(0)
    K = sky.nclusters[0]
    off = [0, K[0], K[0] + K[1]]
    cmb = [[], []]
    for p in range(sky.npix):
        if lab[0, p] < 0:
            assert np.all(np.isnan(s[:, :, p]))
            continue
        bd, td, bs = x[off[0] + lab[0, p]], x[off[1] + lab[1, p]], x[off[2] + lab[2, p]]
        A = np.stack([np.ones(sky.nfreq), skygen.sky_sed_dust(sky.freqs, bd, td), skygen.sky_sed_sync(sky.freqs, bs)], 1)
        for q in range(2):
            sw = np.sqrt(sky.ninv[q])
            sol = np.linalg.lstsq(sw[:, None] * A, sw * d[q, :, p], rcond=None)[0]
            assert np.allclose(s[q, :, p], sol, rtol=1e-9, atol=1e-9 * np.max(np.abs(sol)))
            cmb[q].append(sol[0])
    ref = np.var(cmb[0]) + np.var(cmb[1])
    assert abs(var - ref) <= 1e-10 * ref


def test_component_maps_nan_rules():
    # a pixel without information (zero weights) has no amplitudes; the variance is then undefined
    sky = skygen.make_tiny(6, 15, (1, 1, 1), seed=13)
    w = np.repeat(sky.ninv[:, :, None], 6, axis=2)
    w[:, :, 2] = 0.0
    s, var, st = O.Problem(sky.freqs, sky.item_d(0), w, sky.item_labels(0), (1, 1, 1)).component_maps(sky.x[0])
    assert st & O.NOT_PD and math.isnan(var)
    assert np.all(np.isnan(s[:, :, 2])) and np.all(np.isfinite(np.delete(s, 2, axis=2)))
    lab = np.full((3, 6), -1, dtype=np.int32)  # nothing included
    s, var, st = O.Problem(sky.freqs, sky.item_d(0), sky.ninv, lab, (1, 1, 1)).component_maps(sky.x[0])
    assert st == 0 and math.isnan(var) and np.all(np.isnan(s))


# --------------------------------------------------------------------------------------------
# spherical K-means (Sec. 2.2)
# --------------------------------------------------------------------------------------------

def _partition(lab):
    return sorted(tuple(np.flatnonzero(lab == v)) for v in np.unique(lab))


def _lloyd_score(v, lab):
    # sum over clusters of |sum of members|: the spherical K-means objective at its best centroids
    return sum(np.linalg.norm(v[lab == c].sum(0)) for c in np.unique(lab))


def test_kmeans_recovers_well_separated_groups():
    g = np.random.default_rng(3)
    centres = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, -1.0], [-0.6, -0.8, 0]])
    pts, truth = [], []
    for c, ctr in enumerate(centres):
        x = ctr + 0.05 * g.standard_normal((40, 3))
        pts.append(x / np.linalg.norm(x, axis=1, keepdims=True))
        truth += [c] * 40
    v = np.concatenate(pts)
    truth = np.array(truth)
    init = np.array([0, 40, 80, 120], dtype=np.int32)  # one seed per group, ascending
    lab, keff = O.kmeans(v, 4, init)
    assert keff == 4 and np.array_equal(lab, truth)
    # rotating the sphere rotates the clustering
    q, _ = np.linalg.qr(g.standard_normal((3, 3)))
    lab_r, _ = O.kmeans(v @ q.T, 4, init)
    assert np.array_equal(lab_r, truth)


def test_kmeans_output_is_a_lloyd_fixed_point_and_objective_rises():
    g = np.random.default_rng(4)
    v = skygen.sky.positions(500, g)
    init = np.sort(g.choice(500, 12, replace=False)).astype(np.int32)
    lab, keff = O.kmeans(v, 12, init, iters=200)
    # fixed point, recomputed with numpy: each point's label is its nearest normalised mean
    cen = np.stack([v[lab == c].sum(0) for c in range(keff)])
    cen /= np.linalg.norm(cen, axis=1, keepdims=True)
    dots = v @ cen.T
    assert np.all(dots[np.arange(500), lab] >= dots.max(1) - 1e-12)
    # the objective never decreases along the Lloyd iterations
    scores = [_lloyd_score(v, O.kmeans(v, 12, init, iters=t)[0]) for t in range(0, 15)]
    assert all(b >= a - 1e-9 for a, b in zip(scores, scores[1:]))


def test_kmeans_ties_empty_clusters_and_cap():
    g = np.random.default_rng(5)
    v = skygen.sky.positions(60, g)
    v = np.concatenate([v, v[:1]])  # point 60 duplicates point 0
    # centroids 1 and 2 start on identical vectors: every point prefers index 1 (lowest), so with
    # no update cluster 2 has no member and is compacted away
    init = np.array([5, 0, 60], dtype=np.int32)
    lab, keff = O.kmeans(v, 3, init, iters=0)
    assert keff == 2 and set(np.unique(lab)) == {0, 1}
    lab2, _ = O.kmeans(v, 2, init[:2], iters=0)
    assert np.array_equal(lab, lab2)
    # one update: cluster 2 was empty, so it keeps its starting vector while clusters 0 and 1 move
    # to their normalised means (computed here with numpy); the final assignment uses those three
    a0 = np.argmax(v @ v[init[:2]].T, axis=1)
    cen = np.stack([v[a0 == c].sum(0) for c in range(2)] + [v[0]])
    cen[:2] /= np.linalg.norm(cen[:2], axis=1, keepdims=True)
    want = np.argmax(v @ cen.T, axis=1)
    lab, keff = O.kmeans(v, 3, init, iters=1)
    assert _partition(lab) == _partition(want)
    # the cap: k >= n gives every vector its own cluster, by rank
    lab, keff = O.kmeans(v[:7], 7, np.arange(7, dtype=np.int32))
    assert keff == 7 and np.array_equal(lab, np.arange(7))
    lab, keff = O.kmeans(v, 1, np.array([9], dtype=np.int32))
    assert keff == 1 and np.all(lab == 0)


def test_kmeans_agrees_with_independent_generator_implementation():
    # the seeded sky generator carries its own K-means (tensor cumulative sums, a different
    # rounding order); labels may differ only where rounding decides a near-tie
    g = np.random.default_rng(6)
    v = skygen.sky.positions(3072, g)
    for k in (1, 17, 300):
        gi = np.random.default_rng(100 + k)
        init = gi.choice(3072, size=k, replace=False)
        lab_gen, keff_gen = skygen.sky.spherical_kmeans(v, k, np.random.default_rng(100 + k))
        lab, keff = O.kmeans(v, k, init.astype(np.int32))
        assert keff == keff_gen
        assert np.mean(lab == lab_gen) >= 0.999, k


# --------------------------------------------------------------------------------------------
# AdaTopK (App. A)
# --------------------------------------------------------------------------------------------

def _scipy_opt(pr, x0, lo, hi):
    return scipy.optimize.minimize(lambda z: pr.likelihood_grad(z)[0], x0, jac=lambda z: pr.likelihood_grad(z)[1],
                                   method="L-BFGS-B", bounds=list(zip(lo, hi)),
                                   options=dict(ftol=1e-16, gtol=1e-12, maxiter=5000))


def test_adatopk_matches_scipy_optimum():
    sky = skygen.make_tiny(16, 15, (2, 1, 1), seed=16, model_consistent=True)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0], sky.upper[0]
    x0 = np.array([1.54, 1.54, 20.0, -3.0])
    x, f, it, ne, st = pr.adatopk(x0, lo, hi, max_iter=3000)
    assert st & O.CONVERGED, st
    res = _scipy_opt(pr, x0, lo, hi)
    assert f <= res.fun + 1e-12 * abs(res.fun)
    assert np.all(np.abs(x - res.x) <= 1e-4 * np.maximum(1.0, np.abs(res.x)))


def test_adatopk_pins_an_active_bound_and_meets_kkt():
    # the truth puts beta_d above the box: the optimum sits on the upper bound
    sky = skygen.make_tiny(16, 15, (1, 1, 1), seed=19, model_consistent=True, noiseless=True)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0].copy(), sky.upper[0].copy()
    hi[0] = sky.x[0][0] - 0.2  # beta_d bound below its true value
    x, f, it, ne, st = pr.adatopk(np.array(skygen.X0), lo, hi, max_iter=3000)
    assert st & O.CONVERGED, st
    assert x[0] == hi[0]  # pinned exactly on the bound
    _, g, _, _ = pr.likelihood_grad(x)
    assert g[0] < 0  # F still decreases outward: the bound is active
    res = _scipy_opt(pr, np.array(skygen.X0), lo, hi)
    assert np.all(np.abs(x - res.x) <= 1e-4 * np.maximum(1.0, np.abs(res.x)))


def test_adatopk_rescaling_makes_tiny_objectives_behave_like_unit_ones():
    # multiplying d by 1e-12 multiplies F and g by 1e-24; without the rescaling the AdaBelief
    # epsilon (1e-16 inside the second moment) would dominate and the steps would vanish
    sky = skygen.make_tiny(16, 15, (2, 1, 1), seed=16, model_consistent=True)
    lo, hi = sky.lower[0], sky.upper[0]
    x0 = np.array([1.54, 1.54, 20.0, -3.0])
    pr = O.Problem.from_sky(sky)
    pr_s = O.Problem.from_sky(sky, d=sky.item_d(0) * 1e-12)
    x, f, it, _, st = pr.adatopk(x0, lo, hi, max_iter=3000)
    xs, fs, its, _, sts = pr_s.adatopk(x0, lo, hi, max_iter=3000)
    assert st & O.CONVERGED and sts & O.CONVERGED
    assert np.all(np.abs(xs - x) <= 1e-5 * np.maximum(1.0, np.abs(x)))


def test_adatopk_release_fraction_reaches_the_same_optimum():
    sky = skygen.make_tiny(32, 15, (3, 2, 2), seed=17)
    pr = O.Problem.from_sky(sky)
    lo, hi = sky.lower[0], sky.upper[0]
    x0 = lo.copy()  # every parameter starts pinned at its lower bound
    x_ref = pr.lbfgs(np.concatenate([np.full(3, 1.54), np.full(2, 20.0), np.full(2, -3.0)]), lo, hi)[0]
    for topk in (0.0, 1.0):
        x, f, it, ne, st = pr.adatopk(x0, lo, hi, topk=topk, max_iter=5000)
        assert st & O.CONVERGED, (topk, st)
        assert np.all(np.abs(x - x_ref) <= 1e-4 * np.maximum(1.0, np.abs(x_ref))), topk


def test_fewer_bands_than_components_is_not_positive_definite():
    # with two bands the 3x3 matrix A^T N^-1 A has rank 2 at every pixel; with three or more
    # generic bands it is positive definite
    for nfreq, singular in ((2, True), (3, False), (4, False)):
        sky = skygen.make_tiny(20, nfreq, (1, 1, 1), seed=55)
        pr = O.Problem.from_sky(sky)
        for p in range(20):
            st = pr.pixel(sky.x[0], p)["status"]
            assert bool(st & O.NOT_PD) == singular, (nfreq, p)
