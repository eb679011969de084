"""ctypes front end of the FP64 C oracle (``cs_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the CPU-baseline leg of
the benchmark.  Nothing in the library under ``paper_2604_08463_amd/`` may import it.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cs_oracle.c")
LIB = os.path.join(HERE, "libcs_oracle.so")

NOT_PD, NONFINITE, LS_FAIL, MAXITER, CONVERGED = 1, 2, 4, 8, 16
E_INVALID, E_LABEL = -1, -2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, ISO C11, no fast-math, no FMA contraction."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class _Problem(C.Structure):
    _fields_ = [
        ("nfreq", C.c_int32), ("npix", C.c_int32),
        ("freqs", C.POINTER(C.c_double)),
        ("nu0_dust", C.c_double), ("nu0_sync", C.c_double), ("tcmb", C.c_double),
        ("d", C.POINTER(C.c_double)),
        ("ninv", C.POINTER(C.c_double)),
        ("ninv_per_pixel", C.c_int32),
        ("labels", C.POINTER(C.c_int32)),
        ("nclusters", C.c_int32 * 3),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.POINTER
        dp, ip = P(C.c_double), P(C.c_int32)
        L.orc_sed.argtypes = [C.c_double] * 7 + [dp] * 5
        L.orc_rj_to_cmb.argtypes = [C.c_double, C.c_double]
        L.orc_rj_to_cmb.restype = C.c_double
        L.orc_check_labels.argtypes = [P(_Problem)]
        L.orc_pixel.argtypes = [P(_Problem), dp, C.c_int32, dp, dp, dp, dp, dp, dp]
        L.orc_likelihood_grad.argtypes = [P(_Problem), dp, dp, dp, dp]
        L.orc_grad_abs.argtypes = [P(_Problem), dp, dp]
        L.orc_grad_terms.argtypes = [P(_Problem), dp, dp]
        L.orc_component_maps.argtypes = [P(_Problem), dp, dp, dp]
        L.orc_data_chi2.argtypes = [P(_Problem)]
        L.orc_data_chi2.restype = C.c_double
        L.orc_segments.argtypes = [C.c_int64, ip, C.c_int32, ip, ip]
        L.orc_segments.restype = C.c_int64
        L.orc_adatopk.argtypes = [P(_Problem), dp, dp, dp] + [C.c_double] * 6 + [C.c_int32, C.c_int32, C.c_double,
                                                                                 dp, P(C.c_int32), P(C.c_int64)]
        L.orc_kmeans.argtypes = [C.c_int64, dp, C.c_int32, ip, C.c_int32, ip]
        L.orc_kmeans.restype = C.c_int32
        L.orc_lbfgs.argtypes = [P(_Problem), dp, dp, dp, C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                C.c_double, dp, P(C.c_int32), P(C.c_int64)]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Problem:
    """One item: data ``d[2][F][P]``, weights ``ninv`` ([2][F] or [2][F][P]), labels ``[3][P]``."""

    def __init__(self, freqs, d, ninv, labels, nclusters, nu0_dust=353.0, nu0_sync=23.0, tcmb=2.7255):
        self.freqs = np.ascontiguousarray(freqs, dtype=np.float64)
        self.d = np.ascontiguousarray(d, dtype=np.float64)
        self.ninv = np.ascontiguousarray(ninv, dtype=np.float64)
        self.labels = np.ascontiguousarray(labels, dtype=np.int32)
        F = self.freqs.size
        P = self.labels.shape[-1]
        assert self.d.shape == (2, F, P), self.d.shape
        assert self.labels.shape == (3, P)
        per_pixel = self.ninv.ndim == 3
        assert self.ninv.shape == ((2, F, P) if per_pixel else (2, F))
        self.nclusters = [int(v) for v in nclusters]
        self.K = sum(self.nclusters)
        self._s = _Problem(F, P, _dp(self.freqs), nu0_dust, nu0_sync, tcmb, _dp(self.d), _dp(self.ninv),
                           int(per_pixel), _ip(self.labels), (C.c_int32 * 3)(*self.nclusters))

    @classmethod
    def from_sky(cls, sky, item: int = 0, d=None):
        dd = sky.item_d(item) if d is None else d
        return cls(sky.freqs, dd, sky.ninv, sky.item_labels(item), sky.nclusters[item],
                   sky.nu0_dust, sky.nu0_sync, sky.tcmb)

    def check_labels(self) -> int:
        return lib().orc_check_labels(C.byref(self._s))

    def likelihood_grad(self, x):
        """Returns ``(F, grad[K], cluster_F[K], status)``; raises on a negative error code."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.K
        f = np.zeros(1)
        g = np.zeros(self.K)
        cf = np.zeros(self.K)
        st = lib().orc_likelihood_grad(C.byref(self._s), _dp(x), _dp(f), _dp(g), _dp(cf))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return float(f[0]), g, cf, st

    def grad_abs(self, x):
        """Per cluster (packed like the gradient) the sum over its pixels of |dF_p/dtheta|: the
        scale against which a cluster's gradient error is bounded."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.K
        ga = np.zeros(self.K)
        st = lib().orc_grad_abs(C.byref(self._s), _dp(x), _dp(ga))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return ga

    def grad_terms(self, x):
        """Per cluster (packed like the gradient) the summed magnitude of the terms its gradient
        is built from (|s_c| w |dA/dtheta| (|d| + |A||s|) over pixels, Stokes and bands): the scale
        of the rounding error of sums accumulated in reduced precision."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.size == self.K
        gt = np.zeros(self.K)
        st = lib().orc_grad_terms(C.byref(self._s), _dp(x), _dp(gt))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return gt

    def pixel(self, x, p: int):
        """Per-pixel details: dict(M [2,3,3], b [2,3], s [2,3], r [2,F], f, g [3], status)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        F = self.freqs.size
        m = np.zeros((2, 3, 3))
        b = np.zeros((2, 3))
        s = np.zeros((2, 3))
        r = np.zeros((2, F))
        f = np.zeros(1)
        g = np.zeros(3)
        st = lib().orc_pixel(C.byref(self._s), _dp(x), int(p), _dp(m), _dp(b), _dp(s), _dp(r), _dp(f), _dp(g))
        return dict(M=m, b=b, s=s, r=r, f=float(f[0]), g=g, status=st)

    def component_maps(self, x):
        """GLS amplitudes ``s_hat[2][3][P]`` (NaN where excluded) and sigma^2_CMB (Q + U)."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        P = self.labels.shape[1]
        s = np.zeros((2, 3, P))
        v = np.zeros(1)
        st = lib().orc_component_maps(C.byref(self._s), _dp(x), _dp(s), _dp(v))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return s, float(v[0]), st

    def data_chi2(self) -> float:
        return lib().orc_data_chi2(C.byref(self._s))

    def lbfgs(self, x0, lo, hi, m=10, gtol=1e-8, max_iter=1000, max_backtracks=30, c1=1e-4):
        """Projected L-BFGS; returns ``(x, F, iters, nevals, status)``."""
        x = np.array(x0, dtype=np.float64, copy=True)
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        f = np.zeros(1)
        it = C.c_int32(0)
        ne = C.c_int64(0)
        st = lib().orc_lbfgs(C.byref(self._s), _dp(lo), _dp(hi), _dp(x), m, gtol, max_iter, max_backtracks, c1,
                             _dp(f), C.byref(it), C.byref(ne))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return x, float(f[0]), it.value, ne.value, st

    def adatopk(self, x0, lo, hi, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-16, topk=0.0, gtol=1e-8, max_iter=1000,
                 max_backtracks=30, c1=1e-4):
        """AdaTopK (App. A); returns ``(x, F, iters, nevals, status)``."""
        x = np.array(x0, dtype=np.float64, copy=True)
        lo = np.ascontiguousarray(lo, dtype=np.float64)
        hi = np.ascontiguousarray(hi, dtype=np.float64)
        f = np.zeros(1)
        it = C.c_int32(0)
        ne = C.c_int64(0)
        st = lib().orc_adatopk(C.byref(self._s), _dp(lo), _dp(hi), _dp(x), lr, beta1, beta2, eps, topk, gtol, max_iter,
                               max_backtracks, c1, _dp(f), C.byref(it), C.byref(ne))
        if st < 0:
            raise ValueError(f"oracle error {st}")
        return x, float(f[0]), it.value, ne.value, st


def sed(nu, beta_d, temp_d, beta_s, nu0d=353.0, nu0s=23.0, tcmb=2.7255):
    """Columns and derivatives for one band: ``(a_d, a_s, dad_dbeta, dad_dT, das_dbeta)``."""
    out = [C.c_double() for _ in range(5)]
    lib().orc_sed(nu, nu0d, nu0s, tcmb, beta_d, temp_d, beta_s, *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def rj_to_cmb(nu, tcmb=2.7255) -> float:
    return lib().orc_rj_to_cmb(nu, tcmb)


def segments(labels_j, k: int):
    """Stable CSR of one labelling: ``(perm[n_incl], offsets[k+1])``."""
    lab = np.ascontiguousarray(labels_j, dtype=np.int32)
    perm = np.zeros(lab.size, dtype=np.int32)
    off = np.zeros(k + 1, dtype=np.int32)
    n = lib().orc_segments(lab.size, _ip(lab), int(k), _ip(perm), _ip(off))
    if n < 0:
        raise ValueError(f"oracle error {n}")
    return perm[:n].copy(), off


def kmeans(vecs, k: int, init, iters: int = 20):
    """Spherical K-means of unit vectors ``vecs[n][3]``; returns ``(labels[n], K_eff)``."""
    v = np.ascontiguousarray(vecs, dtype=np.float64)
    n = v.shape[0]
    ini = np.ascontiguousarray(init, dtype=np.int32)
    assert ini.size >= min(k, n) or k >= n
    lab = np.zeros(max(n, 1), dtype=np.int32)
    keff = lib().orc_kmeans(n, _dp(v), int(k), _ip(ini) if ini.size else None, int(iters), _ip(lab))
    if keff < 0:
        raise ValueError(f"oracle error {keff}")
    return lab[:n].copy(), int(keff)
