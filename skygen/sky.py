"""Seeded LiteBIRD-shaped synthetic skies (stand-ins for the paper's PySM3 / Planck / LiteBIRD inputs).

Every array is drawn from NumPy ``PCG64`` streams seeded by
``SeedSequence([2604, 8463, config_id, stream_id, *sub])``, on the host for every target device
(a GPU workload holds the same numbers as its CPU copy).  The simulated sky follows the paper's data
model (Sec. 2.1, eq. data_model): per pixel, multi-band Q/U data equal to CMB + dust + synchrotron
plus white noise.

The emission laws are evaluated the way a sky simulator does it: a specific intensity
(modified blackbody ``nu^beta B_nu(T)`` for dust, a Rayleigh-Jeans power law for synchrotron) is
converted to CMB thermodynamic units by dividing by the derivative of the CMB blackbody,
``dB_nu/dT`` at ``T_CMB``, and normalised at the reference frequency.  Neither the oracle nor the
HIP library uses this code: each builds its own mixing matrix.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

H_PLANCK = 6.62607015e-34  # J s (exact SI value)
K_BOLTZ = 1.380649e-23  # J / K (exact SI value)
C_LIGHT = 299792458.0  # m / s
T_CMB = 2.7255  # K
GHZ = 1.0e9

NU0_DUST = 353.0  # GHz
NU0_SYNC = 23.0  # GHz

#: box bounds of (beta_d, T_d, beta_s); the truth is clipped into the box
BOUNDS = ((0.5, 3.0), (5.0, 50.0), (-5.0, -1.0))
#: starting point of every cluster for the optimiser workloads
X0 = (1.54, 20.0, -3.0)

_STREAM = dict(pos=0, cmb=1, dust=2, sync=3, field_bd=4, field_td=5, field_bs=6, sigma=7,
               noise=8, kmeans=9, mask=10, points=11, kcounts=12)


def _rng(cid: int, stream: str, *sub: int) -> np.random.Generator:
    seq = np.random.SeedSequence([2604, 8463, int(cid), _STREAM[stream], *[int(s) for s in sub]])
    return np.random.Generator(np.random.PCG64(seq))


# ----------------------------------------------------------------------------------------------
# instrument
# ----------------------------------------------------------------------------------------------

def bands(nu_lo: float, nu_hi: float, nfreq: int) -> np.ndarray:
    """Log-spaced band centres in GHz, ``nu_i = nu_lo (nu_hi/nu_lo)^(i/(F-1))``."""
    if nfreq == 1:
        return np.array([nu_lo], dtype=np.float64)
    i = np.arange(nfreq, dtype=np.float64)
    return nu_lo * (nu_hi / nu_lo) ** (i / (nfreq - 1))


# ----------------------------------------------------------------------------------------------
# emission laws (sky simulator route: intensity -> K_CMB through dB/dT at T_CMB)
# ----------------------------------------------------------------------------------------------

def _planck(nu_hz, temp):
    x = H_PLANCK * nu_hz / (K_BOLTZ * temp)
    return 2.0 * H_PLANCK * nu_hz ** 3 / C_LIGHT ** 2 / np.expm1(x)


def _dplanck_dt_cmb(nu_hz):
    x = H_PLANCK * nu_hz / (K_BOLTZ * T_CMB)
    return 2.0 * H_PLANCK * nu_hz ** 3 / C_LIGHT ** 2 * (x / T_CMB) * np.exp(x) / np.expm1(x) ** 2


def sky_sed_dust(nu_ghz, beta, temp, nu0_ghz: float = NU0_DUST):
    """Dust emission in K_CMB normalised to 1 at ``nu0``; ``nu`` [F] x params [...] -> [F, ...]."""
    nu = np.asarray(nu_ghz, np.float64).reshape((-1,) + (1,) * np.ndim(beta)) * GHZ
    nu0 = nu0_ghz * GHZ
    beta = np.asarray(beta, np.float64)
    temp = np.asarray(temp, np.float64)
    num = (nu / nu0) ** beta * _planck(nu, temp) / _dplanck_dt_cmb(nu)
    den = _planck(nu0, temp) / _dplanck_dt_cmb(nu0)
    return num / den


def sky_sed_sync(nu_ghz, beta, nu0_ghz: float = NU0_SYNC):
    """Synchrotron (RJ power law ``T_RJ ~ nu^beta``) in K_CMB normalised to 1 at ``nu0``."""
    nu = np.asarray(nu_ghz, np.float64).reshape((-1,) + (1,) * np.ndim(beta)) * GHZ
    nu0 = nu0_ghz * GHZ
    beta = np.asarray(beta, np.float64)
    rj = 2.0 * K_BOLTZ * nu ** 2 / C_LIGHT ** 2 * (nu / nu0) ** beta
    rj0 = 2.0 * K_BOLTZ * nu0 ** 2 / C_LIGHT ** 2
    return (rj / _dplanck_dt_cmb(nu)) / (rj0 / _dplanck_dt_cmb(nu0))


# ----------------------------------------------------------------------------------------------
# geometry: positions, smooth fields, spherical K-means, masks
# ----------------------------------------------------------------------------------------------

def positions(npix: int, g: np.random.Generator) -> np.ndarray:
    """Unit vectors uniform on the sphere: ``z ~ U[-1,1]``, ``phi ~ U[0, 2 pi)``."""
    z = g.uniform(-1.0, 1.0, npix)
    phi = g.uniform(0.0, 2.0 * math.pi, npix)
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def smooth_field(vecs: np.ndarray, ell_deg: float, mean: float, sigma: float,
                 g: np.random.Generator, nfeat: int = 4096, device="cpu") -> np.ndarray:
    """Gaussian random field with a squared-exponential kernel on chord distance (length ``ell``).

    Sampled with ``nfeat`` random Fourier features: ``f(n) = sqrt(2/M) sum_m cos(w_m . n + b_m)``,
    ``w_m ~ N(0, I / ell^2)``, ``b_m ~ U[0, 2 pi)``; unit variance, then ``mean + sigma f``.
    """
    ell = math.radians(ell_deg)
    omega = g.standard_normal((3, nfeat)) / ell
    phase = g.uniform(0.0, 2.0 * math.pi, nfeat)
    v = torch.as_tensor(vecs, dtype=torch.float64, device=device)
    w = torch.as_tensor(omega, dtype=torch.float64, device=device)
    b = torch.as_tensor(phase, dtype=torch.float64, device=device)
    out = torch.empty(v.shape[0], dtype=torch.float64, device=device)
    step = 8192
    for s in range(0, v.shape[0], step):
        out[s:s + step] = torch.cos(v[s:s + step] @ w + b).sum(dim=1)
    f = out.cpu().numpy() * math.sqrt(2.0 / nfeat)
    return mean + sigma * f


def _assign(v: torch.Tensor, c: torch.Tensor) -> torch.Tensor:
    lab = torch.empty(v.shape[0], dtype=torch.int64, device=v.device)
    step = max(1024, int(2 ** 25 // max(1, c.shape[0])))
    for s in range(0, v.shape[0], step):
        # argmax returns the first maximal index: ties go to the lowest centroid index
        lab[s:s + step] = torch.argmax(v[s:s + step] @ c.T, dim=1)
    return lab


def spherical_kmeans(vecs: np.ndarray, k: int, g: np.random.Generator, iters: int = 20,
                     device="cpu") -> tuple[np.ndarray, int]:
    """Spherical Lloyd K-means on unit vectors (Sec. 2.2).

    Initial centroids: ``k`` distinct points drawn without replacement.  Each of the ``iters``
    iterations assigns every point to the centroid of largest dot product (ties: lowest index),
    then replaces each centroid by the renormalised mean of its members (an empty cluster keeps
    its centroid).  Final labels come from one more assignment, then are compacted to
    ``0..K_eff-1`` in ascending centroid index.  ``k >= n`` returns one cluster per point (the
    patch-count cap of Table 1).  Returns ``(labels int32 [n], K_eff)``.
    """
    n = vecs.shape[0]
    if k >= n:
        return np.arange(n, dtype=np.int32), n
    init = g.choice(n, size=k, replace=False)
    v = torch.as_tensor(vecs, dtype=torch.float64, device=device)
    c = v[torch.as_tensor(init, device=device)].clone()
    zero = torch.zeros((1, 3), dtype=torch.float64, device=device)
    for _ in range(iters):
        lab = _assign(v, c)
        order = torch.argsort(lab, stable=True)
        counts = torch.bincount(lab, minlength=k)
        csum = torch.cat([zero, torch.cumsum(v[order], dim=0)], dim=0)
        ends = torch.cumsum(counts, dim=0)
        sums = csum[ends] - csum[ends - counts]
        norm = torch.linalg.vector_norm(sums, dim=1, keepdim=True)
        ok = (counts > 0).unsqueeze(1) & (norm > 0)
        c = torch.where(ok, sums / torch.where(norm > 0, norm, torch.ones_like(norm)), c)
    lab = _assign(v, c).cpu().numpy()
    used = np.unique(lab)
    remap = np.full(k, -1, dtype=np.int64)
    remap[used] = np.arange(used.size)
    return remap[lab].astype(np.int32), int(used.size)


def kcap_labels(k: int, keep: np.ndarray, vecs: np.ndarray, g: np.random.Generator,
                iters: int = 20, device="cpu") -> tuple[np.ndarray, int]:
    """Labels over all pixels (-1 where masked) for ``k`` requested clusters on the kept pixels."""
    idx = np.flatnonzero(keep)
    lab = np.full(keep.size, -1, dtype=np.int32)
    sub, keff = spherical_kmeans(vecs[idx], k, g, iters=iters, device=device)
    lab[idx] = sub
    return lab, keff


def latitude_mask(z: np.ndarray, fsky: float) -> np.ndarray:
    """Keep the ``round(fsky P)`` pixels of largest ``|z|`` (ties: lower pixel index)."""
    n = int(round(fsky * z.size))
    order = np.lexsort((np.arange(z.size), -np.abs(z)))
    keep = np.zeros(z.size, dtype=bool)
    keep[order[:n]] = True
    return keep


# ----------------------------------------------------------------------------------------------
# sky
# ----------------------------------------------------------------------------------------------

@dataclass
class Sky:
    """One synthetic workload: shared geometry plus a batch of items.

    Arrays follow the library's layouts: ``d`` is ``[B or 1][2][F][P]`` float64 in uK_CMB,
    ``ninv`` is ``[2][F]`` (uK^-2), ``labels`` is ``[B or 1][3][P]`` int32 (-1 = excluded),
    ``nclusters`` is ``[B][3]`` and ``x`` holds one packed parameter vector per item,
    ``[beta_d (K_d) | T_d (K_T) | beta_s (K_s)]``.
    """

    cid: int
    freqs: np.ndarray
    sigma: np.ndarray
    ninv: np.ndarray
    vecs: np.ndarray
    truth: np.ndarray
    signal: np.ndarray
    d: torch.Tensor
    labels: torch.Tensor
    nclusters: np.ndarray
    x: list
    lower: list = field(default_factory=list)
    upper: list = field(default_factory=list)
    nu0_dust: float = NU0_DUST
    nu0_sync: float = NU0_SYNC
    tcmb: float = T_CMB
    meta: dict = field(default_factory=dict)

    @property
    def nitems(self) -> int:
        return int(self.nclusters.shape[0])

    @property
    def npix(self) -> int:
        return int(self.vecs.shape[0])

    @property
    def nfreq(self) -> int:
        return int(self.freqs.size)

    def param_offsets(self) -> np.ndarray:
        k = self.nclusters.sum(axis=1).astype(np.int64)
        return np.concatenate([[0], np.cumsum(k)])

    def x_packed(self) -> np.ndarray:
        return np.concatenate(self.x).astype(np.float64)

    def bounds_packed(self) -> tuple[np.ndarray, np.ndarray]:
        return np.concatenate(self.lower), np.concatenate(self.upper)

    def item_d(self, b: int) -> np.ndarray:
        return self.d[b if self.d.shape[0] > 1 else 0].cpu().numpy()

    def item_labels(self, b: int) -> np.ndarray:
        return self.labels[b if self.labels.shape[0] > 1 else 0].cpu().numpy()


def _box(nc) -> tuple[np.ndarray, np.ndarray]:
    lo = np.concatenate([np.full(int(nc[j]), BOUNDS[j][0]) for j in range(3)])
    hi = np.concatenate([np.full(int(nc[j]), BOUNDS[j][1]) for j in range(3)])
    return lo, hi


def _x0(nc) -> np.ndarray:
    return np.concatenate([np.full(int(nc[j]), X0[j]) for j in range(3)])


def start_and_box(nc) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Optimiser start ``x0`` (X0 for every cluster) and box bounds for cluster counts ``nc``."""
    lo, hi = _box(nc)
    return _x0(nc), lo, hi


def _clip_truth(t: np.ndarray) -> np.ndarray:
    out = t.copy()
    for j in range(3):
        out[j] = np.clip(out[j], BOUNDS[j][0], BOUNDS[j][1])
    return out


def _amplitudes(cid: int, npix: int):
    g = _rng(cid, "cmb")
    cmb = g.normal(0.0, 0.5, (2, npix))

    def polarised(stream, median):
        gg = _rng(cid, stream)
        amp = median * np.exp(0.5 * gg.standard_normal(npix))
        psi = gg.uniform(0.0, math.pi, npix)
        return np.stack([amp * np.cos(2 * psi), amp * np.sin(2 * psi)])

    return cmb, polarised("dust", 10.0), polarised("sync", 5.0)


def _signal(freqs, truth, cmb, dust, sync, nu0d=NU0_DUST, nu0s=NU0_SYNC) -> np.ndarray:
    ad = sky_sed_dust(freqs, truth[0], truth[1], nu0d)  # [F, P]
    as_ = sky_sed_sync(freqs, truth[2], nu0s)  # [F, P]
    return cmb[:, None, :] + ad[None] * dust[:, None, :] + as_[None] * sync[:, None, :]  # [2, F, P]


def _noise(cid: int, sigma: np.ndarray, nreal: int, npix: int, device, first: int = 0) -> torch.Tensor:
    """White noise ``[R][2][F][P]``: realization ``r`` is drawn from its own NumPy ``PCG64`` stream
    ``(cid, noise, first + r)`` on the host whatever the target device, so a GPU workload and its
    CPU copy hold the same numbers.  Realizations are drawn on a few threads (the generator
    releases the GIL) and copied to the device in groups."""
    f = sigma.size
    out = torch.empty((nreal, 2, f, npix), dtype=torch.float64, device=device)

    def draw(r):
        return _rng(cid, "noise", first + r).standard_normal((2, f, npix)) * sigma[None, :, None]

    group = 8
    with ThreadPoolExecutor(max_workers=min(group, max(1, os.cpu_count() or 1))) as ex:
        for r0 in range(0, nreal, group):
            parts = list(ex.map(draw, range(r0, min(nreal, r0 + group))))
            out[r0:r0 + len(parts)] = torch.from_numpy(np.stack(parts)).to(device)
    return out


def _field_truth(cid, vecs, ell_deg, device):
    if ell_deg is None:  # i.i.d. per pixel (deliberately mis-specified single-cluster model)
        npix = vecs.shape[0]
        t = np.stack([
            _rng(cid, "field_bd").normal(1.54, 0.1, npix),
            _rng(cid, "field_td").normal(20.0, 2.0, npix),
            _rng(cid, "field_bs").normal(-3.0, 0.1, npix),
        ])
    else:
        t = np.stack([
            smooth_field(vecs, ell_deg, 1.54, 0.1, _rng(cid, "field_bd"), device=device),
            smooth_field(vecs, ell_deg, 20.0, 2.0, _rng(cid, "field_td"), device=device),
            smooth_field(vecs, ell_deg, -3.0, 0.1, _rng(cid, "field_bs"), device=device),
        ])
    return _clip_truth(t)


_DEFAULTS = {
    1: dict(npix=3072, nfreq=15, band=(40.0, 402.0), sig=(2.0, 20.0), ell=None, k=(1, 1, 1), items=64),
    2: dict(npix=49152, nfreq=15, band=(40.0, 402.0), sig=(2.0, 20.0), ell=5.0, k=(1000, 50, 200), items=8),
    3: dict(npix=3072, nfreq=15, band=(40.0, 402.0), sig=(2.0, 20.0), ell=None, k=(1, 1, 1), items=256),
    4: dict(npix=3072, nfreq=15, band=(40.0, 402.0), sig=(2.0, 20.0), ell=None, k=None, items=1024),
    5: dict(npix=196608, nfreq=22, band=(34.0, 448.0), sig=(1.0, 30.0), ell=2.0, k=(5000, 500, 2000), items=64),
}


def make_config(cid: int, *, npix: int | None = None, nitems: int | None = None,
                k: tuple | None = None, nfreq: int | None = None, device="cpu",
                kmax4: tuple = (3000, 500, 1000)) -> Sky:
    """Build workload ``cid`` (1..5); sizes may be reduced for tests.

    1: 3072 px, 15 bands, one cluster per parameter, 64 parameter points, one noise realization.
    2: 49152 px, smooth fields (5 deg), K-means labels K = (1000, 50, 200), 8 parameter points.
    3: the workload-1 sky with 256 noise realizations, optimiser start x0.
    4: the workload-1 sky, 1024 cluster configurations with seeded K and latitude masks.
    5: 196608 px, 22 bands 34-448 GHz, smooth fields (2 deg), K = (5000, 500, 2000), 64 realizations.
    """
    cfg = dict(_DEFAULTS[cid])
    if npix is not None:
        cfg["npix"] = npix
    if nitems is not None:
        cfg["items"] = nitems
    if k is not None:
        cfg["k"] = k
    if nfreq is not None:
        cfg["nfreq"] = nfreq
    # workloads 3 and 4 reuse the workload-1 sky draws
    sky_id = 1 if cid in (1, 3, 4) else cid
    P, F, B = cfg["npix"], cfg["nfreq"], cfg["items"]
    freqs = bands(cfg["band"][0], cfg["band"][1], F)
    sigma = _rng(sky_id, "sigma").uniform(cfg["sig"][0], cfg["sig"][1], F)
    ninv = np.tile(1.0 / sigma ** 2, (2, 1))
    vecs = positions(P, _rng(sky_id, "pos"))
    truth = _field_truth(sky_id, vecs, cfg["ell"], device)
    cmb, dust, sync = _amplitudes(sky_id, P)
    signal = _signal(freqs, truth, cmb, dust, sync)
    sig_t = torch.as_tensor(signal, dtype=torch.float64, device=device)
    meta = dict(workload=cid, npix=P, nfreq=F, items=B)

    if cid in (1, 2):
        d = sig_t.unsqueeze(0) + _noise(sky_id, sigma, 1, P, device)
        if cid == 1:
            nc = np.array([1, 1, 1], dtype=np.int32)
            labels = np.zeros((1, 3, P), dtype=np.int32)
            g = _rng(cid, "points")
            pts = np.stack([g.uniform(1.24, 1.84, B), g.uniform(14.0, 26.0, B), g.uniform(-3.3, -2.7, B)], axis=1)
            xs = [p.copy() for p in pts]
        else:
            labs, kk = [], []
            for j in range(3):
                lab, keff = spherical_kmeans(vecs, cfg["k"][j], _rng(cid, "kmeans", j), device=device)
                labs.append(lab)
                kk.append(keff)
            nc = np.array(kk, dtype=np.int32)
            labels = np.stack(labs)[None]
            base = []
            for j in range(3):
                s = np.bincount(labs[j], weights=truth[j], minlength=kk[j])
                c = np.bincount(labs[j], minlength=kk[j])
                base.append(s / np.maximum(c, 1))
            base = np.concatenate(base)
            g = _rng(cid, "points")
            scale = np.concatenate([np.full(kk[0], 0.05), np.full(kk[1], 1.0), np.full(kk[2], 0.05)])
            lo, hi = _box(nc)
            xs = [base.copy()] + [np.clip(base + scale * g.standard_normal(base.size), lo, hi) for _ in range(B - 1)]
        ncl = np.tile(nc, (B, 1))
        lo, hi = _box(nc)
        return Sky(cid, freqs, sigma, ninv, vecs, truth, signal, d,
                   torch.as_tensor(labels), ncl, xs, [lo] * B, [hi] * B, meta=meta)

    if cid in (3, 5):
        d = sig_t.unsqueeze(0) + _noise(sky_id, sigma, B, P, device, first=1)
        if cid == 3:
            nc = np.array([1, 1, 1], dtype=np.int32)
            labels = np.zeros((1, 3, P), dtype=np.int32)
        else:
            labs, kk = [], []
            for j in range(3):
                lab, keff = spherical_kmeans(vecs, cfg["k"][j], _rng(cid, "kmeans", j), device=device)
                labs.append(lab)
                kk.append(keff)
            nc = np.array(kk, dtype=np.int32)
            labels = np.stack(labs)[None]
        lo, hi = _box(nc)
        return Sky(cid, freqs, sigma, ninv, vecs, truth, signal, d, torch.as_tensor(labels),
                   np.tile(nc, (B, 1)), [_x0(nc) for _ in range(B)], [lo] * B, [hi] * B, meta=meta)

    # workload 4: cluster-configuration scan on the shared workload-1 data
    d = sig_t.unsqueeze(0) + _noise(sky_id, sigma, 1, P, device)
    kd, kt, ks, fsky = _scan_draws(cid, B, kmax4)
    labels = np.empty((B, 3, P), dtype=np.int32)
    ncl = np.empty((B, 3), dtype=np.int32)
    xs, lows, highs = [], [], []
    for b in range(B):
        keep = latitude_mask(vecs[:, 2], fsky[b])
        for j, kreq in enumerate((kd[b], kt[b], ks[b])):
            lab, keff = kcap_labels(int(kreq), keep, vecs, _rng(cid, "kmeans", b, j), device=device)
            labels[b, j] = lab
            ncl[b, j] = keff
        xs.append(_x0(ncl[b]))
        lo, hi = _box(ncl[b])
        lows.append(lo)
        highs.append(hi)
    meta.update(k_requested=np.stack([kd, kt, ks], axis=1), fsky=fsky)
    return Sky(cid, freqs, sigma, ninv, vecs, truth, signal, d, torch.as_tensor(labels),
               ncl, xs, lows, highs, meta=meta)


def _scan_draws(cid: int, nitems: int, kmax4: tuple):
    """Requested cluster counts and sky fractions of the configuration scan."""
    g = _rng(cid, "kcounts")
    kd = g.integers(10, kmax4[0] + 1, nitems)
    kt = g.integers(1, kmax4[1] + 1, nitems)
    ks = g.integers(1, kmax4[2] + 1, nitems)
    fsky = _rng(cid, "mask").uniform(0.4, 0.8, nitems)
    return kd, kt, ks, fsky


@dataclass
class ScanTasks:
    """Inputs of the configuration scan with its patchings left to be computed: one spherical
    K-means task per (configuration c, parameter j), task t = 3 c + j.

    ``keep[t]`` marks the pixels configuration c keeps (latitude cut), ``k[t]`` the requested
    cluster count and ``init[t, :k[t]]`` (when ``k[t]`` is below the kept count) the indices, into
    the kept pixels in ascending order, of the starting centroids -- the same seeded draws the
    generator's own K-means uses.  ``sky`` holds the shared data (its labels and parameter points
    are workload 1's and play no part here)."""

    sky: Sky
    keep: np.ndarray  # [3C][P] bool
    k: np.ndarray     # [3C] int32
    init: np.ndarray  # [3C][max k] int32

    def task(self, c: int, j: int):
        t = 3 * c + j
        return self.keep[t], int(self.k[t]), self.init[t, :self.k[t]]


def scan_tasks(nitems: int = 1024, kmax4: tuple = (3000, 500, 1000), device="cpu") -> ScanTasks:
    """Workload 4's inputs for patchings computed elsewhere (e.g. on the device)."""
    cid = 4
    base = make_config(1, nitems=1, device=device)
    P = base.npix
    kd, kt, ks, fsky = _scan_draws(cid, nitems, kmax4)
    kreq = np.stack([kd, kt, ks], axis=1).astype(np.int32).reshape(-1)
    keep = np.empty((3 * nitems, P), dtype=bool)
    init = np.zeros((3 * nitems, int(kreq.max())), dtype=np.int32)
    for c in range(nitems):
        kc = latitude_mask(base.vecs[:, 2], fsky[c])
        n = int(kc.sum())
        for j in range(3):
            t = 3 * c + j
            keep[t] = kc
            if kreq[t] < n:  # the generator's K-means draws its start the same way
                init[t, :kreq[t]] = _rng(cid, "kmeans", c, j).choice(n, size=int(kreq[t]), replace=False)
    base.meta.update(workload=4, items=nitems, k_requested=kreq.reshape(nitems, 3), fsky=fsky)
    return ScanTasks(base, keep, kreq, init)


def make_tiny(npix: int, nfreq: int, k=(1, 1, 1), *, seed: int = 0, nitems: int = 1,
              noiseless: bool = False, nu_range=(40.0, 402.0), model_consistent: bool = False,
              mask_frac: float = 0.0) -> Sky:
    """Small skies for oracle pins and parity edge cases (seeded by ``seed``).

    ``model_consistent``: the true parameters are constant on the clusters of a random labelling,
    so the fitted model contains the truth (with ``noiseless`` the truth is an exact optimum).
    """
    cid = 100 + seed
    freqs = bands(nu_range[0], nu_range[1], nfreq)
    sigma = _rng(cid, "sigma").uniform(2.0, 20.0, nfreq)
    ninv = np.tile(1.0 / sigma ** 2, (2, 1))
    vecs = positions(npix, _rng(cid, "pos"))
    g = _rng(cid, "kmeans")
    nc = np.array(k, dtype=np.int32)
    labels = np.stack([g.integers(0, max(1, kk), npix) for kk in k]).astype(np.int32)
    for j in range(3):  # every cluster non-empty when possible
        if k[j] <= npix:
            labels[j, :k[j]] = np.arange(k[j])
    if mask_frac > 0:
        drop = g.random(npix) < mask_frac
        labels[:, drop] = -1
    if model_consistent:
        gp = _rng(cid, "points")
        per = [gp.uniform(1.3, 1.8, k[0]), gp.uniform(15.0, 25.0, k[1]), gp.uniform(-3.2, -2.8, k[2])]
        truth = np.stack([np.where(labels[j] >= 0, per[j][np.maximum(labels[j], 0)], X0[j]) for j in range(3)])
        x_true = np.concatenate(per)
    else:
        t = _rng(cid, "field_bd")
        truth = np.stack([t.normal(1.54, 0.1, npix), t.normal(20.0, 2.0, npix), t.normal(-3.0, 0.1, npix)])
        x_true = None
    truth = _clip_truth(truth)
    cmb, dust, sync = _amplitudes(cid, npix)
    signal = _signal(freqs, truth, cmb, dust, sync)
    if noiseless:
        d = np.repeat(signal[None], nitems, axis=0)
    else:
        d = signal[None] + np.stack([
            _rng(cid, "noise", r).standard_normal((2, nfreq, npix)) * sigma[None, :, None] for r in range(nitems)])
    gx = _rng(cid, "points", 1)
    xs = []
    for _ in range(nitems):
        xs.append(np.concatenate([gx.uniform(1.3, 1.8, k[0]), gx.uniform(15.0, 25.0, k[1]), gx.uniform(-3.2, -2.8, k[2])]))
    lo, hi = _box(nc)
    sky = Sky(cid, freqs, sigma, ninv, vecs, truth, signal, torch.from_numpy(d),
              torch.from_numpy(labels[None].copy()), np.tile(nc, (nitems, 1)), xs, [lo] * nitems, [hi] * nitems,
              meta=dict(workload="tiny", npix=npix, nfreq=nfreq, items=nitems))
    sky.meta["x_true"] = x_true
    return sky
