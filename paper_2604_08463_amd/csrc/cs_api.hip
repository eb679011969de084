// extern "C" entry points: descriptor validation, workspace layout, segment preparation,
// evaluation, optimiser, schedules, autotuning and kernel timing.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cs_internal.h"

namespace csi {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

cs_status hip_fail(hipError_t e, const char *what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return CS_E_HIP;
}

// h / k in kelvin per GHz (exact SI values of the Planck and Boltzmann constants)
constexpr double kHOverK = 6.62607015e-34 / 1.380649e-23 * 1.0e9;

// RJ -> CMB unit conversion g(nu) = (e^y - 1)^2 / (y^2 e^y), y = h nu / (k T_CMB)
static double rj_to_cmb(double nu_ghz, double tcmb) {
    const double y = kHOverK * nu_ghz / tcmb;
    const double em = std::expm1(y);
    return em * em / (y * y * std::exp(y));
}

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

static int bits_for(int64_t n) {
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

static void carve(cs_problem *p) {
    WsLayout &w = p->ws;
    const size_t B = (size_t)p->B, L = (size_t)p->L;
    w.p64 = (size_t)((p->P + kChunk - 1) / kChunk) * kChunk;
    w.nchunk_max = w.p64 / kChunk;
    size_t np2 = 2048;
    while (np2 < (size_t)p->P) np2 <<= 1;
    w.np2 = np2;
    w.keys_stride = np2;
    for (int j = 0; j < 3; ++j) {
        int32_t km = 1;
        for (int b = 0; b < p->B; ++b) km = std::max(km, p->ncl[3 * b + j]);
        w.kmax[j] = (size_t)km;
    }
    const size_t elem = (p->prec == CS_FP64) ? 8 : 4;
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t r = off;
        off += al256(std::max<size_t>(n, 1));
        return r;
    };
    w.band = take(sizeof(BandDev));
    w.items = take(sizeof(ItemDev) * B + sizeof(int64_t) * (B + 1));
    w.layouts = take(sizeof(LayoutDev) * L);
    w.units = take(sizeof(int2) * B * w.nchunk_max);
    w.keys = take(sizeof(uint64_t) * np2 * L);
    w.order = take(sizeof(int32_t) * w.p64 * L);
    w.head = take(sizeof(uint64_t) * w.nchunk_max * L);
    w.seg_base = take(sizeof(int32_t) * (w.nchunk_max + 1) * L);
    w.seg_lab = take(sizeof(int4) * (w.p64 * L + kSegLabPad));
    w.seg_perm = take(sizeof(int32_t) * w.p64 * 3 * L);
    w.seg_off = take(sizeof(int32_t) * (w.kmax[0] + w.kmax[1] + w.kmax[2] + 3) * L);
    w.counts = take(sizeof(int32_t) * 4 * L);
    w.excl = take(sizeof(int32_t) * (size_t)p->P * L);
    w.dpack = take(elem * 2 * (size_t)p->F * kChunk * w.nchunk_max * B);
    w.wpack = take(p->nmode == CS_NINV_PIXEL ? elem * 2 * (size_t)p->F * kChunk * w.nchunk_max * B : 0);
    w.tables = take(sizeof(double) * (size_t)p->F * (size_t)p->taboff[p->B]);
    w.partials = take(sizeof(double) * 4 * w.p64 * B);
    w.segoff = take(sizeof(int64_t) * (B + 1));
    w.istatus = take(sizeof(int32_t) * B);
    w.total = off;
}

static void fill_band(const cs_problem *p, BandDev &b) {
    std::memset(&b, 0, sizeof b);
    const double g0d = rj_to_cmb(p->nu0d, p->tcmb), g0s = rj_to_cmb(p->nu0s, p->tcmb);
    for (int f = 0; f < p->F; ++f) {
        const double nu = p->freqs[f];
        const double gn = rj_to_cmb(nu, p->tcmb);
        for (int s = 0; s < 2; ++s) b.w[s][f] = p->nmode == CS_NINV_BAND ? p->ninv_band[s * p->F + f] : 0.0;
        b.ld[f] = std::log(nu / p->nu0d);
        b.ls[f] = std::log(nu / p->nu0s);
        b.rd[f] = (nu / p->nu0d) * gn / g0d;
        b.gs[f] = gn / g0s;
        b.hk[f] = kHOverK * nu;
        for (int s = 0; s < 2; ++s) b.wf[s][f] = (float)b.w[s][f];
        b.ldf[f] = (float)b.ld[f];
        b.lsf[f] = (float)b.ls[f];
        b.bcd[f][0] = b.w[0][f];
        b.bcd[f][1] = b.ld[f];
        b.bcd[f][2] = b.ls[f];
        b.bcf[f][0] = b.wf[0][f];
        b.bcf[f][1] = b.ldf[f];
        b.bcf[f][2] = b.lsf[f];
    }
    b.hk0d = kHOverK * p->nu0d;
    for (int s = 0; s < 2; ++s) {
        double t = 0.0;
        float tf = 0.0f;
        for (int f = 0; f < p->F; ++f) {
            t += b.w[s][f];
            tf += b.wf[s][f];
        }
        b.wsum[s] = t;
        b.wsumf[s] = tf;
        b.isw[s] = 1.0 / std::sqrt(t);
        b.iswf[s] = 1.0 / std::sqrt((double)(float)t);
    }
}

}  // namespace csi

using namespace csi;

extern "C" {

const char *cs_last_error(void) { return g_error.c_str(); }

const char *cs_status_str(cs_status s) {
    switch (s) {
        case CS_OK: return "ok";
        case CS_E_INVALID: return "invalid argument";
        case CS_E_LABEL: return "invalid cluster label";
        case CS_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case CS_E_HIP: return "HIP runtime error";
        case CS_E_UNSUPPORTED: return "unsupported shape";
        case CS_E_STATE: return "call out of order";
    }
    return "unknown status";
}

static cs_status invalid(const char *msg) {
    set_error(msg);
    return CS_E_INVALID;
}

cs_status cs_problem_create(const cs_problem_desc *d, cs_problem **out) {
    if (!d || !out) return invalid("null descriptor or output");
    *out = nullptr;
    if (d->nfreq < 1) return invalid("nfreq must be >= 1");
    if (d->nfreq > kFMax) {
        set_error("nfreq > 32 is not supported by the register tile");
        return CS_E_UNSUPPORTED;
    }
    if (d->npix < 1 || d->nitems < 1) return invalid("npix and nitems must be >= 1");
    if (!d->freqs_ghz || !d->d || !d->labels || !d->nclusters) return invalid("null array in descriptor");
    for (int f = 0; f < d->nfreq; ++f)
        if (!(d->freqs_ghz[f] > 0.0) || !std::isfinite(d->freqs_ghz[f])) return invalid("band centres must be > 0");
    if (!(d->nu0_dust_ghz > 0) || !(d->nu0_sync_ghz > 0) || !(d->tcmb_k > 0)) return invalid("nu0 and T_CMB must be > 0");
    if (d->precision < CS_FP64 || d->precision > CS_FP32_STORE) return invalid("unknown precision");
    if (d->d_dtype != CS_DTYPE_F64 && d->d_dtype != CS_DTYPE_F32) return invalid("unknown d dtype");
    const int64_t fp2 = 2 * (int64_t)d->nfreq * d->npix;
    if (d->d_item_stride != 0 && d->d_item_stride < fp2) return invalid("d_item_stride must be 0 or >= 2 F P");
    if (d->labels_item_stride != 0 && d->labels_item_stride < 3 * (int64_t)d->npix)
        return invalid("labels_item_stride must be 0 or >= 3 P");
    if (d->ninv_mode == CS_NINV_BAND) {
        if (!d->ninv_band) return invalid("ninv_band is null");
        for (int i = 0; i < 2 * d->nfreq; ++i)
            if (!(d->ninv_band[i] > 0.0) || !std::isfinite(d->ninv_band[i])) return invalid("ninv_band must be > 0");
    } else if (d->ninv_mode == CS_NINV_PIXEL) {
        if (!d->ninv_pixel) return invalid("ninv_pixel is null");
        if (d->ninv_item_stride != 0 && d->ninv_item_stride < fp2) return invalid("ninv_item_stride must be 0 or >= 2 F P");
    } else {
        return invalid("unknown ninv mode");
    }
    for (int b = 0; b < d->nitems; ++b)
        for (int j = 0; j < 3; ++j) {
            const int32_t k = d->nclusters[3 * b + j];
            if (k < 1 || k > (1 << 28)) return invalid("cluster counts must be in [1, 2^28]");
            if (d->labels_item_stride == 0 && k != d->nclusters[j])
                return invalid("shared labels need equal cluster counts for all items");
        }

    cs_problem *p = new cs_problem();
    p->F = d->nfreq;
    p->P = d->npix;
    p->B = d->nitems;
    p->nu0d = d->nu0_dust_ghz;
    p->nu0s = d->nu0_sync_ghz;
    p->tcmb = d->tcmb_k;
    p->prec = d->precision;
    p->dtype = d->d_dtype;
    p->d = d->d;
    p->d_stride = d->d_item_stride;
    p->nmode = d->ninv_mode;
    if (p->nmode == CS_NINV_BAND) p->ninv_band.assign(d->ninv_band, d->ninv_band + 2 * d->nfreq);
    p->ninv_pixel = d->ninv_pixel;
    p->ninv_stride = d->ninv_item_stride;
    p->labels = d->labels;
    p->labels_stride = d->labels_item_stride;
    p->freqs.assign(d->freqs_ghz, d->freqs_ghz + d->nfreq);
    p->ncl.assign(d->nclusters, d->nclusters + 3 * (size_t)d->nitems);
    p->shared_qu = true;
    if (p->nmode == CS_NINV_BAND)
        for (int f = 0; f < p->F; ++f)
            if (p->ninv_band[f] != p->ninv_band[p->F + f]) p->shared_qu = false;
    p->L = d->labels_item_stride == 0 ? 1 : p->B;
    p->xoff.assign(p->B + 1, 0);
    p->taboff.assign(p->B + 1, 0);
    for (int b = 0; b < p->B; ++b) {
        const int64_t kd = p->ncl[3 * b], kt = p->ncl[3 * b + 1], ks = p->ncl[3 * b + 2];
        p->xoff[b + 1] = p->xoff[b] + kd + kt + ks;
        p->kmax_item = std::max<int64_t>(p->kmax_item, kd + kt + ks);
        p->taboff[b + 1] = p->taboff[b] + kd + 2 * kt + ks;
        p->trows_max = std::max<int64_t>(p->trows_max, kd + 2 * kt + ks);
    }
    carve(p);
    const int bits = bits_for((int64_t)p->ws.kmax[0]) + bits_for((int64_t)p->ws.kmax[1]) +
                     bits_for((int64_t)p->ws.kmax[2]) + bits_for(p->P);
    if (bits > 63) {
        delete p;
        set_error("cluster counts and pixel count exceed the 63-bit sort key");
        return CS_E_UNSUPPORTED;
    }
    if (hipGetDevice(&p->device) != hipSuccess) p->device = 0;
    *out = p;
    return CS_OK;
}

cs_status cs_problem_param_offsets(const cs_problem *p, int64_t *host_off) {
    if (!p || !host_off) return invalid("null argument");
    std::memcpy(host_off, p->xoff.data(), sizeof(int64_t) * (p->B + 1));
    return CS_OK;
}

cs_status cs_problem_workspace_bytes(const cs_problem *p, size_t *bytes) {
    if (!p || !bytes) return invalid("null argument");
    *bytes = p->ws.total;
    return CS_OK;
}

cs_status cs_problem_prepare(cs_problem *p, void *workspace, size_t bytes, void *stream) {
    if (!p) return invalid("null problem");
    if (!workspace || ((uintptr_t)workspace & 255) || bytes < p->ws.total) {
        set_error("workspace must be non-null, 256-byte aligned and at least cs_problem_workspace_bytes");
        return CS_E_WORKSPACE;
    }
    hipStream_t s = (hipStream_t)stream;
    p->wsp = (char *)workspace;
    p->prepared = false;
    const WsLayout &w = p->ws;
    char *base = p->wsp;

    BandDev band;
    fill_band(p, band);
    p->layouts.assign(p->L, LayoutDev{});
    for (int l = 0; l < p->L; ++l) {
        LayoutDev &L = p->layouts[l];
        L.labels = p->labels + (int64_t)l * p->labels_stride;
        L.keys = (uint64_t *)(base + w.keys) + (size_t)l * w.keys_stride;
        L.order = (int32_t *)(base + w.order) + (size_t)l * w.p64;
        L.head = (uint64_t *)(base + w.head) + (size_t)l * w.nchunk_max;
        L.seg_base = (int32_t *)(base + w.seg_base) + (size_t)l * (w.nchunk_max + 1);
        L.seg_lab = (int4 *)(base + w.seg_lab) + (size_t)l * w.p64;
        int32_t *so = (int32_t *)(base + w.seg_off) + (size_t)l * (w.kmax[0] + w.kmax[1] + w.kmax[2] + 3);
        for (int j = 0; j < 3; ++j) {
            L.seg_perm[j] = (int32_t *)(base + w.seg_perm) + ((size_t)l * 3 + j) * w.p64;
            L.seg_off[j] = so;
            so += w.kmax[j] + 1;
            L.k[j] = p->ncl[3 * (size_t)l + j];
        }
        L.counts = (int32_t *)(base + w.counts) + 4 * (size_t)l;
        L.excl = (int32_t *)(base + w.excl) + (size_t)l * (size_t)p->P;
    }
    p->items.assign(p->B, ItemDev{});
    for (int b = 0; b < p->B; ++b) {
        ItemDev &it = p->items[b];
        it.layout = p->L == 1 ? 0 : b;
        for (int j = 0; j < 3; ++j) it.k[j] = p->ncl[3 * (size_t)b + j];
        it.xoff = p->xoff[b];
        it.dchunk0 = (int64_t)b * (int64_t)w.nchunk_max;
        it.tab_off = p->taboff[b];
        it.part_off = (int64_t)b * (int64_t)w.p64;
    }
    CSI_HIP(hipMemcpyAsync(base + w.band, &band, sizeof band, hipMemcpyHostToDevice, s));
    CSI_HIP(hipMemcpyAsync(base + w.items, p->items.data(), sizeof(ItemDev) * p->B, hipMemcpyHostToDevice, s));
    CSI_HIP(hipMemcpyAsync(base + w.items + sizeof(ItemDev) * p->B, p->xoff.data(), sizeof(int64_t) * (p->B + 1),
                           hipMemcpyHostToDevice, s));
    CSI_HIP(hipMemcpyAsync(base + w.layouts, p->layouts.data(), sizeof(LayoutDev) * p->L, hipMemcpyHostToDevice, s));
    cs_status st = prepare_layouts(p, s);
    if (st != CS_OK) return st;
    std::vector<int32_t> counts(4 * (size_t)p->L);
    CSI_HIP(hipMemcpyAsync(counts.data(), base + w.counts, sizeof(int32_t) * counts.size(), hipMemcpyDeviceToHost, s));
    CSI_HIP(hipStreamSynchronize(s));
    for (int l = 0; l < p->L; ++l)
        if (counts[4 * l + 2]) {
            set_error("label outside [0, K) or excluded for only some parameters (layout " + std::to_string(l) + ")");
            return CS_E_LABEL;
        }
    std::vector<int2> units;
    units.reserve((size_t)p->B * w.nchunk_max);
    for (int l = 0; l < p->L; ++l) {
        LayoutDev &L = p->layouts[l];
        L.n_incl = counts[4 * l];
        L.nseg = counts[4 * l + 1];
        L.nchunks = (L.n_incl + kChunk - 1) / kChunk;
    }
    for (int b = 0; b < p->B; ++b) {
        const LayoutDev &L = p->layouts[p->items[b].layout];
        for (int c = 0; c < L.nchunks; ++c) units.push_back(make_int2(b, c));
    }
    p->nunits = (int64_t)units.size();
    p->segoff.assign(p->B + 1, 0);
    for (int b = 0; b < p->B; ++b) p->segoff[b + 1] = p->segoff[b] + p->layouts[p->items[b].layout].nseg;
    CSI_HIP(hipMemcpyAsync(base + w.segoff, p->segoff.data(), sizeof(int64_t) * (p->B + 1), hipMemcpyHostToDevice, s));
    CSI_HIP(hipMemcpyAsync(base + w.layouts, p->layouts.data(), sizeof(LayoutDev) * p->L, hipMemcpyHostToDevice, s));
    if (!units.empty())
        CSI_HIP(hipMemcpyAsync(base + w.units, units.data(), sizeof(int2) * units.size(), hipMemcpyHostToDevice, s));
    st = pack_data(p, s);
    if (st != CS_OK) return st;
    CSI_HIP(hipStreamSynchronize(s));
    p->prepared = true;
    return CS_OK;
}

cs_status cs_problem_item_info(const cs_problem *p, int32_t item, int64_t *n_included, int64_t *n_segments) {
    if (!p || item < 0 || item >= p->B) return invalid("bad problem or item");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    const LayoutDev &L = p->layouts[p->items[item].layout];
    if (n_included) *n_included = L.n_incl;
    if (n_segments) *n_segments = L.nseg;
    return CS_OK;
}

cs_status cs_problem_segments(cs_problem *p, int32_t item, int32_t labeling, int32_t *perm, int32_t *offsets,
                              void *stream) {
    if (!p || item < 0 || item >= p->B || labeling < 0 || labeling > 2 || !perm || !offsets)
        return invalid("bad segments request");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    return export_segments(p, item, labeling, perm, offsets, (hipStream_t)stream);
}

static cs_status eval_common(cs_problem *p, const double *x, double *neg2logl, double *grad, double *cf,
                             int32_t *status, bool want_grad, void *stream) {
    if (!p || !x || !neg2logl || (want_grad && !grad)) return invalid("null argument");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    return launch_eval(p, x, nullptr, neg2logl, grad, cf, status, want_grad, p->prec, (hipStream_t)stream);
}

cs_status cs_likelihood(cs_problem *p, const double *x, double *neg2logl, int32_t *status, void *stream) {
    return eval_common(p, x, neg2logl, nullptr, nullptr, status, false, stream);
}

cs_status cs_likelihood_grad(cs_problem *p, const double *x, double *neg2logl, double *grad, double *cluster_f,
                             int32_t *status, void *stream) {
    return eval_common(p, x, neg2logl, grad, cluster_f, status, true, stream);
}

static cs_status maps_common(cs_problem *p, const double *x, double *maps, int64_t maps_item_stride, double *cmb_var,
                             int32_t *status, bool sorted, void *stream) {
    if (!p || !x) return invalid("null argument");
    if (maps_item_stride != 0 && maps_item_stride < 6 * (int64_t)p->P) return invalid("maps_item_stride must be 0 or >= 6 P");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    return launch_maps(p, x, maps, maps_item_stride ? maps_item_stride : 6 * (int64_t)p->P, cmb_var, status, sorted,
                       (hipStream_t)stream);
}

cs_status cs_component_maps(cs_problem *p, const double *x, double *maps, int64_t maps_item_stride,
                            double *cmb_var, int32_t *status, void *stream) {
    return maps_common(p, x, maps, maps_item_stride, cmb_var, status, false, stream);
}

cs_status cs_component_maps_sorted(cs_problem *p, const double *x, double *maps, int64_t maps_item_stride,
                                   double *cmb_var, int32_t *status, void *stream) {
    return maps_common(p, x, maps, maps_item_stride, cmb_var, status, true, stream);
}

cs_status cs_problem_pixel_order(cs_problem *p, int32_t item, int32_t *order, void *stream) {
    if (!p || item < 0 || item >= p->B || !order) return invalid("bad pixel-order request");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    const LayoutDev &L = p->layouts[p->items[item].layout];
    if (L.n_incl > 0)
        CSI_HIP(hipMemcpyAsync(order, L.order, sizeof(int32_t) * (size_t)L.n_incl, hipMemcpyDeviceToDevice,
                               (hipStream_t)stream));
    return CS_OK;
}

static cs_status kmeans_check(int64_t n, int32_t ntasks, const int32_t *k, int64_t *ktot) {
    if (n < 1 || n > INT32_MAX / 2 || ntasks < 1 || ntasks > 65535 || !k)
        return invalid("K-means needs 1 <= n <= 2^30, 1 <= ntasks <= 65535 and host k");
    int64_t t = 0;
    for (int32_t i = 0; i < ntasks; ++i) {
        if (k[i] < 1) return invalid("K-means cluster counts must be >= 1");
        t += k[i];
    }
    *ktot = t;
    return CS_OK;
}

cs_status cs_kmeans_workspace_bytes(int64_t n, int32_t ntasks, const int32_t *k, size_t *bytes) {
    int64_t ktot = 0;
    if (!bytes) return invalid("null argument");
    const cs_status st = kmeans_check(n, ntasks, k, &ktot);
    if (st != CS_OK) return st;
    *bytes = kmeans_bytes(n, ntasks, ktot);
    return CS_OK;
}

cs_status cs_kmeans_batch(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep, int64_t keep_stride,
                          const int32_t *k, const int32_t *init, int64_t init_stride, int32_t iters, int32_t *labels,
                          int64_t labels_stride, int32_t *keff, void *workspace, size_t bytes, void *stream) {
    int64_t ktot = 0;
    cs_status st = kmeans_check(n, ntasks, k, &ktot);
    if (st != CS_OK) return st;
    if (!vecs || !init || !labels || !keff) return invalid("null argument");
    if (iters < 0) return invalid("iters must be >= 0");
    int32_t kmax = 1;
    for (int32_t i = 0; i < ntasks; ++i) kmax = std::max(kmax, k[i]);
    if (keep_stride == 0) keep_stride = n;
    if (labels_stride == 0) labels_stride = n;
    if (init_stride == 0) init_stride = kmax;
    if (keep_stride < n || labels_stride < n || init_stride < kmax) return invalid("row strides too small");
    if (!workspace || ((uintptr_t)workspace & 255) || bytes < kmeans_bytes(n, ntasks, ktot)) {
        set_error("workspace must be non-null, 256-byte aligned and at least cs_kmeans_workspace_bytes");
        return CS_E_WORKSPACE;
    }
    return kmeans_batch(vecs, n, ntasks, keep, keep_stride, k, init, init_stride, iters, labels, labels_stride, keff,
                        workspace, (hipStream_t)stream);
}

cs_status cs_kmeans_batch_static(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep,
                                 int64_t keep_stride, const int32_t *k, const int32_t *init, int64_t init_stride,
                                 int32_t iters, int32_t *labels, int64_t labels_stride, int32_t *keff, void *stream) {
    int64_t ktot = 0;
    cs_status st = kmeans_check(n, ntasks, k, &ktot);
    if (st != CS_OK) return st;
    if (!vecs || !init || !labels || !keff) return invalid("null argument");
    if (iters < 0) return invalid("iters must be >= 0");
    int32_t kmax = 1;
    for (int32_t i = 0; i < ntasks; ++i) kmax = std::max(kmax, k[i]);
    if (keep_stride == 0) keep_stride = n;
    if (labels_stride == 0) labels_stride = n;
    if (init_stride == 0) init_stride = kmax;
    if (keep_stride < n || labels_stride < n || init_stride < kmax) return invalid("row strides too small");
    return kmeans_batch_static(vecs, n, ntasks, keep, keep_stride, k, init, init_stride, iters, labels, labels_stride,
                               keff, kmeans_bytes(n, ntasks, ktot), (hipStream_t)stream);
}

cs_status cs_optim_default_opts(cs_optim_opts *o) {
    if (!o) return invalid("null opts");
    o->m = 10;
    o->gtol_rel = 1e-8;
    o->max_iter = 1000;
    o->iters_per_graph = 8;
    o->max_backtracks = 30;
    o->c1 = 1e-4;
    o->fp64_polish = 1;
    o->solver = CS_SOLVER_LBFGS;
    o->lr = 0.01;
    o->beta1 = 0.9;
    o->beta2 = 0.999;
    o->eps = 1e-16;
    o->topk = 0.0;
    o->switch_rel = 1e-4;
    return CS_OK;
}

cs_status cs_optimizer_workspace_bytes(const cs_problem *p, int32_t m, size_t *bytes) {
    if (!p || !bytes || m < 1 || m > 32) return invalid("bad optimizer workspace query (m in 1..32)");
    *bytes = optimizer_bytes(p, m);
    return CS_OK;
}

cs_status cs_optimize_batch_run(cs_problem *p, const cs_optim_opts *o, const double *lower, const double *upper,
                                double *x, double *f, int32_t *iters, int32_t *status, int64_t *nevals,
                                void *opt_workspace, size_t opt_bytes, int32_t resume, int32_t max_replays,
                                int32_t *running, void *stream) {
    if (running) *running = 0;
    if (!p || !o || !lower || !upper || !x || !f || !iters || !status) return invalid("null argument");
    if (o->m < 1 || o->m > 32 || o->max_iter < 0 || o->iters_per_graph < 1 || o->iters_per_graph > 4096 ||
        o->max_backtracks < 0 || !(o->c1 > 0.0 && o->c1 < 1.0) || !(o->gtol_rel >= 0.0) ||
        !(o->switch_rel >= 0.0 && o->switch_rel < 1.0))
        return invalid("bad optimiser options");
    if (resume != 0 && resume != 1) return invalid("resume must be 0 or 1");
    if (max_replays < 0) return invalid("max_replays must be >= 0");
    if (o->solver != CS_SOLVER_LBFGS && o->solver != CS_SOLVER_ADATOPK) return invalid("unknown solver");
    if (o->solver == CS_SOLVER_ADATOPK &&
        (!(o->lr > 0.0) || !(o->beta1 >= 0.0 && o->beta1 < 1.0) || !(o->beta2 >= 0.0 && o->beta2 < 1.0) ||
         !(o->eps >= 0.0) || !(o->topk >= 0.0 && o->topk <= 1.0)))
        return invalid("bad AdaTopK options");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    if (!opt_workspace || ((uintptr_t)opt_workspace & 255)) {
        set_error("optimizer workspace must be non-null and 256-byte aligned");
        return CS_E_WORKSPACE;
    }
    return optimize(p, o, lower, upper, x, f, iters, status, nevals, opt_workspace, opt_bytes, resume, max_replays,
                    running, (hipStream_t)stream);
}

cs_status cs_optimize_batch(cs_problem *p, const cs_optim_opts *o, const double *lower, const double *upper,
                            double *x, double *f, int32_t *iters, int32_t *status, int64_t *nevals,
                            void *opt_workspace, size_t opt_bytes, void *stream) {
    return cs_optimize_batch_run(p, o, lower, upper, x, f, iters, status, nevals, opt_workspace, opt_bytes, 0, 0,
                                 nullptr, stream);
}

cs_status cs_item_range(int32_t rank, int32_t nranks, int32_t nitems, int32_t *begin, int32_t *end) {
    if (!begin || !end || nranks < 1 || rank < 0 || rank >= nranks || nitems < 0)
        return invalid("cs_item_range needs 0 <= rank < nranks and nitems >= 0");
    *begin = (int32_t)((int64_t)rank * nitems / nranks);
    *end = (int32_t)((int64_t)(rank + 1) * nitems / nranks);
    return CS_OK;
}

cs_status cs_problem_desc_slice(const cs_problem_desc *in, int32_t begin, int32_t end, cs_problem_desc *out) {
    if (!in || !out || begin < 0 || end <= begin || end > in->nitems) return invalid("bad item slice");
    const size_t elem = in->d_dtype == CS_DTYPE_F32 ? 4 : 8;
    cs_problem_desc d = *in;
    d.nitems = end - begin;
    d.d = (const char *)in->d + (size_t)begin * (size_t)in->d_item_stride * elem;
    if (in->ninv_mode == CS_NINV_PIXEL && in->ninv_pixel)
        d.ninv_pixel = (const char *)in->ninv_pixel + (size_t)begin * (size_t)in->ninv_item_stride * elem;
    d.labels = in->labels + (size_t)begin * (size_t)in->labels_item_stride;
    d.nclusters = in->nclusters + 3 * (size_t)begin;
    *out = d;
    return CS_OK;
}

cs_status cs_problem_get_schedule(const cs_problem *p, cs_schedule *s) {
    if (!p || !s) return invalid("null argument");
    *s = p->sched;
    return CS_OK;
}

cs_status cs_problem_set_schedule(cs_problem *p, const cs_schedule *s) {
    if (!p || !s) return invalid("null argument");
    const int w = s->waves_per_block;
    if (!(w == 1 || w == 2 || w == 4 || w == 8) || s->blocks_per_cu < 0 || s->blocks_per_cu > 64 ||
        (s->xcd_remap != 0 && s->xcd_remap != 1) || s->shared_segments < 0 || s->shared_segments > 2)
        return invalid("bad schedule");
    p->sched = *s;
    return CS_OK;
}

cs_status cs_problem_autotune(cs_problem *p, const double *x, double *neg2logl, double *grad, int32_t reps,
                              cs_schedule *best, void *stream) {
    if (!p || !x || !neg2logl || !grad || reps < 1) return invalid("bad autotune arguments");
    if (!p->prepared) {
        set_error("cs_problem_prepare has not completed");
        return CS_E_STATE;
    }
    hipStream_t s = (hipStream_t)stream;
    const cs_schedule keep = p->sched;
    const bool was_timing = p->timing;
    p->timing = false;
    const size_t K = (size_t)p->xoff[p->B];
    std::vector<double> ref(p->B), got(p->B), refg(K), gotg(K);
    hipEvent_t e0, e1;
    CSI_HIP(hipEventCreate(&e0));
    CSI_HIP(hipEventCreate(&e1));
    cs_status rc = launch_eval(p, x, nullptr, neg2logl, grad, nullptr, nullptr, true, p->prec, s);
    if (rc == CS_OK && (hipMemcpyAsync(ref.data(), neg2logl, sizeof(double) * p->B, hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipMemcpyAsync(refg.data(), grad, sizeof(double) * K, hipMemcpyDeviceToHost, s) != hipSuccess))
        rc = CS_E_HIP;
    if (rc == CS_OK && hipStreamSynchronize(s) != hipSuccess) rc = CS_E_HIP;
    cs_schedule bestsch = keep;
    std::vector<std::pair<float, cs_schedule>> cand;  // (time, schedule) of every agreeing schedule
    const int waves[4] = {1, 2, 4, 8};
    const int bpc[3] = {0, 2, 4};
    // tolerances across the rounding orders of the staging modes: F relative, and the gradient
    // normwise per item
    const double cross_tol = p->prec == CS_FP32_BULK ? 1e-6 : 1e-11;
    const double cross_gtol = p->prec == CS_FP32_BULK ? 1e-3 : 1e-8;
    // a candidate is kept only when F and the gradient of every item agree with the reference
    auto agrees = [&](bool same_arith) {
        if (same_arith)  // same arithmetic, work only moved between wavefronts: bit-identical
            return std::memcmp(got.data(), ref.data(), sizeof(double) * p->B) == 0 &&
                   std::memcmp(gotg.data(), refg.data(), sizeof(double) * K) == 0;
        for (int b = 0; b < p->B; ++b) {
            if (!(std::fabs(got[b] - ref[b]) <= cross_tol * std::fabs(ref[b]))) return false;
            double gm = 0.0, dm = 0.0;
            for (int64_t i = p->xoff[b]; i < p->xoff[b + 1]; ++i) {
                gm = std::max(gm, std::fabs(refg[i]));
                const double dv = std::fabs(gotg[i] - refg[i]);
                if (!(dv == dv)) return false;  // NaN
                dm = std::max(dm, dv);
            }
            if (!(dm <= cross_gtol * gm)) return false;
        }
        return true;
    };
    // staging modes that run in this problem's precision (the segment-sum mode needs FP32
    // accumulation, else it runs as the per-pixel mode and is not timed twice)
    auto eff_mode = [&](int sh) {
        const cs_schedule was = p->sched;
        p->sched.shared_segments = sh;
        const int m = staging_mode(p, p->prec);
        p->sched = was;
        return m;
    };
    const int keep_mode = eff_mode(keep.shared_segments);
    for (int sh = 0; sh < 3 && rc == CS_OK; ++sh)
        for (int wi = 0; wi < 4 && rc == CS_OK && eff_mode(sh) == sh; ++wi)
            for (int bi = 0; bi < 3 && rc == CS_OK; ++bi)
                for (int xr = 0; xr < 2 && rc == CS_OK; ++xr) {
                    p->sched = cs_schedule{waves[wi], bpc[bi], xr, sh};
                    rc = launch_eval(p, x, nullptr, neg2logl, grad, nullptr, nullptr, true, p->prec, s);  // warm-up
                    if (rc != CS_OK) break;
                    if (hipEventRecord(e0, s) != hipSuccess) rc = CS_E_HIP;
                    for (int r = 0; r < reps && rc == CS_OK; ++r)
                        rc = launch_eval(p, x, nullptr, neg2logl, grad, nullptr, nullptr, true, p->prec, s);
                    if (rc != CS_OK) break;
                    float ms = 0.f;
                    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                        hipMemcpy(got.data(), neg2logl, sizeof(double) * p->B, hipMemcpyDeviceToHost) != hipSuccess ||
                        hipMemcpy(gotg.data(), grad, sizeof(double) * K, hipMemcpyDeviceToHost) != hipSuccess) {
                        rc = CS_E_HIP;
                        break;
                    }
                    if (agrees(sh == keep_mode)) cand.emplace_back(ms, p->sched);
                }
    // second stage: the four fastest re-timed in turn over three rounds with more repetitions, so
    // that one noisy timing does not decide
    if (rc == CS_OK && !cand.empty()) {
        std::stable_sort(cand.begin(), cand.end(), [](const auto &u, const auto &v) { return u.first < v.first; });
        const size_t ntop = std::min<size_t>(4, cand.size());
        std::vector<double> tot(ntop, 0.0);
        const int reps2 = std::max(reps, 5);
        for (int round = 0; round < 3 && rc == CS_OK; ++round)
            for (size_t c = 0; c < ntop && rc == CS_OK; ++c) {
                p->sched = cand[c].second;
                rc = launch_eval(p, x, nullptr, neg2logl, grad, nullptr, nullptr, true, p->prec, s);  // warm-up
                if (rc != CS_OK) break;
                if (hipEventRecord(e0, s) != hipSuccess) rc = CS_E_HIP;
                for (int r = 0; r < reps2 && rc == CS_OK; ++r)
                    rc = launch_eval(p, x, nullptr, neg2logl, grad, nullptr, nullptr, true, p->prec, s);
                if (rc != CS_OK) break;
                float ms = 0.f;
                if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                    rc = CS_E_HIP;
                    break;
                }
                tot[c] += ms;
            }
        size_t bi = 0;
        for (size_t c = 1; c < ntop; ++c)
            if (tot[c] < tot[bi]) bi = c;
        bestsch = cand[bi].second;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->sched = (rc == CS_OK) ? bestsch : keep;
    p->timing = was_timing;
    if (rc == CS_E_HIP) set_error("HIP error during autotuning");
    if (rc == CS_OK && best) *best = bestsch;
    return rc;
}

cs_status cs_problem_set_timing(cs_problem *p, int32_t enable) {
    if (!p) return invalid("null problem");
    p->timing = enable != 0;
    p->events_used = 0;
    return CS_OK;
}

cs_status cs_problem_kernel_time(cs_problem *p, double *total_ms, int64_t *launches) {
    if (!p || !total_ms) return invalid("null argument");
    double t = 0.0;
    if (p->events_used) CSI_HIP(hipEventSynchronize(p->events[p->events_used - 1].second));
    for (size_t i = 0; i < p->events_used; ++i) {
        float ms = 0.f;
        CSI_HIP(hipEventElapsedTime(&ms, p->events[i].first, p->events[i].second));
        t += ms;
    }
    *total_ms = t;
    if (launches) *launches = (int64_t)p->events_used;
    p->events_used = 0;
    return CS_OK;
}

void cs_problem_destroy(cs_problem *p) {
    if (!p) return;
    for (auto &e : p->events) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete p;
}

}  // extern "C"
