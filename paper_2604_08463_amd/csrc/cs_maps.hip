// Component maps and the CMB map variance at given spectral parameters.
//
// The generalised least-squares amplitudes of one pixel and Stokes parameter are
// s_hat = (A^T N^-1 A)^-1 A^T N^-1 d (paper Sec. 2.3, the reconstruction operator W applied to
// the data).  The CMB variance metric used to choose the number of clusters is the variance of
// the reconstructed CMB amplitude over the analysis mask, here the population variance of Q plus
// that of U (Sec. 2.4, eq. min_var).
//
//   k_fill_excl per (item, excluded pixel): NaN in the six maps at the pixel (pixel order), or at
//               the slots past the included pixels (processing order)
//   k_maps_stage one wavefront per 64-pixel chunk (band weights shared by Q and U): the chunk's
//               SED columns staged in LDS, FP64 normal equations from the stored data streamed
//               through a ring of loads, Cholesky, s_hat written in the caller's pixel order
//               (scattered 8-byte writes when the pixel numbering is not spatial) or in
//               processing order (coalesced), and the chunk's (count, mean, centred sum of
//               squares) of the Q and U CMB amplitudes
//   k_maps      the same with per-lane table gathers (separate Q/U or per-pixel weights)
//   k_maps_var  one workgroup per item: pairwise combination of the chunk moments
//               (Chan, Golub & LeVeque's update), variance and status word
#include <algorithm>

#include "cs_device.h"

namespace csi {

namespace {

constexpr int kMapWaves = 4;
constexpr int kVarThreads = 256;

struct Moments {  // count, then (mean, centred sum of squares) of Q and of U
    double n, mq, sq, mu, su;
};

__device__ __forceinline__ Moments combine(const Moments &a, const Moments &b) {
    if (b.n == 0.0) return a;
    if (a.n == 0.0) return b;
    Moments r;
    r.n = a.n + b.n;
    const double fb = b.n / r.n, fab = a.n * b.n / r.n;
    const double dq = b.mq - a.mq, du = b.mu - a.mu;
    r.mq = a.mq + dq * fb;
    r.sq = a.sq + b.sq + dq * dq * fab;
    r.mu = a.mu + du * fb;
    r.su = a.su + b.su + du * du * fab;
    return r;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// grid (excluded-pixel blocks, item): the P - n_included excluded pixels of the item (pixel order)
// or the slots n_included .. P - 1 (processing order) get NaN in all six maps
__global__ __launch_bounds__(256) void k_fill_excl(const EvalArgs a, double *maps, int64_t stride, int32_t npix,
                                                   int sorted) {
    const int item = blockIdx.y;
    const cptr<LayoutDev> L = as_const(a.layouts) + (as_const(a.items) + item)->layout;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t n_incl = L->n_incl;
    if (e >= (int64_t)npix - n_incl) return;
    const int64_t pos = sorted ? n_incl + e : as_global(L->excl)[e];
    double *o = maps + (int64_t)item * stride + pos;
#pragma unroll
    for (int c = 0; c < 6; ++c) o[(int64_t)c * npix] = __builtin_nan("");
}

// s_hat of the chunk's pixels written, NaN and the status bit at a non-positive-definite pixel,
// and the chunk's moments of the CMB amplitude (NaN propagates from such a pixel)
__device__ __forceinline__ void map_epilogue(const EvalArgs &a, const cptr<ItemDev> it, const cptr<LayoutDev> L,
                                             const int item, const int chunk, const int lane, const int nvalid,
                                             double sh[2][3], const bool ok, double *maps, const int64_t stride,
                                             const int32_t npix, const int sorted) {
    const bool valid = lane < nvalid;
    if (!ok)
        for (int s = 0; s < 2; ++s)
            for (int c = 0; c < 3; ++c) sh[s][c] = __builtin_nan("");
    if (__ballot(valid && !ok) && lane == 0) atomicOr(&a.istatus[item], (int)CS_ITEM_NOT_PD);

    if (maps && valid) {
        const int32_t slot = chunk * kChunk + lane;
        const int32_t pix = sorted ? slot : L->order[slot];
        double *o = maps + (int64_t)item * stride + pix;
        for (int s = 0; s < 2; ++s)
            for (int c = 0; c < 3; ++c) o[(int64_t)(3 * s + c) * npix] = sh[s][c];
    }

    const double n = (double)nvalid;
    const double vq = valid ? sh[0][0] : 0.0, vu = valid ? sh[1][0] : 0.0;
    const double mq = wave_sum(vq) / n, mu = wave_sum(vu) / n;
    const double eq = valid ? vq - mq : 0.0, eu = valid ? vu - mu : 0.0;
    const double sq = wave_sum(eq * eq), su = wave_sum(eu * eu);
    if (lane == 0) {
        double *st = a.partials + it->part_off * 4 + (int64_t)chunk * 8;
        st[0] = n;
        st[1] = mq;
        st[2] = sq;
        st[3] = mu;
        st[4] = su;
    }
}

// FP64 Cholesky of one pixel's M (upper triangle m00, m01, m02, m11, m12, m22) and the solve for
// one Stokes parameter's b; ok is false unless the leading minors are positive relative to the
// products of the diagonal entries
__device__ __forceinline__ void chol_solve(const double *c, const double *b, double *sh, bool &ok) {
    const double l00 = sqrt(c[0]);
    const double l10 = c[1] / l00, l20 = c[2] / l00;
    const double p1 = c[3] - l10 * l10;
    const double l11 = sqrt(p1);
    const double l21 = (c[4] - l20 * l10) / l11;
    const double p2 = c[5] - l20 * l20 - l21 * l21;
    const double l22 = sqrt(p2);
    ok = ok && c[0] > 0.0 && p1 > 1e-12 * c[3] && p1 * p2 > 1e-12 * c[3] * c[5];  // relative minors
    const double z0 = b[0] / l00;
    const double z1 = (b[1] - l10 * z0) / l11;
    const double z2 = (b[2] - l20 * z0 - l21 * z1) / l22;
    sh[2] = z2 / l22;
    sh[1] = (z1 - l21 * sh[2]) / l11;
    sh[0] = (z0 - l10 * sh[1] - l20 * sh[2]) / l00;
}

// Direct-gather form: every lane gathers its segment's table values per band.  For separate Q/U
// (wm = 1) or per-pixel (wm = 2) weights, and for chunks with more segments than the staged
// kernel holds.
template <typename TS>
__device__ __forceinline__ void map_unit_direct(const EvalArgs &a, const int wm, double *maps, const int64_t stride,
                                                const int32_t npix, const int sorted, const int item, const int chunk,
                                                const int lane) {
    const int F = a.nfreq;
    const cptr<ItemDev> it = as_const(a.items) + item;
    const cptr<LayoutDev> L = as_const(a.layouts) + it->layout;
    const uint64_t head = as_const(L->head)[chunk];
    const int segbase = as_const(L->seg_base)[chunk];
    const int nvalid = min(L->n_incl - chunk * kChunk, kChunk);
    const int seg = segbase + __popcll(head & lanemask_le(lane)) - 1;
    const gptr<int> lab = as_global((const int *)L->seg_lab) + 4 * (int64_t)seg;
    const int64_t kd = it->k[0], kt = it->k[1];
    const gptr<double> tab = as_global((const double *)a.tables) + it->tab_off * (int64_t)F;
    const gptr<double> pd = tab + (int64_t)lab[0] * F;
    const gptr<double> bt = tab + (kd + 2 * (int64_t)lab[1]) * F;
    const gptr<double> ss = tab + (kd + 2 * kt + lab[2]) * F;
    const int64_t cbase = (it->dchunk0 + chunk) * (2 * (int64_t)F * kChunk) + lane;
    const gptr<TS> dq = as_global((const TS *)a.dpack) + cbase;
    const gptr<TS> wq = (wm == 2) ? as_global((const TS *)a.wpack) + cbase : nullptr;
    const cptr<BandDev> B = as_const(a.band);

    // normal equations per Stokes parameter: M (upper triangle) and b, in FP64
    double m[2][6], b[2][3];
    for (int s = 0; s < 2; ++s) {
        for (int i = 0; i < 6; ++i) m[s][i] = 0.0;
        for (int i = 0; i < 3; ++i) b[s][i] = 0.0;
    }
    // bands four at a time, so that their gathers and data loads are in flight together; with
    // band weights shared by Q and U (wm == 0) the U sums of M equal the Q sums and are copied
#pragma unroll 4
    for (int f = 0; f < F; ++f) {
        const double ad = pd[f] * bt[2 * f], as = ss[f];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int64_t o = ((int64_t)s * F + f) * kChunk;
            const double w = (wm == 2) ? (double)wq[o] : B->w[s][f];
            const double dv = (double)ld_stream(dq + o);
            const double wad = w * ad, was = w * as;
            if (wm != 0 || s == 0) {
                m[s][0] += w;
                m[s][1] += wad;
                m[s][2] += was;
                m[s][3] += wad * ad;
                m[s][4] += wad * as;
                m[s][5] += was * as;
            }
            b[s][0] += w * dv;
            b[s][1] += wad * dv;
            b[s][2] += was * dv;
        }
    }
    if (wm == 0)
        for (int i = 0; i < 6; ++i) m[1][i] = m[0][i];
    double sh[2][3];
    bool ok = true;
    for (int s = 0; s < 2; ++s) chol_solve(m[s], b[s], sh[s], ok);
    map_epilogue(a, it, L, item, chunk, lane, nvalid, sh, ok, maps, stride, npix, sorted);
}

template <typename TS>
__global__ __launch_bounds__(64 * kMapWaves) void k_maps(const EvalArgs a, const int wm, double *maps,
                                                          const int64_t stride, const int32_t npix, const int sorted) {
    const int lane = threadIdx.x & 63;
    const int64_t u = (int64_t)blockIdx.x * kMapWaves + (threadIdx.x >> 6);
    if (u >= a.nunits) return;
    const int item = __builtin_amdgcn_readfirstlane(a.units[u].x);
    const int chunk = __builtin_amdgcn_readfirstlane(a.units[u].y);
    map_unit_direct<TS>(a, wm, maps, stride, npix, sorted, item, chunk, lane);
}

// Staged form (band weights shared by Q and U): the wavefront first requests a ring of data
// loads, then stages (a_d, a_s) of every (segment, band) of its chunk in its LDS slice; each
// lane then forms M and b of its pixel from LDS and the streamed data, and one Cholesky factor
// serves both Stokes parameters (their weights, hence M, are equal).
constexpr int kMapStageSeg = 12;
#ifndef CS_MAP_RING
#define CS_MAP_RING 5
#endif
constexpr int kMapRing = CS_MAP_RING;  // groups of two bands requested ahead (5 measured best of 4, 5, 8, 11)

template <typename TS>
__global__ __launch_bounds__(64 * kMapWaves) void k_maps_stage(const EvalArgs a, double *maps, const int64_t stride,
                                                               const int32_t npix, const int sorted) {
    extern __shared__ char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t u = (int64_t)blockIdx.x * kMapWaves + wave;
    if (u >= a.nunits) return;
    const int item = __builtin_amdgcn_readfirstlane(a.units[u].x);
    const int chunk = __builtin_amdgcn_readfirstlane(a.units[u].y);
    const int F = a.nfreq;
    const cptr<ItemDev> it = as_const(a.items) + item;
    const cptr<LayoutDev> L = as_const(a.layouts) + it->layout;
    const int segbase = as_const(L->seg_base)[chunk];
    const int nseg = as_const(L->seg_base)[chunk + 1] - segbase;
    if (nseg > kMapStageSeg) {
        map_unit_direct<TS>(a, 0, maps, stride, npix, sorted, item, chunk, lane);
        return;
    }
    const uint64_t head = as_const(L->head)[chunk];
    const int nvalid = min(L->n_incl - chunk * kChunk, kChunk);
    const int segl = __popcll(head & lanemask_le(lane)) - 1;
    const int64_t cbase = (it->dchunk0 + chunk) * (2 * (int64_t)F * kChunk) + lane;
    const gptr<TS> dq = as_global((const TS *)a.dpack) + cbase;
    const gptr<TS> du = dq + (int64_t)F * kChunk;
    const cptr<BandDev> B = as_const(a.band);

    TS rq[kMapRing][2], ru[kMapRing][2];
#pragma unroll
    for (int r = 0; r < kMapRing; ++r)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int f0 = 2 * r + j;
            const int f = f0 < F ? f0 : F - 1;
            rq[r][j] = ld_stream(dq + f * kChunk);
            ru[r][j] = ld_stream(du + f * kChunk);
        }

    // (a_d, a_s) of every (segment, band) pair, one pair per lane per round
    double2 *cols = (double2 *)(smem + (size_t)wave * kMapStageSeg * F * sizeof(double2));
    {
        const int64_t kd = it->k[0], kt = it->k[1];
        const gptr<double> tab = as_global((const double *)a.tables) + it->tab_off * (int64_t)F;
        const gptr<int> sl = as_global((const int *)L->seg_lab) + 4 * (int64_t)segbase;
        const int ne = nseg * F;
        for (int e = lane; e < ne; e += kChunk) {
            const int sg = e / F, f = e - sg * F;
            const int l0 = sl[4 * sg], l1 = sl[4 * sg + 1], l2 = sl[4 * sg + 2];
            const double pd = tab[(int64_t)l0 * F + f], bt = tab[(kd + 2 * (int64_t)l1) * F + 2 * f],
                         ss = tab[(kd + 2 * kt + l2) * F + f];
            cols[e] = double2{pd * bt, ss};
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const double2 *my = cols + segl * F;
    double c[6] = {B->wsum[0], 0.0, 0.0, 0.0, 0.0, 0.0};
    double b[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    auto band = [&](const int f, const double q, const double v) {
        const double2 col = my[f];
        const double w = B->w[0][f];
        const double wad = w * col.x, was = w * col.y;
        c[1] += wad;
        c[2] += was;
        c[3] += wad * col.x;
        c[4] += wad * col.y;
        c[5] += was * col.y;
        b[0][0] += w * q;
        b[0][1] += wad * q;
        b[0][2] += was * q;
        b[1][0] += w * v;
        b[1][1] += wad * v;
        b[1][2] += was * v;
    };
    // consume ring slot r, then refill it kMapRing groups ahead
    for (int g0 = 0; g0 < F; g0 += 2 * kMapRing) {
#pragma unroll
        for (int r = 0; r < kMapRing; ++r) {
            const int fb = g0 + 2 * r;
#pragma unroll
            for (int j = 0; j < 2; ++j)
                if (fb + j < F) band(fb + j, (double)rq[r][j], (double)ru[r][j]);
            if (fb + 2 * kMapRing < F) {
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int f0 = fb + 2 * kMapRing + j;
                    const int f = f0 < F ? f0 : F - 1;
                    rq[r][j] = ld_stream(dq + f * kChunk);
                    ru[r][j] = ld_stream(du + f * kChunk);
                }
            }
        }
    }
    double sh[2][3];
    bool ok = true;
    chol_solve(c, b[0], sh[0], ok);
    chol_solve(c, b[1], sh[1], ok);
    map_epilogue(a, it, L, item, chunk, lane, nvalid, sh, ok, maps, stride, npix, sorted);
}

__global__ __launch_bounds__(kVarThreads) void k_maps_var(const EvalArgs a, double *cmb_var, int32_t *status) {
    const int item = blockIdx.x;
    const ItemDev &it = a.items[item];
    const LayoutDev &L = a.layouts[it.layout];
    const int64_t nc = L.nchunks;
    const double *st = a.partials + it.part_off * 4;
    // thread t folds the contiguous chunk range [t nc / T, (t + 1) nc / T) in order
    const int t = threadIdx.x;
    Moments acc{0.0, 0.0, 0.0, 0.0, 0.0};
    for (int64_t c = t * nc / kVarThreads; c < (t + 1) * nc / kVarThreads; ++c) {
        const double *r = st + c * 8;
        acc = combine(acc, Moments{r[0], r[1], r[2], r[3], r[4]});
    }
    __shared__ Moments sm[kVarThreads];
    sm[t] = acc;
    __syncthreads();
    for (int h = kVarThreads / 2; h > 0; h >>= 1) {
        if (t < h) sm[t] = combine(sm[t], sm[t + h]);
        __syncthreads();
    }
    if (t == 0) {
        int s = a.istatus[item];
        const Moments r = sm[0];
        double v = r.n > 0.0 ? r.sq / r.n + r.su / r.n : __builtin_nan("");
        if (s & CS_ITEM_NOT_PD)
            v = __builtin_nan("");
        else if (!isfinite(v) && r.n > 0.0)
            s |= CS_ITEM_NONFINITE;
        if (cmb_var) cmb_var[item] = v;
        if (status) status[item] = s;
        a.istatus[item] = s;
    }
}

}  // namespace

cs_status launch_maps(cs_problem *p, const double *x, double *maps, int64_t maps_stride, double *cmb_var,
                      int32_t *status, bool sorted, hipStream_t s) {
    const EvalArgs a = make_eval_args(p, x, nullptr);
    cs_status st = launch_sed(p, a, false, s);  // FP64 tables (also resets the status words)
    if (st != CS_OK) return st;
    int64_t nexcl = 0;  // most excluded pixels of one item
    for (int b = 0; b < p->B; ++b)
        nexcl = std::max<int64_t>(nexcl, (int64_t)p->P - p->layouts[p->items[b].layout].n_incl);
    if (maps && nexcl > 0) {
        for (int b0 = 0; b0 < p->B; b0 += kMaxGridY) {
            const dim3 grid((unsigned)((nexcl + 255) / 256), (unsigned)std::min(kMaxGridY, p->B - b0));
            EvalArgs ab = a;
            ab.items = a.items + b0;
            hipLaunchKernelGGL(k_fill_excl, grid, dim3(256), 0, s, ab, maps + (int64_t)b0 * maps_stride, maps_stride,
                               p->P, (int)sorted);
            CSI_HIP(hipGetLastError());
        }
    }
    const int wm = p->nmode == CS_NINV_PIXEL ? 2 : (p->shared_qu ? 0 : 1);
    if (p->nunits > 0) {
        const dim3 grid((unsigned)((p->nunits + kMapWaves - 1) / kMapWaves)), block(64 * kMapWaves);
        const size_t lds = (size_t)kMapWaves * kMapStageSeg * p->F * sizeof(double2);
        if (wm == 0 && p->prec == CS_FP64)
            hipLaunchKernelGGL(k_maps_stage<double>, grid, block, lds, s, a, maps, maps_stride, p->P, (int)sorted);
        else if (wm == 0)
            hipLaunchKernelGGL(k_maps_stage<float>, grid, block, lds, s, a, maps, maps_stride, p->P, (int)sorted);
        else if (p->prec == CS_FP64)
            hipLaunchKernelGGL(k_maps<double>, grid, block, 0, s, a, wm, maps, maps_stride, p->P, (int)sorted);
        else
            hipLaunchKernelGGL(k_maps<float>, grid, block, 0, s, a, wm, maps, maps_stride, p->P, (int)sorted);
        CSI_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_maps_var, dim3(p->B), dim3(kVarThreads), 0, s, a, cmb_var, status);
    CSI_HIP(hipGetLastError());
    return CS_OK;
}

}  // namespace csi
