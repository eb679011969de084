// One batched evaluation of the spectral likelihood and its adjoint (paper Sec. 2.1, 3.3.1).
//
//   k_sed          per (item, cluster, band group): SED tables of the three spectral parameters (a2)
//   k_pixel_stage  per 64-pixel chunk (one wavefront): the chunk's SED columns staged in LDS, the
//                  mixing matrix per pixel (a3), frequency accumulation of A^T N^-1 A, A^T N^-1 d
//                  and the adjoint sums (a4), FP64 3x3 Cholesky (a5), per-pixel gradient (a6),
//                  run-segmented wave reduction (a7, first level); k_pixel is the direct-gather
//                  form for per-Stokes or per-pixel weights
//   k_fin_grad     per (item, cluster): compensated sum over the cluster's segments; per item:
//                  F over all its segments and the status word (a7)
//
// Gradient without a second pass over the data.  With r_s = N^-1 (d_s - A s_hat_s) and
// delta_k(nu) = dA/dtheta_k (only one column depends on theta_k),
//   sum_nu r_s(nu) delta_k(nu) = h_sk - sum_j s_hat_sj G_jk,
//   h_sk = sum_nu w d_s delta_k,   G_jk = sum_nu w a_j delta_k,
// so dF/dtheta_k = -2 sum_s s_hat_s,col(k) (h_sk - sum_j s_hat_sj G_jk).  Both sums are
// accumulated in the same single pass over frequency as M and b.
#include "cs_device.h"

#ifndef CS_WAVES_PER_EU
#define CS_WAVES_PER_EU 1
#endif
#ifndef CS_BAND_GROUP
#define CS_BAND_GROUP 2
#endif
#ifndef CS_SUMS_RING
#define CS_SUMS_RING 11
#endif
#ifndef CS_SUMS_WAVES
#define CS_SUMS_WAVES 5
#endif
#ifndef CS_STAGE0_WAVES
#define CS_STAGE0_WAVES 5
#endif
#ifndef CS_FP64_NOLOOP
#define CS_FP64_NOLOOP 1
#endif
#ifndef CS_FP64_RING
#define CS_FP64_RING 6
#endif

namespace csi {

// ---------------------------------------------------------------------------------------------
// band constants in the accumulation type
// ---------------------------------------------------------------------------------------------
template <typename TA>
struct Band;
template <>
struct Band<double> {
    static __device__ __forceinline__ double w(cptr<BandDev> b, int s, int f) { return b->w[s][f]; }
    static __device__ __forceinline__ double ld(cptr<BandDev> b, int f) { return b->ld[f]; }
    static __device__ __forceinline__ double ls(cptr<BandDev> b, int f) { return b->ls[f]; }
    static __device__ __forceinline__ double wsum(cptr<BandDev> b, int s) { return b->wsum[s]; }
    static __device__ __forceinline__ double isw(cptr<BandDev> b, int s) { return b->isw[s]; }
};
template <>
struct Band<float> {
    static __device__ __forceinline__ float w(cptr<BandDev> b, int s, int f) { return b->wf[s][f]; }
    static __device__ __forceinline__ float ld(cptr<BandDev> b, int f) { return b->ldf[f]; }
    static __device__ __forceinline__ float ls(cptr<BandDev> b, int f) { return b->lsf[f]; }
    static __device__ __forceinline__ float wsum(cptr<BandDev> b, int s) { return b->wsum[s]; }
    static __device__ __forceinline__ double isw(cptr<BandDev> b, int s) { return b->iswf[s]; }
};

// ---------------------------------------------------------------------------------------------
// a2: SED tables.  Rows of an item: PD[K_d][F] = (nu/nu0d)^beta_d;
// BTDT[K_T][F][2] = ((nu/nu0d) expm1(x0)/expm1(x) g(nu)/g(nu0d),  d ln(.)/dT);
// SS[K_s][F] = (nu/nu0s)^beta_s g(nu)/g(nu0s).  The dust column is PD * BT (eq. mixing_columns).
// ---------------------------------------------------------------------------------------------
// Workgroup (nfb, 256 / nfb): x = band group of kSedBands consecutive bands, y = table row;
// grid x over an item's rows, y over items (from item0).  The item is uniform in a workgroup,
// so its descriptor comes through the scalar cache.
constexpr int kSedBands = 4;  // consecutive bands of one table row per thread
constexpr int kSedThreads = 256;

template <typename TT>
__global__ __launch_bounds__(kSedThreads) void k_sed(const EvalArgs a, const int64_t *xoff, int item0) {
    const int F = a.nfreq;
    const int item = item0 + (int)blockIdx.y;
    if (a.active && !as_const(a.active)[item]) return;
    const int64_t x0 = as_const(xoff)[item], kk = as_const(xoff)[item + 1] - x0;
    const int64_t r = (int64_t)blockIdx.x * blockDim.y + threadIdx.y;  // table row (parameter)
    if (r == 0 && threadIdx.x == 0) a.istatus[item] = 0;
    if (r >= kk) return;
    const int fa = (int)threadIdx.x * kSedBands;
    const int fb = fa + kSedBands < F ? fa + kSedBands : F;
    const cptr<ItemDev> it = as_const(a.items) + item;
    const cptr<BandDev> B = as_const(a.band);
    const double x = a.x[x0 + r];
    TT *tab = (TT *)a.tables + it->tab_off * (int64_t)F;
    const int64_t k0 = it->k[0], k1 = it->k[1];
    if (r < k0) {
        for (int f = fa; f < fb; ++f) tab[r * F + f] = (TT)exp(x * B->ld[f]);
    } else if (r < k0 + k1) {
        TT *o = tab + (k0 + 2 * (r - k0)) * F;
        const double xd = B->hk0d / x;
        const double e0 = expm1(xd), q0 = xd / (-expm1(-xd));
        for (int f = fa; f < fb; ++f) {
            const double xf = B->hk[f] / x;
            o[2 * f] = (TT)(B->rd[f] * e0 / expm1(xf));
            o[2 * f + 1] = (TT)((xf / (-expm1(-xf)) - q0) / x);
        }
    } else {
        const int64_t ks = r - k0 - k1;
        for (int f = fa; f < fb; ++f) tab[(k0 + 2 * k1 + ks) * F + f] = (TT)(exp(x * B->ls[f]) * B->gs[f]);
    }
}

// Positive definiteness of M = A^T N^-1 A from its Cholesky pivots m00, p1, p2: the leading
// principal minors m00, m00 p1 and m00 p1 p2 must be positive relative to the products of their
// diagonal entries (p1 / m11 and p1 p2 / (m11 m22) above a tolerance of the accumulation
// precision), so that a rank-deficient M is flagged whatever sign rounding gives its last pivot.
// 1 / sqrt(p) of a Cholesky pivot.  FP64 accumulation: correctly rounded.  FP32 accumulation,
// whose M already carries FP32 rounding: the hardware reciprocal square root (relative error
// below 2^-22) refined by one Newton step to a relative error of about 1e-13, at a quarter of
// the instructions of a rounded square root and division.  A pivot that is zero, negative or
// not finite gives inf or NaN either way and fails the positive-definiteness test.
template <typename TA>
__device__ __forceinline__ double inv_sqrt(double p) {
    if constexpr (sizeof(TA) == 8) {
        return 1.0 / sqrt(p);
    } else {
        const double y = __builtin_amdgcn_rsq(p);
        const double r = fma(-p * y, y, 1.0);  // 1 - p y^2
        return fma(0.5 * y, r, y);
    }
}

template <typename TA>
__device__ __forceinline__ bool pd_pivots(double m00, double m11, double m22, double p1, double p2) {
    constexpr double kTau = sizeof(TA) == 4 ? 1e-6 : 1e-12;
    return m00 > 0.0 && p1 > kTau * m11 && p1 * p2 > kTau * m11 * m22;
}

// ---------------------------------------------------------------------------------------------
// a3-a7 (first level): the per-pixel kernel
// ---------------------------------------------------------------------------------------------
template <typename TA>
struct WAcc {  // accumulators of one weight set: M (upper triangle) and G_jk
    TA m00, m01, m02, m11, m12, m22;
    TA g01, g02, g03, g11, g12, g13, g21, g22, g23;
};
template <typename TA>
struct SAcc {  // accumulators of one Stokes parameter: b and h
    TA b0, b1, b2, h1, h2, h3;
};

// Band loop of one pixel: calls band(f, d_Q, d_U, PD, BT, DT, SS) for f = 0..F-1.
// FM > 0 (compile-time band count): the pixel's whole Q/U data column is requested first (one
// HBM round trip per wavefront), then the SED-table gathers run one group of kG bands ahead of
// the arithmetic.  Vector-memory loads retire in order, so a wait for a gather never waits for
// a data load issued after it.  Scheduling barriers keep the compiler from hoisting the later
// gathers to the top.  FM == 0 (any F): groups of kG bands with the next group's data prefetched
// behind the current group's gathers.  Bands past F read a clamped address and are not used.
template <int FM, int kG, typename TS, typename TA, typename BandFn>
__device__ __forceinline__ void band_loop(const int F, const gptr<TS> dq, const gptr<TS> du, const gptr<TA> pd,
                                          const gptr<TA> bt, const gptr<TA> ss, BandFn &&band) {
    if constexpr (FM > 0) {
        constexpr int NG = (FM + kG - 1) / kG;
        TS vq[FM], vu[FM];
#pragma unroll
        for (int f = 0; f < FM; ++f) {
            vq[f] = ld_stream(dq + f * kChunk);
            vu[f] = ld_stream(du + f * kChunk);
        }
        TA tp[2][kG], tb[2][kG], tt[2][kG], ts[2][kG];
#pragma unroll
        for (int j = 0; j < kG; ++j) {
            const int f = j < FM ? j : FM - 1;
            tp[0][j] = pd[f];
            tb[0][j] = bt[2 * f];
            tt[0][j] = bt[2 * f + 1];
            ts[0][j] = ss[f];
        }
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            if (g + 1 < NG) {
                const int nb = (g + 1) & 1;
#pragma unroll
                for (int j = 0; j < kG; ++j) {
                    const int f = (g + 1) * kG + j < FM ? (g + 1) * kG + j : FM - 1;
                    tp[nb][j] = pd[f];
                    tb[nb][j] = bt[2 * f];
                    tt[nb][j] = bt[2 * f + 1];
                    ts[nb][j] = ss[f];
                }
            }
            __builtin_amdgcn_sched_barrier(0);
            const int cb = g & 1;
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int f = g * kG + j;
                if (f < FM) band(f, (TA)vq[f], (TA)vu[f], tp[cb][j], tb[cb][j], tt[cb][j], ts[cb][j]);
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
        TS nq[kG], nu[kG];
#pragma unroll
        for (int j = 0; j < kG; ++j) {
            const int f = j < F ? j : F - 1;
            nq[j] = ld_stream(dq + f * kChunk);
            nu[j] = ld_stream(du + f * kChunk);
        }
        for (int g0 = 0; g0 < F; g0 += kG) {
            TS cq[kG], cu[kG];
            TA tpd[kG], tbt[kG], tdt[kG], tss[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                cq[j] = nq[j];
                cu[j] = nu[j];
                const int f = g0 + j < F ? g0 + j : F - 1;
                tpd[j] = pd[f];
                tbt[j] = bt[2 * f];
                tdt[j] = bt[2 * f + 1];
                tss[j] = ss[f];
            }
            __builtin_amdgcn_sched_barrier(0);
            if (g0 + kG < F) {
#pragma unroll
                for (int j = 0; j < kG; ++j) {
                    const int f = g0 + kG + j < F ? g0 + kG + j : F - 1;
                    nq[j] = ld_stream(dq + f * kChunk);
                    nu[j] = ld_stream(du + f * kChunk);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < kG; ++j)
                if (g0 + j < F) band(g0 + j, (TA)cq[j], (TA)cu[j], tpd[j], tbt[j], tdt[j], tss[j]);
        }
    }
}

// a7 (first level): inclusive scan inside each constant-label run of the wavefront; the run's
// last lane holds the run total and writes the segment's (f, dF/dbeta_d, dF/dT_d, dF/dbeta_s).
// The scan moves values between lanes by DPP (VALU only, no LDS round trip): within each 16-lane
// row it adds the lane 1, 2, 4 and 8 places below when that lane is in the same run, then each
// odd row adds the last lane of the row below and rows 2 and 3 add lane 31, each again only when
// the source lane is in the same run.  A non-finite gradient partial sets the item's NONFINITE
// bit here (every lane of the wavefront must be active).
// The moved value is undefined in lanes the pattern does not reach (rows outside ROW_MASK, sources
// outside the row); seg_step never adds it there.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_from(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, ROW_MASK, 0xf, false);
    return __hiloint2double(hi, lo);
}
template <bool GRAD, int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_step(bool take, double &f, double &g1, double &g2, double &g3) {
    const double of = dpp_from<CTRL, ROW_MASK>(f);
    double o1 = 0, o2 = 0, o3 = 0;
    if (GRAD) {
        o1 = dpp_from<CTRL, ROW_MASK>(g1);
        o2 = dpp_from<CTRL, ROW_MASK>(g2);
        o3 = dpp_from<CTRL, ROW_MASK>(g3);
    }
    if (take) {
        f += of;
        if (GRAD) {
            g1 += o1;
            g2 += o2;
            g3 += o3;
        }
    }
}
constexpr int kDppRowShr1 = 0x111, kDppRowShr2 = 0x112, kDppRowShr4 = 0x114, kDppRowShr8 = 0x118;
constexpr int kDppRowBcast15 = 0x142, kDppRowBcast31 = 0x143;

template <bool GRAD>
__device__ __forceinline__ void seg_reduce_write(uint64_t head, int lane, double fpix, double g1, double g2,
                                                 double g3, double *out, int32_t *status) {
    const int start = 63 - __clzll(head & lanemask_le(lane));
    const int r16 = lane & 15;
    seg_step<GRAD, kDppRowShr1, 0xf>(r16 >= 1 && lane - 1 >= start, fpix, g1, g2, g3);
    seg_step<GRAD, kDppRowShr2, 0xf>(r16 >= 2 && lane - 2 >= start, fpix, g1, g2, g3);
    seg_step<GRAD, kDppRowShr4, 0xf>(r16 >= 4 && lane - 4 >= start, fpix, g1, g2, g3);
    seg_step<GRAD, kDppRowShr8, 0xf>(r16 >= 8 && lane - 8 >= start, fpix, g1, g2, g3);
    seg_step<GRAD, kDppRowBcast15, 0xa>(((lane >> 4) & 1) && (lane & ~15) - 1 >= start, fpix, g1, g2, g3);
    seg_step<GRAD, kDppRowBcast31, 0xc>(lane >= 32 && 31 >= start, fpix, g1, g2, g3);
    const bool last = (lane == 63) || ((head >> (lane + 1)) & 1ull);
    if (last) {
        out[0] = fpix;
        out[1] = GRAD ? g1 : 0.0;
        out[2] = GRAD ? g2 : 0.0;
        out[3] = GRAD ? g3 : 0.0;
    }
    if (GRAD && __ballot(last && !(isfinite(g1) && isfinite(g2) && isfinite(g3))) && lane == 0)
        atomicOr(status, (int)CS_ITEM_NONFINITE);
}

// WM: 0 = band weights shared by Q and U, 1 = band weights per Stokes, 2 = per-pixel weights.
// One 64-pixel work unit, every per-pixel sum formed by its own lane.
template <typename TS, typename TA, bool GRAD, int WM, int FM>
__device__ __forceinline__ void unit_pixel(const EvalArgs &a, const int item, const int chunk, const int lane) {
    constexpr int NW = (WM == 0) ? 1 : 2;
    const cptr<BandDev> B = as_const(a.band);
    const int F = a.nfreq;
    const cptr<ItemDev> items = as_const(a.items);
    const cptr<LayoutDev> layouts = as_const(a.layouts);
    {
        const cptr<ItemDev> it = items + item;
        const cptr<LayoutDev> L = layouts + it->layout;
        const uint64_t head = as_const(L->head)[chunk];
        const int segbase = as_const(L->seg_base)[chunk];
        const int nvalid = L->n_incl - chunk * kChunk;
        const bool valid = lane < nvalid;
        const int segl = __popcll(head & lanemask_le(lane)) - 1;
        const gptr<int> labp = as_global((const int *)L->seg_lab) + 4 * (int64_t)(segbase + segl);
        const int lab_d = labp[0], lab_t = labp[1], lab_s = labp[2];
        const int64_t kd = it->k[0], kt = it->k[1];

        const gptr<TA> tab = as_global((const TA *)a.tables) + it->tab_off * (int64_t)F;
        const gptr<TA> pd = tab + (int64_t)lab_d * F;
        const gptr<TA> bt = tab + (kd + 2 * (int64_t)lab_t) * F;
        const gptr<TA> ss = tab + (kd + 2 * kt + lab_s) * F;
        const int64_t cbase = (it->dchunk0 + chunk) * (2 * (int64_t)F * kChunk) + lane;
        const gptr<TS> dq = as_global((const TS *)a.dpack) + cbase;
        const gptr<TS> du = dq + (int64_t)F * kChunk;
        const gptr<TS> wq = (WM == 2) ? as_global((const TS *)a.wpack) + cbase : nullptr;
        const gptr<TS> wu = (WM == 2) ? wq + (int64_t)F * kChunk : nullptr;
        const int64_t part_off = it->part_off;

        WAcc<TA> A[NW];
        SAcc<TA> S[2];
#pragma unroll
        for (int n = 0; n < NW; ++n) A[n] = WAcc<TA>{};
        S[0] = SAcc<TA>{};
        S[1] = SAcc<TA>{};

        // One band's contribution to M, G (per weight set) and b, h (per Stokes).
        auto band = [&](const int f, const TA d0, const TA d1, const TA tpd, const TA tbt, const TA dt, const TA as) {
            const TA ad = tpd * tbt;
            const TA lgd = Band<TA>::ld(B, f);
            const TA lgs = Band<TA>::ls(B, f);
            TA w[2];
            if (WM == 2) {
                const int fc = f < F ? f : F - 1;
                w[0] = f < F ? (TA)wq[fc * kChunk] : (TA)0;
                w[1] = f < F ? (TA)wu[fc * kChunk] : (TA)0;
            } else {
                w[0] = Band<TA>::w(B, 0, f);
                w[1] = Band<TA>::w(B, 1, f);
            }
#pragma unroll
            for (int n = 0; n < NW; ++n) {
                const TA wn = w[n];
                const TA wad = wn * ad, was = wn * as;
                WAcc<TA> &c = A[n];
                if (WM == 2) c.m00 += wn;
                c.m01 += wad;
                c.m02 += was;
                c.m11 = fma(wad, ad, c.m11);
                c.m12 = fma(wad, as, c.m12);
                c.m22 = fma(was, as, c.m22);
                if (GRAD) {
                    const TA c1 = wad * lgd, c2 = wad * dt, c3 = was * lgs;
                    c.g01 += c1;
                    c.g02 += c2;
                    c.g03 += c3;
                    c.g11 = fma(c1, ad, c.g11);
                    c.g12 = fma(c2, ad, c.g12);
                    c.g13 = fma(c3, ad, c.g13);
                    c.g21 = fma(c1, as, c.g21);
                    c.g22 = fma(c2, as, c.g22);
                    c.g23 = fma(c3, as, c.g23);
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int n = (NW == 1) ? 0 : s;
                const TA dv = s ? d1 : d0;
                const TA wn = w[n];
                const TA wad = wn * ad, was = wn * as;
                SAcc<TA> &c = S[s];
                c.b0 = fma(wn, dv, c.b0);
                c.b1 = fma(wad, dv, c.b1);
                c.b2 = fma(was, dv, c.b2);
                if (GRAD) {
                    c.h1 = fma(wad * lgd, dv, c.h1);
                    c.h2 = fma(wad * dt, dv, c.h2);
                    c.h3 = fma(was * lgs, dv, c.h3);
                }
            }
        };
        band_loop<FM, CS_BAND_GROUP, TS, TA>(F, dq, du, pd, bt, ss, band);

        // a5: FP64 Cholesky of each weight set's M, then per Stokes z = L^-1 b, b^T M^-1 b = z.z,
        // s_hat = L^-T z; a6: gradient from h and G.
        double fpix = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
        bool ok = true;
#pragma unroll
        for (int n = 0; n < NW; ++n) {
            const WAcc<TA> &c = A[n];
            const double m00 = (WM == 2) ? (double)c.m00 : (double)Band<TA>::wsum(B, n);
            const double m01 = c.m01, m02 = c.m02, m11 = c.m11, m12 = c.m12, m22 = c.m22;
            const double i00 = (WM == 2) ? inv_sqrt<TA>(m00) : Band<TA>::isw(B, n);
            const double l10 = m01 * i00, l20 = m02 * i00;
            const double p1 = m11 - l10 * l10;
            const double i11 = inv_sqrt<TA>(p1);
            const double l21 = (m12 - l20 * l10) * i11;
            const double p2 = m22 - l20 * l20 - l21 * l21;
            const double i22 = inv_sqrt<TA>(p2);
            ok = ok && pd_pivots<TA>(m00, m11, m22, p1, p2);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                if (NW == 2 && s != n) continue;
                const SAcc<TA> &q = S[s];
                const double b0 = q.b0, b1 = q.b1, b2 = q.b2;
                const double z0 = b0 * i00;
                const double z1 = (b1 - l10 * z0) * i11;
                const double z2 = (b2 - l20 * z0 - l21 * z1) * i22;
                fpix -= z0 * z0 + z1 * z1 + z2 * z2;
                if (GRAD) {
                    const double s2 = z2 * i22;
                    const double s1 = (z1 - l21 * s2) * i11;
                    const double s0 = (z0 - l10 * s1 - l20 * s2) * i00;
                    const double e1 = (double)q.h1 - (s0 * (double)c.g01 + s1 * (double)c.g11 + s2 * (double)c.g21);
                    const double e2 = (double)q.h2 - (s0 * (double)c.g02 + s1 * (double)c.g12 + s2 * (double)c.g22);
                    const double e3 = (double)q.h3 - (s0 * (double)c.g03 + s1 * (double)c.g13 + s2 * (double)c.g23);
                    g1 -= 2.0 * s1 * e1;
                    g2 -= 2.0 * s1 * e2;
                    g3 -= 2.0 * s2 * e3;
                }
            }
        }
        if (!valid) {
            fpix = 0.0;
            g1 = g2 = g3 = 0.0;
        } else if (!ok) {
            fpix = g1 = g2 = g3 = __builtin_nan("");
        }
        const uint64_t bad = __ballot(valid && !ok);
        if (bad && lane == 0) atomicOr(&a.istatus[item], (int)CS_ITEM_NOT_PD);

        seg_reduce_write<GRAD>(head, lane, fpix, g1, g2, g3, a.partials + (part_off + segbase + segl) * 4,
                               &a.istatus[item]);
    }
}

template <typename TS, typename TA, bool GRAD, int WM, int FM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(CS_WAVES_PER_EU))) void k_pixel(const EvalArgs a) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = a.waves_per_block;
    const int64_t nb = gridDim.x;
    const int64_t lb = logical_block(a.xcd_remap);
    const cptr<int> units = as_const((const int *)a.units);
    for (int64_t u = lb * wpb + wave; u < a.nunits; u += nb * wpb) {
        const int item = __builtin_amdgcn_readfirstlane(units[2 * u]);
        const int chunk = __builtin_amdgcn_readfirstlane(units[2 * u + 1]);
        if (a.active && !as_const(a.active)[item]) continue;
        unit_pixel<TS, TA, GRAD, WM, FM>(a, item, chunk, lane);
    }
}

// ---------------------------------------------------------------------------------------------
// LDS-staged pixel kernel (band weights shared by Q and U).  Each wavefront first stages, for
// every segment (constant-label run) of its chunk, the per-band coefficients of its sums in its
// own LDS slice -- one parallel round of SED-table gathers -- and the band loop then issues only
// the streaming data loads (a ring of kRing groups prefetched ahead) and reads the coefficients
// from LDS, whose counter is separate from the vector-memory counter: no table gather ever
// waits behind a data load.  M = A^T N^-1 A and the adjoint sums G_jk depend only on a pixel's
// labels; three ways to form them (the staging mode SM):
//   per-pixel (SM = 0): every lane accumulates them over the bands itself;
//   segment-shared (SM = 1): while staging, four lanes per segment accumulate them over
//     interleaved bands and add their partials, and one of them forms the FP64 Cholesky factor
//     of M into the slice; every pixel then accumulates only its data-dependent sums b and h
//     (12 FMAs per band) and reads its segment's factor;
//   segment sums (SM = 2, FP32 accumulation): the staging stores each (segment, band)'s
//     coefficients (w a_d, w a_s, w a_d ln(nu/nu0d), w a_d dlnBT/dT, w a_s ln(nu/nu0s)) and
//     (a_d, a_s); five lanes per segment then each run one coefficient over the bands against
//     (1, a_d, a_s) -- all segments of a chunk in one pass, three sums per lane -- while every
//     pixel accumulates only b and h (12 FMAs per band) and takes its segment's fourteen sums
//     from those lanes by cross-lane reads before its own FP64 Cholesky.
// Chunks with more than kStageSeg segments take the direct-gather per-pixel path.
// ---------------------------------------------------------------------------------------------
// Per segment: the Cholesky factor of M (inverse diagonal), G_jk and a positive-definite flag,
// held field-major in the slice (double [kRecFields][kStageSeg]): the lanes of different segments
// then write and read consecutive words, free of LDS bank conflicts.
enum RecField { kI00, kL10, kL20, kI11, kL21, kI22, kG01, kG02, kG03, kG11, kG12, kG13, kG21, kG22, kG23, kOk,
                kRecFields };

constexpr int kStageSeg = 12;  // segments staged per chunk (more: direct-gather path)
static_assert(kStageSeg <= kSegLabPad, "twelve label records are read past a chunk's first segment");
constexpr int kLanesPerSeg = 4;

template <typename TA>
struct alignas(4 * sizeof(TA)) Col4 {
    TA x, y, z, w;
};

template <typename TA>
struct alignas(2 * sizeof(TA)) Vec2 {
    TA x, y;
};

// LDS slice of one wavefront: Col4 [kStageSeg][F]; the segment-shared mode adds TA [kStageSeg][F]
// (16-byte padded) and double [kRecFields][kStageSeg]; the segment-sum mode adds Vec2
// [kStageSeg][F] and TA [kStageSeg][F]
template <typename TA>
__host__ __device__ constexpr size_t stage_col_bytes(int F) {
    return (size_t)kStageSeg * (size_t)F * sizeof(Col4<TA>);
}
template <typename TA>
__host__ __device__ constexpr size_t stage_c5_bytes(int F) {
    return ((size_t)kStageSeg * (size_t)F * sizeof(TA) + 15) & ~(size_t)15;
}
template <typename TA>
__host__ __device__ constexpr size_t stage_v2_bytes(int F) {
    return (size_t)kStageSeg * (size_t)F * sizeof(Vec2<TA>);
}
template <typename TA, int SM>
__host__ __device__ constexpr size_t stage_bytes_per_wave(int F) {
    return SM == 1   ? stage_col_bytes<TA>(F) + stage_c5_bytes<TA>(F) + (size_t)kRecFields * kStageSeg * sizeof(double)
           : SM == 2 ? stage_col_bytes<TA>(F) + stage_v2_bytes<TA>(F) + stage_c5_bytes<TA>(F)
                     : stage_col_bytes<TA>(F);
}

// Sum over the four lanes of a quad, the same value in each: (v0 + v1) + (v2 + v3) via DPP
// quad permutations (every lane of the wavefront must be active).
template <int kCtrl>
__device__ __forceinline__ float quad_swap(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}
template <int kCtrl>
__device__ __forceinline__ double quad_swap(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), kCtrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T quad_sum(T v) {
    v = v + quad_swap<0xB1>(v);  // lanes (1,0,3,2)
    v = v + quad_swap<0x4E>(v);  // lanes (2,3,0,1)
    return v;
}

template <typename TS, typename TA, bool GRAD, int SM>
__device__ __forceinline__ void unit_staged(const EvalArgs &a, const int item, const int chunk, const int lane,
                                            char *wave_lds) {
    constexpr bool SHARED = SM == 1;
    constexpr bool SUMS = SM == 2;
    static_assert(!SUMS || sizeof(TA) == 4, "the segment-sum mode stages FP32 coefficients");
    // groups of kG bands in flight per lane: the segment-shared band loop is short (12 FMAs per
    // band), so it looks further ahead (measured on gfx950: 8 groups for it; 6 for per-pixel with
    // FP32 accumulation, 4 with FP64, whose registers would otherwise cost it a wavefront)
    constexpr int kRing = SHARED ? 8 : (SUMS ? CS_SUMS_RING : (sizeof(TA) == 4 ? 6 : CS_FP64_RING));
    constexpr int kG = 2;
    const cptr<BandDev> B = as_const(a.band);
    const int F = a.nfreq;
    const cptr<ItemDev> it = as_const(a.items) + item;
    const cptr<LayoutDev> L = as_const(a.layouts) + it->layout;
    const uint64_t head = as_const(L->head)[chunk];
    const int segbase = as_const(L->seg_base)[chunk];
    const int nseg = as_const(L->seg_base)[chunk + 1] - segbase;
    const int nvalid = L->n_incl - chunk * kChunk;
    const bool valid = lane < nvalid;
    const int segl = __popcll(head & lanemask_le(lane)) - 1;
    const int64_t kd = it->k[0], kt = it->k[1];
    // the chunk's data through a buffer descriptor: the band's byte offset in a scalar register,
    // the lane's in one vector register shared by every band, so a load needs no per-lane address
    // arithmetic (and the descriptor's range bounds every access to the chunk)
    const TS *dchunk = (const TS *)a.dpack + (it->dchunk0 + chunk) * (2 * (int64_t)F * kChunk);
    const __amdgpu_buffer_rsrc_t drsrc = __builtin_amdgcn_make_buffer_rsrc(
        (void *)dchunk, (short)0, (int)(2 * F * kChunk * (int)sizeof(TS)), kRawBufferDword3);
    const int lane_bytes = lane * (int)sizeof(TS);
    auto ld_band = [&](int s, int f) { return ld_stream_buf<TS>(drsrc, lane_bytes, (s * F + f) * kChunk * (int)sizeof(TS)); };

    // data ring: groups 0 .. kRing-1, requested before anything else, except on the FP32
    // per-pixel fast path below, which sends it behind its table gathers
    TS rq[kRing][kG], ru[kRing][kG];
    auto issue_ring = [&]() {
#pragma unroll
        for (int r = 0; r < kRing; ++r)
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int f0 = r * kG + j;
                const int f = f0 < F ? f0 : F - 1;
                rq[r][j] = ld_band(0, f);
                ru[r][j] = ld_band(1, f);
            }
    };
    // table offsets of the fast path are 32-bit byte offsets
    const int64_t trows = kd + 2 * kt + it->k[2];
    static_assert(kFMax <= 32, "one band per lane of a half-wavefront");
    const bool fast = sizeof(TA) == 4 && !SHARED && trows * F < (int64_t(1) << 28);
    if (!fast) issue_ring();

    Col4<TA> *cols = (Col4<TA> *)wave_lds;
    // the segment-sum mode keeps (a_d, a_s) between the coefficient columns and the fifth one
    Vec2<TA> *v2 = (Vec2<TA> *)(wave_lds + stage_col_bytes<TA>(F));
    TA *c5 = (TA *)(wave_lds + stage_col_bytes<TA>(F) + (SUMS ? stage_v2_bytes<TA>(F) : 0));
    double *recs = (double *)(wave_lds + stage_col_bytes<TA>(F) + stage_c5_bytes<TA>(F));
    const gptr<TA> tab = as_global((const TA *)a.tables) + it->tab_off * (int64_t)F;
    const gptr<int> seglab = as_global((const int *)L->seg_lab) + 4 * (int64_t)segbase;
    if (fast) {
        // columns (a_d, da_d/dT / a_d, a_s) of every (segment, band): in round r the half-wavefront
        // h stages segment 2 r + h with lane & 31 = band.  The labels arrive through the scalar
        // cache (the array is padded, so the records past the chunk's last segment can be read)
        // and each table's byte offset is formed on the scalar unit as a base plus the second
        // half's difference; all gathers are issued before the first use.  (FP64 accumulation
        // keeps the general path: this one's registers would cost it a wavefront per SIMD.)
        constexpr int kRounds = kStageSeg / 2;
        const cptr<int> sl = as_const((const int *)L->seg_lab) + 4 * (int64_t)segbase;
        const int rb = F * (int)sizeof(TA);  // bytes per table row
        const int kdb = (int)kd * rb, kdtb = (int)(kd + 2 * kt) * rb;
        const bool hi = lane >= 32;
        int hmask = hi ? -1 : 0;  // selects the second half's offset differences
        asm volatile("" : "+v"(hmask));  // kept as a mask: one AND per offset, not a select
        int f = lane & 31;
        // segment-sum mode: the staging's LDS addresses are formed per unit (hoisted out of the
        // unit loop they would hold 18 registers through the band loop)
        if (SUMS) asm volatile("" : "+v"(f));
        const int fb = (f < F ? f : F - 1) * (int)sizeof(TA);
        const int nr = (nseg + 1) >> 1;
        const char *tb = (const char *)(const TA *)tab;
        auto at = [&](int e) { return *(gptr<TA>)(tb + (uint32_t)e); };
        // segment-sum mode: this lane's band constants, requested ahead of the gathers
        TA wl = 0, ldl = 0, lsl = 0;
        if (SUMS) {
            const int fc = f < F ? f : F - 1;
            wl = Band<TA>::w(B, 0, fc);
            ldl = Band<TA>::ld(B, fc);
            lsl = Band<TA>::ls(B, fc);
        }
        TA pdv[kRounds], btv[kRounds], dtv[kRounds], ssv[kRounds];
#pragma unroll
        for (int r = 0; r < kRounds; ++r) {
            if (r < nr) {
                const cptr<int> l0 = sl + 8 * r, l1 = l0 + 4;
                int bd = l0[0] * rb, bt2 = kdb + l0[1] * 2 * rb, bs = kdtb + l0[2] * rb;
                // the second half repeats segment 2 r when 2 r + 1 is past the chunk's last one
                const bool two = 2 * r + 1 < nseg;
                int dd = two ? l1[0] * rb - bd : 0, dt2 = two ? kdb + l1[1] * 2 * rb - bt2 : 0,
                    ds = two ? kdtb + l1[2] * rb - bs : 0;
                // keep the products on the scalar unit (not re-formed per lane after the select)
                asm volatile("" : "+s"(bd), "+s"(bt2), "+s"(bs), "+s"(dd), "+s"(dt2), "+s"(ds));
                const int ed = bd + (dd & hmask) + fb;
                const int et = bt2 + (dt2 & hmask) + 2 * fb;
                const int es = bs + (ds & hmask) + fb;
                pdv[r] = at(ed);
                btv[r] = at(et);
                dtv[r] = at(et + (int)sizeof(TA));
                ssv[r] = at(es);
            }
        }
        // the ring goes out behind the gathers: vector-memory loads complete in order, so the
        // column writes wait only for the gathers while the ring is still in flight
        issue_ring();
        const int lbase = (hi ? F : 0) + f;
#pragma unroll
        for (int r = 0; r < kRounds; ++r)
            if (r < nr && f < F && 2 * r + (hi ? 1 : 0) < nseg) {
                const int e = 2 * r * F + lbase;
                const TA ad = pdv[r] * btv[r], dt = dtv[r], as = ssv[r];
                if (SUMS) {
                    const TA wad = wl * ad, was = wl * as;
                    cols[e] = Col4<TA>{wad, was, wad * ldl, wad * dt};
                    c5[e] = was * lsl;
                    v2[e] = Vec2<TA>{ad, as};
                } else {
                    cols[e] = Col4<TA>{ad, dt, as, (TA)0};
                }
            }
    } else if (!SHARED) {
        // columns (a_d, da_d/dT / a_d, a_s) of every (segment, band), in phases of kPh rounds of
        // the wavefront whose gathers are all issued before their first use
        constexpr int kPh = sizeof(TA) == 4 ? 6 : 3;  // measured best on gfx950 at F = 22
        const int ne = nseg * F;
        for (int e0 = 0; e0 < ne; e0 += kPh * kChunk) {
            int sgi[kPh], fi[kPh];
#pragma unroll
            for (int i = 0; i < kPh; ++i) {
                const int e = e0 + lane + i * kChunk;
                const int ec = e < ne ? e : ne - 1;
                sgi[i] = ec / F;
                fi[i] = ec - sgi[i] * F;
            }
            int lab[kPh][3];
#pragma unroll
            for (int i = 0; i < kPh; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) lab[i][j] = seglab[4 * sgi[i] + j];
            TA pdv[kPh], btv[kPh], dtv[kPh], ssv[kPh];
#pragma unroll
            for (int i = 0; i < kPh; ++i) {
                const int f = fi[i];
                pdv[i] = tab[(int64_t)lab[i][0] * F + f];
                btv[i] = tab[(kd + 2 * (int64_t)lab[i][1]) * F + 2 * f];
                dtv[i] = tab[(kd + 2 * (int64_t)lab[i][1]) * F + 2 * f + 1];
                ssv[i] = tab[(kd + 2 * kt + lab[i][2]) * F + f];
            }
#pragma unroll
            for (int i = 0; i < kPh; ++i) {
                const int e = e0 + lane + i * kChunk;
                if (e < ne) cols[e] = Col4<TA>{pdv[i] * btv[i], dtv[i], ssv[i], (TA)0};
            }
        }
    } else {
        // coefficients (w a_d, w a_s, w a_d ln(nu/nu0d), w da_d/dT, w a_s ln(nu/nu0s)) of every
        // (segment, band), and the segment's M and G sums: lane = 4 segment + part, bands
        // part, part + 4, ...; phases of kPh bands per lane, every gather of a phase issued before
        // its first use
        constexpr int kPh = sizeof(TA) == 4 ? 4 : 2;
        const int sg = lane / kLanesPerSeg, part = lane % kLanesPerSeg;
        const bool act = sg < nseg;
        const int sgc = act ? sg : 0;
        const int ld = seglab[4 * sgc], lt = seglab[4 * sgc + 1], ls = seglab[4 * sgc + 2];
        const gptr<TA> pd = tab + (int64_t)ld * F;
        const gptr<TA> bt = tab + (kd + 2 * (int64_t)lt) * F;
        const gptr<TA> ss = tab + (kd + 2 * kt + ls) * F;
        const BandDev *Bp = a.band;
        const gptr<TA> bc = as_global(sizeof(TA) == 8 ? (const TA *)(const void *)&Bp->bcd[0][0]
                                                      : (const TA *)(const void *)&Bp->bcf[0][0]);
        WAcc<TA> P = WAcc<TA>{};
        for (int f0 = 0; f0 < F; f0 += kLanesPerSeg * kPh) {
            TA pdv[kPh], btv[kPh], dtv[kPh], ssv[kPh], wv[kPh], ldv[kPh], lsv[kPh];
#pragma unroll
            for (int i = 0; i < kPh; ++i) {
                const int fr = f0 + part + kLanesPerSeg * i;
                const int f = fr < F ? fr : F - 1;
                const gptr<TA> c = bc + 4 * f;  // (w, ln(nu/nu0d), ln(nu/nu0s), 0)
                wv[i] = c[0];
                ldv[i] = c[1];
                lsv[i] = c[2];
                pdv[i] = pd[f];
                btv[i] = bt[2 * f];
                dtv[i] = bt[2 * f + 1];
                ssv[i] = ss[f];
            }
#pragma unroll
            for (int i = 0; i < kPh; ++i) {
                const int f = f0 + part + kLanesPerSeg * i;
                const bool use = act && f < F;
                const TA ad = pdv[i] * btv[i], dt = dtv[i], as = ssv[i];
                const TA w = use ? wv[i] : (TA)0;  // nothing past F or past the chunk's segments
                const TA cad = w * ad, cas = w * as;
                const TA c1 = cad * ldv[i], c2 = cad * dt, c3 = cas * lsv[i];
                if (use) {
                    cols[sg * F + f] = Col4<TA>{cad, cas, c1, c2};
                    c5[sg * F + f] = c3;
                }
                P.m01 += cad;
                P.m02 += cas;
                P.m11 = fma(cad, ad, P.m11);
                P.m12 = fma(cad, as, P.m12);
                P.m22 = fma(cas, as, P.m22);
                if (GRAD) {
                    P.g01 += c1;
                    P.g02 += c2;
                    P.g03 += c3;
                    P.g11 = fma(c1, ad, P.g11);
                    P.g12 = fma(c2, ad, P.g12);
                    P.g13 = fma(c3, ad, P.g13);
                    P.g21 = fma(c1, as, P.g21);
                    P.g22 = fma(c2, as, P.g22);
                    P.g23 = fma(c3, as, P.g23);
                }
            }
        }
        P.m01 = quad_sum(P.m01);
        P.m02 = quad_sum(P.m02);
        P.m11 = quad_sum(P.m11);
        P.m12 = quad_sum(P.m12);
        P.m22 = quad_sum(P.m22);
        if (GRAD) {
            P.g01 = quad_sum(P.g01);
            P.g02 = quad_sum(P.g02);
            P.g03 = quad_sum(P.g03);
            P.g11 = quad_sum(P.g11);
            P.g12 = quad_sum(P.g12);
            P.g13 = quad_sum(P.g13);
            P.g21 = quad_sum(P.g21);
            P.g22 = quad_sum(P.g22);
            P.g23 = quad_sum(P.g23);
        }
        if (part == 0 && sg < nseg) {
            const double m00 = (double)Band<TA>::wsum(B, 0);
            const double m01 = P.m01, m02 = P.m02, m11 = P.m11, m12 = P.m12, m22 = P.m22;
            const double i00 = Band<TA>::isw(B, 0);
            const double l10 = m01 * i00, l20 = m02 * i00;
            const double p1 = m11 - l10 * l10;
            const double i11 = inv_sqrt<TA>(p1);
            const double l21 = (m12 - l20 * l10) * i11;
            const double p2 = m22 - l20 * l20 - l21 * l21;
            const double i22 = inv_sqrt<TA>(p2);
            double *r = recs + sg;
            r[kI00 * kStageSeg] = i00;
            r[kL10 * kStageSeg] = l10;
            r[kL20 * kStageSeg] = l20;
            r[kI11 * kStageSeg] = i11;
            r[kL21 * kStageSeg] = l21;
            r[kI22 * kStageSeg] = i22;
            r[kOk * kStageSeg] = pd_pivots<TA>(m00, m11, m22, p1, p2) ? 1.0 : 0.0;
            r[kG01 * kStageSeg] = P.g01;
            r[kG02 * kStageSeg] = P.g02;
            r[kG03 * kStageSeg] = P.g03;
            r[kG11 * kStageSeg] = P.g11;
            r[kG12 * kStageSeg] = P.g12;
            r[kG13 * kStageSeg] = P.g13;
            r[kG21 * kStageSeg] = P.g21;
            r[kG22 * kStageSeg] = P.g22;
            r[kG23 * kStageSeg] = P.g23;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // segment-sum mode: lane 5 s + i runs coefficient i of segment s over the bands against
    // (1, a_d, a_s); the i = 1 lane's a_d sum is not used.  Lanes past the chunk's segments
    // (and lanes 60-63) read slots of the slice that hold no data of this unit and are not read.
    TA ms0 = 0, ms1 = 0, ms2 = 0;
    if (SUMS) {
        const int q = lane / 5;
        const int im = lane - 5 * q;
        const int sgm = q < kStageSeg ? q : kStageSeg - 1;
        const TA *up = im < 4 ? &cols[sgm * F].x + im : c5 + sgm * F;
        const int ust = im < 4 ? 4 : 1;
        const Vec2<TA> *vp = v2 + sgm * F;
        auto add = [&](const TA u, const Vec2<TA> v) {
            ms0 += u;
            ms1 = fma(u, v.x, ms1);
            ms2 = fma(u, v.y, ms2);
        };
        int f = 0;
        for (; f + 4 <= F; f += 4) {  // four bands per step: one pointer step, v2 by immediate offsets
            const TA u0 = up[0], u1 = up[ust], u2 = up[2 * ust], u3 = up[3 * ust];
            up += 4 * ust;
            add(u0, vp[f]);
            add(u1, vp[f + 1]);
            add(u2, vp[f + 2]);
            add(u3, vp[f + 3]);
        }
        for (; f < F; ++f) {
            add(*up, vp[f]);
            up += ust;
        }
    }

    WAcc<TA> A = WAcc<TA>{};
    SAcc<TA> S[2];
    S[0] = SAcc<TA>{};
    S[1] = SAcc<TA>{};
    const Col4<TA> *mycols = cols + segl * F;
    const TA *myc5 = c5 + segl * F;
    auto band = [&](const int f, const TA d0, const TA d1) {
        const Col4<TA> c = mycols[f];
        const TA w = Band<TA>::w(B, 0, f);
        if (SHARED || SUMS) {
            const TA c3 = myc5[f];
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const TA dv = s ? d1 : d0;
                SAcc<TA> &q = S[s];
                q.b0 = fma(w, dv, q.b0);
                q.b1 = fma(c.x, dv, q.b1);
                q.b2 = fma(c.y, dv, q.b2);
                if (GRAD) {
                    q.h1 = fma(c.z, dv, q.h1);
                    q.h2 = fma(c.w, dv, q.h2);
                    q.h3 = fma(c3, dv, q.h3);
                }
            }
            return;
        }
        const TA ad = c.x, dt = c.y, as = c.z;
        const TA lgd = Band<TA>::ld(B, f), lgs = Band<TA>::ls(B, f);
        const TA wad = w * ad, was = w * as;
        const TA c1 = wad * lgd, c2 = wad * dt, c3 = was * lgs;
        A.m01 += wad;
        A.m02 += was;
        A.m11 = fma(wad, ad, A.m11);
        A.m12 = fma(wad, as, A.m12);
        A.m22 = fma(was, as, A.m22);
        if (GRAD) {
            A.g01 += c1;
            A.g02 += c2;
            A.g03 += c3;
            A.g11 = fma(c1, ad, A.g11);
            A.g12 = fma(c2, ad, A.g12);
            A.g13 = fma(c3, ad, A.g13);
            A.g21 = fma(c1, as, A.g21);
            A.g22 = fma(c2, as, A.g22);
            A.g23 = fma(c3, as, A.g23);
        }
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const TA dv = s ? d1 : d0;
            SAcc<TA> &q = S[s];
            q.b0 = fma(w, dv, q.b0);
            q.b1 = fma(wad, dv, q.b1);
            q.b2 = fma(was, dv, q.b2);
            if (GRAD) {
                q.h1 = fma(c1, dv, q.h1);
                q.h2 = fma(c2, dv, q.h2);
                q.h3 = fma(c3, dv, q.h3);
            }
        }
    };
    // band loop: consume ring slot r, then refill it kRing groups ahead
    for (int g0 = 0; g0 < F; g0 += kRing * kG) {
#pragma unroll
        for (int r = 0; r < kRing; ++r) {
            const int fb = g0 + r * kG;
#pragma unroll
            for (int j = 0; j < kG; ++j)
                if (fb + j < F) band(fb + j, (TA)rq[r][j], (TA)ru[r][j]);
            if (fb + kRing * kG < F) {
#pragma unroll
                for (int j = 0; j < kG; ++j) {
                    const int f0 = fb + kRing * kG + j;
                    const int f = f0 < F ? f0 : F - 1;
                    rq[r][j] = ld_band(0, f);
                    ru[r][j] = ld_band(1, f);
                }
            }
        }
    }

    // a5/a6: Cholesky factor (per pixel, or the segment's from the slice), then F and gradient
    double i00, l10, l20, i11, l21, i22, G[9];
    bool ok;
    if (SHARED) {
        const double *R = recs + segl;
        i00 = R[kI00 * kStageSeg];
        l10 = R[kL10 * kStageSeg];
        l20 = R[kL20 * kStageSeg];
        i11 = R[kI11 * kStageSeg];
        l21 = R[kL21 * kStageSeg];
        i22 = R[kI22 * kStageSeg];
        G[0] = R[kG01 * kStageSeg]; G[1] = R[kG02 * kStageSeg]; G[2] = R[kG03 * kStageSeg];
        G[3] = R[kG11 * kStageSeg]; G[4] = R[kG12 * kStageSeg]; G[5] = R[kG13 * kStageSeg];
        G[6] = R[kG21 * kStageSeg]; G[7] = R[kG22 * kStageSeg]; G[8] = R[kG23 * kStageSeg];
        ok = R[kOk * kStageSeg] != 0.0;
    } else {
        if (SUMS) {  // the segment's sums from its five lanes (lanes 5 segl + i <= 59)
            const int src = 20 * segl;  // byte address of lane 5 segl
            auto from = [&](TA v, int i) {
                return __int_as_float(__builtin_amdgcn_ds_bpermute(src + 4 * i, __float_as_int(v)));
            };
            A.m01 = from(ms0, 0);
            A.m11 = from(ms1, 0);
            A.m12 = from(ms2, 0);
            A.m02 = from(ms0, 1);
            A.m22 = from(ms2, 1);
            A.g01 = from(ms0, 2);
            A.g11 = from(ms1, 2);
            A.g21 = from(ms2, 2);
            A.g02 = from(ms0, 3);
            A.g12 = from(ms1, 3);
            A.g22 = from(ms2, 3);
            A.g03 = from(ms0, 4);
            A.g13 = from(ms1, 4);
            A.g23 = from(ms2, 4);
        }
        const double m00 = (double)Band<TA>::wsum(B, 0);
        const double m01 = A.m01, m02 = A.m02, m11 = A.m11, m12 = A.m12, m22 = A.m22;
        i00 = Band<TA>::isw(B, 0);
        l10 = m01 * i00;
        l20 = m02 * i00;
        const double p1 = m11 - l10 * l10;
        i11 = inv_sqrt<TA>(p1);
        l21 = (m12 - l20 * l10) * i11;
        const double p2 = m22 - l20 * l20 - l21 * l21;
        i22 = inv_sqrt<TA>(p2);
        ok = pd_pivots<TA>(m00, m11, m22, p1, p2);
        G[0] = A.g01; G[1] = A.g02; G[2] = A.g03;
        G[3] = A.g11; G[4] = A.g12; G[5] = A.g13;
        G[6] = A.g21; G[7] = A.g22; G[8] = A.g23;
    }
    double fpix = 0.0, g1 = 0.0, g2 = 0.0, g3 = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const SAcc<TA> &q = S[s];
        const double z0 = (double)q.b0 * i00;
        const double z1 = ((double)q.b1 - l10 * z0) * i11;
        const double z2 = ((double)q.b2 - l20 * z0 - l21 * z1) * i22;
        fpix -= z0 * z0 + z1 * z1 + z2 * z2;
        if (GRAD) {
            const double s2 = z2 * i22;
            const double s1 = (z1 - l21 * s2) * i11;
            const double s0 = (z0 - l10 * s1 - l20 * s2) * i00;
            const double e1 = (double)q.h1 - (s0 * G[0] + s1 * G[3] + s2 * G[6]);
            const double e2 = (double)q.h2 - (s0 * G[1] + s1 * G[4] + s2 * G[7]);
            const double e3 = (double)q.h3 - (s0 * G[2] + s1 * G[5] + s2 * G[8]);
            g1 -= 2.0 * s1 * e1;
            g2 -= 2.0 * s1 * e2;
            g3 -= 2.0 * s2 * e3;
        }
    }
    if (!valid) {
        fpix = 0.0;
        g1 = g2 = g3 = 0.0;
    } else if (!ok) {
        fpix = g1 = g2 = g3 = __builtin_nan("");
    }
    const uint64_t bad = __ballot(valid && !ok);
    if (bad && lane == 0) atomicOr(&a.istatus[item], (int)CS_ITEM_NOT_PD);
    seg_reduce_write<GRAD>(head, lane, fpix, g1, g2, g3, a.partials + (it->part_off + segbase + segl) * 4,
                           &a.istatus[item]);
    // the slice is rewritten by the wavefront's next unit
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Minimum wavefronts per SIMD the register allocation must allow: five in the per-pixel and
// segment-sum modes with FP32 accumulation (at most 96 VGPRs), four in the per-pixel mode with
// FP64 accumulation (at most 128); the segment-shared mode is left to the compiler.
template <typename TA, int SM>
constexpr int stage_waves() {
    return SM == 1 ? 1 : (SM == 2 ? CS_SUMS_WAVES : (sizeof(TA) == 4 ? CS_STAGE0_WAVES : 4));
}

// The segment-sum staging forms 32-bit table offsets: items whose tables are larger take the
// direct-gather path (the host selects the mode only when every item fits).  LOOP: persistent
// grid, each wavefront looping over units; otherwise one unit per wavefront, so that nothing is
// hoisted across units into registers (17 VGPRs in the segment-sum mode).
template <typename TS, typename TA, bool GRAD, int SM, bool LOOP>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(stage_waves<TA, SM>()))) void k_pixel_stage(
    const EvalArgs a) {
    extern __shared__ char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wpb = a.waves_per_block;
    const int64_t nb = gridDim.x;
    const int64_t lb = logical_block(a.xcd_remap);
    const cptr<int> units = as_const((const int *)a.units);
    char *wave_lds = smem + (size_t)wave * stage_bytes_per_wave<TA, SM>(a.nfreq);
    auto unit = [&](const int64_t u) {
        const int item = __builtin_amdgcn_readfirstlane(units[2 * u]);
        const int chunk = __builtin_amdgcn_readfirstlane(units[2 * u + 1]);
        if (a.active && !as_const(a.active)[item]) return;
        const cptr<ItemDev> it = as_const(a.items) + item;
        const cptr<LayoutDev> L = as_const(a.layouts) + it->layout;
        const int nseg = as_const(L->seg_base)[chunk + 1] - as_const(L->seg_base)[chunk];
        bool staged = nseg <= kStageSeg;
        if (SM == 2) staged = staged && (it->k[0] + 2 * it->k[1] + it->k[2]) * a.nfreq < (int64_t(1) << 28);
        if (staged)
            unit_staged<TS, TA, GRAD, SM>(a, item, chunk, lane, wave_lds);
        else
            unit_pixel<TS, TA, GRAD, 0, 0>(a, item, chunk, lane);
    };
    if constexpr (LOOP) {
        for (int64_t u = lb * wpb + wave; u < a.nunits; u += nb * wpb) unit(u);
    } else {
        const int64_t u = lb * wpb + wave;
        if (u < a.nunits) unit(u);
    }
}

// ---------------------------------------------------------------------------------------------
// a7 (second level): deterministic compensated sums over each cluster's segments
// ---------------------------------------------------------------------------------------------
// One launch for the second level of a7.  Its first nitems workgroups each add all of one item's
// segment values f (Neumaier per thread over a fixed stride, then a fixed tree over the
// workgroup) and write F and the item's status word: NOT_PD and NONFINITE were set by the pixel
// kernel (a non-positive-definite pixel, a non-finite gradient partial), and F non-finite adds
// NONFINITE.  The remaining workgroups hold kFinLanes lanes per (item, cluster): lane l of a
// cluster's group adds the cluster's segments l, l + kFinLanes, ... in order, and the group's
// lane sums are combined by a fixed butterfly, so no result depends on timing.  (A cluster sum
// of finite partials that overflows is not flagged.)  Workgroups are dealt round-robin to the
// XCDs, so the cluster part of the grid is renumbered in groups of eight items: the blocks of one
// item all land on one XCD, whose L2 then holds its partials.
constexpr int kFinLanes = 4;
constexpr int kFinBlock = 256;
__constant__ int32_t kAllActive = 1;  // read in place of the active flags when the caller passes none

__device__ __forceinline__ void neu_combine(double &s, double &c, int off) {
    const double so = __shfl_xor(s, off, kFinLanes), co = __shfl_xor(c, off, kFinLanes);
    neu_add(s, c, so);  // symmetric in its two sums, so every lane of the group agrees
    c += co;
}

__device__ __forceinline__ void f_item(const EvalArgs &a, const int item, double *neg2logl, int32_t *status) {
    const ItemDev &it = a.items[item];
    const LayoutDev &L = a.layouts[it.layout];
    const int64_t n = L.nseg;
    const double *part = a.partials + it.part_off * 4;
    double s = 0, c = 0;
    constexpr int kU = 8;  // loads in flight per thread
    for (int64_t i0 = threadIdx.x; i0 < n; i0 += kU * kFinBlock) {
        double v[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k) {
            const int64_t i = i0 + (int64_t)k * kFinBlock;
            v[k] = i < n ? part[i * 4] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kU; ++k) neu_add(s, c, v[k]);
    }
    __shared__ double ss[kFinBlock], sc[kFinBlock];
    ss[threadIdx.x] = s;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int st = kFinBlock / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            double s1 = ss[threadIdx.x], c1 = sc[threadIdx.x];
            neu_add(s1, c1, ss[threadIdx.x + st]);
            ss[threadIdx.x] = s1;
            sc[threadIdx.x] = c1 + sc[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int st = a.istatus[item];
        double v = ss[0] + sc[0];
        if (st & CS_ITEM_NOT_PD)
            v = __builtin_nan("");
        else if (!isfinite(v))
            st |= CS_ITEM_NONFINITE;
        neg2logl[item] = v;
        if (status) status[item] = st;
        a.istatus[item] = st;
    }
}

template <bool WG, bool WF>
__global__ __launch_bounds__(kFinBlock) void k_fin_grad(const EvalArgs a, int item0, int nitems,
                                                        int kblocks, double *grad, double *cluster_f,
                                                        double *neg2logl, int32_t *status) {
    if ((int)blockIdx.x < nitems) {  // F and status of one item
        const int item = item0 + (int)blockIdx.x;
        if (a.active && !as_const(a.active)[item]) return;
        f_item(a, item, neg2logl, status);
        return;
    }
    if (!WG && !WF) return;
    const int64_t lin = blockIdx.x - nitems;
    const int64_t grp = lin / (kNumXcd * (int64_t)kblocks);
    const int64_t rem = lin - grp * kNumXcd * (int64_t)kblocks;
    const int ng = (int)min((int64_t)kNumXcd, (int64_t)nitems - grp * kNumXcd);  // items in this group
    const int item = item0 + (int)(grp * kNumXcd + rem % ng);
    const int64_t xb = rem / ng;
    // The descriptors come through the scalar cache in two batches: the kernel arguments, then the
    // item's record, its active flag and the first layout's CSR pointers (the layout of every item
    // when the labels are shared); an item with a layout of its own reads that layout after them.
    asm volatile("" ::"s"(a.items), "s"(a.layouts), "s"(a.active), "s"(a.partials), "s"(grad), "s"(cluster_f));
    const cptr<ItemDev> it = as_const(a.items) + item;
    const cptr<int32_t> actp = a.active ? as_const(a.active) + item : as_const(&kAllActive);
    const int32_t lay = it->layout, act = *actp;
    const int64_t k0 = it->k[0], k1 = it->k[1], k2 = it->k[2], x0 = it->xoff, poff = it->part_off;
    cptr<LayoutDev> L = as_const(a.layouts);
    const int32_t *perm0 = L->seg_perm[0], *perm1 = L->seg_perm[1], *perm2 = L->seg_perm[2];
    const int32_t *off0 = L->seg_off[0], *off1 = L->seg_off[1], *off2 = L->seg_off[2];
    asm volatile("" ::"s"(lay), "s"(act), "s"(k0), "s"(k1), "s"(k2), "s"(x0), "s"(poff), "s"(perm0), "s"(perm1),
                 "s"(perm2), "s"(off0), "s"(off1), "s"(off2));
    if (!act) return;
    const int sub = threadIdx.x % kFinLanes;
    int64_t r = xb * (kFinBlock / kFinLanes) + threadIdx.x / kFinLanes;
    if (r >= k0 + k1 + k2) return;  // whole groups leave together
    const int64_t g = x0 + r;
    if (lay != 0) {
        L = as_const(a.layouts) + lay;
        perm0 = L->seg_perm[0], perm1 = L->seg_perm[1], perm2 = L->seg_perm[2];
        off0 = L->seg_off[0], off1 = L->seg_off[1], off2 = L->seg_off[2];
    }
    int j = 0;
    const int32_t *perm = perm0, *soff = off0;
    if (r >= k0) {
        r -= k0;
        j = 1;
        perm = perm1;
        soff = off1;
        if (r >= k1) {
            r -= k1;
            j = 2;
            perm = perm2;
            soff = off2;
        }
    }
    const int b = soff[r], e = soff[r + 1];
    const double *part = a.partials + poff * 4;
    double gs = 0, gc = 0, fs = 0, fc = 0;
    // segments are scattered in the partials: kB of the lane's segments are requested at a time,
    // with the next batch's segment indices already in flight
    constexpr int kB = 4;
    constexpr int kStep = kB * kFinLanes;
    int idx[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
        const int i = b + sub + k * kFinLanes;
        idx[k] = i < e ? perm[i] : 0;
    }
    for (int i0 = b + sub; i0 < e; i0 += kStep) {
        double vg[kB], vf[kB];
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            if (WG) vg[k] = part[idx[k] * 4 + 1 + j];
            if (WF) vf[k] = part[idx[k] * 4];
        }
#pragma unroll
        for (int k = 0; k < kB; ++k) {
            const int i = i0 + kStep + k * kFinLanes;
            idx[k] = i < e ? perm[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < kB; ++k)
            if (i0 + k * kFinLanes < e) {
                if (WG) neu_add(gs, gc, vg[k]);
                if (WF) neu_add(fs, fc, vf[k]);
            }
    }
#pragma unroll
    for (int off = kFinLanes / 2; off > 0; off >>= 1) {
        if (WG) neu_combine(gs, gc, off);
        if (WF) neu_combine(fs, fc, off);
    }
    if (sub != 0) return;
    if (WG) grad[g] = gs + gc;
    if (WF) cluster_f[g] = fs + fc;
}

// ---------------------------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------------------------
// wm == 0 (band weights shared by Q and U): the LDS-staged kernel in staging mode sm, lds bytes
// per workgroup; otherwise the direct-gather kernel with separate Q/U (wm = 1) or per-pixel
// (wm = 2) weights.
// The segment-sum mode takes its one-unit-per-wavefront form unless the grid is persistent; the
// per-pixel and segment-shared modes keep the unit loop (measured faster for them on gfx950:
// without it the per-pixel mode drops to 79 VGPRs and its sixth wavefront per SIMD costs time).
template <typename TS, typename TA, bool GRAD>
static void launch_pixel_t(int wm, int sm, bool loop, size_t lds, dim3 grid, dim3 block, hipStream_t s,
                           const EvalArgs &a) {
    if constexpr (sizeof(TA) == 4)
        if (wm == 0 && sm == 2) {
            if (loop)
                hipLaunchKernelGGL((k_pixel_stage<TS, TA, GRAD, 2, true>), grid, block, lds, s, a);
            else
                hipLaunchKernelGGL((k_pixel_stage<TS, TA, GRAD, 2, false>), grid, block, lds, s, a);
            return;
        }
    if (wm == 0 && sm == 1)
        hipLaunchKernelGGL((k_pixel_stage<TS, TA, GRAD, 1, true>), grid, block, lds, s, a);
    else if (wm == 0 && sizeof(TA) == 8 && CS_FP64_NOLOOP && !loop)
        hipLaunchKernelGGL((k_pixel_stage<TS, TA, GRAD, 0, false>), grid, block, lds, s, a);
    else if (wm == 0)  // sm 0, or 2 where it runs as 0
        hipLaunchKernelGGL((k_pixel_stage<TS, TA, GRAD, 0, true>), grid, block, lds, s, a);
    else if (wm == 1)
        hipLaunchKernelGGL((k_pixel<TS, TA, GRAD, 1, 0>), grid, block, 0, s, a);
    else
        hipLaunchKernelGGL((k_pixel<TS, TA, GRAD, 2, 0>), grid, block, 0, s, a);
}

template <typename TS, typename TA>
static void launch_pixel_g(bool grad, int wm, int sm, bool loop, size_t lds, dim3 grid, dim3 block, hipStream_t s,
                           const EvalArgs &a) {
    if (grad)
        launch_pixel_t<TS, TA, true>(wm, sm, loop, lds, grid, block, s, a);
    else
        launch_pixel_t<TS, TA, false>(wm, sm, loop, lds, grid, block, s, a);
}

// LDS slice of one wavefront of the staged kernel in an arithmetic and staging mode
static size_t stage_bytes(cs_precision mode, int sm, int F) {
    if (mode == CS_FP32_BULK)
        return sm == 1   ? stage_bytes_per_wave<float, 1>(F)
               : sm == 2 ? stage_bytes_per_wave<float, 2>(F)
                         : stage_bytes_per_wave<float, 0>(F);
    return sm == 1 ? stage_bytes_per_wave<double, 1>(F) : stage_bytes_per_wave<double, 0>(F);
}

// Staging mode of a launch: the segment-sum mode needs FP32 accumulation and 32-bit table
// offsets; otherwise it runs as the per-pixel mode (the same sums in another rounding order).
int staging_mode(const cs_problem *p, cs_precision mode) {
    const int sm = p->sched.shared_segments;
    if (sm == 2 && !(mode == CS_FP32_BULK && p->trows_max * p->F < (int64_t(1) << 28))) return 0;
    return sm;
}

EvalArgs make_eval_args(const cs_problem *p, const double *x, const int32_t *active) {
    const WsLayout &w = p->ws;
    EvalArgs a;
    a.units = (const int2 *)(p->wsp + w.units);
    a.nunits = p->nunits;
    a.items = (const ItemDev *)(p->wsp + w.items);
    a.layouts = (const LayoutDev *)(p->wsp + w.layouts);
    a.dpack = p->wsp + w.dpack;
    a.wpack = p->wsp + w.wpack;
    a.tables = p->wsp + w.tables;
    a.band = (const BandDev *)(p->wsp + w.band);
    a.partials = (double *)(p->wsp + w.partials);
    a.istatus = (int32_t *)(p->wsp + w.istatus);
    a.active = active;
    a.x = x;
    a.nitems = p->B;
    a.nfreq = p->F;
    a.xcd_remap = p->sched.xcd_remap;
    a.waves_per_block = p->sched.waves_per_block;
    return a;
}

cs_status launch_sed(const cs_problem *p, const EvalArgs &a, bool fp32_tables, hipStream_t s) {
    const int64_t *xoff_dev = (const int64_t *)(p->wsp + p->ws.items + sizeof(ItemDev) * (size_t)p->B);
    const int nfb = (p->F + kSedBands - 1) / kSedBands;  // band groups per row
    const int rpb = kSedThreads / nfb;                   // rows per workgroup
    const unsigned sblocks = (unsigned)((p->kmax_item + rpb - 1) / rpb);
    for (int b0 = 0; b0 < p->B; b0 += kMaxGridY) {
        const dim3 grid(sblocks, (unsigned)std::min(kMaxGridY, p->B - b0)), block((unsigned)nfb, (unsigned)rpb);
        if (fp32_tables)
            hipLaunchKernelGGL(k_sed<float>, grid, block, 0, s, a, xoff_dev, b0);
        else
            hipLaunchKernelGGL(k_sed<double>, grid, block, 0, s, a, xoff_dev, b0);
        CSI_HIP(hipGetLastError());
    }
    return CS_OK;
}

cs_status launch_eval(cs_problem *p, const double *x, const int32_t *active, double *neg2logl, double *grad,
                      double *cluster_f, int32_t *status, bool want_grad, cs_precision mode, hipStream_t s) {
    const WsLayout &w = p->ws;
    EvalArgs a = make_eval_args(p, x, active);
    const bool t32 = (mode == CS_FP32_BULK);
    const unsigned kblocks = (unsigned)((p->kmax_item * kFinLanes + kFinBlock - 1) / kFinBlock);

    const cs_status sst = launch_sed(p, a, t32, s);
    if (sst != CS_OK) return sst;

    const int wm = p->nmode == CS_NINV_PIXEL ? 2 : (p->shared_qu ? 0 : 1);
    const int sm = staging_mode(p, mode);
    // the staged kernel's workgroup holds at most 64 KiB of LDS: fewer wavefronts per workgroup
    // when the slices do not fit (same arithmetic, work only regrouped)
    int wpb = p->sched.waves_per_block;
    const size_t per_wave = wm == 0 ? stage_bytes(mode, sm, p->F) : 0;
    while (wpb > 1 && per_wave * (size_t)wpb > 65536) wpb >>= 1;
    a.waves_per_block = wpb;
    int64_t nblocks = (p->nunits + wpb - 1) / wpb;
    if (p->sched.blocks_per_cu > 0) nblocks = std::min<int64_t>(nblocks, (int64_t)p->sched.blocks_per_cu * kNumCu);
    if (nblocks < 1) nblocks = 1;
    const bool loop = nblocks * wpb < p->nunits;  // persistent grid: wavefronts loop over units
    const dim3 grid((unsigned)nblocks), block((unsigned)(64 * wpb));
    const size_t lds = per_wave * (size_t)wpb;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (p->timing) {
        if (p->events_used == p->events.size()) {
            hipEvent_t x0, x1;
            CSI_HIP(hipEventCreate(&x0));
            CSI_HIP(hipEventCreate(&x1));
            p->events.emplace_back(x0, x1);
        }
        e0 = p->events[p->events_used].first;
        e1 = p->events[p->events_used].second;
        ++p->events_used;
        CSI_HIP(hipEventRecord(e0, s));
    }
    if (mode == CS_FP64)
        launch_pixel_g<double, double>(want_grad, wm, sm, loop, lds, grid, block, s, a);
    else if (mode == CS_FP32_BULK)
        launch_pixel_g<float, float>(want_grad, wm, sm, loop, lds, grid, block, s, a);
    else
        launch_pixel_g<float, double>(want_grad, wm, sm, loop, lds, grid, block, s, a);
    CSI_HIP(hipGetLastError());
    if (p->timing) CSI_HIP(hipEventRecord(e1, s));

    {
        // items per launch: the 1D grid stays below 2^31 workgroups
        const int64_t per_item = 1 + ((want_grad || cluster_f) ? (int64_t)kblocks : 0);
        const int per = (int)std::min<int64_t>(p->B, std::max<int64_t>(1, ((int64_t(1) << 31) - 1) / per_item));
        for (int b0 = 0; b0 < p->B; b0 += per) {
            const int nb = std::min(per, p->B - b0);
            const dim3 fgrid((unsigned)(per_item * nb));
            const int kb = (int)kblocks;
            if (want_grad && cluster_f)
                hipLaunchKernelGGL((k_fin_grad<true, true>), fgrid, dim3(kFinBlock), 0, s, a, b0, nb, kb, grad,
                                   cluster_f, neg2logl, status);
            else if (want_grad)
                hipLaunchKernelGGL((k_fin_grad<true, false>), fgrid, dim3(kFinBlock), 0, s, a, b0, nb, kb, grad,
                                   cluster_f, neg2logl, status);
            else if (cluster_f)
                hipLaunchKernelGGL((k_fin_grad<false, true>), fgrid, dim3(kFinBlock), 0, s, a, b0, nb, kb, grad,
                                   cluster_f, neg2logl, status);
            else
                hipLaunchKernelGGL((k_fin_grad<false, false>), fgrid, dim3(kFinBlock), 0, s, a, b0, nb, kb, grad,
                                   cluster_f, neg2logl, status);
            CSI_HIP(hipGetLastError());
        }
    }
    return CS_OK;
}

}  // namespace csi
