// Batched bound-constrained optimisers on the device (a8): projected L-BFGS and AdaTopK, driven by
// HIP-graph replays (a9).
//
// Every item (realization / configuration) runs its own optimisation in the internal box
// y = (x - l)/(u - l) in [0,1]^K (paper App. A.1); trial points are clamped to the box, the
// bound logic of Alg. 1.  One graph replay holds `iters_per_graph` steps; a step is one batched
// evaluation of every active item followed by k_opt_update, a small state machine per item:
//   INIT / REINIT : take F, g at the start point (REINIT keeps the curvature pairs)
//   SEARCH        : line-search test of the pending trial (Armijo, or F unchanged to 1e-12
//                   relative with g_trial.(y_trial - y) <= 0); accept -> curvature pair,
//                   convergence test, new direction; reject -> halve the step (max_backtracks)
//   DONE          : converged, line-search failure, iteration limit or bad evaluation
// The direction is the two-loop recursion restricted to the free set (variables not held at a
// bound by the sign of their gradient).  Items that finish are masked out of the evaluation
// kernels through active[].  The host reads one counter after each replay.
#include <algorithm>
#include <vector>

#include "cs_device.h"

namespace csi {

enum : int32_t { ST_INIT = 0, ST_REINIT = 1, ST_SEARCH = 2, ST_DONE = 3 };

struct OptItem {
    double f, pg0, alpha, dec;
    int64_t nevals;
    int32_t state, status, iter, nbt, npairs, newest;
    int32_t iter0;  // iterations before this phase
    int32_t sd;     // the direction is -Pg
    // AdaTopK: objective scale, bias-correction powers, last accepted step, step limit
    double scale, b1t, b2t, aprev, amax;
    int32_t t, lim, hit, pad2;
};

struct OptArgs {
    OptItem *st;
    int32_t *active;
    int32_t *nactive;
    const double *fe;      // [B] objective at the trial (evaluation output)
    const int32_t *estat;  // [B] evaluation status
    const double *ge;      // [Ktot] physical gradient at the trial (evaluation output)
    double *y, *g, *p, *yt, *xt;  // [Ktot]
    double *S, *T;         // [m][Ktot]
    const double *lo, *hi;
    const int64_t *xoff;
    int64_t ktot;
    int32_t m, max_iter, max_backtracks, solver;
    double gtol, c1;
    double gsw;  // FP32 phase of the mixed-precision run: leave it at |Pg| <= gsw |Pg_0| (0 = off)
    int32_t *piv;  // [Ktot] AdaTopK pivots: -1 lower bound, +1 upper bound, 0 free
    double lr, b1, b2, eps, topk;
};

// An item's state record read through the scalar cache: it is the same for every thread of the
// item's workgroup, so it stays in scalar registers.
__device__ __forceinline__ OptItem load_uniform(const OptItem *p) {
    constexpr int kW = sizeof(OptItem) / 4;
    const cptr<uint32_t> q = (cptr<uint32_t>)as_const(p);
    uint32_t w[kW];
#pragma unroll
    for (int i = 0; i < kW; ++i) w[i] = q[i];
    OptItem s;
    __builtin_memcpy(&s, w, sizeof s);
    return s;
}

constexpr int kOptThreads = 256;   // block size of the small per-item kernels
constexpr int32_t kSwitch = 1 << 8;  // internal status bit: the item reached the FP32 phase's tolerance
constexpr double kFlatRel = 1e-12;  // relative change of F below which Armijo is not resolved

// Wave-level sums and maxima by DPP lane moves (VALU only, no LDS round trip): swap neighbouring
// lanes, then the lane pairs of each quad, mirror each half-row, mirror each row, so every lane
// of a 16-lane row holds that row's result; the four row results are then read in row order.
// Each step combines two lanes' values symmetrically, so the lanes of a row agree bit for bit and
// the result is independent of timing.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_f64(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}
constexpr int kDppSwap1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppSwap2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror
constexpr int kDppMirror = 0x140;      // row_mirror
__device__ __forceinline__ double wave_sum(double x) {
    x += dpp_f64<kDppSwap1>(x);
    x += dpp_f64<kDppSwap2>(x);
    x += dpp_f64<kDppHalfMirror>(x);
    x += dpp_f64<kDppMirror>(x);
    return ((lane_f64(x, 0) + lane_f64(x, 16)) + lane_f64(x, 32)) + lane_f64(x, 48);
}
__device__ __forceinline__ double wave_max(double x) {
    x = fmax(x, dpp_f64<kDppSwap1>(x));
    x = fmax(x, dpp_f64<kDppSwap2>(x));
    x = fmax(x, dpp_f64<kDppHalfMirror>(x));
    x = fmax(x, dpp_f64<kDppMirror>(x));
    return fmax(fmax(fmax(lane_f64(x, 0), lane_f64(x, 16)), lane_f64(x, 32)), lane_f64(x, 48));
}

// deterministic block sum of N values (the wave sums above, then the waves in order)
template <int N, int NT>
__device__ __forceinline__ void block_sum(double (&v)[N], double (*sh)[16]) {
    constexpr int NWV = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        v[n] = wave_sum(v[n]);
        if (NWV > 1 && lane == 0) sh[n][wave] = v[n];
    }
    if (NWV > 1) {
        __syncthreads();
#pragma unroll
        for (int n = 0; n < N; ++n) {
            double x = 0;
#pragma unroll
            for (int w = 0; w < NWV; ++w) x += sh[n][w];
            v[n] = lane_f64(x, 0);  // the same in every lane; held in scalar registers from here
        }
        __syncthreads();
    }
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double *sh) {
    constexpr int NWV = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    v = wave_max(v);
    if (NWV == 1) return v;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double x = sh[0];
#pragma unroll
    for (int w = 1; w < NWV; ++w) x = fmax(x, sh[w]);
    __syncthreads();
    return lane_f64(x, 0);
}

// Stopping tests after an accepted step, in order: the relative projected-gradient tolerance,
// the switch tolerance of the FP32 phase of a mixed-precision run, the phase's iteration budget.
__device__ __forceinline__ int32_t stop_test(const OptArgs &a, const OptItem &s, double pgn) {
    if (pgn <= a.gtol * s.pg0) return CS_ITEM_CONVERGED;
    if (pgn <= a.gsw * s.pg0) return kSwitch;
    if (s.iter - s.iter0 >= a.max_iter) return CS_ITEM_MAXITER;
    return 0;
}

__device__ __forceinline__ bool is_free(double y, double g) {
    return !((y <= 0.0 && g > 0.0) || (y >= 1.0 && g < 0.0));
}

__global__ __launch_bounds__(kOptThreads) void k_opt_init(OptArgs a, const double *x0, int32_t nitems) {
    const int item = blockIdx.x;
    const int64_t o = a.xoff[item], K = a.xoff[item + 1] - o;
    for (int64_t i = threadIdx.x; i < K; i += blockDim.x) {
        const double l = a.lo[o + i], u = a.hi[o + i];
        double yi = (x0[o + i] - l) / (u - l);
        yi = yi < 0.0 ? 0.0 : (yi > 1.0 ? 1.0 : yi);
        a.y[o + i] = yi;
        a.yt[o + i] = yi;
        a.xt[o + i] = l + yi * (u - l);
        if (a.solver == CS_SOLVER_ADATOPK) {
            a.piv[o + i] = yi <= 0.0 ? -1 : (yi >= 1.0 ? 1 : 0);
            a.S[o + i] = 0.0;  // first moment
            a.T[o + i] = 0.0;  // second moment
        }
    }
    if (threadIdx.x == 0) {
        OptItem s{};
        s.state = ST_INIT;
        s.scale = 1.0;
        s.b1t = 1.0;
        s.b2t = 1.0;
        s.aprev = 1.0;
        s.lim = -1;
        a.st[item] = s;
        a.active[item] = 1;
        if (item == 0) *a.nactive = nitems;
    }
}

// One optimiser step per active item (one workgroup of NT threads per item).  The two-loop
// recursion runs as fused passes over the item's vectors: the pass for pair j first applies the
// previous pair's update, then forms pair j's products, so each pair costs one pass per loop.
template <int NT>
__global__ __launch_bounds__(NT) void k_opt_update(OptArgs a) {
    const int item = blockIdx.x;
    if (!as_const(a.active)[item]) return;
    __shared__ double red[8][16];
    __shared__ double rho[32], alp[32];
    const int64_t o = a.xoff[item], K = a.xoff[item + 1] - o;
    const int tid = threadIdx.x;
    const double *lo = a.lo + o, *hi = a.hi + o, *ge = a.ge + o;
    double *y = a.y + o, *g = a.g + o, *p = a.p + o, *yt = a.yt + o, *xt = a.xt + o;
    OptItem s = load_uniform(a.st + item);  // every thread holds the same copy, in scalar registers
    s.nevals += 1;
    const double fe = as_const(a.fe)[item];
    const int32_t est = as_const(a.estat)[item];
    const bool evalok = !(est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE)) && isfinite(fe);
    int32_t finish = 0;
    bool need_dir = false;

    if (s.state == ST_INIT || s.state == ST_REINIT) {
        if (!evalok) {
            finish = est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE);
            if (!finish) finish = CS_ITEM_NONFINITE;
        } else {
            double v[1] = {0.0};
            for (int64_t i = tid; i < K; i += NT) {
                const double gi = ge[i] * (hi[i] - lo[i]);
                g[i] = gi;
                if (is_free(y[i], gi)) v[0] += gi * gi;
            }
            block_sum<1, NT>(v, red);
            s.f = fe;
            if (s.state == ST_INIT) {
                s.pg0 = sqrt(v[0]);
                if (!isfinite(s.pg0))
                    finish = CS_ITEM_NONFINITE;
                else if (s.pg0 == 0.0)
                    finish = CS_ITEM_CONVERGED;
            }
            if (!finish && s.iter - s.iter0 >= a.max_iter) finish = CS_ITEM_MAXITER;
            need_dir = !finish;
        }
    } else if (s.state == ST_SEARCH) {
        // s = yt - y, t = g_trial - g (internal gradients): s.t, s.s, t.t and g_trial.s
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (evalok) {
            for (int64_t i = tid; i < K; i += NT) {
                const double si = yt[i] - y[i], gti = ge[i] * (hi[i] - lo[i]), ti = gti - g[i];
                v[0] += si * ti;
                v[1] += si * si;
                v[2] += ti * ti;
                v[3] += gti * si;
            }
        }
        block_sum<4, NT>(v, red);
        // Armijo, or (at the rounding floor of F) F unchanged and still non-increasing at the trial
        const bool flat = fabs(fe - s.f) <= kFlatRel * fabs(s.f) && v[3] <= 0.0;
        if (evalok && v[1] > 0.0 && (fe <= s.f + a.c1 * s.dec || flat)) {  // never accept a null step
            const bool keep = v[0] > 1e-12 * sqrt(v[1]) * sqrt(v[2]);
            const int nw = keep ? (s.newest + 1) % a.m : s.newest;
            double *Sn = a.S + (int64_t)nw * a.ktot + o, *Tn = a.T + (int64_t)nw * a.ktot + o;
            double pg[1] = {0.0};
            for (int64_t i = tid; i < K; i += NT) {
                const double gi = ge[i] * (hi[i] - lo[i]);
                if (keep) {
                    Sn[i] = yt[i] - y[i];
                    Tn[i] = gi - g[i];
                }
                y[i] = yt[i];
                g[i] = gi;
                if (is_free(yt[i], gi)) pg[0] += gi * gi;
            }
            block_sum<1, NT>(pg, red);
            if (keep) {
                s.newest = nw;
                if (s.npairs < a.m) s.npairs += 1;
            }
            s.f = fe;
            s.iter += 1;
            finish = stop_test(a, s, sqrt(pg[0]));
            need_dir = !finish;
        } else {
            s.nbt += 1;
            if (s.nbt > a.max_backtracks)
                finish = CS_ITEM_LS_FAIL;
            else
                s.alpha *= 0.5;
        }
    }

    if (need_dir) {
        // Two-loop recursion on the free set, q = P g held in p.  Backward (newest pair first):
        // the pass of pair j applies the pending q -= alpha t of the previous used pair, then forms
        // the masked s.t, s.s, t.t and s.q of pair j.  Forward (oldest first): the pass of pair j
        // applies gamma (first pass) and the pending r += s (alpha - beta), then forms t.r.
        const int np = s.npairs, m = a.m;
        double gamma = 1.0;
        bool gamma_set = false;
        int used = 0;
        bool qinit = false;            // p holds q
        const double *pendT = nullptr;  // pending backward update
        double penda = 0.0;
        for (int c = 0; c < np; ++c) {
            const int j = ((s.newest - c) % m + m) % m;
            const double *Sj = a.S + (int64_t)j * a.ktot + o, *Tj = a.T + (int64_t)j * a.ktot + o;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t i = tid; i < K; i += NT) {
                const bool fr = is_free(y[i], g[i]);
                double q = qinit ? p[i] : (fr ? g[i] : 0.0);
                if (pendT && fr) q -= penda * pendT[i];
                if (!qinit || pendT) p[i] = q;
                if (fr) {
                    const double si = Sj[i], ti = Tj[i];
                    v[0] += si * ti;
                    v[1] += si * si;
                    v[2] += ti * ti;
                    v[3] += si * q;
                }
            }
            block_sum<4, NT>(v, red);
            qinit = true;
            pendT = nullptr;
            if (!(v[0] > 1e-12 * sqrt(v[1]) * sqrt(v[2])) || v[2] == 0.0) {
                if (tid == 0) rho[j] = 0.0;
                continue;
            }
            const double rj = 1.0 / v[0];
            if (!gamma_set) {
                gamma = v[0] / v[2];
                gamma_set = true;
            }
            const double aj = rj * v[3];
            if (tid == 0) {
                rho[j] = rj;
                alp[j] = aj;
            }
            pendT = Tj;
            penda = aj;
            ++used;
        }
        __syncthreads();  // rho / alp visible to every thread
        bool scaled = false;            // gamma applied
        const double *pendS = nullptr;  // pending forward update
        double pendc = 0.0;
        for (int c = np - 1; c >= 0; --c) {
            const int j = ((s.newest - c) % m + m) % m;
            const double rj = rho[j];
            if (rj == 0.0) continue;
            const double *Sj = a.S + (int64_t)j * a.ktot + o, *Tj = a.T + (int64_t)j * a.ktot + o;
            double v[1] = {0.0};
            for (int64_t i = tid; i < K; i += NT) {
                const bool fr = is_free(y[i], g[i]);
                double r = p[i];
                if (!scaled) {
                    if (pendT && fr) r -= penda * pendT[i];
                    r *= gamma;
                }
                if (pendS && fr) r += pendS[i] * pendc;
                p[i] = r;
                if (fr) v[0] += Tj[i] * r;
            }
            block_sum<1, NT>(v, red);
            scaled = true;
            pendT = nullptr;
            pendS = Sj;
            pendc = alp[j] - rj * v[0];
        }
        // final pass: remaining pending updates, p = -(H P g) on the free set, p.g, max |p|
        double v[2] = {0.0, 0.0};
        double pm = 0.0;
        for (int64_t i = tid; i < K; i += NT) {
            const bool fr = is_free(y[i], g[i]);
            double r = qinit ? p[i] : (fr ? g[i] : 0.0);
            if (!scaled) {
                if (pendT && fr) r -= penda * pendT[i];
                r *= gamma;
            }
            if (pendS && fr) r += pendS[i] * pendc;
            const double pi = fr ? -r : 0.0;
            p[i] = pi;
            v[0] += pi * g[i];
            v[1] += isfinite(pi) ? 0.0 : 1.0;
            pm = fmax(pm, fabs(pi));
        }
        block_sum<2, NT>(v, red);
        if (!(v[0] < 0.0) || v[1] != 0.0) {  // not a finite descent direction: clear memory, -Pg
            s.npairs = 0;
            s.newest = -1;
            used = 0;
            pm = 0.0;
            for (int64_t i = tid; i < K; i += NT) {
                const double pi = is_free(y[i], g[i]) ? -g[i] : 0.0;
                p[i] = pi;
                pm = fmax(pm, fabs(pi));
            }
        }
        pm = block_max<NT>(pm, red[0]);
        s.alpha = used ? 1.0 : (pm > 1.0 ? 1.0 / pm : 1.0);
        s.sd = used ? 0 : 1;
        s.nbt = 0;
    }

    if (!finish && s.state != ST_DONE) {
        // trial point y(alpha) = clip(y + alpha p, 0, 1) and the Armijo reference g.(yt - y).  The
        // clamp can turn a descent direction into an ascending step (a coordinate next to a bound
        // that p drives out of the box carries the descent); such a trial is not evaluated: unless
        // p is already -Pg, the memory is cleared and the search restarts along -Pg, whose clamped
        // steps always descend
        for (;;) {
            double v[1] = {0.0};
            for (int64_t i = tid; i < K; i += NT) {
                double t = y[i] + s.alpha * p[i];
                t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                yt[i] = t;
                xt[i] = lo[i] + t * (hi[i] - lo[i]);
                v[0] += g[i] * (t - y[i]);
            }
            block_sum<1, NT>(v, red);
            s.dec = v[0];
            if (s.dec < 0.0 || s.sd) break;
            s.npairs = 0;
            s.newest = -1;
            s.sd = 1;
            s.nbt = 0;
            double pm = 0.0;
            for (int64_t i = tid; i < K; i += NT) {
                const double pi = is_free(y[i], g[i]) ? -g[i] : 0.0;
                p[i] = pi;
                pm = fmax(pm, fabs(pi));
            }
            pm = block_max<NT>(pm, red[0]);
            s.alpha = pm > 1.0 ? 1.0 / pm : 1.0;
        }
        s.state = ST_SEARCH;
    }
    if (finish) {
        s.status |= finish;
        s.state = ST_DONE;
    }
    __syncthreads();
    if (tid == 0) {
        a.st[item] = s;
        if (finish) {
            a.active[item] = 0;
            atomicSub(a.nactive, 1);
        }
    }
}

// The same step with the work spread over a workgroup's registers: thread t owns elements k NT + t,
// k < PT (K <= NT PT), so every load instruction of a wavefront is one contiguous span.  y and g
// live in memory (the item's vectors stay in L2 between the phases): each phase reads what it
// needs, and y and g are written back as soon as they change, so only the direction (and the
// two-loop buffers) occupy registers across phases.  Each two-loop pass streams only its pair
// (s_j, t_j), requested during the previous pass's block reduction, and keeps the vector the next
// pass's pending update needs.  Each thread's partial sums run over its elements in order, as in
// k_opt_update; the workgroup size (and so the reduction tree) may differ.
template <int NT, int PT>
__global__ __launch_bounds__(NT) void k_opt_update_tile(OptArgs a) {
    const int item = blockIdx.x;
    if (!as_const(a.active)[item]) return;
    __shared__ double red[8][16];
    __shared__ double rho[32], alp[32];
    const int64_t o = as_const(a.xoff)[item], K = as_const(a.xoff)[item + 1] - o;
    const int tid = threadIdx.x;
    const double *lo = a.lo + o, *hi = a.hi + o, *ge = a.ge + o;
    double *yg = a.y + o, *gg = a.g + o, *pgl = a.p + o, *ytg = a.yt + o, *xtg = a.xt + o;
    OptItem s = load_uniform(a.st + item);  // every thread holds the same copy, in scalar registers
    s.nevals += 1;
    const double fe = as_const(a.fe)[item];
    const int32_t est = as_const(a.estat)[item];
    const bool evalok = !(est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE)) && isfinite(fe);
    int32_t finish = 0;
    bool need_dir = false;
    auto in = [&](int k) { return tid < K - (int64_t)k * NT; };
    auto at = [&](auto *v, int k) { return v + (int64_t)k * NT + tid; };  // element k of the thread
    // gradient at the trial in the box coordinates
    auto gtrial = [&](int k) { return *at(ge, k) * (*at(hi, k) - *at(lo, k)); };
    // phases re-read y and g from memory rather than holding them in registers
    auto phase_break = [] { asm volatile("" ::: "memory"); };

    if (s.state == ST_INIT || s.state == ST_REINIT) {
        if (!evalok) {
            finish = est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE);
            if (!finish) finish = CS_ITEM_NONFINITE;
        } else {
            double v[1] = {0.0};
#pragma unroll
            for (int k = 0; k < PT; ++k)
                if (in(k)) {
                    const double gk = gtrial(k);
                    *at(gg, k) = gk;
                    if (is_free(*at(yg, k), gk)) v[0] += gk * gk;
                }
            block_sum<1, NT>(v, red);
            s.f = fe;
            if (s.state == ST_INIT) {
                s.pg0 = sqrt(v[0]);
                if (!isfinite(s.pg0))
                    finish = CS_ITEM_NONFINITE;
                else if (s.pg0 == 0.0)
                    finish = CS_ITEM_CONVERGED;
            }
            if (!finish && s.iter - s.iter0 >= a.max_iter) finish = CS_ITEM_MAXITER;
            need_dir = !finish;
        }
    } else if (s.state == ST_SEARCH) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        if (evalok) {
#pragma unroll
            for (int k = 0; k < PT; ++k)
                if (in(k)) {
                    const double si = *at(ytg, k) - *at(yg, k), gti = gtrial(k), ti = gti - *at(gg, k);
                    v[0] += si * ti;
                    v[1] += si * si;
                    v[2] += ti * ti;
                    v[3] += gti * si;
                }
        }
        block_sum<4, NT>(v, red);
        const bool flat = fabs(fe - s.f) <= kFlatRel * fabs(s.f) && v[3] <= 0.0;
        if (evalok && v[1] > 0.0 && (fe <= s.f + a.c1 * s.dec || flat)) {  // never accept a null step
            const bool keep = v[0] > 1e-12 * sqrt(v[1]) * sqrt(v[2]);
            const int nw = keep ? (s.newest + 1) % a.m : s.newest;
            double *Sn = a.S + (int64_t)nw * a.ktot + o, *Tn = a.T + (int64_t)nw * a.ktot + o;
            double pg[1] = {0.0};
            phase_break();
#pragma unroll
            for (int k = 0; k < PT; ++k)
                if (in(k)) {
                    const double yti = *at(ytg, k), gti = gtrial(k);
                    if (keep) {
                        *at(Sn, k) = yti - *at(yg, k);
                        *at(Tn, k) = gti - *at(gg, k);
                    }
                    *at(yg, k) = yti;
                    *at(gg, k) = gti;
                    if (is_free(yti, gti)) pg[0] += gti * gti;
                }
            block_sum<1, NT>(pg, red);
            if (keep) {
                s.newest = nw;
                if (s.npairs < a.m) s.npairs += 1;
            }
            s.f = fe;
            s.iter += 1;
            finish = stop_test(a, s, sqrt(pg[0]));
            need_dir = !finish;
        } else {
            s.nbt += 1;
            if (s.nbt > a.max_backtracks)
                finish = CS_ITEM_LS_FAIL;
            else
                s.alpha *= 0.5;
        }
    }
    phase_break();

    double pv[PT];  // the direction, also the two-loop vector
    bool pv_new = need_dir;  // the direction differs from the stored one
    if (need_dir) {
        // two-loop recursion on the free set, q (in pv) = P g; carry = t (backward) or s (forward)
        // of the last used pair, whose update is applied at the start of the next pass.  Each
        // pass requests the next pair (s_j, t_j) before its block reduction, so the history stream
        // overlaps the reductions; the oldest pair, last of the backward pass, is the forward
        // pass's first.
        unsigned fr = 0;
        double carry[PT];
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const double gk = in(k) ? *at(gg, k) : 0.0;
            const bool f = in(k) && is_free(*at(yg, k), gk);
            fr |= (unsigned)f << k;
            pv[k] = f ? gk : 0.0;
            carry[k] = 0.0;
        }
        const int np = s.npairs, m = a.m;
        auto pair_at = [&](int c) { return ((s.newest - c) % m + m) % m; };
        double sn[PT], tn[PT];  // the pair of the coming pass
        auto fetch = [&](int j) {
            const double *Sj = a.S + (int64_t)j * a.ktot + o, *Tj = a.T + (int64_t)j * a.ktot + o;
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const int64_t kb = (int64_t)k * NT;
                const bool f = (fr >> k) & 1u;
                sn[k] = f ? (Sj + kb)[tid] : 0.0;
                tn[k] = f ? (Tj + kb)[tid] : 0.0;
            }
        };
        if (np > 0) fetch(pair_at(0));
        double gamma = 1.0;
        bool gamma_set = false;
        int used = 0;
        bool pend = false;
        double penda = 0.0;
        for (int c = 0; c < np; ++c) {
            const int j = pair_at(c);
            double v[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                // no free-set test: s, t and q are zero outside the free set, so those elements
                // add exact zeros
                if (pend) pv[k] -= penda * carry[k];
                const double si = sn[k], ti = tn[k];
                v[0] += si * ti;
                v[1] += si * si;
                v[2] += ti * ti;
                v[3] += si * pv[k];
                carry[k] = ti;
            }
            if (c + 1 < np) fetch(pair_at(c + 1));  // the oldest pair stays in sn, tn
            block_sum<4, NT>(v, red);
            if (!(v[0] > 1e-12 * sqrt(v[1]) * sqrt(v[2])) || v[2] == 0.0) {
                if (tid == 0) rho[j] = 0.0;
                pend = false;
                continue;
            }
            const double rj = 1.0 / v[0];
            if (!gamma_set) {
                gamma = v[0] / v[2];
                gamma_set = true;
            }
            const double aj = rj * v[3];
            if (tid == 0) {
                rho[j] = rj;
                alp[j] = aj;
            }
            pend = true;
            penda = aj;
            ++used;
        }
        __syncthreads();  // rho / alp visible to every thread
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            if (pend && ((fr >> k) & 1u)) pv[k] -= penda * carry[k];
            pv[k] *= gamma;
        }
        bool spend = false;
        double pendc = 0.0;
        // the forward pass over the pairs with rho != 0, oldest first; sn, tn hold the oldest
        auto next_used = [&](int c) {
            while (c >= 0 && rho[pair_at(c)] == 0.0) --c;
            return c;
        };
        int c = next_used(np - 1);
        if (c >= 0 && c != np - 1) fetch(pair_at(c));
        while (c >= 0) {
            const int j = pair_at(c);
            const double rj = rho[j];
            double v[1] = {0.0};
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                if (spend) pv[k] += carry[k] * pendc;
                const double si = sn[k];
                v[0] += tn[k] * pv[k];
                carry[k] = si;
            }
            const int cn = next_used(c - 1);
            if (cn >= 0) fetch(pair_at(cn));
            block_sum<1, NT>(v, red);
            spend = true;
            pendc = alp[j] - rj * v[0];
            c = cn;
        }
        // p = -(H P g) on the free set, p.g, max |p|
        phase_break();
        double v[2] = {0.0, 0.0};
        double pm = 0.0;
#pragma unroll
        for (int k = 0; k < PT; ++k) {
            const bool f = (fr >> k) & 1u;
            if (spend && f) pv[k] += carry[k] * pendc;
            const double pi = f ? -pv[k] : 0.0;
            pv[k] = pi;
            v[0] += pi * (in(k) ? *at(gg, k) : 0.0);
            v[1] += isfinite(pi) ? 0.0 : 1.0;
            pm = fmax(pm, fabs(pi));
        }
        block_sum<2, NT>(v, red);
        if (!(v[0] < 0.0) || v[1] != 0.0) {  // not a finite descent direction: clear memory, -Pg
            s.npairs = 0;
            s.newest = -1;
            used = 0;
            pm = 0.0;
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                pv[k] = ((fr >> k) & 1u) ? -*at(gg, k) : 0.0;
                pm = fmax(pm, fabs(pv[k]));
            }
        }
        pm = block_max<NT>(pm, red[0]);
        s.alpha = used ? 1.0 : (pm > 1.0 ? 1.0 / pm : 1.0);
        s.sd = used ? 0 : 1;
        s.nbt = 0;
    }

    if (!finish && s.state != ST_DONE) {
        if (!need_dir) {  // a backtracking step keeps its direction
#pragma unroll
            for (int k = 0; k < PT; ++k) pv[k] = in(k) ? *at(pgl, k) : 0.0;
        }
        // trial point y(alpha) = clip(y + alpha p, 0, 1) and the Armijo reference g.(yt - y); a
        // clamped step that does not descend restarts the search along -Pg (as in k_opt_update)
        for (;;) {
            phase_break();
            double v[1] = {0.0};
#pragma unroll
            for (int k = 0; k < PT; ++k)
                if (in(k)) {
                    const double yk = *at(yg, k);
                    double t = yk + s.alpha * pv[k];
                    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                    *at(ytg, k) = t;
                    *at(xtg, k) = *at(lo, k) + t * (*at(hi, k) - *at(lo, k));
                    v[0] += *at(gg, k) * (t - yk);
                }
            block_sum<1, NT>(v, red);
            s.dec = v[0];
            if (s.dec < 0.0 || s.sd) break;
            s.npairs = 0;
            s.newest = -1;
            s.sd = 1;
            s.nbt = 0;
            pv_new = true;
            double pm = 0.0;
            phase_break();
#pragma unroll
            for (int k = 0; k < PT; ++k) {
                const double gk = in(k) ? *at(gg, k) : 0.0;
                pv[k] = (in(k) && is_free(*at(yg, k), gk)) ? -gk : 0.0;
                pm = fmax(pm, fabs(pv[k]));
            }
            pm = block_max<NT>(pm, red[0]);
            s.alpha = pm > 1.0 ? 1.0 / pm : 1.0;
        }
        s.state = ST_SEARCH;
    }
    if (pv_new) {
#pragma unroll
        for (int k = 0; k < PT; ++k)
            if (in(k)) *at(pgl, k) = pv[k];
    }
    if (finish) {
        s.status |= finish;
        s.state = ST_DONE;
    }
    __syncthreads();
    if (tid == 0) {
        a.st[item] = s;
        if (finish) {
            a.active[item] = 0;
            atomicSub(a.nactive, 1);
        }
    }
}

// ---------------------------------------------------------------------------------------------
// AdaTopK (paper App. A), one workgroup per item.  Each iteration: release the pinned bounds whose
// descent direction points into the box (the largest scores p_i g_i, max(1, floor(topk n)) of
// them), stop on the projected-gradient test, rescale the objective and the moments when the
// scaled gradient norm leaves [1e-15, 1e15], take the AdaBelief direction on the free set, limit
// the step by the nearest bound (pinning it at once when the limit is zero), then backtrack from
// min(limit, 1, 2 x last step): Armijo for a descent step, a strict decrease otherwise, or the flat-F
// rule.  A failed search resets the moments once; a failure with fresh moments stops the item.
// ---------------------------------------------------------------------------------------------
// best (value, index) over a workgroup: the largest value (kMax) or the smallest, ties to the
// lowest index; every thread receives the result
template <int NT, bool kMax>
__device__ __forceinline__ void block_best(double &v, int64_t &idx, double *shv, int64_t *shi) {
    constexpr int NWV = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto better = [](double va, int64_t ia, double vb, int64_t ib) {
        if (ib < 0) return false;
        if (ia < 0) return true;
        if (kMax ? (vb > va) : (vb < va)) return true;
        return vb == va && ib < ia;
    };
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v, off, 64);
        const int64_t oi = __shfl_xor(idx, off, 64);
        if (better(v, idx, ov, oi)) {
            v = ov;
            idx = oi;
        }
    }
    if (NWV == 1) return;
    if (lane == 0) {
        shv[wave] = v;
        shi[wave] = idx;
    }
    __syncthreads();
    v = shv[0];
    idx = shi[0];
    for (int w = 1; w < NWV; ++w)
        if (better(v, idx, shv[w], shi[w])) {
            v = shv[w];
            idx = shi[w];
        }
    __syncthreads();
}

template <int NT>
__global__ __launch_bounds__(NT) void k_ada_update(OptArgs a) {
    const int item = blockIdx.x;
    if (!as_const(a.active)[item]) return;
    __shared__ double red[8][16];
    __shared__ double bv[16];
    __shared__ int64_t bi[16];
    const int64_t o = a.xoff[item], K = a.xoff[item + 1] - o;
    const int tid = threadIdx.x;
    const double *lo = a.lo + o, *hi = a.hi + o, *ge = a.ge + o;
    double *y = a.y + o, *g = a.g + o, *d = a.p + o, *yt = a.yt + o, *xt = a.xt + o;
    double *mm = a.S + o, *vv = a.T + o;
    int32_t *piv = a.piv + o;
    OptItem s = load_uniform(a.st + item);  // every thread holds the same copy, in scalar registers
    s.nevals += 1;
    const double fe = as_const(a.fe)[item];
    const int32_t est = as_const(a.estat)[item];
    const bool evalok = !(est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE)) && isfinite(fe);
    int32_t finish = 0;
    bool iterate = false;  // start a new iteration from the current point

    if (s.state == ST_INIT || s.state == ST_REINIT) {
        if (!evalok) {
            finish = est & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE);
            if (!finish) finish = CS_ITEM_NONFINITE;
        } else {
            for (int64_t i = tid; i < K; i += NT) g[i] = ge[i] * (hi[i] - lo[i]);
            s.f = fe;
            iterate = true;
        }
    } else if (s.state == ST_SEARCH) {
        // g.(y_t - y), |y_t - y|^2 and g_t.(y_t - y) at the evaluated trial
        double v[3] = {0.0, 0.0, 0.0};
        for (int64_t i = tid; i < K; i += NT) {
            const double st = yt[i] - y[i];
            v[0] += g[i] * st;
            v[1] += st * st;
            v[2] += ge[i] * (hi[i] - lo[i]) * st;
        }
        block_sum<3, NT>(v, red);
        bool ok = false;
        if (evalok && v[1] > 0.0) {
            const bool dec_ok = v[0] < 0.0 ? (fe <= s.f + a.c1 * v[0]) : (fe < s.f);
            ok = dec_ok || (fabs(fe - s.f) <= kFlatRel * fabs(s.f) && v[2] <= 0.0);
        }
        if (ok) {
            s.aprev = s.alpha;
            for (int64_t i = tid; i < K; i += NT) {
                y[i] = yt[i];
                g[i] = ge[i] * (hi[i] - lo[i]);
            }
            if (s.hit && tid == 0) piv[s.lim] = d[s.lim] > 0.0 ? 1 : -1;
            s.f = fe;
            s.iter += 1;
            iterate = true;
        } else {
            s.nbt += 1;
            if (s.nbt > a.max_backtracks) {
                if (s.t <= 1) {
                    finish = CS_ITEM_LS_FAIL;
                } else {  // reset the moments once and start again from the same point
                    for (int64_t i = tid; i < K; i += NT) {
                        mm[i] = 0.0;
                        vv[i] = 0.0;
                    }
                    s.t = 0;
                    s.b1t = s.b2t = 1.0;
                    s.aprev = 1.0;
                    s.iter += 1;
                    iterate = true;
                }
            } else {
                s.alpha *= 0.5;
                s.hit = (s.lim >= 0 && s.alpha == s.amax) ? 1 : 0;
            }
        }
    }
    __syncthreads();  // pivot and point updates visible to the whole workgroup

    bool trial = !finish && s.state == ST_SEARCH && !iterate;  // a halved step of the same direction
    while (iterate && !finish) {
        // 1. Top-K release among the pinned coordinates with a positive score p_i g_i
        double cnt[1] = {0.0};
        for (int64_t i = tid; i < K; i += NT)
            if (piv[i] != 0 && piv[i] * g[i] > 0.0) cnt[0] += 1.0;
        block_sum<1, NT>(cnt, red);
        const int64_t ncand = (int64_t)cnt[0];
        if (ncand > 0) {
            int64_t nrel = (int64_t)floor(a.topk * (double)ncand);
            if (nrel < 1) nrel = 1;
            if (nrel >= ncand) {
                for (int64_t i = tid; i < K; i += NT)
                    if (piv[i] != 0 && piv[i] * g[i] > 0.0) piv[i] = 0;
            } else {
                for (int64_t r = 0; r < nrel; ++r) {
                    double bvv = 0.0;
                    int64_t bix = -1;
                    for (int64_t i = tid; i < K; i += NT)
                        if (piv[i] != 0 && piv[i] * g[i] > 0.0) {
                            const double sc = piv[i] * g[i];
                            if (bix < 0 || sc > bvv) {
                                bvv = sc;
                                bix = i;
                            }
                        }
                    block_best<NT, true>(bvv, bix, bv, bi);
                    if (bix < 0) break;
                    if (tid == 0) piv[bix] = 0;
                    __syncthreads();
                }
            }
        }
        __syncthreads();
        // 2. projected gradient and the stopping tests
        double pg[1] = {0.0};
        for (int64_t i = tid; i < K; i += NT)
            if (piv[i] == 0) pg[0] += g[i] * g[i];
        block_sum<1, NT>(pg, red);
        const double pgn = sqrt(pg[0]);
        if (s.state == ST_INIT) {
            s.pg0 = pgn;
            if (!isfinite(pgn)) {
                finish = CS_ITEM_NONFINITE;
                break;
            }
        }
        finish = stop_test(a, s, pgn);
        if (finish) break;
        s.state = ST_SEARCH;  // any later pass of this loop is a continuation
        // 3. rescaling of the objective scale and the moments
        const double cpg = s.scale * pgn;
        double fs = 1.0;
        if (cpg < 1e-15 || cpg > 1e15) {
            fs = 1.0 / cpg;
            s.scale *= fs;
        }
        // 4. AdaBelief on the scaled projected gradient; 5. distance to the nearest bound
        s.t += 1;
        s.b1t *= a.b1;
        s.b2t *= a.b2;
        double amin = 0.0;
        int64_t lim = -1;
        for (int64_t i = tid; i < K; i += NT) {
            double m = mm[i], v = vv[i];
            if (fs != 1.0) {
                m *= fs;
                v *= fs * fs;
            }
            const double gi = piv[i] != 0 ? 0.0 : s.scale * g[i];
            m = a.b1 * m + (1.0 - a.b1) * gi;
            const double dv = gi - m;
            v = a.b2 * v + (1.0 - a.b2) * dv * dv + a.eps;
            mm[i] = m;
            vv[i] = v;
            const double mh = m / (1.0 - s.b1t), vh = v / (1.0 - s.b2t);
            const double di = piv[i] != 0 ? 0.0 : -a.lr * mh / (sqrt(vh) + a.eps);
            d[i] = di;
            if (piv[i] == 0 && di != 0.0) {
                const double ai = di > 0.0 ? (1.0 - y[i]) / di : -y[i] / di;
                if (lim < 0 || ai < amin) {
                    amin = ai;
                    lim = i;
                }
            }
        }
        block_best<NT, false>(amin, lim, bv, bi);
        s.amax = lim >= 0 ? amin : INFINITY;
        s.lim = (int32_t)lim;
        __syncthreads();  // d complete before any thread reads another's entry
        if (lim >= 0 && amin <= 0.0) {  // zero step to the bound: pin it without an evaluation
            if (tid == 0) {
                const bool up = d[lim] > 0.0;
                piv[lim] = up ? 1 : -1;
                y[lim] = up ? 1.0 : 0.0;
            }
            s.iter += 1;
            __syncthreads();
            continue;
        }
        // 6. first trial step
        const double a0 = 2.0 * s.aprev < 1.0 ? 2.0 * s.aprev : 1.0;
        s.alpha = s.amax < a0 ? s.amax : a0;
        s.hit = (lim >= 0 && s.alpha == s.amax) ? 1 : 0;
        s.nbt = 0;
        trial = true;
        break;
    }

    if (finish) {
        s.status |= finish;
        s.state = ST_DONE;
    } else if (trial) {
        for (int64_t i = tid; i < K; i += NT) {
            double t = y[i] + s.alpha * d[i];
            t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
            if (s.hit && i == s.lim) t = d[i] > 0.0 ? 1.0 : 0.0;
            yt[i] = t;
            xt[i] = lo[i] + t * (hi[i] - lo[i]);
        }
        s.state = ST_SEARCH;
    }
    __syncthreads();
    if (tid == 0) {
        a.st[item] = s;
        if (finish) {
            a.active[item] = 0;
            atomicSub(a.nactive, 1);
        }
    }
}

// Start of the FP64-accumulation phase of a mixed-precision run: every item that stopped in the
// FP32 phase for a reason other than convergence or a bad evaluation (its line search failed, it
// reached the switch tolerance or spent the phase's iteration budget) continues from its point with
// its curvature pairs and a fresh budget.
__global__ __launch_bounds__(kOptThreads) void k_opt_repolish(OptArgs a) {
    const int item = blockIdx.x;
    OptItem *s = a.st + item;
    constexpr int32_t kResume = CS_ITEM_LS_FAIL | CS_ITEM_MAXITER | kSwitch;
    if (!(s->state == ST_DONE && (s->status & kResume) && !(s->status & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE))))
        return;
    const int64_t o = a.xoff[item], K = a.xoff[item + 1] - o;
    for (int64_t i = threadIdx.x; i < K; i += blockDim.x) {
        a.yt[o + i] = a.y[o + i];
        a.xt[o + i] = a.lo[o + i] + a.y[o + i] * (a.hi[o + i] - a.lo[o + i]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s->status &= ~kResume;
        s->state = ST_REINIT;
        s->iter0 = s->iter;
        a.active[item] = 1;
        atomicAdd(a.nactive, 1);
    }
}

// x, f, iters, status and nevals of every item.  An item still running carries CS_ITEM_RUNNING when
// the caller's replay limit stopped the run (paused), else CS_ITEM_MAXITER (the replay bound).  When
// the run is paused before its FP64-accumulation phase (polish_pending), an item that has left the
// FP32 phase without converging will continue too, and is reported running.
__global__ __launch_bounds__(kOptThreads) void k_opt_output(OptArgs a, double *x, double *f, int32_t *iters,
                                                            int32_t *status, int64_t *nevals, int32_t paused,
                                                            int32_t polish_pending) {
    const int item = blockIdx.x;
    OptItem s = a.st[item];
    const int64_t o = a.xoff[item], K = a.xoff[item + 1] - o;
    for (int64_t i = threadIdx.x; i < K; i += blockDim.x)
        x[o + i] = a.lo[o + i] + a.y[o + i] * (a.hi[o + i] - a.lo[o + i]);
    if (threadIdx.x == 0) {
        constexpr int32_t kResume = CS_ITEM_LS_FAIL | CS_ITEM_MAXITER | kSwitch;
        int32_t stt = s.status;
        if (s.state != ST_DONE) {
            stt |= paused ? CS_ITEM_RUNNING : CS_ITEM_MAXITER;
        } else if (polish_pending && (stt & kResume) && !(stt & (CS_ITEM_NOT_PD | CS_ITEM_NONFINITE))) {
            stt = (stt & ~kResume) | CS_ITEM_RUNNING;
        }
        stt &= ~kSwitch;
        f[item] = s.f;
        iters[item] = s.iter;
        status[item] = stt;
        if (nevals) nevals[item] = s.nevals;
    }
}

// ---------------------------------------------------------------------------------------------
// host driver
// ---------------------------------------------------------------------------------------------
static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// First record of the optimiser workspace: what the state belongs to and how far the run is.  The
// rest of the workspace (per-item records, vectors, curvature pairs) holds no pointers, so a byte
// copy of the workspace is a complete checkpoint.
struct OptHeader {
    uint64_t magic;
    int64_t ktot;
    int32_t nitems, m, solver, precision;
    int32_t phase;   // 0: first (working-precision) phase; 1: FP64-accumulation phase started
    int32_t phases;  // 1, or 2 for a mixed-precision run
    int64_t replays; // graph replays so far (all calls)
};
constexpr uint64_t kOptMagic = 0x6373306f70743031ull;  // state format 1

size_t optimizer_bytes(const cs_problem *p, int32_t m) {
    const size_t B = (size_t)p->B, K = (size_t)p->xoff[p->B];
    size_t t = al256(sizeof(OptHeader));
    t += al256(sizeof(OptItem) * B);
    t += al256(sizeof(int32_t) * B) * 2 + al256(sizeof(int32_t));
    t += al256(sizeof(double) * B);
    t += al256(sizeof(double) * K) * 6;
    t += al256(sizeof(double) * K * (size_t)m) * 2;
    t += al256(sizeof(int32_t) * K);  // AdaTopK pivots
    return t;
}

cs_status optimize(cs_problem *p, const cs_optim_opts *o, const double *lo, const double *hi, double *x, double *f,
                   int32_t *iters, int32_t *status, int64_t *nevals, void *ws, size_t bytes, int32_t resume,
                   int32_t max_replays, int32_t *running, hipStream_t caller) {
    const int B = p->B;
    const int64_t K = p->xoff[B];
    int64_t kmax = 0;
    for (int b = 0; b < B; ++b) kmax = std::max<int64_t>(kmax, p->xoff[b + 1] - p->xoff[b]);
    if (bytes < optimizer_bytes(p, o->m)) {
        set_error("optimizer workspace too small");
        return CS_E_WORKSPACE;
    }
    char *w = (char *)ws;
    size_t off = 0;
    auto take = [&](size_t n) {
        char *r = w + off;
        off += al256(n);
        return r;
    };
    OptHeader *hdr_dev = (OptHeader *)take(sizeof(OptHeader));
    OptArgs a;
    a.st = (OptItem *)take(sizeof(OptItem) * B);
    a.active = (int32_t *)take(sizeof(int32_t) * B);
    int32_t *estat = (int32_t *)take(sizeof(int32_t) * B);
    a.estat = estat;
    a.nactive = (int32_t *)take(sizeof(int32_t));
    double *fe = (double *)take(sizeof(double) * B);
    a.fe = fe;
    double *ge = (double *)take(sizeof(double) * K);
    a.ge = ge;
    a.y = (double *)take(sizeof(double) * K);
    a.g = (double *)take(sizeof(double) * K);
    a.p = (double *)take(sizeof(double) * K);
    a.yt = (double *)take(sizeof(double) * K);
    a.xt = (double *)take(sizeof(double) * K);
    a.S = (double *)take(sizeof(double) * K * o->m);
    a.T = (double *)take(sizeof(double) * K * o->m);
    a.piv = (int32_t *)take(sizeof(int32_t) * K);
    a.lo = lo;
    a.hi = hi;
    a.xoff = (const int64_t *)(p->wsp + p->ws.items + sizeof(ItemDev) * (size_t)B);
    a.ktot = K;
    a.m = o->m;
    a.max_iter = o->max_iter;
    a.max_backtracks = o->max_backtracks;
    a.gtol = o->gtol_rel;
    a.c1 = o->c1;
    a.solver = o->solver;
    a.lr = o->lr;
    a.b1 = o->beta1;
    a.b2 = o->beta2;
    a.eps = o->eps;
    a.topk = o->topk;
    const int phases = (p->prec == CS_FP32_BULK && o->fp64_polish) ? 2 : 1;

    CSI_HIP(hipStreamSynchronize(caller));
    OptHeader hdr{};
    if (resume) {
        CSI_HIP(hipMemcpy(&hdr, hdr_dev, sizeof hdr, hipMemcpyDeviceToHost));
        if (hdr.magic != kOptMagic || hdr.ktot != K || hdr.nitems != B || hdr.m != o->m || hdr.solver != o->solver ||
            hdr.precision != (int32_t)p->prec || hdr.phases != phases || hdr.phase < 0 || hdr.phase >= phases) {
            set_error("optimizer workspace does not hold a state of this problem shape, m, solver and precision");
            return CS_E_STATE;
        }
    } else {
        hdr.magic = kOptMagic;
        hdr.ktot = K;
        hdr.nitems = B;
        hdr.m = o->m;
        hdr.solver = o->solver;
        hdr.precision = (int32_t)p->prec;
        hdr.phase = 0;
        hdr.phases = phases;
        hdr.replays = 0;
    }
    hipStream_t s;
    CSI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    cs_status rc = CS_OK;
    const bool was_timing = p->timing;
    p->timing = false;  // no event records inside captured graphs
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int32_t *hcount = nullptr;
    int32_t nrun = 0;
    bool paused = false;
    do {
        hipError_t eh = hipHostMalloc((void **)&hcount, sizeof(int32_t), hipHostMallocDefault);
        if (eh != hipSuccess) {
            hcount = nullptr;
            rc = hip_fail(eh, "hipHostMalloc");
            break;
        }
        if (!resume) {
            hipLaunchKernelGGL(k_opt_init, dim3(B), dim3(kOptThreads), 0, s, a, x, B);
            hipError_t e0 = hipGetLastError();
            if (e0 != hipSuccess) {
                rc = hip_fail(e0, "k_opt_init");
                break;
            }
        }
        // bound on replays of one call: every item needs at most max_iter * (max_backtracks + 1) + 1
        // evaluations per phase
        const int64_t max_steps = (int64_t)(o->max_iter + 1) * (o->max_backtracks + 1) + 2;
        int64_t replays_left = max_replays > 0 ? max_replays : INT64_MAX;
        for (int ph = hdr.phase; ph < phases && rc == CS_OK; ++ph) {
            const cs_precision mode = (ph == 0) ? p->prec : CS_FP32_STORE;
            a.gsw = (phases == 2 && ph == 0) ? o->switch_rel : 0.0;
            if (ph > hdr.phase) {
                // entering the FP64-accumulation phase (not when resuming inside it)
                hipLaunchKernelGGL(k_opt_repolish, dim3(B), dim3(kOptThreads), 0, s, a);
                hipError_t e3 = hipGetLastError();
                if (e3 != hipSuccess) {
                    rc = hip_fail(e3, "k_opt_repolish");
                    break;
                }
                hdr.phase = ph;
            }
            hipError_t ecap = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (ecap != hipSuccess) {
                rc = hip_fail(ecap, "hipStreamBeginCapture");
                break;
            }
            for (int k = 0; k < o->iters_per_graph && rc == CS_OK; ++k) {
                rc = launch_eval(p, a.xt, a.active, fe, ge, nullptr, estat, true, mode, s);
                if (rc == CS_OK) {
                    if (o->solver == CS_SOLVER_ADATOPK && kmax <= 1024)
                        hipLaunchKernelGGL(k_ada_update<256>, dim3(B), dim3(256), 0, s, a);
                    else if (o->solver == CS_SOLVER_ADATOPK)
                        hipLaunchKernelGGL(k_ada_update<1024>, dim3(B), dim3(1024), 0, s, a);
                    else if (kmax <= 64 * 8)
                        hipLaunchKernelGGL((k_opt_update_tile<64, 8>), dim3(B), dim3(64), 0, s, a);
                    else if (kmax <= 512 * 15)  // fits its registers without spilling
                        hipLaunchKernelGGL((k_opt_update_tile<512, 15>), dim3(B), dim3(512), 0, s, a);
                    else if (kmax <= 512 * 16)
                        hipLaunchKernelGGL((k_opt_update_tile<512, 16>), dim3(B), dim3(512), 0, s, a);
                    else
                        hipLaunchKernelGGL(k_opt_update<1024>, dim3(B), dim3(1024), 0, s, a);
                    hipError_t eu = hipGetLastError();
                    if (eu != hipSuccess) rc = hip_fail(eu, "k_opt_update");
                }
            }
            hipError_t ec = hipStreamEndCapture(s, &graph);
            if (rc != CS_OK) break;
            if (ec != hipSuccess) {
                rc = hip_fail(ec, "hipStreamEndCapture");
                break;
            }
            ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ec != hipSuccess) {
                rc = hip_fail(ec, "hipGraphInstantiate");
                break;
            }
            // the active count of a resumed run decides whether its phase still has work
            ec = hipMemcpyAsync(hcount, a.nactive, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            if (ec == hipSuccess) ec = hipStreamSynchronize(s);
            if (ec != hipSuccess) {
                rc = hip_fail(ec, "optimizer state read");
                break;
            }
            int64_t steps = 0;
            while (*hcount > 0 && steps < max_steps) {
                if (replays_left <= 0) {
                    paused = true;
                    break;
                }
                hipError_t e1 = hipGraphLaunch(exec, s);
                if (e1 == hipSuccess) e1 = hipMemcpyAsync(hcount, a.nactive, sizeof(int32_t), hipMemcpyDeviceToHost, s);
                if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
                if (e1 != hipSuccess) {
                    rc = hip_fail(e1, "optimizer graph replay");
                    break;
                }
                steps += o->iters_per_graph;
                --replays_left;
                ++hdr.replays;
            }
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            exec = nullptr;
            graph = nullptr;
            if (paused) break;
        }
        if (rc != CS_OK) break;
        const int32_t polish_pending = paused && hdr.phase + 1 < phases;
        hipError_t e2 = hipMemcpyAsync(hdr_dev, &hdr, sizeof hdr, hipMemcpyHostToDevice, s);
        if (e2 == hipSuccess) {
            hipLaunchKernelGGL(k_opt_output, dim3(B), dim3(kOptThreads), 0, s, a, x, f, iters, status, nevals,
                               (int32_t)paused, polish_pending);
            e2 = hipGetLastError();
        }
        std::vector<int32_t> hst;
        if (e2 == hipSuccess && paused) {  // items reported running, for the caller's count
            hst.resize(B);
            e2 = hipMemcpyAsync(hst.data(), status, sizeof(int32_t) * B, hipMemcpyDeviceToHost, s);
        }
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        if (e2 != hipSuccess) rc = hip_fail(e2, "k_opt_output");
        for (int32_t v : hst) nrun += (v & CS_ITEM_RUNNING) ? 1 : 0;
    } while (false);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (hcount) (void)hipHostFree(hcount);
    (void)hipStreamDestroy(s);
    p->timing = was_timing;
    if (running) *running = nrun;
    return rc;
}

}  // namespace csi
