// Internal declarations shared by the library's translation units (host + device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "cs.h"

namespace csi {

constexpr int kChunk = 64;  // pixels per work unit = lanes of one wavefront
constexpr int kFMax = 32;   // largest supported band count (register tile)
constexpr int kSegLabPad = 16;  // records past the end of each seg_lab array (read, never used)
constexpr int kNumXcd = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each
constexpr int kNumCu = 256;
constexpr int kMaxGridY = 65535;  // largest grid dimension y

// Per-band constants, computed on the host in FP64 and stored once in the workspace.
struct BandDev {
    double w[2][kFMax];   // N^-1 per Stokes and band (band mode)
    double ld[kFMax];     // ln(nu / nu0_dust)
    double ls[kFMax];     // ln(nu / nu0_sync)
    double rd[kFMax];     // (nu / nu0_dust) * g(nu) / g(nu0_dust)
    double gs[kFMax];     // g(nu) / g(nu0_sync)
    double hk[kFMax];     // h nu / k  (kelvin)
    double hk0d;          // h nu0_dust / k
    double wsum[2];       // sum_f w[s][f]
    float wf[2][kFMax];   // FP32 copies for the FP32-bulk accumulation
    float ldf[kFMax];
    float lsf[kFMax];
    float wsumf[2];
    float bcf[kFMax][4];   // (w[0][f], ld[f], ls[f], 0) packed, FP32 copies
    double bcd[kFMax][4];  // the same in FP64
    double isw[2];         // 1 / sqrt(wsum[s]): the first Cholesky pivot's inverse
    double iswf[2];        // the same of wsum[s] rounded to FP32 (the FP32-accumulation m00)
};

// One label layout: the labelling of one item, or the labelling shared by every item.
struct LayoutDev {
    const int32_t *labels;  // caller's labels [3][P]
    uint64_t *keys;         // [np2] sort scratch
    int32_t *order;         // [P64] processing slot -> original pixel index
    uint64_t *head;         // [nchunk_max] bit i set = lane i starts a segment
    int32_t *seg_base;      // [nchunk_max + 1] first segment of each chunk
    int4 *seg_lab;          // [P64] (l_d, l_T, l_s, first slot) of each segment
    int32_t *seg_perm[3];   // [P64] segments grouped by the cluster of labelling j
    int32_t *seg_off[3];    // [K_j + 1]
    int32_t *excl;          // [P] excluded pixels (label -1), in no particular order
    int32_t *counts;        // [4]: n_included, n_segments, label error, n_excluded
    int32_t k[3];
    int32_t n_incl;         // filled after prepare
    int32_t nchunks;
    int32_t nseg;
    int32_t pad;
};

struct ItemDev {
    int32_t layout;
    int32_t k[3];
    int64_t xoff;      // first packed parameter
    int64_t dchunk0;   // first packed data chunk
    int64_t tab_off;   // first table row (rows of F elements)
    int64_t part_off;  // first segment partial
};

struct EvalArgs {
    const int2 *units;  // (item, chunk) per work unit, item-major
    int64_t nunits;
    const ItemDev *items;
    const LayoutDev *layouts;
    const void *dpack;   // packed d, [chunk][2][F][64]
    const void *wpack;   // packed per-pixel N^-1 (PIXEL mode)
    void *tables;        // per item: PD [K_d][F], BTDT [K_T][F][2], SS [K_s][F]
    const BandDev *band;
    double *partials;    // [segment][4]: f, dF/dbeta_d, dF/dT_d, dF/dbeta_s
    int32_t *istatus;    // [B] status bits of the current evaluation
    const int32_t *active;  // nullable [B]: 0 = skip item (converged optimiser items)
    const double *x;     // packed parameters
    int32_t nitems;
    int32_t nfreq;
    int32_t xcd_remap;
    int32_t waves_per_block;
};

// Workspace regions (byte offsets, 256-aligned), see carve_workspace().
struct WsLayout {
    size_t band, items, layouts, units, keys, order, head, seg_base, seg_lab, seg_perm, seg_off,
        counts, excl, dpack, wpack, tables, partials, segoff, istatus, total;
    size_t keys_stride, p64, nchunk_max, np2, kmax[3];
};

}  // namespace csi

struct cs_problem {
    // descriptor copies
    int32_t F = 0, P = 0, B = 0;
    double nu0d = 0, nu0s = 0, tcmb = 0;
    cs_precision prec = CS_FP64;
    cs_dtype dtype = CS_DTYPE_F64;
    const void *d = nullptr;
    int64_t d_stride = 0;
    cs_ninv_mode nmode = CS_NINV_BAND;
    std::vector<double> ninv_band;
    const void *ninv_pixel = nullptr;
    int64_t ninv_stride = 0;
    const int32_t *labels = nullptr;
    int64_t labels_stride = 0;
    std::vector<double> freqs;
    std::vector<int32_t> ncl;  // [B][3]
    // derived
    bool shared_qu = true;  // band weights equal for Q and U
    int32_t L = 1;          // number of label layouts
    int key_bits[4] = {0, 0, 0, 0};
    std::vector<int64_t> xoff;     // [B+1]
    int64_t kmax_item = 1;         // largest parameter count of one item
    std::vector<int64_t> taboff;   // [B+1] table rows
    int64_t trows_max = 0;         // largest table row count of one item
    std::vector<int64_t> segoff;   // [B+1] segments of the items (after prepare)
    csi::WsLayout ws;
    char *wsp = nullptr;
    int device = 0;
    bool prepared = false;
    // host mirrors filled by prepare
    std::vector<csi::ItemDev> items;
    std::vector<csi::LayoutDev> layouts;
    int64_t nunits = 0;
    cs_schedule sched{2, 0, 1, 2};
    // kernel timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    size_t events_used = 0;
};

namespace csi {

void set_error(const std::string &msg);
cs_status hip_fail(hipError_t e, const char *what);

#define CSI_HIP(call)                                          \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return csi::hip_fail(e_, #call); \
    } while (0)

// a1: segment preparation (cs_prep.hip)
cs_status prepare_layouts(cs_problem *p, hipStream_t s);
cs_status pack_data(cs_problem *p, hipStream_t s);
// Ascending bitonic sort of nlayouts arrays of n keys (n a power of two >= 2048) spaced lstride
// apart; layouts with active_layout[l] == 0 are skipped (active_layout nullable).
cs_status bitonic_sort(uint64_t *base, int64_t lstride, int64_t n, int nlayouts, const int32_t *active_layout,
                       hipStream_t s);
cs_status export_segments(cs_problem *p, int32_t item, int32_t j, int32_t *perm, int32_t *offsets,
                          hipStream_t s);

// a2-a7: one batched evaluation (cs_eval.hip)
EvalArgs make_eval_args(const cs_problem *p, const double *x, const int32_t *active);
// staging mode that a launch in arithmetic mode `mode` runs under the problem's schedule
int staging_mode(const cs_problem *p, cs_precision mode);
cs_status launch_sed(const cs_problem *p, const EvalArgs &a, bool fp32_tables, hipStream_t s);
cs_status launch_eval(cs_problem *p, const double *x, const int32_t *active, double *neg2logl,
                      double *grad, double *cluster_f, int32_t *status, bool want_grad,
                      cs_precision mode, hipStream_t s);

// component maps and the CMB map variance (cs_maps.hip)
// sorted: maps in processing order (slot i of an item = pixel order[i]) instead of pixel order
cs_status launch_maps(cs_problem *p, const double *x, double *maps, int64_t maps_stride, double *cmb_var,
                      int32_t *status, bool sorted, hipStream_t s);

// spherical K-means patching (cs_kmeans.hip)
size_t kmeans_bytes(int64_t n, int32_t ntasks, int64_t ktot);
cs_status kmeans_batch(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep, int64_t keep_stride,
                       const int32_t *k_host, const int32_t *init, int64_t init_stride, int32_t iters,
                       int32_t *labels, int64_t labels_stride, int32_t *keff, void *ws, hipStream_t s);
// the same on this device's library-owned scratch array; bytes = kmeans_bytes of the arguments
cs_status kmeans_batch_static(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep,
                              int64_t keep_stride, const int32_t *k_host, const int32_t *init, int64_t init_stride,
                              int32_t iters, int32_t *labels, int64_t labels_stride, int32_t *keff, size_t bytes,
                              hipStream_t s);

// a8: batched projected L-BFGS (cs_optim.hip)
size_t optimizer_bytes(const cs_problem *p, int32_t m);
cs_status optimize(cs_problem *p, const cs_optim_opts *o, const double *lo, const double *hi,
                   double *x, double *f, int32_t *iters, int32_t *status, int64_t *nevals, void *ws,
                   size_t bytes, int32_t resume, int32_t max_replays, int32_t *running, hipStream_t s);

}  // namespace csi
