// Segment preparation (once per clustering).
//
// Patches are disjoint pixel sets and each spectral parameter has its own patching (paper
// Sec. 2.2-2.3).  The evaluation kernels want the pixels of one item ordered so that every
// 64-pixel chunk (one wavefront) holds few runs of constant (l_d, l_T, l_s), and every data
// byte is streamed once, coalesced.  Everything here runs on the device:
//   1. keys  = (l_T, l_d, l_s, p) packed in 64 bits (unique), invalid labels flagged: the
//      segments of one T_d patch, and those of one beta_d patch inside it, are then
//      neighbours in the partials that the per-patch sums gather;
//   2. bitonic sort of the keys (unique keys => the order is deterministic);
//   3. chunk heads (ballot of run starts), per-chunk segment counts, segment triples;
//   4. per labelling, a bitonic sort of (label, segment) -> segment CSR;
//   5. the item's d (and per-pixel N^-1) gathered into [chunk][2][F][64] in working precision.
#include "cs_internal.h"

namespace csi {

constexpr int kSortTile = 2048;   // keys held in LDS by one workgroup
constexpr int kSortThreads = 1024;
constexpr uint64_t kInvalid = ~0ull;

__device__ __forceinline__ void cmpswap(uint64_t &a, uint64_t &b, bool asc) {
    if ((a > b) == asc) {
        uint64_t t = a;
        a = b;
        b = t;
    }
}

// All bitonic stages k = 2..kSortTile inside each tile (global index decides the direction).
__global__ __launch_bounds__(kSortThreads) void k_bitonic_presort(uint64_t *base, int64_t lstride,
                                                                   const int32_t *active_layout) {
    __shared__ uint64_t s[kSortTile];
    const int l = blockIdx.y;
    if (active_layout && !active_layout[l]) return;
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    uint64_t *a = base + l * lstride + tile0;
    const int t = threadIdx.x;
    s[t] = a[t];
    s[t + kSortThreads] = a[t + kSortThreads];
    __syncthreads();
    for (int k = 2; k <= kSortTile; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int i = 2 * j * (t / j) + (t % j);
            const bool asc = ((tile0 + i) & k) == 0;
            cmpswap(s[i], s[i + j], asc);
            __syncthreads();
        }
    }
    a[t] = s[t];
    a[t + kSortThreads] = s[t + kSortThreads];
}

// Stage k, steps j = kSortTile/2 .. 1 inside each tile.
__global__ __launch_bounds__(kSortThreads) void k_bitonic_merge_tile(uint64_t *base, int64_t lstride,
                                                                      int64_t k, const int32_t *active_layout) {
    __shared__ uint64_t s[kSortTile];
    const int l = blockIdx.y;
    if (active_layout && !active_layout[l]) return;
    const int64_t tile0 = (int64_t)blockIdx.x * kSortTile;
    uint64_t *a = base + l * lstride + tile0;
    const int t = threadIdx.x;
    s[t] = a[t];
    s[t + kSortThreads] = a[t + kSortThreads];
    __syncthreads();
    const bool asc = (tile0 & k) == 0;  // k > kSortTile: direction constant over the tile
    for (int j = kSortTile >> 1; j > 0; j >>= 1) {
        const int i = 2 * j * (t / j) + (t % j);
        cmpswap(s[i], s[i + j], asc);
        __syncthreads();
    }
    a[t] = s[t];
    a[t + kSortThreads] = s[t + kSortThreads];
}

// One global step (k, j) with j >= kSortTile: thread per compared pair.
__global__ __launch_bounds__(256) void k_bitonic_global(uint64_t *base, int64_t lstride, int64_t n,
                                                        int64_t k, int64_t j, const int32_t *active_layout) {
    const int l = blockIdx.y;
    if (active_layout && !active_layout[l]) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n / 2) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    uint64_t *a = base + l * lstride;
    uint64_t x = a[i], y = a[i + j];
    const bool asc = (i & k) == 0;
    if ((x > y) == asc) {
        a[i] = y;
        a[i + j] = x;
    }
}

cs_status bitonic_sort(uint64_t *base, int64_t lstride, int64_t n, int nlayouts,
                              const int32_t *active_layout, hipStream_t s) {
    // n is a power of two >= kSortTile
    const int tiles = (int)(n / kSortTile);
    hipLaunchKernelGGL(k_bitonic_presort, dim3(tiles, nlayouts), dim3(kSortThreads), 0, s, base, lstride,
                       active_layout);
    CSI_HIP(hipGetLastError());
    for (int64_t k = 2 * kSortTile; k <= n; k <<= 1) {
        for (int64_t j = k >> 1; j >= kSortTile; j >>= 1) {
            const int64_t pairs = n / 2;
            hipLaunchKernelGGL(k_bitonic_global, dim3((unsigned)((pairs + 255) / 256), nlayouts), dim3(256), 0, s,
                               base, lstride, n, k, j, active_layout);
            CSI_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_bitonic_merge_tile, dim3(tiles, nlayouts), dim3(kSortThreads), 0, s, base, lstride, k,
                           active_layout);
        CSI_HIP(hipGetLastError());
    }
    return CS_OK;
}

struct KeyBits {
    int bd, bt, bs, bp;
};

// 1. keys = (l_T, l_d, l_s, p); invalid labels set the error flag; excluded pixels sort last and
//    are listed (in no particular order) for the component maps, which write NaN there.
__global__ __launch_bounds__(256) void k_make_keys(const LayoutDev *lays, int32_t npix, int64_t np2, KeyBits kb) {
    const LayoutDev L = lays[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np2) return;
    uint64_t key = kInvalid;
    if (i < npix) {
        const int32_t a = L.labels[i], b = L.labels[npix + i], c = L.labels[2 * (int64_t)npix + i];
        const int nexcl = (a == -1) + (b == -1) + (c == -1);
        const bool inrange = a >= 0 && a < L.k[0] && b >= 0 && b < L.k[1] && c >= 0 && c < L.k[2];
        if (nexcl == 0 && inrange) {
            key = ((uint64_t)b << (kb.bd + kb.bs + kb.bp)) | ((uint64_t)a << (kb.bs + kb.bp)) |
                  ((uint64_t)c << kb.bp) | (uint64_t)i;
        } else if (nexcl != 3) {
            atomicOr(&L.counts[2], 1);
        } else {
            L.excl[atomicAdd(&L.counts[3], 1)] = (int32_t)i;
        }
    }
    L.keys[i] = key;
}

// number of valid keys = index of the first kInvalid (keys sorted ascending)
__global__ void k_count_valid(const LayoutDev *lays, int64_t np2, int slot, const int32_t *active_layout) {
    const LayoutDev L = lays[blockIdx.x];
    if (active_layout && !active_layout[blockIdx.x]) return;
    if (threadIdx.x != 0) return;
    int64_t lo = 0, hi = np2;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (L.keys[mid] == kInvalid)
            hi = mid;
        else
            lo = mid + 1;
    }
    L.counts[slot] = (int32_t)lo;
}

// 3a. one wavefront per chunk: processing order, run starts, per-chunk segment counts
__global__ __launch_bounds__(64) void k_chunk_heads(const LayoutDev *lays, KeyBits kb, int32_t nchunk_max) {
    const LayoutDev L = lays[blockIdx.y];
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t n = L.counts[0];
    const int64_t slot = (int64_t)chunk * kChunk + lane;
    const bool valid = slot < n;
    const uint64_t pmask = (kb.bp >= 64) ? ~0ull : ((1ull << kb.bp) - 1);
    uint64_t key = valid ? L.keys[slot] : 0;
    uint64_t prev = (valid && lane > 0) ? L.keys[slot - 1] : 0;
    const bool head = valid && (lane == 0 || (key >> kb.bp) != (prev >> kb.bp));
    const uint64_t mask = __ballot(head);
    L.order[slot] = valid ? (int32_t)(key & pmask) : -1;
    if (lane == 0) {
        L.head[chunk] = mask;
        L.seg_base[chunk + 1] = __popcll(mask);
    }
    (void)nchunk_max;
}

// 3b. exclusive scan of the per-chunk segment counts (serial: once per clustering)
__global__ void k_seg_scan(const LayoutDev *lays, int32_t nchunk_max) {
    const LayoutDev L = lays[blockIdx.x];
    if (threadIdx.x != 0) return;
    int32_t acc = 0;
    L.seg_base[0] = 0;
    for (int c = 0; c < nchunk_max; ++c) {
        acc += L.seg_base[c + 1];
        L.seg_base[c + 1] = acc;
    }
    L.counts[1] = acc;
}

// 3c. segment triples
__global__ __launch_bounds__(64) void k_seg_lab(const LayoutDev *lays, KeyBits kb) {
    const LayoutDev L = lays[blockIdx.y];
    const int chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const uint64_t mask = L.head[chunk];
    if (!((mask >> lane) & 1ull)) return;
    const int64_t slot = (int64_t)chunk * kChunk + lane;
    const uint64_t key = L.keys[slot];
    const int seg = L.seg_base[chunk] + __popcll(mask & ((1ull << lane) - 1ull));
    int4 v;
    v.y = (int)((key >> (kb.bd + kb.bs + kb.bp)) & ((1ull << kb.bt) - 1ull));
    v.x = (int)((key >> (kb.bs + kb.bp)) & ((1ull << kb.bd) - 1ull));
    v.z = (int)((key >> kb.bp) & ((1ull << kb.bs) - 1ull));
    v.w = (int)slot;
    L.seg_lab[seg] = v;
}

// 4a. keys of the segments by the cluster of labelling j
__global__ __launch_bounds__(256) void k_seg_keys(const LayoutDev *lays, int j, int64_t np2, int bp) {
    const LayoutDev L = lays[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np2) return;
    uint64_t key = kInvalid;
    if (i < L.counts[1]) {
        const int4 v = L.seg_lab[i];
        const int lab = j == 0 ? v.x : (j == 1 ? v.y : v.z);
        key = ((uint64_t)lab << bp) | (uint64_t)i;
    }
    L.keys[i] = key;
}

// 4b. CSR from sorted (label, index) keys: perm and lower-bound offsets
__device__ int64_t lower_bound_keys(const uint64_t *keys, int64_t n, uint64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(256) void k_csr_from_keys(const uint64_t *keys, int64_t n, int k, int bp,
                                                       int32_t *perm, int32_t *offsets) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t pmask = (1ull << bp) - 1ull;
    if (i < n) perm[i] = (int32_t)(keys[i] & pmask);
    if (i <= k) offsets[i] = (i == k) ? (int32_t)n : (int32_t)lower_bound_keys(keys, n, (uint64_t)i << bp);
}

__global__ __launch_bounds__(256) void k_seg_csr(const LayoutDev *lays, int j, int bp) {
    const LayoutDev L = lays[blockIdx.y];
    const int64_t n = L.counts[1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t pmask = (1ull << bp) - 1ull;
    if (i < n) L.seg_perm[j][i] = (int32_t)(L.keys[i] & pmask);
    const int k = L.k[j];
    if (i <= k) L.seg_off[j][i] = (i == k) ? (int32_t)n : (int32_t)lower_bound_keys(L.keys, n, (uint64_t)i << bp);
}

// pixel keys (l_j, p) of one layout for the exported per-labelling pixel CSR, rebuilt from the
// prepared order and segment triples (the caller's label array is not read again)
__global__ __launch_bounds__(64) void k_pixel_keys(const LayoutDev *lays, int lay, int j, int64_t np2, int bp) {
    const LayoutDev L = lays[lay];
    const int64_t chunk = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t slot = chunk * kChunk + lane;
    if (slot >= np2) return;
    uint64_t key = kInvalid;
    if (slot < L.n_incl) {
        const uint64_t mask = L.head[chunk];
        const uint64_t le = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const int seg = L.seg_base[chunk] + __popcll(mask & le) - 1;
        const int4 v = L.seg_lab[seg];
        const int lab = j == 0 ? v.x : (j == 1 ? v.y : v.z);
        key = ((uint64_t)lab << bp) | (uint64_t)L.order[slot];
    }
    L.keys[slot] = key;
}

// 5. gather one item's d (and per-pixel N^-1) into [chunk][2][F][64] in working precision
template <typename TI, typename TO>
__global__ __launch_bounds__(256) void k_pack(const ItemDev *items, const LayoutDev *lays, const TI *src,
                                              int64_t item_stride, TO *dst, int32_t nfreq, int32_t npix,
                                              int32_t nchunk_max) {
    const int b = blockIdx.y;
    const ItemDev it = items[b];
    const LayoutDev L = lays[it.layout];
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= (int64_t)nchunk_max * kChunk) return;
    const int64_t chunk = slot / kChunk;
    const int lane = (int)(slot % kChunk);
    if (chunk >= L.nchunks) return;
    const bool valid = slot < L.n_incl;
    const int32_t p = valid ? L.order[slot] : 0;
    const TI *s = src + (int64_t)b * item_stride;
    TO *o = dst + (it.dchunk0 + chunk) * (2 * (int64_t)nfreq * kChunk) + lane;
    for (int sf = 0; sf < 2 * nfreq; ++sf) {
        const TI v = valid ? s[(int64_t)sf * npix + p] : (TI)0;
        o[(int64_t)sf * kChunk] = (TO)v;
    }
}

static int bits_for(int64_t n) {  // bits needed for values 0..n-1 (at least 1)
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

cs_status prepare_layouts(cs_problem *p, hipStream_t s) {
    const WsLayout &w = p->ws;
    KeyBits kb{bits_for(w.kmax[0]), bits_for(w.kmax[1]), bits_for(w.kmax[2]), bits_for(p->P)};
    const LayoutDev *dl = (const LayoutDev *)(p->wsp + w.layouts);
    const int L = p->L;
    const int64_t np2 = (int64_t)w.np2;
    // clear counts of every layout (fill kernel-free: counts are contiguous)
    CSI_HIP(hipMemsetAsync(p->wsp + w.counts, 0, sizeof(int32_t) * 4 * (size_t)L, s));
    hipLaunchKernelGGL(k_make_keys, dim3((unsigned)((np2 + 255) / 256), L), dim3(256), 0, s, dl, p->P, np2, kb);
    CSI_HIP(hipGetLastError());
    cs_status st = bitonic_sort((uint64_t *)(p->wsp + w.keys), (int64_t)w.keys_stride, np2, L, nullptr, s);
    if (st != CS_OK) return st;
    hipLaunchKernelGGL(k_count_valid, dim3(L), dim3(64), 0, s, dl, np2, 0, nullptr);
    CSI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_chunk_heads, dim3((unsigned)w.nchunk_max, L), dim3(64), 0, s, dl, kb, (int32_t)w.nchunk_max);
    CSI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_scan, dim3(L), dim3(64), 0, s, dl, (int32_t)w.nchunk_max);
    CSI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_seg_lab, dim3((unsigned)w.nchunk_max, L), dim3(64), 0, s, dl, kb);
    CSI_HIP(hipGetLastError());
    const int bseg = kb.bp;
    for (int j = 0; j < 3; ++j) {
        hipLaunchKernelGGL(k_seg_keys, dim3((unsigned)((np2 + 255) / 256), L), dim3(256), 0, s, dl, j, np2, bseg);
        CSI_HIP(hipGetLastError());
        st = bitonic_sort((uint64_t *)(p->wsp + w.keys), (int64_t)w.keys_stride, np2, L, nullptr, s);
        if (st != CS_OK) return st;
        const int64_t nthr = std::max<int64_t>((int64_t)w.p64, (int64_t)w.kmax[j] + 1);
        hipLaunchKernelGGL(k_seg_csr, dim3((unsigned)((nthr + 255) / 256), L), dim3(256), 0, s, dl, j, bseg);
        CSI_HIP(hipGetLastError());
    }
    return CS_OK;
}

cs_status pack_data(cs_problem *p, hipStream_t s) {
    const WsLayout &w = p->ws;
    const ItemDev *di = (const ItemDev *)(p->wsp + w.items);
    const LayoutDev *dl = (const LayoutDev *)(p->wsp + w.layouts);
    const int64_t slots = (int64_t)w.nchunk_max * kChunk;
    dim3 grid((unsigned)((slots + 255) / 256), p->B);
    const bool out32 = p->prec != CS_FP64;
    const int32_t nch = (int32_t)w.nchunk_max;
    auto pack = [&](const void *src, int64_t stride, void *dst) -> cs_status {
        if (p->dtype == CS_DTYPE_F64) {
            if (out32)
                hipLaunchKernelGGL((k_pack<double, float>), grid, dim3(256), 0, s, di, dl, (const double *)src, stride,
                                   (float *)dst, p->F, p->P, nch);
            else
                hipLaunchKernelGGL((k_pack<double, double>), grid, dim3(256), 0, s, di, dl, (const double *)src, stride,
                                   (double *)dst, p->F, p->P, nch);
        } else {
            if (out32)
                hipLaunchKernelGGL((k_pack<float, float>), grid, dim3(256), 0, s, di, dl, (const float *)src, stride,
                                   (float *)dst, p->F, p->P, nch);
            else
                hipLaunchKernelGGL((k_pack<float, double>), grid, dim3(256), 0, s, di, dl, (const float *)src, stride,
                                   (double *)dst, p->F, p->P, nch);
        }
        CSI_HIP(hipGetLastError());
        return CS_OK;
    };
    cs_status st = pack(p->d, p->d_stride, p->wsp + w.dpack);
    if (st != CS_OK) return st;
    if (p->nmode == CS_NINV_PIXEL) st = pack(p->ninv_pixel, p->ninv_stride, p->wsp + w.wpack);
    return st;
}

cs_status export_segments(cs_problem *p, int32_t item, int32_t j, int32_t *perm, int32_t *offsets, hipStream_t s) {
    const WsLayout &w = p->ws;
    const LayoutDev *dl = (const LayoutDev *)(p->wsp + w.layouts);
    const int lay = p->items[item].layout;
    const int64_t np2 = (int64_t)w.np2;
    const int bp = bits_for(p->P);
    hipLaunchKernelGGL(k_pixel_keys, dim3((unsigned)(np2 / kChunk)), dim3(kChunk), 0, s, dl, lay, j, np2, bp);
    CSI_HIP(hipGetLastError());
    uint64_t *keys = (uint64_t *)(p->wsp + w.keys) + (int64_t)lay * (int64_t)w.keys_stride;
    cs_status st = bitonic_sort(keys, 0, np2, 1, nullptr, s);
    if (st != CS_OK) return st;
    const int64_t n = p->layouts[lay].n_incl;
    const int k = p->layouts[lay].k[j];
    const int64_t nthr = std::max<int64_t>(n, (int64_t)k + 1);
    hipLaunchKernelGGL(k_csr_from_keys, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, s, keys, n, k, bp, perm,
                       offsets);
    CSI_HIP(hipGetLastError());
    return CS_OK;
}

}  // namespace csi
