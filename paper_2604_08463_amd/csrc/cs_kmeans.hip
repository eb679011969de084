// Spherical K-means patching (paper Sec. 2.2) for many independent clustering tasks at once.
//
// A task clusters the vectors it keeps (a mask over one shared set of unit vectors) into k
// patches.  The nearest centroid in angular separation is the one of largest dot product; each
// centroid is replaced by the direction of the sum of its members.  The labels must come out
// identical to a sequential reference, so every floating-point decision is reproduced exactly:
//   - the dot product is (x cx + y cy) + z cz with each product and sum rounded on its own
//     (contraction into FMA is switched off in this file), ties go to the lowest index;
//   - a centroid sums its members one after another in ascending vector order.  The members
//     come from a sort of the unique keys (label, kept index), after which one thread per
//     cluster walks its contiguous key range.
// Kernels per launch:
//   k_km_compact  per task: kept-vector list (ascending) and its length, by a block scan
//   k_km_init     per (task, cluster): starting centroid = kept vector init[t][j]
//   k_km_assign   per (task, kept vector): argmax over the task's centroids, staged through LDS
//                 in tiles; writes the label and the sort key
//   bitonic sort of the keys of every task (shared with segment preparation)
//   k_km_update   per (task, cluster): ordered member sum, norm, division
//   k_km_used / k_km_remap / k_km_write: compaction to 0..K_eff-1 and the caller's labels
#include <algorithm>
#include <mutex>

#include "cs_device.h"

#pragma clang fp contract(off)

namespace csi {

namespace {

constexpr int kKmThreads = 256;
constexpr int kKmTile = 256;  // centroids per LDS tile
constexpr int kScanThreads = 1024;
constexpr uint64_t kNoKey = ~0ull;

struct KmArgs {
    const double *vecs;      // [n][3]
    const uint8_t *keep;     // nullable [T][keep_stride]
    int64_t keep_stride;
    const int32_t *init;     // [T][init_stride]
    int64_t init_stride;
    int64_t n;
    int32_t ntasks;
    const int32_t *k;        // [T]
    const int64_t *coff;     // [T + 1] first centroid of each task
    int32_t *nkept;          // [T]
    int32_t *err;            // [T]
    int32_t *idx;            // [T][n] kept vector -> pixel index
    int32_t *lab;            // [T][n] current assignment (kept order)
    uint64_t *keys;          // [T][np2]
    int64_t np2;
    double *cen;             // [sum k][3]
    int32_t *flag;           // [sum k] used flags, then the compacted label
};

__device__ __forceinline__ double dot3(double x, double y, double z, double cx, double cy, double cz) {
    const double xy = x * cx + y * cy;
    return xy + z * cz;
}

// Block-wide exclusive scan of one int per thread (kScanThreads threads); returns the total.
__device__ __forceinline__ int block_scan(int v, int &excl, int *sh) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    int incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o);
        if (lane >= o) incl += u;
    }
    if (lane == 63) sh[w] = incl;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int i = 0; i < kScanThreads / 64; ++i) {
            const int c = sh[i];
            sh[i] = run;
            run += c;
        }
        sh[kScanThreads / 64] = run;
    }
    __syncthreads();
    excl = sh[w] + incl - v;
    const int total = sh[kScanThreads / 64];
    __syncthreads();
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_km_compact(const KmArgs a) {
    __shared__ int sh[kScanThreads / 64 + 1];
    const int t = blockIdx.x;
    const uint8_t *keep = a.keep ? a.keep + (int64_t)t * a.keep_stride : nullptr;
    int32_t *idx = a.idx + (int64_t)t * a.n;
    int base = 0;
    for (int64_t p0 = 0; p0 < a.n; p0 += kScanThreads) {
        const int64_t p = p0 + threadIdx.x;
        const int v = (p < a.n && (!keep || keep[p])) ? 1 : 0;
        int excl;
        const int tot = block_scan(v, excl, sh);
        if (v) idx[base + excl] = (int32_t)p;
        base += tot;
    }
    if (threadIdx.x == 0) {
        a.nkept[t] = base;
        a.err[t] = 0;
    }
}

__global__ __launch_bounds__(kKmThreads) void k_km_init(const KmArgs a) {
    const int t = blockIdx.y;
    const int j = blockIdx.x * kKmThreads + threadIdx.x;
    const int k = a.k[t], nk = a.nkept[t];
    if (j >= k || k >= nk) return;
    const int i = a.init[(int64_t)t * a.init_stride + j];
    double *c = a.cen + 3 * (a.coff[t] + j);
    if (i < 0 || i >= nk) {
        atomicOr(&a.err[t], 1);
        c[0] = c[1] = c[2] = 0.0;
        return;
    }
    const int64_t p = a.idx[(int64_t)t * a.n + i];
    c[0] = a.vecs[3 * p];
    c[1] = a.vecs[3 * p + 1];
    c[2] = a.vecs[3 * p + 2];
}

// Tasks that iterate: 2 <= k < n_kept and no error (k = 1 puts everything in cluster 0; k >= n_kept
// gives each vector its own cluster).
__device__ __forceinline__ bool km_active(const KmArgs &a, int t) {
    const int k = a.k[t], nk = a.nkept[t];
    return k >= 2 && k < nk && a.err[t] == 0;
}

__global__ __launch_bounds__(kKmThreads) void k_km_assign(const KmArgs a) {
    __shared__ double sc[3 * kKmTile];
    const int t = blockIdx.y;
    if (!km_active(a, t)) return;
    const int k = a.k[t], nk = a.nkept[t];
    const int64_t i = (int64_t)blockIdx.x * kKmThreads + threadIdx.x;
    if ((int64_t)blockIdx.x * kKmThreads >= a.np2) return;
    const bool live = i < nk;
    double x = 0.0, y = 0.0, z = 0.0;
    if (live) {
        const int64_t p = a.idx[(int64_t)t * a.n + i];
        x = a.vecs[3 * p];
        y = a.vecs[3 * p + 1];
        z = a.vecs[3 * p + 2];
    }
    const double *cen = a.cen + 3 * a.coff[t];
    double best = 0.0;
    int bi = -1;
    for (int j0 = 0; j0 < k; j0 += kKmTile) {
        const int nt = min(kKmTile, k - j0);
        __syncthreads();
        for (int e = threadIdx.x; e < 3 * nt; e += kKmThreads) sc[e] = cen[3 * (int64_t)j0 + e];
        __syncthreads();
        if (live)
            for (int j = 0; j < nt; ++j) {
                const double d = dot3(x, y, z, sc[3 * j], sc[3 * j + 1], sc[3 * j + 2]);
                if (bi < 0 || d > best) {
                    best = d;
                    bi = j0 + j;
                }
            }
    }
    if (i < a.np2) {
        uint64_t key = kNoKey;
        if (live) {
            a.lab[(int64_t)t * a.n + i] = bi;
            key = ((uint64_t)(uint32_t)bi << 32) | (uint64_t)i;
        }
        a.keys[(int64_t)t * a.np2 + i] = key;
    }
}

__device__ __forceinline__ int64_t lower_key(const uint64_t *keys, int64_t n, uint64_t v) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kKmThreads) void k_km_update(const KmArgs a) {
    const int t = blockIdx.y;
    if (!km_active(a, t)) return;
    const int j = blockIdx.x * kKmThreads + threadIdx.x;
    const int k = a.k[t], nk = a.nkept[t];
    if (j >= k) return;
    const uint64_t *keys = a.keys + (int64_t)t * a.np2;
    const int64_t b = lower_key(keys, nk, (uint64_t)j << 32);
    const int64_t e = lower_key(keys, nk, (uint64_t)(j + 1) << 32);
    if (e == b) return;  // no member: the centroid stays
    const int32_t *idx = a.idx + (int64_t)t * a.n;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int64_t m = b; m < e; ++m) {
        const int64_t p = idx[(uint32_t)keys[m]];
        sx = sx + a.vecs[3 * p];
        sy = sy + a.vecs[3 * p + 1];
        sz = sz + a.vecs[3 * p + 2];
    }
    const double n2 = (sx * sx + sy * sy) + sz * sz;
    const double nrm = __builtin_sqrt(n2);
    if (!(nrm > 0.0)) return;
    double *c = a.cen + 3 * (a.coff[t] + j);
    c[0] = sx / nrm;
    c[1] = sy / nrm;
    c[2] = sz / nrm;
}

__global__ __launch_bounds__(kKmThreads) void k_km_clear_flags(const KmArgs a, int64_t total) {
    const int64_t i = (int64_t)blockIdx.x * kKmThreads + threadIdx.x;
    if (i < total) a.flag[i] = 0;
}

__global__ __launch_bounds__(kKmThreads) void k_km_used(const KmArgs a) {
    const int t = blockIdx.y;
    if (!km_active(a, t)) return;
    const int64_t i = (int64_t)blockIdx.x * kKmThreads + threadIdx.x;
    if (i >= a.nkept[t]) return;
    a.flag[a.coff[t] + a.lab[(int64_t)t * a.n + i]] = 1;  // every writer stores the same value
}

__global__ __launch_bounds__(kScanThreads) void k_km_remap(const KmArgs a, int32_t *keff) {
    __shared__ int sh[kScanThreads / 64 + 1];
    const int t = blockIdx.x;
    const int k = a.k[t], nk = a.nkept[t];
    if (a.err[t]) {
        if (threadIdx.x == 0) keff[t] = -1;
        return;
    }
    if (!km_active(a, t)) {
        if (threadIdx.x == 0) keff[t] = (k >= nk) ? nk : (nk > 0 ? 1 : 0);
        return;
    }
    int32_t *f = a.flag + a.coff[t];
    int base = 0;
    for (int j0 = 0; j0 < k; j0 += kScanThreads) {
        const int j = j0 + threadIdx.x;
        const int v = (j < k) ? f[j] : 0;
        int excl;
        const int tot = block_scan(v, excl, sh);
        if (j < k) f[j] = v ? base + excl : -1;
        base += tot;
    }
    if (threadIdx.x == 0) keff[t] = base;
}

__global__ __launch_bounds__(kKmThreads) void k_km_write(const KmArgs a, int32_t *labels, int64_t lstride) {
    const int t = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * kKmThreads + threadIdx.x;
    if (i >= a.n) return;
    int32_t *out = labels + (int64_t)t * lstride;
    const uint8_t *keep = a.keep ? a.keep + (int64_t)t * a.keep_stride : nullptr;
    const int k = a.k[t], nk = a.nkept[t];
    if (a.err[t]) {
        out[i] = -1;
        return;
    }
    if (keep && !keep[i]) out[i] = -1;  // vectors outside the task
    if (i < nk) {
        int v;
        if (k >= nk)
            v = (int)i;  // one cluster per vector, by rank
        else if (k == 1)
            v = 0;
        else
            v = a.flag[a.coff[t] + a.lab[(int64_t)t * a.n + i]];
        out[a.idx[(int64_t)t * a.n + i]] = v;
    }
}

}  // namespace

// Workspace of the allocation-free entry point: one copy of this array on every GPU the library
// runs on, held until the process ends.  In host code its name stands for the symbol only; the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) char km_scratch[CS_KMEANS_STATIC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // device address of km_scratch per device id
}  // namespace

// Device address of this device's km_scratch (looked up on the first call on the device).
static cs_status km_scratch_address(void **out) {
    int dev = 0;
    CSI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device id beyond the 64 the allocation-free K-means supports");
        return CS_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(km_scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(km_scratch)");
        if (!ptr) {
            set_error("hipGetSymbolAddress(km_scratch) returned a null address");
            return CS_E_HIP;
        }
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return CS_OK;
}

size_t kmeans_bytes(int64_t n, int32_t ntasks, int64_t ktot) {
    int64_t np2 = 2048;
    while (np2 < n) np2 <<= 1;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t T = (size_t)ntasks;
    return al(sizeof(int32_t) * T) + al(sizeof(int64_t) * (T + 1)) + al(sizeof(int32_t) * T) * 2 +
           al(sizeof(int32_t) * T * (size_t)n) * 2 + al(sizeof(uint64_t) * T * (size_t)np2) +
           al(sizeof(double) * 3 * (size_t)ktot) + al(sizeof(int32_t) * (size_t)ktot);
}

cs_status kmeans_batch(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep, int64_t keep_stride,
                       const int32_t *k_host, const int32_t *init, int64_t init_stride, int32_t iters,
                       int32_t *labels, int64_t labels_stride, int32_t *keff, void *ws, hipStream_t s) {
    int64_t np2 = 2048;
    while (np2 < n) np2 <<= 1;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t T = (size_t)ntasks;
    std::vector<int64_t> coff(T + 1, 0);
    int32_t kmax = 1;
    for (size_t t = 0; t < T; ++t) {
        coff[t + 1] = coff[t] + k_host[t];
        kmax = std::max(kmax, k_host[t]);
    }
    const int64_t ktot = coff[T];
    char *w = (char *)ws;
    KmArgs a;
    int32_t *kdev = (int32_t *)w;
    w += al(sizeof(int32_t) * T);
    int64_t *cdev = (int64_t *)w;
    w += al(sizeof(int64_t) * (T + 1));
    a.nkept = (int32_t *)w;
    w += al(sizeof(int32_t) * T);
    a.err = (int32_t *)w;
    w += al(sizeof(int32_t) * T);
    a.idx = (int32_t *)w;
    w += al(sizeof(int32_t) * T * (size_t)n);
    a.lab = (int32_t *)w;
    w += al(sizeof(int32_t) * T * (size_t)n);
    a.keys = (uint64_t *)w;
    w += al(sizeof(uint64_t) * T * (size_t)np2);
    a.cen = (double *)w;
    w += al(sizeof(double) * 3 * (size_t)ktot);
    a.flag = (int32_t *)w;
    a.vecs = vecs;
    a.keep = keep;
    a.keep_stride = keep_stride;
    a.init = init;
    a.init_stride = init_stride;
    a.n = n;
    a.ntasks = ntasks;
    a.k = kdev;
    a.coff = cdev;
    a.np2 = np2;

    CSI_HIP(hipMemcpyAsync(kdev, k_host, sizeof(int32_t) * T, hipMemcpyHostToDevice, s));
    CSI_HIP(hipMemcpyAsync(cdev, coff.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice, s));
    CSI_HIP(hipStreamSynchronize(s));  // the host arrays may go out of scope after this
    hipLaunchKernelGGL(k_km_compact, dim3(ntasks), dim3(kScanThreads), 0, s, a);
    CSI_HIP(hipGetLastError());
    const unsigned kb = (unsigned)((kmax + kKmThreads - 1) / kKmThreads);
    hipLaunchKernelGGL(k_km_init, dim3(kb, ntasks), dim3(kKmThreads), 0, s, a);
    CSI_HIP(hipGetLastError());
    const unsigned pb = (unsigned)((np2 + kKmThreads - 1) / kKmThreads);
    for (int it = 0; it <= iters; ++it) {
        hipLaunchKernelGGL(k_km_assign, dim3(pb, ntasks), dim3(kKmThreads), 0, s, a);
        CSI_HIP(hipGetLastError());
        if (it == iters) break;  // the final assignment
        cs_status st = bitonic_sort(a.keys, np2, np2, ntasks, nullptr, s);
        if (st != CS_OK) return st;
        hipLaunchKernelGGL(k_km_update, dim3(kb, ntasks), dim3(kKmThreads), 0, s, a);
        CSI_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_km_clear_flags, dim3((unsigned)((ktot + kKmThreads - 1) / kKmThreads)), dim3(kKmThreads), 0,
                       s, a, ktot);
    CSI_HIP(hipGetLastError());
    const unsigned nb = (unsigned)((n + kKmThreads - 1) / kKmThreads);
    hipLaunchKernelGGL(k_km_used, dim3(nb, ntasks), dim3(kKmThreads), 0, s, a);
    CSI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_km_remap, dim3(ntasks), dim3(kScanThreads), 0, s, a, keff);
    CSI_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_km_write, dim3(nb, ntasks), dim3(kKmThreads), 0, s, a, labels, labels_stride);
    CSI_HIP(hipGetLastError());
    return CS_OK;
}

cs_status kmeans_batch_static(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep,
                              int64_t keep_stride, const int32_t *k_host, const int32_t *init, int64_t init_stride,
                              int32_t iters, int32_t *labels, int64_t labels_stride, int32_t *keff, size_t bytes,
                              hipStream_t s) {
    if (bytes > CS_KMEANS_STATIC_BYTES) {
        set_error("K-means workspace of " + std::to_string(bytes) + " bytes exceeds the " +
                  std::to_string((size_t)CS_KMEANS_STATIC_BYTES) +
                  " bytes of the allocation-free entry point: use cs_kmeans_batch or fewer tasks per call");
        return CS_E_WORKSPACE;
    }
    void *ws = nullptr;
    const cs_status st = km_scratch_address(&ws);
    if (st != CS_OK) return st;
    return kmeans_batch(vecs, n, ntasks, keep, keep_stride, k_host, init, init_stride, iters, labels, labels_stride,
                        keff, ws, s);
}

}  // namespace csi
