/*
 * cs.h -- C ABI of the MI355X (gfx950) library for the clustered spectral likelihood of
 * parametric CMB component separation (arXiv 2604.08463).
 *
 * Every entry point is extern "C", takes plain pointers and sizes, never throws, and reports
 * argument errors synchronously through cs_status.  Unless a parameter is marked "host", a
 * pointer is a DEVICE pointer (HIP global memory of the current device).  "stream" is a
 * hipStream_t passed as void* (NULL = the legacy default stream).  The library never allocates
 * device memory: the caller provides every buffer, including the workspaces.
 *
 * Method (paper Sec. 2.1-2.3, Sec. 3.3.1):
 *   For pixel p with spectral parameters beta_p = (beta_d, T_d, beta_s), each read from its own
 *   cluster label (one independent patching per parameter, Sec. 2.2-2.3), the F x 3 mixing
 *   matrix A_p has the columns CMB = 1, dust modified blackbody and synchrotron power law
 *   (eq. mixing_columns), converted from Rayleigh-Jeans to CMB units with
 *   g(nu) = (e^y - 1)^2 / (y^2 e^y), y = h nu / (k T_CMB), and normalised to 1 at nu0.
 *   Per Stokes parameter s in {Q, U}: M = A^T N^-1 A, b_s = A^T N^-1 d_s (eq. mle_solution),
 *   and the objective is F = -2 ln L_spec without its constant (eq. spectral_likelihood):
 *       F = - sum_p sum_s b_s^T M^-1 b_s.
 *   Its gradient uses the GLS residuals r = N^-1 (d - A s_hat) with s_hat held fixed
 *   (Sec. 3.3.1): dF/dtheta = -2 r^T (dA/dtheta) s_hat, summed over the pixels of each cluster.
 *
 * Parameter vectors (x, grad, lower, upper) are packed per item as
 *   [ beta_d (K_d values) | T_d (K_T values) | beta_s (K_s values) ]
 * and items are concatenated; cs_problem_param_offsets returns the item offsets.
 */
#ifndef CS_H
#define CS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_problem cs_problem; /* opaque handle in host memory */

typedef enum {
    CS_OK = 0,
    CS_E_INVALID = 1,     /* bad argument, shape or size                                    */
    CS_E_LABEL = 2,       /* label outside [0, K_j) or excluded (-1) for only some parameters */
    CS_E_WORKSPACE = 3,   /* workspace missing, misaligned or too small                      */
    CS_E_HIP = 4,         /* a HIP runtime call failed; cs_last_error() has the text          */
    CS_E_UNSUPPORTED = 5, /* shape outside what the kernels support (e.g. F > 32)             */
    CS_E_STATE = 6        /* call out of order (e.g. evaluation before cs_problem_prepare)    */
} cs_status;

/* Working precision of the per-pixel data stream (d and per-pixel N^-1).
 *   CS_FP64       : FP64 storage, FP64 frequency accumulation, FP64 solve and reductions.
 *   CS_FP32_BULK  : FP32 storage and FP32 frequency accumulation of every per-band sum
 *                   (A^T N^-1 A, A^T N^-1 d and the adjoint sums), whichever schedule forms them
 *                   (per pixel, or once per segment inside the pixel kernel); FP64 3x3 Cholesky
 *                   solve from those sums; FP64 compensated per-cluster reductions.
 *   CS_FP32_STORE : FP32 storage, FP64 accumulation, solve and reductions.  */
typedef enum { CS_FP64 = 0, CS_FP32_BULK = 1, CS_FP32_STORE = 2 } cs_precision;

/* Element type of the caller's d (and per-pixel N^-1) arrays. */
typedef enum { CS_DTYPE_F64 = 0, CS_DTYPE_F32 = 1 } cs_dtype;

/* Noise weights: one value per Stokes and band (host [2][F]) or per pixel (device [2][F][P]). */
typedef enum { CS_NINV_BAND = 0, CS_NINV_PIXEL = 1 } cs_ninv_mode;

/* per-item status bits, written to int32 status[B] */
#define CS_ITEM_NOT_PD 1     /* some pixel's M failed the Cholesky pivot test -> F = NaN  */
#define CS_ITEM_NONFINITE 2  /* F or a gradient entry is not finite                       */
#define CS_ITEM_LS_FAIL 4    /* optimiser: line search exhausted its backtracks           */
#define CS_ITEM_MAXITER 8    /* optimiser: iteration limit reached                        */
#define CS_ITEM_CONVERGED 16 /* optimiser: projected-gradient tolerance reached           */
#define CS_ITEM_RUNNING 32   /* optimiser: paused by the caller's replay limit (resumable)  */

typedef struct {
    int32_t nfreq;  /* F, 1..32                                                         */
    int32_t npix;   /* P >= 1: pixels per item (before exclusion)                       */
    int32_t nitems; /* B >= 1: realizations / configurations / parameter points         */
    const double *freqs_ghz;  /* host [F] band centres (delta bandpasses), > 0          */
    double nu0_dust_ghz;      /* dust reference frequency (353 in the workloads)        */
    double nu0_sync_ghz;      /* synchrotron reference frequency (23)                   */
    double tcmb_k;            /* CMB temperature (2.7255)                               */
    cs_precision precision;
    cs_dtype d_dtype;
    const void *d;            /* device [B][2][F][P] uK_CMB, pixel fastest               */
    int64_t d_item_stride;    /* elements between items; 0 = one sky shared by all items */
    cs_ninv_mode ninv_mode;
    const double *ninv_band;  /* host [2][F] uK^-2 (> 0), used when ninv_mode = BAND     */
    const void *ninv_pixel;   /* device [B][2][F][P] (dtype d_dtype, >= 0) when PIXEL    */
    int64_t ninv_item_stride; /* elements between items; 0 = shared                      */
    const int32_t *labels;    /* device [B][3][P]: cluster of each pixel for beta_d, T_d,
                                 beta_s; -1 on all three = pixel excluded (mask)          */
    int64_t labels_item_stride; /* elements between items; 0 = one labelling for all     */
    const int32_t *nclusters; /* host [B][3]: K_d, K_T, K_s >= 1 of each item (equal for
                                 all items when labels are shared)                        */
} cs_problem_desc;

/* Validates the descriptor on the host and copies the host arrays (freqs, ninv_band,
 * nclusters).  The device arrays d, ninv_pixel and labels are only read by
 * cs_problem_prepare.  Ownership of *out passes to the caller (cs_problem_destroy). */
cs_status cs_problem_create(const cs_problem_desc *desc, cs_problem **out);

/* host [B+1]: offset of each item's packed parameter vector; host_off[B] = total length. */
cs_status cs_problem_param_offsets(const cs_problem *prob, int64_t *host_off);

/* Device workspace needed by cs_problem_prepare and every evaluation (an upper bound that
 * depends only on the descriptor).  The caller owns the buffer; it must be 256-byte aligned
 * and stay alive and untouched until cs_problem_destroy. */
cs_status cs_problem_workspace_bytes(const cs_problem *prob, size_t *bytes);

/* Segment preparation, once per clustering (paper Sec. 2.2-2.3: patches are disjoint pixel
 * sets, one patching per parameter).  On the device: validates the labels, orders the
 * included pixels by (l_T, l_d, l_s, p), cuts the order into 64-pixel chunks and constant-
 * label runs (segments), builds each labelling's segment CSR, and packs d (and per-pixel
 * N^-1) into the workspace in that order and in the working precision.  Synchronises the
 * stream.  Returns CS_E_LABEL on a bad label.  After it returns, d / ninv_pixel / labels are
 * no longer read. */
cs_status cs_problem_prepare(cs_problem *prob, void *workspace, size_t bytes, void *stream);

/* host: number of included pixels and of segments of an item (after prepare). */
cs_status cs_problem_item_info(const cs_problem *prob, int32_t item, int64_t *n_included,
                               int64_t *n_segments);

/* Segment structure of one labelling (0 = beta_d, 1 = T_d, 2 = beta_s) of one item (paper
 * Sec. 2.2: each patch is a disjoint set of pixels sharing one parameter value; Sec. 2.3: one
 * patching per spectral parameter), for bit-exact checks: perm[n_included] lists the included pixel indices grouped by cluster,
 * ascending pixel index inside a cluster (a stable sort by label); offsets[K_j + 1] is the
 * exclusive prefix sum of cluster sizes.  Device outputs; enqueued on the stream. */
cs_status cs_problem_segments(cs_problem *prob, int32_t item, int32_t labeling, int32_t *perm,
                              int32_t *offsets, void *stream);

/* neg2logL[B] = F of each item at x (packed, FP64): the spectral likelihood of paper Sec. 2.1,
 * eq. spectral_likelihood, with s profiled out by the GLS solution of eq. mle_solution, and
 * the parameters of each pixel read through its three patch labels (Sec. 2.2-2.3).  The 3x3
 * system per pixel is solved by an FP64 Cholesky factorisation (the central step of Sec.
 * 3.3.1).  status[B] (nullable) gets the item bits; a pixel whose A^T N^-1 A fails the
 * positive-definiteness test sets CS_ITEM_NOT_PD and F = NaN; a non-finite F sets
 * CS_ITEM_NONFINITE.  x, neg2logL and status are caller-owned device arrays.
 * Asynchronous on the stream; no allocation; capturable in a HIP graph. */
cs_status cs_likelihood(cs_problem *prob, const double *x, double *neg2logL, int32_t *status,
                        void *stream);

/* As cs_likelihood, plus grad (packed like x) = dF/dx summed per cluster (the adjoint of
 * paper Sec. 3.3.1: the gradient of the profiled likelihood with the GLS amplitudes held fixed,
 * -2 r^T (dA/dtheta) s_hat with r = N^-1 (d - A s_hat), routed to each parameter's patch by
 * summing over its pixels), and optional
 * cluster_neg2logL (nullable, packed like x): entry k of labelling j is the sum of the
 * per-pixel terms of F over the pixels of cluster k of labelling j (each labelling's entries
 * sum to F).  Per-cluster sums are FP64 and compensated. */
cs_status cs_likelihood_grad(cs_problem *prob, const double *x, double *neg2logL, double *grad,
                             double *cluster_neg2logL, int32_t *status, void *stream);

/* Component maps and the CMB map variance at x (packed, FP64).  The generalised least-squares
 * amplitudes s_hat = (A^T N^-1 A)^-1 A^T N^-1 d of every included pixel (paper Sec. 2.3, the
 * reconstruction operator W applied to d) are formed in FP64 from the data as stored by
 * prepare (FP32 for the FP32 precisions).
 *   maps      nullable device double; item b's block starts at maps + b * maps_item_stride
 *             and is [2 Stokes Q, U][3 components CMB, dust, sync][P] in the caller's pixel
 *             order; excluded pixels and pixels whose A^T N^-1 A is not positive definite
 *             hold NaN.
 *   maps_item_stride  0 = 6 P, else >= 6 P elements.
 *   cmb_var   nullable device double [B]: population variance over the included pixels of
 *             the CMB amplitude of Q plus that of U (Sec. 2.4, eq. min_var, the statistic that
 *             selects the number of clusters); NaN for an item with a non-positive-definite
 *             pixel or with no included pixel.
 *   status    nullable device int32 [B]: item bits of this call.
 * Asynchronous on the stream; no allocation.  Shares the workspace scratch with the
 * evaluations, so calls on one problem must not overlap. */
cs_status cs_component_maps(cs_problem *prob, const double *x, double *maps, int64_t maps_item_stride,
                            double *cmb_var, int32_t *status, void *stream);

/* As cs_component_maps, with each item's maps in processing order instead of the caller's pixel
 * order: entry i of every [P] row is the amplitude of pixel order[i] (cs_problem_pixel_order), for
 * i < n_included; entries n_included .. P - 1 hold NaN.  Every map write is coalesced, where the
 * pixel-order variant scatters 8-byte writes whenever neighbouring pixels of a patch are not
 * neighbours in the caller's numbering. */
cs_status cs_component_maps_sorted(cs_problem *prob, const double *x, double *maps,
                                   int64_t maps_item_stride, double *cmb_var, int32_t *status,
                                   void *stream);

/* Processing order of an item (after prepare): order[i] (device int32, n_included entries) is the
 * caller's index of the pixel in slot i -- included pixels sorted by (l_T, l_d, l_s, pixel).
 * Enqueued on the stream. */
cs_status cs_problem_pixel_order(cs_problem *prob, int32_t item, int32_t *order, void *stream);

/* Spherical K-means patching (paper Sec. 2.2) of ntasks independent tasks over one set of n
 * unit vectors, on the device.  Task t clusters the vectors it keeps into k[t] patches: the
 * nearest centroid in angular separation is the one of largest dot product (ties: lowest
 * index), and each of the iters Lloyd iterations replaces a centroid by the direction of the
 * sum of its members (a cluster without members keeps its centroid).  Labels come from one more
 * assignment and are compacted to 0..K_eff-1 in ascending centroid index; with k[t] >= the kept
 * count every kept vector is its own patch (by rank), and k[t] = 1 puts all in patch 0.  Every
 * floating-point decision is taken in FP64 with a fixed operation order, so results are
 * reproducible bit for bit.
 *   vecs      device double [n][3] unit vectors (pixel order)
 *   keep      nullable device uint8, row t at keep + t * keep_stride (0 = n): 1 = vector i takes
 *             part in task t; null = every vector in every task
 *   k         host int32 [ntasks], >= 1
 *   init      device int32, row t at init + t * init_stride (0 = max k): when k[t] is below the
 *             kept count, indices (into the task's kept vectors in ascending pixel order) of the
 *             k[t] starting centroids -- the random draw, made by the caller
 *   labels    device int32, row t at labels + t * labels_stride (0 = n): the patch of each
 *             vector, -1 where not kept
 *   keff      device int32 [ntasks]: number of patches; -1 if an init index was out of range
 *             (that task's labels are then all -1)
 *   workspace device, 256-byte aligned, >= cs_kmeans_workspace_bytes; caller owned.
 * Synchronises the stream once (upload of k); the rest is asynchronous. */
cs_status cs_kmeans_workspace_bytes(int64_t n, int32_t ntasks, const int32_t *k, size_t *bytes);
cs_status cs_kmeans_batch(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep,
                          int64_t keep_stride, const int32_t *k, const int32_t *init,
                          int64_t init_stride, int32_t iters, int32_t *labels,
                          int64_t labels_stride, int32_t *keff, void *workspace, size_t bytes,
                          void *stream);

/* Allocation-free K-means, for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cs_kmeans_batch with its
 * workspace taken from a device array owned by the library, CS_KMEANS_STATIC_BYTES (128 MiB) on
 * every GPU it runs on, held from the module load until the process ends.  Returns CS_E_WORKSPACE
 * when cs_kmeans_workspace_bytes of the arguments exceeds that size (split the tasks over several
 * calls).  Every call on one GPU uses the same array, which keeps the last call's contents (each
 * call initialises what it reads): calls that overlap on one GPU -- on other streams or host
 * threads -- race, so the caller serialises them.  Calls no hipMalloc, hipFree or other allocating
 * routine.  Synchronises the stream once (upload of k), like cs_kmeans_batch. */
#define CS_KMEANS_STATIC_BYTES ((size_t)128 << 20)
cs_status cs_kmeans_batch_static(const double *vecs, int64_t n, int32_t ntasks, const uint8_t *keep,
                                 int64_t keep_stride, const int32_t *k, const int32_t *init,
                                 int64_t init_stride, int32_t iters, int32_t *labels,
                                 int64_t labels_stride, int32_t *keff, void *stream);

/* Batched bound-constrained optimisers on the device, in the internal box y = (x - l)/(u - l)
 * (paper App. A.1) with bound clamping as in Alg. 1:
 *   CS_SOLVER_LBFGS    projected L-BFGS (two-loop recursion on the free set, Armijo backtracking)
 *   CS_SOLVER_ADATOPK  AdaTopK (App. A): AdaBelief directions, Top-K release of pinned bounds,
 *                      dynamic rescaling of the objective and moments, step limited by the
 *                      nearest bound (which is then pinned), backtracking line search
 * Defaults: solver = L-BFGS, m = 10, gtol_rel = 1e-8, max_iter = 1000, iters_per_graph = 8,
 * max_backtracks = 30, c1 = 1e-4, fp64_polish = 1, lr = 0.01, beta1 = 0.9, beta2 = 0.999,
 * eps = 1e-16, topk = 0, switch_rel = 1e-4.
 * Mixed precision (CS_FP32_BULK with fp64_polish): the FP32-accumulation phase runs until an item
 * converges, reaches |P g|_2 <= switch_rel |P g_0|_2, fails its line search or spends max_iter
 * iterations; every such item that has not converged then continues from its point, with its
 * curvature pairs, in FP64 accumulation on the same FP32 data, with max_iter more iterations.  The
 * FP32 gradient carries a rounding error of order F u times the magnitude of its terms, which near
 * the optimum is far above 1e-8 |P g_0|, so the last decades need the FP64 sums. */
#define CS_SOLVER_LBFGS 0
#define CS_SOLVER_ADATOPK 1
typedef struct {
    int32_t m;               /* history pairs, 1..32                                        */
    double gtol_rel;         /* stop when |P g|_2 <= gtol_rel |P g_0|_2 (internal units)    */
    int32_t max_iter;        /* accepted iterations per item                                */
    int32_t iters_per_graph; /* evaluations captured per HIP-graph replay (host polls once) */
    int32_t max_backtracks;  /* step halvings per line search                               */
    double c1;               /* Armijo constant                                             */
    int32_t fp64_polish;     /* CS_FP32_BULK only: items whose line search fails continue
                                with FP64 accumulation on the same FP32 data                */
    int32_t solver;          /* CS_SOLVER_LBFGS or CS_SOLVER_ADATOPK                         */
    double lr;               /* AdaTopK: AdaBelief step size (internal units)                */
    double beta1, beta2;     /* AdaTopK: moment decay rates, in [0, 1)                       */
    double eps;              /* AdaTopK: AdaBelief epsilon, >= 0                             */
    double topk;             /* AdaTopK: fraction in [0, 1] of the releasable bounds freed per
                                iteration (at least one)                                     */
    double switch_rel;       /* mixed precision: leave the FP32 phase at |P g|_2 <= switch_rel
                                |P g_0|_2, in [0, 1) (0 = only on a line-search failure or the
                                iteration limit)                                             */
} cs_optim_opts;

cs_status cs_optim_default_opts(cs_optim_opts *opts); /* host */

/* Device workspace of the optimiser for history m (AdaTopK uses it with any m >= 1). */
cs_status cs_optimizer_workspace_bytes(const cs_problem *prob, int32_t m, size_t *bytes);

/* Minimises F per item inside [lower, upper] (packed like x, lower < upper).  x: in = start
 * point (clipped into the box), out = minimiser.  f[B], iters[B], status[B] (device) receive
 * the final objective, accepted iterations and status bits; nevals[B] (nullable, int64) the
 * number of evaluations.  Runs HIP-graph replays of iters_per_graph evaluations and reads one
 * 4-byte counter back after each replay, so it synchronises the stream. */
cs_status cs_optimize_batch(cs_problem *prob, const cs_optim_opts *opts, const double *lower,
                            const double *upper, double *x, double *f, int32_t *iters,
                            int32_t *status, int64_t *nevals, void *opt_workspace, size_t opt_bytes,
                            void *stream);

/* The optimiser in resumable steps (paper Sec. 3.1: a campaign's batches are checkpointed and
 * resumed).  As cs_optimize_batch, and:
 *   resume       0 = start from x; 1 = continue from the state held in opt_workspace, left there
 *                by an earlier call on a problem of the same shape (items, parameter counts,
 *                precision) with the same opts.m and opts.solver; x is then output only.
 *   max_replays  0 = run until every item has stopped; n > 0 = return after at most n graph
 *                replays (n * iters_per_graph evaluation steps).  Items still running then carry
 *                CS_ITEM_RUNNING, and x, f, iters and nevals describe their current point.
 *   running      host, nullable: number of items still running on return.
 * Whenever the call returns, the first cs_optimizer_workspace_bytes bytes of opt_workspace hold
 * the optimiser's complete state (no pointers): a byte copy of them is a checkpoint, and copying
 * it back into a 256-byte aligned workspace -- in this or another process, for a problem prepared
 * from the same inputs -- and calling with resume = 1 continues the run.  With the same schedule the
 * result is bit for bit that of an uninterrupted run.  Returns CS_E_STATE when the workspace does
 * not hold a state of this shape, m, solver and precision.  Synchronises the stream. */
cs_status cs_optimize_batch_run(cs_problem *prob, const cs_optim_opts *opts, const double *lower,
                                const double *upper, double *x, double *f, int32_t *iters,
                                int32_t *status, int64_t *nevals, void *opt_workspace,
                                size_t opt_bytes, int32_t resume, int32_t max_replays,
                                int32_t *running, void *stream);

/* Contiguous item chunking (paper Sec. 3.1: worker k of P takes the items
 * [floor(k N / P), floor((k + 1) N / P))).  host outputs; 0 <= rank < nranks, nitems >= 0. */
cs_status cs_item_range(int32_t rank, int32_t nranks, int32_t nitems, int32_t *begin, int32_t *end);

/* *out = the descriptor of items [begin, end) of *in (0 <= begin < end <= in->nitems): the item
 * arrays (d, per-pixel N^-1, labels, nclusters) are offset by their item strides; arrays shared
 * by all items (stride 0) stay shared.  No copy is made: *out points into *in's arrays, which must
 * outlive it.  A problem created from each chunk gives bit for bit the results of those items in
 * the whole batch. */
cs_status cs_problem_desc_slice(const cs_problem_desc *in, int32_t begin, int32_t end,
                                cs_problem_desc *out);

/* Launch schedule of the per-pixel kernel (chosen by cs_problem_autotune or set by hand). */
typedef struct {
    int32_t waves_per_block; /* 1, 2, 4 or 8 wavefronts of 64 lanes per workgroup        */
    int32_t blocks_per_cu;   /* 0 = one 64-pixel unit per wavefront (no grid-stride loop);
                                n > 0 = persistent grid of n * 256 workgroups              */
    int32_t xcd_remap;       /* 1 = give each of the 8 XCDs a contiguous range of units    */
    int32_t shared_segments; /* staging mode of the LDS-staged kernel (band weights shared
                                by Q and U only): 0 = every pixel forms A^T N^-1 A and the
                                adjoint sums itself; 1 = formed once per segment
                                (constant-label run) with its Cholesky factor in LDS and
                                shared across its pixels; 2 = formed once per segment by
                                five lanes per segment, each pixel then taking them by
                                cross-lane reads and forming its own Cholesky factor
                                (CS_FP32_BULK only; in other precisions it runs as 0)      */
} cs_schedule;

cs_status cs_problem_get_schedule(const cs_problem *prob, cs_schedule *sched);
cs_status cs_problem_set_schedule(cs_problem *prob, const cs_schedule *sched);

/* Times every candidate schedule on cs_likelihood_grad at x (reps evaluations each, HIP
 * events on the stream), then re-times the four fastest in turn over three rounds of
 * max(reps, 5) evaluations and keeps the one with the least total.  Candidates that only move
 * work between wavefronts must reproduce the current schedule's F and gradient bit for bit;
 * candidates that change shared_segments (a different rounding order) must agree on F to 1e-11
 * relative and on each item's gradient to 1e-8 normwise (1e-6 and 1e-3 for CS_FP32_BULK);
 * others are rejected.  grad / neg2logL are scratch outputs.  Writes the chosen schedule to
 * *best (nullable).  Synchronises the stream. */
cs_status cs_problem_autotune(cs_problem *prob, const double *x, double *neg2logL, double *grad,
                              int32_t reps, cs_schedule *best, void *stream);

/* Kernel timing: when enabled, every per-pixel kernel launch is bracketed by a pair of HIP
 * events on its stream; cs_problem_kernel_time sums the elapsed times of the completed
 * launches (synchronising on the last event) and resets the counters. */
cs_status cs_problem_set_timing(cs_problem *prob, int32_t enable);
cs_status cs_problem_kernel_time(cs_problem *prob, double *total_ms, int64_t *launches);

void cs_problem_destroy(cs_problem *prob);
const char *cs_status_str(cs_status status);
const char *cs_last_error(void); /* thread-local text of the last error */

#ifdef __cplusplus
}
#endif
#endif /* CS_H */
