/*
 * kdt.h -- C ABI of the MI355X (gfx950) left-balanced k-d tree builder.
 *
 * The library builds the left-balanced, complete k-d tree of Wald,
 * "GPU-friendly, Parallel, and (Almost-)In-Place Construction of Left-Balanced
 * k-d Trees" (arXiv 2211.00120) over N float32 (or int32) points of
 * dimension k:
 *
 *   - the tree is stored in level order, node s has children 2s+1 and 2s+2,
 *     and only the array order carries the topology (Sec. 1, Sec. 2);
 *   - it is built by O(log N) iterations over the whole point set, each a
 *     sort by (subtree tag, coordinate in the split dimension) followed by a
 *     per-point tag update that fixes every subtree's pivot with the O(1)
 *     subtree-size and segment-begin formulas (Sec. 3, Sec. 4);
 *   - the split dimension is either level(s) mod k (round robin, Sec. 2) or
 *     the widest extent of the subtree's domain, i.e. the scene bounding box
 *     clipped by all ancestors' planes (split-widest, Sec. 6).
 *
 * Equal coordinates are ordered by the points' original indices, which makes
 * the tree unique (the paper's comparison has no tie-break, Sec. 3.1).
 *
 * Conventions for every entry point below:
 *   - pointers named d_* are device memory of the current HIP device; h_* are
 *     host memory;
 *   - points are row-major float32, point i's coordinate d at [i*k + d];
 *   - work is enqueued asynchronously on `stream` (0 = the null stream); the
 *     call returns once it is enqueued, without synchronising;
 *   - argument errors are detected on the host before anything is enqueued;
 *     no call throws, and no call leaves partial work on the stream when it
 *     returns an error;
 *   - the caller owns every buffer it passes in.
 */
#ifndef KDT_H
#define KDT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum kdt_status {
    KDT_OK = 0,
    KDT_EINVAL = 1,      /* bad argument (null pointer, k outside 1..4, N too large, workspace too small) */
    KDT_ENOMEM = 2,      /* the library could not allocate device memory it owns */
    KDT_EDEVICE = 3,     /* a HIP call failed; kdt_last_error() has its message */
    KDT_ENONFINITE = 4,  /* device status word: an input coordinate is NaN or +-inf */
    KDT_EBUSY = 5,       /* server: the request has not finished yet */
    KDT_ENOTFOUND = 6    /* server: unknown ticket */
} kdt_status;

/* Split-dimension rule: level(s) mod k (Sec. 2) or widest domain extent
 * (Sec. 6). */
typedef enum kdt_dim_mode {
    KDT_DIM_ROUND_ROBIN = 0,
    KDT_DIM_WIDEST = 1
} kdt_dim_mode;

/* Largest supported point count (2^30 - 1): positions and lookback counts
 * are kept in 30-bit fields. */
#define KDT_MAX_POINTS 1073741823u

/* Bit of a device status word (kdt_build_ws, kdt_build_batched, server
 * results): an internal consistency check of the build failed -- a bounds
 * guard on a scatter or gather, or a bounded wait of the onesweep look-back
 * or a pivot search that gave up.  The outputs are then unspecified.  No
 * build of valid arguments in a valid workspace sets it; it turns a corrupt
 * workspace or a device fault into an error instead of a wrong tree. */
#define KDT_STATUS_INTERNAL_BIT 0x100u

/* Bytes of device workspace kdt_build_ws needs for (n, k, mode); 0 when the
 * arguments are invalid.  The size depends only on the arguments. */
size_t kdt_workspace_bytes(uint32_t n, uint32_t k, int dim_mode);

/*
 * Build the tree of d_points into caller-provided outputs.
 *
 *   d_points   n*k float32, read only; must not overlap any output;
 *              16-byte aligned for k = 4, 8-byte for k = 2, 4-byte
 *              otherwise (rows move as whole vectors; KDT_EINVAL if not).
 *   n, k       point count (0..KDT_MAX_POINTS) and dimension (1..4).
 *   dim_mode   KDT_DIM_ROUND_ROBIN or KDT_DIM_WIDEST.
 *   d_tree     nullable; n*k float32, aligned as d_points; d_tree[s*k + d] = coordinate d of the
 *              point stored at level-order node s.
 *   d_perm     nullable; n uint32: original index of the point at node s.
 *   d_dim      nullable; n uint8: split dimension of node s (round robin:
 *              level(s) mod k; split-widest: widest extent of s's domain,
 *              lowest dimension on ties; defined for leaves too).
 *   d_status   nullable; one uint32 the device sets to KDT_OK or, if any
 *              input coordinate is NaN or infinite, KDT_ENONFINITE (the
 *              outputs are then unspecified); KDT_STATUS_INTERNAL_BIT may be
 *              or-ed in if an internal check failed (see above).
 *   d_ws       device workspace of at least kdt_workspace_bytes(n,k,mode)
 *              bytes, 256-byte aligned; contents on entry are ignored.
 *
 * Never allocates and never synchronises.  Builds that use different
 * workspaces may run concurrently on different streams.
 */
kdt_status kdt_build_ws(const float* d_points, uint32_t n, uint32_t k, int dim_mode,
                        float* d_tree, uint32_t* d_perm, uint8_t* d_dim,
                        uint32_t* d_status, void* d_ws, size_t ws_bytes,
                        hipStream_t stream);

/*
 * kdt_build_ws for int32 coordinates (the paper's int1 workload, Table 1;
 * Sec. 7.2 templates the builder over the point type).  Same arguments,
 * workspace size (kdt_workspace_bytes) and outputs, with int32 points and
 * tree.  Coordinates compare as signed integers, ties by original index;
 * the split-widest extent of a domain is the exact difference hi - lo (no
 * int32 overflow).  The status word is always KDT_OK (plus
 * KDT_STATUS_INTERNAL_BIT on an internal failure): every int32 is finite.
 */
kdt_status kdt_build_ws_i32(const int32_t* d_points, uint32_t n, uint32_t k, int dim_mode,
                            int32_t* d_tree, uint32_t* d_perm, uint8_t* d_dim,
                            uint32_t* d_status, void* d_ws, size_t ws_bytes,
                            hipStream_t stream);

/*
 * Per-point payload in tree order (Sec. 7.2: whatever a point carries moves
 * with it): record s of d_out is record d_perm[s] of d_in, records of
 * stride_bytes bytes, for s < n, d_perm being the permutation a build wrote.
 * d_out must not overlap d_in or d_perm.  An entry d_perm[s] >= n leaves
 * record s unwritten and sets KDT_STATUS_INTERNAL_BIT in d_status (nullable).
 * Records move in 16-, 4- or 1-byte units, whichever the pointers and the
 * stride are aligned to.  Never allocates and never synchronises.
 */
kdt_status kdt_permute_payload(const uint32_t* d_perm, uint32_t n, const void* d_in, uint32_t stride_bytes,
                               void* d_out, uint32_t* d_status, hipStream_t stream);

/*
 * Low-memory in-place build (Sec. 7: the method needs one int per node of
 * temporary storage, and a sort made only of swaps, such as bitonic sort,
 * needs no more).  On completion d_points holds the tree in level order and
 * d_perm[s] the original index of the point at node s.  d_perm is the one
 * int per node: during the build it carries each point's original index
 * (the tie-break of the order), so it is required.  Every data movement is
 * a compare-exchange or a swap of (point, index) pairs; the tree, perm and
 * dims are the same as kdt_build_ws's.  Slower than kdt_build_ws (whose
 * workspace is about 95-130 bytes per point), for callers short of memory.
 *
 *   d_points   n*k float32, read and overwritten; 4-, 8- or 16-byte aligned
 *              for k = 1 or 3, 2, 4.
 *   d_perm     n uint32 (required).
 *   d_dim      nullable; n uint8, as in kdt_build_ws.
 *   d_status   nullable; as in kdt_build_ws (KDT_OK, KDT_ENONFINITE, plus
 *              KDT_STATUS_INTERNAL_BIT if an internal bound check failed).
 *   d_ws       at least kdt_inplace_workspace_bytes(n,k,mode) bytes,
 *              256-byte aligned: a 256-byte header plus one byte (round
 *              robin) or 33 bytes (split-widest) per subtree of the level
 *              whose subtrees first fit 2047 points, i.e. about n/1024
 *              subtrees.
 * Buffers must not overlap.  Never allocates and never synchronises.
 */
size_t kdt_inplace_workspace_bytes(uint32_t n, uint32_t k, int dim_mode);
kdt_status kdt_build_inplace(float* d_points, uint32_t n, uint32_t k, int dim_mode, uint32_t* d_perm,
                             uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                             hipStream_t stream);
/* The same for int32 coordinates (as kdt_build_ws_i32). */
kdt_status kdt_build_inplace_i32(int32_t* d_points, uint32_t n, uint32_t k, int dim_mode, uint32_t* d_perm,
                                 uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream);

/*
 * Build in place: on return (once `stream` has run the work) d_points holds
 * the tree in level order.  The library keeps one cached workspace per
 * (device, stream) pair, allocated on first use and grown when needed, so
 * this entry point may allocate.  Non-finite input is not reported (use
 * kdt_build_ws with a status word for that).  d_points is aligned as for
 * kdt_build_ws.
 */
kdt_status kdt_build(float* d_points, uint32_t n, uint32_t k, int dim_mode,
                     hipStream_t stream);

/*
 * Batched build: C independent trees (one per cloud) in one call.
 *
 * Cloud c is the points [h_offsets[c], h_offsets[c+1]) of d_points (row-major
 * float32, k per point; d_points and d_tree aligned as for kdt_build_ws); its tree, permutation and dimensions go to the same
 * entry range of d_tree / d_perm / d_dim, exactly as kdt_build_ws would write
 * them for that cloud alone (d_perm holds indices local to the cloud).  All
 * clouds share k and dim_mode.  The build is the same sequence of iterations
 * for every cloud (Sec. 3); one launch runs a step for every cloud that has
 * that step, each cloud a separate key range of the segmented sorts, so a
 * batch costs the launches of its largest cloud.
 *
 *   h_offsets  host array of C+1 non-decreasing entries, h_offsets[0] = 0,
 *              h_offsets[C] <= KDT_MAX_POINTS (empty clouds are allowed).
 *   d_status   nullable; set to KDT_OK, or KDT_ENONFINITE if any coordinate of
 *              any cloud is NaN or infinite.
 *   d_ws       at least kdt_batched_workspace_bytes(h_offsets, C, k, mode)
 *              bytes, 256-byte aligned.
 *
 * The first call for a given (h_offsets, k, mode) plans the batch on the host
 * and keeps the plan, with its launch tables in pinned host memory, until
 * kdt_release_cached(); each call uploads the tables into d_ws on `stream`.
 * Apart from that first planning the call neither allocates nor
 * synchronises, so it can be captured into a HIP graph (the graph then
 * refers to the cached tables: release the cache only after the graph).
 */
size_t kdt_batched_workspace_bytes(const uint32_t* h_offsets, uint32_t C, uint32_t k, int dim_mode);

kdt_status kdt_build_batched(const float* d_points, const uint32_t* h_offsets, uint32_t C,
                             uint32_t k, int dim_mode, float* d_tree, uint32_t* d_perm,
                             uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                             hipStream_t stream);

/*
 * kdt_build_ws for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * The workspace is a fixed device array of KDT_STATIC_WS_BYTES bytes that
 * the library holds on every device it runs on until the process ends (its
 * address is looked up once per device, on the first call with that device
 * current).  Arguments, outputs and status word as for kdt_build_ws; the
 * caller still provides the points and every output buffer.
 *
 *   - Builds whose kdt_workspace_bytes(n, k, dim_mode) exceeds
 *     KDT_STATIC_WS_BYTES are rejected with KDT_EINVAL before anything is
 *     enqueued (about 0.5M points at k = 4, 0.67M at k = 3, 1.4M at k = 1).
 *   - Allocates no device or pinned memory and never synchronises.
 *   - Every call on one device shares that device's array, and each call
 *     starts by clearing what it needs cleared: calls ordered on one stream
 *     are fine, but calls that overlap in time on one device (other streams,
 *     other threads) race and corrupt each other's trees.
 */
#define KDT_STATIC_WS_BYTES (64u << 20)

kdt_status kdt_build_static(const float* d_points, uint32_t n, uint32_t k, int dim_mode,
                            float* d_tree, uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status,
                            hipStream_t stream);

/* kdt_build_batched for int32 coordinates (see kdt_build_ws_i32). */
kdt_status kdt_build_batched_i32(const int32_t* d_points, const uint32_t* h_offsets, uint32_t C,
                                 uint32_t k, int dim_mode, int32_t* d_tree, uint32_t* d_perm,
                                 uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream);

/* Free every workspace cached by kdt_build and every cached batch plan
 * (synchronises the device first). */
void kdt_release_cached(void);

/*
 * Autotuner.  The level sorts can run with 8-, 9- or 10-bit digits (fewer
 * bits: more passes, smaller histograms and look-back tables) and with tiles
 * of 512 x 4 or 512 x 10 records; the presort's digit passes can run one
 * dimension per launch or all dimensions per launch.  Without tuning the
 * planner picks the fewest passes, the largest tile the level's subtrees
 * fill, and all dimensions per launch.
 * kdt_tune_batched times a whole kdt_build_batched of the given batch (in
 * device memory) for every combination, `reps` builds each after one
 * warm-up, and records the fastest for builds of this k, split rule and
 * rank width (bits of the largest cloud's n-1, counting only clouds of more
 * than 2048 points); single, batched and served builds of that class use it
 * from then on.  The choice never changes the tree.  Synchronises `stream`;
 * d_ws needs kdt_batched_workspace_bytes(...) bytes (those sizes, like
 * kdt_workspace_bytes, already hold every choice).
 */
typedef struct kdt_tuning {
    uint32_t radix_bits;   /* 0 (planner's choice) or 8..10 */
    uint32_t level_items;  /* records per thread of the split tiles: 0 (planner's choice), 4 (tiles of
                              512 x 4 records only) or 10 (also tiles of 512 x 10 records, where an
                              iteration's subtrees fill them) */
    uint32_t rank_layout;  /* 0 (planner's choice: 2 when the largest tree's rank table exceeds 128 MiB), 1 (each
                              dimension's last presort pass writes a point-major rank table, which iteration 0
                              gathers by index) or 2 (the root dimension is sorted first; every other dimension's
                              sort carries each point's root rank, and its ranks go to an array of its own by root
                              position through a windowed scatter, which iteration 0 streams); never swept by
                              kdt_tune_batched */
    uint32_t presort_dims; /* 0 (planner's choice: all k) or 1..4 (clamped to k): presort dimensions whose digit
                              passes share a launch, each with its own look-back chain (with rank_layout 2 the
                              root dimension's passes run alone, before the others) */
    double ms;             /* kdt_tune_batched: time of one build with this choice */
} kdt_tuning;

kdt_status kdt_tune_batched(const float* d_points, const uint32_t* h_offsets, uint32_t C, uint32_t k,
                            int dim_mode, void* d_ws, size_t ws_bytes, uint32_t reps,
                            hipStream_t stream, kdt_tuning* best);

/* Read or set the recorded choice for (k, dim_mode, rank_bits). */
kdt_status kdt_tuning_get(uint32_t k, int dim_mode, uint32_t rank_bits, kdt_tuning* out);
kdt_status kdt_tuning_set(uint32_t k, int dim_mode, uint32_t rank_bits, const kdt_tuning* t);

/* Text file of recorded choices, one "k dim_mode rank_bits radix_bits
 * level_items rank_layout presort_dims" line each; load merges into the current table and fails
 * without changing it on a malformed file. */
kdt_status kdt_tuning_save(const char* path);
kdt_status kdt_tuning_load(const char* path);
void kdt_tuning_clear(void);

/*
 * Build server: a request loop that builds trees for a stream of requests of
 * mixed size, k and split rule on one device.
 *
 * The server owns one device pool of hbm_budget_bytes, allocated once.  A
 * worker thread admits queued requests in arrival order whenever a batch
 * slot is free and their buffers fit the pool: the oldest request together
 * with the queued requests of the same k and split rule (up to
 * max_batch_requests and max_batch_points) becomes one batched build
 * (kdt_build_batched's kernels) on the slot's own stream, so up to
 * max_inflight batches run on the device at once and requests that arrive
 * while others run start as soon as a slot and memory free up.  A request's
 * points are copied from its host buffer when it is admitted; its tree,
 * permutation and split dimensions stay in the pool, at the device
 * addresses the result reports, until kdt_server_release.  Each result is
 * exactly the tree kdt_build_ws builds for that request alone.
 *
 * Timestamps are seconds on the clock kdt_clock() reads (monotonic).
 * The calls are thread-safe.  No stream priority other than the default is
 * used.
 */
typedef struct kdt_server kdt_server;

typedef struct kdt_server_config {
    size_t hbm_budget_bytes;     /* device pool; every request must fit it alone */
    uint32_t max_inflight;       /* batches on the device at once, 1..8 (one stream each) */
    uint32_t max_batch_requests; /* requests merged into one batch, >= 1 */
    uint64_t max_batch_points;   /* points merged into one batch (a larger request runs alone) */
} kdt_server_config;

typedef struct kdt_request {
    const float* h_points;       /* host, n*k float32; must stay valid until the request is done */
    uint32_t n, k;               /* 0..KDT_MAX_POINTS points of dimension 1..4 */
    int dim_mode;                /* KDT_DIM_ROUND_ROBIN or KDT_DIM_WIDEST */
} kdt_request;

typedef struct kdt_result {
    int status;                  /* KDT_OK, or KDT_ENONFINITE for a NaN/inf coordinate */
    uint32_t n, k;
    const float* d_tree;         /* device, n*k float32 (level order), owned by the server */
    const uint32_t* d_perm;      /* device, n uint32: original index of node s */
    const uint8_t* d_dim;        /* device, n uint8: split dimension of node s */
    double t_submit, t_admit, t_done;
    double device_ms;            /* device time of the batch that built it (copy-in included) */
    uint32_t batch_requests;     /* requests in that batch */
} kdt_result;

/* Create a server on the current device.  KDT_EINVAL for a bad config,
 * KDT_ENOMEM if the pool cannot be allocated. */
kdt_status kdt_server_create(const kdt_server_config* cfg, kdt_server** out);

/* Queue a request; *ticket identifies it.  KDT_EINVAL for bad arguments,
 * KDT_ENOMEM if the request cannot fit the pool even alone. */
kdt_status kdt_server_submit(kdt_server* server, const kdt_request* req, uint64_t* ticket);

/* KDT_OK and *out filled once the request is done, KDT_EBUSY before,
 * KDT_ENOTFOUND for an unknown or released ticket. */
kdt_status kdt_server_poll(kdt_server* server, uint64_t ticket, kdt_result* out);

/* As kdt_server_poll, but blocks until the request is done. */
kdt_status kdt_server_wait(kdt_server* server, uint64_t ticket, kdt_result* out);

/* Copy a done request's tree, permutation and dimensions (each nullable)
 * into caller device buffers of n*k float32 / n uint32 / n uint8, enqueued on
 * `stream`.  KDT_EBUSY if it is not done yet. */
kdt_status kdt_server_copy_out(kdt_server* server, uint64_t ticket, float* d_tree, uint32_t* d_perm,
                               uint8_t* d_dim, hipStream_t stream);

/* Give a done request's buffers back to the pool; its device pointers become
 * invalid.  KDT_EBUSY if it is not done yet. */
kdt_status kdt_server_release(kdt_server* server, uint64_t ticket);

/* Finish the queued and running requests, then free everything. */
kdt_status kdt_server_destroy(kdt_server* server);

/* Seconds on the monotonic clock of the server's timestamps. */
double kdt_clock(void);

/*
 * Measurement hook for benchmarks.  While enabled, every kernel a build
 * enqueues is bracketed by a pair of hipEvents recorded on the build's own
 * stream and tagged with the kernel's name and two byte counts:
 *   - alg_bytes: the bytes this implementation's step moves by design (e.g.
 *     a split pass reads and writes a 4k-byte rank record per live point);
 *   - method_bytes: the bytes the paper's method moves for the work the
 *     step completes: each iteration reads and writes every live point's k
 *     coordinates and 32-bit tag once, 8(k+1) bytes per live point (Sec. 3),
 *     and the final placement moves every point once more, 8k bytes
 *     (Sec. 5); steps that only prepare an iteration count 0.
 * Enabling adds two event records per launch.
 */
typedef struct kdt_kernel_stat {
    char name[32];        /* kernel name, e.g. "k_level_part" */
    uint64_t launches;    /* launches recorded since the last collect */
    double total_ms;      /* sum of event-measured durations */
    double alg_bytes;     /* sum of the implementation's bytes */
    double method_bytes;  /* sum of the paper method's bytes */
} kdt_kernel_stat;

kdt_status kdt_profile_enable(int on);

/* Wait for the recorded events, write one entry per kernel name (at most
 * max_entries) into out, clear the records and return the number of entries;
 * -1 if an event could not be read. */
int kdt_profile_collect(kdt_kernel_stat* out, int max_entries);

/* Static text for a status code. */
const char* kdt_status_string(int status);

/* Message of the last KDT_EDEVICE / KDT_EINVAL in the calling thread. */
const char* kdt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KDT_H */
