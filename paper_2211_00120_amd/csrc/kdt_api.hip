// kdt_api.hip -- host driver and C ABI (include/kdt.h) of the k-d tree build.
//
// A call builds a list of independent trees (one for kdt_build_ws, one per
// cloud for kdt_build_batched).  The planner splits them:
//
//   * a tree of at most TAIL_CAP points is built whole by one workgroup
//     (k_tail from the points: keys, per-dimension orders and every
//     iteration in LDS);
//   * larger trees go through init, prep, [root dims], k presorts x 4
//     passes, iteration 0, then iterations 1.. while some subtree is larger
//     than TAIL_CAP (each: radix select of every subtree's pivot key, the
//     pivot kernel that reads it off the histograms and places the node, then
//     one segmented onesweep split pass that applies the tag update), then
//     one tail launch that runs each tree's remaining iterations, each tree
//     from its own level.
//
// Every launch covers all trees that have work at that step, so the launch
// count of a batch is that of its largest tree.  With a single share the
// share travels in the kernel arguments; otherwise the launch reads a table
// that the call uploads into its workspace (from pinned host memory that the
// plan cache owns).
//
// The loop bounds follow the paper's iteration count with the two savings of
// Sec. 7.1: entries of fixed nodes are dropped from every iteration, and the
// lowest level needs no iteration of its own (iteration L-2 places the
// leaves directly, which replaces the final sort by tag of Sec. 5).
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/kdt.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"
#include "kdt_host.h"
#include "kdt_plan.h"

static_assert(kdt::KDT_STATUS_INTERNAL == KDT_STATUS_INTERNAL_BIT, "status bit of include/kdt.h");

// The workspace of kdt_build_static: a fixed array on every device the
// library runs on.  In host code this name is only a handle for the
// symbol lookup below; host code never passes it to a kernel or a copy, only
// the per-device address hipGetSymbolAddress returns.
static __device__ __align__(256) uint8_t scratch[KDT_STATIC_WS_BYTES];
static_assert(kdt::KDT_STATUS_NONFINITE == (uint32_t)KDT_ENONFINITE, "status code of include/kdt.h");

namespace {

using namespace kdt;

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

constexpr size_t ALIGN = WS_ALIGN;

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            set_err("%s failed: %s", #expr, hipGetErrorString(e_));                         \
            return KDT_EDEVICE;                                                             \
        }                                                                                   \
    } while (0)

kdt_status check_launch(const char* what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_err("%s launch failed: %s", what, hipGetErrorString(e));
        return KDT_EDEVICE;
    }
    return KDT_OK;
}

// ------------------------------------------------------------ profiling
// While enabled, every kernel enqueued by a build is bracketed by two
// hipEvents on the build's stream and tagged with its kind and two byte
// counts: the bytes this build's design moves in that step (`bytes`), and
// the bytes the paper's method moves for the work the step completes
// (`mbytes`): every iteration reads and writes each live point -- k
// coordinates and its 32-bit tag, 8(k+1) bytes -- once (Sec. 3), and the
// final placement moves each point once more, 8k bytes (Sec. 5).  Steps
// that only prepare an iteration (key prep, presorts, pivot selects) do no
// such work and count 0.
const char* const kind_names[KIND_COUNT] = {"k_init", "k_prep", "k_root_dim", "k_presort_pass",
                                            "k_level0", "k_level_select", "k_level_pivot", "k_level_part",
                                            "k_tail", "k_tail_whole", "share_tables", "k_word", "k_rank_bucket",
                                            "k_rank_window", "k_ip_init", "k_ip_setup", "k_ip_block", "k_ip_mgroup",
                                            "k_ip_group", "k_ip_deep", "k_ip_perm"};

struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes, mbytes;
};
struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<ProfRec> recs;
    hipEvent_t take()
    {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};
Profiler g_prof;

// Enqueue one kernel (or copy) through `fn`, with profiling events when enabled.
template <class F>
kdt_status run_kernel(hipStream_t st, int kind, double bytes, double mbytes, F&& fn)
{
    hipEvent_t a = nullptr, b = nullptr;
    const bool on = g_prof.on;
    if (on) {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        a = g_prof.take();
        b = g_prof.take();
        if (a) (void)hipEventRecord(a, st);
    }
    fn();
    if (kdt_status s = check_launch(kind_names[kind])) return s;
    if (on && a && b) {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        (void)hipEventRecord(b, st);
        g_prof.recs.push_back({kind, a, b, bytes, mbytes});
    }
    return KDT_OK;
}

// Bytes the paper's method moves in the iterations l0 .. L-2 of an n-point
// tree plus its final placement (see the profiling note above).
double method_bytes(uint32_t n, uint32_t k, uint32_t l0)
{
    const uint32_t L = num_levels(n);
    double b = 8.0 * k * n;
    for (uint32_t l = l0; l + 2u <= L; ++l) b += 8.0 * (k + 1.0) * (n - full_nodes(l));
    return b;
}

// method_bytes over the trees built by digit passes.
double method_bytes_large(const Plan& p, uint32_t k)
{
    double b = 0;
    for (uint32_t t : p.large) b += method_bytes(p.trees[t].n, k, 0u);
    return b;
}

kdt_status validate_k_mode(uint32_t k, int mode)
{
    if (k < 1 || k > 4) {
        set_err("k must be in 1..4 (got %u)", k);
        return KDT_EINVAL;
    }
    if (mode != KDT_DIM_ROUND_ROBIN && mode != KDT_DIM_WIDEST) {
        set_err("dim_mode must be KDT_DIM_ROUND_ROBIN or KDT_DIM_WIDEST (got %d)", mode);
        return KDT_EINVAL;
    }
    return KDT_OK;
}

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    if (!a || !b || !na || !nb) return false;
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

// Points and tree rows move as whole 16-byte (k = 4) or 8-byte (k = 2)
// vectors, so those arrays must be aligned to that.
kdt_status validate_row_align(uint32_t k, const void* pts, const void* tree)
{
    const uintptr_t a = k == 4 ? 16 : k == 2 ? 8 : 4;
    if (((uintptr_t)pts | (uintptr_t)tree) % a) {
        set_err("points and tree must be %zu-byte aligned for k = %u", (size_t)a, k);
        return KDT_EINVAL;
    }
    return KDT_OK;
}

// Checks shared by the caller-workspace entry points.
kdt_status validate_buffers(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim,
                            uint32_t* status, void* ws, size_t ws_bytes)
{
    if (p.ntotal > 0 && !pts) {
        set_err("points is null");
        return KDT_EINVAL;
    }
    if (!ws || ws_bytes < p.total) {
        set_err("workspace of %zu bytes needed (got %zu)", p.total, ws ? ws_bytes : (size_t)0);
        return KDT_EINVAL;
    }
    if (((uintptr_t)ws) % ALIGN) {
        set_err("workspace must be %zu-byte aligned", ALIGN);
        return KDT_EINVAL;
    }
    if (kdt_status s = validate_row_align(p.k, pts, tree)) return s;
    const size_t n = p.ntotal;
    const size_t pb = n * p.k * 4;
    if (overlaps(pts, pb, tree, pb) || overlaps(pts, pb, perm, n * 4) || overlaps(pts, pb, dim, n) ||
        overlaps(pts, pb, ws, ws_bytes) || overlaps(tree, pb, ws, ws_bytes) || overlaps(perm, n * 4, ws, ws_bytes) ||
        overlaps(dim, n, ws, ws_bytes) || overlaps(status, 4, ws, ws_bytes)) {
        set_err("points, outputs and workspace must not overlap");
        return KDT_EINVAL;
    }
    return KDT_OK;
}

// Shares of one launch: inline for a single share, else the device table.
Shares shares(const Plan& p, const std::vector<TreeStep>& steps, size_t table_off, const char* ws)
{
    Shares s{};
    s.nsteps = (uint32_t)steps.size();
    if (steps.size() == 1) {
        s.step0 = steps[0];
        s.tree0 = p.trees[steps[0].tree];
    } else {
        s.trees = (const TreeInfo*)(ws + p.o_tables + p.t_trees);
        s.steps = (const TreeStep*)(ws + p.o_tables + table_off);
    }
    return s;
}

// Enqueue every kernel of a planned call on `st`.  h_tables: the plan's
// share tables in pinned host memory (needed when p.tables).
kdt_status enqueue(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim, uint32_t* status,
                   char* ws, const void* h_tables, hipStream_t st, bool i32 = false)
{
    const uint32_t k = p.k;
    const bool widest = p.widest;
    const double K = k;
    uint32_t* dstatus = (uint32_t*)(ws + p.o_status);
    uint32_t* counters = (uint32_t*)(ws + p.o_counters);
    uint32_t* hist_rank = (uint32_t*)(ws + p.o_hist_rank);
    uint32_t* hist = (uint32_t*)(ws + p.o_hist);
    uint32_t* lb[2] = {(uint32_t*)(ws + p.o_lb[0]), (uint32_t*)(ws + p.o_lb[1])};
    uint32_t* keys = (uint32_t*)(ws + p.o_keys);
    uint32_t* perms = (uint32_t*)(ws + p.o_perms);
    uint32_t* ranks = (uint32_t*)(ws + p.o_ranks);
    uint32_t* recbase = (uint32_t*)(ws + p.o_rec);
    uint32_t* piv = (uint32_t*)(ws + p.o_piv);
    uint32_t* wcount = (uint32_t*)(ws + p.o_wcount);
    uint32_t* rec[2] = {recbase, recbase + p.rec_words};
    const uint32_t ntotal = (uint32_t)p.ntotal;
    const uint32_t nlarge_trees = (uint32_t)p.large.size();

    Outs o{};
    o.pts = pts;
    o.tree = tree;
    o.dim = widest ? nullptr : dim;
    o.nodeperm = perm ? perm : (uint32_t*)(ws + p.o_nodeperm);
    o.dimnode = (widest && dim) ? dim : (uint8_t*)(ws + p.o_dimnode);
    o.status = dstatus;
    o.tstatus = (uint32_t*)(ws + p.o_tstatus);
    o.box[0] = (uint32_t*)(ws + p.o_box[0]);
    o.box[1] = (uint32_t*)(ws + p.o_box[1]);
    o.i32 = i32 ? 1u : 0u;
    o.bbox = (uint32_t*)(ws + p.o_bbox);

    if (p.tables) {
        if (!h_tables) {
            set_err("internal: share tables missing");
            return KDT_EINVAL;
        }
        if (kdt_status s = run_kernel(st, KIND_TABLES, (double)p.blob.size(), 0.0, [&] {
                (void)hipMemcpyAsync(ws + p.o_tables, h_tables, p.blob.size(), hipMemcpyHostToDevice, st);
            }))
            return s;
    }

    // the look-back buffer of onesweep pass q is lb[q & 1]; init clears the
    // first one, pass q clears the one of pass q+1
    const std::vector<uint32_t>& pw = p.pass_words;
    auto next_words = [&](uint32_t q) { return q + 1 < pw.size() ? pw[q + 1] : 0u; };
    // histogram thirds 1 and 2 (iterations 1 and 2) start cleared; the split
    // of iteration l clears the third of iteration l+2
    const uint32_t hist12_words = p.levels.empty() ? 0u : p.hist_words * 2u;
    // split keys of iteration l live in skey[(l-1) & 1]: the presort keys
    // (free after the presorts) and the rank table (free after iteration 0)
    uint32_t* skey[2] = {keys, ranks};

    // a single tree of at most TAIL_CAP points: one launch, which zeroes the
    // status words itself and reports into the caller's (and the tree's own)
    if (p.large.empty() && p.small.size() == 1 && !p.tables) {
        o.status = status ? status : dstatus;
        TailArgs a{};
        a.sh = shares(p, p.small, p.t_small, ws);
        a.from_points = 1;
        a.init_status = 1;
        a.o = o;
        const uint32_t n1 = p.trees[p.small[0].tree].n;
        return run_kernel(st, KIND_WHOLE, n1 * (8.0 * K + 4.0), method_bytes(n1, k, 0u),
                          [&] { launch_tail((int)k, a, 1u, widest, st); });
    }

    if (kdt_status s = run_kernel(st, KIND_INIT, 0.0, 0.0, [&] {
            launch_init(dstatus, counters, hist_rank, nlarge_trees * k * 4 * RADIX_HOST, lb[0],
                        pw.empty() ? 0u : pw[0], hist + p.hist_words, hist12_words, wcount,
                        p.rank_dm ? k * RANK_MAX_WIN : 0u, o.tstatus, (uint32_t)p.trees.size(), o.bbox,
                        nlarge_trees, st);
        }))
        return s;

    // ---- whole trees of at most TAIL_CAP points ----
    if (!p.small.empty()) {
        TailArgs a{};
        a.sh = shares(p, p.small, p.t_small, ws);
        a.from_points = 1;
        a.o = o;
        double bytes = 0, mbytes = 0;
        for (const TreeStep& s : p.small) {
            bytes += p.trees[s.tree].n * (8.0 * K + 4.0);
            mbytes += method_bytes(p.trees[s.tree].n, k, 0u);
        }
        if (kdt_status s = run_kernel(st, KIND_WHOLE, bytes, mbytes,
                                      [&] { launch_tail((int)k, a, (uint32_t)p.small.size(), widest, st); }))
            return s;
    }

    if (!p.large.empty()) {
        double nlarge = 0;
        for (uint32_t t : p.large) nlarge += p.trees[t].n;
        PrepArgs pa{};
        pa.sh = shares(p, p.prep, p.t_prep, ws);
        pa.keys = keys;
        pa.hist = hist_rank;
        pa.ntotal = ntotal;
        pa.o = o;
        if (kdt_status s = run_kernel(st, KIND_PREP, nlarge * 8.0 * K, 0.0,
                                      [&] { launch_prep((int)k, pa, p.prep_tiles, widest, st); }))
            return s;
        // key summaries combined; split-widest: scene boxes and root dims
        if (kdt_status s = run_kernel(st, KIND_ROOT, 0.0, 0.0, [&] {
                launch_root_dim((int)k, shares(p, p.roots, p.t_roots, ws), o, nlarge_trees, widest, st);
            }))
            return s;

        // presort: per presort role (the root's dimension first, then the
        // others, see PresortArgs), 4 stable digit passes of (key, payload);
        // the (key, payload) ping-pongs live in the record region (>= 4 *
        // presort_group * ntotal words), which is free until iteration 0.  A
        // pass whose digit is the same in all keys of a tree is skipped for
        // that tree; for the profile's byte counts, the key summaries (and
        // the split-widest root dimensions) are read back (profiling builds
        // only)
        std::vector<uint32_t> keysum;
        std::vector<uint8_t> rootdim(nlarge_trees, 0u);
        if (g_prof.on) {
            keysum.resize((size_t)nlarge_trees * KEYSUM_WORDS);
            HIP_TRY(hipMemcpyAsync(keysum.data(), o.bbox, keysum.size() * 4, hipMemcpyDeviceToHost, st));
            if (widest)
                for (uint32_t i = 0; i < nlarge_trees; ++i)
                    HIP_TRY(hipMemcpyAsync(&rootdim[i], o.dimnode + p.trees[p.large[i]].off, 1,
                                           hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        // the plan's launches, each over a group of roles, the group's role j
        // with its own ping-pong (slot j: words [4j, 4j+4) * ntotal of the
        // record region)
        uint32_t q = 0;
        for (const Plan::PresortLaunch& pl : p.presort_launches) {
            const uint32_t r0 = pl.role0, nd = pl.ndims, ps = pl.pass;
            {
                PresortArgs a{};
                a.sh = shares(p, p.presort, p.t_presort, ws);
                a.keys = keys;
                a.kv_words = 2 * (size_t)ntotal;
                a.kv = recbase;
                a.keysum = o.bbox;
                a.pass = ps;
                a.role0 = r0;
                a.ndims = nd;
                a.hist = hist_rank;
                a.hist_stride = k * 4 * RADIX_HOST;
                a.lb = lb[q & 1];
                a.lb_dim_words = p.presort_tiles * RADIX_HOST;
                a.lb_zero = lb[(q + 1) & 1];
                a.lb_zero_n = next_words(q);
                a.counter = counters + q;
                if (p.xq) {
                    a.xq = (const uint32_t*)(ws + p.o_tables + p.t_xq);
                    a.xq_cnt = counters + MAX_PASSES + 8 * (size_t)(&pl - p.presort_launches.data());
                }
                a.perms = perms;
                // per-role arrays are written by the windowed scatter below
                a.rank_table = p.rank_dm ? nullptr : ranks;
                a.root_ranks = p.rank_dm ? ranks : nullptr;    // role 0's array
                a.k = k;
                a.dimnode = widest ? o.dimnode : nullptr;
                a.ntotal = ntotal;
                a.status = dstatus;
                a.place1 = (k == 1 && ps == 3) ? 1u : 0u;
                a.o = o;
                double bytes = 0;
                if (g_prof.on) {
                    for (uint32_t r = r0; r < r0 + nd; ++r)
                        for (uint32_t i = 0; i < nlarge_trees; ++i) {
                            const uint32_t d = role_dim(r, rootdim[i]);
                            const uint32_t vary =
                                keysum[i * KEYSUM_WORDS + 8 + d] ^ keysum[i * KEYSUM_WORDS + 12 + d];
                            auto runs = [&](uint32_t qq) { return ((vary >> (8 * qq)) & 0xFFu) != 0u; };
                            if (ps < 3 && !runs(ps)) continue;
                            bool first = true;
                            for (uint32_t qq = 0; qq < ps; ++qq) first = first && !runs(qq);
                            // a first pass reads the key (and, but for the root's
                            // role, the payload), a later one the pair
                            bytes += p.trees[p.large[i]].n * (first ? (r && p.rank_dm ? 16.0 : 12.0) : 16.0);
                        }
                }
                // with k = 1 the last pass places the trees: it completes
                // every iteration of the method
                const double mb = a.place1 ? method_bytes_large(p, k) : 0.0;
                if (kdt_status s = run_kernel(st, KIND_PRESORT, bytes, mb,
                                              [&] { launch_presort_pass(a, ps == 3, nd * p.presort_tiles, st); }))
                    return s;
            }
            ++q;
            if (p.rank_dm && ps == 3 && k > 1) {
                // the roles' ranks into their arrays, window by window; the
                // buckets take the ping-pong of the role just sorted
                for (uint32_t r = r0; r < r0 + nd; ++r) {
                    RankBucketArgs b{};
                    b.sh = shares(p, p.presort, p.t_presort, ws);
                    b.perm = perms + (size_t)r * ntotal;
                    b.pairs = recbase + 4 * (size_t)(r - r0) * ntotal;
                    b.wcount = wcount + (size_t)r * RANK_MAX_WIN;
                    b.wbits = p.rank_wbits;
                    b.nwin = p.rank_nwin;
                    b.status = dstatus;
                    if (kdt_status s = run_kernel(st, KIND_BUCKET, nlarge * 12.0, 0.0,
                                                  [&] { launch_rank_bucket(b, p.presort_tiles, st); }))
                        return s;
                    RankWindowArgs wa{};
                    wa.pairs = b.pairs;
                    wa.wcount = b.wcount;
                    wa.dm = ranks + (size_t)r * ntotal;
                    wa.wbits = p.rank_wbits;
                    wa.nwin = p.rank_nwin;
                    wa.chunks = std::max(1u, (1u << p.rank_wbits) / RANK_WIN_CHUNK);
                    wa.ntotal = ntotal;
                    if (kdt_status s = run_kernel(st, KIND_WINDOW, nlarge * 12.0, 0.0, [&] { launch_rank_window(wa, st); }))
                        return s;
                }
            }
        }

        if (k == 1) {
            // one dimension: the last presort pass has placed every large
            // tree (the sorted order is the tree's in-order sequence)
            if (status)
                if (kdt_status s = run_kernel(st, KIND_STATUS, 8.0, 0.0, [&] { launch_copy_word(status, dstatus, st); }))
                    return s;
            return KDT_OK;
        }

        // iteration 0 reads the ranks (per-role arrays: by root position,
        // streaming; point-major table: by index) and writes the records of
        // iteration 1 into rec[0]
        int cur = 0;
        {
            const bool keys1 = !p.levels.empty() && !p.levels[0].sorted;
            Level0Args a{};
            a.sh = shares(p, p.level0, p.t_level0, ws);
            a.perms = perms;
            a.rank_table = p.rank_dm ? nullptr : ranks;
            a.role_ranks = p.rank_dm ? ranks : nullptr;
            a.rout = rec[cur];
            a.kout = skey[0];
            a.hist = hist;
            a.keys_next = keys1 ? 1u : 0u;
            a.ntotal = ntotal;
            a.passes = p.P;
            a.radix_bits = p.RB;
            a.o = o;
            a.xmap = p.xmap0.empty() ? nullptr : (const uint32_t*)(ws + p.o_tables + p.t_xmap0);
            const uint32_t grid = p.xmap0.empty() ? p.prep_tiles : (uint32_t)p.xmap0.size();
            if (kdt_status s = run_kernel(st, KIND_LEVEL0, nlarge * (4.0 + 8.0 * K + (keys1 ? 4.0 : 0.0)),
                                          nlarge * 8.0 * (K + 1.0),
                                          [&] { launch_level0((int)k, a, grid, widest, st); }))
                return s;
        }

        // iterations 1 .. : pivot selects, then the split
        for (size_t li = 0; li < p.levels.size(); ++li) {
            const LevelLaunch& ll = p.levels[li];
            const uint32_t l = ll.level;
            double live = 0;
            for (const TreeStep& s : ll.steps) live += p.trees[s.tree].n - full_nodes(l);
            if (!ll.sorted) {
                for (int j = (int)p.P - 2; j >= 0; --j) {
                    LevelSelectArgs sa{};
                    sa.sh = shares(p, ll.ssteps, p.t_select[li], ws);
                    sa.kin = skey[(l - 1u) & 1u];
                    sa.hist = hist;
                    sa.passes = p.P;
                    sa.digit = (uint32_t)j;
                    sa.radix_bits = p.RB;
                    sa.status = dstatus;
                    sa.dimnode = widest ? o.dimnode : nullptr;
                    if (kdt_status s = run_kernel(st, KIND_SELECT, live * 4.0, 0.0,
                                                  [&] { launch_level_select(sa, ll.select_tiles, st); }))
                        return s;
                }
            }
            {
                LevelPivotArgs pa{};
                pa.sh = shares(p, ll.psteps, p.t_pivot[li], ws);
                pa.rin = rec[cur];
                pa.hist = hist;
                pa.piv = piv;
                pa.perms = perms;
                pa.root_payload = p.rank_dm ? 1u : 0u;
                pa.ntotal = ntotal;
                pa.passes = p.P;
                pa.radix_bits = p.RB;
                pa.sorted = ll.sorted ? 1u : 0u;
                pa.k = k;
                pa.o = o;
                double segs = 0;
                for (const TreeStep& s : ll.psteps) segs += make_level(p.trees[s.tree].n, l).nseg;
                const double per_seg = ll.sorted ? 4.0 * K : 4.0 * p.P * (1u << p.RB);
                if (kdt_status s = run_kernel(st, KIND_PIVOT, segs * per_seg, 0.0,
                                              [&] { launch_level_pivot((int)k, pa, ll.pivot_tiles, widest, st); }))
                    return s;
            }
            const bool keys_next = li + 1 < p.levels.size() && !p.levels[li + 1].sorted;
            const uint32_t zero_words = li + 2 < p.levels.size() ? p.levels[li + 2].hist_words : 0u;
            LevelPartArgs a{};
            a.sh = shares(p, ll.steps, p.t_level[li], ws);
            a.rin = rec[cur];
            a.rout = rec[cur ^ 1];
            a.kout = skey[l & 1u];
            a.hist = hist;
            a.piv = piv;
            a.passes = p.P;
            a.radix_bits = p.RB;
            a.items = ll.items;
            a.keys_next = keys_next ? 1u : 0u;
            a.lb = lb[q & 1];
            a.lb_zero = lb[(q + 1) & 1];
            a.lb_zero_n = next_words(q);
            a.zero2 = zero_words ? hist + ((l + 2u) % 3u) * p.hist_words : nullptr;
            a.zero2_n = zero_words;
            a.counter = counters + q;
            a.k = k;
            a.o = o;
            if (kdt_status s = run_kernel(st, KIND_PART, live * (8.0 * K + (keys_next ? 4.0 : 0.0)), live * 8.0 * (K + 1.0),
                                          [&] { launch_level_part((int)k, a, ll.tiles, widest, st); }))
                return s;
            cur ^= 1;
            ++q;
        }

        // every large tree's remaining iterations, each from its own level
        TailArgs a{};
        a.sh = shares(p, p.tail, p.t_tail, ws);
        a.rin[0] = rec[0];
        a.rin[1] = rec[1];
        a.from_points = 0;
        a.o = o;
        a.xmap = p.xmapt.empty() ? nullptr : (const uint32_t*)(ws + p.o_tables + p.t_xmapt);
        const uint32_t tail_grid = p.xmapt.empty() ? p.tail_groups : (uint32_t)p.xmapt.size();
        double tail_live = 0, tail_m = 0;
        for (const TreeStep& s : p.tail) {
            tail_live += p.trees[s.tree].n - full_nodes(s.level);
            tail_m += method_bytes(p.trees[s.tree].n, k, s.level);
        }
        if (kdt_status s = run_kernel(st, KIND_TAIL, tail_live * 4.0 * K, tail_m,
                                      [&] { launch_tail((int)k, a, tail_grid, widest, st); }))
            return s;
    }
    if (status)
        if (kdt_status s = run_kernel(st, KIND_STATUS, 8.0, 0.0, [&] { launch_copy_word(status, dstatus, st); }))
            return s;
    return KDT_OK;
}

// Plans of batched calls, keyed by (k, mode, offsets), with their share
// tables in pinned host memory.  A plan lives until kdt_release_cached(), so
// an enqueued (or graph-captured) upload always reads valid memory.
struct CachedPlan {
    Plan plan;
    void* pinned = nullptr;
};
std::mutex g_plan_mu;
std::map<std::string, std::shared_ptr<CachedPlan>> g_plans;

// pinned: also make sure the plan's tables are in pinned host memory
kdt_status batched_plan(const uint32_t* h_offsets, uint32_t C, uint32_t k, bool widest, bool pinned,
                        std::shared_ptr<CachedPlan>& out)
{
    std::vector<uint32_t> n(C);
    for (uint32_t c = 0; c < C; ++c) n[c] = h_offsets[c + 1] - h_offsets[c];
    // the tuning in effect is part of the key
    const PlanOptions opt = tuned_options(k, widest, plan_rank_bits(n));
    std::string key(24 + (size_t)(C + 1) * 4, '\0');
    const uint32_t head[6] = {k, widest ? 1u : 0u, opt.radix_bits, opt.max_items, opt.rank_layout, opt.presort_dims};
    memcpy(&key[0], head, 24);
    memcpy(&key[24], h_offsets, (size_t)(C + 1) * 4);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    std::shared_ptr<CachedPlan> cp;
    auto it = g_plans.find(key);
    if (it != g_plans.end()) {
        cp = it->second;
    } else {
        cp = std::make_shared<CachedPlan>();
        cp->plan = make_plan(n, k, widest, opt);
        g_plans.emplace(key, cp);
    }
    if (pinned && cp->plan.tables && !cp->pinned) {
        if (hipHostMalloc(&cp->pinned, cp->plan.blob.size(), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            cp->pinned = nullptr;
            set_err("hipHostMalloc of %zu bytes failed", cp->plan.blob.size());
            return KDT_ENOMEM;
        }
        memcpy(cp->pinned, cp->plan.blob.data(), cp->plan.blob.size());
    }
    out = cp;
    return KDT_OK;
}

kdt_status validate_offsets(const uint32_t* h_offsets, uint32_t C)
{
    if (!h_offsets || C == 0) {
        set_err("h_offsets must hold C+1 entries with C >= 1");
        return KDT_EINVAL;
    }
    if (h_offsets[0] != 0) {
        set_err("h_offsets[0] must be 0 (got %u)", h_offsets[0]);
        return KDT_EINVAL;
    }
    for (uint32_t c = 0; c < C; ++c)
        if (h_offsets[c + 1] < h_offsets[c]) {
            set_err("h_offsets must be non-decreasing (cloud %u)", c);
            return KDT_EINVAL;
        }
    if (h_offsets[C] > KDT_MAX_POINTS) {
        set_err("total point count %u exceeds KDT_MAX_POINTS", h_offsets[C]);
        return KDT_EINVAL;
    }
    return KDT_OK;
}

// Workspaces cached by kdt_build, one per (device, stream).
struct Cached {
    void* ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_cache_mu;
std::map<std::pair<int, hipStream_t>, Cached> g_cache;

kdt_status write_ok_status(uint32_t* d_status, hipStream_t stream)
{
    if (!d_status) return KDT_OK;
    kdt::launch_set_word(d_status, 0u, stream);
    return check_launch("status");
}

// Device address of `scratch` on the current device, looked up on the first
// call with that device current and kept (each device holds its own copy of
// the array at its own address).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};

kdt_status scratch_address(void** out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_err("device %d out of range for the static workspace", dev);
        return KDT_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_err("hipGetSymbolAddress of the static workspace failed: %s", hipGetErrorString(e));
            return KDT_EDEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return KDT_OK;
}

}  // namespace

namespace kdt {

kdt_status enqueue_plan(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim,
                        uint32_t* status, char* ws, const void* h_tables, hipStream_t st)
{
    return enqueue(p, pts, tree, perm, dim, status, ws, h_tables, st);
}

kdt_status launch_profiled(hipStream_t st, int kind, double bytes, double mbytes, const std::function<void()>& fn)
{
    return run_kernel(st, kind, bytes, mbytes, fn);
}

void set_last_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

}  // namespace kdt

extern "C" {

size_t kdt_workspace_bytes(uint32_t n, uint32_t k, int dim_mode)
{
    if (validate_k_mode(k, dim_mode) || n > KDT_MAX_POINTS) return 0;
    return workspace_bytes_any(std::vector<uint32_t>{n}, k, dim_mode == KDT_DIM_WIDEST);
}

static kdt_status build_ws_any(const float* d_points, uint32_t n, uint32_t k, int dim_mode, float* d_tree,
                               uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                               hipStream_t stream, bool i32)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (n > KDT_MAX_POINTS) {
        set_err("n = %u exceeds KDT_MAX_POINTS", n);
        return KDT_EINVAL;
    }
    const Plan p = make_plan(std::vector<uint32_t>{n}, k, dim_mode == KDT_DIM_WIDEST);
    if (kdt_status s = validate_buffers(p, d_points, d_tree, d_perm, d_dim, d_status, d_ws, ws_bytes)) return s;
    if (n == 0) return write_ok_status(d_status, stream);
    return enqueue(p, d_points, d_tree, d_perm, d_dim, d_status, (char*)d_ws, nullptr, stream, i32);
}

kdt_status kdt_build_ws(const float* d_points, uint32_t n, uint32_t k, int dim_mode, float* d_tree,
                        uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                        hipStream_t stream)
{
    return build_ws_any(d_points, n, k, dim_mode, d_tree, d_perm, d_dim, d_status, d_ws, ws_bytes, stream, false);
}

kdt_status kdt_build_ws_i32(const int32_t* d_points, uint32_t n, uint32_t k, int dim_mode, int32_t* d_tree,
                            uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                            hipStream_t stream)
{
    // the kernels move coordinates as 32-bit words; only their keys differ
    return build_ws_any((const float*)d_points, n, k, dim_mode, (float*)d_tree, d_perm, d_dim, d_status, d_ws,
                        ws_bytes, stream, true);
}

kdt_status kdt_permute_payload(const uint32_t* d_perm, uint32_t n, const void* d_in, uint32_t stride_bytes,
                               void* d_out, uint32_t* d_status, hipStream_t stream)
{
    if (n == 0 || stride_bytes == 0) return KDT_OK;
    if (!d_perm || !d_in || !d_out) {
        set_err("perm, payload and output must not be null");
        return KDT_EINVAL;
    }
    const size_t bytes = (size_t)n * stride_bytes;
    if (overlaps(d_in, bytes, d_out, bytes) || overlaps(d_perm, (size_t)n * 4, d_out, bytes)) {
        set_err("the payload output must not overlap its input or the permutation");
        return KDT_EINVAL;
    }
    kdt::launch_permute(d_perm, n, d_in, d_out, stride_bytes, d_status, stream);
    return check_launch("k_permute");
}

kdt_status kdt_build_static(const float* d_points, uint32_t n, uint32_t k, int dim_mode, float* d_tree,
                            uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status, hipStream_t stream)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (n > KDT_MAX_POINTS) {
        set_err("n = %u exceeds KDT_MAX_POINTS", n);
        return KDT_EINVAL;
    }
    const Plan p = make_plan(std::vector<uint32_t>{n}, k, dim_mode == KDT_DIM_WIDEST);
    const size_t need = workspace_bytes_any(std::vector<uint32_t>{n}, k, dim_mode == KDT_DIM_WIDEST);
    if (need > KDT_STATIC_WS_BYTES) {
        set_err("kdt_build_static: n = %u, k = %u needs %zu bytes of workspace, more than the %u-byte static "
                "workspace holds",
                n, k, need, KDT_STATIC_WS_BYTES);
        return KDT_EINVAL;
    }
    void* ws = nullptr;
    if (kdt_status s = scratch_address(&ws)) return s;
    if (kdt_status s = validate_buffers(p, d_points, d_tree, d_perm, d_dim, d_status, ws, KDT_STATIC_WS_BYTES))
        return s;
    if (n == 0) return write_ok_status(d_status, stream);
    return enqueue(p, d_points, d_tree, d_perm, d_dim, d_status, (char*)ws, nullptr, stream);
}

kdt_status kdt_build(float* d_points, uint32_t n, uint32_t k, int dim_mode, hipStream_t stream)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (n > KDT_MAX_POINTS || (n > 0 && !d_points)) {
        set_err("points is null or n exceeds KDT_MAX_POINTS");
        return KDT_EINVAL;
    }
    if (kdt_status s = validate_row_align(k, d_points, nullptr)) return s;
    if (n == 0) return KDT_OK;
    const Plan p = make_plan(std::vector<uint32_t>{n}, k, dim_mode == KDT_DIM_WIDEST);
    const size_t pb = align_up((size_t)n * k * 4);
    const size_t need = p.total + pb;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        Cached& c = g_cache[{dev, stream}];
        if (c.bytes < need) {
            if (c.ptr) {
                HIP_TRY(hipStreamSynchronize(stream));
                HIP_TRY(hipFree(c.ptr));
                c.ptr = nullptr;
                c.bytes = 0;
            }
            if (hipMalloc(&c.ptr, need) != hipSuccess) {
                (void)hipGetLastError();
                c.ptr = nullptr;
                set_err("hipMalloc of %zu bytes failed", need);
                return KDT_ENOMEM;
            }
            c.bytes = need;
        }
        ws = c.ptr;
    }
    // the build reads the points until the last node is placed, so it works
    // from a copy and writes the tree over the caller's array
    float* copy = (float*)((char*)ws + p.total);
    HIP_TRY(hipMemcpyAsync(copy, d_points, (size_t)n * k * 4, hipMemcpyDeviceToDevice, stream));
    return enqueue(p, copy, d_points, nullptr, nullptr, nullptr, (char*)ws, nullptr, stream);
}

size_t kdt_batched_workspace_bytes(const uint32_t* h_offsets, uint32_t C, uint32_t k, int dim_mode)
{
    if (validate_k_mode(k, dim_mode) || validate_offsets(h_offsets, C)) return 0;
    std::vector<uint32_t> n(C);
    for (uint32_t c = 0; c < C; ++c) n[c] = h_offsets[c + 1] - h_offsets[c];
    return workspace_bytes_any(n, k, dim_mode == KDT_DIM_WIDEST);
}

static kdt_status build_batched_any(const float* d_points, const uint32_t* h_offsets, uint32_t C, uint32_t k,
                                    int dim_mode, float* d_tree, uint32_t* d_perm, uint8_t* d_dim,
                                    uint32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream, bool i32)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (kdt_status s = validate_offsets(h_offsets, C)) return s;
    std::shared_ptr<CachedPlan> cp;
    if (kdt_status s = batched_plan(h_offsets, C, k, dim_mode == KDT_DIM_WIDEST, false, cp)) return s;
    const Plan& p = cp->plan;
    if (kdt_status s = validate_buffers(p, d_points, d_tree, d_perm, d_dim, d_status, d_ws, ws_bytes)) return s;
    if (p.ntotal == 0) return write_ok_status(d_status, stream);
    if (kdt_status s = batched_plan(h_offsets, C, k, dim_mode == KDT_DIM_WIDEST, true, cp)) return s;
    return enqueue(p, d_points, d_tree, d_perm, d_dim, d_status, (char*)d_ws, cp->pinned, stream, i32);
}

kdt_status kdt_build_batched(const float* d_points, const uint32_t* h_offsets, uint32_t C, uint32_t k,
                             int dim_mode, float* d_tree, uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status,
                             void* d_ws, size_t ws_bytes, hipStream_t stream)
{
    return build_batched_any(d_points, h_offsets, C, k, dim_mode, d_tree, d_perm, d_dim, d_status, d_ws, ws_bytes,
                             stream, false);
}

kdt_status kdt_build_batched_i32(const int32_t* d_points, const uint32_t* h_offsets, uint32_t C, uint32_t k,
                                 int dim_mode, int32_t* d_tree, uint32_t* d_perm, uint8_t* d_dim,
                                 uint32_t* d_status, void* d_ws, size_t ws_bytes, hipStream_t stream)
{
    return build_batched_any((const float*)d_points, h_offsets, C, k, dim_mode, (float*)d_tree, d_perm, d_dim,
                             d_status, d_ws, ws_bytes, stream, true);
}

kdt_status kdt_tune_batched(const float* d_points, const uint32_t* h_offsets, uint32_t C, uint32_t k, int dim_mode,
                            void* d_ws, size_t ws_bytes, uint32_t reps, hipStream_t stream, kdt_tuning* best)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (kdt_status s = validate_offsets(h_offsets, C)) return s;
    if (!best) {
        set_err("best is null");
        return KDT_EINVAL;
    }
    const bool widest = dim_mode == KDT_DIM_WIDEST;
    std::vector<uint32_t> n(C);
    for (uint32_t c = 0; c < C; ++c) n[c] = h_offsets[c + 1] - h_offsets[c];
    const uint64_t ntotal = h_offsets[C];
    if (ntotal > 0 && !d_points) {
        set_err("points is null");
        return KDT_EINVAL;
    }
    const size_t need = workspace_bytes_any(n, k, widest);
    if (!d_ws || ws_bytes < need || ((uintptr_t)d_ws) % ALIGN) {
        set_err("a %zu-byte aligned workspace of %zu bytes is needed", (size_t)ALIGN, need);
        return KDT_EINVAL;
    }
    memset(best, 0, sizeof *best);
    const uint32_t bits = plan_rank_bits(n);
    if (ntotal == 0 || bits == 0) return KDT_OK;   // no tree is built by digit passes: nothing to choose
    reps = reps ? reps : 1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    kdt_status rc = KDT_OK;
    PlanOptions chosen;
    float best_ms = 0.f;
    for (const PlanOptions& cand : tuning_candidates()) {
        const Plan p = make_plan(n, k, widest, cand);
        void* pinned = nullptr;
        if (p.tables) {
            if (hipHostMalloc(&pinned, p.blob.size(), hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                set_err("hipHostMalloc of %zu bytes failed", p.blob.size());
                rc = KDT_ENOMEM;
                break;
            }
            memcpy(pinned, p.blob.data(), p.blob.size());
        }
        float ms = 0.f;
        rc = enqueue(p, d_points, nullptr, nullptr, nullptr, nullptr, (char*)d_ws, pinned, stream);   // warm-up
        if (rc == KDT_OK && hipEventRecord(e0, stream) != hipSuccess) rc = KDT_EDEVICE;
        for (uint32_t r = 0; rc == KDT_OK && r < reps; ++r)
            rc = enqueue(p, d_points, nullptr, nullptr, nullptr, nullptr, (char*)d_ws, pinned, stream);
        if (rc == KDT_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            rc = KDT_EDEVICE;
        (void)hipStreamSynchronize(stream);
        if (pinned) (void)hipHostFree(pinned);
        if (rc != KDT_OK) break;
        ms /= (float)reps;
        if (best_ms == 0.f || ms < best_ms) {
            best_ms = ms;
            chosen = cand;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != KDT_OK) {
        if (rc == KDT_EDEVICE && !g_err[0]) set_err("HIP error while timing a candidate");
        return rc;
    }
    set_tuned_options(k, widest, bits, chosen);
    best->radix_bits = chosen.radix_bits;
    best->level_items = chosen.max_items;
    best->rank_layout = chosen.rank_layout;
    best->presort_dims = chosen.presort_dims;
    best->ms = best_ms;
    return KDT_OK;
}

kdt_status kdt_tuning_get(uint32_t k, int dim_mode, uint32_t rank_bits, kdt_tuning* out)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (!out || rank_bits > 32) {
        set_err("bad arguments");
        return KDT_EINVAL;
    }
    const PlanOptions o = tuned_options(k, dim_mode == KDT_DIM_WIDEST, rank_bits);
    memset(out, 0, sizeof *out);
    out->radix_bits = o.radix_bits;
    out->level_items = o.max_items;
    out->rank_layout = o.rank_layout;
    out->presort_dims = o.presort_dims;
    return KDT_OK;
}

kdt_status kdt_tuning_set(uint32_t k, int dim_mode, uint32_t rank_bits, const kdt_tuning* t)
{
    if (kdt_status s = validate_k_mode(k, dim_mode)) return s;
    if (!t || rank_bits > 32 || (t->radix_bits && (t->radix_bits < 8 || t->radix_bits > 10)) ||
        (t->level_items && t->level_items != 4 && t->level_items != (uint32_t)PART_ITEMS) || t->rank_layout > 2 ||
        t->presort_dims > 4) {
        set_err("tuning must have radix_bits 0 or 8..10, level_items 0, 4 or %d, rank_layout 0..2 and "
                "presort_dims 0..4", PART_ITEMS);
        return KDT_EINVAL;
    }
    PlanOptions o;
    o.radix_bits = t->radix_bits;
    o.max_items = t->level_items;
    o.rank_layout = t->rank_layout;
    o.presort_dims = t->presort_dims;
    set_tuned_options(k, dim_mode == KDT_DIM_WIDEST, rank_bits, o);
    return KDT_OK;
}

kdt_status kdt_tuning_save(const char* path)
{
    if (!path || !save_tuning(path)) {
        set_err("could not write the tuning file");
        return KDT_EINVAL;
    }
    return KDT_OK;
}

kdt_status kdt_tuning_load(const char* path)
{
    if (!path || !load_tuning(path)) {
        set_err("could not read a valid tuning file");
        return KDT_EINVAL;
    }
    return KDT_OK;
}

void kdt_tuning_clear(void) { clear_tuning(); }

void kdt_release_cached(void)
{
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        int prev = 0;
        (void)hipGetDevice(&prev);
        for (auto& kv : g_cache) {
            if (!kv.second.ptr) continue;
            (void)hipSetDevice(kv.first.first);
            (void)hipStreamSynchronize(kv.first.second);
            (void)hipFree(kv.second.ptr);
        }
        g_cache.clear();
        (void)hipSetDevice(prev);
    }
    std::lock_guard<std::mutex> lk(g_plan_mu);
    if (!g_plans.empty()) {
        // uploads of batched share tables may still be queued on any stream
        (void)hipDeviceSynchronize();
        for (auto& kv : g_plans)
            if (kv.second->pinned) (void)hipHostFree(kv.second->pinned);
        g_plans.clear();
    }
}

const char* kdt_status_string(int status)
{
    switch (status) {
    case KDT_OK: return "ok";
    case KDT_EINVAL: return "invalid argument";
    case KDT_ENOMEM: return "out of device memory";
    case KDT_EDEVICE: return "HIP error";
    case KDT_ENONFINITE: return "non-finite input coordinate";
    case KDT_EBUSY: return "request not finished";
    case KDT_ENOTFOUND: return "unknown ticket";
    default: return "unknown status";
    }
}

const char* kdt_last_error(void) { return g_err; }

kdt_status kdt_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on != 0;
    return KDT_OK;
}

int kdt_profile_collect(kdt_kernel_stat* out, int max_entries)
{
    std::lock_guard<std::mutex> lk(g_prof.mu);
    kdt_kernel_stat acc[KIND_COUNT];
    memset(acc, 0, sizeof acc);
    int rc = 0;
    for (const ProfRec& r : g_prof.recs) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) {
            set_err("profiling events could not be read");
            rc = -1;
            continue;
        }
        acc[r.kind].launches += 1;
        acc[r.kind].total_ms += ms;
        acc[r.kind].alg_bytes += r.bytes;
        acc[r.kind].method_bytes += r.mbytes;
    }
    g_prof.recs.clear();
    g_prof.used = 0;
    if (rc < 0) return rc;
    int m = 0;
    for (int kk = 0; kk < KIND_COUNT && m < max_entries; ++kk) {
        if (!acc[kk].launches) continue;
        acc[kk].name[0] = 0;
        strncpy(acc[kk].name, kind_names[kk], sizeof acc[kk].name - 1);
        if (out) out[m] = acc[kk];
        ++m;
    }
    return m;
}

}  // extern "C"
