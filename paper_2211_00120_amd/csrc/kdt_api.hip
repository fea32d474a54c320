// kdt_api.hip -- host driver and C ABI (include/kdt.h) of the k-d tree build.
//
// The driver validates arguments, carves the caller's workspace, and
// enqueues the kernel sequence of one build on the caller's stream:
//
//   init, prep, [root dim], k presorts x 4 passes, iteration 0,
//   iterations 1.. with segmented onesweep passes while a subtree is larger
//   than one workgroup's tile, then block-local iterations down to L-2.
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

#include <map>
#include <vector>
#include <mutex>
#include <utility>

#include "../../include/kdt.h"
#include "kdt_kernels.h"
#include "kdt_layout.h"

namespace {

thread_local char g_err[512] = "";

void set_err(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) & ~(ALIGN - 1); }

// Everything about one build that depends only on (n, k, mode).
struct Plan {
    uint32_t n = 0, k = 0;
    bool widest = false;
    uint32_t L = 0;            // levels of the tree
    uint32_t B = 0;            // bits of a rank
    uint32_t P = 0;            // digit passes per level sort
    uint32_t RB = 8;           // bits per digit of the level sorts
    uint32_t first_local = 0;  // first iteration run block-locally
    uint32_t max_tiles = 1;    // look-back words per buffer / 256
    uint32_t max_hist_segs = 2;
    // workspace offsets (bytes)
    size_t o_ctl, o_counters, o_hist_rank, o_hist[2], o_lb[2], o_keys, o_perms, o_ranks, o_rec, o_nodeperm,
        o_dimnode, o_box[2], total;
    size_t rec_words;          // words per record buffer
};

// Records per thread of the level-l sort tiles (tile = 512 * items): the
// largest tile that the level's biggest subtree still fills.
#ifndef KDT_LEVEL_MAX_ITEMS
#define KDT_LEVEL_MAX_ITEMS 8
#endif
uint32_t level_items(uint32_t n, uint32_t l)
{
    const kdt::Level v = kdt::make_level(n, l);
    const uint32_t big = 2u * v.W - 1u;
    uint32_t items = big >= 8192u ? 16u : (big >= 4096u ? 8u : 4u);
    return items < KDT_LEVEL_MAX_ITEMS ? items : KDT_LEVEL_MAX_ITEMS;
}

bool level_is_global(const Plan& p, uint32_t l)
{
    return l >= 1 && l + 2 <= p.L && l < p.first_local;
}

Plan make_plan(uint32_t n, uint32_t k, bool widest)
{
    using namespace kdt;
    Plan p;
    p.n = n;
    p.k = k;
    p.widest = widest;
    p.L = num_levels(n);
    p.B = rank_bits(n);
    // fewest digit passes over a B-bit rank with 8..10-bit digits, then the
    // narrowest digit that keeps that pass count
    {
        const uint32_t pmin = p.B ? (p.B + 9u) / 10u : 0u;
        p.RB = 10;
        for (uint32_t rb = 8; rb <= 10; ++rb)
            if (p.B == 0 || (p.B + rb - 1u) / rb == pmin) { p.RB = rb; break; }
        p.P = p.B ? (p.B + p.RB - 1u) / p.RB : 0u;
    }
    // first iteration whose largest subtree (2W - 1 points) fits a local tile
    p.first_local = 1;
    while (p.first_local + 2 <= p.L) {
        const uint32_t W = 1u << (p.L - p.first_local - 1u);
        if (2u * W - 1u <= TAIL_CAP) break;
        ++p.first_local;
    }
    p.max_tiles = n ? ceil_div(n, PRESORT_TILE) : 1u;
    for (uint32_t l = 1; l + 2 <= p.L; ++l) {
        if (!level_is_global(p, l)) continue;
        const Level v = make_level(n, l);
        const SegTiles t = tiles_level(v, 512u * level_items(n, l));
        if (t.tiles > p.max_tiles) p.max_tiles = t.tiles;
        if (v.nseg * 2u > p.max_hist_segs) p.max_hist_segs = v.nseg * 2u;
    }
    const size_t N = n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    p.o_ctl = take(CTL_WORDS * 4);
    p.o_counters = take(MAX_PASSES * 4);
    p.o_hist_rank = take((size_t)k * 4 * RADIX_HOST * 4);
    const size_t hist_bytes = (size_t)p.max_hist_segs * (p.P ? p.P : 1u) * (1u << p.RB) * 4;
    p.o_hist[0] = take(hist_bytes);
    p.o_hist[1] = take(hist_bytes);
    const size_t lb_bytes = (size_t)p.max_tiles * MAX_BINS * 4;
    p.o_lb[0] = take(lb_bytes);
    p.o_lb[1] = take(lb_bytes);
    p.o_keys = take(N * k * 4);
    p.o_perms = take(N * k * 4);
    p.o_ranks = take(N * k * 4);
    p.rec_words = N * k > 2 * N ? N * k : 2 * N;     // also holds the presort's (key, value) ping-pong
    p.o_rec = take(p.rec_words * 2 * 4);
    p.o_nodeperm = take(N * 4);
    p.o_dimnode = take(N);
    // split-widest domain tables: levels up to the tail's first level
    const uint32_t box_level = p.L >= 2 ? (p.first_local < p.L - 2 ? p.first_local : p.L - 2) : 0u;
    const size_t box_bytes = ((size_t)1 << box_level) * 8 * 4;
    p.o_box[0] = take(box_bytes);
    p.o_box[1] = take(box_bytes);
    p.total = off;
    return p;
}

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
// hipEvents on the build's stream and tagged with its kind and algorithmic
// bytes (the bytes the step must move by definition).
enum Kind { KIND_INIT, KIND_PREP, KIND_ROOT, KIND_PRESORT, KIND_LEVEL0, KIND_HIST, KIND_PASS, KIND_TAIL,
            KIND_STATUS, KIND_COUNT };
const char* const kind_names[KIND_COUNT] = {"k_init", "k_prep", "k_root_dim", "k_presort_pass", "k_level0",
                                            "k_level_hist", "k_level_pass", "k_tail", "k_word"};

struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes;
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

// Enqueue one kernel through `fn`, with profiling events when enabled.
template <class F>
kdt_status run_kernel(hipStream_t st, int kind, double bytes, F&& fn)
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
        g_prof.recs.push_back({kind, a, b, bytes});
    }
    return KDT_OK;
}

kdt_status validate(const float* pts, uint32_t n, uint32_t k, int mode)
{
    if (k < 1 || k > 4) {
        set_err("k must be in 1..4 (got %u)", k);
        return KDT_EINVAL;
    }
    if (mode != KDT_DIM_ROUND_ROBIN && mode != KDT_DIM_WIDEST) {
        set_err("dim_mode must be KDT_DIM_ROUND_ROBIN or KDT_DIM_WIDEST (got %d)", mode);
        return KDT_EINVAL;
    }
    if (n > KDT_MAX_POINTS) {
        set_err("n = %u exceeds KDT_MAX_POINTS", n);
        return KDT_EINVAL;
    }
    if (n > 0 && !pts) {
        set_err("points is null");
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

kdt_status enqueue_build(const Plan& p, const float* pts, float* tree, uint32_t* perm, uint8_t* dim,
                         uint32_t* status, char* ws, hipStream_t st)
{
    using namespace kdt;
    const uint32_t n = p.n, k = p.k;
    const bool widest = p.widest;
    uint32_t* ctl = (uint32_t*)(ws + p.o_ctl);
    uint32_t* counters = (uint32_t*)(ws + p.o_counters);
    uint32_t* hist_rank = (uint32_t*)(ws + p.o_hist_rank);
    uint32_t* hist[2] = {(uint32_t*)(ws + p.o_hist[0]), (uint32_t*)(ws + p.o_hist[1])};
    uint32_t* lb[2] = {(uint32_t*)(ws + p.o_lb[0]), (uint32_t*)(ws + p.o_lb[1])};
    uint32_t* keys = (uint32_t*)(ws + p.o_keys);
    uint32_t* perms = (uint32_t*)(ws + p.o_perms);
    uint32_t* ranks = (uint32_t*)(ws + p.o_ranks);
    uint32_t* recbase = (uint32_t*)(ws + p.o_rec);
    uint32_t* rec[2] = {recbase, recbase + p.rec_words};
    uint32_t* nodeperm = perm ? perm : (uint32_t*)(ws + p.o_nodeperm);
    uint8_t* dimnode = (widest && dim) ? dim : (uint8_t*)(ws + p.o_dimnode);

    if (n == 0) return KDT_OK;

    // Onesweep passes of the build, in order, with their tile counts: the
    // look-back buffer of pass q is lb[q & 1], cleared by pass q-1 (or init).
    const uint32_t presort_tiles = ceil_div(n, PRESORT_TILE);
    // (look-back words a pass uses = its tiles * its digit values)
    uint32_t pass_words[MAX_PASSES];
    uint32_t npass = 0;
    for (uint32_t d = 0; d < k; ++d)
        for (int q = 0; q < 4; ++q) pass_words[npass++] = presort_tiles * RADIX_HOST;
    for (uint32_t l = 1; l + 2 <= p.L; ++l)
        if (level_is_global(p, l)) {
            const uint32_t t = tiles_level(make_level(n, l), 512u * level_items(n, l)).tiles;
            for (uint32_t q = 0; q < p.P; ++q) pass_words[npass++] = t << p.RB;
        }
    auto next_words = [&](uint32_t q) { return q + 1 < npass ? pass_words[q + 1] : 0u; };
    const uint32_t NBL = 1u << p.RB;

    const bool level1_global = level_is_global(p, 1);
    const double N = n, K = k;
    if (kdt_status s = run_kernel(st, KIND_INIT, 4.0 * (pass_words[0] + (k * 4 + 2 * p.P) * RADIX_HOST), [&] {
            launch_init(ctl, counters, hist_rank, k * 4 * RADIX_HOST, lb[0], pass_words[0],
                        level1_global ? hist[1] : nullptr, 2u * p.P * NBL, st);
        }))
        return s;
    if (kdt_status s = run_kernel(st, KIND_PREP, N * 8.0 * K,
                                  [&] { launch_prep((int)k, pts, n, keys, hist_rank, ctl, widest, st); }))
        return s;
    if (widest)
        if (kdt_status s = run_kernel(st, KIND_ROOT, 0.0,
                                      [&] { launch_root_dim((int)k, ctl, dimnode, (float*)(ws + p.o_box[0]), st); }))
            return s;

    // presort: per dimension, 4 stable digit passes of (key, index)
    uint32_t q = 0;
    // (key, index) ping-pong of the presort: two n-pair arrays inside the
    // record region (2 * rec_words >= 4n words), free until iteration 0
    uint32_t* kv[2] = {recbase, recbase + 2 * (size_t)n};
    for (uint32_t d = 0; d < k; ++d) {
        for (uint32_t ps = 0; ps < 4; ++ps, ++q) {
            PresortArgs a{};
            a.kin = keys + (size_t)d * n;
            a.kvin = ps == 0 ? nullptr : kv[(ps - 1) & 1];
            a.kvout = kv[ps & 1];
            a.hist = hist_rank + (d * 4 + ps) * RADIX_HOST;
            a.lb = lb[q & 1];
            a.lb_zero = lb[(q + 1) & 1];
            a.lb_zero_n = next_words(q);
            a.counter = counters + q;
            a.n = n;
            a.shift = 8 * ps;
            a.perm_out = perms + (size_t)d * n;
            a.rank_table = ranks;
            a.k = k;
            a.dim = d;
            a.status = ctl + CTL_STATUS;
            if (kdt_status s = run_kernel(st, KIND_PRESORT, N * (ps == 0 ? 12.0 : 16.0),
                                          [&] { launch_presort_pass(a, ps == 0, ps == 3, presort_tiles, st); }))
                return s;
        }
    }

    Outs o{};
    o.pts = pts;
    o.tree = tree;
    o.dim = widest ? nullptr : dim;
    o.nodeperm = nodeperm;
    o.dimnode = dimnode;
    o.perm0 = perms;
    o.ctl = ctl;
    o.status = ctl + CTL_STATUS;
    o.box[0] = (float*)(ws + p.o_box[0]);
    o.box[1] = (float*)(ws + p.o_box[1]);
    o.n = n;

    // iteration 0
    int cur = 0;    // record buffer holding the current iteration's input
    {
        Level0Args a{};
        a.perms = perms;
        a.rank_table = ranks;
        a.rout = rec[cur];
        a.hist_next = (level1_global && !widest) ? hist[1] : nullptr;
        a.next_passes = p.P;
        a.radix_bits = p.RB;
        a.o = o;
        if (kdt_status s = run_kernel(st, KIND_LEVEL0, N * (4.0 + 8.0 * K),
                                      [&] { launch_level0((int)k, a, widest, st); }))
            return s;
    }

    // iterations 1 .. L-2
    for (uint32_t l = 1; l + 2 <= p.L; ++l) {
        const Level v = make_level(n, l);
        if (level_is_global(p, l)) {
            const uint32_t items = level_items(n, l);
            const SegTiles tl = tiles_level(v, 512u * items);
            uint32_t* h = hist[l & 1];
            if (widest) {
                LevelHistArgs ha{};
                ha.rin = rec[cur];
                ha.dimnode = dimnode;
                ha.hist = h;
                ha.passes = p.P;
                ha.radix_bits = p.RB;
                ha.v = v;
                ha.tl = tiles_level(v, HIST_TILE);
                ha.status = ctl + CTL_STATUS;
                if (kdt_status s = run_kernel(st, KIND_HIST, (double)(n - v.Fl) * 4.0 * K,
                                              [&] { launch_level_hist((int)k, ha, st); }))
                    return s;
            }
            const bool next_global = level_is_global(p, l + 1);
            const uint32_t next_hist_n = next_global ? 2u * v.nseg * p.P * NBL : 0u;
            for (uint32_t ps = 0; ps < p.P; ++ps, ++q) {
                const bool last = ps + 1 == p.P;
                LevelPassArgs a{};
                a.rin = rec[cur];
                a.rout = rec[cur ^ 1];
                a.hist = h;
                a.passes = p.P;
                a.pass = ps;
                a.shift = p.RB * ps;
                a.radix_bits = p.RB;
                a.items = items;
                a.lb = lb[q & 1];
                a.lb_zero = lb[(q + 1) & 1];
                a.lb_zero_n = next_words(q);
                a.zero2 = (ps == 0 && next_global) ? hist[(l + 1) & 1] : nullptr;
                a.zero2_n = (ps == 0) ? next_hist_n : 0u;
                a.counter = counters + q;
                a.v = v;
                a.tl = tl;
                a.dim_rr = l % k;
                a.hist_next = (last && next_global && !widest) ? hist[(l + 1) & 1] : nullptr;
                a.next_passes = p.P;
                a.dim_next_rr = (l + 1) % k;
                a.o = o;
                if (kdt_status s = run_kernel(st, KIND_PASS, (double)(n - v.Fl) * 8.0 * K,
                                              [&] { launch_level_pass((int)k, a, last, widest, st); }))
                    return s;
                cur ^= 1;
            }
        } else {
            // every subtree of iteration l fits one workgroup: the tail runs
            // iterations l .. L-2 in one launch
            TailArgs a{};
            a.rin = rec[cur];
            a.v0 = v;
            const uint32_t big = 2u * v.W - 1u;
            a.G = TAIL_CAP / big;
            if (a.G > v.nseg) a.G = v.nseg;
            if (a.G > 2u) a.G = 2u;
            a.rank_bits = p.B;
            a.o = o;
            if (kdt_status s = run_kernel(st, KIND_TAIL, (double)(n - v.Fl) * 4.0 * K,
                                          [&] { launch_tail((int)k, a, widest, st); }))
                return s;
            break;
        }
    }
    if (status) {
        if (kdt_status s = run_kernel(st, KIND_STATUS, 8.0,
                                      [&] { launch_copy_word(status, ctl + CTL_STATUS, st); }))
            return s;
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

}  // namespace

extern "C" {

size_t kdt_workspace_bytes(uint32_t n, uint32_t k, int dim_mode)
{
    if (k < 1 || k > 4 || n > KDT_MAX_POINTS) return 0;
    if (dim_mode != KDT_DIM_ROUND_ROBIN && dim_mode != KDT_DIM_WIDEST) return 0;
    return make_plan(n, k, dim_mode == KDT_DIM_WIDEST).total;
}

kdt_status kdt_build_ws(const float* d_points, uint32_t n, uint32_t k, int dim_mode, float* d_tree,
                        uint32_t* d_perm, uint8_t* d_dim, uint32_t* d_status, void* d_ws, size_t ws_bytes,
                        hipStream_t stream)
{
    if (kdt_status s = validate(d_points, n, k, dim_mode)) return s;
    const Plan p = make_plan(n, k, dim_mode == KDT_DIM_WIDEST);
    if (!d_ws || ws_bytes < p.total) {
        set_err("workspace of %zu bytes needed (got %zu)", p.total, d_ws ? ws_bytes : (size_t)0);
        return KDT_EINVAL;
    }
    if (((uintptr_t)d_ws) % ALIGN) {
        set_err("workspace must be %zu-byte aligned", ALIGN);
        return KDT_EINVAL;
    }
    const size_t pb = (size_t)n * k * 4;
    if (overlaps(d_points, pb, d_tree, pb) || overlaps(d_points, pb, d_perm, (size_t)n * 4) ||
        overlaps(d_points, pb, d_dim, n) || overlaps(d_points, pb, d_ws, ws_bytes) ||
        overlaps(d_tree, pb, d_ws, ws_bytes) || overlaps(d_perm, (size_t)n * 4, d_ws, ws_bytes) ||
        overlaps(d_dim, n, d_ws, ws_bytes) || overlaps(d_status, 4, d_ws, ws_bytes)) {
        set_err("points, outputs and workspace must not overlap");
        return KDT_EINVAL;
    }
    if (n == 0) {
        if (d_status) {
            kdt::launch_set_word(d_status, 0u, stream);
            return check_launch("status");
        }
        return KDT_OK;
    }
    return enqueue_build(p, d_points, d_tree, d_perm, d_dim, d_status, (char*)d_ws, stream);
}

kdt_status kdt_build(float* d_points, uint32_t n, uint32_t k, int dim_mode, hipStream_t stream)
{
    if (kdt_status s = validate(d_points, n, k, dim_mode)) return s;
    if (n == 0) return KDT_OK;
    const Plan p = make_plan(n, k, dim_mode == KDT_DIM_WIDEST);
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
    return enqueue_build(p, copy, d_points, nullptr, nullptr, nullptr, (char*)ws, stream);
}

void kdt_release_cached(void)
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
