// Host-side structures of the engine shared by the executor (engine.cpp) and
// the batch / serving layer (serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "../../include/atrapos.h"
#include "internal.hpp"
#include "otree.hpp"
#include "planner.hpp"

namespace atp {

// Per-kernel event timing of one lane (ATP_OPT_PROFILE).
struct KernelTimer {
    struct Rec {
        std::string name;
        hipEvent_t e0, e1;
    };
    std::string suffix;  // appended to kernel names (per-product breakdown)
    std::string only;    // time only launches of this kernel name (empty: all)
    bool skip = false;   // the current launch is not timed
    std::vector<hipEvent_t> free_events;
    std::vector<Rec> pending;
    std::map<std::string, std::pair<double, int64_t>> acc;
    std::map<std::string, double> bytes;
    hipEvent_t take() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void flush() {
        for (auto &r : pending) {
            float ms = 0;
            if (r.e0 && r.e1 && hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess) {
                auto &a = acc[r.name];
                a.first += ms;
                a.second += 1;
            }
            if (r.e0) free_events.push_back(r.e0);
            if (r.e1) free_events.push_back(r.e1);
        }
        pending.clear();
    }
    ~KernelTimer() {
        for (auto &r : pending) {
            if (r.e0) (void)hipEventDestroy(r.e0);
            if (r.e1) (void)hipEventDestroy(r.e1);
        }
        for (auto e : free_events) (void)hipEventDestroy(e);
    }
};

// ---------------------------------------------------------------------------
// device memory: caching pool (or caller callbacks) with an optional budget

struct Pool {
    void *(*user_alloc)(size_t, void *) = nullptr;
    void (*user_free)(void *, void *) = nullptr;
    void *user = nullptr;
    uint64_t budget = 0;
    int64_t held = 0;  // bytes obtained from the runtime (in use + cached)
    std::multimap<size_t, void *> cache;
    std::map<void *, size_t> live;
    std::recursive_mutex mu;  // lanes release each other's buffers (cache eviction, results)
    size_t cached = 0;                // bytes of free blocks in `cache`
    size_t cache_limit = (size_t)32 << 30;  // an allocation that fails releases every pool's free blocks
    // Arena mode (atp_eval_noalloc): allocations are carved in order out of a
    // fixed device region (the library's static workspace); nothing is
    // obtained from or returned to the runtime, releases of arena blocks are
    // ignored (they are not in `live`), and running past the region's end
    // fails with ATP_EBUDGET.
    char *arena = nullptr;
    size_t arena_size = 0, arena_used = 0;
    int64_t n_malloc = 0, n_free = 0;  // runtime allocations and frees (diagnostics)
    double malloc_s = 0, free_s = 0;

    static size_t round(size_t n) {
        if (n < 256) return 256;
        size_t r = 256;
        while (r < n && r < ((size_t)1 << 21)) r <<= 1;
        if (r >= n) return r;
        const size_t mb2 = (size_t)1 << 21;
        return (n + mb2 - 1) / mb2 * mb2;
    }
    void release_cache() {
        std::lock_guard<std::recursive_mutex> g(mu);
        const auto t0 = std::chrono::steady_clock::now();
        for (auto &kv : cache) {
            (void)hipFree(kv.second);
            held -= (int64_t)kv.first;
            n_free += 1;
        }
        cache.clear();
        cached = 0;
        free_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    // every free block, taken out of this pool (held drops with them); for another pool's adopt()
    std::vector<std::pair<size_t, void *>> take_cache() {
        std::lock_guard<std::recursive_mutex> g(mu);
        std::vector<std::pair<size_t, void *>> out(cache.begin(), cache.end());
        for (auto &kv : out) held -= (int64_t)kv.first;
        cache.clear();
        cached = 0;
        return out;
    }
    // a free block of n bytes from another pool of the same device; the caller has ordered
    // every use of it before this pool's stream (no runtime allocation or free either way)
    void adopt(size_t n, void *p) {
        std::lock_guard<std::recursive_mutex> g(mu);
        cache.emplace(n, p);
        cached += n;
        held += (int64_t)n;
    }
    std::function<void()> on_oom;  // frees the cached blocks of every pool of the context
    atp_status alloc(size_t bytes, void **out) {
        if (arena) return alloc_arena(bytes, out);
        atp_status st = alloc_once(bytes, out);
        if (st == ATP_ENOMEM && on_oom) {  // other lanes may hold the memory in their caches
            on_oom();
            st = alloc_once(bytes, out);
        }
        return st;
    }
    atp_status alloc_arena(size_t bytes, void **out) {
        std::lock_guard<std::recursive_mutex> g(mu);
        *out = nullptr;
        const size_t n = ((bytes ? bytes : 1) + 255) / 256 * 256;
        if (n > arena_size - arena_used) return ATP_EBUDGET;
        *out = arena + arena_used;
        arena_used += n;
        return ATP_OK;
    }
    atp_status alloc_once(size_t bytes, void **out) {
        std::lock_guard<std::recursive_mutex> g(mu);
        *out = nullptr;
        if (bytes == 0) bytes = 1;
        size_t n = round(bytes);
        if (user_alloc) {
            if (budget && (uint64_t)(held + n) > budget) return ATP_EBUDGET;
            void *p = user_alloc(n, user);
            if (!p) return ATP_ENOMEM;
            live[p] = n;
            held += (int64_t)n;
            *out = p;
            return ATP_OK;
        }
        // a free block of up to 1.25x the request is reused (2x for blocks of 64 MiB and more: a large
        // runtime allocation costs milliseconds, and large requests vary from query to query)
        auto it = cache.lower_bound(n);
        const size_t slack = n >= ((size_t)64 << 20) ? n : n / 4;
        if (it != cache.end() && it->first <= n + slack) {
            void *p = it->second;
            size_t sz = it->first;
            cache.erase(it);
            cached -= sz;
            live[p] = sz;
            *out = p;
            return ATP_OK;
        }
        if (budget && (uint64_t)(held + n) > budget) {
            release_cache();
            if ((uint64_t)(held + n) > budget) return ATP_EBUDGET;
        }
        void *p = nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            release_cache();
            if (hipMalloc(&p, n) != hipSuccess) {
                (void)hipGetLastError();
                return ATP_ENOMEM;
            }
        }
        n_malloc += 1;
        malloc_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        held += (int64_t)n;
        live[p] = n;
        *out = p;
        return ATP_OK;
    }
    void release(void *p) {
        if (!p) return;
        std::lock_guard<std::recursive_mutex> g(mu);
        auto it = live.find(p);
        if (it == live.end()) return;
        size_t n = it->second;
        live.erase(it);
        if (user_free) {
            user_free(p, user);
            held -= (int64_t)n;
            return;
        }
        cache.emplace(n, p);
        cached += n;
        // keep at most cache_limit bytes of free blocks: drop the largest first
        while (!arena && cached > cache_limit && !cache.empty()) {
            auto last = std::prev(cache.end());
            (void)hipFree(last->second);
            held -= (int64_t)last->first;
            cached -= last->first;
            n_free += 1;
            cache.erase(last);
        }
    }
    void destroy() {
        std::lock_guard<std::recursive_mutex> g(mu);
        release_cache();
        for (auto &kv : live) {
            if (user_free)
                user_free(kv.first, user);
            else
                (void)hipFree(kv.first);
        }
        live.clear();
        held = 0;
    }
};

// RAII device buffer from the pool
struct Buf {
    Pool *pool = nullptr;
    void *p = nullptr;
    size_t bytes = 0;
    Buf() = default;
    Buf(const Buf &) = delete;
    Buf &operator=(const Buf &) = delete;
    Buf(Buf &&o) noexcept : pool(o.pool), p(o.p), bytes(o.bytes) { o.p = nullptr; }
    Buf &operator=(Buf &&o) noexcept {
        reset();
        pool = o.pool;
        p = o.p;
        bytes = o.bytes;
        o.p = nullptr;
        return *this;
    }
    ~Buf() { reset(); }
    void reset() {
        if (p && pool) pool->release(p);
        p = nullptr;
    }
    atp_status alloc(Pool *pl, size_t n) {
        reset();
        pool = pl;
        bytes = n;
        return pl->alloc(n, &p);
    }
    template <typename T>
    T *as() const {
        return (T *)p;
    }
};

#define TRY(x)                               \
    do {                                     \
        atp_status _st = (x);                \
        if (_st != ATP_OK) return _st;       \
    } while (0)
#define HIPTRY(x)                            \
    do {                                     \
        if ((x) != hipSuccess) {             \
            (void)hipGetLastError();         \
            return ATP_EDEVICE;              \
        }                                    \
    } while (0)

struct NodeType {
    std::string name;
    int64_t count;
};

struct Rel {
    int32_t src, dst;
    int64_t nnz;
    Buf rp, col;
    std::vector<int64_t> h_rp;      // host row pointers (planner statistics)
    std::vector<int32_t> h_indeg;   // host column counts
    int64_t nonempty_rows = 0, nonempty_cols = 0;
};

struct Prop {
    int32_t type;
    int32_t dtype;
    std::string name;
    Buf values;
};

Tuning tuning_from_env();

// One execution lane: a stream with its own memory pool, pinned header and
// timers.  The context's main lane runs atp_eval; batch and serving workers
// each own another, so their work overlaps on the device.
// Side streams on which the numeric kernels of different bins run beside
// the lane's stream (fork/join through events).
constexpr int kSideStreams = 3;
struct Lane {
    int id = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Pool pool;
    StepHeader *h_hdr = nullptr;  // pinned; device-writable (mailbox of posted values)
    uint64_t *h_flag = nullptr;   // pinned: sequence number of the last post
    int64_t *d_mailbox = nullptr; // device addresses of h_hdr and h_flag (nullptr: read by copies)
    uint64_t *d_flag = nullptr;
    uint64_t seq = 0;
    double wait_limit_s = 600.0;  // longest wait for posted values before the lane gives up (ATP_EDEVICE)
    KernelTimer timer;
    hipStream_t side[kSideStreams] = {};
    hipEvent_t fork = nullptr, join[kSideStreams] = {};
};
// creates the lane's side streams and events on first use
atp_status lane_sides(Lane *L);
// pinned step header + post flag of a lane
atp_status lane_mailbox(Lane *L);
void lane_free_mailbox(Lane *L);
void lane_release_sides(Lane *L);

// Device-resident cached results and their bookkeeping (Sec. 3.3-3.4).
struct CachePayload {
    Buf rp, col, val, active;
    int64_t rows = 0, cols = 0, nnz = 0, n_active = -1;
    double bytes = 0;
    hipEvent_t ready = nullptr;  // recorded on the producing stream after the data is written
    ~CachePayload() {
        if (ready) (void)hipEventDestroy(ready);
    }
};
using PayloadRef = std::shared_ptr<CachePayload>;  // an evicted payload lives on while a query uses it
struct CacheItemInfo {
    int node = -1;                    // Overlap Tree node, -1 if the string is not in the tree
    std::vector<int32_t> types;       // the sub-metapath
    std::vector<int32_t> rels;
    std::vector<std::string> pos;     // constraint key of every position
};
struct CacheState {
    std::mutex mu;  // every field below; lanes share the cache
    int32_t policy = ATP_CACHE_OFF;
    uint64_t budget = 0;
    std::unique_ptr<OverlapTree> tree;
    std::unique_ptr<CachePolicy> pol;
    std::map<std::string, int64_t> item_by_key;
    std::map<int64_t, CacheItemInfo> info;
    std::map<int64_t, PayloadRef> payload;
    atp_cache_stats stats{};
};

// Admission of per-multiplication slot reservations across lanes: a
// reservation waits while it does not fit next to the ones held (one that
// exceeds the budget alone proceeds when nothing else is held).  Each lane
// holds at most one reservation at a time, so waiting cannot deadlock.
struct MemGate {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t budget = 0;  // 0 = no admission control
    uint64_t used = 0;
    int held = 0;
    bool acquire(uint64_t b) {  // false: no admission control, nothing held
        std::unique_lock<std::mutex> lk(mu);
        if (!budget) return false;
        cv.wait(lk, [&] { return held == 0 || used + b <= budget; });
        used += b;
        ++held;
        return true;
    }
    void release(uint64_t b) {
        std::lock_guard<std::mutex> g(mu);
        used -= b;
        --held;
        cv.notify_all();
    }
};
struct GateHold {
    MemGate *g;
    uint64_t b;
    bool counted;
    GateHold(MemGate *g_, uint64_t b_) : g(g_), b(b_), counted(g_->acquire(b_)) {}
    GateHold(const GateHold &) = delete;
    GateHold &operator=(const GateHold &) = delete;
    ~GateHold() {
        if (counted) g->release(b);
    }
};

// Products of different lanes overlap, except that a heavy product runs
// alone: concurrent work evicts the right operand it re-reads from the
// caches.  Writer-preferring shared/exclusive gate, held for one product.
struct ProductGate {
    std::mutex mu;
    std::condition_variable cv;
    int shared = 0, waiting = 0;
    bool exclusive = false;
    void lock(bool excl) {
        std::unique_lock<std::mutex> lk(mu);
        if (excl) {
            ++waiting;
            cv.wait(lk, [&] { return !exclusive && shared == 0; });
            --waiting;
            exclusive = true;
        } else {
            cv.wait(lk, [&] { return !exclusive && waiting == 0; });
            ++shared;
        }
    }
    void unlock(bool excl) {
        std::lock_guard<std::mutex> lk(mu);
        if (excl)
            exclusive = false;
        else
            --shared;
        cv.notify_all();
    }
};
struct ProductHold {
    ProductGate *g;
    bool excl;
    ProductHold(ProductGate *g_, bool e) : g(g_), excl(e) { g->lock(excl); }
    ProductHold(const ProductHold &) = delete;
    ProductHold &operator=(const ProductHold &) = delete;
    ~ProductHold() { g->unlock(excl); }
};

struct Server;  // serve.cpp

// Identity of constraint id sets (cache keys, mask sharing, popcount memo):
// each distinct canonical id list (sorted, unique) gets a serial number; a
// lookup compares the whole list against the candidates of its hash, so two
// different sets never share a number.  Lists are kept for the context's
// lifetime (the keys that name them live as long).
struct IdSets {
    std::mutex mu;
    std::map<uint64_t, std::vector<std::pair<std::vector<int32_t>, int64_t>>> by_hash;
    int64_t next = 0;
    int64_t serial(std::vector<int32_t> &&ids, uint64_t hash) {
        std::lock_guard<std::mutex> g(mu);
        auto &cands = by_hash[hash];
        for (const auto &c : cands)
            if (c.first == ids) return c.second;
        cands.emplace_back(std::move(ids), next);
        return next++;
    }
};

}  // namespace atp

struct atp_ctx {
    int device = 0;
    uint32_t flags = 0;
    atp::Lane main;  // its pool also holds the network
    std::vector<std::unique_ptr<atp::Lane>> lanes;  // batch / serving lanes (created on demand)
    std::vector<atp::NodeType> types;
    std::vector<std::unique_ptr<atp::Rel>> rels;
    std::vector<std::unique_ptr<atp::Prop>> props;
    std::mutex stat_mu;  // planner statistics below, filled on first use
    std::map<std::pair<int, int>, atp::JunctionSketch> sketches;
    std::map<int, atp::ColumnHist> col_hists;
    std::map<std::string, int64_t> pop_memo;  // mask popcount by (type, position constraint key)
    atp::IdSets idsets;                       // id-set identities used in those keys
    atp::CostCoeffs cost;                     // Eq. 2 coefficients of the planner
    std::vector<std::array<double, 4>> *cost_sink = nullptr;  // (nnz(X), N_op, nnz(Z), ms) per multiplication
    atp::CacheState cache;
    std::mutex results_mu;
    std::set<atp_result *> results;
    std::atomic<bool> broken{false};
    bool step_names = std::getenv("ATP_PROFILE_STEPS") != nullptr;  // diagnostics: kernel names per product
    atp::Tuning tune = atp::tuning_from_env();
    atp::MemGate gate;
    // free blocks the pools in use keep for reuse, in all (half the device's memory, set at
    // creation): the main pool may keep all of it, each of n lanes in use an n-th.  A multi-GB
    // block dropped and obtained again costs milliseconds each way, so a query whose
    // intermediates exceed a small limit would pay that on every run.
    size_t pool_cache_total = (size_t)32 << 30;
    atp::ProductGate products;     // a product above heavy_ops products runs alone across lanes
    // a product above this many products runs alone across lanes (ATP_HEAVY_OPS overrides it)
    int64_t heavy_ops = std::getenv("ATP_HEAVY_OPS") ? std::atoll(std::getenv("ATP_HEAVY_OPS")) : 64ll << 20;
    int64_t tile_index_cap = std::getenv("ATP_TILE_INDEX_CAP") ? std::atoll(std::getenv("ATP_TILE_INDEX_CAP"))
                                                               : (int64_t)256 << 20;  // entries (4 B each)
    // the numeric bins of a product on the lane's side streams (ATP_SERIAL_BINS=1: all on one stream);
    // only while at most one lane is busy (several lanes already keep the GPU busy, and their side
    // streams would outnumber the hardware queues)
    bool concurrent_bins = std::getenv("ATP_SERIAL_BINS") == nullptr;
    std::atomic<int> busy_lanes{0};  // lanes a batch or the server runs at once
    // per-chunk tile counts of the bucket path kept up to this many entries (ATP_CHUNK_HIST_CAP)
    int64_t chunk_hist_cap = std::getenv("ATP_CHUNK_HIST_CAP") ? std::atoll(std::getenv("ATP_CHUNK_HIST_CAP"))
                                                               : atp::kChunkHistCap;
    atp::Server *server = nullptr;  // owned; created and destroyed by serve.cpp
    void *scratch = nullptr;        // this device's copy of the static workspace (atp_eval_noalloc)
    // longest host wait for values a lane's kernels post (ATP_WAIT_LIMIT_S, seconds): a stream that
    // neither finishes nor fails within it is treated as a device error
    double wait_limit_s = std::getenv("ATP_WAIT_LIMIT_S") ? std::atof(std::getenv("ATP_WAIT_LIMIT_S")) : 600.0;
    atp::KernelTimer *kt(atp::Lane *L) { return (flags & ATP_OPT_PROFILE) ? &L->timer : nullptr; }
};

struct atp_result {
    atp_ctx *ctx;
    hipStream_t stream;  // the lane stream that produced it
    int64_t rows, cols, nnz;
    atp::Buf rp, col, val;   // the arrays, unless `shared` holds them
    atp::PayloadRef shared;  // arrays shared with a cached item (a result kept whole, or a whole hit)
    atp_eval_stats stats;
    std::string plan;
    const void *rp_ptr() const { return shared ? shared->rp.p : rp.p; }
    const void *col_ptr() const { return shared ? shared->col.p : col.p; }
    const void *val_ptr() const { return shared ? shared->val.p : val.p; }
};

namespace atp {

// One metapath query (Def. 2-3) as the C-ABI passes it.
struct QueryRef {
    const int32_t *types;
    int32_t n_types;
    const int32_t *rel_ids;
    const atp_constraint *cons;
    int32_t n_cons;
};

// Evaluate one query on lane L.  weight = number of submitted queries this
// evaluation stands for (Overlap Tree frequencies of a fused batch).
atp_status eval_query(atp_ctx *c, Lane *L, const QueryRef &q, const char *plan, int weight, atp_result **out);
atp_status lane_init(atp_ctx *c, Lane *L, int id);
void lane_destroy(Lane *L);
void register_result(atp_ctx *c, atp_result *r);
// workload cache, whole-query items (used by the batch layer): is q's result
// cached; offer a result computed elsewhere (a fused batch member)
bool cache_has_whole(atp_ctx *c, const QueryRef &q);
// (the result's arrays move into the cached item, which the result then shares)
atp_status cache_offer_whole(atp_ctx *c, Lane *L, const QueryRef &q, atp_result &r, double cost_s);
void release_pool_caches(atp_ctx *c);
void server_shutdown(atp_ctx *c);

}  // namespace atp
