// Batches and the serving loop over a workload of metapath queries
// (Problem 2, MQWE): lanes, fusion of queries that differ only in their start
// set, and a request queue with continuous batching.  The arithmetic is that
// of the one-query path; every result is bit-identical to its own atp_eval.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <thread>

#include "engine.hpp"

using namespace atp;

namespace atp {

namespace {

constexpr int kMaxLanes = 16;

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// A query with owned storage (the queue outlives the caller's arrays).
struct OwnedQuery {
    std::vector<int32_t> types, rels;
    bool has_rels = false;
    std::vector<atp_constraint> cons;
    std::vector<std::vector<int32_t>> ids;  // storage of every id-set constraint
    QueryRef ref() const {
        return QueryRef{types.data(), (int32_t)types.size(), has_rels ? rels.data() : nullptr,
                        cons.empty() ? nullptr : cons.data(), (int32_t)cons.size()};
    }
};

OwnedQuery copy_query(const atp_query &q) {
    OwnedQuery o;
    o.types.assign(q.types, q.types + q.n_types);
    if (q.rel_ids) {
        o.has_rels = true;
        o.rels.assign(q.rel_ids, q.rel_ids + (q.n_types - 1));
    }
    o.cons.assign(q.cons, q.cons + q.n_cons);
    o.ids.resize(o.cons.size());
    for (size_t z = 0; z < o.cons.size(); ++z) {
        if (o.cons[z].kind != ATP_C_IDSET) continue;
        o.ids[z].assign(o.cons[z].ids, o.cons[z].ids + o.cons[z].n_ids);
        o.cons[z].ids = o.ids[z].empty() ? nullptr : o.ids[z].data();
    }
    return o;
}

// Shape checks that need no context state (the full validation is eval's).
bool well_formed(const atp_query &q) {
    if (!q.types || q.n_types < 2 || q.n_cons < 0 || (q.n_cons > 0 && !q.cons)) return false;
    for (int32_t z = 0; z < q.n_cons; ++z)
        if (q.cons[z].kind == ATP_C_IDSET && (q.cons[z].n_ids < 0 || (q.cons[z].n_ids > 0 && !q.cons[z].ids)))
            return false;
    return true;
}

// One query as a member of a fusion group.
struct Member {
    QueryRef q;
    int fuse = -1;                 // index of the id-set constraint on position 0 that is unioned, -1 = none
    std::vector<int32_t> start;    // its ids, ascending and unique
    std::string key;               // equal keys fuse
    atp_result *res = nullptr;
    atp_status st = ATP_EINVAL;
    int batch = 1;
};

void append_i64(std::string &k, int64_t v) { k.append((const char *)&v, sizeof(v)); }

// The fusion key: everything but the unioned start set.
void prepare(Member &m) {
    const QueryRef &q = m.q;
    int n_first = 0;
    for (int32_t z = 0; z < q.n_cons; ++z)
        if (q.cons[z].kind == ATP_C_IDSET && q.cons[z].position == 0) {
            ++n_first;
            m.fuse = z;
        }
    if (n_first != 1) m.fuse = -1;  // none, or an intersection of several sets: evaluated alone
    std::string &k = m.key;
    k.clear();
    append_i64(k, q.n_types);
    for (int32_t i = 0; i < q.n_types; ++i) append_i64(k, q.types[i]);
    append_i64(k, q.rel_ids ? 1 : 0);
    if (q.rel_ids)
        for (int32_t i = 0; i + 1 < q.n_types; ++i) append_i64(k, q.rel_ids[i]);
    // constraints in a canonical order (their order does not change the query)
    std::vector<std::string> parts;
    for (int32_t z = 0; z < q.n_cons; ++z) {
        if (z == m.fuse) continue;
        const atp_constraint &c = q.cons[z];
        std::string p;
        append_i64(p, c.position);
        append_i64(p, c.kind);
        if (c.kind == ATP_C_RANGE) {
            append_i64(p, c.prop_id);
            append_i64(p, c.lo);
            append_i64(p, c.hi);
        } else {
            std::vector<int32_t> ids(c.ids, c.ids + c.n_ids);
            std::sort(ids.begin(), ids.end());
            ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
            append_i64(p, (int64_t)ids.size());
            p.append((const char *)ids.data(), ids.size() * sizeof(int32_t));
        }
        parts.push_back(std::move(p));
    }
    std::sort(parts.begin(), parts.end());
    for (auto &p : parts) k += p;
    if (m.fuse < 0) {  // never fuses: make the key unique
        k += "#solo";
        append_i64(k, (int64_t)(intptr_t)&m);
    } else {
        const atp_constraint &c = q.cons[m.fuse];
        m.start.assign(c.ids, c.ids + c.n_ids);
        std::sort(m.start.begin(), m.start.end());
        m.start.erase(std::unique(m.start.begin(), m.start.end()), m.start.end());
    }
}

// Rows `ids` of the fused result R as a result of R's shape.  cnt is a
// zeroed-per-call buffer of R.rows int64.
atp_status gather_member(atp_ctx *c, Lane *L, const atp_result &R, const Buf &d_ids, int64_t n_ids, Buf &cnt,
                         Buf &tmp, int64_t *d_total, atp_result *out) {
    hipStream_t s = L->stream;
    KernelTimer *t = c->kt(L);
    TRY(out->rp.alloc(&L->pool, 8 * (size_t)(R.rows + 1)));
    launch_fill_i64(cnt.as<int64_t>(), R.rows, 0, s, t);
    launch_gather_count((const int64_t *)R.rp_ptr(), d_ids.as<int32_t>(), n_ids, cnt.as<int64_t>(), s, t);
    launch_scan_i64(cnt.as<int64_t>(), out->rp.as<int64_t>(), R.rows, tmp.as<int64_t>(), s, t, d_total);
    return ATP_OK;
}

atp_result *new_result(atp_ctx *c, Lane *L, const atp_result &R) {
    atp_result *r = new atp_result();
    r->ctx = c;
    r->stream = L->stream;
    r->rows = R.rows;
    r->cols = R.cols;
    r->nnz = 0;
    r->stats = R.stats;
    r->plan = R.plan;
    return r;
}

void run_fused(atp_ctx *c, Lane *L, std::vector<Member *> &g);

// Evaluate one fusion group on lane L.  With a cache, members whose whole
// result is cached are answered from it; the others are fused.
void run_group(atp_ctx *c, Lane *L, std::vector<Member *> &g) {
    if (g.size() > 1) {
        std::vector<Member *> rest;
        for (Member *m : g) {
            if (cache_has_whole(c, m->q)) {
                m->batch = 1;
                m->st = eval_query(c, L, m->q, nullptr, 1, &m->res);
            } else {
                rest.push_back(m);
            }
        }
        if (rest.size() != g.size()) {
            if (!rest.empty()) run_fused(c, L, rest);
            return;
        }
    }
    run_fused(c, L, g);
}

void run_fused(atp_ctx *c, Lane *L, std::vector<Member *> &g) {
    for (Member *m : g) m->batch = (int)g.size();
    auto alone = [&]() {
        for (Member *m : g) {
            m->batch = 1;
            m->st = eval_query(c, L, m->q, nullptr, 1, &m->res);
        }
    };
    if (g.size() == 1) {
        alone();
        return;
    }
    const auto t_0 = std::chrono::steady_clock::now();
    // the union of the start sets
    std::vector<int32_t> uni;
    for (Member *m : g) {
        std::vector<int32_t> merged;
        merged.reserve(uni.size() + m->start.size());
        std::set_union(uni.begin(), uni.end(), m->start.begin(), m->start.end(), std::back_inserter(merged));
        uni.swap(merged);
    }
    const Member &m0 = *g[0];
    std::vector<atp_constraint> cons(m0.q.cons, m0.q.cons + m0.q.n_cons);
    cons[m0.fuse].ids = uni.empty() ? nullptr : uni.data();
    cons[m0.fuse].n_ids = (int64_t)uni.size();
    QueryRef qu = m0.q;
    qu.cons = cons.data();
    atp_result *R = nullptr;
    atp_status st = eval_query(c, L, qu, nullptr, (int)g.size(), &R);
    if (st != ATP_OK) {  // e.g. overflow in another member's rows: each query on its own
        alone();
        return;
    }
    hipStream_t s = L->stream;
    KernelTimer *t = c->kt(L);
    auto fail = [&](atp_status e) {
        for (Member *m : g) {
            if (m->res) atp_result_free(m->res);
            m->res = nullptr;
            m->st = e;
        }
        if (e == ATP_EDEVICE) c->broken = true;
    };
    {
        const size_t ng = g.size();
        Buf cnt, tmp, totals;
        std::vector<Buf> ids(ng);
        std::vector<atp_result *> outs(ng, nullptr);
        atp_status e = ATP_OK;
        if ((e = cnt.alloc(&L->pool, 8 * (size_t)std::max<int64_t>(R->rows, 1))) != ATP_OK ||
            (e = tmp.alloc(&L->pool, 8 * (size_t)scan_tmp_elems(R->rows))) != ATP_OK ||
            (e = totals.alloc(&L->pool, 8 * ng)) != ATP_OK) {
            atp_result_free(R);
            alone();
            return;
        }
        for (size_t z = 0; z < ng && e == ATP_OK; ++z) {
            Member &m = *g[z];
            if ((e = ids[z].alloc(&L->pool, 4 * std::max<size_t>(m.start.size(), 1))) != ATP_OK) break;
            if (!m.start.empty() &&
                hipMemcpyAsync(ids[z].p, m.start.data(), 4 * m.start.size(), hipMemcpyHostToDevice, s) != hipSuccess) {
                e = ATP_EDEVICE;
                break;
            }
            outs[z] = new_result(c, L, *R);
            m.res = outs[z];
            e = gather_member(c, L, *R, ids[z], (int64_t)m.start.size(), cnt, tmp, totals.as<int64_t>() + z, outs[z]);
        }
        std::vector<int64_t> h_tot(ng, 0);
        if (e == ATP_OK && (hipMemcpyAsync(h_tot.data(), totals.p, 8 * ng, hipMemcpyDeviceToHost, s) != hipSuccess ||
                            hipStreamSynchronize(s) != hipSuccess))
            e = ATP_EDEVICE;
        for (size_t z = 0; z < ng && e == ATP_OK; ++z) {
            atp_result *o = outs[z];
            o->nnz = h_tot[z];
            o->stats.nnz_result = h_tot[z];
            if ((e = o->col.alloc(&L->pool, 4 * (size_t)std::max<int64_t>(o->nnz, 1))) != ATP_OK ||
                (e = o->val.alloc(&L->pool, 8 * (size_t)std::max<int64_t>(o->nnz, 1))) != ATP_OK)
                break;
            launch_gather_copy((const int64_t *)R->rp_ptr(), (const int32_t *)R->col_ptr(),
                               (const uint64_t *)R->val_ptr(), ids[z].as<int32_t>(),
                               (int64_t)g[z]->start.size(), o->rp.as<int64_t>(), o->col.as<int32_t>(),
                               o->val.as<uint64_t>(), s, t);
        }
        if (e == ATP_OK && hipStreamSynchronize(s) != hipSuccess) e = ATP_EDEVICE;
        if (e != ATP_OK) {
            (void)hipStreamSynchronize(s);
            for (size_t z = 0; z < ng; ++z) delete outs[z];
            for (Member *m : g) m->res = nullptr;
            atp_result_free(R);
            if (e == ATP_EDEVICE) {
                fail(e);
                return;
            }
            alone();
            return;
        }
        for (size_t z = 0; z < ng; ++z) {
            register_result(c, outs[z]);
            g[z]->st = ATP_OK;
        }
        // each member's result is a whole-query cache candidate of its own
        const double share = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_0).count() / ng;
        for (size_t z = 0; z < ng; ++z) (void)cache_offer_whole(c, L, g[z]->q, *outs[z], share);
    }
    if (t) t->flush();
    atp_result_free(R);
}

// Lanes run groups concurrently; a group whose queries ran out of device
// memory next to the others is re-run alone once every other lane is idle.
struct LaneGate {
    std::mutex mu;
    std::condition_variable cv;
    int running = 0;
    bool exclusive = false;
    void enter() {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return !exclusive; });
        ++running;
    }
    void leave() {
        std::lock_guard<std::mutex> lk(mu);
        --running;
        cv.notify_all();
    }
    void enter_exclusive() {  // called without holding a shared entry
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [&] { return !exclusive; });
        exclusive = true;
        cv.wait(lk, [&] { return running == 0; });
    }
    void leave_exclusive() {
        std::lock_guard<std::mutex> lk(mu);
        exclusive = false;
        cv.notify_all();
    }
};

bool out_of_memory(atp_status st) { return st == ATP_ENOMEM || st == ATP_EBUDGET; }

void run_group_gated(atp_ctx *c, Lane *L, std::vector<Member *> &g, LaneGate &gate, int lanes) {
    gate.enter();
    run_group(c, L, g);
    gate.leave();
    if (lanes < 2) return;
    bool again = false;
    for (Member *m : g) again |= out_of_memory(m->st);
    if (!again) return;
    gate.enter_exclusive();
    release_pool_caches(c);
    for (Member *m : g)
        if (out_of_memory(m->st)) {
            m->batch = 1;
            m->st = eval_query(c, L, m->q, nullptr, 1, &m->res);
        }
    gate.leave_exclusive();
}

// Fusion groups of at most max_batch members, in order of first appearance.
std::vector<std::vector<Member *>> make_groups(const std::vector<Member *> &ms, int max_batch) {
    std::vector<std::vector<Member *>> groups;
    std::map<std::string, size_t> open;  // key -> index of the group still filling
    for (Member *m : ms) {
        auto it = open.find(m->key);
        if (it != open.end() && (int)groups[it->second].size() < max_batch) {
            groups[it->second].push_back(m);
            continue;
        }
        open[m->key] = groups.size();
        groups.push_back({m});
    }
    return groups;
}

atp_status ensure_lanes(atp_ctx *c, int n) {
    while ((int)c->lanes.size() < n) {
        auto ln = std::make_unique<Lane>();
        atp_status st = lane_init(c, ln.get(), (int)c->lanes.size() + 1);
        if (st != ATP_OK) {
            lane_destroy(ln.get());
            return st;
        }
        c->lanes.push_back(std::move(ln));
    }
    // the n lanes about to run share the free-block allowance (a pool above its new limit
    // drops blocks on its next release)
    for (int i = 0; i < n; ++i) {
        std::lock_guard<std::recursive_mutex> g(c->lanes[i]->pool.mu);
        c->lanes[i]->pool.cache_limit = c->pool_cache_total / (size_t)n;
    }
    // the main pool's free blocks, idle while lanes run, move to the lanes (largest first, each
    // to the lane holding the fewest free bytes) once the main stream has finished with them:
    // returning them to the runtime and obtaining them again costs milliseconds per large block
    if (!c->main.pool.arena && !c->main.pool.user_alloc && !c->main.pool.cache.empty()) {
        if (hipStreamSynchronize(c->main.stream) != hipSuccess) {
            (void)hipGetLastError();
            return ATP_EDEVICE;
        }
        auto blocks = c->main.pool.take_cache();
        std::sort(blocks.begin(), blocks.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
        for (auto &kv : blocks) {
            Pool *best = &c->lanes[0]->pool;
            for (int i = 1; i < n; ++i)
                if (c->lanes[i]->pool.cached < best->cached) best = &c->lanes[i]->pool;
            best->adopt(kv.first, kv.second);
        }
    }
    return ATP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// serving loop

struct Request {
    uint64_t tag = 0;
    OwnedQuery q;
    Member m;
    double t_submit = 0;
};

struct Server {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::unique_ptr<Request>> queue;
    std::deque<atp_completion> done;
    std::vector<std::thread> workers;
    int running = 0;  // requests taken by workers and not yet completed
    bool stopping = false;
    int max_batch = 1;
    int lanes = 1;
    LaneGate gate;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

namespace {

// Worker `rank` (0 = first lane) takes a request only while more than `rank`
// requests are queued: at low load one lane serves everything (its products'
// bins then run side by side on its side streams, and nothing else competes
// for the device), and further lanes join as a backlog builds up.
void worker(atp_ctx *c, Lane *L, int rank) {
    (void)hipSetDevice(c->device);
    Server &sv = *c->server;
    for (;;) {
        std::vector<std::unique_ptr<Request>> batch;
        {
            std::unique_lock<std::mutex> lk(sv.mu);
            sv.cv_work.wait(lk, [&] { return sv.stopping || (int)sv.queue.size() > rank; });
            if (sv.queue.empty()) return;  // stopping and drained
            batch.push_back(std::move(sv.queue.front()));
            sv.queue.pop_front();
            const std::string &key = batch[0]->m.key;
            for (auto it = sv.queue.begin(); it != sv.queue.end() && (int)batch.size() < sv.max_batch;) {
                if ((*it)->m.key == key) {
                    batch.push_back(std::move(*it));
                    it = sv.queue.erase(it);
                } else {
                    ++it;
                }
            }
            sv.running += (int)batch.size();
        }
        c->busy_lanes += 1;  // lanes running a group now
        const double t_start = now_s(sv.t0);
        std::vector<Member *> g;
        for (auto &r : batch) g.push_back(&r->m);
        run_group_gated(c, L, g, sv.gate, sv.lanes);
        const double t_done = now_s(sv.t0);
        c->busy_lanes -= 1;
        {
            std::lock_guard<std::mutex> lk(sv.mu);
            for (auto &r : batch) {
                atp_completion cp{};
                cp.tag = r->tag;
                cp.status = r->m.st;
                cp.result = r->m.res;
                cp.t_submit = r->t_submit;
                cp.t_start = t_start;
                cp.t_done = t_done;
                cp.batch_size = r->m.batch;
                cp.lane = L->id;
                sv.done.push_back(cp);
            }
            sv.running -= (int)batch.size();
        }
        sv.cv_done.notify_all();
    }
}

}  // namespace

void server_shutdown(atp_ctx *c) {
    if (!c->server) return;
    {
        std::lock_guard<std::mutex> lk(c->server->mu);
        c->server->stopping = true;
    }
    c->server->cv_work.notify_all();
    for (auto &w : c->server->workers) w.join();
    c->busy_lanes.store(0);
    for (auto &cp : c->server->done)
        if (cp.result) atp_result_free(cp.result);
    delete c->server;
    c->server = nullptr;
    std::lock_guard<std::mutex> g(c->gate.mu);
    c->gate.budget = 0;
}

}  // namespace atp

// ---------------------------------------------------------------------------
// C-ABI

extern "C" {

atp_status atp_eval_batch(atp_ctx *c, const atp_query *queries, int32_t n, int32_t lanes, int32_t max_batch,
                          uint64_t mem_budget_bytes, atp_result **out, atp_status *status) {
    if (!c || n < 0 || (n > 0 && (!queries || !out || !status))) return ATP_EINVAL;
    if (lanes < 1 || lanes > kMaxLanes || max_batch < 1) return ATP_EINVAL;
    if (c->server) return ATP_ESTATE;
    if (c->broken) return ATP_EDEVICE;
    (void)hipSetDevice(c->device);
    TRY(ensure_lanes(c, lanes));
    std::vector<Member> ms(n);
    std::vector<Member *> valid;  // members that pass the shape check, in submission order
    for (int32_t i = 0; i < n; ++i) {
        out[i] = nullptr;
        status[i] = ATP_EINVAL;
        if (!well_formed(queries[i])) continue;
        ms[i].q = QueryRef{queries[i].types, queries[i].n_types, queries[i].rel_ids, queries[i].cons,
                           queries[i].n_cons};
        prepare(ms[i]);
        valid.push_back(&ms[i]);
    }
    std::vector<std::vector<Member *>> groups = make_groups(valid, max_batch);
    {
        std::lock_guard<std::mutex> g(c->gate.mu);
        c->gate.budget = mem_budget_bytes;
    }
    std::atomic<size_t> next{0};
    LaneGate gate;
    const int nl = std::min<int>(lanes, (int)std::max<size_t>(groups.size(), 1));
    auto drain = [&](Lane *L) {
        (void)hipSetDevice(c->device);
        for (size_t gi; (gi = next.fetch_add(1)) < groups.size();) run_group_gated(c, L, groups[gi], gate, nl);
    };
    std::vector<std::thread> th;
    c->busy_lanes.store(nl);
    for (int l = 1; l < nl; ++l) th.emplace_back(drain, c->lanes[l].get());
    drain(c->lanes[0].get());
    for (auto &x : th) x.join();
    c->busy_lanes.store(0);
    {
        std::lock_guard<std::mutex> g(c->gate.mu);
        c->gate.budget = 0;
    }
    for (int32_t i = 0; i < n; ++i) {
        out[i] = ms[i].res;
        status[i] = ms[i].st;
    }
    return ATP_OK;
}

atp_status atp_server_start(atp_ctx *c, const atp_server_options *o) {
    if (!c || !o || o->lanes < 1 || o->lanes > kMaxLanes || o->max_batch < 1) return ATP_EINVAL;
    if (c->server) return ATP_ESTATE;
    if (c->broken) return ATP_EDEVICE;
    (void)hipSetDevice(c->device);
    TRY(ensure_lanes(c, o->lanes));
    {
        std::lock_guard<std::mutex> g(c->gate.mu);
        c->gate.budget = o->mem_budget_bytes;
    }
    c->server = new Server();
    c->server->max_batch = o->max_batch;
    c->server->lanes = o->lanes;
    c->busy_lanes.store(0);
    for (int l = 0; l < o->lanes; ++l) c->server->workers.emplace_back(worker, c, c->lanes[l].get(), l);
    return ATP_OK;
}

atp_status atp_submit(atp_ctx *c, const atp_query *q, uint64_t tag) {
    if (!c || !q || !well_formed(*q)) return ATP_EINVAL;
    if (!c->server) return ATP_ESTATE;
    auto r = std::make_unique<Request>();
    r->tag = tag;
    r->q = copy_query(*q);
    r->m.q = r->q.ref();
    prepare(r->m);
    Server &sv = *c->server;
    {
        std::lock_guard<std::mutex> lk(sv.mu);
        r->t_submit = now_s(sv.t0);
        sv.queue.push_back(std::move(r));
    }
    sv.cv_work.notify_all();  // a longer queue may wake a further lane
    return ATP_OK;
}

int32_t atp_poll(atp_ctx *c, atp_completion *out, int32_t max, int32_t wait_ms) {
    if (!c || max < 0 || (max > 0 && !out)) return ATP_EINVAL;
    if (!c->server) return ATP_ESTATE;
    Server &sv = *c->server;
    std::unique_lock<std::mutex> lk(sv.mu);
    if (sv.done.empty() && wait_ms > 0)
        sv.cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !sv.done.empty(); });
    int32_t k = 0;
    while (k < max && !sv.done.empty()) {
        out[k++] = sv.done.front();
        sv.done.pop_front();
    }
    return k;
}

int32_t atp_server_pending(atp_ctx *c) {
    if (!c || !c->server) return 0;
    std::lock_guard<std::mutex> lk(c->server->mu);
    return (int32_t)c->server->queue.size() + c->server->running;
}

atp_status atp_server_stop(atp_ctx *c) {
    if (!c) return ATP_EINVAL;
    if (!c->server) return ATP_ESTATE;
    server_shutdown(c);
    return ATP_OK;
}

}  // extern "C"
