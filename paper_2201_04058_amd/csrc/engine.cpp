// Host side of the engine: the C-ABI of atrapos.h, the HIN registry (Def. 1),
// constraint masks (Def. 3, the diagonal matrices M_c of Sec. 2), the
// planner call (Sec. 3.1-3.2) and the post-order executor of the plan tree.
#include "engine.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>

using namespace atp;

// Device workspace of atp_eval_noalloc: every temporary of such a call is
// carved out of it in order (Pool arena mode).  One copy per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel or
// a copy (on the host it only names the symbol): it uses the per-device
// address looked up once by scratch_address().
static __device__ __align__(256) unsigned char scratch[ATP_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device ordinal -> address of that device's copy

// The current device's copy of `scratch` (the device must be current).
atp_status scratch_address(int device, void **out) {
    std::lock_guard<std::mutex> g(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return ATP_EDEVICE;
        }
        it = g_scratch_ptr.emplace(device, ptr).first;
    }
    *out = it->second;
    return ATP_OK;
}
}  // namespace

namespace atp {

void timer_begin(KernelTimer *t, const char *name, hipStream_t s) {
    if (!t) return;
    t->skip = !t->only.empty() && t->only != name;
    if (t->skip) return;
    KernelTimer::Rec r{std::string(name) + t->suffix, t->take(), t->take()};
    if (r.e0) (void)hipEventRecord(r.e0, s);
    t->pending.push_back(r);
}

void timer_end(KernelTimer *t, hipStream_t s) {
    if (!t || t->pending.empty()) return;
    if (t->skip) {
        t->skip = false;
        return;
    }
    auto &r = t->pending.back();
    if (r.e1) (void)hipEventRecord(r.e1, s);
}
}  // namespace atp

Tuning atp::tuning_from_env() {
    Tuning t;
    auto get = [](const char *name, int64_t &v) {
        if (const char *e = std::getenv(name)) v = std::atoll(e);
    };
    get("ATP_PART_TARGET", t.part_target);
    get("ATP_PART_HASH_CAP", t.part_hash_cap);
    get("ATP_TASK_OPS", t.task_ops);
    get("ATP_BUCKET_PCT", t.bucket_pct);
    get("ATP_SPLIT_OPS", t.split_ops);
    get("ATP_BUCKET_CHUNK", t.bucket_chunk);
    if (t.bucket_chunk < 64) t.bucket_chunk = 64;
    if (t.split_ops < 1024) t.split_ops = 1024;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        t.wg_slots = 2 * (int64_t)cus;
    (void)hipGetLastError();
    if (t.part_hash_cap > kRankCap) t.part_hash_cap = kRankCap;  // rank parts overlay one 8192-column tile
    if (t.part_target < 1) t.part_target = 1;
    if (t.task_ops < 1) t.task_ops = 1;
    return t;
}


// ---------------------------------------------------------------------------

namespace {

atp_status sync(Lane *L) {
    HIPTRY(hipStreamSynchronize(L->stream));
    return ATP_OK;
}

// n int64 values from device memory into the lane's pinned header area: a
// posting kernel writes them and a sequence number into host memory and the
// host polls the number (no stream synchronisation on the way); while the
// stream still runs, it is queried now and then so that a device error ends
// the wait.  Without a device-writable mailbox: a copy and a synchronisation.
atp_status read_values(Lane *L, const int64_t *src, int64_t n) {
    if (!L->d_mailbox) {
        HIPTRY(hipMemcpyAsync(L->h_hdr, src, 8 * (size_t)n, hipMemcpyDeviceToHost, L->stream));
        return sync(L);
    }
    const uint64_t seq = ++L->seq;
    launch_post(src, n, L->d_mailbox, L->d_flag, seq, L->stream);
    HIPTRY(hipGetLastError());
    const auto t0 = std::chrono::steady_clock::now();
    for (uint64_t it = 1;; ++it) {
        if (__atomic_load_n(L->h_flag, __ATOMIC_ACQUIRE) == seq) return ATP_OK;
        if ((it & 63) == 0 &&
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > L->wait_limit_s)
            return ATP_EDEVICE;  // the caller synchronises the stream on its error path
        if ((it & 1023) == 0) {
            const hipError_t e = hipStreamQuery(L->stream);
            if (e == hipSuccess) {  // the post has run: its values are visible after a synchronisation
                HIPTRY(hipStreamSynchronize(L->stream));
                return __atomic_load_n(L->h_flag, __ATOMIC_ACQUIRE) == seq ? ATP_OK : ATP_EDEVICE;
            }
            if (e != hipErrorNotReady) {
                (void)hipGetLastError();
                return ATP_EDEVICE;
            }
        }
        __builtin_ia32_pause();
    }
}

atp_status read_header(Lane *L, const StepHeader *d_hdr) {
    return read_values(L, (const int64_t *)d_hdr, (int64_t)(sizeof(StepHeader) / 8));
}

// A matrix produced by (or feeding) one plan node.
struct Mat {
    bool leaf = false;
    Operand op;
    int64_t rows = 0, cols = 0, nnz = 0;
    Buf rp, col, val;          // owned storage of products
    Buf active;                // ascending non-empty rows (products used as a left operand)
    int64_t n_active = -1;     // -1 = no list
    const int32_t *active_ptr = nullptr;  // the list (owned above, or a cached result's)
    bool view = false;                    // a cached result, not owned
    const int32_t *cand = nullptr;  // leaf: candidate rows from an id-set constraint
    int64_t n_cand = 0;
    // the product's step header (kept for the value bound at hdr->vmax).  A
    // product whose size was not read back: nnz is an upper bound (the
    // arrays' capacity), the true count is at nnz_dev in the kept header, and
    // the active list holds every candidate row, non-empty ones first
    Buf hdr;
    const int64_t *nnz_dev = nullptr;
    // some count reached 2^63 (known when the size was read back; a deferred
    // product is never cached, so it never needs the flag)
    bool saturated = false;
};

struct PosMask {
    Buf bits;
    int64_t pop = -1;       // -1 = no constraint at this position
    Buf ids;                // sorted unique ids of an id-set constraint (smallest set)
    int64_t n_ids = -1;
    std::vector<int32_t> h_ids;
    std::vector<std::vector<int32_t>> staged;  // host sources of asynchronous copies
    std::vector<Buf> spent;                    // device id lists of the other id sets
    const PosMask *alias = nullptr;            // the same constraints at an earlier position of the query
    const uint32_t *bits_ptr() const { return alias ? alias->bits.as<uint32_t>() : bits.as<uint32_t>(); }
    const int32_t *ids_ptr() const { return alias ? alias->ids.as<int32_t>() : ids.as<int32_t>(); }
};

struct StepStats {
    int64_t n_op = 0, nnz = 0, slots = 0;
};


// Counting mode: algorithmic bytes of the numeric launches of one product,
// by kernel name (operands read once, results written once).
atp_status count_bytes(atp_ctx *c, Lane *L, const Mat &X, const Mat &Y, const int32_t *cand, const int32_t *bin_lists,
                       int64_t n_cand, const StepHeader &h1, const int64_t *row_nnz) {
    struct Group {
        const char *name;
        int b0, b1;
    } groups[] = {{"hash_wave", BIN_W64, BIN_W512}, {"hash_block", BIN_B1024, BIN_B8192}, {"dense", BIN_DENSE, BIN_DENSE},
                  {"bucket", BIN_BUCKET, BIN_BUCKET}};
    hipStream_t s = L->stream;
    const double vx = X.op.val ? 8.0 : 0.0, vy = Y.op.val ? 8.0 : 0.0;
    for (const Group &g : groups) {
        int64_t rows_in_group = 0;
        for (int b = g.b0; b <= g.b1; ++b) rows_in_group += h1.bin_count[b];
        if (!rows_in_group) continue;
        Buf ymark, acc;
        const int64_t words = (Y.rows + 31) / 32;
        TRY(ymark.alloc(&L->pool, 4 * (size_t)std::max<int64_t>(words, 1)));
        TRY(acc.alloc(&L->pool, 8 * 5));
        launch_fill_u32(ymark.as<uint32_t>(), words, 0u, s, nullptr);
        launch_fill_i64(acc.as<int64_t>(), 5, 0, s, nullptr);
        for (int b = g.b0; b <= g.b1; ++b)
            launch_bin_stats(bin_lists + (int64_t)b * n_cand, h1.bin_count[b], X.op, cand, row_nnz,
                             ymark.as<uint32_t>(), acc.as<int64_t>(), s);
        launch_mark_bytes(ymark.as<uint32_t>(), Y.op.rp, Y.rows, acc.as<int64_t>(), s);
        int64_t h[5];
        HIPTRY(hipMemcpyAsync(h, acc.p, sizeof(h), hipMemcpyDeviceToHost, s));
        TRY(sync(L));
        L->timer.bytes[g.name] += 16.0 * h[0] + (4.0 + vx) * h[1] + 12.0 * h[2] + 16.0 * h[3] + (4.0 + vy) * h[4];
    }
    return ATP_OK;
}

// Z = X * Y, one product of the plan (Sec. 3.2).  ycols_eff bounds the
// columns that can occur (mask popcount of Y's last position, or Y's width).
// need_active: Z will be the left operand of a later product.
// defer: Z is an intermediate (not the result, no cache): its sizes are not
// read back (no host synchronisation after the numeric phase); its true
// nonzero count is added to *nnz_acc on the device.  defer_below > 0: defer
// too when the symbolic bound on Z's nonzeros is below it (a caller that
// compares Z's size with that limit gets the same answer from the bound).
atp_status spgemm(atp_ctx *c, Lane *L, const Mat &X, const Mat &Y, int64_t ycols_eff, bool need_active, Mat &Z,
                  StepStats &st, bool &saturated, bool defer, int64_t *nnz_acc, int64_t defer_below = 0,
                  bool operand = true) {
    Pool *pool = &L->pool;
    hipStream_t s = L->stream;
    KernelTimer *t = c->kt(L);
    Z.leaf = false;
    Z.rows = X.rows;
    Z.cols = Y.cols;
    saturated = false;

    const int32_t *cand = nullptr;
    int64_t n_cand = X.rows;
    if (X.leaf && X.cand) {
        cand = X.cand;
        n_cand = X.n_cand;
    } else if (!X.leaf && X.n_active >= 0 && X.active_ptr) {
        cand = X.active_ptr;
        n_cand = X.n_active;
    }
    TRY(Z.rp.alloc(pool, sizeof(int64_t) * (Z.rows + 1)));
    auto finish_empty = [&]() -> atp_status {
        launch_fill_i64(Z.rp.as<int64_t>(), Z.rows + 1, 0, s, t);
        Z.nnz = 0;
        TRY(Z.col.alloc(pool, 4));
        TRY(Z.val.alloc(pool, 8));
        if (need_active) {
            TRY(Z.active.alloc(pool, 4));
            Z.n_active = 0;
            Z.active_ptr = Z.active.as<int32_t>();
        }
        Z.op = Operand{Z.rp.as<int64_t>(), Z.col.as<int32_t>(), Z.val.as<uint64_t>(), nullptr, nullptr,
                       Z.rows, Z.cols, 0};
        return ATP_OK;
    };
    if (n_cand == 0 || ycols_eff == 0) return finish_empty();

    Buf hdr, nop, ub, nseg, bin, long_len, long_off, bin_lists, dense_chunks, slot_off, seg_base, task_base, tmp;
    Buf bucket_chunks, bucket_nop, chunk_base, prod_base, dense_split;
    TRY(hdr.alloc(pool, sizeof(StepHeader)));
    TRY(nop.alloc(pool, 8 * n_cand));
    TRY(ub.alloc(pool, 8 * n_cand));
    TRY(nseg.alloc(pool, 8 * n_cand));
    TRY(bin.alloc(pool, 4 * n_cand));
    TRY(long_len.alloc(pool, 8 * n_cand));
    TRY(long_off.alloc(pool, 8 * (n_cand + 1)));
    TRY(bin_lists.alloc(pool, 4 * (size_t)n_cand * BIN_COUNT));
    TRY(dense_chunks.alloc(pool, 8 * n_cand));
    TRY(slot_off.alloc(pool, 8 * (n_cand + 1)));
    TRY(seg_base.alloc(pool, 8 * (n_cand + 1)));
    TRY(task_base.alloc(pool, 8 * (n_cand + 1)));
    TRY(bucket_chunks.alloc(pool, 8 * n_cand));
    TRY(dense_split.alloc(pool, 8 * n_cand));
    TRY(bucket_nop.alloc(pool, 8 * n_cand));
    TRY(chunk_base.alloc(pool, 8 * (n_cand + 1)));
    TRY(prod_base.alloc(pool, 8 * (n_cand + 1)));
    const int64_t tmp_n = 5 * scan_tmp_elems(n_cand);
    TRY(tmp.alloc(pool, 8 * tmp_n));

    StepHeader *d_hdr = hdr.as<StepHeader>();
    launch_fill_i64((int64_t *)d_hdr, sizeof(StepHeader) / 8, 0, s, t);
    // a product that feeds another one records its largest value (the dense tiles' bound)
    uint64_t *vmax = operand ? &d_hdr->vmax : nullptr;

    SymbolicArgs sa;
    sa.X = X.op;
    sa.Y = Y.op;
    sa.cand = cand;
    sa.n_cand = n_cand;
    sa.ycols_eff = ycols_eff;
    sa.nop = nop.as<int64_t>();
    sa.ub = ub.as<int64_t>();
    sa.nseg = nseg.as<int64_t>();
    sa.bin = bin.as<int32_t>();
    sa.long_len = long_len.as<int64_t>();
    sa.long_off = long_off.as<int64_t>();
    sa.scan_tmp = tmp.as<int64_t>();
    sa.bin_lists = bin_lists.as<int32_t>();
    sa.dense_chunks = dense_chunks.as<int64_t>();
    sa.bucket_chunks = bucket_chunks.as<int64_t>();
    sa.dense_split = dense_split.as<int64_t>();
    sa.bucket_nop = bucket_nop.as<int64_t>();
    sa.hdr = d_hdr;
    sa.tune = c->tune;
    launch_symbolic(sa, s, t);
    launch_bin_rows(sa, s, t);
    const ScanJob jobs[5] = {{ub.as<int64_t>(), slot_off.as<int64_t>(), &d_hdr->slots_total, n_cand},
                             {nseg.as<int64_t>(), seg_base.as<int64_t>(), &d_hdr->segs_total, n_cand},
                             {dense_chunks.as<int64_t>(), task_base.as<int64_t>(), &d_hdr->dense_tasks, n_cand},
                             {bucket_chunks.as<int64_t>(), chunk_base.as<int64_t>(), &d_hdr->bucket_chunks, n_cand},
                             {bucket_nop.as<int64_t>(), prod_base.as<int64_t>(), &d_hdr->bucket_products, n_cand}};
    launch_scan_multi(jobs, 5, tmp.as<int64_t>(), s, t);
    TRY(read_header(L, d_hdr));
    const StepHeader h1 = *L->h_hdr;
    st.n_op += h1.n_op_total;
    st.slots += h1.slots_total;
    if (h1.slots_total == 0) return finish_empty();

    // the numeric phase of a heavy product runs alone across lanes
    ProductHold alone(&c->products, h1.n_op_total > c->heavy_ops);
    // admission: reserve the slot arrays (and the split accumulators) against the lanes' budget
    const int64_t ntiles_y = (Y.cols + kTileW - 1) / kTileW;
    GateHold hold(&c->gate, 12ull * (uint64_t)h1.slots_total +
                                (uint64_t)h1.n_split * (uint64_t)ntiles_y * (uint64_t)kTileW * 9ull);
    Buf slot_col, slot_val, seg_cnt, seg_src, seg_dst, row_cursor, row_nnz, dqueue;
    TRY(slot_col.alloc(pool, 4 * (size_t)h1.slots_total));
    TRY(slot_val.alloc(pool, 8 * (size_t)h1.slots_total));
    TRY(seg_cnt.alloc(pool, 8 * (size_t)h1.segs_total));
    TRY(seg_src.alloc(pool, 8 * (size_t)h1.segs_total));
    TRY(seg_dst.alloc(pool, 8 * ((size_t)h1.segs_total + 1)));
    TRY(row_cursor.alloc(pool, 8 * n_cand));
    TRY(row_nnz.alloc(pool, 8 * (size_t)Z.rows));
    TRY(dqueue.alloc(pool, 8 * kQueues));
    const FillJob zero[4] = {{seg_cnt.as<int64_t>(), h1.segs_total, 0}, {row_cursor.as<int64_t>(), n_cand, 0},
                             {row_nnz.as<int64_t>(), Z.rows, 0}, {dqueue.as<int64_t>(), kQueues, 0}};
    launch_fill_multi(zero, 4, s, t);

    NumericArgs na{};
    na.X = X.op;
    na.Y = Y.op;
    na.cand = cand;
    na.nop = nop.as<int64_t>();
    na.slot_off = slot_off.as<int64_t>();
    na.seg_base = seg_base.as<int64_t>();
    na.row_cursor = row_cursor.as<int64_t>();
    na.slot_col = slot_col.as<int32_t>();
    na.slot_val = slot_val.as<uint64_t>();
    na.seg_cnt = seg_cnt.as<int64_t>();
    na.seg_src = seg_src.as<int64_t>();
    na.row_nnz = row_nnz.as<int64_t>();
    na.hdr = d_hdr;
    na.ycols = Y.cols;
    na.tune = c->tune;
    na.dense_split = dense_split.as<int64_t>();
    na.dense_queue = dqueue.as<int64_t>();
    Buf split_acc, split_sat, split_done;
    if (h1.n_split > 0) {
        const int64_t ntiles = (Y.cols + kTileW - 1) / kTileW;
        const int64_t nt = h1.n_split * ntiles;
        TRY(split_acc.alloc(pool, 8 * (size_t)nt * kTileW));
        TRY(split_sat.alloc(pool, 4 * (size_t)nt * (kTileW / 32)));
        TRY(split_done.alloc(pool, 4 * (size_t)nt));
        launch_fill_i64(split_acc.as<int64_t>(), nt * kTileW, 0, s, t);
        launch_fill_u32(split_sat.as<uint32_t>(), nt * (kTileW / 32), 0u, s, t);
        launch_fill_u32((uint32_t *)split_done.as<int32_t>(), nt, 0u, s, t);
        na.split_acc = split_acc.as<unsigned long long>();
        na.split_sat = split_sat.as<uint32_t>();
        na.split_done = split_done.as<int32_t>();
    }
    Buf ytile;
    na.ytile = nullptr;
    const int64_t ntiles_z = (Y.cols + kTileW - 1) / kTileW;
    if (h1.bin_count[BIN_DENSE] > 0) {
        // segment bounds from a per-row tile index instead of searches, when it is small enough
        const int64_t entries = (Y.rows) * (ntiles_z + 1);
        if (ntiles_z > 1 && entries <= c->tile_index_cap && Y.nnz < ((int64_t)1 << 31)) {
            TRY(ytile.alloc(pool, 4 * (size_t)entries));
            na.ytile = ytile.as<int32_t>();
        }
    }
    Buf tile_cnt, tile_off, prod_col, prod_val, chunk_hist, parts;
    const int64_t nb = h1.bin_count[BIN_BUCKET];
    const bool valued = X.op.val || Y.op.val;
    if (nb > 0) {
        TRY(parts.alloc(pool, 8 * (size_t)bucket_parts_elems(nb)));
        if (h1.bucket_chunks * ntiles_z <= c->chunk_hist_cap)
            TRY(chunk_hist.alloc(pool, 8 * (size_t)std::max<int64_t>(h1.bucket_chunks * ntiles_z, 1)));
        TRY(tile_cnt.alloc(pool, 8 * (size_t)nb * (ntiles_z + 1)));
        TRY(tile_off.alloc(pool, 8 * (size_t)nb * (ntiles_z + 1)));
        TRY(prod_col.alloc(pool, 4 * (size_t)std::max<int64_t>(h1.bucket_products, 1)));
        if (valued) TRY(prod_val.alloc(pool, 8 * (size_t)std::max<int64_t>(h1.bucket_products, 1)));
    }
    // The bins are independent (disjoint rows and slots): wavefront-hash rows,
    // workgroup-hash rows and bucketed rows go to the lane's side streams and
    // run beside the dense rows on the lane's stream.
    bool any_wave = false, any_block = false;
    for (int b = BIN_W64; b <= BIN_W512; ++b) any_wave |= h1.bin_count[b] > 0;
    for (int b = BIN_B1024; b <= BIN_B8192; ++b) any_block |= h1.bin_count[b] > 0;
    const int groups = (int)any_wave + (int)any_block + (int)(nb > 0) + (int)(h1.bin_count[BIN_DENSE] > 0);
    hipStream_t s_wave = s, s_block = s, s_bucket = s;
    struct Join {
        Lane *L = nullptr;
        hipStream_t s = nullptr;
        int n = 0;  // side streams forked
        atp_status run() {
            atp_status st = ATP_OK;
            for (int i = 0; i < n; ++i)
                if (hipEventRecord(L->join[i], L->side[i]) != hipSuccess || hipStreamWaitEvent(s, L->join[i], 0) != hipSuccess)
                    st = ATP_EDEVICE;
            n = 0;
            return st;
        }
        ~Join() { (void)run(); }
    } join;
    if (groups >= 2 && c->concurrent_bins && !(c->flags & ATP_OPT_SERIAL_BINS) && c->busy_lanes.load() <= 1) {
        // the dense rows (else the first other group) keep the lane's stream; each
        // further non-empty group takes a side stream forked from it
        TRY(lane_sides(L));
        bool main_taken = h1.bin_count[BIN_DENSE] > 0;
        int used = 0;
        auto take = [&](bool present) -> hipStream_t {
            if (!present) return s;
            if (!main_taken) {
                main_taken = true;
                return s;
            }
            return L->side[used++];
        };
        s_wave = take(any_wave);
        s_block = take(any_block);
        s_bucket = take(nb > 0);
        HIPTRY(hipEventRecord(L->fork, s));
        for (int i = 0; i < used; ++i) HIPTRY(hipStreamWaitEvent(L->side[i], L->fork, 0));
        join.L = L;
        join.s = s;
        join.n = used;
    }
    // the largest hash bins first: their rows take longest, and they get CUs before the
    // dense kernel's persistent workgroups fill the LDS
    for (int b = BIN_B8192; b >= BIN_W64; --b)
        launch_numeric_hash(b, bin_lists.as<int32_t>() + (int64_t)b * n_cand, h1.bin_count[b], na,
                            b <= BIN_W512 ? s_wave : s_block, t);
    if (nb > 0) {
        launch_fill_i64(tile_cnt.as<int64_t>(), nb * (ntiles_z + 1), 0, s_bucket, t);
        launch_numeric_bucket(bin_lists.as<int32_t>() + (int64_t)BIN_BUCKET * n_cand, nb, chunk_base.as<int64_t>(),
                              h1.bucket_chunks, prod_base.as<int64_t>(), ntiles_z, tile_cnt.as<int64_t>(),
                              tile_off.as<int64_t>(), prod_col.as<int32_t>(),
                              valued ? prod_val.as<uint64_t>() : nullptr, chunk_hist.as<int64_t>(),
                              parts.as<int64_t>(), na, s_bucket, t);
    }
    if (na.ytile) launch_tile_index(Y.op, ntiles_z, ytile.as<int32_t>(), s, t);
    if (h1.bin_count[BIN_DENSE] > 0)
        launch_numeric_dense(bin_lists.as<int32_t>() + (int64_t)BIN_DENSE * n_cand, h1.bin_count[BIN_DENSE],
                             task_base.as<int64_t>(), h1.dense_tasks, na, s, t);
    TRY(join.run());

    if (c->flags & ATP_OPT_COUNT_BYTES) TRY(count_bytes(c, L, X, Y, cand, bin_lists.as<int32_t>(), n_cand, h1,
                                                       row_nnz.as<int64_t>()));

    // row pointers over every row of X, segment destinations in (row, tile)
    // order and (for a left operand) the non-empty rows: one scan sequence
    Buf flags, flags_scan;
    ScanJob jobs2[3] = {{row_nnz.as<int64_t>(), Z.rp.as<int64_t>(), &d_hdr->nnz_total, Z.rows},
                        {seg_cnt.as<int64_t>(), seg_dst.as<int64_t>(), nullptr, h1.segs_total},
                        {nullptr, nullptr, nullptr, 0}};
    int n_jobs2 = 2;
    if (need_active) {
        TRY(flags.alloc(pool, 8 * n_cand));
        TRY(flags_scan.alloc(pool, 8 * (n_cand + 1)));
        launch_active_flags(cand, n_cand, row_nnz.as<int64_t>(), flags.as<int64_t>(), s, t);
        jobs2[n_jobs2++] = ScanJob{flags.as<int64_t>(), flags_scan.as<int64_t>(), &d_hdr->n_active, n_cand};
    }
    Buf tmp2;
    TRY(tmp2.alloc(pool, 8 * (size_t)scan_multi_tmp_elems(jobs2, n_jobs2)));
    launch_scan_multi(jobs2, n_jobs2, tmp2.as<int64_t>(), s, t);
    if (defer_below > 0 && h1.slots_total < defer_below && nnz_acc) defer = true;
    if (defer) {
        // capacities from the symbolic bounds; the counts stay on the device
        Z.nnz = h1.slots_total;
        TRY(Z.col.alloc(pool, 4 * (size_t)std::max<int64_t>(Z.nnz, 1)));
        TRY(Z.val.alloc(pool, 8 * (size_t)std::max<int64_t>(Z.nnz, 1)));
        launch_copy_segments(seg_cnt.as<int64_t>(), seg_src.as<int64_t>(), seg_dst.as<int64_t>(), h1.segs_total,
                             slot_col.as<int32_t>(), slot_val.as<uint64_t>(), Z.col.as<int32_t>(),
                             Z.val.as<uint64_t>(), vmax, s, t);
        if (need_active) {
            Z.n_active = n_cand;
            TRY(Z.active.alloc(pool, 4 * (size_t)std::max<int64_t>(n_cand, 1)));
            Z.active_ptr = Z.active.as<int32_t>();
            launch_active_scatter(cand, n_cand, flags_scan.as<int64_t>(), Z.active.as<int32_t>(), true, s, t);
        }
        if (nnz_acc) launch_accum_step(d_hdr, nnz_acc, s);
        Z.nnz_dev = &d_hdr->nnz_total;
        Z.hdr = std::move(hdr);
    } else {
        TRY(read_header(L, d_hdr));
        const StepHeader h2 = *L->h_hdr;
        if (h2.fault) {  // an LDS hash table ran out of probes: the product is invalid
            c->broken = true;
            return ATP_EDEVICE;
        }
        saturated = h2.saturated != 0;
        Z.saturated = saturated;
        Z.nnz = h2.nnz_total;
        st.nnz += Z.nnz;
        TRY(Z.col.alloc(pool, 4 * (size_t)std::max<int64_t>(Z.nnz, 1)));
        TRY(Z.val.alloc(pool, 8 * (size_t)std::max<int64_t>(Z.nnz, 1)));
        launch_copy_segments(seg_cnt.as<int64_t>(), seg_src.as<int64_t>(), seg_dst.as<int64_t>(), h1.segs_total,
                             slot_col.as<int32_t>(), slot_val.as<uint64_t>(), Z.col.as<int32_t>(),
                             Z.val.as<uint64_t>(), vmax, s, t);
        if (need_active) {
            Z.n_active = h2.n_active;
            TRY(Z.active.alloc(pool, 4 * (size_t)std::max<int64_t>(Z.n_active, 1)));
            Z.active_ptr = Z.active.as<int32_t>();
            launch_active_scatter(cand, n_cand, flags_scan.as<int64_t>(), Z.active.as<int32_t>(), false, s, t);
        }
        Z.hdr = std::move(hdr);  // holds the value bound
    }
    Z.op = Operand{Z.rp.as<int64_t>(), Z.col.as<int32_t>(), Z.val.as<uint64_t>(), nullptr, nullptr,
                   Z.rows, Z.cols, Z.nnz};
    Z.op.vmax = vmax;
    if (c->flags & ATP_OPT_COUNT_BYTES) L->timer.bytes["copy"] += 24.0 * (double)Z.nnz + 24.0 * (double)h1.segs_total;
    // temporaries go back to the pool here; later work on the stream is ordered after this step
    return ATP_OK;
}

// Build the mask of one metapath position from its constraints (ANDed).
atp_status build_mask(atp_ctx *c, Lane *L, int pos_type, const atp_constraint *cons, int n_cons, int pos, PosMask &m) {
    Pool *pool = &L->pool;
    hipStream_t s = L->stream;
    KernelTimer *t = c->kt(L);
    const int64_t n = c->types[pos_type].count;
    const int64_t words = (n + 31) / 32;
    bool first = true;
    for (int q = 0; q < n_cons; ++q) {
        const atp_constraint &k = cons[q];
        if (k.position != pos) continue;
        if (first) {
            TRY(m.bits.alloc(pool, 4 * (size_t)std::max<int64_t>(words, 1)));
        }
        if (k.kind == ATP_C_RANGE) {
            const Prop &p = *c->props[k.prop_id];
            launch_mask_range(p.values.p, p.dtype, n, k.lo, k.hi, m.bits.as<uint32_t>(), first ? 0 : 1, s, t);
        } else {
            std::vector<int32_t> ids(k.ids, k.ids + k.n_ids);
            std::sort(ids.begin(), ids.end());
            ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
            Buf d_ids;
            TRY(d_ids.alloc(pool, 4 * std::max<size_t>(ids.size(), 1)));
            if (!ids.empty())  // the host copy lives in m.staged until the query ends
                HIPTRY(hipMemcpyAsync(d_ids.p, ids.data(), 4 * ids.size(), hipMemcpyHostToDevice, s));
            if (first) {
                launch_fill_u32(m.bits.as<uint32_t>(), words, 0u, s, t);
                launch_mask_ids(d_ids.as<int32_t>(), (int64_t)ids.size(), m.bits.as<uint32_t>(), s, t);
            } else {
                Buf tmpb;
                TRY(tmpb.alloc(pool, 4 * (size_t)std::max<int64_t>(words, 1)));
                launch_fill_u32(tmpb.as<uint32_t>(), words, 0u, s, t);
                launch_mask_ids(d_ids.as<int32_t>(), (int64_t)ids.size(), tmpb.as<uint32_t>(), s, t);
                launch_mask_and(m.bits.as<uint32_t>(), tmpb.as<uint32_t>(), words, s, t);
                // tmpb returns to this lane's pool; its reuse is ordered after these launches
            }
            if (m.n_ids < 0 || (int64_t)ids.size() < m.n_ids) {
                m.n_ids = (int64_t)ids.size();
                m.h_ids = ids;
                m.ids = std::move(d_ids);
            } else {
                m.spent.push_back(std::move(d_ids));  // the mask kernel may still read it
            }
            m.staged.push_back(std::move(ids));
        }
        first = false;
    }
    if (!first) m.pop = 0;  // popcount filled in by the caller
    return ATP_OK;
}

double est_rows_with_ids(const Rel &r, const std::vector<int32_t> &ids, double *nnz) {
    double rows = 0, z = 0;
    for (int32_t u : ids) {
        int64_t d = r.h_rp[u + 1] - r.h_rp[u];
        if (d > 0) {
            rows += 1;
            z += (double)d;
        }
    }
    *nnz = z;
    return rows;
}

const JunctionSketch &sketch_for(atp_ctx *c, int rin, int rout) {
    std::lock_guard<std::mutex> g(c->stat_mu);  // map nodes are stable: the reference outlives the lock
    auto key = std::make_pair(rin, rout);
    auto it = c->sketches.find(key);
    if (it != c->sketches.end()) return it->second;
    const Rel &a = *c->rels[rin];
    const Rel &b = *c->rels[rout];
    JunctionSketch js = make_sketch(a.h_indeg.data(), b.h_rp.data(), (int64_t)b.h_rp.size() - 1);
    return c->sketches.emplace(key, std::move(js)).first->second;
}

// ---- cache keys (Sec. 3.3, "Handling constrained queries") ----------------

uint64_t fnv1a64(const void *data, size_t n, uint64_t h = 1469598103934665603ull) {
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// canonical constraint string of every metapath position; an id set is
// named by its size and its context-wide serial number (exact identity)
std::vector<std::string> position_keys(atp_ctx *c, int32_t n_types, const atp_constraint *cons, int32_t n_cons) {
    std::vector<std::vector<std::string>> per(n_types);
    for (int q = 0; q < n_cons; ++q) {
        const atp_constraint &k = cons[q];
        char buf[96];
        if (k.kind == ATP_C_RANGE) {
            std::snprintf(buf, sizeof(buf), "R%d:%lld:%lld", k.prop_id, (long long)k.lo, (long long)k.hi);
        } else {
            std::vector<int32_t> ids(k.ids, k.ids + k.n_ids);
            std::sort(ids.begin(), ids.end());
            ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
            const size_t n = ids.size();
            const uint64_t h = fnv1a64(ids.data(), n * sizeof(int32_t));
            std::snprintf(buf, sizeof(buf), "I%zu:#%lld", n, (long long)c->idsets.serial(std::move(ids), h));
        }
        per[k.position].push_back(buf);
    }
    std::vector<std::string> out(n_types);
    for (int i = 0; i < n_types; ++i) {
        std::sort(per[i].begin(), per[i].end());
        for (auto &x : per[i]) out[i] += (out[i].empty() ? "" : "&") + x;
    }
    return out;
}

std::string item_key(const std::vector<int32_t> &types, const std::vector<int32_t> &rels,
                     const std::vector<std::string> &pos) {
    std::string k = "t";
    for (int32_t t : types) k += ":" + std::to_string(t);
    k += "|r";
    for (int32_t r : rels) k += ":" + std::to_string(r);
    k += "|c";
    for (auto &x : pos) k += ";" + x;
    return k;
}

// cached items whose sub-metapath extends item q's to the right with the same
// relations and constraints on q's positions (q's Overlap-Tree subtree)
std::vector<int64_t> cache_subtree(const CacheState &cs, int64_t q) {
    std::vector<int64_t> out;
    auto iq = cs.info.find(q);
    if (iq == cs.info.end() || !cs.tree) return out;
    const CacheItemInfo &qi = iq->second;
    const int node = cs.tree->find(qi.types);
    if (node < 0) return out;
    cs.tree->for_subtree(node, [&](int u) {
        for (const auto &kv : cs.tree->node(u).keys) {
            const int64_t e = kv.second.item;
            if (e < 0 || e == q || !cs.payload.count(e)) continue;
            const CacheItemInfo &ei = cs.info.at(e);
            bool ok = ei.types.size() > qi.types.size();
            for (size_t z = 0; ok && z < qi.rels.size(); ++z) ok = ei.rels[z] == qi.rels[z];
            for (size_t z = 0; ok && z < qi.pos.size(); ++z) ok = ei.pos[z] == qi.pos[z];
            if (ok) out.push_back(e);
        }
    });
    return out;
}

// A product computed by the current query: leaves lo..hi, cumulative cost (s).
struct KeptMat {
    int lo, hi;
    double cost;
    bool partial;  // computed on a subset of its rows (row restriction): not a cacheable result
    Mat m;
};

// The relation of every step of a metapath (Def. 2): the given ids, checked
// against the types, or the unique relation between each pair of types.
atp_status resolve_rels(const atp_ctx *c, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                        std::vector<int> &rel) {
    const int ntypes_reg = (int)c->types.size();
    for (int i = 0; i < n_types; ++i)
        if (types[i] < 0 || types[i] >= ntypes_reg) return ATP_EINVAL;
    const int p = n_types - 1;
    rel.assign(p, -1);
    for (int i = 0; i < p; ++i) {
        if (rel_ids) {
            int r = rel_ids[i];
            if (r < 0 || r >= (int)c->rels.size()) return ATP_EINVAL;
            if (c->rels[r]->src != types[i] || c->rels[r]->dst != types[i + 1]) return ATP_ESCHEMA;
            rel[i] = r;
        } else {
            int found = -1, nfound = 0;
            for (int r = 0; r < (int)c->rels.size(); ++r)
                if (c->rels[r]->src == types[i] && c->rels[r]->dst == types[i + 1]) {
                    found = r;
                    ++nfound;
                }
            if (nfound != 1) return ATP_ESCHEMA;
            rel[i] = found;
        }
    }
    return ATP_OK;
}

// Bookkeeping of one insertion attempt (Sec. 3.4.1): find or create the item
// of `key`, count the attempt and let the policy admit it, evicting as it
// decides.  Returns the item id to store, or -1 (already cached / refused).
// The caller holds cs.mu.
int64_t admit_item(CacheState &cs, const std::string &key, const std::vector<int32_t> &ty,
                   const std::vector<int32_t> &rl, const std::vector<std::string> &ps, double bytes, double cost) {
    int64_t id;
    auto it = cs.item_by_key.find(key);
    if (it != cs.item_by_key.end()) {
        id = it->second;
        if (cs.payload.count(id)) return -1;  // already cached
    } else {
        id = cs.pol->add_item(bytes, std::max(cost, 1e-9));
        const int node = cs.tree->find(ty);
        cs.info[id] = CacheItemInfo{node, ty, rl, ps};
        cs.item_by_key[key] = id;
        if (node >= 0) cs.tree->node(node).keys[key].item = id;
    }
    cs.stats.insert_attempts += 1;
    std::vector<int64_t> ev;
    const bool ok = cs.pol->request(id, ev);
    for (int64_t e : ev) {
        cs.payload.erase(e);  // a query still using it holds its own reference
        cs.stats.evictions += 1;
    }
    return ok ? id : -1;
}

// Keep the arrays of a computed CSR result as item id's payload: they move
// into the cache (no copy); a result handed to the caller shares them
// (the caller holds cs.mu).
PayloadRef store_moved(CacheState &cs, Lane *L, int64_t id, int64_t rows, int64_t cols, int64_t nnz, Buf &rp,
                       Buf &col, Buf &val, atp_status &st) {
    auto P = std::make_shared<CachePayload>();
    P->rows = rows;
    P->cols = cols;
    P->nnz = nnz;
    P->bytes = cs.pol->item(id).size;
    P->rp = std::move(rp);
    P->col = std::move(col);
    P->val = std::move(val);
    P->n_active = -1;
    st = ATP_OK;
    if (hipEventCreateWithFlags(&P->ready, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(P->ready, L->stream) != hipSuccess) {
        (void)hipGetLastError();
        st = ATP_EDEVICE;
    }
    cs.payload[id] = P;
    cs.stats.inserts += 1;
    return P;
}

// Cache insertion after a query (Sec. 3.4.1): record the hits on cached
// sub-results, then try to insert the policy's candidates -- the whole query
// and, for the Overlap-Tree policies, the longest computed sub-metapath whose
// string is an overlap (an internal Overlap-Tree node); CBS1 only the whole
// query; CBS2 every computed product.  Replacement follows the policy.
atp_status cache_insert(atp_ctx *c, Lane *L, Mat &R, double root_cost, std::vector<KeptMat> &kept,
                        const std::vector<int64_t> &used, const int32_t *types, const std::vector<int> &rel,
                        const std::vector<std::string> &pkeys, int p, int weight, PayloadRef *root_payload) {
    CacheState &cs = c->cache;  // the caller holds cs.mu
    hipStream_t s = L->stream;
    for (int64_t id : used)
        for (int w = 0; w < weight; ++w) {
            std::vector<int64_t> ev;
            cs.pol->request(id, ev);
            cs.stats.sub_hits += 1;
        }
    struct Cand {
        int lo, hi;
        double cost;
        Mat *m;
        bool root;
    };
    std::vector<Cand> cands;
    cands.push_back(Cand{0, p - 1, root_cost, &R, true});
    // a product holding a count of 2^63 or more is never kept: as a whole
    // query it must answer ATP_EOVERFLOW, which only a recomputation reports;
    // nor is one whose size stayed on the device (its arrays are sized by the
    // symbolic bound: it was not a candidate when it was computed, though the
    // Overlap Tree may have changed since, other lanes inserting queries)
    auto keepable = [](const KeptMat &k) { return !k.partial && !k.m.saturated && !k.m.nnz_dev; };
    if (cs.policy == ATP_CACHE_CBS2) {
        for (auto &k : kept)
            if (keepable(k)) cands.push_back(Cand{k.lo, k.hi, k.cost, &k.m, false});
    } else if (cs.policy != ATP_CACHE_CBS1) {
        KeptMat *best = nullptr;
        for (auto &k : kept) {
            if (!keepable(k)) continue;
            const int node = cs.tree->find(std::vector<int32_t>(types + k.lo, types + k.hi + 2));
            if (node < 0 || cs.tree->node(node).leaf()) continue;
            if (!best || (k.hi - k.lo) > (best->hi - best->lo)) best = &k;
        }
        if (best) cands.push_back(Cand{best->lo, best->hi, best->cost, &best->m, false});
    }
    for (const Cand &cd : cands) {
        const std::vector<int32_t> ty(types + cd.lo, types + cd.hi + 2);
        const std::vector<int32_t> rl(rel.begin() + cd.lo, rel.begin() + cd.hi + 1);
        const std::vector<std::string> ps(pkeys.begin() + cd.lo, pkeys.begin() + cd.hi + 2);
        const Mat &m = *cd.m;
        const double bytes = 8.0 * (m.rows + 1) + 12.0 * m.nnz + (m.n_active >= 0 ? 4.0 * m.n_active : 0.0);
        const int64_t id = admit_item(cs, item_key(ty, rl, ps), ty, rl, ps, bytes, cd.cost);
        if (id < 0) continue;
        if (cd.root) {  // the result the caller receives shares the kept arrays
            atp_status st = ATP_OK;
            *root_payload = store_moved(cs, L, id, m.rows, m.cols, m.nnz, cd.m->rp, cd.m->col, cd.m->val, st);
            TRY(st);
            continue;
        }
        auto P = std::make_shared<CachePayload>();
        P->rows = m.rows;
        P->cols = m.cols;
        P->nnz = m.nnz;
        P->bytes = cs.pol->item(id).size;
        P->rp = std::move(cd.m->rp);
        P->col = std::move(cd.m->col);
        P->val = std::move(cd.m->val);
        P->n_active = cd.m->n_active;
        if (cd.m->n_active >= 0) P->active = std::move(cd.m->active);
        // other lanes order their reads after this lane's writes through the event
        HIPTRY(hipEventCreateWithFlags(&P->ready, hipEventDisableTiming));
        HIPTRY(hipEventRecord(P->ready, s));
        cs.payload[id] = std::move(P);
        cs.stats.inserts += 1;
    }
    return ATP_OK;
}

atp_status eval_impl(atp_ctx *c, Lane *L, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                     const atp_constraint *cons, int32_t n_cons, const char *plan, int weight, atp_result **out,
                     bool use_cache = true) {
    if (out) *out = nullptr;
    if (!c || !types || !out) return ATP_EINVAL;
    if (c->broken) return ATP_EDEVICE;
    if (n_types < 2) return ATP_EINVAL;
    if (n_cons < 0 || (n_cons > 0 && !cons)) return ATP_EINVAL;
    // relations of every step (Def. 2; one matrix per edge type)
    const int p = n_types - 1;
    std::vector<int> rel;
    TRY(resolve_rels(c, types, n_types, rel_ids, rel));
    for (int q = 0; q < n_cons; ++q) {
        const atp_constraint &k = cons[q];
        if (k.position < 0 || k.position >= n_types) return ATP_EINVAL;
        if (k.kind == ATP_C_RANGE) {
            if (k.prop_id < 0 || k.prop_id >= (int)c->props.size()) return ATP_EINVAL;
            if (c->props[k.prop_id]->type != types[k.position]) return ATP_EINVAL;
        } else if (k.kind == ATP_C_IDSET) {
            if (k.n_ids < 0 || (k.n_ids > 0 && !k.ids)) return ATP_EINVAL;
            const int64_t n = c->types[types[k.position]].count;
            for (int64_t z = 0; z < k.n_ids; ++z)
                if (k.ids[z] < 0 || k.ids[z] >= n) return ATP_EINVAL;
        } else {
            return ATP_EINVAL;
        }
    }
    std::vector<PlanTree> forced;
    int forced_root = -1;
    if (plan && !parse_plan(plan, p, forced, forced_root)) return ATP_EINVAL;

    hipStream_t s = L->stream;
    KernelTimer *t = c->kt(L);
    // masks M_1..M_n (Def. 3).  Their popcounts (planner selectivities) come
    // from the id count of a lone id-set constraint, from a memo of range
    // constraints seen before, or from the device (one readback)
    const std::vector<std::string> mkeys = position_keys(c, n_types, cons, n_cons);
    std::vector<int> n_at(n_types, 0), ranges_at(n_types, 0);
    for (int q = 0; q < n_cons; ++q) {
        n_at[cons[q].position] += 1;
        ranges_at[cons[q].position] += cons[q].kind == ATP_C_RANGE;
    }
    std::vector<PosMask> masks(n_types);
    Buf pops;
    TRY(pops.alloc(&L->pool, 8 * n_types));
    std::vector<std::string> memo_key(n_types);
    bool readback = false;
    std::vector<int> same(n_types, -1);  // an earlier position of the same type with the same constraints
    for (int i = 0; i < n_types; ++i)
        for (int j = 0; j < i && !mkeys[i].empty(); ++j)
            if (types[j] == types[i] && mkeys[j] == mkeys[i]) {
                same[i] = j;
                break;
            }
    for (int i = 0; i < n_types; ++i) {
        if (same[i] >= 0) continue;  // shares that position's mask (below)
        TRY(build_mask(c, L, types[i], cons, n_cons, i, masks[i]));
        if (masks[i].pop < 0) continue;
        if (n_at[i] == 1 && ranges_at[i] == 0) {
            masks[i].pop = masks[i].n_ids;
            continue;
        }
        memo_key[i] = std::to_string(types[i]) + "|" + mkeys[i];
        {
            std::lock_guard<std::mutex> g(c->stat_mu);
            auto it = c->pop_memo.find(memo_key[i]);
            if (it != c->pop_memo.end()) {
                masks[i].pop = it->second;
                memo_key[i].clear();
                continue;
            }
        }
        if (!readback) launch_fill_i64(pops.as<int64_t>(), n_types, 0, s, t);
        readback = true;
        launch_popcount(masks[i].bits.as<uint32_t>(), (c->types[types[i]].count + 31) / 32, pops.as<int64_t>() + i,
                        s, t);
    }
    if (readback) {
        std::vector<int64_t> h_pop(n_types, 0);
        HIPTRY(hipMemcpyAsync(h_pop.data(), pops.p, 8 * n_types, hipMemcpyDeviceToHost, s));
        TRY(sync(L));
        std::lock_guard<std::mutex> g(c->stat_mu);
        for (int i = 0; i < n_types; ++i)
            if (!memo_key[i].empty()) {
                masks[i].pop = h_pop[i];
                c->pop_memo[memo_key[i]] = h_pop[i];
            }
    }
    for (int i = 0; i < n_types; ++i)
        if (same[i] >= 0) {
            const PosMask &m0 = masks[same[i]];
            masks[i].alias = &m0;
            masks[i].pop = m0.pop;
            masks[i].n_ids = m0.n_ids;
            masks[i].h_ids = m0.h_ids;
        }
    auto sel_of = [&](int i) {
        const double n = (double)c->types[types[i]].count;
        return masks[i].pop >= 0 ? (n > 0 ? masks[i].pop / n : 0.0) : 1.0;
    };

    // leaves: relation i with masks of positions i and i+1
    std::vector<Mat> leaves(p);
    std::vector<ChainStats> lst(p);
    for (int i = 0; i < p; ++i) {
        const Rel &r = *c->rels[rel[i]];
        Mat &L = leaves[i];
        L.leaf = true;
        L.rows = c->types[types[i]].count;
        L.cols = c->types[types[i + 1]].count;
        L.nnz = r.nnz;
        L.op = Operand{r.rp.as<int64_t>(), r.col.as<int32_t>(), nullptr,
                       masks[i].pop >= 0 ? masks[i].bits_ptr() : nullptr,
                       masks[i + 1].pop >= 0 ? masks[i + 1].bits_ptr() : nullptr, L.rows, L.cols, r.nnz};
        if (masks[i].n_ids >= 0) {
            L.cand = masks[i].ids_ptr();
            L.n_cand = masks[i].n_ids;
        }
        ChainStats cs;
        cs.dim_r = (double)L.rows;
        cs.dim_c = (double)L.cols;
        const double sr = sel_of(i), sc = sel_of(i + 1);
        if (masks[i].n_ids >= 0) {
            double z = 0;
            // rows of the id list with edges, thinned by any other constraint at the position
            const double thin = masks[i].n_ids > 0 ? std::min(1.0, sr * L.rows / (double)masks[i].n_ids) : 0.0;
            cs.rows = est_rows_with_ids(r, masks[i].h_ids, &z) * thin;
            z *= thin;
            cs.nnz = z * sc;
        } else {
            cs.rows = (double)r.nonempty_rows * sr;
            cs.nnz = (double)r.nnz * sr * sc;
        }
        cs.cols = (double)r.nonempty_cols * sc;
        lst[i] = cs;
    }
    // ---- workload cache: Overlap Tree update and cached sub-chains ----
    CacheState &cs = c->cache;
    std::unique_lock<std::mutex> cache_lock(cs.mu);
    const bool caching = use_cache && cs.policy != ATP_CACHE_OFF && p >= 2;
    const int32_t cache_policy = cs.policy;
    std::vector<std::string> pkeys;
    std::vector<std::vector<int64_t>> cached_item(p, std::vector<int64_t>(p, -1));
    std::map<int64_t, PayloadRef> pins;  // cached results this query may read
    std::vector<std::vector<int64_t>> kfreq(p, std::vector<int64_t>(p, 0));  // Overlap Tree f of each sub-chain's key
    std::vector<std::vector<char>> overlap(p, std::vector<char>(p, 0));    // its string is an internal node
    std::vector<ChainStats> cached_stats_store(p * p);
    std::vector<std::vector<const ChainStats *>> cached_stats(p, std::vector<const ChainStats *>(p, nullptr));
    auto sub_types = [&](int a, int b) { return std::vector<int32_t>(types + a, types + b + 2); };
    auto sub_rels = [&](int a, int b) { return std::vector<int32_t>(rel.begin() + a, rel.begin() + b + 1); };
    auto sub_pos = [&](int a, int b) { return std::vector<std::string>(pkeys.begin() + a, pkeys.begin() + b + 2); };
    uint64_t cache_budget = 0;
    if (caching) {
        cache_budget = cs.budget;
        pkeys = position_keys(c, n_types, cons, n_cons);
        for (int w = 0; w < weight; ++w) cs.tree->insert(std::vector<int32_t>(types, types + n_types));
        cs.stats.queries += weight;
        for (int a = 0; a < p; ++a)
            for (int b = a; b < p; ++b) {
                const std::vector<int32_t> st_ = sub_types(a, b);
                const std::string key = item_key(st_, sub_rels(a, b), sub_pos(a, b));
                const int node = cs.tree->find(st_);
                if (node >= 0) {
                    cs.tree->node(node).keys[key].f += weight;
                    kfreq[a][b] = cs.tree->node(node).keys[key].f;
                }
                overlap[a][b] = node >= 0 && !cs.tree->node(node).leaf();
                auto it = cs.item_by_key.find(key);
                if (it == cs.item_by_key.end()) continue;
                if (node >= 0) cs.tree->node(node).keys[key].item = it->second;
                cs.info[it->second].node = node;
                auto pl = cs.payload.find(it->second);
                if (pl == cs.payload.end() || b == a) continue;
                cached_item[a][b] = it->second;
                pins[it->second] = pl->second;
                ChainStats &z = cached_stats_store[a * p + b];
                const CachePayload &P = *pl->second;
                z.dim_r = (double)P.rows;
                z.dim_c = (double)P.cols;
                z.nnz = (double)P.nnz;
                z.rows = P.n_active >= 0 ? (double)P.n_active : std::min((double)P.rows, (double)P.nnz);
                z.cols = std::min((double)P.cols, (double)P.nnz);
                cached_stats[a][b] = &z;
            }
    }
    cache_lock.unlock();

    std::string plan_str;
    std::vector<std::vector<double>> span_nnz;  // planner estimate of every sub-chain (none for a given plan)
    // Eq. 1 over the leaves, with cached sub-chains at no cost when with_cache
    auto choose_plan = [&](bool with_cache) -> atp_status {
        std::vector<JunctionSketch> js;
        std::vector<double> jsel, csel;
        std::vector<ColumnHist> ch;
        const bool uniform = (c->flags & ATP_OPT_PLAN_EAC) != 0;
        for (int k = 0; k + 1 < p; ++k) {
            if (!uniform) js.push_back(sketch_for(c, rel[k], rel[k + 1]));
            jsel.push_back(sel_of(k + 1));
        }
        for (int k = 0; k < p && !uniform; ++k) {
            std::lock_guard<std::mutex> g(c->stat_mu);
            auto it = c->col_hists.find(rel[k]);
            if (it == c->col_hists.end()) {
                const Rel &r = *c->rels[rel[k]];
                it = c->col_hists.emplace(rel[k], make_column_hist(r.h_indeg.data(), (int64_t)r.h_indeg.size()))
                         .first;
            }
            ch.push_back(it->second);
            csel.push_back(sel_of(k + 1));
        }
        const CostCoeffs cc = c->cost;
        PlanResult pr = plan_chain(lst, js, jsel, ch, csel, uniform ? Estimator::Uniform : Estimator::Sketch, cc,
                                   with_cache ? &cached_stats : nullptr);
        plan_str = pr.plan;
        span_nnz = std::move(pr.span_nnz);
        return parse_plan(plan_str.c_str(), p, forced, forced_root) ? ATP_OK : ATP_ESTATE;
    };
    if (plan) {
        plan_str = plan;
        for (const PlanTree &nd : forced)
            if (nd.block_lo >= 0 && (!caching || cached_item[nd.block_lo][nd.block_hi] < 0)) return ATP_EINVAL;
    } else {
        TRY(choose_plan(caching));
    }

    // a single relation: multiply by the identity so the masked relation is
    // materialised with values by the same kernels
    Buf ident_rp, ident_col;
    Mat ident;
    if (p == 1) {
        const int64_t n = leaves[0].cols;
        TRY(ident_rp.alloc(&L->pool, 8 * (n + 1)));
        TRY(ident_col.alloc(&L->pool, 4 * std::max<int64_t>(n, 1)));
        std::vector<int64_t> h_rp(n + 1);
        std::vector<int32_t> h_col(n);
        for (int64_t z = 0; z <= n; ++z) h_rp[z] = z;
        for (int64_t z = 0; z < n; ++z) h_col[z] = (int32_t)z;
        HIPTRY(hipMemcpyAsync(ident_rp.p, h_rp.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));
        if (n) HIPTRY(hipMemcpyAsync(ident_col.p, h_col.data(), 4 * n, hipMemcpyHostToDevice, s));
        TRY(sync(L));
        ident.leaf = true;
        ident.rows = ident.cols = n;
        ident.nnz = n;
        ident.op = Operand{ident_rp.as<int64_t>(), ident_col.as<int32_t>(), nullptr, nullptr, nullptr, n, n, n};
    }


    StepStats st;
    int n_products = 0;
    bool overflow = false;
    std::vector<PlanTree> &tree = forced;
    std::vector<Buf> keep;  // restriction buffers, alive until the query ends
    const bool restrict_rows = (c->flags & ATP_OPT_NO_RESTRICT) == 0;
    // leaves covered by a plan node
    std::function<std::pair<int, int>(int)> span = [&](int v) -> std::pair<int, int> {
        const PlanTree &nd = tree[v];
        if (nd.leaf >= 0) return {nd.leaf, nd.leaf};
        if (nd.block_lo >= 0) return {nd.block_lo, nd.block_hi};
        return {span(nd.left).first, span(nd.right).second};
    };
    // a product whose right operand is itself a product: its rows can be
    // restricted to the left operand's columns (a base relation's rows are
    // only read where the left operand points, so it gains nothing)
    auto internal = [&](int v) { return tree[v].leaf < 0 && tree[v].block_lo < 0; };
    std::vector<char> feeds_restriction;
    auto mark_restrictions = [&]() {
        feeds_restriction.assign(tree.size(), 0);
        for (size_t v = 0; v < tree.size(); ++v)
            if (restrict_rows && internal((int)v) && internal(tree[v].right)) feeds_restriction[tree[v].left] = 1;
    };
    mark_restrictions();
    // intermediates whose sizes stay on the device (no read-back per product):
    // not the result, not kept by the cache, not timed or byte-counted, and not
    // a left operand whose size decides a restriction
    // with a cache, only the products its insertion policy may keep need exact
    // sizes: the result, and sub-chains computed on all their rows that CBS2
    // keeps (every one) or the Overlap-Tree policies keep (overlaps)
    const bool may_defer = !(c->flags & ATP_OPT_COUNT_BYTES) && !c->cost_sink;
    auto cache_candidate = [&](int lo_, int hi_, bool partial) -> bool {
        if (!caching || partial) return false;
        if (cache_policy == ATP_CACHE_CBS2) return true;
        if (cache_policy == ATP_CACHE_CBS1) return false;
        return overlap[lo_][hi_] != 0;
    };
    Buf nnz_acc;
    if (may_defer && p >= 3) {  // nonzeros and fault flag of the deferred products
        TRY(nnz_acc.alloc(&L->pool, 16));
        launch_fill_i64(nnz_acc.as<int64_t>(), 2, 0, s, t);
    }
    // Rows of a right sub-chain that can matter: the columns its left neighbour uses.
    struct Restriction {
        const uint32_t *bits = nullptr;
        const int32_t *list = nullptr;
        int64_t n = 0;
    };
    auto make_restriction = [&](const Mat &X, int64_t n_rows_y, Restriction &r) -> atp_status {
        const int64_t words = (n_rows_y + 31) / 32;
        Buf bits, cnt, scan, tmpb, list;
        TRY(bits.alloc(&L->pool, 4 * (size_t)std::max<int64_t>(words, 1)));
        TRY(cnt.alloc(&L->pool, 8 * (size_t)std::max<int64_t>(words, 1)));
        TRY(scan.alloc(&L->pool, 8 * (size_t)(words + 1)));
        TRY(tmpb.alloc(&L->pool, 8 * (size_t)scan_tmp_elems(words)));
        launch_fill_u32(bits.as<uint32_t>(), words, 0u, s, t);
        Buf len, off, tmpc;
        if (X.leaf) {
            TRY(len.alloc(&L->pool, 8 * (size_t)std::max<int64_t>(X.n_cand, 1)));
            TRY(off.alloc(&L->pool, 8 * (size_t)(X.n_cand + 1)));
            TRY(tmpc.alloc(&L->pool, 8 * (size_t)scan_tmp_elems(X.n_cand)));
            launch_leaf_cols_to_bits(X.op, X.cand, X.n_cand, len.as<int64_t>(), off.as<int64_t>(), tmpc.as<int64_t>(),
                                     bits.as<uint32_t>(), s, t);
        } else
            launch_cols_to_bits(X.op.col, X.nnz, X.nnz_dev, bits.as<uint32_t>(), s, t);
        launch_bits_count(bits.as<uint32_t>(), words, cnt.as<int64_t>(), scan.as<int64_t>(), tmpb.as<int64_t>(), s, t);
        TRY(read_values(L, scan.as<int64_t>() + words, 1));
        const int64_t n = *(const int64_t *)L->h_hdr;
        TRY(list.alloc(&L->pool, 4 * (size_t)std::max<int64_t>(n, 1)));
        launch_bits_scatter(bits.as<uint32_t>(), words, scan.as<int64_t>(), list.as<int32_t>(), s, t);
        r.bits = bits.as<uint32_t>();
        r.list = list.as<int32_t>();
        r.n = n;
        keep.push_back(std::move(bits));
        keep.push_back(std::move(list));
        keep.push_back(std::move(scan));  // the scatter may still be reading it
        return ATP_OK;
    };
    std::vector<KeptMat> kept;  // products kept for the cache's insertion policy
    struct CostRecord {
        double nnz_x = 0, n_op = 0, nnz_z = 0;
        hipEvent_t e0 = nullptr, e1 = nullptr;
    };
    struct CostRecords : std::vector<CostRecord> {
        ~CostRecords() {
            for (auto &r : *this) {
                if (r.e0) (void)hipEventDestroy(r.e0);
                if (r.e1) (void)hipEventDestroy(r.e1);
            }
        }
    } cost_recs;
    std::vector<int64_t> used_items;
    bool whole_allowed = true;
    bool whole_taken = false;  // a sub-chain was computed on all its rows for the cache
    // post-order evaluation of node v into outm; rs restricts v's rows; cost =
    // seconds to compute it from the base relations in this query
    std::function<atp_status(int, bool, const Restriction *, Mat &, int &, int &, double &)> run =
        [&](int v, bool as_left, const Restriction *rs, Mat &outm, int &lo, int &hi, double &cost) -> atp_status {
        const PlanTree &nd = tree[v];
        cost = 0;
        if (nd.block_lo >= 0) {  // a cached result, computed on all its rows
            lo = nd.block_lo;
            hi = nd.block_hi;
            const int64_t id = cached_item[lo][hi];
            const CachePayload &P = *pins.at(id);
            HIPTRY(hipStreamWaitEvent(s, P.ready, 0));
            outm = Mat();
            outm.view = true;
            outm.rows = P.rows;
            outm.cols = P.cols;
            outm.nnz = P.nnz;
            outm.n_active = P.n_active;
            outm.active_ptr = P.n_active >= 0 ? P.active.as<int32_t>() : nullptr;
            if (rs && (P.n_active < 0 || rs->n < P.n_active)) {
                // as a left operand under a restriction only the listed rows are multiplied
                // (a listed row that is empty in the result adds nothing)
                outm.n_active = rs->n;
                outm.active_ptr = rs->list;
            }
            outm.op = Operand{P.rp.as<int64_t>(), P.col.as<int32_t>(), P.val.as<uint64_t>(), nullptr, nullptr,
                              P.rows, P.cols, P.nnz};
            used_items.push_back(id);
            return ATP_OK;
        }
        if (nd.leaf >= 0) {
            lo = hi = nd.leaf;
            outm = Mat();
            outm.leaf = true;
            const Mat &L = leaves[nd.leaf];
            outm.op = L.op;
            outm.rows = L.rows;
            outm.cols = L.cols;
            outm.nnz = L.nnz;
            outm.cand = L.cand;
            outm.n_cand = L.n_cand;
            if (rs) {
                // rs.bits is a subset of this position's mask (it is the masked column set of the
                // left neighbour), so it replaces the row mask; an id list stays the candidate list
                outm.op.rmask = rs->bits;
                if (!outm.cand) {
                    outm.cand = rs->list;
                    outm.n_cand = rs->n;
                }
            }
            return ATP_OK;
        }
        Mat X, Y;
        int l0, l1, r0, r1;
        double cx = 0, cy = 0;
        TRY(run(nd.left, true, rs, X, l0, l1, cx));
        Restriction r2;
        const Restriction *rp = nullptr;
        const int64_t y_rows = c->types[types[l1 + 1]].count;
        const bool x_small = X.leaf ? (X.cand != nullptr && X.n_cand < y_rows) : (X.nnz < y_rows / 2);
        // with a cache, a right sub-chain that is an overlap (seen in an earlier
        // query) is computed on all its rows so that its result can be kept
        // (only when its estimated columns and values fit an item the cache admits, at most
        // 80% of its budget, and not on the retry of a query that ran out of memory with it)
        const std::pair<int, int> ysp = span(nd.right);
        const bool fits =
            span_nnz.empty() || 12.0 * span_nnz[ysp.first][ysp.second] <= 0.8 * (double)cache_budget;
        const int64_t f_y = kfreq[ysp.first][ysp.second];
        const bool whole_candidate = caching && whole_allowed && fits && ysp.second > ysp.first && f_y >= 2;
        if (restrict_rows && x_small && internal(nd.right)) {
            // computing the sub-chain whole costs about 1/share times its restricted form, where
            // share is the part of its rows the left operand reaches; a sub-chain seen f times
            // with the same constraints (its item key) is expected back about f - 1 times, so the
            // whole form is kept only when share * f >= 1
            TRY(make_restriction(X, y_rows, r2));
            if (!(whole_candidate && (double)r2.n * (double)f_y >= (double)y_rows))
                rp = &r2;
            else
                whole_taken = true;
        }
        TRY(run(nd.right, false, rp, Y, r0, r1, cy));
        lo = l0;
        hi = r1;
        const int last_pos = r1 + 1;  // metapath position of Y's last type
        const int64_t ycols_eff = masks[last_pos].pop >= 0 ? masks[last_pos].pop : Y.cols;
        bool sat = false;
        if (c->step_names) L->timer.suffix = "#" + std::to_string(n_products);
        const auto t_0 = std::chrono::steady_clock::now();
        CostRecord rec;
        if (c->cost_sink) {  // device time of this multiplication, for the cost-model fit
            rec.nnz_x = X.leaf ? lst[l0].nnz : (double)X.nnz;
            rec.n_op = (double)st.n_op;
            HIPTRY(hipEventCreate(&rec.e0));
            HIPTRY(hipEventCreate(&rec.e1));
            HIPTRY(hipEventRecord(rec.e0, s));
        }
        const bool defer_ok = may_defer && !cache_candidate(lo, hi, rs != nullptr);
        const bool defer = defer_ok && v != forced_root && !feeds_restriction[v];
        // a left operand whose size decides its parent's restriction (size below half the rows
        // of the parent's right operand) can keep its size on the device when its bound decides
        const int64_t defer_below = defer_ok && v != forced_root && feeds_restriction[v]
                                        ? c->types[types[r1 + 1]].count / 2
                                        : 0;
        TRY(spgemm(c, L, X, Y, ycols_eff, as_left, outm, st, sat, defer, nnz_acc.as<int64_t>(), defer_below,
                   v != forced_root));
        if (c->cost_sink) {
            HIPTRY(hipEventRecord(rec.e1, s));
            rec.n_op = (double)st.n_op - rec.n_op;
            rec.nnz_z = (double)outm.nnz;
            cost_recs.push_back(rec);
            rec.e0 = rec.e1 = nullptr;
        }
        cost = cx + cy + std::chrono::duration<double>(std::chrono::steady_clock::now() - t_0).count();
        L->timer.suffix.clear();
        ++n_products;
        if (v == forced_root && sat) overflow = true;
        if (caching) {  // keep computed operands for the insertion policy
            if (!X.leaf && !X.view) kept.push_back(KeptMat{l0, l1, cx, rs != nullptr, std::move(X)});
            if (!Y.leaf && !Y.view) kept.push_back(KeptMat{r0, r1, cy, rp != nullptr, std::move(Y)});
        }
        return ATP_OK;
    };
    Mat R;
    PayloadRef result_payload;  // set when the result's arrays are (or become) a cached item's
    int lo = 0, hi = 0;
    atp_status stt;
    if (p == 1) {
        const int64_t ycols_eff = masks[1].pop >= 0 ? masks[1].pop : leaves[0].cols;
        Mat X;
        X.leaf = true;
        X.op = leaves[0].op;
        X.op.cmask = nullptr;  // the column mask is applied through the identity's columns
        X.rows = leaves[0].rows;
        X.cols = leaves[0].cols;
        X.nnz = leaves[0].nnz;
        X.cand = leaves[0].cand;
        X.n_cand = leaves[0].n_cand;
        ident.op.cmask = leaves[0].op.cmask;
        bool sat = false;
        stt = spgemm(c, L, X, ident, ycols_eff, false, R, st, sat, false, nullptr, 0, false);
        n_products = 1;
        overflow = sat;
    } else if (caching && tree[forced_root].block_lo == 0 && tree[forced_root].block_hi == p - 1) {
        // the whole query is cached: the result shares the item's arrays (read-only, kept alive by
        // the result even if the item is evicted)
        const int64_t id = cached_item[0][p - 1];
        result_payload = pins.at(id);
        const CachePayload &P = *result_payload;
        R.rows = P.rows;
        R.cols = P.cols;
        R.nnz = P.nnz;
        stt = hipStreamWaitEvent(s, P.ready, 0) == hipSuccess ? ATP_OK : ATP_EDEVICE;
        std::lock_guard<std::mutex> g(cs.mu);
        for (int w = 0; w < weight; ++w) {
            std::vector<int64_t> ev;
            cs.pol->request(id, ev);
            cs.stats.whole_hits += 1;
        }
    } else {
        double root_cost = 0;
        stt = run(forced_root, false, nullptr, R, lo, hi, root_cost);
        bool plan_blocks = false;  // the plan reads cached blocks
        for (const PlanTree &nd : forced) plan_blocks |= nd.block_lo >= 0;
        if ((stt == ATP_ENOMEM || stt == ATP_EBUDGET) && caching && (whole_taken || plan_blocks)) {
            // out of memory with the cache's choices (cached blocks in the plan, a sub-chain
            // computed on all its rows to be kept): once more as without the cache (a query
            // that made neither choice would only fail the same way again)
            (void)hipStreamSynchronize(s);
            for (auto &r : cost_recs) {
                if (r.e0) (void)hipEventDestroy(r.e0);
                if (r.e1) (void)hipEventDestroy(r.e1);
            }
            cost_recs.clear();
            kept.clear();
            keep.clear();
            used_items.clear();
            R = Mat();
            st = StepStats();
            n_products = 0;
            overflow = false;
            whole_allowed = false;
            stt = plan ? ATP_OK : choose_plan(false);
            mark_restrictions();
            if (stt == ATP_OK) stt = run(forced_root, false, nullptr, R, lo, hi, root_cost);
        }
        if (stt == ATP_OK && caching && !overflow) {
            std::lock_guard<std::mutex> g(cs.mu);
            if (cs.pol)  // the cache may have been switched off meanwhile
                stt = cache_insert(c, L, R, root_cost, kept, used_items, types, rel, pkeys, p, weight,
                                   &result_payload);
        }
    }
    if (stt != ATP_OK) {
        if (stt == ATP_EDEVICE) c->broken = true;
        (void)hipStreamSynchronize(s);
        return stt;
    }
    // the deferred count comes back through the lane's pinned header, which
    // the last product has finished reading
    if (nnz_acc.p) HIPTRY(hipMemcpyAsync(L->h_hdr, nnz_acc.p, 16, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    if (nnz_acc.p) {
        st.nnz += ((const int64_t *)L->h_hdr)[0];
        if (((const int64_t *)L->h_hdr)[1]) {  // a deferred product's hash table overflowed
            c->broken = true;
            return ATP_EDEVICE;
        }
    }
    if (t) t->flush();
    if (c->cost_sink && !cost_recs.empty()) {
        std::lock_guard<std::mutex> g(c->stat_mu);
        for (auto &r : cost_recs) {
            float ms = 0;
            if (hipEventElapsedTime(&ms, r.e0, r.e1) == hipSuccess)
                c->cost_sink->push_back({r.nnz_x, r.n_op, r.nnz_z, (double)ms});
        }
    }
    if (overflow) return ATP_EOVERFLOW;
    atp_result *res = new atp_result();
    res->ctx = c;
    res->stream = s;
    res->rows = R.rows;
    res->cols = R.cols;
    res->nnz = R.nnz;
    if (result_payload) {
        res->shared = std::move(result_payload);
    } else {
        res->rp = std::move(R.rp);
        res->col = std::move(R.col);
        res->val = std::move(R.val);
    }
    res->plan = plan_str;
    res->stats.n_products = n_products;
    res->stats.n_op_total = st.n_op;
    res->stats.nnz_result = R.nnz;
    res->stats.nnz_intermediate_total = st.nnz - R.nnz;
    res->stats.slots_total = st.slots;
    register_result(c, res);
    *out = res;
    return ATP_OK;
}

}  // namespace

namespace atp {

void register_result(atp_ctx *c, atp_result *r) {
    std::lock_guard<std::mutex> g(c->results_mu);
    c->results.insert(r);
}

atp_status eval_query(atp_ctx *c, Lane *L, const QueryRef &q, const char *plan, int weight, atp_result **out) {
    return eval_impl(c, L, q.types, q.n_types, q.rel_ids, q.cons, q.n_cons, plan, weight < 1 ? 1 : weight, out);
}

void release_pool_caches(atp_ctx *c) {
    c->main.pool.release_cache();
    for (auto &ln : c->lanes) ln->pool.release_cache();
}

// Whole-query cache key of q, or "" when q does not resolve.
static std::string whole_key(atp_ctx *c, const QueryRef &q, std::vector<int32_t> &ty, std::vector<int32_t> &rl,
                             std::vector<std::string> &ps) {
    if (!q.types || q.n_types < 2) return "";
    std::vector<int> rel;
    if (resolve_rels(c, q.types, q.n_types, q.rel_ids, rel) != ATP_OK) return "";
    ty.assign(q.types, q.types + q.n_types);
    rl.assign(rel.begin(), rel.end());
    ps = position_keys(c, q.n_types, q.cons, q.n_cons);
    return item_key(ty, rl, ps);
}

bool cache_has_whole(atp_ctx *c, const QueryRef &q) {
    CacheState &cs = c->cache;
    {
        std::lock_guard<std::mutex> g(cs.mu);
        if (cs.policy == ATP_CACHE_OFF) return false;
    }
    std::vector<int32_t> ty, rl;
    std::vector<std::string> ps;
    const std::string key = whole_key(c, q, ty, rl, ps);
    if (key.empty()) return false;
    std::lock_guard<std::mutex> g(cs.mu);
    auto it = cs.item_by_key.find(key);
    return it != cs.item_by_key.end() && cs.payload.count(it->second) > 0;
}

atp_status cache_offer_whole(atp_ctx *c, Lane *L, const QueryRef &q, atp_result &r, double cost_s) {
    std::vector<int32_t> ty, rl;
    std::vector<std::string> ps;
    const std::string key = whole_key(c, q, ty, rl, ps);
    if (key.empty()) return ATP_OK;
    CacheState &cs = c->cache;
    std::lock_guard<std::mutex> g(cs.mu);
    if (cs.policy == ATP_CACHE_OFF || !cs.pol) return ATP_OK;
    const int node = cs.tree->find(ty);
    if (node >= 0) cs.tree->node(node).keys[key].f += 1;
    const double bytes = 8.0 * (r.rows + 1) + 12.0 * r.nnz;
    const int64_t id = admit_item(cs, key, ty, rl, ps, bytes, cost_s);
    if (id < 0) return ATP_OK;
    if (r.shared) return ATP_OK;  // already an item's arrays
    atp_status st = ATP_OK;
    r.shared = store_moved(cs, L, id, r.rows, r.cols, r.nnz, r.rp, r.col, r.val, st);
    return st;
}

atp_status lane_init(atp_ctx *c, Lane *L, int id) {
    L->id = id;
    L->wait_limit_s = c->wait_limit_s;
    // each lane has its own pool: a block it frees is reused only by later work on its own stream,
    // which is ordered after the work that used the block
    L->pool.on_oom = [c]() { release_pool_caches(c); };
    L->pool.cache_limit = c->pool_cache_total;  // until ensure_lanes shares it out
    L->pool.budget = c->main.pool.budget;
    L->pool.user_alloc = c->main.pool.user_alloc;
    L->pool.user_free = c->main.pool.user_free;
    L->pool.user = c->main.pool.user;
    if (hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return ATP_EDEVICE;
    }
    L->own_stream = true;
    return lane_mailbox(L);
}

// The pinned block holds the step header (a mailbox of posted values) and,
// 64-byte aligned after it, the post flag; both get device addresses when
// the runtime maps them (else values are read by copies).
atp_status lane_mailbox(Lane *L) {
    constexpr size_t hdr_bytes = (sizeof(StepHeader) + 63) / 64 * 64;
    void *p = nullptr;
    if (hipHostMalloc(&p, hdr_bytes + 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return ATP_ENOMEM;
    }
    std::memset(p, 0, hdr_bytes + 64);
    L->h_hdr = (StepHeader *)p;
    L->h_flag = (uint64_t *)((char *)p + hdr_bytes);
    L->seq = 0;
    void *dp = nullptr;
    if (hipHostGetDevicePointer(&dp, p, 0) == hipSuccess && dp) {
        L->d_mailbox = (int64_t *)dp;
        L->d_flag = (uint64_t *)((char *)dp + hdr_bytes);
    } else {
        (void)hipGetLastError();
        L->d_mailbox = nullptr;
        L->d_flag = nullptr;
    }
    if (std::getenv("ATP_NO_MAILBOX")) {  // read posted values by copies instead
        L->d_mailbox = nullptr;
        L->d_flag = nullptr;
    }
    return ATP_OK;
}

void lane_free_mailbox(Lane *L) {
    if (L->h_hdr) (void)hipHostFree(L->h_hdr);
    L->h_hdr = nullptr;
    L->h_flag = nullptr;
    L->d_mailbox = nullptr;
    L->d_flag = nullptr;
}

atp_status lane_sides(Lane *L) {
    if (L->fork) return ATP_OK;
    for (int i = 0; i < kSideStreams; ++i) {
        if (hipStreamCreateWithFlags(&L->side[i], hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L->join[i], hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            lane_release_sides(L);
            return ATP_EDEVICE;
        }
    }
    if (hipEventCreateWithFlags(&L->fork, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        lane_release_sides(L);
        return ATP_EDEVICE;
    }
    return ATP_OK;
}
void lane_release_sides(Lane *L) {
    for (int i = 0; i < kSideStreams; ++i) {
        if (L->side[i]) {
            (void)hipStreamSynchronize(L->side[i]);
            (void)hipStreamDestroy(L->side[i]);
        }
        if (L->join[i]) (void)hipEventDestroy(L->join[i]);
        L->side[i] = nullptr;
        L->join[i] = nullptr;
    }
    if (L->fork) (void)hipEventDestroy(L->fork);
    L->fork = nullptr;
}
void lane_destroy(Lane *L) {
    if (L->stream) (void)hipStreamSynchronize(L->stream);
    lane_release_sides(L);
    L->timer.flush();
    L->pool.destroy();
    lane_free_mailbox(L);
    if (L->own_stream && L->stream) (void)hipStreamDestroy(L->stream);
    L->stream = nullptr;
}

}  // namespace atp

// ---------------------------------------------------------------------------
// C-ABI

extern "C" {

const char *atp_status_str(atp_status st) {
    switch (st) {
        case ATP_OK: return "ok";
        case ATP_EINVAL: return "invalid argument";
        case ATP_ENOMEM: return "device out of memory";
        case ATP_EOVERFLOW: return "path count does not fit int64";
        case ATP_ESCHEMA: return "metapath does not follow the schema";
        case ATP_EDEVICE: return "HIP runtime error";
        case ATP_EBUDGET: return "memory budget exceeded";
        case ATP_ESTATE: return "invalid state";
        default: return "unknown status";
    }
}

atp_status atp_create(const atp_options *o, atp_ctx **out) {
    if (!out) return ATP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        (void)hipGetLastError();
        return ATP_ESTATE;
    }
    atp_options d{};
    if (o) d = *o;
    if (d.device < 0 || d.device >= ndev) return ATP_EINVAL;
    if ((d.alloc == nullptr) != (d.free == nullptr)) return ATP_EINVAL;
    if (hipSetDevice(d.device) != hipSuccess) return ATP_EDEVICE;
    atp_ctx *c = new atp_ctx();
    c->device = d.device;
    c->main.stream = (hipStream_t)d.hip_stream;
    c->flags = d.flags;
    c->main.pool.user_alloc = d.alloc;
    c->main.pool.user_free = d.free;
    c->main.pool.user = d.alloc_user;
    c->main.pool.budget = d.mem_budget_bytes;
    c->main.pool.on_oom = [c]() { release_pool_caches(c); };
    {  // free blocks kept for reuse: up to half the device's memory
        size_t fr = 0, total = 0;
        if (hipMemGetInfo(&fr, &total) == hipSuccess && total > 0)
            c->pool_cache_total = std::max<size_t>(c->pool_cache_total, total / 2);
        (void)hipGetLastError();
        if (const char *e = std::getenv("ATP_POOL_CACHE_GB"))  // diagnostics
            c->pool_cache_total = (size_t)(std::atof(e) * (double)(1ull << 30));
        c->main.pool.cache_limit = c->pool_cache_total;
    }
    c->main.wait_limit_s = c->wait_limit_s;
    // the static workspace of atp_eval_noalloc on this device (looked up once per device)
    if (scratch_address(d.device, &c->scratch) != ATP_OK) {
        delete c;
        return ATP_EDEVICE;
    }
    if (lane_mailbox(&c->main) != ATP_OK) {
        delete c;
        return ATP_ENOMEM;
    }
    *out = c;
    return ATP_OK;
}

atp_status atp_destroy(atp_ctx *c) {
    if (!c) return ATP_EINVAL;
    (void)hipSetDevice(c->device);
    server_shutdown(c);
    if (std::getenv("ATP_POOL_STATS")) {  // diagnostics: runtime allocations per lane
        std::fprintf(stderr, "pool main: %lld mallocs %.3f s, %lld frees %.3f s, held %.2f GB\n",
                     (long long)c->main.pool.n_malloc, c->main.pool.malloc_s, (long long)c->main.pool.n_free,
                     c->main.pool.free_s, c->main.pool.held / 1e9);
        for (auto &ln : c->lanes)
            std::fprintf(stderr, "pool lane %d: %lld mallocs %.3f s, %lld frees %.3f s, held %.2f GB\n", ln->id,
                         (long long)ln->pool.n_malloc, ln->pool.malloc_s, (long long)ln->pool.n_free, ln->pool.free_s,
                         ln->pool.held / 1e9);
    }
    (void)hipStreamSynchronize(c->main.stream);
    for (auto &ln : c->lanes) (void)hipStreamSynchronize(ln->stream);
    for (atp_result *r : c->results) delete r;
    c->results.clear();
    c->cache.payload.clear();
    for (auto &ln : c->lanes) lane_destroy(ln.get());
    c->lanes.clear();
    c->rels.clear();
    c->props.clear();
    lane_release_sides(&c->main);
    c->main.timer.flush();
    c->main.pool.destroy();
    lane_free_mailbox(&c->main);
    delete c;
    return ATP_OK;
}

atp_status atp_add_node_type(atp_ctx *c, const char *name, int64_t count, int32_t *type_id) {
    if (!c || count < 0 || count >= (int64_t)0x7FFFFFFF) return ATP_EINVAL;
    c->types.push_back(NodeType{name ? name : "", count});
    if (type_id) *type_id = (int32_t)c->types.size() - 1;
    return ATP_OK;
}

static atp_status add_rel_host(atp_ctx *c, int32_t src, int32_t dst, std::vector<int64_t> &&rp,
                               std::vector<int32_t> &&col, int32_t *rel_id) {
    auto r = std::make_unique<Rel>();
    r->src = src;
    r->dst = dst;
    r->nnz = (int64_t)col.size();
    const int64_t m = c->types[src].count, n = c->types[dst].count;
    TRY(r->rp.alloc(&c->main.pool, 8 * (m + 1)));
    TRY(r->col.alloc(&c->main.pool, 4 * std::max<int64_t>(r->nnz, 1)));
    HIPTRY(hipMemcpyAsync(r->rp.p, rp.data(), 8 * (m + 1), hipMemcpyHostToDevice, c->main.stream));
    if (r->nnz) HIPTRY(hipMemcpyAsync(r->col.p, col.data(), 4 * r->nnz, hipMemcpyHostToDevice, c->main.stream));
    r->h_indeg.assign(n, 0);
    for (int32_t j : col) r->h_indeg[j]++;
    for (int64_t i = 0; i < m; ++i) r->nonempty_rows += rp[i + 1] > rp[i];
    for (int64_t j = 0; j < n; ++j) r->nonempty_cols += r->h_indeg[j] > 0;
    HIPTRY(hipStreamSynchronize(c->main.stream));
    r->h_rp = std::move(rp);
    c->rels.push_back(std::move(r));
    if (rel_id) *rel_id = (int32_t)c->rels.size() - 1;
    return ATP_OK;
}

atp_status atp_add_relation(atp_ctx *c, int32_t src, int32_t dst, const int64_t *row_ptr, const int32_t *col,
                            int64_t nnz, uint32_t flags, int32_t *rel_id) {
    if (!c || !row_ptr || nnz < 0 || (nnz > 0 && !col)) return ATP_EINVAL;
    if (c->broken) return ATP_EDEVICE;
    if (src < 0 || dst < 0 || src >= (int)c->types.size() || dst >= (int)c->types.size()) return ATP_EINVAL;
    const int64_t m = c->types[src].count, n = c->types[dst].count;
    std::vector<int64_t> rp(m + 1);
    std::vector<int32_t> cl(nnz);
    if (flags & ATP_REL_DEVICE_PTRS) {
        HIPTRY(hipMemcpy(rp.data(), row_ptr, 8 * (m + 1), hipMemcpyDeviceToHost));
        if (nnz) HIPTRY(hipMemcpy(cl.data(), col, 4 * nnz, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(rp.data(), row_ptr, 8 * (m + 1));
        if (nnz) std::memcpy(cl.data(), col, 4 * nnz);
    }
    // validation: canonical CSR of a 0/1 matrix
    if (rp[0] != 0 || rp[m] != nnz) return ATP_EINVAL;
    for (int64_t i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) return ATP_EINVAL;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            if (cl[e] < 0 || cl[e] >= n) return ATP_EINVAL;
            if (e > rp[i] && cl[e] <= cl[e - 1]) return ATP_EINVAL;
        }
    }
    std::vector<int64_t> trp;
    std::vector<int32_t> tcol;
    const bool rev = (flags & ATP_REL_ADD_REVERSE) != 0;
    if (rev) {
        trp.assign(n + 1, 0);
        for (int32_t j : cl) trp[j + 1]++;
        for (int64_t j = 0; j < n; ++j) trp[j + 1] += trp[j];
        tcol.resize(nnz);
        std::vector<int64_t> cur(trp.begin(), trp.end() - 1);
        for (int64_t i = 0; i < m; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) tcol[cur[cl[e]]++] = (int32_t)i;
    }
    int32_t id = -1;
    TRY(add_rel_host(c, src, dst, std::move(rp), std::move(cl), &id));
    if (rev) {
        int32_t id2 = -1;
        TRY(add_rel_host(c, dst, src, std::move(trp), std::move(tcol), &id2));
    }
    if (rel_id) *rel_id = id;
    return ATP_OK;
}

atp_status atp_add_property(atp_ctx *c, int32_t type_id, const char *name, int32_t dtype, const void *values,
                            int32_t *prop_id) {
    if (!c || type_id < 0 || type_id >= (int)c->types.size()) return ATP_EINVAL;
    if (dtype != ATP_I16 && dtype != ATP_I32 && dtype != ATP_I64) return ATP_EINVAL;
    const int64_t n = c->types[type_id].count;
    if (n > 0 && !values) return ATP_EINVAL;
    if (c->broken) return ATP_EDEVICE;
    const size_t es = dtype == ATP_I16 ? 2 : dtype == ATP_I32 ? 4 : 8;
    auto p = std::make_unique<Prop>();
    p->type = type_id;
    p->dtype = dtype;
    p->name = name ? name : "";
    TRY(p->values.alloc(&c->main.pool, es * std::max<int64_t>(n, 1)));
    if (n) HIPTRY(hipMemcpyAsync(p->values.p, values, es * n, hipMemcpyHostToDevice, c->main.stream));
    HIPTRY(hipStreamSynchronize(c->main.stream));
    c->props.push_back(std::move(p));
    if (prop_id) *prop_id = (int32_t)c->props.size() - 1;
    return ATP_OK;
}

atp_status atp_eval(atp_ctx *c, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                    const atp_constraint *cons, int32_t n_cons, atp_result **out) {
    if (c) (void)hipSetDevice(c->device);
    return eval_impl(c, &c->main, types, n_types, rel_ids, cons, n_cons, nullptr, 1, out);
}

atp_status atp_eval_plan(atp_ctx *c, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                         const atp_constraint *cons, int32_t n_cons, const char *plan, atp_result **out) {
    if (c) (void)hipSetDevice(c->device);
    return eval_impl(c, &c->main, types, n_types, rel_ids, cons, n_cons, plan, 1, out);
}

atp_status atp_eval_noalloc(atp_ctx *c, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                            const atp_constraint *cons, int32_t n_cons, const char *plan, int64_t *row_ptr,
                            int32_t *col, int64_t *val, int64_t cap, int64_t *nnz) {
    if (nnz) *nnz = -1;
    if (!c || !row_ptr || !nnz || cap < 0 || (cap > 0 && (!col || !val))) return ATP_EINVAL;
    if (c->broken) return ATP_EDEVICE;
    if (!c->scratch) return ATP_ESTATE;
    (void)hipSetDevice(c->device);
    Lane *L = &c->main;
    {
        std::lock_guard<std::recursive_mutex> g(L->pool.mu);
        L->pool.arena = (char *)c->scratch;
        L->pool.arena_size = ATP_NOALLOC_SCRATCH_BYTES;
        L->pool.arena_used = 0;
    }
    // the bins of a product stay on the context's stream (side streams would be created on first use)
    const uint32_t saved_flags = c->flags;
    c->flags |= ATP_OPT_SERIAL_BINS;
    atp_result *r = nullptr;
    atp_status st = eval_impl(c, L, types, n_types, rel_ids, cons, n_cons, plan, 1, &r, false);
    if (st == ATP_OK) {
        // eval_impl has synchronised the stream: the result is complete in the workspace
        *nnz = r->nnz;
        if (r->nnz > cap) {
            st = ATP_EINVAL;
        } else if (hipMemcpyAsync(row_ptr, r->rp_ptr(), 8 * (size_t)(r->rows + 1), hipMemcpyDeviceToDevice,
                                  L->stream) !=
                       hipSuccess ||
                   (r->nnz && hipMemcpyAsync(col, r->col_ptr(), 4 * (size_t)r->nnz, hipMemcpyDeviceToDevice,
                                             L->stream) != hipSuccess) ||
                   (r->nnz && hipMemcpyAsync(val, r->val_ptr(), 8 * (size_t)r->nnz, hipMemcpyDeviceToDevice,
                                             L->stream) != hipSuccess) ||
                   hipStreamSynchronize(L->stream) != hipSuccess) {
            (void)hipGetLastError();
            c->broken = true;
            st = ATP_EDEVICE;
        }
    }
    if (r) (void)atp_result_free(r);  // its arrays are workspace blocks: nothing is released
    c->flags = saved_flags;
    {
        std::lock_guard<std::recursive_mutex> g(L->pool.mu);
        L->pool.arena = nullptr;
        L->pool.arena_size = L->pool.arena_used = 0;
    }
    return st;
}

atp_status atp_result_csr(const atp_result *r, int64_t *n_rows, int64_t *n_cols, int64_t *nnz,
                          const int64_t **row_ptr, const int32_t **col, const int64_t **val) {
    if (!r) return ATP_EINVAL;
    if (n_rows) *n_rows = r->rows;
    if (n_cols) *n_cols = r->cols;
    if (nnz) *nnz = r->nnz;
    if (row_ptr) *row_ptr = (const int64_t *)r->rp_ptr();
    if (col) *col = (const int32_t *)r->col_ptr();
    if (val) *val = (const int64_t *)r->val_ptr();
    return ATP_OK;
}

atp_status atp_result_to_host(const atp_result *r, int64_t *row_ptr, int32_t *col, int64_t *val) {
    if (!r) return ATP_EINVAL;
    hipStream_t s = r->stream;
    if (row_ptr) HIPTRY(hipMemcpyAsync(row_ptr, r->rp_ptr(), 8 * (r->rows + 1), hipMemcpyDeviceToHost, s));
    if (col && r->nnz) HIPTRY(hipMemcpyAsync(col, r->col_ptr(), 4 * r->nnz, hipMemcpyDeviceToHost, s));
    if (val && r->nnz) HIPTRY(hipMemcpyAsync(val, r->val_ptr(), 8 * r->nnz, hipMemcpyDeviceToHost, s));
    HIPTRY(hipStreamSynchronize(s));
    return ATP_OK;
}

atp_status atp_result_stats(const atp_result *r, atp_eval_stats *stats, char *plan, size_t plan_cap) {
    if (!r) return ATP_EINVAL;
    if (stats) *stats = r->stats;
    if (plan && plan_cap) {
        std::snprintf(plan, plan_cap, "%s", r->plan.c_str());
    }
    return ATP_OK;
}

atp_status atp_result_free(atp_result *r) {
    if (!r) return ATP_EINVAL;
    {
        std::lock_guard<std::mutex> g(r->ctx->results_mu);
        r->ctx->results.erase(r);
    }
    delete r;
    return ATP_OK;
}

atp_status atp_plan_chain(int32_t n_mats, const int64_t *dims, const int64_t *nnz, double alpha, double beta,
                          double gamma, int32_t dense, char *plan, size_t plan_cap, double *cost) {
    if (n_mats < 1 || !dims || (!dense && !nnz)) return ATP_EINVAL;
    const int p = n_mats;
    if (dense) {
        // standard product of Sec. 3.1: m*k*l operations per multiplication
        std::vector<std::vector<double>> C(p, std::vector<double>(p, 0.0));
        std::vector<std::vector<int>> S(p, std::vector<int>(p, -1));
        for (int len = 2; len <= p; ++len)
            for (int i = 0; i + len - 1 < p; ++i) {
                int j = i + len - 1;
                C[i][j] = 1e300;
                for (int k = i; k < j; ++k) {
                    double v = C[i][k] + C[k + 1][j] + (double)dims[i] * (double)dims[k + 1] * (double)dims[j + 1];
                    if (v < C[i][j]) {
                        C[i][j] = v;
                        S[i][j] = k;
                    }
                }
            }
        std::function<std::string(int, int)> str = [&](int i, int j) -> std::string {
            if (i == j) return std::to_string(i);
            return "(" + str(i, S[i][j]) + "," + str(S[i][j] + 1, j) + ")";
        };
        std::string ps = str(0, p - 1);
        if (plan && plan_cap) std::snprintf(plan, plan_cap, "%s", ps.c_str());
        if (cost) *cost = C[0][p - 1];
        return ATP_OK;
    }
    std::vector<ChainStats> leaves(p);
    for (int i = 0; i < p; ++i) {
        if (dims[i] < 0 || dims[i + 1] < 0 || nnz[i] < 0) return ATP_EINVAL;
        leaves[i].dim_r = (double)dims[i];
        leaves[i].dim_c = (double)dims[i + 1];
        leaves[i].nnz = (double)nnz[i];
        leaves[i].rows = (double)dims[i];
        leaves[i].cols = (double)dims[i + 1];
    }
    CostCoeffs cc;
    cc.alpha = alpha;
    cc.beta = beta;
    cc.gamma = gamma;
    cc.delta = 0;
    PlanResult pr = plan_chain(leaves, {}, {}, {}, {}, Estimator::Uniform, cc);
    if (plan && plan_cap) std::snprintf(plan, plan_cap, "%s", pr.plan.c_str());
    if (cost) *cost = pr.cost;
    return ATP_OK;
}

atp_status atp_set_flags(atp_ctx *c, uint32_t flags) {
    if (!c) return ATP_EINVAL;
    c->flags = flags;
    return ATP_OK;
}

int32_t atp_kernel_times(atp_ctx *c, const char **names, double *ms, int64_t *launches, double *bytes, int32_t cap) {
    if (!c) return 0;
    c->main.timer.flush();
    std::map<std::string, int> keys;
    for (auto &kv : c->main.timer.acc) keys[kv.first] = 1;
    for (auto &kv : c->main.timer.bytes) keys[kv.first] = 1;
    int32_t n = 0;
    for (auto &kv : keys) {
        if (n >= cap) break;
        auto it = c->main.timer.acc.find(kv.first);
        auto ib = c->main.timer.bytes.find(kv.first);
        if (names) names[n] = kv.first == "" ? "" : (it != c->main.timer.acc.end() ? it->first.c_str() : ib->first.c_str());
        if (ms) ms[n] = it != c->main.timer.acc.end() ? it->second.first : 0.0;
        if (launches) launches[n] = it != c->main.timer.acc.end() ? it->second.second : 0;
        if (bytes) bytes[n] = ib != c->main.timer.bytes.end() ? ib->second : 0.0;
        ++n;
    }
    return n;
}

atp_status atp_set_profile_kernel(atp_ctx *c, const char *name) {
    if (!c) return ATP_EINVAL;
    c->main.timer.only = name ? name : "";
    for (auto &ln : c->lanes) ln->timer.only = c->main.timer.only;
    return ATP_OK;
}

void atp_kernel_times_reset(atp_ctx *c) {
    if (!c) return;
    c->main.timer.flush();
    c->main.timer.acc.clear();
    c->main.timer.bytes.clear();
}

int64_t atp_device_bytes(const atp_ctx *c) {
    if (!c) return 0;
    int64_t n = c->main.pool.held;
    for (auto &ln : c->lanes) n += ln->pool.held;
    return n;
}

atp_status atp_cache_configure(atp_ctx *c, int32_t policy, uint64_t budget_bytes) {
    if (!c || policy < ATP_CACHE_OFF || policy > ATP_CACHE_CBS2) return ATP_EINVAL;
    (void)hipStreamSynchronize(c->main.stream);
    CacheState &cs = c->cache;
    std::lock_guard<std::mutex> g(cs.mu);
    cs.payload.clear();
    cs.info.clear();
    cs.item_by_key.clear();
    cs.stats = atp_cache_stats{};
    cs.policy = policy;
    cs.budget = budget_bytes;
    cs.tree.reset(policy == ATP_CACHE_OFF ? nullptr : new OverlapTree());
    cs.pol.reset();
    if (policy != ATP_CACHE_OFF) {
        const Policy pol = policy == ATP_CACHE_OTREE ? Policy::Otree : policy == ATP_CACHE_PGDS ? Policy::Pgds
                                                                                                 : Policy::Lru;
        cs.pol.reset(new CachePolicy(pol, (double)budget_bytes));
        CacheState *csp = &cs;
        cs.pol->set_subtree_fn([csp](int64_t id) { return cache_subtree(*csp, id); });
    }
    return ATP_OK;
}

atp_status atp_cache_get_stats(const atp_ctx *c, atp_cache_stats *st) {
    if (!c || !st) return ATP_EINVAL;
    CacheState &cs = const_cast<atp_ctx *>(c)->cache;
    std::lock_guard<std::mutex> g(cs.mu);
    *st = cs.stats;
    st->items = cs.pol ? cs.pol->cached_count() : 0;
    st->bytes = cs.pol ? (int64_t)cs.pol->used() : 0;
    st->otree_nodes = cs.tree ? cs.tree->size() : 0;
    st->otree_leaves = cs.tree ? cs.tree->leaves() : 0;
    return ATP_OK;
}

// ---- tunables and the autotuner ----

static atp_tuning to_abi(const Tuning &t) {
    return atp_tuning{t.part_target, t.part_hash_cap, t.task_ops, t.bucket_pct, t.split_ops, t.bucket_chunk};
}

atp_status atp_get_tuning(const atp_ctx *c, atp_tuning *t) {
    if (!c || !t) return ATP_EINVAL;
    *t = to_abi(c->tune);
    return ATP_OK;
}

atp_status atp_set_tuning(atp_ctx *c, const atp_tuning *t) {
    if (!c || !t) return ATP_EINVAL;
    if (t->part_target < 1 || t->part_hash_cap < 0 || t->part_hash_cap > kRankCap || t->task_ops < 1 ||
        t->bucket_pct < 0 || t->split_ops < 1024 || t->bucket_chunk < 64)
        return ATP_EINVAL;
    c->tune.part_target = t->part_target;
    c->tune.part_hash_cap = t->part_hash_cap;
    c->tune.task_ops = t->task_ops;
    c->tune.bucket_pct = t->bucket_pct;
    c->tune.split_ops = t->split_ops;
    c->tune.bucket_chunk = t->bucket_chunk;
    return ATP_OK;
}

atp_status atp_autotune(atp_ctx *c, const atp_query *sample, int32_t n, int32_t rounds, atp_tuning *chosen,
                        double *ms_before, double *ms_after) {
    if (!c || n < 1 || !sample || rounds < 1) return ATP_EINVAL;
    if (c->server) return ATP_ESTATE;
    {
        std::lock_guard<std::mutex> g(c->cache.mu);
        if (c->cache.policy != ATP_CACHE_OFF) return ATP_ESTATE;
    }
    (void)hipSetDevice(c->device);
    const Tuning start = c->tune;
    // wall time of the sample (best of two), every query synchronised
    auto run = [&](double &ms) -> atp_status {
        ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            for (int32_t i = 0; i < n; ++i) {
                const atp_query &q = sample[i];
                atp_result *r = nullptr;
                atp_status st = eval_impl(c, &c->main, q.types, q.n_types, q.rel_ids, q.cons, q.n_cons, nullptr, 1, &r);
                if (st != ATP_OK) return st;
                atp_result_free(r);
            }
            ms = std::min(ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        return ATP_OK;
    };
    struct Knob {
        int64_t Tuning::*field;
        std::vector<int64_t> grid;
    };
    const std::vector<Knob> knobs = {
        {&Tuning::bucket_pct, {25, 50, 100, 200, 400, 800}},
        {&Tuning::part_target, {600, 1200, 2400, 3600}},
        {&Tuning::task_ops, {8192, 16384, 32768, 65536}},
        {&Tuning::split_ops, {16384, 65536, 262144}},
        {&Tuning::part_hash_cap, {1024, 2048, 4096}},
        {&Tuning::bucket_chunk, {1024, 2048, 4096, 8192}},
    };
    double best = 0;
    atp_status st = run(best);  // also warms the pool and the planner statistics
    if (st == ATP_OK) st = run(best);
    if (st != ATP_OK) {
        c->tune = start;
        return st;
    }
    const double before = best;
    for (int r = 0; r < rounds; ++r)
        for (const Knob &k : knobs) {
            const int64_t keep = c->tune.*(k.field);
            int64_t arg = keep;
            for (int64_t v : k.grid) {
                if (v == keep) continue;
                c->tune.*(k.field) = v;
                double ms = 0;
                if ((st = run(ms)) != ATP_OK) {
                    c->tune = start;
                    return st;
                }
                if (ms < best) {
                    best = ms;
                    arg = v;
                }
            }
            c->tune.*(k.field) = arg;
        }
    if (chosen) *chosen = to_abi(c->tune);
    if (ms_before) *ms_before = before;
    if (ms_after) *ms_after = best;
    return ATP_OK;
}

// ---- cost model (Eq. 2) ----

atp_status atp_cost_fit(int32_t n, const double *nnz_x, const double *n_op, const double *nnz_z, const double *t_ms,
                        double coeffs[4], double *r2) {
    if (n < 1 || !nnz_x || !n_op || !nnz_z || !t_ms || !coeffs) return ATP_EINVAL;
    CostCoeffs cc;
    const double q = fit_cost(std::vector<double>(nnz_x, nnz_x + n), std::vector<double>(n_op, n_op + n),
                              std::vector<double>(nnz_z, nnz_z + n), std::vector<double>(t_ms, t_ms + n), cc);
    coeffs[0] = cc.alpha;
    coeffs[1] = cc.beta;
    coeffs[2] = cc.gamma;
    coeffs[3] = cc.delta;
    if (r2) *r2 = q;
    return ATP_OK;
}

atp_status atp_get_cost_model(const atp_ctx *c, double coeffs[4]) {
    if (!c || !coeffs) return ATP_EINVAL;
    coeffs[0] = c->cost.alpha;
    coeffs[1] = c->cost.beta;
    coeffs[2] = c->cost.gamma;
    coeffs[3] = c->cost.delta;
    return ATP_OK;
}

atp_status atp_set_cost_model(atp_ctx *c, const double coeffs[4]) {
    if (!c || !coeffs) return ATP_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (!(coeffs[k] >= 0) || !std::isfinite(coeffs[k])) return ATP_EINVAL;
    if (coeffs[0] + coeffs[1] + coeffs[2] <= 0) return ATP_EINVAL;
    c->cost.alpha = coeffs[0];
    c->cost.beta = coeffs[1];
    c->cost.gamma = coeffs[2];
    c->cost.delta = coeffs[3];
    return ATP_OK;
}

atp_status atp_calibrate_cost_model(atp_ctx *c, const atp_query *sample, int32_t n, double coeffs[4], double *r2,
                                    int32_t *n_products) {
    if (!c || !sample || n < 1) return ATP_EINVAL;
    if (c->server) return ATP_ESTATE;
    (void)hipSetDevice(c->device);
    std::vector<std::array<double, 4>> recs;
    {
        std::lock_guard<std::mutex> g(c->stat_mu);
        c->cost_sink = &recs;
    }
    atp_status st = ATP_OK;
    for (int32_t i = 0; i < n && st == ATP_OK; ++i) {
        const atp_query &q = sample[i];
        atp_result *r = nullptr;
        st = eval_impl(c, &c->main, q.types, q.n_types, q.rel_ids, q.cons, q.n_cons, nullptr, 1, &r);
        if (st == ATP_OK) atp_result_free(r);
    }
    {
        std::lock_guard<std::mutex> g(c->stat_mu);
        c->cost_sink = nullptr;
    }
    if (st != ATP_OK) return st;
    if (recs.size() < 4) return ATP_EINVAL;  // too few multiplications to fit four coefficients
    std::vector<double> x(recs.size()), o(recs.size()), z(recs.size()), t(recs.size());
    for (size_t k = 0; k < recs.size(); ++k) {
        x[k] = recs[k][0];
        o[k] = recs[k][1];
        z[k] = recs[k][2];
        t[k] = recs[k][3];
    }
    CostCoeffs cc;
    const double q = fit_cost(x, o, z, t, cc);
    if (cc.alpha + cc.beta + cc.gamma <= 0) return ATP_ESTATE;  // the fit explains nothing: keep the model
    c->cost = cc;
    if (coeffs) {
        coeffs[0] = cc.alpha;
        coeffs[1] = cc.beta;
        coeffs[2] = cc.gamma;
        coeffs[3] = cc.delta;
    }
    if (r2) *r2 = q;
    if (n_products) *n_products = (int32_t)recs.size();
    return ATP_OK;
}

}  // extern "C"
