// Internal declarations shared by the host engine and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace atp {

constexpr uint64_t kSat = 0x8000000000000000ull;  // saturated count (true value >= 2^63)
constexpr int32_t kEmptyKey = 0x7FFFFFFF;          // empty hash slot; sorts after every column id

// Dense LDS tile: TW columns of uint64 accumulators plus presence/saturation bitmaps.
constexpr int kTileShift = 13;
constexpr int kTileW = 1 << kTileShift;
constexpr int kDenseThreads = 512;
constexpr int kCursorCap = 512;     // X entries whose cursors fit in LDS (multi-tile chunks)
constexpr int64_t kTaskOps = 8192;  // target products per dense task
constexpr int64_t kPartTarget = 3600;  // expected products per part of a sparse long row
constexpr int kRankCap = 4096;         // most products of a part accumulated by column rank
constexpr int64_t kPartHashCap = kRankCap;  // default part_hash_cap: parts of at most this many products go by rank
constexpr int kPartMaxTiles = 16;      // ... if it spans at most this many tiles (its presence bitmap)
constexpr int64_t kSplitOps = 16384;   // products per (row, tile) beyond which the row's entries are split
constexpr int kMaxSplit = 64;
constexpr int64_t kPartGroup = 4;      // most sparse parts handed out to one dense task
constexpr int kQueues = 8;             // task counters of the dense kernel
constexpr int64_t kAlignTiles = 16;    // products with this many column tiles align dense tasks to the counters
constexpr int kMaxBucketTiles = 4096;  // column tiles a bucketed row may span
constexpr int kBucketThreads = 512;

// Hash bins: table sizes (slots); wave-level tables for small rows, block-level otherwise.
enum Bin : int32_t {
    BIN_NONE = 0,
    BIN_W64, BIN_W128, BIN_W256, BIN_W512,         // one wavefront per row
    BIN_B1024, BIN_B2048, BIN_B4096, BIN_B8192,    // one workgroup per row
    BIN_DENSE,                                     // dense LDS tiles over column ranges
    BIN_BUCKET,                                    // products bucketed by column tile, then dense tiles
    BIN_COUNT
};

// One operand of Z = X * Y.  Leaves are base relations (no values) and carry
// the masks of their two metapath positions; products carry int64 values and
// are already masked.
struct Operand {
    const int64_t *rp = nullptr;
    const int32_t *col = nullptr;
    const uint64_t *val = nullptr;   // nullptr: every stored entry is 1
    const uint32_t *rmask = nullptr; // row mask bits (leaf X only)
    const uint32_t *cmask = nullptr; // column mask bits (leaf only)
    int64_t rows = 0, cols = 0, nnz = 0;
    const uint64_t *vmax = nullptr;  // device: no stored value exceeds *vmax (nullptr: no bound known)
};

// Runtime tunables of the binning and numeric kernels (defaults above).
struct Tuning {
    int64_t part_target = kPartTarget;
    int64_t part_hash_cap = kPartHashCap;
    int64_t task_ops = kTaskOps;
    int64_t bucket_pct = 400;  // bucket a row when left entries x tiles x 100 > pct x products
    int64_t split_ops = kSplitOps;
    int64_t wg_slots = 512;    // resident dense workgroups (2 per compute unit)
    int64_t bucket_chunk = 8192;  // left-operand entries per bucketing work item
};

// Per-step device scratch header read back by the host (one small copy).
struct StepHeader {
    int64_t slots_total;      // sum of per-row upper bounds
    int64_t segs_total;       // number of output segments
    int64_t n_op_total;       // products
    int64_t bin_count[BIN_COUNT];
    int64_t dense_tasks;      // dense-bin tasks
    int64_t bucket_chunks;    // bucket-bin work items
    int64_t n_split;          // dense rows whose entries are split over several workgroups
    int64_t bucket_products;  // products buffered by the bucket bin
    int64_t nnz_total;        // result nonzeros (after numeric)
    int64_t n_active;         // non-empty result rows
    uint64_t vmax;            // largest result value (the compaction copy's maximum)
    int32_t saturated;        // some emitted value is saturated
    int32_t fault;            // an LDS hash table overflowed its probe bound (a sizing error): result invalid
};

// ---- launchers (kernels.hip) -------------------------------------------------

// Post n int64 values from device memory to mapped pinned host memory, then
// set *flag = seq (system-scope release): the host polls the flag instead of
// synchronising the stream.  One workgroup.
void launch_post(const int64_t *src, int64_t n, int64_t *dst_host, uint64_t *flag_host, uint64_t seq,
                 hipStream_t s);
struct KernelTimer;  // host-side profiler hook (engine.cpp)

void timer_begin(KernelTimer *t, const char *name, hipStream_t s);
void timer_end(KernelTimer *t, hipStream_t s);

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s, KernelTimer *t);
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s, KernelTimer *t);

// exclusive scan of n int64 values; out has n+1 entries (out[n] = total,
// also stored to *total when given); tmp must hold scan_tmp_elems(n) int64.
int64_t scan_tmp_elems(int64_t n);
void launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s,
                     KernelTimer *t, int64_t *total = nullptr);
// up to kMaxScanJobs scans in one launch sequence; tmp holds
// scan_multi_tmp_elems(jobs) int64.  When every array has at most
// kSmallScanTiles * 2048 elements the sequence is a single launch.
constexpr int kMaxScanJobs = 8;
constexpr int64_t kSmallScanTiles = 8;
// up to this many tiles, the tile sums are added up by each tile (two launches instead of three)
constexpr int64_t kScanFoldTiles = 1024;
struct ScanJob {
    const int64_t *in;
    int64_t *out;    // n + 1 entries
    int64_t *total;  // optional
    int64_t n;
};
int64_t scan_multi_tmp_elems(const ScanJob *jobs, int n_jobs);
void launch_scan_multi(const ScanJob *jobs, int n_jobs, int64_t *tmp, hipStream_t s, KernelTimer *t);
// up to kMaxFillJobs int64 fills in one launch
constexpr int kMaxFillJobs = 4;
struct FillJob {
    int64_t *p;
    int64_t n;
    int64_t v;
};
void launch_fill_multi(const FillJob *jobs, int n_jobs, hipStream_t s, KernelTimer *t);

// masks
void launch_mask_range(const void *prop, int32_t dtype, int64_t n, int64_t lo, int64_t hi,
                       uint32_t *bits, int and_mode, hipStream_t s, KernelTimer *t);
void launch_mask_ids(const int32_t *ids, int64_t n_ids, uint32_t *bits, hipStream_t s, KernelTimer *t);
void launch_mask_and(uint32_t *dst, const uint32_t *src, int64_t words, hipStream_t s, KernelTimer *t);
void launch_popcount(const uint32_t *bits, int64_t words, int64_t *out, hipStream_t s, KernelTimer *t);

// symbolic: per candidate row the products, the upper bound, bin, segments
struct SymbolicArgs {
    Operand X, Y;
    const int32_t *cand;      // candidate rows (ascending) or nullptr = all rows 0..n_cand-1
    int64_t n_cand;
    int64_t ycols_eff;        // columns that can appear (mask popcount or Y cols)
    int64_t *nop;             // [n_cand]
    int64_t *ub;              // [n_cand]
    int64_t *nseg;            // [n_cand]
    int32_t *bin;             // [n_cand]
    int64_t *long_len;        // [n_cand] chunks of rows left to the long-row pass
    int64_t *long_off;        // [n_cand + 1] their exclusive scan
    int64_t *scan_tmp;        // scan_tmp_elems(n_cand)
    int32_t *bin_lists;       // [BIN_COUNT * n_cand]
    int64_t *dense_chunks;    // [n_cand] tasks per dense candidate (indexed by dense list position)
    int64_t *dense_split;     // [n_cand] per dense candidate: split slot * 256 + split factor (> 1), or
                              // tiles per part << 16 | parts per task << 8 | 1
    int64_t *bucket_chunks;   // [n_cand] work items per bucket candidate (indexed by bucket list position)
    int64_t *bucket_nop;      // [n_cand] products per bucket candidate (indexed by bucket list position)
    StepHeader *hdr;
    Tuning tune;
};
void launch_symbolic(const SymbolicArgs &a, hipStream_t s, KernelTimer *t);
void launch_bin_rows(const SymbolicArgs &a, hipStream_t s, KernelTimer *t);

// numeric
struct NumericArgs {
    Operand X, Y;
    const int32_t *cand;       // nullptr = identity
    const int64_t *nop;        // [n_cand]
    const int64_t *slot_off;   // [n_cand + 1]
    const int64_t *seg_base;   // [n_cand + 1]
    int64_t *row_cursor;       // [n_cand] (dense rows: reserved slots so far)
    int32_t *slot_col;         // [slots_total]
    uint64_t *slot_val;        // [slots_total]
    int64_t *seg_cnt;          // [segs_total]
    int64_t *seg_src;          // [segs_total]
    int64_t *row_nnz;          // [X.rows] (zeroed)
    StepHeader *hdr;
    int64_t ycols;
    const int64_t *dense_split;        // [n_dense] as SymbolicArgs::dense_split
    unsigned long long *split_acc;     // [n_split * ntiles * kTileW] (zeroed)
    uint32_t *split_sat;               // [n_split * ntiles * kTileW / 32] (zeroed)
    int32_t *split_done;               // [n_split * ntiles] (zeroed)
    const int32_t *ytile;              // [Y.rows * (ntiles + 1)] tile index of Y, or nullptr
    int64_t *dense_queue;              // [kQueues] task counters of the dense kernel (zeroed)
    Tuning tune;
};
void launch_numeric_hash(int32_t bin, const int32_t *list, int64_t n, const NumericArgs &a, hipStream_t s,
                         KernelTimer *t);
void launch_numeric_dense(const int32_t *list, int64_t n_list, const int64_t *task_base, int64_t n_tasks,
                          const NumericArgs &a, hipStream_t s, KernelTimer *t);

// per-row column-tile offsets of Y (the dense kernel's segment bounds)
void launch_tile_index(const Operand &Y, int64_t ntiles, int32_t *ytile, hipStream_t s, KernelTimer *t);
// chunk_hist: [n_chunks * ntiles] int64 scratch (per-chunk tile counts, then bucket bases), or
// nullptr (the scatter pass then counts its chunk's products again); parts: int64 scratch of
// bucket_parts_elems(n_list) entries (accumulation parts per row, their scan and its temporaries)
void launch_numeric_bucket(const int32_t *list, int64_t n_list, const int64_t *chunk_base, int64_t n_chunks,
                           const int64_t *prod_base, int64_t ntiles, int64_t *tile_cnt, int64_t *tile_off,
                           int32_t *prod_col, uint64_t *prod_val, int64_t *chunk_hist, int64_t *parts,
                           const NumericArgs &a, hipStream_t s, KernelTimer *t);
inline int64_t bucket_parts_elems(int64_t n_list) { return 2 * n_list + 1 + scan_tmp_elems(n_list); }
constexpr int64_t kChunkHistCap = (int64_t)64 << 20;  // per-chunk tile counts kept up to this many entries

// compaction
void launch_copy_segments(const int64_t *seg_cnt, const int64_t *seg_src, const int64_t *seg_dst, int64_t n_segs,
                          const int32_t *slot_col, const uint64_t *slot_val, int32_t *col, uint64_t *val,
                          uint64_t *vmax, hipStream_t s, KernelTimer *t);
void launch_active_flags(const int32_t *cand, int64_t n_cand, const int64_t *row_nnz, int64_t *flags,
                         hipStream_t s, KernelTimer *t);
// the non-empty candidate rows in order; with partition the empty ones
// follow, so that `active` holds n_cand rows
void launch_active_scatter(const int32_t *cand, int64_t n_cand, const int64_t *flags_scan, int32_t *active,
                           bool partition, hipStream_t s, KernelTimer *t);
// dst[0] += h->nnz_total, dst[1] |= h->fault on the stream (a deferred product's totals)
void launch_accum_step(const StepHeader *h, int64_t *dst, hipStream_t s);

// row restriction: columns used by a left operand -> bitmap -> ascending list
// nnz_dev (optional) holds the true entry count on the device, nnz its upper bound
void launch_cols_to_bits(const int32_t *col, int64_t nnz, const int64_t *nnz_dev, uint32_t *bits, hipStream_t s,
                         KernelTimer *t);
// len/off hold n_cand (+1) int64, tmp scan_tmp_elems(n_cand)
void launch_leaf_cols_to_bits(const Operand &X, const int32_t *cand, int64_t n_cand, int64_t *len, int64_t *off,
                              int64_t *tmp, uint32_t *bits, hipStream_t s, KernelTimer *t);
// per-word popcounts (cnt[words]) and their exclusive scan (scan[words+1], tmp scan_tmp_elems(words))
void launch_bits_count(const uint32_t *bits, int64_t words, int64_t *cnt, int64_t *scan, int64_t *tmp, hipStream_t s,
                       KernelTimer *t);
// ascending list of set bits (list holds scan[words] entries)
void launch_bits_scatter(const uint32_t *bits, int64_t words, const int64_t *scan, int32_t *list, hipStream_t s,
                         KernelTimer *t);

// rows ids (ascending, unique) of a CSR R into a CSR of the same shape:
// cnt[rows] (zeroed) receives their lengths; after its exclusive scan orp,
// the copy fills ocol/oval
void launch_gather_count(const int64_t *rrp, const int32_t *ids, int64_t n, int64_t *cnt, hipStream_t s,
                         KernelTimer *t);
void launch_gather_copy(const int64_t *rrp, const int32_t *rcol, const uint64_t *rval, const int32_t *ids, int64_t n,
                        const int64_t *orp, int32_t *ocol, uint64_t *oval, hipStream_t s, KernelTimer *t);

// algorithmic-byte accounting: acc[5] = rows, left entries, result entries,
// distinct right rows, their entries
void launch_bin_stats(const int32_t *list, int64_t n, const Operand &X, const int32_t *cand, const int64_t *row_nnz,
                      uint32_t *ymark, int64_t *acc, hipStream_t s);
void launch_mark_bytes(const uint32_t *ymark, const int64_t *yrp, int64_t yrows, int64_t *acc, hipStream_t s);

}  // namespace atp
