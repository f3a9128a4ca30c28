/*
 * atrapos.h -- C-ABI of the MI355X metapath query engine.
 *
 * The engine evaluates constrained metapath queries over a heterogeneous
 * information network (HIN) held in GPU memory and returns, for every pair of
 * end nodes connected by at least one instance of the metapath, the number of
 * instances (paper Sec. 2: Def. 1 HIN, Def. 2 metapath and instance, Def. 3
 * constrained metapath, Problem 1 MQE).  Evaluation is a chain of sparse
 * matrix products over the typed 0/1 adjacency matrices A_r, with each
 * constraint c_i applied as the 0/1 diagonal matrix M_{c_i} (Sec. 2, the
 * paragraph after Problem 1):
 *
 *      R = M_1 A_{r_1} M_2 A_{r_2} ... A_{r_{n-1}} M_n .
 *
 * The multiplication order is chosen by dynamic programming over estimated
 * sparse-product costs (Sec. 3.1 Eq. 1, Sec. 3.2 Eq. 2); the order never
 * changes the result (associativity, Sec. 3.1).
 *
 * Conventions shared by every call
 *   - Every call returns an atp_status; it never aborts the process.  On error
 *     no output handle is created and *out (where present) is set to NULL.
 *     A context stays usable after any error except ATP_EDEVICE.
 *   - Node ids are 0-based indices within their node type.
 *   - Sparse matrices are CSR: int64 row pointers (rows + 1 entries, first 0,
 *     non-decreasing), int32 column indices strictly ascending within a row.
 *   - Input arrays are host pointers unless a flag says otherwise; they are
 *     copied, the caller keeps ownership and may free them after the call.
 *   - All GPU work of a context is issued on the stream given in atp_options
 *     (NULL = the default stream) of the device given there.
 *   - A context is not internally locked: use one context per host thread.
 */
#ifndef ATRAPOS_H
#define ATRAPOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t atp_status;
enum {
    ATP_OK = 0,
    ATP_EINVAL = -1,     /* malformed argument: bad CSR, id out of range, bad kind, n_types < 2 */
    ATP_ENOMEM = -2,     /* a device allocation failed */
    ATP_EOVERFLOW = -3,  /* some path count of the result is >= 2^63 (does not fit int64) */
    ATP_ESCHEMA = -4,    /* metapath step without a (unique) relation between the two types */
    ATP_EDEVICE = -5,    /* HIP runtime error; the context must be destroyed */
    ATP_EBUDGET = -6,    /* the context's memory budget would be exceeded */
    ATP_ESTATE = -7      /* call not valid in the current state (e.g. no GPU present) */
};

typedef struct atp_ctx atp_ctx;
typedef struct atp_result atp_result;

/* flags of atp_options.flags */
#define ATP_OPT_PROFILE (1u << 0)   /* time every kernel launch with HIP events (atp_kernel_times) */
#define ATP_OPT_PLAN_EAC (1u << 1)  /* planner uses the paper's uniform E_ac estimate (Sec. 3.2) */
#define ATP_OPT_COUNT_BYTES (1u << 2) /* count algorithmic bytes per kernel (extra passes; not for timing) */
#define ATP_OPT_NO_RESTRICT (1u << 3) /* compute right sub-chains on all rows, not only on the rows the left
                                         operand reaches (same result; keeps sub-results start-independent) */
#define ATP_OPT_SERIAL_BINS (1u << 4) /* run a product's numeric bins one after another on the context's
                                         stream instead of beside each other on side streams (same result;
                                         uncontended per-kernel times) */

typedef struct {
    int device;                 /* HIP device ordinal */
    void *hip_stream;           /* hipStream_t to issue work on, or NULL for the default stream */
    /* optional device allocator; both NULL = the library's own caching pools, which keep
     * freed blocks for reuse, up to half the device's memory in all (mem_budget_bytes
     * bounds what each pool holds; a failed allocation releases every pool's free blocks) */
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *alloc_user;
    uint64_t mem_budget_bytes;  /* 0 = unlimited; otherwise allocations beyond it fail with ATP_EBUDGET */
    uint32_t flags;             /* ATP_OPT_* */
} atp_options;

/* Create a context on options->device (options may be NULL: device 0,
 * default stream, own pool).  ATP_ESTATE if no HIP device is present. */
atp_status atp_create(const atp_options *options, atp_ctx **out);
/* Release every device buffer, result handle and the context itself. */
atp_status atp_destroy(atp_ctx *ctx);

/* --- the network (Def. 1): node types, relations, properties -------------- */

/* Register a node type with `count` nodes (ids 0..count-1). */
atp_status atp_add_node_type(atp_ctx *ctx, const char *name, int64_t count, int32_t *type_id);

#define ATP_REL_DEVICE_PTRS (1u << 0)  /* row_ptr / col are device pointers (still copied) */
#define ATP_REL_ADD_REVERSE (1u << 1)  /* also register the transpose as relation dst -> src */

/* Register the 0/1 adjacency matrix A_r of an edge type from src_type to
 * dst_type (the adjacency-matrix definition after Def. 1) as CSR with
 * count(src_type) rows and count(dst_type) columns.  ATP_EINVAL on
 * non-monotone row_ptr, unsorted or duplicate columns, or ids out of range.
 * *rel_id receives the relation id; with ATP_REL_ADD_REVERSE the transpose
 * gets id *rel_id + 1. */
atp_status atp_add_relation(atp_ctx *ctx, int32_t src_type, int32_t dst_type,
                            const int64_t *row_ptr, const int32_t *col, int64_t nnz,
                            uint32_t flags, int32_t *rel_id);

enum { ATP_I16 = 1, ATP_I32 = 2, ATP_I64 = 3 };

/* Register a node property (Sec. 2, v.prop): one value per node of type_id,
 * of dtype ATP_I16 / ATP_I32 / ATP_I64, host pointer, copied. */
atp_status atp_add_property(atp_ctx *ctx, int32_t type_id, const char *name, int32_t dtype,
                            const void *values, int32_t *prop_id);

/* --- queries (Def. 3, Problem 1) ------------------------------------------ */

enum { ATP_C_RANGE = 1, ATP_C_IDSET = 2 };

/* One constraint c_i of a constrained metapath (Def. 3).  It restricts the
 * nodes allowed at metapath position `position` (0-based):
 *   ATP_C_RANGE: lo <= v.prop <= hi (inclusive) on property prop_id, which must
 *                belong to the node type at that position;
 *   ATP_C_IDSET: v is one of ids[0..n_ids) (host pointer, any order,
 *                duplicates allowed, each in range).
 * Several constraints at one position are ANDed. */
typedef struct {
    int32_t position;
    int32_t kind;
    int32_t prop_id;
    int64_t lo, hi;
    const int32_t *ids;
    int64_t n_ids;
} atp_constraint;

/* Evaluate the constrained metapath types[0] .. types[n_types-1] (node type
 * ids).  rel_ids (n_types-1 entries) names the relation of every step; NULL
 * means the unique relation registered from types[i] to types[i+1]
 * (ATP_ESCHEMA if there is none or more than one).  The result is the
 * count(types[0]) x count(types[n-1]) matrix R in canonical CSR: int64 row
 * pointers, int32 columns ascending per row, int64 counts >= 1, no stored
 * zeros; rows excluded by constraints are empty.  If any count is >= 2^63
 * the call returns ATP_EOVERFLOW and no result.  The result lives in device
 * memory owned by the library until atp_result_free. */
atp_status atp_eval(atp_ctx *ctx, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                    const atp_constraint *cons, int32_t n_cons, atp_result **out);

/* As atp_eval, with the multiplication order forced by `plan` instead of the
 * planner's choice.  `plan` parenthesises the relation indices 0..n_types-2
 * in order, e.g. "((0,1),(2,3))" or "(((0,1),2),3)"; NULL = planner.  The
 * result is identical for every plan.  ATP_EINVAL on a malformed plan. */
atp_status atp_eval_plan(atp_ctx *ctx, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                         const atp_constraint *cons, int32_t n_cons, const char *plan,
                         atp_result **out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): atp_eval /
 * atp_eval_plan (plan may be NULL) writing the result into caller-owned
 * device arrays, with every temporary of the evaluation taken from a static
 * device workspace of ATP_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on until the process ends.  The call allocates no device
 * memory and creates no stream: the masks, per-product arrays and slot
 * arrays of the whole query must fit the workspace together, and the cache
 * (if configured) is neither read nor updated.
 *   row_ptr  device, count(types[0]) + 1 int64
 *   col      device, cap int32;  val  device, cap int64  (NULL allowed when cap = 0)
 *   *nnz     the result's nonzero count (set whenever the evaluation finished)
 * The result is identical to atp_eval's.  Errors: ATP_EBUDGET when the query
 * needs more workspace than ATP_NOALLOC_SCRATCH_BYTES; ATP_EINVAL for bad
 * arguments or when the result has more than cap nonzeros (*nnz then tells
 * the size needed); otherwise as atp_eval.  The call returns after the
 * result is written (the context's stream is synchronised).  All calls on
 * one GPU share its workspace: calls that overlap in time on the same GPU
 * (from several contexts or threads) race and must not be made. */
#define ATP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
atp_status atp_eval_noalloc(atp_ctx *ctx, const int32_t *types, int32_t n_types, const int32_t *rel_ids,
                            const atp_constraint *cons, int32_t n_cons, const char *plan, int64_t *row_ptr,
                            int32_t *col, int64_t *val, int64_t cap, int64_t *nnz);

/* Shape and device arrays of a result.  Pointers stay valid until
 * atp_result_free; any output pointer argument may be NULL. */
atp_status atp_result_csr(const atp_result *res, int64_t *n_rows, int64_t *n_cols, int64_t *nnz,
                          const int64_t **row_ptr, const int32_t **col, const int64_t **val);

/* Copy a result to host arrays of n_rows+1, nnz and nnz entries (synchronous). */
atp_status atp_result_to_host(const atp_result *res, int64_t *row_ptr, int32_t *col, int64_t *val);

/* Per-query statistics: chosen plan (NUL-terminated, truncated to plan_cap),
 * multiplications performed, total products (N_op, Sec. 3.2) and nonzeros of
 * every intermediate and of the result. */
typedef struct {
    int32_t n_products;
    int64_t n_op_total;
    int64_t nnz_intermediate_total;
    int64_t nnz_result;
    int64_t slots_total;         /* sum of per-row upper bounds reserved */
} atp_eval_stats;
atp_status atp_result_stats(const atp_result *res, atp_eval_stats *stats, char *plan, size_t plan_cap);

atp_status atp_result_free(atp_result *res);

/* --- workload evaluation with an intermediate-result cache (Sec. 3.3-3.4) ---
 *
 * With a cache configured, every atp_eval / atp_eval_plan call is one query
 * of a metapath query workload (Problem 2, MQWE).  The query's type string is
 * inserted into the context's Overlap Tree (Sec. 3.3: a generalised suffix
 * tree of metapaths with per-node occurrence frequency and a constraints
 * index), the planner prices every sub-chain whose result is cached at zero
 * (Sec. 3.2, last paragraph), and after evaluation the cache insertion policy
 * tries to keep results in device memory:
 *   ATP_CACHE_OTREE  Atrapos-OTree: the whole query and the longest computed
 *                    sub-metapath that is an Overlap-Tree overlap (Sec. 3.4.1),
 *                    replaced by Algorithm 1 (PGDS utility f*c/s + L, with the
 *                    cost of cached entries in an evicted / inserted entry's
 *                    subtree reinstated / subtracted);
 *   ATP_CACHE_PGDS   same insertion, plain PGDS replacement;
 *   ATP_CACHE_LRU    same insertion, LRU replacement;
 *   ATP_CACHE_CBS1   LRU of final query results only (Sec. 4.1 baseline CBS1);
 *   ATP_CACHE_CBS2   LRU of every intermediate result (baseline CBS2).
 * Items larger than 80% of the budget are never cached (Sec. 4.1).  Only
 * full sub-metapath results are kept: a right sub-chain is restricted to the
 * rows its left neighbour reaches (and then not cached) unless its type string
 * already occurred in an earlier query (Overlap-Tree frequency >= 2), in which
 * case it is computed on all rows and becomes a cache candidate, provided the
 * planner's size estimate of it fits an item the cache admits.  A cached
 * sub-metapath that is the left operand of a restricted product multiplies
 * only the restricted rows.  A query that runs out of device memory (or over
 * the context's budget) with the cache's choices is evaluated once more with
 * a plan chosen without cached results and every right sub-chain restricted.
 * Results are identical with and without a cache. */
enum { ATP_CACHE_OFF = 0, ATP_CACHE_OTREE = 1, ATP_CACHE_PGDS = 2, ATP_CACHE_LRU = 3, ATP_CACHE_CBS1 = 4,
       ATP_CACHE_CBS2 = 5 };

/* Set the cache policy and its device-memory budget in bytes; drops every
 * cached result and resets the Overlap Tree and statistics. */
atp_status atp_cache_configure(atp_ctx *ctx, int32_t policy, uint64_t budget_bytes);

typedef struct {
    int64_t queries;          /* queries evaluated since configuration */
    int64_t whole_hits;       /* queries answered entirely from the cache */
    int64_t sub_hits;         /* cached sub-chain results used by plans */
    int64_t insert_attempts;
    int64_t inserts;
    int64_t evictions;
    int64_t items;            /* results currently cached */
    int64_t bytes;            /* device bytes they hold */
    int64_t otree_nodes;      /* Overlap Tree nodes (root included) */
    int64_t otree_leaves;
} atp_cache_stats;
atp_status atp_cache_get_stats(const atp_ctx *ctx, atp_cache_stats *stats);

/* --- batches and serving (Problem 2, MQWE: a workload of metapath queries) --
 *
 * Both forms leave the arithmetic unchanged: every query's result is
 * bit-identical to its own atp_eval.  Queries are executed on lanes: a lane
 * is a HIP stream with its own memory pool, driven by its own host thread, so
 * the kernels of queries on different lanes overlap on the device.  The
 * context's cache (if configured) is shared by all lanes.
 *
 * Fusion: queries whose metapath, relations and constraints are the same
 * except for a single id-set constraint on the first position are evaluated
 * as ONE chain over the union of their start sets (every SpGEMM launch of the
 * chain serves all of them: R[u,:] depends only on u and the rest of the
 * chain, Def. 2-3); each query's rows are then copied out on the device.  A
 * fused chain that fails (int64 overflow in another member's rows, memory)
 * is retried one query at a time, so each query gets its own status.
 *
 * Memory admission: while lanes run, the slot arrays of each multiplication
 * (12 bytes per unit of the symbolic per-row upper bound, Sec. 3.2's N_op
 * bounded by the output width) are reserved against mem_budget_bytes before
 * they are allocated; a lane whose reservation does not fit waits until
 * other lanes release theirs (a reservation that exceeds the budget alone
 * proceeds when no other is held). */
typedef struct {
    const int32_t *types;              /* n_types node-type ids (a metapath, Def. 2) */
    int32_t n_types;
    const int32_t *rel_ids;            /* n_types-1 relation ids, or NULL (as in atp_eval) */
    const atp_constraint *cons;        /* as in atp_eval */
    int32_t n_cons;
} atp_query;

/* Evaluate n queries on `lanes` lanes (1..16) with at most max_batch queries
 * per fused chain (1 disables fusion).  out[i] / status[i] receive query i's
 * result handle (NULL on error) and status.  Returns ATP_OK when every query
 * was attempted (see status[]), ATP_EINVAL for bad arguments, ATP_ESTATE while
 * a server runs on the context.  The input arrays are read during the call. */
atp_status atp_eval_batch(atp_ctx *ctx, const atp_query *queries, int32_t n, int32_t lanes, int32_t max_batch,
                          uint64_t mem_budget_bytes, atp_result **out, atp_status *status);

/* Serving loop: a request queue drained by `lanes` worker lanes.  A free lane
 * takes the oldest queued request together with up to max_batch-1 queued
 * requests it can fuse with (continuous batching: requests that arrive while
 * others run join the next batch).  atp_submit copies the query and returns
 * at once; atp_poll hands out finished requests in completion order. */
typedef struct {
    int32_t lanes;                     /* 1..16 */
    int32_t max_batch;                 /* >= 1 */
    uint64_t mem_budget_bytes;         /* slot-array admission budget, 0 = none */
} atp_server_options;

typedef struct {
    uint64_t tag;                      /* the caller's tag from atp_submit */
    atp_status status;
    atp_result *result;                /* owned by the caller (atp_result_free); NULL on error */
    double t_submit, t_start, t_done;  /* seconds on a monotonic clock since atp_server_start */
    int32_t batch_size;                /* queries in the fused chain that served it */
    int32_t lane;
} atp_completion;

/* ATP_ESTATE if a server already runs on the context. */
atp_status atp_server_start(atp_ctx *ctx, const atp_server_options *opts);
/* Copy the query into the queue.  ATP_EINVAL for malformed arguments (checked
 * as atp_eval does), ATP_ESTATE if no server runs. */
atp_status atp_submit(atp_ctx *ctx, const atp_query *query, uint64_t tag);
/* Move up to max finished requests into out, waiting up to wait_ms
 * milliseconds for the first one (0 = do not wait).  Returns how many were
 * written, or a negative status. */
int32_t atp_poll(atp_ctx *ctx, atp_completion *out, int32_t max, int32_t wait_ms);
/* Requests queued or running (not yet polled-ready). */
int32_t atp_server_pending(atp_ctx *ctx);
/* Finish every queued request, stop the workers; completions not yet polled
 * are freed.  ATP_ESTATE if no server runs. */
atp_status atp_server_stop(atp_ctx *ctx);

/* --- kernel tunables and the autotuner ---------------------------------------
 *
 * Thresholds of the row binning and the numeric kernels.  They change which
 * kernel handles a row and how its work is split, never a result.
 *   part_target    expected products per part of a sparse row spanning several
 *                  column tiles (parts group consecutive tiles), >= 1
 *   part_hash_cap  a part with at most this many products is accumulated by
 *                  column rank (a presence bitmap over its columns, then one
 *                  value per present column) instead of in dense tiles, 0..4096
 *   task_ops       target products per dense task, >= 1
 *   bucket_pct     a row with more than 512 left entries whose entries x column
 *                  tiles x 100 exceed bucket_pct x its products is bucketed by
 *                  column tile (products materialised once) instead of searched
 *                  per tile, >= 0
 *   split_ops      products per (row, tile) beyond which a dense row's left
 *                  entries are split over several workgroups, >= 1024
 *   bucket_chunk   left entries per work item of a bucketed row, >= 64 */
typedef struct {
    int64_t part_target;
    int64_t part_hash_cap;
    int64_t task_ops;
    int64_t bucket_pct;
    int64_t split_ops;
    int64_t bucket_chunk;
} atp_tuning;
atp_status atp_get_tuning(const atp_ctx *ctx, atp_tuning *t);
/* Between queries (not while a server or batch runs).  ATP_EINVAL if a value
 * is out of its range. */
atp_status atp_set_tuning(atp_ctx *ctx, const atp_tuning *t);

/* Pick the tunables for a workload: coordinate descent over a fixed grid of
 * each tunable (bucket_pct, part_target, task_ops, split_ops, part_hash_cap),
 * `rounds` passes, timing the n sample queries end to end on the context's
 * stream (best of two runs per setting).  The fastest setting found is kept
 * in the context and written to *chosen; *ms_before / *ms_after receive the
 * sample's time with the starting and the chosen setting (either may be
 * NULL).  ATP_ESTATE while a cache is configured or a server runs (cached
 * results would hide the kernels).  A query that fails stops the search with
 * its status, the starting setting restored. */
atp_status atp_autotune(atp_ctx *ctx, const atp_query *sample, int32_t n, int32_t rounds, atp_tuning *chosen,
                        double *ms_before, double *ms_after);

/* --- Overlap Tree and cache policy as standalone host objects (no GPU) ---- */

typedef struct atp_otree atp_otree;
atp_status atp_otree_create(atp_otree **out);
atp_status atp_otree_destroy(atp_otree *t);
/* insert a metapath given as n >= 1 non-negative symbols (and all its suffixes) */
atp_status atp_otree_insert(atp_otree *t, const int32_t *symbols, int32_t n);
/* occurrences of symbols[0..n) as a substring of the inserted metapaths */
atp_status atp_otree_frequency(const atp_otree *t, const int32_t *symbols, int32_t n, int64_t *f);
/* node count (root included), leaves, sum of inserted lengths (lambda),
 * internal nodes below the root with fewer than two children, and leaves with f != 1 */
atp_status atp_otree_shape(const atp_otree *t, int64_t *nodes, int64_t *leaves, int64_t *lambda,
                           int64_t *thin_internal, int64_t *leaves_f_not_1);

/* Replay n_req requests of items 0..n_items-1 (size, cost; parent[i] is the
 * item whose Overlap-Tree subtree holds item i, or -1) through a policy
 * (ATP_CACHE_OTREE / PGDS / LRU) with the given budget.  hit[r] = item was
 * cached before request r; cached_after[r] = it is cached after it;
 * final_cached[i] = item i is cached at the end. */
atp_status atp_cache_simulate(int32_t policy, double budget, int32_t n_items, const double *size,
                              const double *cost, const int32_t *parent, int32_t n_req, const int32_t *req,
                              int32_t *hit, int32_t *cached_after, int32_t *final_cached);

/* --- planner (host only; usable without a GPU) ----------------------------- */

/* Dynamic-programming chain order (Sec. 3.1, Eq. 1) for p = n_mats matrices
 * with dims[0..p] (matrix i is dims[i] x dims[i+1]) and per-matrix nonzeros
 * nnz[0..p) under the sparse cost of Eq. 2 with the uniform E_ac density
 * estimate (Sec. 3.2): cost = alpha*nnz(X) + beta*N_op + gamma*nnz(Z),
 * N_op = nnz(X)*nnz(Y)/k for X (m x k), Y (k x l), and
 * rho_Z = 1 - (1 - rho_X*rho_Y)^k.  With dense != 0 the cost of X*Y is
 * m*k*l instead (the standard product of Sec. 3.1).  Ties go to the smallest
 * split.  Writes the parenthesisation (same syntax as atp_eval_plan) and
 * the optimal total cost. */
atp_status atp_plan_chain(int32_t n_mats, const int64_t *dims, const int64_t *nnz, double alpha,
                          double beta, double gamma, int32_t dense, char *plan, size_t plan_cap,
                          double *cost);

/* --- cost model of the planner (Eq. 2) -------------------------------------
 *
 * Eq. 2 prices one multiplication Z = X*Y as alpha*nnz(X) + beta*N_op +
 * gamma*nnz(Z); the paper fits alpha, beta, gamma by least squares on measured
 * multiplications.  The engine adds delta per multiplication (launches and
 * host synchronisation).  coeffs = {alpha, beta, gamma, delta}, all >= 0.
 * Coefficients change plans only, never results. */

/* Host-only least squares over n measured multiplications (t_ms ~ alpha *
 * nnz_x + beta * n_op + gamma * nnz_z + delta); a coefficient that would be
 * negative is fixed at 0 and the others refit.  *r2 = coefficient of
 * determination (may be NULL). */
atp_status atp_cost_fit(int32_t n, const double *nnz_x, const double *n_op, const double *nnz_z, const double *t_ms,
                        double coeffs[4], double *r2);
atp_status atp_get_cost_model(const atp_ctx *ctx, double coeffs[4]);
/* ATP_EINVAL for a negative or non-finite value, or alpha = beta = gamma = 0. */
atp_status atp_set_cost_model(atp_ctx *ctx, const double coeffs[4]);
/* Evaluate the sample queries once, timing every multiplication with HIP
 * events on the context's stream (nnz(X) of a base relation is the planner's
 * masked estimate), fit the coefficients and install them.  ATP_EINVAL with
 * fewer than four multiplications in the sample; ATP_ESTATE while a server
 * runs or when the fit leaves alpha = beta = gamma = 0 (the model is kept). */
atp_status atp_calibrate_cost_model(atp_ctx *ctx, const atp_query *sample, int32_t n, double coeffs[4], double *r2,
                                    int32_t *n_products);

/* --- diagnostics ------------------------------------------------------------ */

/* Replace the context's ATP_OPT_* flags (between queries). */
atp_status atp_set_flags(atp_ctx *ctx, uint32_t flags);

/* Per kernel name since the last reset: accumulated device time in ms and
 * launch count (ATP_OPT_PROFILE, HIP events on the context's stream), and
 * algorithmic bytes (ATP_OPT_COUNT_BYTES): operands read once and results
 * written once, i.e. for a numeric launch 16 B per row pointer pair,
 * (4 + 8 if valued) B per left-operand entry, 16 + (4 + 8 if valued) B per
 * distinct right-operand row and its entries, 12 B per result entry.  Any
 * output array may be NULL; returns the number of kernels written (<= cap). */
int32_t atp_kernel_times(atp_ctx *ctx, const char **names, double *ms, int64_t *launches, double *bytes,
                         int32_t cap);
void atp_kernel_times_reset(atp_ctx *ctx);

/* Restrict ATP_OPT_PROFILE to the launches of one kernel name (as reported by
 * atp_kernel_times, e.g. "dense"); NULL or "" times every launch again.  A
 * timed launch records two HIP events, so timing one kernel leaves the rest
 * of a query's launch sequence as it runs unprofiled.  The name is copied.
 * Returns ATP_EINVAL for a NULL context. */
atp_status atp_set_profile_kernel(atp_ctx *ctx, const char *name);

/* Bytes of device memory currently held by the context (pool included). */
int64_t atp_device_bytes(const atp_ctx *ctx);

const char *atp_status_str(atp_status status);

#ifdef __cplusplus
}
#endif
#endif /* ATRAPOS_H */
