/*
 * CPU oracle for constrained metapath query evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code with
 * the GPU library and must never serve a product call.
 *
 * What it computes (paper Sec. 2, Problem 1 "MQE", and the constrained
 * adjacency matrices defined right after it): for a metapath o_1 ... o_n over
 * relations r_1 ... r_{n-1} with per-position 0/1 masks M_1 ... M_n,
 *
 *      R = M_1 A_{r_1} M_2 A_{r_2} ... A_{r_{n-1}} M_n ,
 *
 * where R[u,v] is the number of metapath instances from u to v.  The result is
 * every pair with R[u,v] >= 1 together with its count.
 *
 * Method: fixed left-to-right row-by-row evaluation (Gustavson's row-wise
 * sparse product applied to one row vector at a time).  For a start node u
 * that passes M_1 the row vector e_u is pushed through every relation in
 * metapath order; each step scatters into a dense accumulator of the next
 * type's width and gathers the touched entries.  Counts are accumulated in
 * signed 128-bit integers, so a final count of 2^63 or more is detected
 * exactly (status ORC_OVERFLOW); values are then reported saturated at 2^63.
 *
 * orc_spgemm is the plain row-wise product Z = X * Y of two CSR matrices with
 * optional int64 values (absent values mean every stored entry is 1).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

enum { ORC_OK = 0, ORC_OVERFLOW = 1, ORC_RANGE = 2, ORC_NOMEM = 3 };

#define SAT63 ((uint64_t)1 << 63)

typedef struct {
    int64_t n_rows;
    int64_t *row_len;  /* [n_rows] */
    int64_t nnz;
    int32_t *col;      /* [nnz], ascending within a row */
    uint64_t *val;     /* [nnz], min(count, 2^63) */
    int32_t status;
} orc_result;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static uint64_t sat_u64(i128 v) { return v >= (i128)SAT63 ? SAT63 : (uint64_t)v; }

/* One row of the chain.  Buffers are per thread. */
typedef struct {
    i128 *acc;        /* dense accumulator, width max_dim, kept all-zero between uses */
    int32_t *cur_idx, *nxt_idx;
    i128 *cur_val, *nxt_val;
} worker;

static int chain_row(int n_types, const int64_t *const *row_ptr, const int32_t *const *col,
                     const uint8_t *const *mask, int64_t u, worker *w,
                     int64_t *out_len, int32_t **out_col, uint64_t **out_val, int *overflow) {
    *out_len = 0; *out_col = NULL; *out_val = NULL;
    if (mask[0] && !mask[0][u]) return ORC_OK;
    int64_t n_cur = 1;
    w->cur_idx[0] = (int32_t)u;
    w->cur_val[0] = 1;
    for (int i = 0; i + 1 < n_types; ++i) {
        const int64_t *rp = row_ptr[i];
        const int32_t *cl = col[i];
        const uint8_t *mk = mask[i + 1];
        int64_t n_nxt = 0;
        for (int64_t t = 0; t < n_cur; ++t) {
            int32_t k = w->cur_idx[t];
            i128 x = w->cur_val[t];
            for (int64_t e = rp[k]; e < rp[k + 1]; ++e) {
                int32_t j = cl[e];
                if (mk && !mk[j]) continue;
                if (w->acc[j] == 0) w->nxt_idx[n_nxt++] = j;
                i128 s;
                if (__builtin_add_overflow(w->acc[j], x, &s)) return ORC_RANGE;
                w->acc[j] = s;
            }
        }
        for (int64_t t = 0; t < n_nxt; ++t) {
            int32_t j = w->nxt_idx[t];
            w->nxt_val[t] = w->acc[j];
            w->acc[j] = 0;
        }
        int32_t *ti = w->cur_idx; w->cur_idx = w->nxt_idx; w->nxt_idx = ti;
        i128 *tv = w->cur_val; w->cur_val = w->nxt_val; w->nxt_val = tv;
        n_cur = n_nxt;
        if (n_cur == 0) return ORC_OK;
    }
    /* canonical order: ascending column */
    int32_t *oc = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_cur);
    uint64_t *ov = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n_cur);
    if (!oc || !ov) { free(oc); free(ov); return ORC_NOMEM; }
    /* sort indices, then look values up through the (re-filled) accumulator */
    for (int64_t t = 0; t < n_cur; ++t) w->acc[w->cur_idx[t]] = w->cur_val[t];
    memcpy(oc, w->cur_idx, sizeof(int32_t) * (size_t)n_cur);
    qsort(oc, (size_t)n_cur, sizeof(int32_t), cmp_i32);
    for (int64_t t = 0; t < n_cur; ++t) {
        i128 v = w->acc[oc[t]];
        if (v >= (i128)SAT63) *overflow = 1;
        ov[t] = sat_u64(v);
        w->acc[oc[t]] = 0;
    }
    *out_len = n_cur; *out_col = oc; *out_val = ov;
    return ORC_OK;
}

/*
 * Evaluate rows ``rows[0..n_rows)`` of R.  dims[i] = node count of o_{i+1};
 * row_ptr[i], col[i] = relation i (dims[i] rows, columns in [0, dims[i+1]));
 * mask[i] = 0/1 byte per node of o_{i+1}, or NULL for "no constraint".
 * nthreads <= 0 uses one thread.  Caller frees the result with orc_free.
 */
int orc_chain_rows(int n_types, const int64_t *dims, const int64_t *const *row_ptr,
                   const int32_t *const *col, const uint8_t *const *mask,
                   const int64_t *rows, int64_t n_rows, int nthreads, orc_result *res) {
    memset(res, 0, sizeof(*res));
    res->n_rows = n_rows;
    int64_t max_dim = 1;
    for (int i = 0; i < n_types; ++i) if (dims[i] > max_dim) max_dim = dims[i];
    res->row_len = (int64_t *)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(int64_t));
    int32_t **rc = (int32_t **)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(int32_t *));
    uint64_t **rv = (uint64_t **)calloc((size_t)(n_rows > 0 ? n_rows : 1), sizeof(uint64_t *));
    if (!res->row_len || !rc || !rv) { free(rc); free(rv); res->status = ORC_NOMEM; return ORC_NOMEM; }
    if (nthreads <= 0) nthreads = 1;
    int status = ORC_OK, overflow = 0;
#pragma omp parallel num_threads(nthreads)
    {
        worker w;
        w.acc = (i128 *)calloc((size_t)max_dim, sizeof(i128));
        w.cur_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_dim);
        w.nxt_idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)max_dim);
        w.cur_val = (i128 *)malloc(sizeof(i128) * (size_t)max_dim);
        w.nxt_val = (i128 *)malloc(sizeof(i128) * (size_t)max_dim);
        int ok = w.acc && w.cur_idx && w.nxt_idx && w.cur_val && w.nxt_val;
        int my_over = 0, my_status = ok ? ORC_OK : ORC_NOMEM;
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n_rows; ++r) {
            if (my_status != ORC_OK) continue;
            int s = chain_row(n_types, row_ptr, col, mask, rows[r], &w, &res->row_len[r], &rc[r], &rv[r],
                              &my_over);
            if (s != ORC_OK) my_status = s;
        }
#pragma omp critical
        {
            if (my_status != ORC_OK) status = my_status;
            if (my_over) overflow = 1;
        }
        free(w.acc); free(w.cur_idx); free(w.nxt_idx); free(w.cur_val); free(w.nxt_val);
    }
    int64_t nnz = 0;
    for (int64_t r = 0; r < n_rows; ++r) nnz += res->row_len[r];
    res->nnz = nnz;
    res->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    res->val = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nnz > 0 ? nnz : 1));
    if (!res->col || !res->val) status = ORC_NOMEM;
    int64_t o = 0;
    for (int64_t r = 0; r < n_rows; ++r) {
        if (status == ORC_OK && res->row_len[r]) {
            memcpy(res->col + o, rc[r], sizeof(int32_t) * (size_t)res->row_len[r]);
            memcpy(res->val + o, rv[r], sizeof(uint64_t) * (size_t)res->row_len[r]);
            o += res->row_len[r];
        }
        free(rc[r]); free(rv[r]);
    }
    free(rc); free(rv);
    if (status == ORC_OK && overflow) status = ORC_OVERFLOW;
    res->status = status;
    return status;
}

/*
 * Z = X * Y, X: m x k (xrp, xcol, xval or NULL), Y: k x n (yrp, ycol, yval or
 * NULL).  Values are non-negative int64.  Plain row-wise product with a dense
 * 128-bit accumulator of width n; entries equal to zero are not stored.  Result
 * values are min(value, 2^63); status ORC_OVERFLOW if any reached 2^63.
 */
int orc_spgemm(int64_t m, int64_t n, const int64_t *xrp, const int32_t *xcol, const int64_t *xval,
               const int64_t *yrp, const int32_t *ycol, const int64_t *yval, orc_result *res) {
    memset(res, 0, sizeof(*res));
    res->n_rows = m;
    res->row_len = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
    i128 *acc = (i128 *)calloc((size_t)(n > 0 ? n : 1), sizeof(i128));
    int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    size_t cap = 1024;
    res->col = (int32_t *)malloc(sizeof(int32_t) * cap);
    res->val = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    if (!res->row_len || !acc || !touched || !res->col || !res->val) {
        free(acc); free(touched); res->status = ORC_NOMEM; return ORC_NOMEM;
    }
    int status = ORC_OK, overflow = 0;
    int64_t nnz = 0;
    for (int64_t i = 0; i < m && status == ORC_OK; ++i) {
        int64_t nt = 0;
        for (int64_t e = xrp[i]; e < xrp[i + 1] && status == ORC_OK; ++e) {
            int32_t k = xcol[e];
            i128 x = xval ? (i128)xval[e] : 1;
            for (int64_t f = yrp[k]; f < yrp[k + 1]; ++f) {
                int32_t j = ycol[f];
                i128 y = yval ? (i128)yval[f] : 1;
                i128 p = x * y, s;  /* operands are below 2^63: the product fits */
                if (p == 0) continue;
                if (acc[j] == 0) touched[nt++] = j;
                if (__builtin_add_overflow(acc[j], p, &s)) { status = ORC_RANGE; break; }
                acc[j] = s;
            }
        }
        qsort(touched, (size_t)nt, sizeof(int32_t), cmp_i32);
        if ((size_t)(nnz + nt) > cap) {
            while ((size_t)(nnz + nt) > cap) cap *= 2;
            int32_t *nc = (int32_t *)realloc(res->col, sizeof(int32_t) * cap);
            if (nc) res->col = nc;
            uint64_t *nv = (uint64_t *)realloc(res->val, sizeof(uint64_t) * cap);
            if (nv) res->val = nv;
            if (!nc || !nv) { status = ORC_NOMEM; break; }
        }
        for (int64_t t = 0; t < nt; ++t) {
            int32_t j = touched[t];
            if (acc[j] >= (i128)SAT63) overflow = 1;
            res->col[nnz + t] = j;
            res->val[nnz + t] = sat_u64(acc[j]);
            acc[j] = 0;
        }
        res->row_len[i] = nt;
        nnz += nt;
    }
    free(acc); free(touched);
    res->nnz = nnz;
    if (status == ORC_OK && overflow) status = ORC_OVERFLOW;
    res->status = status;
    return status;
}

void orc_free(orc_result *res) {
    free(res->row_len); free(res->col); free(res->val);
    memset(res, 0, sizeof(*res));
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
