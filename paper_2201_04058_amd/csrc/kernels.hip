// gfx950 kernels of the metapath SpGEMM chain.
//
// One sparse product Z = X * Y (paper Sec. 3.2, the sparse product that the
// planner's Eq. 2 prices) runs as
//   symbolic  per X row: products N_op (Eq. 2's N_op, exact here) and an upper
//             bound ub = min(N_op, usable columns) on the row's nonzeros; the
//             row is binned by ub;
//   numeric   per bin: small rows accumulate in a wavefront-private LDS hash,
//             mid rows in a workgroup LDS hash, long rows in dense LDS tiles
//             over column ranges; hash rows are bitonic-sorted by column;
//   compact   scan of per-row nonzeros -> row pointers; segments are copied
//             from the ub-sized slots into exact-size arrays.
// Constraints (the diagonal masks M_c of Sec. 2) are bitsets tested while the
// operands are read.  Counts are int64 with saturation at 2^63: a count
// reaching 2^63 is carried as the value 2^63, so every stored value equals
// min(true count, 2^63) whatever the multiplication order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace atp {

namespace {

constexpr int kLongRow = 128;     // X rows longer than this go to the chunked symbolic pass
constexpr int kProdUnroll = 4;    // products per lane per step of a flattened product walk
constexpr int kHashUnroll = 2;    // ... in the hash kernels
constexpr int64_t kSymChunk = 4096;

__device__ __forceinline__ bool bit_test(const uint32_t *b, int64_t i) {
    return (b[i >> 5] >> (i & 31)) & 1u;
}

__device__ __forceinline__ uint64_t sat_mul(uint64_t a, uint64_t b) {
    if (((a | b) >> 32) == 0) {  // both below 2^32: one 32x32->64 product
        const uint64_t p = (uint64_t)(uint32_t)a * (uint32_t)b;
        return (p & kSat) ? kSat : p;
    }
    if ((a | b) & kSat) return kSat;
    uint64_t hi = __umul64hi(a, b);
    uint64_t lo = a * b;
    return (hi != 0 || (lo & kSat)) ? kSat : lo;
}

// Add contribution c to accumulator slot `slot` (value v, saturation bitmap
// satw).  The first addition whose running sum reaches 2^63 sees an old value
// below 2^63 and a new one at or above it, so the flag is exact.
__device__ __forceinline__ void acc_add(unsigned long long *v, uint32_t *satw, uint32_t slot, uint64_t c) {
    if (c & kSat) {
        atomicOr(&satw[slot >> 5], 1u << (slot & 31));
        return;
    }
    unsigned long long old = atomicAdd(v, (unsigned long long)c);
    if (old < kSat && old + c >= kSat) atomicOr(&satw[slot >> 5], 1u << (slot & 31));
}

__device__ __forceinline__ int64_t lower_bound_col(const int32_t *col, int64_t lo, int64_t hi, int32_t key) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (col[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Lower bound of `key` in the ascending arr[lo, hi), searched by a group of g
// lanes of one wavefront (g a power of two <= 64, li = lane within the group,
// gmask = the group's lanes in the wavefront).  Each round probes g evenly
// spaced positions and keeps the gap that holds the answer, so a range of n
// entries takes about log(n)/log(g+1) dependent loads.
template <typename T, typename K>
__device__ __forceinline__ int64_t group_lower_bound(const T *arr, int64_t lo, int64_t hi, K key, int g, int li,
                                                     uint64_t gmask) {
    while (hi - lo > g) {
        const int64_t span = hi - lo;
        const int64_t pos = lo + span * (li + 1) / (g + 1);
        const bool pred = arr[pos] < key;
        const int cnt = __popcll(__ballot(pred) & gmask);
        const int64_t nlo = cnt > 0 ? lo + span * cnt / (g + 1) + 1 : lo;
        const int64_t nhi = cnt < g ? lo + span * (cnt + 1) / (g + 1) : hi;
        lo = nlo;
        hi = nhi;
    }
    const bool pred = (lo + li < hi) && arr[lo + li] < key;
    return lo + __popcll(__ballot(pred) & gmask);
}

__device__ __forceinline__ uint64_t group_mask(int g) {
    const int lane = threadIdx.x & 63;
    const uint64_t base = g == 64 ? ~0ull : ((1ull << g) - 1ull);
    return base << (lane & ~(g - 1));
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Task ids 0 .. n-1 handed out by kQueues counters q[0 .. kQueues) (zeroed
// before the launch): counter g hands out g, g + kQueues, ...  A workgroup
// starts at counter blockIdx.x mod kQueues and moves on to the next one when
// a counter runs dry; -1 once all have.  Called by one thread, which keeps
// the cursor.
struct QueueCursor {
    int grp, tried;
};
__device__ __forceinline__ QueueCursor queue_start() { return QueueCursor{(int)(blockIdx.x & (kQueues - 1)), 0}; }
__device__ __forceinline__ int64_t queue_next(int64_t *q, int64_t n, QueueCursor &cur) {
    while (cur.tried < kQueues) {
        const int64_t idx = (int64_t)atomicAdd((unsigned long long *)&q[cur.grp], 1ull);
        const int64_t t = cur.grp + (int64_t)kQueues * idx;
        if (t < n) return t;
        cur.grp = (cur.grp + 1) & (kQueues - 1);
        ++cur.tried;
    }
    return -1;
}

// The workgroup's next task from the queue (every thread calls it; slot is
// a __shared__ int64_t).
__device__ __forceinline__ int64_t block_next_task(int64_t *q, int64_t n, QueueCursor &cur, int64_t *slot) {
    if (threadIdx.x == 0) *slot = queue_next(q, n, cur);
    __syncthreads();
    const int64_t t = *slot;
    __syncthreads();  // read by all before the next call writes it
    return t;
}

// lanes per X entry: power of two near the average Y-row length, in [1, 64]
__host__ __device__ inline int group_size(int64_t avg) {
    int g = 1;
    while (g < 64 && (int64_t)g * 2 <= avg + (avg >> 1)) g <<= 1;
    return g;
}

__device__ __forceinline__ uint32_t hash_of(int32_t j, int log2s) {
    return ((uint32_t)j * 0x9E3779B1u) >> (32 - log2s);
}

// Slot of column j in an open-addressing LDS table of S slots, inserted if
// absent.  Tables hold at least twice the distinct columns they receive, so a
// probe sequence ends within S steps; should it not (a sizing error), *fault
// is set and slot 0 is returned: the product's result is then wrong, and the
// host, which reads the fault flag, discards it (ATP_EDEVICE).
template <int S>
__device__ __forceinline__ uint32_t hash_find(int32_t *keys, int32_t j, int32_t *fault) {
    constexpr int L = __builtin_ctz(S);
    uint32_t h = hash_of(j, L);
    for (int n = 0; n < S; ++n) {
        int32_t k = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (k == j) return h;
        if (k == kEmptyKey) {
            int32_t prev = atomicCAS(&keys[h], kEmptyKey, j);
            if (prev == kEmptyKey || prev == j) return h;
        }
        h = (h + 1) & (S - 1);
    }
    atomicOr(fault, 1);
    return 0;
}

// Accumulate row i of X*Y into an LDS hash table.  Groups of g lanes walk one
// X entry each; the lanes of a group stride over the Y row.
template <int S>
__device__ __forceinline__ void accumulate_hash(const Operand &X, const Operand &Y, int64_t xb, int64_t xe,
                                                int gid, int ng, int li, int g, int32_t *keys,
                                                unsigned long long *vals, uint32_t *satw, int32_t *fault) {
    for (int64_t e = xb + gid; e < xe; e += ng) {
        int32_t k = X.col[e];
        if (X.cmask && !bit_test(X.cmask, k)) continue;
        uint64_t xv = X.val ? X.val[e] : 1ull;
        int64_t yb = Y.rp[k], ye = Y.rp[k + 1];
        for (int64_t f = yb + li; f < ye; f += g) {
            int32_t j = Y.col[f];
            if (Y.cmask && !bit_test(Y.cmask, j)) continue;
            uint64_t c = Y.val ? sat_mul(xv, Y.val[f]) : xv;
            uint32_t h = hash_find<S>(keys, j, fault);
            acc_add(&vals[h], satw, h, c);
        }
    }
}

// ---------------------------------------------------------------------------
// fills, scans

__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// inclusive scan across a 256-thread block; returns the inclusive value, *total = block sum
__device__ int64_t block_inclusive_scan(int64_t x, int64_t *smem_waves, int64_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int64_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) smem_waves[wave] = v;
    __syncthreads();
    int64_t pre = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        int64_t s = smem_waves[w];
        if (w < wave) pre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return v + pre;
}

// Several scans of the same length in one launch sequence: job = blockIdx.y.
struct ScanJobs {
    ScanJob job[kMaxScanJobs];
    int64_t stride;  // tmp entries per job
};

__device__ __forceinline__ int64_t scan_blocks(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return nb > 0 ? nb : 1;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(ScanJobs sj, int64_t *tmp) {
    __shared__ int64_t sw[kScanThreads / 64];
    const ScanJob &j = sj.job[blockIdx.y];
    if ((int64_t)blockIdx.x >= scan_blocks(j.n)) return;  // uniform: this job has fewer tiles
    const int64_t *in = j.in;
    int64_t *t = tmp + blockIdx.y * sj.stride;
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        int64_t i = base + (int64_t)r * kScanThreads + threadIdx.x;
        if (i < j.n) s += in[i];
    }
    int64_t tot;
    block_inclusive_scan(s, sw, &tot);
    if (threadIdx.x == 0) t[blockIdx.x] = tot;
}

// exclusive scan of tmp[0..nb) in place, tmp[nb] = total; one block per job
__global__ __launch_bounds__(kScanThreads) void k_scan_top(ScanJobs sj, int64_t *tmp) {
    __shared__ int64_t sw[kScanThreads / 64];
    const int64_t nb = scan_blocks(sj.job[blockIdx.x].n);
    int64_t *t = tmp + blockIdx.x * sj.stride;
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        int64_t i = base + threadIdx.x;
        int64_t x = i < nb ? t[i] : 0;
        int64_t tot;
        int64_t inc = block_inclusive_scan(x, sw, &tot);
        if (i < nb) t[i] = carry + inc - x;
        carry += tot;
    }
    if (threadIdx.x == 0) t[nb] = carry;
}

// one tile [base, base + kScanTile) of job j with offset `carry`; returns the tile sum
__device__ __forceinline__ int64_t scan_tile(const ScanJob &j, int64_t n, int64_t tile_base, int64_t carry,
                                             int64_t *sw) {
    const int64_t base = tile_base + (int64_t)threadIdx.x * kScanItems;
    int64_t x[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        int64_t i = base + r;
        x[r] = i < n ? j.in[i] : 0;
        s += x[r];
    }
    int64_t tot;
    int64_t inc = block_inclusive_scan(s, sw, &tot);
    int64_t run = carry + inc - s;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        int64_t i = base + r;
        if (i < n) j.out[i] = run;
        run += x[r];
    }
    return tot;
}

// per block: exclusive scan of its tile with offset tmp[block]
__global__ __launch_bounds__(kScanThreads) void k_scan_down(ScanJobs sj, const int64_t *tmp) {
    __shared__ int64_t sw[kScanThreads / 64];
    const ScanJob &j = sj.job[blockIdx.y];
    const int64_t nb = scan_blocks(j.n);
    if ((int64_t)blockIdx.x >= nb) return;  // uniform
    const int64_t *t = tmp + blockIdx.y * sj.stride;
    scan_tile(j, j.n, (int64_t)blockIdx.x * kScanTile, t[blockIdx.x], sw);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        j.out[j.n] = t[nb];
        if (j.total) *j.total = t[nb];
    }
}

// As k_scan_down after k_scan_top, from the raw tile sums of k_scan_reduce:
// each block adds up the sums of the tiles before it (block 0: of every
// tile, the total) instead of a separate scan of the sums.  For at most
// kScanFoldTiles tiles, so that the re-read sums stay few.
__global__ __launch_bounds__(kScanThreads) void k_scan_down_fold(ScanJobs sj, const int64_t *tmp) {
    __shared__ int64_t sw[kScanThreads / 64];
    const ScanJob &j = sj.job[blockIdx.y];
    const int64_t nb = scan_blocks(j.n);
    if ((int64_t)blockIdx.x >= nb) return;  // uniform
    const int64_t *t = tmp + blockIdx.y * sj.stride;
    const int64_t upto = blockIdx.x == 0 ? nb : (int64_t)blockIdx.x;
    int64_t x = 0;
    for (int64_t i = threadIdx.x; i < upto; i += kScanThreads) x += t[i];
    int64_t sum;
    block_inclusive_scan(x, sw, &sum);  // its closing barrier frees sw for the tile scan
    scan_tile(j, j.n, (int64_t)blockIdx.x * kScanTile, blockIdx.x == 0 ? 0 : sum, sw);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        j.out[j.n] = sum;
        if (j.total) *j.total = sum;
    }
}

// short arrays: one block per job walks its tiles with a running carry
__global__ __launch_bounds__(kScanThreads) void k_scan_small(ScanJobs sj) {
    __shared__ int64_t sw[kScanThreads / 64];
    const ScanJob &j = sj.job[blockIdx.x];
    int64_t carry = 0;
    for (int64_t base = 0; base < j.n; base += kScanTile) carry += scan_tile(j, j.n, base, carry, sw);
    if (threadIdx.x == 0) {
        j.out[j.n] = carry;
        if (j.total) *j.total = carry;
    }
}

// ---------------------------------------------------------------------------
// masks (diagonal M_c as a bitset)

// One bit per node: lo <= prop <= hi.  Each wavefront covers 64 consecutive
// nodes per step (one ballot, two words), striding over the grid until every
// node is covered, so any node count fits the launch.
template <typename T>
__global__ void k_mask_range(const T *prop, int64_t n, int64_t lo, int64_t hi, uint32_t *bits, int64_t words,
                             int and_mode) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = blockIdx.x * (int64_t)blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
        const int64_t gid = base + (threadIdx.x & 63);
        bool keep = false;
        if (gid < n) {
            int64_t v = (int64_t)prop[gid];
            keep = v >= lo && v <= hi;
        }
        uint64_t b = __ballot(keep);
        if ((threadIdx.x & 63) == 0) {
            int64_t w = base >> 5;
            uint32_t w0 = (uint32_t)b, w1 = (uint32_t)(b >> 32);
            if (w < words) bits[w] = and_mode ? (bits[w] & w0) : w0;
            if (w + 1 < words) bits[w + 1] = and_mode ? (bits[w + 1] & w1) : w1;
        }
    }
}

__global__ void k_mask_ids(const int32_t *ids, int64_t n, uint32_t *bits) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = ids[i];
        atomicOr(&bits[v >> 5], 1u << (v & 31));
    }
}

__global__ void k_mask_and(uint32_t *dst, const uint32_t *src, int64_t words) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] &= src[i];
}

__global__ void k_popcount(const uint32_t *bits, int64_t words, int64_t *out) {
    int64_t s = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        s += __popc(bits[i]);
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd((unsigned long long *)out, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// symbolic pass

// Sum of |Y row k| over the X entries k at positions p0, p0 + stride, ...
// below e that pass X's column mask; UN entries' loads are in flight
// together (column ids, then mask words, then row-pointer pairs).
template <int UN = 4>
__device__ __forceinline__ int64_t sum_right_rows(const Operand &X, const Operand &Y, int64_t p0, int64_t e,
                                                  int stride) {
    int64_t s = 0;
    for (int64_t p = p0; p < e; p += UN * (int64_t)stride) {
        int32_t k[UN];
        bool ok[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            const int64_t q = p + (int64_t)u * stride;
            ok[u] = q < e;
            k[u] = ok[u] ? X.col[q] : 0;
        }
        if (X.cmask) {
#pragma unroll
            for (int u = 0; u < UN; ++u)
                if (ok[u]) ok[u] = bit_test(X.cmask, k[u]);
        }
        int64_t lo[UN], hi[UN];
#pragma unroll
        for (int u = 0; u < UN; ++u) {
            lo[u] = ok[u] ? Y.rp[k[u]] : 0;
            hi[u] = ok[u] ? Y.rp[k[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < UN; ++u) s += hi[u] - lo[u];
    }
    return s;
}

// Eight lanes per candidate row (they stride over its entries); rows longer
// than kLongRow are left to the chunked pass.
constexpr int kSymLanes = 8;
constexpr int kBinThreads = 1024;  // rows per binning workgroup
__global__ __launch_bounds__(256) void k_symbolic(SymbolicArgs a) {
    const int64_t c = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kSymLanes;
    const int li = threadIdx.x & (kSymLanes - 1);
    int64_t nop = 0, deferred = 0;
    if (c < a.n_cand) {  // uniform within the group
        const int64_t i = a.cand ? a.cand[c] : c;
        if (!(a.X.rmask && !bit_test(a.X.rmask, i))) {
            const int64_t b = a.X.rp[i], e = a.X.rp[i + 1];
            if (e - b > kLongRow) {
                deferred = (e - b + kSymChunk - 1) / kSymChunk;
            } else {
                nop = sum_right_rows<4>(a.X, a.Y, b + li, e, kSymLanes);
            }
        }
    }
    for (int d = kSymLanes / 2; d > 0; d >>= 1) nop += __shfl_xor(nop, d, kSymLanes);
    if (c < a.n_cand && li == 0) {
        a.nop[c] = nop;
        a.long_len[c] = deferred;  // chunks left to the long-row pass
        // per-bin-list-position counts that the binning fills sparsely (scanned over all n_cand)
        a.dense_chunks[c] = 0;
        a.bucket_chunks[c] = 0;
        a.bucket_nop[c] = 0;
    }
    // the step's product total: one atomic per workgroup
    __shared__ int64_t s_sum[4];
    int64_t wsum = li == 0 ? nop : 0;
    for (int d = 32; d > 0; d >>= 1) wsum += __shfl_xor(wsum, d, 64);
    if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = wsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t bsum = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
        if (bsum) atomicAdd((unsigned long long *)&a.hdr->n_op_total, (unsigned long long)bsum);
    }
}

// Long rows are cut into chunks of kSymChunk entries (long_len holds each
// candidate's chunk count, long_off its exclusive scan); one workgroup per
// chunk sums the products and adds them to the row with one atomic.
__global__ __launch_bounds__(256) void k_symbolic_long(SymbolicArgs a, const int64_t *long_off) {
    __shared__ int64_t sw[4];
    __shared__ int64_t s_c;
    const int64_t n_chunks = long_off[a.n_cand];
    int64_t block_total = 0;  // thread 0's sum over the workgroup's chunks
    for (int64_t id = blockIdx.x; id < n_chunks; id += gridDim.x) {
        if (threadIdx.x < 64) {
            const int64_t c = group_lower_bound(long_off, 0, a.n_cand, id + 1, 64, threadIdx.x, ~0ull) - 1;
            if (threadIdx.x == 0) s_c = c;
        }
        __syncthreads();
        const int64_t c = s_c;
        const int64_t i = a.cand ? a.cand[c] : c;
        const int64_t q = id - long_off[c];
        const int64_t b = a.X.rp[i] + q * kSymChunk;
        const int64_t e = (b + kSymChunk < a.X.rp[i + 1]) ? b + kSymChunk : a.X.rp[i + 1];
        const int64_t s = sum_right_rows<8>(a.X, a.Y, b + threadIdx.x, e, blockDim.x);
        int64_t tot;
        block_inclusive_scan(s, sw, &tot);
        if (threadIdx.x == 0 && tot) {
            atomicAdd((unsigned long long *)&a.nop[c], (unsigned long long)tot);
            block_total += tot;
        }
    }
    // the step's product total: one atomic per workgroup
    if (threadIdx.x == 0 && block_total) atomicAdd((unsigned long long *)&a.hdr->n_op_total, (unsigned long long)block_total);
}

__global__ __launch_bounds__(kBinThreads) void k_bin_rows(SymbolicArgs a) {
    constexpr int NWV = kBinThreads / 64;
    __shared__ int32_t s_cnt[BIN_COUNT][NWV];           // members per (bin, wavefront)
    __shared__ unsigned long long s_base[BIN_COUNT][NWV];  // list position of each wavefront's first
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = c < a.n_cand;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t nop = live ? a.nop[c] : 0;
    int64_t ub = nop < a.ycols_eff ? nop : a.ycols_eff;
    int32_t bin = BIN_NONE;
    int64_t nseg = 0;
    const int64_t ycols = a.Y.cols;
    const int64_t ntiles = (ycols + kTileW - 1) / kTileW;
    if (live && ub > 0) {
        if (ub > 4096 || (ycols <= kTileW && ycols <= 8 * ub)) {
            bin = BIN_DENSE;
            nseg = ntiles;
            if (ntiles > 1 && ntiles <= kMaxBucketTiles) {
                const int64_t i = a.cand ? a.cand[c] : c;
                const int64_t xlen = a.X.rp[i + 1] - a.X.rp[i];
                if (xlen > kCursorCap && xlen * ntiles * 100 > a.tune.bucket_pct * nop) bin = BIN_BUCKET;
            }
        } else {
            nseg = 1;
            bin = ub <= 32 ? BIN_W64 : ub <= 64 ? BIN_W128 : ub <= 128 ? BIN_W256 : ub <= 256 ? BIN_W512
                : ub <= 512 ? BIN_B1024 : ub <= 1024 ? BIN_B2048 : ub <= 2048 ? BIN_B4096 : BIN_B8192;
        }
    }
    if (live) {
        a.ub[c] = ub;
        a.nseg[c] = nseg;
        a.bin[c] = bin;
    }
    // bin lists: one atomic per (workgroup, bin); wavefronts take consecutive ranges
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int b = BIN_W64; b < BIN_COUNT; ++b) {
        const uint64_t m = __ballot(bin == b);
        if (lane == 0) s_cnt[b][wave] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x >= BIN_W64 && threadIdx.x < BIN_COUNT) {
        const int b = threadIdx.x;
        unsigned long long tot = 0;
        for (int w = 0; w < NWV; ++w) tot += (unsigned long long)s_cnt[b][w];
        unsigned long long base = tot ? atomicAdd((unsigned long long *)&a.hdr->bin_count[b], tot) : 0ull;
        for (int w = 0; w < NWV; ++w) {
            s_base[b][w] = base;
            base += (unsigned long long)s_cnt[b][w];
        }
    }
    __syncthreads();
    for (int b = BIN_W64; b < BIN_COUNT; ++b) {
        const uint64_t m = __ballot(bin == b);
        if (m == 0) continue;
        const unsigned long long base = s_base[b][wave];
        if (bin == b) {
            const int64_t pos = (int64_t)base + __popcll(m & lt);
            a.bin_lists[(int64_t)b * a.n_cand + pos] = (int32_t)c;
            if (b == BIN_BUCKET) {
                int64_t i = a.cand ? a.cand[c] : c;
                int64_t xlen = a.X.rp[i + 1] - a.X.rp[i];
                a.bucket_chunks[pos] = (xlen + a.tune.bucket_chunk - 1) / a.tune.bucket_chunk;
                a.bucket_nop[pos] = nop;
            }
            if (b == BIN_DENSE) {
                int64_t nch = 1;
                int64_t m = ntiles;  // tiles per part
                int64_t grp = 1;     // parts per task
                if (ntiles > 1) {
                    int64_t i = a.cand ? a.cand[c] : c;
                    int64_t xlen = a.X.rp[i + 1] - a.X.rp[i];
                    const int64_t per_tile = nop / ntiles;
                    m = 1;
                    if (per_tile < a.tune.part_target) {
                        m = a.tune.part_target / (per_tile > 0 ? per_tile : 1);
                        m = m > kPartMaxTiles ? kPartMaxTiles : m;
                        // small parts are handed out several to a task (the
                        // row's set-up is paid once), while the step still
                        // gives each resident workgroup several tasks
                        grp = a.hdr->n_op_total / (a.tune.part_target * 4 * a.tune.wg_slots);
                        grp = grp < 1 ? 1 : (grp > kPartGroup ? kPartGroup : grp);
                    } else if (xlen <= kCursorCap) {
                        int64_t chunks = (nop + a.tune.task_ops - 1) / a.tune.task_ops;
                        chunks = chunks < 1 ? 1 : chunks;
                        m = (ntiles + chunks - 1) / chunks;
                    }
                    m = m < 1 ? 1 : (m > ntiles ? ntiles : m);
                    const int64_t nparts = (ntiles + m - 1) / m;
                    nch = (nparts + grp - 1) / grp;
                }
                // heavy rows: split the left entries over several workgroups per tile
                int64_t ks = 1;
                {
                    const int64_t i = a.cand ? a.cand[c] : c;
                    const int64_t xlen = a.X.rp[i + 1] - a.X.rp[i];
                    const int64_t per_tile = nop / ntiles;
                    // a straggler holds more than the step's work per resident workgroup
                    int64_t thr = a.hdr->n_op_total / (2 * a.tune.wg_slots);
                    thr = thr > a.tune.split_ops ? thr : a.tune.split_ops;
                    if (per_tile > thr) {
                        ks = (per_tile + thr - 1) / thr;
                        const int64_t cap = xlen / 8 < kMaxSplit ? xlen / 8 : kMaxSplit;
                        ks = ks > cap ? cap : ks;
                    }
                }
                if (ks > 1) {
                    nch = ntiles * ks;  // one part per tile
                    const unsigned long long slot = atomicAdd((unsigned long long *)&a.hdr->n_split, 1ull);
                    a.dense_split[pos] = (int64_t)slot * 256 + ks;
                } else {
                    a.dense_split[pos] = (m << 16) | (grp << 8) | 1;
                }
                // with many column tiles, every row's task count is padded to a multiple
                // of kQueues (the extra tasks do nothing): a row's tasks then start at a
                // multiple of kQueues, task q of a row goes out through counter q mod
                // kQueues, whose workgroups sit mostly on one XCD, and the tasks of a
                // column tile (one part per task) gather that tile's slice of Y on one XCD
                // (its L2) for every row
                if (ntiles >= kAlignTiles) nch = (nch + kQueues - 1) / kQueues * kQueues;
                a.dense_chunks[pos] = nch;
            }
        }
    }
}

// Visit the flattened products of a batch of at most NT left entries (NT
// threads cooperate: a block, or one wavefront when NT = 64): entry e's
// segment is right-operand entries [seg_s[e], seg_s[e] + len) and its items
// are [seg_o[e], seg_o[e+1]) of the batch's tot items (tot < 2^31; seg_o has
// NT + 1 entries).  f(column, value) per product whose column passes Y's
// column mask.  Each wavefront takes a contiguous chunk of items,
// U items per lane per step (unit stride between lanes), and tracks
// its entry with a forward walk; the step's gathers of the right operand are
// all issued before the first is used, so their latencies overlap.  XV / YV:
// the left / right operand carries values (else every value is 1).
template <bool XV, bool YV, int NT, int U, typename F>
__device__ __forceinline__ void walk_products(const Operand &Y, const int32_t *seg_o, const int64_t *seg_s,
                                              int32_t tot, const uint64_t *xval, F f, int nb = NT,
                                              bool plain = false) {
    constexpr int NWV = NT / 64;
    const int lane = threadIdx.x & 63, wave = (threadIdx.x >> 6) & (NWV - 1);
    const int32_t chunk = (((tot + NWV - 1) / NWV) + 63) & ~63;
    const int32_t beg = wave * chunk;
    const int32_t end = (beg + chunk < tot) ? beg + chunk : tot;
    if (beg >= end) return;
    int32_t item = beg + lane;
    const int32_t first = item < end ? item : end - 1;
    int lo = 0, hi = nb;  // last entry with seg_o <= first (entries from nb on are empty)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg_o[mid] <= first)
            lo = mid;
        else
            hi = mid;
    }
    int ent = lo;
    int32_t o0 = seg_o[ent], o1 = seg_o[ent + 1];
    int64_t s0 = seg_s[ent];
    uint64_t xv = XV ? xval[ent] : 1ull;
    for (; item < end; item += 64 * U) {
        // an item past the chunk repeats the lane's previous one (loads stay
        // in bounds and unconditional) and is skipped when applied
        int64_t fpos[U];
        uint64_t xs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t it = item + 64 * u;
            if (u == 0 || it < end) {
                while (it >= o1) {
                    ++ent;
                    o0 = o1;
                    o1 = seg_o[ent + 1];
                    s0 = seg_s[ent];
                    if (XV) xv = xval[ent];
                }
                fpos[u] = s0 + (it - o0);
            } else {
                fpos[u] = fpos[u - 1];
            }
            if (XV) xs[u] = xv;
        }
        int32_t js[U];
        uint64_t ys[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            js[u] = Y.col[fpos[u]];
            if (YV) ys[u] = Y.val[fpos[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (item + 64 * u >= end) break;
            if (Y.cmask && !bit_test(Y.cmask, js[u])) continue;
            f(js[u], YV ? (XV ? (plain ? xs[u] * ys[u] : sat_mul(xs[u], ys[u])) : ys[u]) : (XV ? xs[u] : 1ull));
        }
    }
}

// walk_products for whichever operands carry values
// (plain: no product can reach 2^63, so values multiply without the
// saturation check)
template <int NT, int U = kProdUnroll, typename F>
__device__ __forceinline__ void walk_products_any(const Operand &Y, const int32_t *seg_o, const int64_t *seg_s,
                                                  int32_t tot, const uint64_t *xval, F f, int nb = NT,
                                                  bool plain = false) {
    if (xval) {
        if (Y.val)
            walk_products<true, true, NT, U>(Y, seg_o, seg_s, tot, xval, f, nb, plain);
        else
            walk_products<true, false, NT, U>(Y, seg_o, seg_s, tot, xval, f, nb);
    } else {
        if (Y.val)
            walk_products<false, true, NT, U>(Y, seg_o, seg_s, tot, xval, f, nb);
        else
            walk_products<false, false, NT, U>(Y, seg_o, seg_s, tot, xval, f, nb);
    }
}

// A batch's products are walked flattened when they number below this.
constexpr int64_t kWalkMax = (int64_t)1 << 30;

// Segments of left entries [e0, e0 + nb) (nb <= NT): each entry's whole right
// row (empty when the column mask excludes it).  NT = blockDim.x threads, or
// one wavefront (NT = 64).  Returns the batch's product count (uniform).
template <int NT>
__device__ __forceinline__ int64_t row_segments(const Operand &X, const Operand &Y, int64_t e0, int64_t nb,
                                                int64_t *seg_s, int32_t *seg_o, int64_t *sw) {
    const int tid = NT == 64 ? (int)(threadIdx.x & 63) : (int)threadIdx.x;
    int64_t len = 0;
    if (tid < nb) {
        const int32_t k = X.col[e0 + tid];
        if (!X.cmask || bit_test(X.cmask, k)) {
            const int64_t yb = Y.rp[k];
            len = Y.rp[k + 1] - yb;
            seg_s[tid] = yb;
        }
    }
    int64_t tot, inc;
    if (NT == 64) {
        inc = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t o = __shfl_up(inc, d, 64);
            if (tid >= d) inc += o;
        }
        tot = __shfl(inc, 63, 64);
    } else {
        inc = block_inclusive_scan(len, sw, &tot);
    }
    seg_o[tid] = (int32_t)(inc - len);
    if (tid == NT - 1) seg_o[NT] = (int32_t)inc;
    if (NT == 64)
        wave_sync();
    else
        __syncthreads();
    return tot;
}

// ---------------------------------------------------------------------------
// numeric: LDS hash, one wavefront per row


// Wavefront bitonic sort of the first n (power of two) pairs.
__device__ void bitonic_sort_wave_rt(int32_t *keys, unsigned long long *vals, int n, int lane) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = lane; t < n / 2; t += 64) {
                int a = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                int b = a + j;
                bool up = (a & k) == 0;
                int32_t ka = keys[a], kb = keys[b];
                if ((ka > kb) == up) {
                    keys[a] = kb;
                    keys[b] = ka;
                    unsigned long long va = vals[a];
                    vals[a] = vals[b];
                    vals[b] = va;
                }
            }
            wave_sync();
        }
    }
}

template <int S>
__global__ __launch_bounds__(256) void k_hash_wave(const int32_t *list, int64_t n, NumericArgs a) {
    __shared__ int32_t keys_all[4][S];
    __shared__ unsigned long long vals_all[4][S];
    __shared__ uint32_t sat_all[4][(S + 31) / 32];
    __shared__ int cnt_all[4];
    __shared__ int64_t segs_all[4][64];
    __shared__ int32_t sego_all[4][65];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t *keys = keys_all[wave];
    unsigned long long *vals = vals_all[wave];
    uint32_t *satw = sat_all[wave];
    int64_t *seg_s = segs_all[wave];
    int32_t *seg_o = sego_all[wave];
    for (int t = lane; t < S; t += 64) {
        keys[t] = kEmptyKey;
        vals[t] = 0;
    }
    for (int t = lane; t < (S + 31) / 32; t += 64) satw[t] = 0;
    if (lane == 0) cnt_all[wave] = 0;
    wave_sync();
    for (int64_t r = (int64_t)blockIdx.x * 4 + wave; r < n; r += (int64_t)gridDim.x * 4) {
        const int32_t c = list[r];
        const int64_t i = a.cand ? a.cand[c] : c;
        const int64_t xb = a.X.rp[i], xe = a.X.rp[i + 1];
        // batches of 64 left entries, their products walked flattened
        for (int64_t eb = xb; eb < xe; eb += 64) {
            const int64_t nb = (xe - eb < 64) ? xe - eb : 64;
            const int64_t tot = row_segments<64>(a.X, a.Y, eb, nb, seg_s, seg_o, nullptr);
            if (tot < kWalkMax)
                walk_products_any<64, kHashUnroll>(a.Y, seg_o, seg_s, (int32_t)tot, a.X.val ? a.X.val + eb : nullptr,
                                      [&](int32_t j, uint64_t v) {
                                          const uint32_t h = hash_find<S>(keys, j, &a.hdr->fault);
                                          acc_add(&vals[h], satw, h, v);
                                      }, (int)nb);
            else
                accumulate_hash<S>(a.X, a.Y, eb, eb + nb, 0, 1, lane, 64, keys, vals, satw, &a.hdr->fault);
            wave_sync();
        }
        // compact the occupied slots to the front in one pass (a slot is read
        // before any write can reach it: positions written stay below the
        // current group of 64), then sort the next power of two of them
        int local = 0;
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        for (int t0 = 0; t0 < S; t0 += 64) {
            const int t = t0 + lane;
            const int32_t kk = keys[t];
            unsigned long long vv = vals[t];
            const bool occ = kk != kEmptyKey;
            if (occ && ((satw[t >> 5] >> (t & 31)) & 1u)) vv = kSat;
            const uint64_t m = __ballot(occ);
            if (occ) {
                const int pos = local + __popcll(m & lt);
                keys[pos] = kk;
                vals[pos] = vv;
            }
            local += __popcll(m);
            wave_sync();
        }
        int p2 = 1;
        while (p2 < local) p2 <<= 1;
        for (int t = local + lane; t < p2; t += 64) keys[t] = kEmptyKey;
        wave_sync();
        bitonic_sort_wave_rt(keys, vals, p2, lane);
        const int64_t off = a.slot_off[c];
        bool sat = false;
        for (int t = lane; t < local; t += 64) {
            a.slot_col[off + t] = keys[t];
            unsigned long long v = vals[t];
            a.slot_val[off + t] = v;
            sat |= (v & kSat) != 0;
        }
        wave_sync();
        for (int t = lane; t < S; t += 64) {  // the whole table back to empty
            keys[t] = kEmptyKey;
            vals[t] = 0;
        }
        if (__ballot(sat) != 0 && lane == 0) atomicOr(&a.hdr->saturated, 1);
        for (int t = lane; t < (S + 31) / 32; t += 64) satw[t] = 0;
        if (lane == 0) {
            const int64_t sb = a.seg_base[c];
            a.seg_cnt[sb] = local;
            a.seg_src[sb] = off;
            a.row_nnz[i] = local;
        }
        wave_sync();
    }
}

// ---------------------------------------------------------------------------
// numeric: LDS hash, one workgroup per row

// Sort keys/vals[0, n) ascending by key within a workgroup of NT threads
// (keys unique; n <= S/2 and entries [n, S) free).  128-entry chunks are
// bitonic-sorted by one wavefront each (no workgroup barriers); then runs
// are merged pairwise, every entry placed at its index in its run plus the
// number of entries of the other run that precede it (a binary search:
// keys below it from a right run, keys up to it from a left run), moving
// between the two halves of the arrays.  Returns the offset of the sorted
// entries.
template <int S, int NT>
__device__ int merge_sort_block(int32_t *keys, unsigned long long *vals, int n) {
    constexpr int C = 128;
    constexpr int NWV = NT / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int np = (n + C - 1) / C * C;  // whole chunks, padded with keys above every column
    for (int t = n + threadIdx.x; t < np; t += NT) keys[t] = kEmptyKey;
    __syncthreads();
    for (int c = wave; c * C < np; c += NWV) bitonic_sort_wave_rt(keys + c * C, vals + c * C, C, lane);
    __syncthreads();
    int src = 0, dst = S / 2;
    for (int L = C; L < np; L <<= 1) {
        for (int t = threadIdx.x; t < np; t += NT) {
            const int run = t / L;
            const int base = (run & ~1) * L;  // start of the run pair
            const bool left = (run & 1) == 0;
            const int32_t k = keys[src + t];
            const unsigned long long v = vals[src + t];
            // the pair's other run [ob, oe) (empty for a left run without a partner)
            const int ob = left ? base + L : base;
            int oe = left ? base + 2 * L : base + L;
            if (oe > np) oe = np;
            int lo = ob, hi = oe > ob ? oe : ob;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                const int32_t km = keys[src + mid];
                if (left ? (km < k) : (km <= k))
                    lo = mid + 1;
                else
                    hi = mid;
            }
            const int pos = base + (t - run * L) + (lo - ob);
            keys[dst + pos] = k;
            vals[dst + pos] = v;
        }
        __syncthreads();
        const int tmp = src;
        src = dst;
        dst = tmp;
    }
    return src;
}

template <int S, int NT>
__global__ __launch_bounds__(NT) void k_hash_block(const int32_t *list, int64_t n, NumericArgs a) {
    __shared__ int32_t keys[S];
    __shared__ unsigned long long vals[S];
    __shared__ uint32_t satw[S / 32];
    __shared__ int64_t sw[NT / 64];
    __shared__ int64_t seg_s[NT];
    __shared__ int32_t seg_o[NT + 1];
    __shared__ int any_sat;
    for (int t = threadIdx.x; t < S; t += NT) {
        keys[t] = kEmptyKey;
        vals[t] = 0;
    }
    for (int t = threadIdx.x; t < S / 32; t += NT) satw[t] = 0;
    if (threadIdx.x == 0) any_sat = 0;
    __syncthreads();
    for (int64_t r = blockIdx.x; r < n; r += gridDim.x) {
        const int32_t c = list[r];
        const int64_t i = a.cand ? a.cand[c] : c;
        const int64_t xb = a.X.rp[i], xe = a.X.rp[i + 1];
        // batches of NT left entries, their products walked flattened
        for (int64_t eb = xb; eb < xe; eb += NT) {
            const int64_t nb = (xe - eb < NT) ? xe - eb : NT;
            const int64_t tot = row_segments<NT>(a.X, a.Y, eb, nb, seg_s, seg_o, sw);
            if (tot < kWalkMax)
                walk_products_any<NT, kHashUnroll>(a.Y, seg_o, seg_s, (int32_t)tot, a.X.val ? a.X.val + eb : nullptr,
                                      [&](int32_t j, uint64_t v) {
                                          const uint32_t h = hash_find<S>(keys, j, &a.hdr->fault);
                                          acc_add(&vals[h], satw, h, v);
                                      }, (int)nb);
            else
                accumulate_hash<S>(a.X, a.Y, eb, eb + nb, threadIdx.x >> 6, NT / 64, threadIdx.x & 63, 64, keys,
                                   vals, satw, &a.hdr->fault);
            __syncthreads();
        }
        // compact the occupied slots to the front (each thread's slots pass
        // through registers), then sort them
        constexpr int PER = S / NT;
        int32_t kk[PER];
        unsigned long long vv[PER];
        int64_t local = 0;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int t = q * NT + threadIdx.x;
            kk[q] = keys[t];
            vv[q] = vals[t];
            if (kk[q] != kEmptyKey) {
                ++local;
                if ((satw[t >> 5] >> (t & 31)) & 1u) vv[q] = kSat;
            }
        }
        int64_t tot64;
        int64_t pos = block_inclusive_scan(local, sw, &tot64) - local;  // its barriers order reads before writes
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (kk[q] != kEmptyKey) {
                keys[pos] = kk[q];
                vals[pos] = vv[q];
                ++pos;
            }
        }
        const int total = (int)tot64;
        __syncthreads();
        const int so = merge_sort_block<S, NT>(keys, vals, total);
        const int64_t off = a.slot_off[c];
        bool sat = false;
        for (int t = threadIdx.x; t < total; t += NT) {
            a.slot_col[off + t] = keys[so + t];
            unsigned long long v = vals[so + t];
            a.slot_val[off + t] = v;
            sat |= (v & kSat) != 0;
        }
        __syncthreads();
        for (int t = threadIdx.x; t < S; t += NT) {  // the whole table back to empty
            keys[t] = kEmptyKey;
            vals[t] = 0;
        }
        if (sat) any_sat = 1;
        for (int t = threadIdx.x; t < S / 32; t += NT) satw[t] = 0;
        __syncthreads();
        if (threadIdx.x == 0) {
            const int64_t sb = a.seg_base[c];
            a.seg_cnt[sb] = total;
            a.seg_src[sb] = off;
            a.row_nnz[i] = total;
            if (any_sat) atomicOr(&a.hdr->saturated, 1);
            any_sat = 0;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// numeric: dense LDS tiles over column ranges

// Write one dense LDS tile (columns c0 .. c0+kTileW) of row i in column order
// into the row's slots, then clear it.  A slot is present when its
// accumulator is non-zero or its saturation bit is set (every contribution is
// at least 1; a saturated one only sets the bit).  Each wavefront handles
// groups of 64 consecutive slots, one slot per lane: a ballot gives the
// group's presence mask, a block scan of the group counts gives positions,
// and lanes write consecutive outputs.  gcnt holds kTileW/64 int32.  The
// tile's entries go at `base` within the row's slots when base >= 0, else at
// a position taken from the row's cursor.  Every thread of the block calls it.
__device__ void emit_dense_tile(const NumericArgs &a, int32_t c, int64_t i, int64_t t, int64_t c0,
                                unsigned long long *acc, uint32_t *satw, int32_t *gcnt, int64_t *sw,
                                int64_t *s_base, int *s_sat, int64_t base = -1) {
    constexpr int NG = kTileW / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    for (int g = wave; g < NG; g += nwaves) {
        const int slot = g * 64 + lane;
        const bool pr = acc[slot] != 0 || ((satw[slot >> 5] >> (slot & 31)) & 1u);
        const uint64_t m = __ballot(pr);
        if (lane == 0) gcnt[g] = __popcll(m);
    }
    __syncthreads();
    int64_t x = 0;
    for (int g = tid; g < NG; g += blockDim.x) x += gcnt[g];  // NG <= blockDim: one group per thread
    int64_t tot;
    const int64_t inc = block_inclusive_scan(x, sw, &tot);
    if (tid < NG) gcnt[tid] = (int32_t)(inc - x);
    if (tid == 0 && base < 0)
        *s_base = tot > 0 ? (int64_t)atomicAdd((unsigned long long *)&a.row_cursor[c], (unsigned long long)tot) : 0;
    __syncthreads();
    if (tot > 0) {
        const int64_t off = a.slot_off[c] + (base >= 0 ? base : *s_base);
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        bool sat = false;
        for (int g = wave; g < NG; g += nwaves) {
            const int slot = g * 64 + lane;
            const unsigned long long v = acc[slot];
            const bool sb = (satw[slot >> 5] >> (slot & 31)) & 1u;
            const bool pr = v != 0 || sb;
            const uint64_t m = __ballot(pr);
            if (pr) {
                const int64_t pos = off + gcnt[g] + __popcll(m & lt);
                const unsigned long long out = sb ? kSat : v;
                sat |= sb;
                a.slot_col[pos] = (int32_t)(c0 + slot);
                a.slot_val[pos] = out;
                acc[slot] = 0;
            }
        }
        for (int w = tid; w < kTileW / 32; w += blockDim.x) satw[w] = 0;
        if (sat) *s_sat = 1;
        if (tid == 0) {
            const int64_t sg = a.seg_base[c] + t;
            a.seg_cnt[sg] = tot;
            a.seg_src[sg] = off;
            atomicAdd((unsigned long long *)&a.row_nnz[i], (unsigned long long)tot);
        }
    }
}

// As emit_dense_tile, for a sparse tile whose present slots are marked in the
// bitmap pres (one bit per column): one thread per bitmap word, the word's
// entries written in column order; pres is cleared.
__device__ void emit_sparse_tile(const NumericArgs &a, int32_t c, int64_t i, int64_t t, int64_t c0,
                                 unsigned long long *acc, uint32_t *pres, uint32_t *satw, int64_t *sw,
                                 int64_t *s_base, int *s_sat) {
    constexpr int NW = kTileW / 32;
    const int tid = threadIdx.x;
    const uint32_t word = tid < NW ? pres[tid] : 0u;
    const int64_t cntw = __popc(word);
    int64_t tot;
    const int64_t inc = block_inclusive_scan(cntw, sw, &tot);
    if (tid == 0)
        *s_base = tot > 0 ? (int64_t)atomicAdd((unsigned long long *)&a.row_cursor[c], (unsigned long long)tot) : 0;
    __syncthreads();
    if (tot > 0) {
        const int64_t off = a.slot_off[c] + *s_base;
        int64_t pos = off + inc - cntw;
        bool sat = false;
        if (tid < NW) {
            const uint32_t sbits = satw[tid];
            uint32_t wbits = word;
            while (wbits) {
                const int b = __builtin_ctz(wbits);
                wbits &= wbits - 1;
                const int slot = tid * 32 + b;
                const bool sb = (sbits >> b) & 1u;
                sat |= sb;
                a.slot_col[pos] = (int32_t)(c0 + slot);
                a.slot_val[pos] = sb ? kSat : acc[slot];
                ++pos;
                acc[slot] = 0;
            }
            pres[tid] = 0;
            satw[tid] = 0;
        }
        if (sat) *s_sat = 1;
        if (tid == 0) {
            const int64_t sg = a.seg_base[c] + t;
            a.seg_cnt[sg] = tot;
            a.seg_src[sg] = off;
            atomicAdd((unsigned long long *)&a.row_nnz[i], (unsigned long long)tot);
        }
    }
}

// Split rows: add this workgroup's partial tile into the tile's global
// accumulator (device-scope atomics; a partial is exact below 2^63, so the
// first crossing of 2^63 is seen by the adding workgroup, as in acc_add),
// clear the LDS tile, and let the last of the ks workgroups emit the tile in
// column order from the global accumulator.
__device__ void flush_split_tile(const NumericArgs &a, int64_t gt, int64_t ks, int32_t c, int64_t i, int64_t t,
                                 int64_t c0, unsigned long long *acc, uint32_t *satw, int32_t *gcnt, int64_t *sw,
                                 int64_t *s_base, int *s_sat, int *s_last) {
    constexpr int NG = kTileW / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    unsigned long long *gacc = a.split_acc + gt * kTileW;
    uint32_t *gsat = a.split_sat + gt * (kTileW / 32);
    for (int g = wave; g < NG; g += nwaves) {
        const int slot = g * 64 + lane;
        const unsigned long long v = acc[slot];
        const bool sb = (satw[slot >> 5] >> (slot & 31)) & 1u;
        if (sb) {
            atomicOr(&gsat[slot >> 5], 1u << (slot & 31));
        } else if (v) {
            const unsigned long long old = atomicAdd(&gacc[slot], v);
            if (old < kSat && old + v >= kSat) atomicOr(&gsat[slot >> 5], 1u << (slot & 31));
        }
        acc[slot] = 0;
    }
    for (int w = tid; w < kTileW / 32; w += blockDim.x) satw[w] = 0;
    __threadfence();
    __syncthreads();
    if (tid == 0) {
        const int done = atomicAdd(&a.split_done[gt], 1);
        *s_last = (done == ks - 1);
    }
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
    // last workgroup: emit from the global accumulator
    for (int g = wave; g < NG; g += nwaves) {
        const int slot = g * 64 + lane;
        const unsigned long long v = __hip_atomic_load(&gacc[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t sw32 = __hip_atomic_load(&gsat[slot >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool pr = v != 0 || ((sw32 >> (slot & 31)) & 1u);
        const uint64_t m = __ballot(pr);
        if (lane == 0) gcnt[g] = __popcll(m);
    }
    __syncthreads();
    const int64_t x = tid < NG ? gcnt[tid] : 0;
    int64_t tot;
    const int64_t inc = block_inclusive_scan(x, sw, &tot);
    if (tid < NG) gcnt[tid] = (int32_t)(inc - x);
    if (tid == 0)
        *s_base = tot > 0 ? (int64_t)atomicAdd((unsigned long long *)&a.row_cursor[c], (unsigned long long)tot) : 0;
    __syncthreads();
    if (tot > 0) {
        const int64_t off = a.slot_off[c] + *s_base;
        const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        bool sat = false;
        for (int g = wave; g < NG; g += nwaves) {
            const int slot = g * 64 + lane;
            const unsigned long long v = __hip_atomic_load(&gacc[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t sw32 = __hip_atomic_load(&gsat[slot >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool sb = (sw32 >> (slot & 31)) & 1u;
            const bool pr = v != 0 || sb;
            const uint64_t m = __ballot(pr);
            if (pr) {
                const int64_t pos = off + gcnt[g] + __popcll(m & lt);
                sat |= sb;
                a.slot_col[pos] = (int32_t)(c0 + slot);
                a.slot_val[pos] = sb ? kSat : v;
            }
        }
        if (sat) *s_sat = 1;
        if (tid == 0) {
            const int64_t sg = a.seg_base[c] + t;
            a.seg_cnt[sg] = tot;
            a.seg_src[sg] = off;
            atomicAdd((unsigned long long *)&a.row_nnz[i], (unsigned long long)tot);
        }
    }
}

// Sparse parts (columns [c0p, c1p) of one row, at most kPartMaxTiles tiles
// and kRankCap products) are accumulated by column rank in the tile memory:
// a presence bitmap over the part's columns (marked by a first walk of the
// products), each bitmap word's rank (present columns in the words before
// it, a block scan of the words' popcounts), and one value slot per present
// column in column order, which a second walk adds into.  No probing, and
// emission is in column order by construction.  The memory is left all zero.
constexpr int kRankWrOff = kPartMaxTiles * kTileW / 64;         // u64 words of the bitmap
constexpr int kRankValOff = kRankWrOff + kPartMaxTiles * kTileW / 128;  // ... then u16 word ranks
static_assert(kRankValOff + kRankCap <= kTileW, "rank parts fit the tile memory");
static_assert(kRankCap <= 65535 && kRankCap <= kTileW, "word ranks and saturation bits");

// Word ranks of a marked bitmap of nwords words (every thread of the block
// calls it); returns the number of present columns.
template <int NT>
__device__ int64_t rank_words(const uint32_t *bm, uint16_t *wr, int nwords, int64_t *sw) {
    const int tid = threadIdx.x;
    const int wpt = (nwords + NT - 1) / NT;  // words per thread, contiguous
    const int w0 = tid * wpt, w1 = (w0 + wpt < nwords) ? w0 + wpt : nwords;
    int64_t local = 0;
    for (int w = w0; w < w1; ++w) local += __popc(bm[w]);
    int64_t cnt;
    int64_t run = block_inclusive_scan(local, sw, &cnt) - local;
    for (int w = w0; w < w1; ++w) {
        wr[w] = (uint16_t)run;
        run += __popc(bm[w]);
    }
    __syncthreads();
    return cnt;
}

// Value slot of part column r (marked in the bitmap)
__device__ __forceinline__ uint32_t rank_of(const uint32_t *bm, const uint16_t *wr, int64_t r) {
    const int w = (int)(r >> 5);
    return (uint32_t)wr[w] + (uint32_t)__popc(bm[w] & ((1u << (r & 31)) - 1u));
}

// Emit a sparse part of row i (candidate c): its cnt present columns in
// column order, as one segment at tile t0.  The entries go at `base` within
// the row's slots when base >= 0, else at a position taken from the row's
// cursor.  Bitmap words, word ranks, values and saturation bits are cleared
// as they are emitted.  Every thread of the block calls it.
template <int NT>
__device__ void emit_rank_part(const NumericArgs &a, int32_t c, int64_t i, int64_t t0, int64_t c0p, int nwords,
                               int64_t cnt, uint32_t *bm, uint16_t *wr, unsigned long long *vals, uint32_t *satw,
                               int64_t *s_base, int *s_sat, int64_t base) {
    const int tid = threadIdx.x;
    if (tid == 0 && base < 0)
        *s_base = cnt > 0 ? (int64_t)atomicAdd((unsigned long long *)&a.row_cursor[c], (unsigned long long)cnt) : 0;
    __syncthreads();
    const int64_t off = a.slot_off[c] + (base >= 0 ? base : *s_base);
    const int wpt = (nwords + NT - 1) / NT;
    const int w0 = tid * wpt, w1 = (w0 + wpt < nwords) ? w0 + wpt : nwords;
    bool sat = false;
    for (int w = w0; w < w1; ++w) {
        uint32_t bits = bm[w];
        uint32_t k = wr[w];
        while (bits) {
            const int b = __builtin_ctz(bits);
            bits &= bits - 1;
            const bool sb = (satw[k >> 5] >> (k & 31)) & 1u;
            sat |= sb;
            a.slot_col[off + k] = (int32_t)(c0p + (int64_t)w * 32 + b);
            a.slot_val[off + k] = sb ? kSat : vals[k];
            vals[k] = 0;
            if (sb) atomicAnd(&satw[k >> 5], ~(1u << (k & 31)));
            ++k;
        }
        bm[w] = 0;
        wr[w] = 0;
    }
    if (sat) *s_sat = 1;
    if (tid == 0 && cnt > 0) {
        const int64_t sg = a.seg_base[c] + t0;
        a.seg_cnt[sg] = cnt;
        a.seg_src[sg] = off;
        atomicAdd((unsigned long long *)&a.row_nnz[i], (unsigned long long)cnt);
    }
    __syncthreads();
}

// One task = one row and a part of m consecutive column tiles.  Each left
// entry's segment of its right row inside the part is located (from the right
// operand's tile index when there is one, else by binary search or the row
// start), the segment lengths are block-scanned, and:
//  * a part with at most part_hash_cap products is accumulated by column
//    rank (a presence bitmap over the part's columns, word ranks, one value
//    slot per present column), overlaid on the tile memory;
//  * otherwise the part is walked tile by tile: per tile the segments are
//    found again (cursors carried between tiles when the row's entries fit one
//    batch and there is no tile index), and the flattened products are shared
//    evenly by the wavefronts into a dense LDS tile.
// Left entries are taken in batches of kDenseThreads.
__global__ __launch_bounds__(kDenseThreads, 4) void k_dense(const int32_t *list, int64_t n_list, const int64_t *task_base,
                                                         int64_t n_tasks, NumericArgs a) {
    constexpr int W = kTileW;
    constexpr int NW = W / 32;
    constexpr int NT = kDenseThreads;
    __shared__ unsigned long long acc[W];
    __shared__ uint32_t satw[NW];
    __shared__ int64_t cur[kCursorCap];  // next segment start per entry (single-batch rows)
    __shared__ int64_t seg_s[NT];        // segment start of each entry of the batch
    __shared__ int32_t seg_l[NT];        // segment length (first: remaining row length)
    __shared__ int32_t seg_o[NT + 1];    // exclusive scan of segment lengths
    __shared__ int64_t sw[NT / 64];
    __shared__ int64_t s_task[4];
    __shared__ int64_t s_base;
    __shared__ int s_sat;
    __shared__ int s_last;
    const int tid = threadIdx.x;
    for (int t = tid; t < W; t += NT) acc[t] = 0;
    for (int t = tid; t < NW; t += NT) satw[t] = 0;
    if (tid == 0) s_sat = 0;
    __syncthreads();
    const int64_t ycols = a.ycols;
    const int64_t ntiles = (ycols + W - 1) / W;
    // bound of every product value (an operand without values holds ones; one
    // without a known bound gives 2^63).  A row of nop products, each at most
    // vm, cannot bring any column to 2^63 when nop * vm < 2^63: its tiles add
    // without the returning atomic of the saturation check.
    const uint64_t xm = a.X.val ? (a.X.vmax ? *a.X.vmax : kSat) : 1;
    const uint64_t ym = a.Y.val ? (a.Y.vmax ? *a.Y.vmax : kSat) : 1;
    const uint64_t vm = sat_mul(xm, ym);

    // segments of the batch starting at eb over columns [c0, c1); start from
    // cur[] when from_cursor.  The bound searches are shared out to groups of
    // lanes (all 512 threads on few entries, one thread per entry on many).
    // Returns the batch's product count (block-uniform).
    // With the tile index, a row of at most NT entries keeps each entry's
    // right row (column id and row start, or -1 when X's column mask drops
    // it) in ent_k / ent_b for the whole task (the cursor memory, unused then).
    static_assert(kCursorCap >= NT, "the kept entries overlay the cursor memory");
    int32_t *ent_k = reinterpret_cast<int32_t *>(cur);
    int32_t *ent_b = ent_k + NT;
    auto segments = [&](int64_t xb, int64_t xlen, int64_t eb, int64_t c0, int64_t c1, bool from_cursor,
                        bool keep_cursor) -> int64_t {
        const int64_t nb = (xlen - eb < NT) ? xlen - eb : NT;
        if (a.ytile) {  // the right operand's tile index gives both bounds directly
            if (tid < nb) {
                int32_t k;
                int64_t yb;
                if (from_cursor) {  // entries kept for the task
                    k = ent_k[tid];
                    yb = ent_b[tid];
                } else {
                    k = a.X.col[xb + eb + tid];
                    if (a.X.cmask && !bit_test(a.X.cmask, k)) k = -1;
                    yb = k >= 0 ? a.Y.rp[k] : 0;
                }
                if (k < 0) {
                    seg_s[tid] = 0;
                    seg_l[tid] = 0;
                } else {
                    const int32_t *yt = a.ytile + (int64_t)k * (ntiles + 1);
                    const int32_t lo = yt[c0 >> kTileShift], hi = yt[(c1 + W - 1) >> kTileShift];
                    seg_s[tid] = yb + lo;
                    seg_l[tid] = hi - lo;
                }
            }
            __syncthreads();
            const int64_t len = tid < nb ? seg_l[tid] : 0;
            int64_t tot;
            const int64_t inc = block_inclusive_scan(len, sw, &tot);
            seg_o[tid] = (int32_t)(inc - len);
            if (tid == NT - 1) seg_o[NT] = (int32_t)inc;
            __syncthreads();
            return tot;
        }
        if (tid < nb) {
            const int64_t e = eb + tid;
            const int32_t k = a.X.col[xb + e];
            if (a.X.cmask && !bit_test(a.X.cmask, k)) {
                seg_s[tid] = 0;
                seg_l[tid] = 0;
            } else {
                const int64_t yb = a.Y.rp[k], ye = a.Y.rp[k + 1];
                const int64_t s0 = from_cursor ? cur[e] : yb;
                seg_s[tid] = s0;
                seg_l[tid] = (int32_t)(ye - s0);
            }
        }
        __syncthreads();
        int g = 64;
        while (g > 1 && (int64_t)(NT / g) < nb) g >>= 1;
        const int li = tid & (g - 1);
        const int64_t ngroups = NT / g;
        const uint64_t gm = group_mask(g);
        if (!from_cursor && c0 > 0) {
            for (int64_t x = tid / g; x < nb; x += ngroups) {
                const int64_t lo = seg_s[x], hi = lo + seg_l[x];
                const int64_t r = group_lower_bound(a.Y.col, lo, hi, (int32_t)c0, g, li, gm);
                if (li == 0) {
                    seg_s[x] = r;
                    seg_l[x] = (int32_t)(hi - r);
                }
            }
            __syncthreads();
        }
        if (c1 < ycols) {
            for (int64_t x = tid / g; x < nb; x += ngroups) {
                const int64_t lo = seg_s[x], hi = lo + seg_l[x];
                const int64_t r = group_lower_bound(a.Y.col, lo, hi, (int32_t)c1, g, li, gm);
                if (li == 0) seg_l[x] = (int32_t)(r - lo);
            }
            __syncthreads();
        }
        const int64_t len = tid < nb ? seg_l[tid] : 0;
        if (keep_cursor && tid < nb) cur[eb + tid] = seg_s[tid] + len;
        int64_t tot;
        const int64_t inc = block_inclusive_scan(len, sw, &tot);
        seg_o[tid] = (int32_t)(inc - len);
        if (tid == NT - 1) seg_o[NT] = (int32_t)inc;
        __syncthreads();
        return tot;
    };
    // visit the flattened products of the current batch: f(column, value)
    auto products = [&](int64_t tot, int64_t nb, const uint64_t *xval, bool plain, auto f) {
        walk_products_any<NT>(a.Y, seg_o, seg_s, (int32_t)tot, xval, f, nb < NT ? (int)nb : NT, plain);
    };

    // tasks from the dense queue (rows of very different cost stay balanced)
    QueueCursor qc = queue_start();
    while (true) {
        const int64_t task = block_next_task(a.dense_queue, n_tasks, qc, &s_task[3]);
        if (task < 0) break;
        if (tid < 64) {  // last p with task_base[p] <= task, by the first wavefront
            const int64_t pp = group_lower_bound(task_base, 0, n_list, task + 1, 64, tid, ~0ull) - 1;
            if (tid == 0) {
                s_task[0] = pp;
                s_task[1] = task - task_base[pp];
            }
        }
        __syncthreads();
        const int64_t p = s_task[0], qq = s_task[1];
        const int64_t sp = a.dense_split[p];
        const int64_t ks = sp & 255;
        const int64_t sslot = ks > 1 ? sp >> 8 : 0;
        const int64_t m = ks > 1 ? 1 : sp >> 16;           // tiles per part
        const int64_t grp = ks > 1 ? 1 : (sp >> 8) & 255;  // parts per task
        const int64_t nparts = (ntiles + m - 1) / m;
        const int64_t q = qq / ks, r = qq % ks;  // task of the row, split
        const int32_t c = list[p];
        const int64_t i = a.cand ? a.cand[c] : c;
        int64_t xb = a.X.rp[i], xlen = a.X.rp[i + 1] - xb;
        if (ks > 1) {  // this workgroup's share of the left entries
            const int64_t per = (xlen + ks - 1) / ks;
            const int64_t e0 = r * per, e1 = (e0 + per < xlen) ? e0 + per : xlen;
            xb += e0 < xlen ? e0 : xlen;
            xlen = e1 > e0 ? e1 - e0 : 0;
        }
        const int64_t pa = q * grp, pb = (pa + grp < nparts) ? pa + grp : nparts;
        if (pa >= pb) continue;  // block-uniform
        const bool single = xlen <= NT;
        const int64_t nop_c = a.nop[c];
        // Where the row's parts write: the row has ub = min(products, usable
        // columns) slots.  With a slot per column of Y, a part's entries go
        // at its first column; with a slot per product (and the tile index),
        // at the row's products in tiles below the part, which bound the
        // entries before it; otherwise at a position taken from the row's
        // cursor.  Every task of a row takes the same choice.
        const int64_t cap = a.slot_off[c + 1] - a.slot_off[c];
        const int mode = ks > 1 ? 0 : cap >= ycols ? 1 : (a.ytile && cap >= nop_c) ? 2 : 0;
        const bool keep = a.ytile && single;  // the row's entries kept for the task
        const bool no_sat = sat_mul(vm, (uint64_t)nop_c) < kSat;  // plain adds (see vm)
        int64_t pbase = 0;  // mode 2: the row's products in tiles below the current part
        if (keep) {  // (with the prefix of mode 2 from the same round of loads)
            int64_t lo = 0;
            if (tid < xlen) {
                int32_t k = a.X.col[xb + tid];
                if (a.X.cmask && !bit_test(a.X.cmask, k)) k = -1;
                ent_k[tid] = k;
                ent_b[tid] = k >= 0 ? (int32_t)a.Y.rp[k] : 0;
                if (mode == 2 && pa > 0 && k >= 0) lo = a.ytile[(int64_t)k * (ntiles + 1) + pa * m];
            }
            if (mode == 2 && pa > 0) block_inclusive_scan(lo, sw, &pbase);
            __syncthreads();
        } else if (mode == 2 && pa > 0) {
            const int64_t tb = pa * m;
            for (int64_t eb = 0; eb < xlen; eb += NT) {
                int64_t lo = 0;
                if (eb + tid < xlen) {
                    const int32_t k = a.X.col[xb + eb + tid];
                    if (!(a.X.cmask && !bit_test(a.X.cmask, k))) lo = a.ytile[(int64_t)k * (ntiles + 1) + tb];
                }
                int64_t tot;
                block_inclusive_scan(lo, sw, &tot);
                pbase += tot;
                __syncthreads();
            }
        }

        for (int64_t part = pa; part < pb; ++part) {
            const int64_t t0 = part * m;
            const int64_t t1 = (t0 + m < ntiles) ? t0 + m : ntiles;
            const int64_t c0p = t0 * W, c1p = (t1 * W < ycols) ? t1 * W : ycols;

            // part-level product count, when the part may be sparse enough to
            // go by column rank (a row whose mean part holds more than twice
            // the rank capacity goes straight to the dense tiles)
            const bool may_rank = ks == 1 && (c1p - c0p) <= (int64_t)kPartMaxTiles * W &&
                                  nop_c <= 2 * a.tune.part_hash_cap * nparts;
            int64_t ltot = 0;
            if (may_rank) {
                for (int64_t eb = 0; eb < xlen; eb += NT) ltot += segments(xb, xlen, eb, c0p, c1p, keep, false);
                if (ltot == 0) continue;
            }

            if (may_rank && ltot <= a.tune.part_hash_cap) {
                // sparse part, accumulated by column rank: mark, rank the words, add
                const int nwords = (int)((c1p - c0p + 31) / 32);
                uint32_t *bm = reinterpret_cast<uint32_t *>(acc);
                uint16_t *wr = reinterpret_cast<uint16_t *>(acc + kRankWrOff);
                unsigned long long *vals = acc + kRankValOff;
                for (int64_t eb = 0; eb < xlen; eb += NT) {
                    const int64_t tot = single ? ltot : segments(xb, xlen, eb, c0p, c1p, false, false);
                    const int nb = (int)(xlen - eb < NT ? xlen - eb : NT);
                    walk_products<false, false, NT, kProdUnroll>(a.Y, seg_o, seg_s, (int32_t)tot, nullptr,
                                                                 [&](int32_t j, uint64_t) {
                                                                     const int64_t r = j - c0p;
                                                                     atomicOr(&bm[r >> 5], 1u << (r & 31));
                                                                 }, nb);
                    __syncthreads();
                }
                const int64_t cnt = rank_words<NT>(bm, wr, nwords, sw);
                for (int64_t eb = 0; eb < xlen; eb += NT) {
                    const int64_t tot = single ? ltot : segments(xb, xlen, eb, c0p, c1p, false, false);
                    const uint64_t *xval = a.X.val ? a.X.val + xb + eb : nullptr;
                    products(tot, xlen - eb, xval, no_sat, [&](int32_t j, uint64_t v) {
                        const uint32_t k = rank_of(bm, wr, j - c0p);
                        acc_add(&vals[k], satw, k, v);
                    });
                    __syncthreads();
                }
                emit_rank_part<NT>(a, c, i, t0, c0p, nwords, cnt, bm, wr, vals, satw, &s_base, &s_sat,
                                   mode == 1 ? c0p : mode == 2 ? pbase : -1);
                pbase += ltot;
                continue;
            }

            // dense part: tile by tile (cursors only without the tile index)
            const bool cursors = single && !a.ytile;
            if (cursors) {  // cursors at the part start
                for (int64_t e = tid; e < xlen; e += NT) {
                    int32_t k = a.X.col[xb + e];
                    cur[e] = a.Y.rp[k];
                }
                __syncthreads();
                if (c0p > 0) {
                    int g = 64;
                    while (g > 1 && (int64_t)(NT / g) < xlen) g >>= 1;
                    const int li = tid & (g - 1);
                    const uint64_t gm = group_mask(g);
                    for (int64_t x = tid / g; x < xlen; x += NT / g) {
                        const int32_t k = a.X.col[xb + x];
                        const int64_t r = group_lower_bound(a.Y.col, a.Y.rp[k], a.Y.rp[k + 1], (int32_t)c0p, g, li, gm);
                        if (li == 0) cur[x] = r;
                    }
                    __syncthreads();
                }
            }
            for (int64_t t = t0; t < t1; ++t) {
                const int64_t c0 = t * W;
                const int64_t c1 = (c0 + W < ycols) ? c0 + W : ycols;
                int64_t ttot = 0;
                for (int64_t eb = 0; eb < xlen; eb += NT) {
                    const int64_t tot = segments(xb, xlen, eb, c0, c1, cursors || keep, cursors);
                    ttot += tot;
                    const uint64_t *xval = a.X.val ? a.X.val + xb + eb : nullptr;
                    products(tot, xlen - eb, xval, no_sat, [&](int32_t j, uint64_t v) {
                        const uint32_t slot = (uint32_t)(j - c0);
                        if (no_sat)
                            (void)__hip_atomic_fetch_add(&acc[slot], (unsigned long long)v, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
                        else
                            acc_add(&acc[slot], satw, slot, v);
                    });
                    __syncthreads();
                }
                if (ks == 1) {
                    emit_dense_tile(a, c, i, t, c0, acc, satw, seg_o, sw, &s_base, &s_sat,
                                    mode == 1 ? c0 : mode == 2 ? pbase : -1);
                    pbase += ttot;
                } else {
                    const int64_t gt = sslot * ntiles + t;
                    flush_split_tile(a, gt, ks, c, i, t, c0, acc, satw, seg_o, sw, &s_base, &s_sat, &s_last);
                }
                __syncthreads();
            }
        }
    }
    __syncthreads();
    if (tid == 0 && s_sat) atomicOr(&a.hdr->saturated, 1);
}

// Tile index of a right operand: ytile[k * (ntiles + 1) + t] = entries of
// row k in column tiles below t (so tile t of row k is entries
// [ytile[..t], ytile[..t+1]) from the row start).  One thread per (row,
// boundary): a binary search of the boundary column; consecutive threads
// write consecutive words.
__global__ __launch_bounds__(256) void k_tile_index(Operand Y, int64_t ntiles, int32_t *ytile) {
    const int64_t per = ntiles + 1, n = Y.rows * per;
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t k = idx / per, t = idx - k * per;
        const int64_t yb = Y.rp[k], ye = Y.rp[k + 1];
        int64_t v;
        if (t == 0)
            v = 0;
        else if (t == ntiles)
            v = ye - yb;
        else
            v = lower_bound_col(Y.col, yb, ye, (int32_t)(t << kTileShift)) - yb;
        ytile[idx] = (int32_t)v;
    }
}

// ---------------------------------------------------------------------------
// numeric: tile buckets for rows with very many left-operand entries and many
// column tiles.  Their products are generated once, counting-sorted into
// column-tile buckets, and each bucket is accumulated in a dense LDS tile.

// Last p in [0, n) with base[p] <= key (base[0] <= key), found by the first
// wavefront (a 64-ary search: a few dependent loads instead of log2 n) and
// handed to the workgroup through *slot.  Every thread calls it; the caller
// keeps the slot from being rewritten before every thread has read it.
__device__ __forceinline__ int64_t block_find_row(const int64_t *base, int64_t n, int64_t key, int64_t *slot) {
    if (threadIdx.x < 64) {
        const int64_t p = group_lower_bound(base, 0, n, key + 1, 64, (int)threadIdx.x, ~0ull) - 1;
        if (threadIdx.x == 0) *slot = p;
    }
    __syncthreads();
    return *slot;
}

// Runs of one lane group: consecutive active lanes whose products fall into
// the same column tile (the lanes of a group read consecutive entries of one
// sorted right-operand row, so a row's products in one tile are adjacent).
// Every lane of the group calls it together.
struct TileRun {
    bool head;      // first lane of its run
    int head_lane;  // wavefront lane of the run's head
    int len;        // lanes in the run (valid at the head)
    int rank;       // position within the run
};

__device__ __forceinline__ TileRun tile_run(bool act, int32_t tile, int lane, int g) {
    const int li = lane & (g - 1);
    const int gbase = lane - li;
    const uint64_t gmask = (g == 64 ? ~0ull : ((1ull << g) - 1)) << gbase;
    const int key = act ? tile : -1 - lane;  // an inactive lane matches no neighbour
    const int prev = __shfl_up(key, 1, g);
    const bool head = act && (li == 0 || prev != key);
    const uint64_t hm = __ballot(head) & gmask;
    const uint64_t bound = hm | (~__ballot(act) & gmask);
    TileRun r;
    r.head = head;
    const uint64_t upto = (2ull << lane) - 1;  // lanes 0..lane (all lanes when lane = 63)
    r.head_lane = (act && (hm & upto)) ? 63 - __builtin_clzll(hm & upto) : lane;
    const uint64_t above = bound & ~((2ull << r.head_lane) - 1);
    const int end = above ? __builtin_ctzll(above) : gbase + g;
    r.len = end - r.head_lane;
    r.rank = lane - r.head_lane;
    return r;
}

// Products of X entries [e0, e1) of one row, one X entry per group of g lanes
// (g a power of two); the group walks the right row in steps of g entries so
// that its lanes stay together.  f(act, tile, col, value, run) is called by
// every lane of the group in every step; act = the lane holds a product.
template <typename F>
__device__ __forceinline__ void for_product_runs(const Operand &X, const Operand &Y, int64_t e0, int64_t e1, int g,
                                                 F f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per_wave = 64 / g;
    const int gid = wave * per_wave + lane / g, ng = (blockDim.x / 64) * per_wave, li = lane & (g - 1);
    for (int64_t e = e0 + gid; e < e1; e += ng) {  // uniform within the group
        const int32_t k = X.col[e];
        if (X.cmask && !bit_test(X.cmask, k)) continue;
        const uint64_t xv = X.val ? X.val[e] : 1ull;
        const int64_t yb = Y.rp[k], ye = Y.rp[k + 1];
        for (int64_t base = yb; base < ye; base += g) {
            const int64_t fpos = base + li;
            bool act = fpos < ye;
            const int32_t j = act ? Y.col[fpos] : 0;
            if (act && Y.cmask) act = bit_test(Y.cmask, j);
            const uint64_t v = act ? (Y.val ? sat_mul(xv, Y.val[fpos]) : xv) : 0ull;
            const int32_t tile = j >> kTileShift;
            const TileRun r = tile_run(act, tile, lane, g);
            f(act, tile, j, v, r);
        }
    }
}

// right rows of at least this many lanes' worth of entries are walked in
// tile runs (one LDS atomic per run); shorter rows one product per lane
constexpr int kRunMinLanes = 16;

struct BucketArgs {
    const int32_t *list;        // bucket rows (candidate indices)
    int64_t n_list;
    const int64_t *chunk_base;  // [n_list + 1] X-entry chunks per row
    int64_t n_chunks;
    const int64_t *prod_base;   // [n_list + 1] products per row
    int64_t ntiles;
    int64_t *tile_cnt;          // [n_list * (ntiles + 1)] counts, then cursors
    int64_t *tile_off;          // [n_list * (ntiles + 1)] absolute bucket offsets
    int32_t *prod_col;
    uint64_t *prod_val;
    int g;                      // lanes per left entry (power of two <= 64)
    int64_t *chunk_hist;        // [n_chunks * ntiles] per-chunk tile counts, then bucket bases; or nullptr
    int64_t *part_cnt;          // [n_list] parts per row
    int64_t *part_base;         // [n_list + 1] exclusive scan of part_cnt
};

// tiles per accumulation part of a bucket row with nop products: the part
// target over the row's mean products per tile, at most kPartMaxTiles
__device__ __forceinline__ int64_t bucket_part_tiles(int64_t nop, int64_t ntiles, const Tuning &tune) {
    const int64_t per_tile = nop / ntiles;
    int64_t m = 1;
    if (per_tile < tune.part_target) {
        m = tune.part_target / (per_tile > 0 ? per_tile : 1);
        m = m > kPartMaxTiles ? kPartMaxTiles : (m < 1 ? 1 : m);
    }
    return m;
}

constexpr int kBucketUnroll = 2;  // products per lane per step of the bucket passes' walk

// Products of X entries [e0, e1) of one row, f(column, value) for each: every
// wavefront takes batches of 64 consecutive entries in turn (its batches are
// kBucketThreads entries apart) and walks each batch's products flattened,
// with no workgroup barrier between batches.  The batch set-up is pipelined:
// a batch's left columns are loaded two batches ahead and their column-mask
// words one batch ahead, so that only the right row bounds and the walk's
// gathers wait within a batch.  seg_s holds 64 and seg_o 65 entries per
// wavefront.
template <typename F>
__device__ __forceinline__ void walk_entry_range(const NumericArgs &a, int64_t e0, int64_t e1, int64_t *seg_s,
                                                 int32_t *seg_o, F f) {
    constexpr int64_t B = kBucketThreads;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t *ws = seg_s + wave * 64;
    int32_t *wo = seg_o + wave * 65;
    const uint32_t *cm = a.X.cmask;
    int64_t eb = e0 + (int64_t)wave * 64;
    // stages (an entry past e1 reads column 0, in bounds, and is not used)
    int32_t k0 = eb + lane < e1 ? a.X.col[eb + lane] : 0;          // this batch's columns
    int32_t k1 = eb + B + lane < e1 ? a.X.col[eb + B + lane] : 0;  // the next batch's
    uint32_t w0 = cm ? cm[k0 >> 5] : ~0u;                          // this batch's mask words
    for (; eb < e1; eb += B) {
        const int64_t nb = (e1 - eb < 64) ? e1 - eb : 64;
        const int32_t k = k0;
        const uint32_t w = w0;
        w0 = cm ? cm[k1 >> 5] : ~0u;
        k0 = k1;
        k1 = eb + 2 * B + lane < e1 ? a.X.col[eb + 2 * B + lane] : 0;
        int64_t len = 0;
        if (lane < nb && ((w >> (k & 31)) & 1u)) {
            const int64_t yb = a.Y.rp[k];
            len = a.Y.rp[k + 1] - yb;
            ws[lane] = yb;
        }
        int64_t inc = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        const int64_t tot = __shfl(inc, 63, 64);
        wo[lane] = (int32_t)(inc - len);
        if (lane == 63) wo[64] = (int32_t)inc;
        wave_sync();
        if (tot < kWalkMax) {
            walk_products_any<64, kBucketUnroll>(a.Y, wo, ws, (int32_t)tot, a.X.val ? a.X.val + eb : nullptr, f,
                                                 (int)nb);
        } else {
            for (int64_t e = eb; e < eb + nb; ++e) {
                const int32_t kk = a.X.col[e];
                if (cm && !bit_test(cm, kk)) continue;
                const uint64_t xv = a.X.val ? a.X.val[e] : 1ull;
                for (int64_t fpos = a.Y.rp[kk] + lane; fpos < a.Y.rp[kk + 1]; fpos += 64) {
                    const int32_t j = a.Y.col[fpos];
                    if (a.Y.cmask && !bit_test(a.Y.cmask, j)) continue;
                    f(j, a.Y.val ? sat_mul(xv, a.Y.val[fpos]) : xv);
                }
            }
        }
        wave_sync();
    }
}

__global__ __launch_bounds__(kBucketThreads) void k_bucket_count(BucketArgs b, NumericArgs a) {
    __shared__ int32_t hist[kMaxBucketTiles];
    __shared__ int64_t s_row;
    __shared__ int64_t seg_s[kBucketThreads];
    __shared__ int32_t seg_o[kBucketThreads / 64 * 65];
    for (int64_t id = blockIdx.x; id < b.n_chunks; id += gridDim.x) {  // the body ends with a barrier
        const int64_t p = block_find_row(b.chunk_base, b.n_list, id, &s_row);
        const int64_t q = id - b.chunk_base[p];
        const int32_t c = b.list[p];
        const int64_t i = a.cand ? a.cand[c] : c;
        const int64_t xb = a.X.rp[i], xe = a.X.rp[i + 1];
        const int64_t bc = a.tune.bucket_chunk;
        const int64_t e0 = xb + q * bc, e1 = e0 + bc < xe ? e0 + bc : xe;
        for (int t = threadIdx.x; t < b.ntiles; t += blockDim.x) hist[t] = 0;
        __syncthreads();
        if (b.g >= kRunMinLanes)
            for_product_runs(a.X, a.Y, e0, e1, b.g, [&](bool, int32_t tile, int32_t, uint64_t, const TileRun &r) {
                if (r.head) atomicAdd(&hist[tile], r.len);
            });
        else
            walk_entry_range(a, e0, e1, seg_s, seg_o,
                             [&](int32_t j, uint64_t) { atomicAdd(&hist[j >> kTileShift], 1); });
        __syncthreads();
        int64_t *cnt = b.tile_cnt + p * (b.ntiles + 1);
        for (int t = threadIdx.x; t < b.ntiles; t += blockDim.x) {
            if (hist[t]) atomicAdd((unsigned long long *)&cnt[t], (unsigned long long)hist[t]);
            if (b.chunk_hist) b.chunk_hist[id * b.ntiles + t] = hist[t];
        }
        __syncthreads();
    }
}

// per bucket row: tile_off = prod_base + exclusive scan of the tile counts.
// Without per-chunk counts: one workgroup per row, and the counts become the
// scatter's cursors.  With per-chunk counts, each chunk's count of a tile
// becomes the chunk's base in that bucket (the tile's offset plus the counts
// of the row's earlier chunks): a row's tiles are spread over workgroups of
// kBucketScanThreads tiles (each scans the row's counts up to its own tiles),
// and when a workgroup has fewer tiles than threads, each tile's chunks are
// split over a group of threads (a sum per thread, a scan across the group,
// then a second pass that writes the bases).
constexpr int kBucketScanThreads = 256;
constexpr int kBucketScanLoads = 16;  // chunk counts loaded together

__global__ __launch_bounds__(kBucketScanThreads) void k_bucket_scan(BucketArgs b, Tuning tune) {
    constexpr int NT = kBucketScanThreads, U = kBucketScanLoads;
    __shared__ int64_t sw[NT / 64];
    __shared__ int64_t s_off[NT];
    __shared__ int64_t s_inc[NT];
    const int tid = threadIdx.x;
    const int64_t tbn = b.chunk_hist ? (b.ntiles + NT - 1) / NT : 1;  // workgroups per row
    for (int64_t id = blockIdx.x; id < b.n_list * tbn; id += gridDim.x) {
        const int64_t p = id / tbn, tb = id - p * tbn;
        if (tb == 0 && tid == 0) {
            const int64_t m = bucket_part_tiles(b.prod_base[p + 1] - b.prod_base[p], b.ntiles, tune);
            b.part_cnt[p] = (b.ntiles + m - 1) / m;
        }
        int64_t *cnt = b.tile_cnt + p * (b.ntiles + 1);
        int64_t *off = b.tile_off + p * (b.ntiles + 1);
        // tiles [0, t_end): up to this workgroup's own tiles (all of them in the
        // row's last workgroup, which writes the total)
        const int64_t t_end = (tb == tbn - 1) ? b.ntiles : (tb + 1) * NT;
        int64_t carry = b.prod_base[p];
        for (int64_t base = 0; base < t_end; base += NT) {
            const int64_t t = base + tid;
            const int64_t x = t < b.ntiles ? cnt[t] : 0;
            int64_t tot;
            const int64_t inc = block_inclusive_scan(x, sw, &tot);
            if (base >= tb * NT) {  // own tiles (with one workgroup per row: every pass)
                const int64_t o = carry + inc - x;
                s_off[tid] = o;
                if (t < b.ntiles) {
                    off[t] = o;
                    if (!b.chunk_hist) cnt[t] = o;
                }
            }
            carry += tot;
        }
        if (tb == tbn - 1 && tid == 0) off[b.ntiles] = carry;
        __syncthreads();
        if (b.chunk_hist) {  // tbn > 1 only with chunk counts: s_off holds this workgroup's tiles
            const int64_t q0 = b.chunk_base[p], q1 = b.chunk_base[p + 1], nq = q1 - q0;
            const int64_t own = (b.ntiles - tb * NT < NT) ? b.ntiles - tb * NT : NT;
            int g = 1;  // threads per tile (uniform)
            while (2 * g * own <= NT && 2 * g <= nq) g *= 2;
            const int lt = tid / g, r = tid & (g - 1);
            const bool live = lt < own;
            const int64_t t = tb * NT + lt;
            const int64_t per = (nq + g - 1) / g;
            const int64_t qa = q0 + r * per < q1 ? q0 + r * per : q1;
            const int64_t qz = qa + per < q1 ? qa + per : q1;
            int64_t run = live ? s_off[lt] : 0;
            if (g > 1) {  // the counts of the group's earlier threads
                int64_t sum = 0;
                if (live)
                    for (int64_t q = qa; q < qz; q += U) {
                        int64_t v[U];
#pragma unroll
                        for (int u = 0; u < U; ++u) v[u] = q + u < qz ? b.chunk_hist[(q + u) * b.ntiles + t] : 0;
#pragma unroll
                        for (int u = 0; u < U; ++u) sum += v[u];
                    }
                int64_t tot;
                const int64_t inc = block_inclusive_scan(sum, sw, &tot);
                s_inc[tid] = inc;
                __syncthreads();
                const int g0 = tid & ~(g - 1);
                run += inc - sum - (g0 > 0 ? s_inc[g0 - 1] : 0);
            }
            if (live)
                for (int64_t q = qa; q < qz; q += U) {
                    int64_t v[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) v[u] = q + u < qz ? b.chunk_hist[(q + u) * b.ntiles + t] : 0;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (q + u < qz) b.chunk_hist[(q + u) * b.ntiles + t] = run;
                        run += v[u];
                    }
                }
        }
        __syncthreads();  // LDS reuse by the next row
    }
}

// dynamic LDS: base[ntiles] (int64), then hist[ntiles] (int32), sized to the
// product's tiles (at most kMaxBucketTiles) so that more workgroups fit a CU
__global__ __launch_bounds__(kBucketThreads) void k_bucket_scatter(BucketArgs b, NumericArgs a) {
    extern __shared__ int64_t scatter_lds[];
    int64_t *base = scatter_lds;
    int32_t *hist = reinterpret_cast<int32_t *>(scatter_lds + b.ntiles);
    __shared__ int64_t s_row;
    __shared__ int64_t seg_s[kBucketThreads];
    __shared__ int32_t seg_o[kBucketThreads / 64 * 65];
    for (int64_t id = blockIdx.x; id < b.n_chunks; id += gridDim.x) {  // the body ends with a barrier
        const int64_t p = block_find_row(b.chunk_base, b.n_list, id, &s_row);
        const int64_t q = id - b.chunk_base[p];
        const int32_t c = b.list[p];
        const int64_t i = a.cand ? a.cand[c] : c;
        const int64_t xb = a.X.rp[i], xe = a.X.rp[i + 1];
        const int64_t bc = a.tune.bucket_chunk;
        const int64_t e0 = xb + q * bc, e1 = e0 + bc < xe ? e0 + bc : xe;
        if (b.chunk_hist) {  // the chunk's bucket bases from the scan
            for (int t = threadIdx.x; t < b.ntiles; t += blockDim.x) {
                base[t] = b.chunk_hist[id * b.ntiles + t];
                hist[t] = 0;
            }
            __syncthreads();
        } else {  // count the chunk's products per tile again and reserve its ranges
            for (int t = threadIdx.x; t < b.ntiles; t += blockDim.x) hist[t] = 0;
            __syncthreads();
            if (b.g >= kRunMinLanes)
                for_product_runs(a.X, a.Y, e0, e1, b.g,
                                 [&](bool, int32_t tile, int32_t, uint64_t, const TileRun &r) {
                                     if (r.head) atomicAdd(&hist[tile], r.len);
                                 });
            else
                walk_entry_range(a, e0, e1, seg_s, seg_o,
                                 [&](int32_t j, uint64_t) { atomicAdd(&hist[j >> kTileShift], 1); });
            __syncthreads();
            int64_t *cur = b.tile_cnt + p * (b.ntiles + 1);
            for (int t = threadIdx.x; t < b.ntiles; t += blockDim.x) {
                int32_t h = hist[t];
                base[t] = h ? (int64_t)atomicAdd((unsigned long long *)&cur[t], (unsigned long long)h) : 0;
                hist[t] = 0;
            }
            __syncthreads();
        }
        const bool valued = b.prod_val != nullptr;
        if (b.g >= kRunMinLanes)
            for_product_runs(a.X, a.Y, e0, e1, b.g,
                             [&](bool act, int32_t tile, int32_t j, uint64_t v, const TileRun &r) {
                int32_t at = 0;
                if (r.head) at = atomicAdd(&hist[tile], r.len);
                at = __shfl(at, r.head_lane);  // the run's lanes take consecutive positions
                if (act) {
                    const int64_t pos = base[tile] + at + r.rank;
                    b.prod_col[pos] = j;
                    if (valued) b.prod_val[pos] = v;
                }
            });
        else
            walk_entry_range(a, e0, e1, seg_s, seg_o, [&](int32_t j, uint64_t v) {
                const int32_t tile = j >> kTileShift;
                const int64_t pos = base[tile] + atomicAdd(&hist[tile], 1);
                b.prod_col[pos] = j;
                if (valued) b.prod_val[pos] = v;
            });
        __syncthreads();
    }
}

constexpr int kBucketAccLoads = 4;  // bucket entries per thread loaded together

// f(column, value) for bucket entries [lo, hi), kDenseThreads threads, each
// loading kBucketAccLoads entries before applying them (a heavy row's tile
// holds up to ~10^6 entries, walked by one workgroup); value 1 when !valued.
template <typename F>
__device__ __forceinline__ void bucket_products(const BucketArgs &b, int64_t lo, int64_t hi, bool valued, F f) {
    constexpr int U = kBucketAccLoads;
    for (int64_t e = lo + threadIdx.x; e < hi; e += (int64_t)kDenseThreads * U) {
        int32_t js[U];
        uint64_t vs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t x = e + (int64_t)kDenseThreads * u;
            const int64_t y = x < hi ? x : e;  // past the range: repeat the first (in bounds), not applied
            js[u] = b.prod_col[y];
            vs[u] = valued ? b.prod_val[y] : 1ull;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (e + (int64_t)kDenseThreads * u < hi) f(js[u], vs[u]);
    }
}

__global__ __launch_bounds__(kDenseThreads) void k_bucket_accumulate(BucketArgs b, NumericArgs a) {
    constexpr int W = kTileW;
    constexpr int NW = W / 32;
    __shared__ unsigned long long acc[W];
    __shared__ uint32_t satw[NW];
    __shared__ uint32_t pres[NW];
    __shared__ int32_t gcnt[W / 64];
    __shared__ int64_t sw[kDenseThreads / 64];
    __shared__ int64_t s_base;
    __shared__ int64_t s_rows[2];
    __shared__ int s_sat;
    const int tid = threadIdx.x;
    for (int t = tid; t < W; t += kDenseThreads) acc[t] = 0;
    for (int t = tid; t < NW; t += kDenseThreads) {
        satw[t] = 0;
        pres[t] = 0;
    }
    if (tid == 0) s_sat = 0;
    __syncthreads();
    // one task per part of m consecutive tiles of a row (m from the row's
    // mean products per tile); part_base enumerates them
    const int64_t n_tasks = b.part_base[b.n_list];
    const bool valued = b.prod_val != nullptr;
    int parity = 0;  // the row slot alternates: a task may end without a barrier
    for (int64_t task = blockIdx.x; task < n_tasks; task += gridDim.x, parity ^= 1) {
        const int64_t p = block_find_row(b.part_base, b.n_list, task, &s_rows[parity]);
        const int64_t m = bucket_part_tiles(b.prod_base[p + 1] - b.prod_base[p], b.ntiles, a.tune);
        const int64_t t = (task - b.part_base[p]) * m;
        const int64_t t1 = (t + m < b.ntiles) ? t + m : b.ntiles;
        const int64_t *off = b.tile_off + p * (b.ntiles + 1);
        if (off[t] == off[t1]) continue;  // uniform across the block
        const int32_t c = b.list[p];
        const int64_t i = a.cand ? a.cand[c] : c;
        if (t1 - t > 1 && off[t1] - off[t] <= a.tune.part_hash_cap) {
            // a sparse part, accumulated by column rank (as the dense kernel's sparse parts)
            const int64_t c0p = t * W, c1p = (t1 * W < a.ycols) ? t1 * W : a.ycols;
            const int nwords = (int)((c1p - c0p + 31) / 32);
            uint32_t *bm = reinterpret_cast<uint32_t *>(acc);
            uint16_t *wr = reinterpret_cast<uint16_t *>(acc + kRankWrOff);
            unsigned long long *vals = acc + kRankValOff;
            bucket_products(b, off[t], off[t1], false, [&](int32_t j, uint64_t) {
                const int64_t r = j - c0p;
                atomicOr(&bm[r >> 5], 1u << (r & 31));
            });
            __syncthreads();
            const int64_t cnt = rank_words<kDenseThreads>(bm, wr, nwords, sw);
            bucket_products(b, off[t], off[t1], valued, [&](int32_t j, uint64_t v) {
                const uint32_t k = rank_of(bm, wr, j - c0p);
                acc_add(&vals[k], satw, k, v);
            });
            __syncthreads();
            emit_rank_part<kDenseThreads>(a, c, i, t, c0p, nwords, cnt, bm, wr, vals, satw, &s_base, &s_sat, -1);
            continue;
        }
        for (int64_t tt = t; tt < t1; ++tt) {  // tile by tile
            const int64_t lo = off[tt], hi = off[tt + 1];
            if (lo == hi) continue;  // uniform across the block
            const int64_t c0 = tt * W;
            const bool sparse = (hi - lo) < (int64_t)(W / 4);  // block-uniform
            bucket_products(b, lo, hi, valued, [&](int32_t j, uint64_t v) {
                const uint32_t slot = (uint32_t)(j - c0);
                if (sparse) atomicOr(&pres[slot >> 5], 1u << (slot & 31));
                acc_add(&acc[slot], satw, slot, v);
            });
            __syncthreads();
            if (sparse)
                emit_sparse_tile(a, c, i, tt, c0, acc, pres, satw, sw, &s_base, &s_sat);
            else
                emit_dense_tile(a, c, i, tt, c0, acc, satw, gcnt, sw, &s_base, &s_sat);
            __syncthreads();
        }
    }
    __syncthreads();
    if (tid == 0 && s_sat) atomicOr(&a.hdr->saturated, 1);
}

// ---------------------------------------------------------------------------
// compaction

// Segments of slots -> exact-size arrays; with vmax, also raises *vmax to the
// largest value copied (one atomic per workgroup at most).  256 threads.
__global__ __launch_bounds__(256) void k_copy_segments(const int64_t *__restrict__ seg_cnt,
                                                       const int64_t *__restrict__ seg_src,
                                                       const int64_t *__restrict__ seg_dst, int64_t n_segs,
                                                       const int32_t *__restrict__ slot_col,
                                                       const uint64_t *__restrict__ slot_val,
                                                       int32_t *__restrict__ col, uint64_t *__restrict__ val,
                                                       unsigned long long *vmax) {
    __shared__ unsigned long long s_max[4];
    unsigned long long m = 0;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t sgm = wave; sgm < n_segs; sgm += nwaves) {
        const int64_t n = seg_cnt[sgm];
        if (n == 0) continue;
        const int64_t src = seg_src[sgm], dst = seg_dst[sgm];
        int64_t t = lane;
        for (; t + 192 < n; t += 256) {  // four loads of each array in flight per lane
            int32_t c[4];
            uint64_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = slot_col[src + t + 64 * u];
                v[u] = slot_val[src + t + 64 * u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                col[dst + t + 64 * u] = c[u];
                val[dst + t + 64 * u] = v[u];
                m = v[u] > m ? v[u] : m;
            }
        }
        for (; t < n; t += 64) {
            col[dst + t] = slot_col[src + t];
            const uint64_t v = slot_val[src + t];
            val[dst + t] = v;
            m = v > m ? v : m;
        }
    }
    if (!vmax) return;  // kernel-uniform
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(m, o, 64);
        m = y > m ? y : m;
    }
    if (lane == 0) s_max[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 4; ++w) m = s_max[w] > m ? s_max[w] : m;
        if (m > __hip_atomic_load(vmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(vmax, m);
    }
}

__global__ void k_active_flags(const int32_t *cand, int64_t n_cand, const int64_t *row_nnz, int64_t *flags) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    int64_t i = cand ? cand[c] : c;
    flags[c] = row_nnz[i] > 0 ? 1 : 0;
}

// non-empty rows first (ascending); with `partition` the empty ones follow
// (ascending), so the list has n_cand entries
__global__ void k_active_scatter(const int32_t *cand, int64_t n_cand, const int64_t *scan, int32_t *active,
                                 int partition) {
    int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= n_cand) return;
    const int32_t row = cand ? cand[c] : (int32_t)c;
    if (scan[c + 1] != scan[c])
        active[scan[c]] = row;
    else if (partition)
        active[scan[n_cand] + (c - scan[c])] = row;
}

// *dst += *src (one value; per-query statistics kept on the device)
// a deferred product's step header into the query's totals: nonzeros added,
// fault flag or-ed
__global__ void k_accum_step(const StepHeader *h, int64_t *dst) {
    dst[0] += h->nnz_total;
    dst[1] |= h->fault;
}

// ---------------------------------------------------------------------------
// rows of a fused batch result handed to one member query

// cnt[ids[z]] = length of row ids[z] of R (cnt zeroed; ids ascending, unique)
__global__ void k_gather_count(const int64_t *rrp, const int32_t *ids, int64_t n, int64_t *cnt) {
    for (int64_t z = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; z < n; z += (int64_t)gridDim.x * blockDim.x) {
        const int32_t i = ids[z];
        cnt[i] = rrp[i + 1] - rrp[i];
    }
}

// one wavefront per listed row: copy its entries to the member's row pointers
__global__ __launch_bounds__(256) void k_gather_copy(const int64_t *rrp, const int32_t *rcol, const uint64_t *rval,
                                                     const int32_t *ids, int64_t n, const int64_t *orp,
                                                     int32_t *ocol, uint64_t *oval) {
    const int lane = threadIdx.x & 63;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t z = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; z < n; z += nwaves) {
        const int32_t i = ids[z];
        const int64_t b = rrp[i], len = rrp[i + 1] - b, o = orp[i];
        for (int64_t e = lane; e < len; e += 64) {
            ocol[o + e] = rcol[b + e];
            oval[o + e] = rval[b + e];
        }
    }
}

// ---------------------------------------------------------------------------
// row restriction of a right subtree: the columns that a left operand uses

// bits |= columns of every stored entry of a product (all entries are live)
// nnz_dev (when given) holds the true entry count, nnz its upper bound
__global__ void k_cols_to_bits(const int32_t *col, int64_t nnz, const int64_t *nnz_dev, uint32_t *bits) {
    const int64_t n = nnz_dev ? *nnz_dev : nnz;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = col[e];
        atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
}

// lengths of the candidate rows of a relation (0 for rows outside the row mask)
__global__ void k_cand_lengths(Operand X, const int32_t *cand, int64_t n_cand, int64_t *len) {
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cand; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = cand ? cand[c] : c;
        len[c] = (X.rmask && !bit_test(X.rmask, i)) ? 0 : X.rp[i + 1] - X.rp[i];
    }
}

// bits |= columns of the candidate rows (column mask applied), entries
// flattened over the grid via the exclusive scan of the row lengths
__global__ void k_leaf_cols_to_bits(Operand X, const int32_t *cand, int64_t n_cand, const int64_t *off,
                                    uint32_t *bits) {
    const int64_t total = off[n_cand];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n_cand;  // last row with off <= e
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) >> 1;
            if (off[mid] <= e)
                lo = mid;
            else
                hi = mid;
        }
        const int64_t i = cand ? cand[lo] : lo;
        const int32_t j = X.col[X.rp[i] + (e - off[lo])];
        if (X.cmask && !bit_test(X.cmask, j)) continue;
        atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
}

__global__ void k_word_counts(const uint32_t *bits, int64_t words, int64_t *cnt) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x)
        cnt[w] = __popc(bits[w]);
}

// ascending list of set bits, given the exclusive scan of the word counts
__global__ void k_bits_to_list(const uint32_t *bits, int64_t words, const int64_t *scan, int32_t *list) {
    for (int64_t w = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; w < words; w += (int64_t)gridDim.x * blockDim.x) {
        uint32_t b = bits[w];
        int64_t pos = scan[w];
        while (b) {
            const int k = __builtin_ctz(b);
            b &= b - 1;
            list[pos++] = (int32_t)(w * 32 + k);
        }
    }
}

// ---------------------------------------------------------------------------
// algorithmic-byte accounting (counting mode only, never on the timed path)

// acc[0] rows, acc[1] left-operand entries, acc[2] result entries; marks the
// right-operand rows the bin reads.
__global__ __launch_bounds__(256) void k_bin_stats(const int32_t *list, int64_t n, Operand X, const int32_t *cand,
                                                    const int64_t *row_nnz, uint32_t *ymark, unsigned long long *acc) {
    // one wavefront per row; its lanes stride over the row's entries
    const int lane = threadIdx.x & 63;
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned long long rows = 0, xent = 0, outn = 0;
    for (int64_t r = wave; r < n; r += nwaves) {
        const int32_t c = list[r];
        const int64_t i = cand ? cand[c] : c;
        const int64_t xb = X.rp[i], xe = X.rp[i + 1];
        if (lane == 0) {
            rows += 1;
            xent += (unsigned long long)(xe - xb);
            outn += (unsigned long long)row_nnz[i];
        }
        for (int64_t p = xb + lane; p < xe; p += 64) {
            int32_t k = X.col[p];
            if (X.cmask && !bit_test(X.cmask, k)) continue;
            atomicOr(&ymark[k >> 5], 1u << (k & 31));
        }
    }
    if (rows) {
        atomicAdd(&acc[0], rows);
        atomicAdd(&acc[1], xent);
        atomicAdd(&acc[2], outn);
    }
}

// acc[3] distinct right-operand rows, acc[4] their entries
__global__ void k_mark_bytes(const uint32_t *ymark, const int64_t *yrp, int64_t yrows, unsigned long long *acc) {
    unsigned long long rows = 0, ent = 0;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < yrows; k += (int64_t)gridDim.x * blockDim.x) {
        if (bit_test(ymark, k)) {
            rows += 1;
            ent += (unsigned long long)(yrp[k + 1] - yrp[k]);
        }
    }
    if (rows) {
        atomicAdd(&acc[3], rows);
        atomicAdd(&acc[4], ent);
    }
}

inline int grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    }
    return cus;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

#define ATP_LAUNCH(name, grid, block, stream, ...)                    \
    do {                                                              \
        timer_begin(t, name, stream);                                 \
        hipLaunchKernelGGL(__VA_ARGS__);                              \
        timer_end(t, stream);                                         \
    } while (0)

__global__ void k_post(const int64_t *src, int64_t n, int64_t *dst, uint64_t *flag, uint64_t seq) {
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_post(const int64_t *src, int64_t n, int64_t *dst_host, uint64_t *flag_host, uint64_t seq,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, s, src, n, dst_host, flag_host, seq);
}

void launch_fill_i64(int64_t *p, int64_t n, int64_t v, hipStream_t s, KernelTimer *t) {
    if (n <= 0) return;
    ATP_LAUNCH("fill", 0, 0, s, k_fill_i64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
}

void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s, KernelTimer *t) {
    if (n <= 0) return;
    ATP_LAUNCH("fill", 0, 0, s, k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
}

int64_t scan_tmp_elems(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

int64_t scan_multi_tmp_elems(const ScanJob *jobs, int n_jobs) {
    int64_t n = 0;
    for (int z = 0; z < n_jobs; ++z) n = std::max(n, jobs[z].n);
    return n_jobs * scan_tmp_elems(n);
}

void launch_scan_multi(const ScanJob *jobs, int n_jobs, int64_t *tmp, hipStream_t s, KernelTimer *t) {
    if (n_jobs < 1 || n_jobs > kMaxScanJobs) return;
    ScanJobs sj{};
    int64_t n = 0;
    for (int z = 0; z < n_jobs; ++z) {
        if (jobs[z].n < 0) return;
        sj.job[z] = jobs[z];
        n = std::max(n, jobs[z].n);
    }
    sj.stride = scan_tmp_elems(n);
    const int64_t nb = std::max<int64_t>((n + kScanTile - 1) / kScanTile, 1);
    if (nb <= kSmallScanTiles) {
        ATP_LAUNCH("scan", 0, 0, s, k_scan_small, dim3((unsigned)n_jobs), dim3(kScanThreads), 0, s, sj);
        return;
    }
    ATP_LAUNCH("scan", 0, 0, s, k_scan_reduce, dim3((unsigned)nb, (unsigned)n_jobs), dim3(kScanThreads), 0, s, sj,
               tmp);
    if (nb <= kScanFoldTiles) {
        ATP_LAUNCH("scan", 0, 0, s, k_scan_down_fold, dim3((unsigned)nb, (unsigned)n_jobs), dim3(kScanThreads), 0, s,
                   sj, (const int64_t *)tmp);
        return;
    }
    ATP_LAUNCH("scan", 0, 0, s, k_scan_top, dim3((unsigned)n_jobs), dim3(kScanThreads), 0, s, sj, tmp);
    ATP_LAUNCH("scan", 0, 0, s, k_scan_down, dim3((unsigned)nb, (unsigned)n_jobs), dim3(kScanThreads), 0, s, sj,
               (const int64_t *)tmp);
}

void launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s, KernelTimer *t,
                     int64_t *total) {
    const ScanJob j{in, out, total, n};
    launch_scan_multi(&j, 1, tmp, s, t);
}

// several int64 fills in one launch (job = blockIdx.y)
struct FillJobs {
    FillJob job[kMaxFillJobs];
};
__global__ void k_fill_multi(FillJobs fj) {
    const FillJob &j = fj.job[blockIdx.y];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < j.n; i += (int64_t)gridDim.x * blockDim.x)
        j.p[i] = j.v;
}

void launch_fill_multi(const FillJob *jobs, int n_jobs, hipStream_t s, KernelTimer *t) {
    if (n_jobs < 1 || n_jobs > kMaxFillJobs) return;
    FillJobs fj{};
    int64_t n = 0;
    for (int z = 0; z < n_jobs; ++z) {
        fj.job[z] = jobs[z];
        n = std::max(n, jobs[z].n);
    }
    if (n <= 0) return;
    ATP_LAUNCH("fill", 0, 0, s, k_fill_multi, dim3(grid_for(n, 256, 4096), (unsigned)n_jobs), dim3(256), 0, s, fj);
}

void launch_mask_range(const void *prop, int32_t dtype, int64_t n, int64_t lo, int64_t hi, uint32_t *bits,
                       int and_mode, hipStream_t s, KernelTimer *t) {
    int64_t words = (n + 31) / 32;
    // the kernel strides over the nodes: a capped grid covers any count
    dim3 g(grid_for(((n + 63) / 64) * 64, 256, 4096)), b(256);
    if (dtype == 1)
        ATP_LAUNCH("mask", 0, 0, s, k_mask_range<int16_t>, g, b, 0, s, (const int16_t *)prop, n, lo, hi, bits, words,
                   and_mode);
    else if (dtype == 2)
        ATP_LAUNCH("mask", 0, 0, s, k_mask_range<int32_t>, g, b, 0, s, (const int32_t *)prop, n, lo, hi, bits, words,
                   and_mode);
    else
        ATP_LAUNCH("mask", 0, 0, s, k_mask_range<int64_t>, g, b, 0, s, (const int64_t *)prop, n, lo, hi, bits, words,
                   and_mode);
}

void launch_mask_ids(const int32_t *ids, int64_t n_ids, uint32_t *bits, hipStream_t s, KernelTimer *t) {
    if (n_ids <= 0) return;
    ATP_LAUNCH("mask", 0, 0, s, k_mask_ids, dim3(grid_for(n_ids, 256, 4096)), dim3(256), 0, s, ids, n_ids, bits);
}

void launch_mask_and(uint32_t *dst, const uint32_t *src, int64_t words, hipStream_t s, KernelTimer *t) {
    if (words <= 0) return;
    ATP_LAUNCH("mask", 0, 0, s, k_mask_and, dim3(grid_for(words, 256, 4096)), dim3(256), 0, s, dst, src, words);
}

void launch_popcount(const uint32_t *bits, int64_t words, int64_t *out, hipStream_t s, KernelTimer *t) {
    if (words <= 0) return;
    ATP_LAUNCH("mask", 0, 0, s, k_popcount, dim3(grid_for(words, 256, 2048)), dim3(256), 0, s, bits, words, out);
}

void launch_symbolic(const SymbolicArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.n_cand <= 0) return;
    const int64_t threads = a.n_cand * kSymLanes;
    if ((threads + 255) / 256 > 0x7FFFFFFF) return;
    ATP_LAUNCH("symbolic", 0, 0, s, k_symbolic, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, a);
    launch_scan_i64(a.long_len, a.long_off, a.n_cand, a.scan_tmp, s, t);
    ATP_LAUNCH("symbolic", 0, 0, s, k_symbolic_long, dim3(device_cus() * 8), dim3(256), 0, s, a,
               (const int64_t *)a.long_off);
}

void launch_bin_rows(const SymbolicArgs &a, hipStream_t s, KernelTimer *t) {
    if (a.n_cand <= 0) return;
    ATP_LAUNCH("binning", 0, 0, s, k_bin_rows, dim3((unsigned)((a.n_cand + kBinThreads - 1) / kBinThreads)),
               dim3(kBinThreads), 0, s, a);
}

void launch_numeric_hash(int32_t bin, const int32_t *list, int64_t n, const NumericArgs &a, hipStream_t s,
                         KernelTimer *t) {
    if (n <= 0) return;
    const int cus = device_cus();
    auto waves = [&](int per_block) { return dim3((unsigned)grid_for(n, per_block, (int64_t)cus * 16)); };
    switch (bin) {
        case BIN_W64: ATP_LAUNCH("hash_wave", 0, 0, s, k_hash_wave<64>, waves(4), dim3(256), 0, s, list, n, a); break;
        case BIN_W128: ATP_LAUNCH("hash_wave", 0, 0, s, k_hash_wave<128>, waves(4), dim3(256), 0, s, list, n, a); break;
        case BIN_W256: ATP_LAUNCH("hash_wave", 0, 0, s, k_hash_wave<256>, waves(4), dim3(256), 0, s, list, n, a); break;
        case BIN_W512: ATP_LAUNCH("hash_wave", 0, 0, s, k_hash_wave<512>, waves(4), dim3(256), 0, s, list, n, a); break;
        case BIN_B1024:
            ATP_LAUNCH("hash_block", 0, 0, s, (k_hash_block<1024, 256>), waves(1), dim3(256), 0, s, list, n, a);
            break;
        case BIN_B2048:
            ATP_LAUNCH("hash_block", 0, 0, s, (k_hash_block<2048, 256>), waves(1), dim3(256), 0, s, list, n, a);
            break;
        case BIN_B4096:
            ATP_LAUNCH("hash_block", 0, 0, s, (k_hash_block<4096, 512>), waves(1), dim3(512), 0, s, list, n, a);
            break;
        case BIN_B8192:
            ATP_LAUNCH("hash_block", 0, 0, s, (k_hash_block<8192, 1024>), waves(1), dim3(1024), 0, s, list, n, a);
            break;
        default: break;
    }
}

void launch_numeric_dense(const int32_t *list, int64_t n_list, const int64_t *task_base, int64_t n_tasks,
                          const NumericArgs &a, hipStream_t s, KernelTimer *t) {
    if (n_tasks <= 0) return;
    const int cus = device_cus();
    int64_t g = n_tasks < (int64_t)cus * 2 ? n_tasks : (int64_t)cus * 2;
    ATP_LAUNCH("dense", 0, 0, s, k_dense, dim3((unsigned)g), dim3(kDenseThreads), 0, s, list, n_list, task_base,
               n_tasks, a);
}

void launch_tile_index(const Operand &Y, int64_t ntiles, int32_t *ytile, hipStream_t s, KernelTimer *t) {
    if (Y.rows <= 0) return;
    const int cus = device_cus();
    ATP_LAUNCH("tile_index", 0, 0, s, k_tile_index, dim3(grid_for(Y.rows * (ntiles + 1), 256, (int64_t)cus * 64)),
               dim3(256), 0, s, Y, ntiles, ytile);
}

void launch_numeric_bucket(const int32_t *list, int64_t n_list, const int64_t *chunk_base, int64_t n_chunks,
                           const int64_t *prod_base, int64_t ntiles, int64_t *tile_cnt, int64_t *tile_off,
                           int32_t *prod_col, uint64_t *prod_val, int64_t *chunk_hist, int64_t *parts,
                           const NumericArgs &a, hipStream_t s, KernelTimer *t) {
    if (n_list <= 0 || n_chunks <= 0) return;
    const int64_t yavg = a.Y.rows > 0 ? a.Y.nnz / a.Y.rows : 1;
    BucketArgs b{list, n_list, chunk_base, n_chunks, prod_base, ntiles, tile_cnt, tile_off, prod_col, prod_val,
                 group_size(yavg), chunk_hist, parts, parts + n_list};
    const int cus = device_cus();
    const int64_t gc = n_chunks < (int64_t)cus * 4 ? n_chunks : (int64_t)cus * 4;
    ATP_LAUNCH("bucket", 0, 0, s, k_bucket_count, dim3((unsigned)gc), dim3(kBucketThreads), 0, s, b, a);
    const int64_t gs_n = n_list * (chunk_hist ? (ntiles + kBucketScanThreads - 1) / kBucketScanThreads : 1);
    const int64_t gs = gs_n < (int64_t)cus * 8 ? gs_n : (int64_t)cus * 8;
    ATP_LAUNCH("bucket", 0, 0, s, k_bucket_scan, dim3((unsigned)gs), dim3(kBucketScanThreads), 0, s, b, a.tune);
    launch_scan_i64(b.part_cnt, b.part_base, n_list, b.part_base + n_list + 1, s, t);
    ATP_LAUNCH("bucket", 0, 0, s, k_bucket_scatter, dim3((unsigned)gc), dim3(kBucketThreads),
               (unsigned)(12 * ntiles), s, b, a);
    const int64_t n_tasks = n_list * ntiles;
    const int64_t ga = n_tasks < (int64_t)cus * 2 ? n_tasks : (int64_t)cus * 2;
    ATP_LAUNCH("bucket_acc", 0, 0, s, k_bucket_accumulate, dim3((unsigned)ga), dim3(kDenseThreads), 0, s, b, a);
}

void launch_copy_segments(const int64_t *seg_cnt, const int64_t *seg_src, const int64_t *seg_dst, int64_t n_segs,
                          const int32_t *slot_col, const uint64_t *slot_val, int32_t *col, uint64_t *val,
                          uint64_t *vmax, hipStream_t s, KernelTimer *t) {
    if (n_segs <= 0) return;
    const int cus = device_cus();
    ATP_LAUNCH("copy", 0, 0, s, k_copy_segments, dim3(grid_for(n_segs * 64, 256, (int64_t)cus * 8)), dim3(256), 0, s,
               seg_cnt, seg_src, seg_dst, n_segs, slot_col, slot_val, col, val, (unsigned long long *)vmax);
}

void launch_active_flags(const int32_t *cand, int64_t n_cand, const int64_t *row_nnz, int64_t *flags,
                         hipStream_t s, KernelTimer *t) {
    if (n_cand <= 0) return;
    ATP_LAUNCH("active", 0, 0, s, k_active_flags, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, cand,
               n_cand, row_nnz, flags);
}

void launch_active_scatter(const int32_t *cand, int64_t n_cand, const int64_t *flags_scan, int32_t *active,
                           bool partition, hipStream_t s, KernelTimer *t) {
    if (n_cand <= 0) return;
    ATP_LAUNCH("active", 0, 0, s, k_active_scatter, dim3((unsigned)((n_cand + 255) / 256)), dim3(256), 0, s, cand,
               n_cand, flags_scan, active, partition ? 1 : 0);
}

void launch_accum_step(const StepHeader *h, int64_t *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_accum_step, dim3(1), dim3(1), 0, s, h, dst);
}

void launch_bin_stats(const int32_t *list, int64_t n, const Operand &X, const int32_t *cand, const int64_t *row_nnz,
                      uint32_t *ymark, int64_t *acc, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_bin_stats, dim3(grid_for(n * 64, 256, 4096)), dim3(256), 0, s, list, n, X, cand, row_nnz, ymark,
                       (unsigned long long *)acc);
}

void launch_mark_bytes(const uint32_t *ymark, const int64_t *yrp, int64_t yrows, int64_t *acc, hipStream_t s) {
    if (yrows <= 0) return;
    hipLaunchKernelGGL(k_mark_bytes, dim3(grid_for(yrows, 256, 4096)), dim3(256), 0, s, ymark, yrp, yrows,
                       (unsigned long long *)acc);
}

void launch_cols_to_bits(const int32_t *col, int64_t nnz, const int64_t *nnz_dev, uint32_t *bits, hipStream_t s,
                         KernelTimer *t) {
    if (nnz <= 0) return;
    ATP_LAUNCH("restrict", 0, 0, s, k_cols_to_bits, dim3(grid_for(nnz, 256, 8192)), dim3(256), 0, s, col, nnz, nnz_dev,
               bits);
}

void launch_leaf_cols_to_bits(const Operand &X, const int32_t *cand, int64_t n_cand, int64_t *len, int64_t *off,
                              int64_t *tmp, uint32_t *bits, hipStream_t s, KernelTimer *t) {
    if (n_cand <= 0) return;
    ATP_LAUNCH("restrict", 0, 0, s, k_cand_lengths, dim3(grid_for(n_cand, 256, 8192)), dim3(256), 0, s, X, cand, n_cand,
               len);
    launch_scan_i64(len, off, n_cand, tmp, s, t);
    ATP_LAUNCH("restrict", 0, 0, s, k_leaf_cols_to_bits, dim3(device_cus() * 8), dim3(256), 0, s, X, cand, n_cand,
               (const int64_t *)off, bits);
}

void launch_bits_count(const uint32_t *bits, int64_t words, int64_t *cnt, int64_t *scan, int64_t *tmp, hipStream_t s,
                       KernelTimer *t) {
    if (words <= 0) return;
    ATP_LAUNCH("restrict", 0, 0, s, k_word_counts, dim3(grid_for(words, 256, 8192)), dim3(256), 0, s, bits, words, cnt);
    launch_scan_i64(cnt, scan, words, tmp, s, t);
}

void launch_bits_scatter(const uint32_t *bits, int64_t words, const int64_t *scan, int32_t *list, hipStream_t s,
                         KernelTimer *t) {
    if (words <= 0) return;
    ATP_LAUNCH("restrict", 0, 0, s, k_bits_to_list, dim3(grid_for(words, 256, 8192)), dim3(256), 0, s, bits, words,
               scan, list);
}


void launch_gather_count(const int64_t *rrp, const int32_t *ids, int64_t n, int64_t *cnt, hipStream_t s,
                         KernelTimer *t) {
    if (n <= 0) return;
    ATP_LAUNCH("gather", 0, 0, s, k_gather_count, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, rrp, ids, n, cnt);
}

void launch_gather_copy(const int64_t *rrp, const int32_t *rcol, const uint64_t *rval, const int32_t *ids, int64_t n,
                        const int64_t *orp, int32_t *ocol, uint64_t *oval, hipStream_t s, KernelTimer *t) {
    if (n <= 0) return;
    ATP_LAUNCH("gather", 0, 0, s, k_gather_copy, dim3(grid_for(n * 64, 256, 8192)), dim3(256), 0, s, rrp, rcol, rval,
               ids, n, orp, ocol, oval);
}

}  // namespace atp
