// topk_kernels.hpp -- ranking on the device.  Targets scoring at least the
// threshold are ranked by (score descending, target index ascending); each
// target gets a unique 64-bit key, high word = score with the sign bit
// flipped, low word = bitwise-not of the index, so that the top k keys are
// exactly the k best ranks.
//
// Fast path (exact): the scoring pass leaves the maximum score M; a
// histogram of the scores in the window [M - 2047, M] finds the k-th best
// score T; a collect pass gathers every key with score >= T; one workgroup
// sorts them and keeps the first k.  When the window does not reach the k-th
// best score, or too many keys tie at T to sort in one workgroup, a
// single-workgroup radix select over all keys takes over (never for the
// workloads here, kept so that every input is ranked exactly).
// Every kernel handles one query per blockIdx.y.
#pragma once

#include "device_common.hpp"

namespace hs {

constexpr int kWinBins = 2048;          // histogram window, in score units
constexpr int kSortCap = 8192;          // keys one workgroup sorts in LDS

struct TopkState {
    int32_t max_score;      // written by the scoring pass (atomic max)
    int32_t thr;            // k-th best score T
    int32_t n_sel;          // min(k, eligible targets)
    int32_t fallback;       // 1: the fast path cannot decide, use the radix select
    int32_t count;          // keys gathered by the collect pass
    int32_t min_score;      // eligibility threshold of the query
    int32_t pad_[2];
};

struct DevHit {
    int64_t target_id;
    int32_t score;
    int32_t round;
};

__device__ __forceinline__ uint64_t rank_key(int32_t score, int32_t id) {
    return ((uint64_t)((uint32_t)score ^ 0x80000000u) << 32) | (uint64_t)(~(uint32_t)id);
}
__device__ __forceinline__ int32_t rank_key_score(uint64_t key) {
    return (int32_t)((uint32_t)(key >> 32) ^ 0x80000000u);
}
__device__ __forceinline__ int32_t rank_key_id(uint64_t key) { return (int32_t)(~(uint32_t)key); }

// Per query: state plus histogram.
struct TopkWs {
    TopkState* st;          // [nq]
    uint32_t* hist;         // [nq][kWinBins]
    uint64_t* keys;         // [nq][kSortCap]
};

// Initial ranking state of query q (eligibility threshold min_score), and
// its histogram cleared by the calling workgroup's threads.
__device__ __forceinline__ void topk_state_init(const TopkWs& w, int q, int32_t min_score,
                                                int32_t first, int32_t step) {
    if (first == 0) {
        TopkState s;
        s.max_score = INT32_MIN;
        s.thr = 0;
        s.n_sel = 0;
        s.fallback = 0;
        s.count = 0;
        s.min_score = min_score;
        s.pad_[0] = s.pad_[1] = 0;
        w.st[q] = s;
    }
    uint32_t* h = w.hist + (int64_t)q * kWinBins;
    for (int i = first; i < kWinBins; i += step) h[i] = 0;
}

// Before the scoring pass: reset the state and the histogram of every query
// and, if given, two work counters (ctr[0], ctr[1]).  The threshold is qs[q].kp.min_score for a
// batch, min_score otherwise.
__global__ __launch_bounds__(256) void k_topk_reset(TopkWs w, int32_t min_score,
                                                    const BatchQuery* __restrict__ qs,
                                                    uint32_t* ctr) {
    const int q = blockIdx.y;
    const int32_t first = blockIdx.x * blockDim.x + threadIdx.x;
    topk_state_init(w, q, qs ? qs[q].kp.min_score : min_score, first, gridDim.x * blockDim.x);
    if (first == 0 && ctr && q == 0) {
        ctr[0] = 0;
        ctr[1] = 0;
    }
}

// Histogram of eligible scores within [M - kWinBins + 1, M].
__global__ __launch_bounds__(256) void k_topk_hist(const int32_t* __restrict__ scores, int64_t stride,
                                                   int32_t n, TopkWs w) {
    __shared__ uint32_t h[kWinBins];
    const int q = blockIdx.y;
    const int32_t* sc = scores + (int64_t)q * stride;
    const int32_t M = w.st[q].max_score;
    const int32_t min_score = w.st[q].min_score;
    for (int i = threadIdx.x; i < kWinBins; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const int32_t lo = M - (kWinBins - 1);
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t s = sc[i];
        if (s < min_score || s < lo) continue;
        atomicAdd(&h[M - s], 1u);        // bin 0 = the best score
    }
    __syncthreads();
    uint32_t* gh = w.hist + (int64_t)q * kWinBins;
    for (int i = threadIdx.x; i < kWinBins; i += blockDim.x)
        if (h[i]) atomicAdd(&gh[i], h[i]);
}

// One workgroup per query: the k-th best score from the window histogram.
__global__ __launch_bounds__(256) void k_topk_pick(int32_t k, int32_t n, TopkWs w) {
    __shared__ uint32_t part[256];
    const int q = blockIdx.y;
    TopkState* st = w.st + q;
    const uint32_t* gh = w.hist + (int64_t)q * kWinBins;
    const int32_t M = st->max_score;
    const int32_t min_score = st->min_score;
    if (n == 0 || M == INT32_MIN) {          // empty database
        if (threadIdx.x == 0) { st->n_sel = 0; st->thr = INT32_MAX; }
        return;
    }
    // chunk t = bins [8t, 8t + 8) (best scores first)
    constexpr int per = kWinBins / 256;
    uint32_t c[per];
    uint32_t cs = 0;
#pragma unroll
    for (int i = 0; i < per; ++i) {
        c[i] = gh[threadIdx.x * per + i];
        cs += c[i];
    }
    part[threadIdx.x] = cs;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint32_t x = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
        __syncthreads();
        part[threadIdx.x] += x;
        __syncthreads();
    }
    const uint32_t total = part[255];
    const int32_t lo = M - (kWinBins - 1);
    if (total < (uint32_t)k) {
        // fewer than k eligible scores in the window: all of them are ranked
        // if nothing eligible lies below it, otherwise the window is too narrow
        if (threadIdx.x == 0) {
            if (min_score >= lo) {
                st->n_sel = (int32_t)total;
                st->thr = min_score > lo ? min_score : lo;
                if (total > (uint32_t)kSortCap) st->fallback = 1;
            } else {
                st->fallback = 1;
            }
        }
        return;
    }
    const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    if (before < (uint32_t)k && part[threadIdx.x] >= (uint32_t)k) {
        uint32_t acc = before;
        for (int i = 0; i < per; ++i) {
            acc += c[i];
            if (acc >= (uint32_t)k) {
                st->thr = M - (threadIdx.x * per + i);
                st->n_sel = k;
                if (acc > (uint32_t)kSortCap) st->fallback = 1;
                break;
            }
        }
    }
}

// Gathers every eligible key with score >= T (fast path only).
__global__ __launch_bounds__(256) void k_topk_collect(const int32_t* __restrict__ scores, int64_t stride,
                                                      int32_t n, TopkWs w) {
    const int q = blockIdx.y;
    TopkState* st = w.st + q;
    if (st->fallback) return;
    const int32_t thr = st->thr;
    const int32_t min_score = st->min_score;
    const int32_t* sc = scores + (int64_t)q * stride;
    uint64_t* keys = w.keys + (int64_t)q * kSortCap;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t s = sc[i];
        if (s < thr || s < min_score) continue;
        const int32_t slot = atomicAdd(&st->count, 1);
        if (slot < kSortCap) keys[slot] = rank_key(s, i);
    }
}

// Bitonic sort (descending) of m keys in LDS, m a power of two.
__device__ __forceinline__ void bitonic_desc(uint64_t* s, int m) {
    for (int size = 2; size <= m; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < m; i += blockDim.x) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool desc = (i & size) == 0;
                    const uint64_t a = s[i], b = s[j];
                    if (desc ? (a < b) : (a > b)) {
                        s[i] = b;
                        s[j] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Exact radix select over all eligible keys by one workgroup, most
// significant digit first, 8 bits at a time; returns the k-th largest key.
__device__ uint64_t radix_select_block(const int32_t* sc, int32_t n, int32_t min_score, int32_t k,
                                       uint32_t* hist, uint32_t* part) {
    uint64_t prefix = 0, mask = 0;
    int32_t remaining = k;
    for (int shift = 56; shift >= 0; shift -= 8) {
        for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const int32_t s = sc[i];
            if (s < min_score) continue;
            const uint64_t key = rank_key(s, i);
            if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1u);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t acc = 0;
            int d = 255;
            for (; d >= 0; --d) {
                if (acc + hist[d] >= (uint32_t)remaining) break;
                acc += hist[d];
            }
            part[0] = (uint32_t)d;
            part[1] = acc;
        }
        __syncthreads();
        const uint32_t d = part[0];
        remaining -= (int32_t)part[1];
        prefix |= (uint64_t)d << shift;
        mask |= (uint64_t)0xFF << shift;
        __syncthreads();
    }
    return prefix;
}

// Keys ranked per workgroup of k_topk_final's fast path.
constexpr int kFinalThreads = 256;
constexpr int kFinalGroups = kSortCap / kFinalThreads;

// Writes the ranked hits: blockIdx.y is the query.  Fast path: every
// workgroup loads all gathered keys into LDS and ranks its share of them
// (keys blockIdx.x * kFinalThreads + t, strided by the grid) -- a key's rank
// is the number of larger keys (all keys differ) -- writing each hit
// straight to its rank, so that the workgroups need no synchronisation.
// Fallback: workgroup 0 runs the radix select and sorts.
__global__ __launch_bounds__(kFinalThreads) void k_topk_final(
    const int32_t* __restrict__ scores, int64_t stride, const int32_t* __restrict__ rounds,
    int32_t n, int32_t k, TopkWs w, DevHit* __restrict__ hits, int32_t* __restrict__ n_hits) {
    extern __shared__ __align__(16) uint64_t s[];        // kSortCap + 8 keys
    __shared__ uint32_t hist[256];
    __shared__ uint32_t part[4];
    __shared__ uint32_t cnt;
    const int q = blockIdx.y;
    TopkState* st = w.st + q;
    const int32_t min_score = st->min_score;
    const int32_t* sc = scores + (int64_t)q * stride;
    const int32_t* rd = rounds + (int64_t)q * stride;
    DevHit* out = hits + (int64_t)q * k;
    if (!st->fallback) {
        const int32_t c = st->count < kSortCap ? st->count : kSortCap;
        const int32_t n_out = st->n_sel < c ? st->n_sel : c;
        if (blockIdx.x == 0 && threadIdx.x == 0) n_hits[q] = n_out;
        const int32_t first = blockIdx.x * kFinalThreads;
        if (first >= c) return;
        const uint64_t* keys = w.keys + (int64_t)q * kSortCap;
        for (int32_t i = threadIdx.x; i < c; i += kFinalThreads) s[i] = keys[i];
        // keys past c are 0 and never larger, so the scan may run to a
        // multiple of 8 (two keys per LDS read, four reads in flight)
        if (threadIdx.x < 8u) s[c + threadIdx.x] = 0ull;
        __syncthreads();
        // keys first, first + 1, ... of every kFinalThreads * gridDim.x
        for (int32_t i = first + (int32_t)threadIdx.x; i < c; i += kFinalThreads * (int32_t)gridDim.x) {
            const uint64_t mine = s[i];
            int32_t r = 0;
            const uint4* s2 = (const uint4*)s;
            for (int32_t j = 0; j < c; j += 8) {
                const uint4 a = s2[j / 2], b = s2[j / 2 + 1], e = s2[j / 2 + 2], f = s2[j / 2 + 3];
                r += (((uint64_t)a.y << 32 | a.x) > mine) + (((uint64_t)a.w << 32 | a.z) > mine);
                r += (((uint64_t)b.y << 32 | b.x) > mine) + (((uint64_t)b.w << 32 | b.z) > mine);
                r += (((uint64_t)e.y << 32 | e.x) > mine) + (((uint64_t)e.w << 32 | e.z) > mine);
                r += (((uint64_t)f.y << 32 | f.x) > mine) + (((uint64_t)f.w << 32 | f.z) > mine);
            }
            if (r < n_out) {
                const int32_t id = rank_key_id(mine);
                DevHit h;
                h.target_id = id;
                h.score = rank_key_score(mine);
                h.round = (id >= 0 && id < n) ? rd[id] : -1;
                out[r] = h;
            }
        }
        return;
    }
    if (blockIdx.x != 0) return;
    // k-th largest key, then gather the keys at or above it and sort them
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x)
        if (sc[i] >= min_score) atomicAdd(&cnt, 1u);
    __syncthreads();
    const int32_t eligible = (int32_t)cnt;
    int32_t n_out = eligible < k ? eligible : k;
    const uint64_t kth = n_out > 0 ? radix_select_block(sc, n, min_score, n_out, hist, part) : ~0ull;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int32_t v = sc[i];
        if (v < min_score) continue;
        const uint64_t key = rank_key(v, i);
        if (key >= kth) {
            const uint32_t slot = atomicAdd(&cnt, 1u);
            if (slot < (uint32_t)kSortCap) s[slot] = key;
        }
    }
    __syncthreads();
    const int32_t c = (int32_t)cnt < kSortCap ? (int32_t)cnt : kSortCap;
    int32_t m = 1;
    while (m < c) m <<= 1;
    for (int i = c + threadIdx.x; i < m; i += blockDim.x) s[i] = 0ull;
    __syncthreads();
    bitonic_desc(s, m);
    n_out = n_out < c ? n_out : c;
    for (int i = threadIdx.x; i < n_out; i += blockDim.x) {
        const uint64_t key = s[i];
        const int32_t id = rank_key_id(key);
        DevHit h;
        h.target_id = id;
        h.score = rank_key_score(key);
        h.round = (id >= 0 && id < n) ? rd[id] : -1;
        out[i] = h;
    }
    if (threadIdx.x == 0) n_hits[q] = n_out;
}

}  // namespace hs
