// topk_kernels.hpp -- ranking on the device.  Targets scoring at least the
// threshold are ranked by (score descending, target index ascending); each
// target gets a unique 64-bit key, high word = score with the sign bit
// flipped, low word = bitwise-not of the index, so that the top k keys are
// exactly the k best ranks.  A most-significant-digit radix select (digits of
// 12, 12, 8, 12, 12, 8 bits) narrows to the k-th key, a collect pass gathers
// every key at or above it, and one workgroup sorts those k keys.
#pragma once

#include "device_common.hpp"

namespace hs {

constexpr int kTopkBins = 4096;
constexpr int kTopkPasses = 6;
__host__ __device__ constexpr int topk_shift(int pass) {
    return pass == 0 ? 52 : pass == 1 ? 40 : pass == 2 ? 32 : pass == 3 ? 20 : pass == 4 ? 8 : 0;
}
__host__ __device__ constexpr int topk_bits(int pass) { return (pass == 2 || pass == 5) ? 8 : 12; }

struct TopkState {
    uint64_t prefix;      // digits fixed so far (lower bits zero)
    uint64_t mask;        // bits fixed so far
    int32_t remaining;    // ranks still to fill among keys matching prefix
    int32_t done;         // every selected key is >= prefix
    uint32_t ticket;      // workgroups finished in the current pass
    int32_t count;        // keys gathered by the collect pass
    int32_t n_sel;        // min(k, eligible targets)
    int32_t pad_;
};

__device__ __forceinline__ uint64_t rank_key(int32_t score, int32_t id) {
    return ((uint64_t)((uint32_t)score ^ 0x80000000u) << 32) | (uint64_t)(~(uint32_t)id);
}

__global__ void k_topk_init(TopkState* st, uint32_t* hist, int32_t k) {
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->mask = 0;
        st->remaining = k;
        st->done = 0;
        st->ticket = 0;
        st->count = 0;
        st->n_sel = 0;
    }
    for (int i = threadIdx.x; i < kTopkBins; i += blockDim.x) hist[i] = 0;
}

__global__ __launch_bounds__(256) void k_topk_pass(const int32_t* __restrict__ scores, int32_t n,
                                                   int32_t min_score, TopkState* st,
                                                   uint32_t* hist, int32_t pass) {
    __shared__ uint32_t h[kTopkBins];
    __shared__ uint32_t part[256];
    __shared__ int32_t is_last;
    if (__hip_atomic_load(&st->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    const int shift = topk_shift(pass);
    const int nb = 1 << topk_bits(pass);
    for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix, mask = st->mask;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t s = scores[i];
        if (s < min_score) continue;
        const uint64_t key = rank_key(s, i);
        if ((key & mask) != prefix) continue;
        atomicAdd(&h[(uint32_t)(key >> shift) & (uint32_t)(nb - 1)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        if (h[i]) atomicAdd(&hist[i], h[i]);
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) is_last = (atomicAdd(&st->ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    // Last workgroup: pull the global histogram, find the digit holding the
    // remaining-th largest key, fix it, and reset the histogram.
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
        h[i] = __hip_atomic_load(&hist[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        hist[i] = 0;
    }
    __syncthreads();
    // chunk c = bins [c * per, (c + 1) * per), counted from the top bin down
    const int per = nb / 256;
    uint32_t cs = 0;
    for (int i = 0; i < per; ++i) cs += h[nb - 1 - (threadIdx.x * per + i)];
    part[threadIdx.x] = cs;
    __syncthreads();
    // inclusive prefix over chunks (top-down order)
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t v = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    const int32_t remaining = st->remaining;
    const uint32_t total = part[255];
    if (pass == 0 && total <= (uint32_t)remaining) {
        // every eligible target is ranked
        if (threadIdx.x == 0) {
            st->n_sel = (int32_t)total;
            st->done = 1;
            st->prefix = 0;
            st->mask = 0;
            st->ticket = 0;
        }
        return;
    }
    if (pass == 0 && threadIdx.x == 0) st->n_sel = remaining;
    const uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
    if (before < (uint32_t)remaining && part[threadIdx.x] >= (uint32_t)remaining) {
        uint32_t above = before;
        for (int i = 0; i < per; ++i) {
            const int bin = nb - 1 - (threadIdx.x * per + i);
            const uint32_t c = h[bin];
            if (above + c >= (uint32_t)remaining) {
                const int32_t rem = remaining - (int32_t)above;
                st->remaining = rem;
                st->prefix |= (uint64_t)bin << shift;
                st->mask |= (uint64_t)(nb - 1) << shift;
                st->done = (c == (uint32_t)rem) ? 1 : 0;
                break;
            }
            above += c;
        }
        st->ticket = 0;
    }
}

__global__ __launch_bounds__(256) void k_topk_collect(const int32_t* __restrict__ scores, int32_t n,
                                                      int32_t min_score, TopkState* st,
                                                      uint64_t* __restrict__ keys, int32_t cap) {
    const uint64_t thr = st->prefix;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t s = scores[i];
        if (s < min_score) continue;
        const uint64_t key = rank_key(s, i);
        if (key >= thr) {
            const int32_t slot = atomicAdd(&st->count, 1);
            if (slot < cap) keys[slot] = key;
        }
    }
}

// One workgroup of 1024 threads: bitonic sort (descending) of the gathered
// keys, padded with zeros, then the ranked hits.
struct DevHit {
    int64_t target_id;
    int32_t score;
    int32_t round;
};

__global__ __launch_bounds__(1024) void k_topk_sort(const TopkState* st, const uint64_t* keys,
                                                    const int32_t* __restrict__ rounds,
                                                    int32_t n_targets, int32_t cap,
                                                    DevHit* __restrict__ hits,
                                                    int32_t* __restrict__ n_hits) {
    __shared__ uint64_t s[4096];
    // the collect pass gathers exactly n_sel keys; the clamps only keep a
    // broken invariant from reaching memory out of range
    int32_t n = st->n_sel < st->count ? st->n_sel : st->count;
    n = n < cap ? n : cap;
    int32_t m = 1;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += blockDim.x) s[i] = i < n ? keys[i] : 0ull;
    __syncthreads();
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
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const uint64_t key = s[i];
        const int32_t id = (int32_t)(~(uint32_t)key);
        DevHit h;
        h.target_id = id;
        h.score = (int32_t)((uint32_t)(key >> 32) ^ 0x80000000u);
        h.round = (id >= 0 && id < n_targets) ? rounds[id] : -1;
        hits[i] = h;
    }
    if (threadIdx.x == 0) *n_hits = n;
}

}  // namespace hs
