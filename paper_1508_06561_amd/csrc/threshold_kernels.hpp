// threshold_kernels.hpp -- threshold reporting: every target whose score
// reaches the query's threshold, in rank order (score descending, target
// index ascending), however many there are (Section IV reports the database
// sequences scoring above a threshold).
//
// A stable least-significant-digit radix sort of v = M - score (M = the
// largest score of the search, so that ascending v is descending score),
// eight bits per pass, over the eligible targets taken in index order:
// stability keeps equal scores in index order.  Pass 0 reads the score
// array and drops the targets below the threshold.  A pass whose digit is
// zero for every key would leave the order unchanged: it is skipped, and
// so are all later passes (their digits are zero too).
//
// A pass is three launches: per-tile digit histograms, one exclusive scan
// over (digit, tile), and a stable scatter in which every tile places its
// keys round by round, a wavefront's equal digits ranked by lane order
// (ballots over the digit bits), wavefronts in order.
#pragma once

#include "device_common.hpp"
#include "topk_kernels.hpp"

namespace hs {

constexpr int kRsThreads = 256;
constexpr int kRsWaves = kRsThreads / kLanes;
constexpr int kRsRounds = 8;
constexpr int kRsTile = kRsThreads * kRsRounds;   // keys per tile
constexpr int kRsBins = 256;
constexpr int kRsScanThreads = 1024;

struct RsState {
    uint32_t m;         // eligible targets
    uint32_t maxv;      // largest v among them
    int32_t n_out;      // ranks written: min(m, cap), as the alignment kernel reads it
    uint32_t pad_;
};

struct RsWs {
    RsState* st;
    uint32_t* hist;     // [kRsBins][tiles], digit-major
    uint32_t* v[2];     // keys, ping-pong
    int32_t* id[2];
};

__host__ __device__ inline int64_t rs_tiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }

// A pass p > 0 runs only if some key has a non-zero digit p or above.
__device__ __forceinline__ bool rs_pass_live(const RsState* st, int pass) {
    return pass == 0 || (st->maxv >> (8 * pass)) != 0u;
}

__global__ __launch_bounds__(64) void k_rs_reset(RsState* st) {
    if (threadIdx.x == 0) {
        RsState s;
        s.m = 0;
        s.maxv = 0;
        s.n_out = 0;
        s.pad_ = 0;
        *st = s;
    }
}

// Key i of a pass: pass 0 takes target i if its score reaches the
// threshold; later passes take key i of the previous pass's output.
struct RsKey {
    bool live;
    uint32_t v;
    int32_t id;
};
__device__ __forceinline__ RsKey rs_key(int pass, int64_t i, const int32_t* __restrict__ scores,
                                        int32_t n, int32_t min_score, int32_t M, const RsWs& w,
                                        uint32_t m) {
    RsKey k;
    k.live = false;
    k.v = 0;
    k.id = 0;
    if (pass == 0) {
        if (i < n) {
            const int32_t s = scores[i];
            if (s >= min_score) {
                k.live = true;
                k.v = (uint32_t)M - (uint32_t)s;   // M >= s, so no wrap
                k.id = (int32_t)i;
            }
        }
    } else if (i < (int64_t)m) {
        const int src = (pass - 1) & 1;
        k.live = true;
        k.v = w.v[src][i];
        k.id = w.id[src][i];
    }
    return k;
}

// Digit histogram of tile blockIdx.x, written to hist[d][tile] for all d.
// Pass 0 also counts the eligible keys and their largest v.
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(int pass, const int32_t* __restrict__ scores,
                                                        int32_t n, const TopkState* __restrict__ tst,
                                                        RsWs w, int32_t ntiles) {
    __shared__ uint32_t h[kRsBins];
    __shared__ uint32_t s_m, s_max;
    if (!rs_pass_live(w.st, pass)) return;
    const int32_t min_score = tst->min_score, M = tst->max_score;
    const uint32_t m = pass == 0 ? 0u : w.st->m;
    for (int i = threadIdx.x; i < kRsBins; i += kRsThreads) h[i] = 0;
    if (threadIdx.x == 0) {
        s_m = 0;
        s_max = 0;
    }
    __syncthreads();
    uint32_t cnt = 0, mx = 0;
    const int64_t base = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        const RsKey k = rs_key(pass, base + r * kRsThreads + threadIdx.x, scores, n, min_score, M, w, m);
        if (k.live) {
            atomicAdd(&h[(k.v >> (8 * pass)) & 255u], 1u);
            ++cnt;
            mx = k.v > mx ? k.v : mx;
        }
    }
    if (pass == 0) {
        if (cnt) atomicAdd(&s_m, cnt);
        if (mx) atomicMax(&s_max, mx);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads) w.hist[(int64_t)d * ntiles + blockIdx.x] = h[d];
    if (pass == 0 && threadIdx.x == 0) {
        if (s_m) atomicAdd(&w.st->m, s_m);
        if (s_max) atomicMax(&w.st->maxv, s_max);
    }
}

// Exclusive scan of hist (kRsBins * ntiles entries) in place, one workgroup.
__global__ __launch_bounds__(kRsScanThreads) void k_rs_scan(int pass, RsWs w, int32_t ntiles) {
    __shared__ uint32_t part[kRsScanThreads];
    if (!rs_pass_live(w.st, pass)) return;
    const int64_t L = (int64_t)kRsBins * ntiles;
    const int64_t per = (L + kRsScanThreads - 1) / kRsScanThreads;
    const int64_t lo = threadIdx.x * per;
    const int64_t hi = lo + per < L ? lo + per : L;
    uint32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += w.hist[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    // inclusive scan of the per-thread sums (Hillis-Steele)
    for (int off = 1; off < kRsScanThreads; off <<= 1) {
        const uint32_t add = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        const uint32_t c = w.hist[i];
        w.hist[i] = run;
        run += c;
    }
}

// Lanes of the wavefront holding the same 8-bit digit as this lane (among
// the live lanes).
__device__ __forceinline__ uint64_t rs_match(uint32_t d, bool live) {
    uint64_t m = __ballot(live);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const bool bit = ((d >> b) & 1u) != 0u;
        const uint64_t bb = __ballot(live && bit);
        m &= bit ? bb : ~bb;
    }
    return m;
}

// Stable scatter of tile blockIdx.x into the output buffer of the pass.
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(int pass, const int32_t* __restrict__ scores,
                                                           int32_t n, const TopkState* __restrict__ tst,
                                                           RsWs w, int32_t ntiles) {
    __shared__ uint32_t base[kRsBins], run[kRsBins];
    __shared__ uint32_t wcnt[kRsWaves][kRsBins];
    if (!rs_pass_live(w.st, pass)) return;
    const int32_t min_score = tst->min_score, M = tst->max_score;
    const uint32_t m = pass == 0 ? 0u : w.st->m;
    const int dst = pass & 1;
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    for (int d = threadIdx.x; d < kRsBins; d += kRsThreads) {
        base[d] = w.hist[(int64_t)d * ntiles + blockIdx.x];
        run[d] = 0;
    }
    const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsRounds; ++r) {
        for (int i = threadIdx.x; i < kRsWaves * kRsBins; i += kRsThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        const RsKey k = rs_key(pass, tile0 + r * kRsThreads + threadIdx.x, scores, n, min_score, M, w, m);
        const uint32_t d = (k.v >> (8 * pass)) & 255u;
        const uint64_t same = rs_match(d, k.live);
        const uint64_t below = same & ((1ull << lane) - 1ull);
        const uint32_t rank = (uint32_t)__popcll(below);
        // the last lane of each digit group publishes the group's size
        if (k.live && (same >> lane) == 1ull) wcnt[wave][d] = rank + 1u;
        __syncthreads();
        if (k.live) {
            uint32_t pos = base[d] + run[d] + rank;
            for (int v = 0; v < wave; ++v) pos += wcnt[v][d];
            w.v[dst][pos] = k.v;
            w.id[dst][pos] = k.id;
        }
        __syncthreads();
        for (int dd = threadIdx.x; dd < kRsBins; dd += kRsThreads) {
            uint32_t add = 0;
            for (int v = 0; v < kRsWaves; ++v) add += wcnt[v][dd];
            run[dd] += add;
        }
        __syncthreads();
    }
}

// Ranked hits from the last pass's output: the first min(m, cap) ranks,
// each with its winning round; *n_total = m.
__global__ __launch_bounds__(256) void k_rs_out(const TopkState* __restrict__ tst, RsWs w,
                                                const int32_t* __restrict__ rounds, int64_t cap,
                                                DevHit* __restrict__ hits, int64_t* n_total) {
    const RsState* st = w.st;
    const uint32_t m = st->m;
    int last = 0;
    for (int p = 1; p < 4; ++p)
        if ((st->maxv >> (8 * p)) != 0u) last = p;
    const int src = last & 1;
    const int64_t n_out = (int64_t)m < cap ? (int64_t)m : cap;
    const int32_t M = tst->max_score;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_out;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t id = w.id[src][i];
        DevHit h;
        h.target_id = id;
        h.score = (int32_t)((uint32_t)M - w.v[src][i]);
        h.round = rounds ? rounds[id] : 0;
        hits[i] = h;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *n_total = (int64_t)m;
        w.st->n_out = (int32_t)(n_out < 0x7FFFFFFF ? n_out : 0x7FFFFFFF);
    }
}

}  // namespace hs
