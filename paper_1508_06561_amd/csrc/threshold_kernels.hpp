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
// A pass is per-tile digit histograms, an exclusive scan over (digit, tile)
// (segment sums, a scan of those, then each segment scanned with its
// offset), and a stable scatter in which every tile places its keys round by
// round, a wavefront's equal digits ranked by lane order (ballots over the
// digit bits), wavefronts in order.
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
constexpr int kRsSeg = 4 * kRsThreads;        // histogram entries per scan segment

struct RsState {
    uint32_t m;         // eligible targets
    uint32_t maxv;      // largest v among them
    int32_t n_out;      // ranks written: min(m, cap), as the alignment kernel reads it
    uint32_t pad_;
};

struct RsWs {
    RsState* st;
    uint32_t* hist;     // [kRsBins][tiles], digit-major
    uint32_t* part;     // one sum per scan segment of hist
    uint32_t* v[2];     // keys, ping-pong
    int32_t* id[2];
};

__host__ __device__ inline int64_t rs_tiles(int64_t n) { return (n + kRsTile - 1) / kRsTile; }
// Scan segments of a histogram of `tiles` tiles.
__host__ __device__ inline int64_t rs_segments(int64_t tiles) {
    return (kRsBins * tiles + kRsSeg - 1) / kRsSeg;
}

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

// Inclusive prefix sum over the wavefront (all lanes active).
__device__ __forceinline__ uint32_t rs_wave_inclusive(uint32_t x, int lane) {
    for (int o = 1; o < kLanes; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, kLanes);
        if (lane >= o) x += y;
    }
    return x;
}

// The scan of hist (L = kRsBins * ntiles entries, a multiple of 4) in three
// launches.  First the sum of each segment of kRsSeg entries, one workgroup
// per segment, each thread reading four consecutive entries.
__global__ __launch_bounds__(kRsThreads) void k_rs_scan_reduce(int pass, RsWs w, int64_t L) {
    __shared__ uint32_t wsum[kRsWaves];
    if (!rs_pass_live(w.st, pass)) return;
    const int64_t i = (int64_t)blockIdx.x * kRsSeg + 4 * (int64_t)threadIdx.x;
    uint32_t s = 0;
    if (i < L) {
        const uint4 v = *(const uint4*)(w.hist + i);
        s = v.x + v.y + v.z + v.w;
    }
    for (int o = kLanes / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kLanes);
    if ((threadIdx.x & (kLanes - 1)) == 0) wsum[threadIdx.x / kLanes] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kRsWaves; ++k) t += wsum[k];
        w.part[blockIdx.x] = t;
    }
}

// Exclusive scan of the G segment sums in place, one workgroup, 1,024 at a
// time with the running total carried over.
__global__ __launch_bounds__(kRsScanThreads) void k_rs_scan_top(int pass, RsWs w, int64_t G) {
    constexpr int kW = kRsScanThreads / kLanes;
    __shared__ uint32_t tot[kW];
    if (!rs_pass_live(w.st, pass)) return;
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    uint32_t carry = 0;
    for (int64_t base = 0; base < G; base += kRsScanThreads) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < G ? w.part[i] : 0u;
        const uint32_t inc = rs_wave_inclusive(v, lane);
        if (lane == kLanes - 1) tot[wave] = inc;
        __syncthreads();
        uint32_t before = carry, all = carry;
        for (int k = 0; k < kW; ++k) {
            before += k < wave ? tot[k] : 0u;
            all += tot[k];
        }
        if (i < G) w.part[i] = before + inc - v;
        __syncthreads();              // tot is rewritten by the next chunk
        carry = all;
    }
}

// Each segment's exclusive scan plus the segment's offset, written back.
__global__ __launch_bounds__(kRsThreads) void k_rs_scan_down(int pass, RsWs w, int64_t L) {
    __shared__ uint32_t wsum[kRsWaves];
    if (!rs_pass_live(w.st, pass)) return;
    const int64_t i = (int64_t)blockIdx.x * kRsSeg + 4 * (int64_t)threadIdx.x;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (i < L) v = *(const uint4*)(w.hist + i);
    const uint32_t t = v.x + v.y + v.z + v.w;
    const int lane = threadIdx.x & (kLanes - 1), wave = threadIdx.x / kLanes;
    const uint32_t inc = rs_wave_inclusive(t, lane);
    if (lane == kLanes - 1) wsum[wave] = inc;
    __syncthreads();
    uint32_t run = w.part[blockIdx.x] + inc - t;
    for (int k = 0; k < wave; ++k) run += wsum[k];
    if (i < L) {
        uint4 o;
        o.x = run;
        run += v.x;
        o.y = run;
        run += v.y;
        o.z = run;
        run += v.z;
        o.w = run;
        *(uint4*)(w.hist + i) = o;
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
