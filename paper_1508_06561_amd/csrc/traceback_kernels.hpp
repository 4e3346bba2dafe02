// traceback_kernels.hpp -- alignments for the best hits only.  The scoring
// pass keeps no per-pair state beyond the score and the winning round (the
// constant auxiliary space of Section III.B.4); the aligned rows of the top
// hits are recovered by replaying that round, which is deterministic because
// every draw is keyed by (seed, target, round, draw index).
#pragma once

#include "device_common.hpp"
#include "score_kernels.hpp"
#include "topk_kernels.hpp"

namespace hs {

constexpr uint32_t kOpM = 0, kOpI = 1, kOpD = 2;

struct DevAln {
    int64_t target_id;
    int32_t score;
    int32_t n_ops;
    int64_t ops_off;
};

// Run-length writer that merges adjacent runs of the same op.
struct OpWriter {
    uint32_t* out;
    int32_t n;
    uint32_t op, len;
    __device__ __forceinline__ void init(uint32_t* o) { out = o; n = 0; op = 0; len = 0; }
    __device__ __forceinline__ void emit(uint32_t o, int32_t l) {
        if (l <= 0) return;
        if (len && o == op) {
            len += (uint32_t)l;
            return;
        }
        flush();
        op = o;
        len = (uint32_t)l;
    }
    __device__ __forceinline__ void flush() {
        if (len) out[n++] = (len << 2) | op;
        len = 0;
    }
};

// Replays the winning round of hit a (a < min(n_aln, n_hits)) and writes its
// alignment as ops oriented (query, target).  Inside the chop-and-consume
// loop only the small sequence receives gaps (Section III.B.3): the k* skipped
// letters of large are target letters over gaps (D) when the target is large
// and query letters over gaps (I) otherwise; after the loop the rest of
// whichever sequence is left goes against gaps.
__global__ __launch_bounds__(64) void k_traceback(DbView db, const uint8_t* __restrict__ qcodes,
                                                  int32_t qlen, int32_t ps, KParams kp, KMatrix km,
                                                  const DevHit* __restrict__ hits,
                                                  const int32_t* __restrict__ n_hits, int32_t n_aln,
                                                  int32_t n_targets, DevAln* __restrict__ alns,
                                                  uint32_t* __restrict__ ops, int64_t ops_stride) {
    extern __shared__ int8_t prof[];
    build_profile(prof, ps, qcodes, qlen, km);
    __syncthreads();
    const int32_t a = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nh = *n_hits;
    if (a >= n_aln || a >= nh) return;
    const int32_t id = (int32_t)hits[a].target_id;
    const int32_t r = hits[a].round;
    if (id < 0 || id >= n_targets || r < 0 || r >= kp.rounds) return;   // never for a valid hit
    const int32_t slot = db.loc[id];
    const int32_t g = slot / kLanes, lane = slot % kLanes;
    const int32_t tlen = db.slot_len[slot];
    const uint32_t* lane_base = db.words + db.group_base[g] + lane;

    const bool target_large = tlen >= qlen;
    const int32_t nl = target_large ? tlen : qlen;
    const int32_t ns = target_large ? qlen : tlen;
    const uint32_t gap_in_small = target_large ? kOpD : kOpI;   // large letter over a gap
    const uint32_t gap_in_large = target_large ? kOpI : kOpD;   // small letter over a gap

    DrawStream ds;
    ds.init(kp.seed, (uint64_t)id, (uint32_t)r);
    uint32_t lf = ds.get(0), sf = ds.get(1);
    lf = lf < kp.minfactor ? kp.minfactor : lf;
    sf = sf < kp.minfactor ? kp.minfactor : sf;
    const uint32_t LF = (uint32_t)(((uint64_t)kp.lfactor * lf) >> 16);
    const uint32_t SF = (uint32_t)(((uint64_t)kp.sfactor * sf) >> 16);
    OpWriter w;
    w.init(ops + (int64_t)a * ops_stride);
    int32_t pL = 0, pS = 0, t = 0, score = 0;
    while (pL < nl && pS < ns) {
        const int32_t ls = window_large(nl - pL, LF);
        const int32_t ss = window_small(ns - pS, SF, ds.get(2u + (uint32_t)t), ls);
        int32_t kb, db_;
        best_shift_lane(prof, ps, lane_base, target_large, pL, pS, ls, ss, kb, db_);
        score += db_ - shift_penalty(kp, t, kb);
        w.emit(gap_in_small, kb);
        w.emit(kOpM, ss);
        pL += kb + ss;
        pS += ss;
        ++t;
    }
    score -= kp.pgp * ((nl - pL) + (ns - pS));
    w.emit(gap_in_small, nl - pL);
    w.emit(gap_in_large, ns - pS);
    w.flush();
    DevAln out;
    out.target_id = id;
    out.score = score;
    out.n_ops = w.n;
    out.ops_off = (int64_t)a * ops_stride;
    alns[a] = out;
}

}  // namespace hs
