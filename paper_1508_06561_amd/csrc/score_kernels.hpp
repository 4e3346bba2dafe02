// score_kernels.hpp -- pair scoring: the search-mode heuristic of Fig. 1
// (Section III.B.3: Rounds = 1 by default, contained shifts only) for every
// (query, target) pair, one lane per target.
#pragma once

#include "device_common.hpp"

namespace hs {

// Query profile in LDS: prof[r * ps + c] = B[r][query[c]] for target letter
// r and query position c; columns qlen..ps-1 are zero padding.
__device__ __forceinline__ void build_profile(int8_t* prof, int32_t ps, const uint8_t* qcodes,
                                              int32_t qlen, const KMatrix& km) {
    for (int32_t idx = threadIdx.x; idx < kNsym * ps; idx += blockDim.x) {
        const int32_t r = idx / ps;
        const int32_t c = idx - r * ps;
        prof[idx] = c < qlen ? km.m[r * kNsym + qcodes[c]] : (int8_t)0;
    }
}

// Best contained shift (PROCEDURE getBestSubsequenceAlignment with
// start = len(small) - 1, end = len(large) - 1): the ss-letter window of
// small at every shift k in [0, ls - ss] of the ls-letter window of large;
// each placement scores the sum of substitution scores over its ss pairs
// (getVirtualAlignmentScore).  The first shift reaching the maximum wins.
// The cell (k, j) pairs large[pL + k + j] with small[pS + j]; in the profile
// the target letter picks the row and the query position the column.
__device__ __forceinline__ void best_shift_lane(const int8_t* prof, int32_t ps,
                                                const uint32_t* lane_base, bool target_large,
                                                int32_t pL, int32_t pS, int32_t ls, int32_t ss,
                                                int32_t& kbest, int32_t& dbest) {
    const int32_t nk = ls - ss + 1;
    dbest = INT32_MIN;
    kbest = 0;
    TargetStream ts;
    for (int32_t k = 0; k < nk; ++k) {
        int32_t D = 0;
        const int8_t* col;
        if (target_large) {
            ts.seek(lane_base, pL + k);
            col = prof + pS;
        } else {
            ts.seek(lane_base, pS);
            col = prof + pL + k;
        }
        for (int32_t j = 0; j < ss; ++j) D += col[(int32_t)ts.next() * ps + j];
        if (D > dbest) {
            dbest = D;
            kbest = k;
        }
    }
}

// One (query, target) pair: AlignSequences over `rounds` rounds, each an
// Align run whose score is accumulated on the fly: the sum of the chosen
// placements' scores, minus the gap cost of each chosen shift, minus the
// trailing periphery gaps left when one sequence runs out (SCORE).
__device__ __forceinline__ void score_pair_lane(const KParams& kp, const int8_t* prof,
                                                int32_t ps, int32_t qlen,
                                                const uint32_t* lane_base, int32_t tlen,
                                                uint64_t target_id, int32_t& best,
                                                int32_t& best_round, uint64_t& cells) {
    const bool target_large = tlen >= qlen;
    const int32_t nl = target_large ? tlen : qlen;
    const int32_t ns = target_large ? qlen : tlen;
    best = INT32_MIN;
    best_round = 0;
    cells = 0;
    DrawStream ds;
    for (int32_t r = 0; r < kp.rounds; ++r) {
        ds.init(kp.seed, target_id, (uint32_t)r);
        uint32_t lf = ds.get(0), sf = ds.get(1);
        lf = lf < kp.minfactor ? kp.minfactor : lf;
        sf = sf < kp.minfactor ? kp.minfactor : sf;
        const uint32_t LF = (uint32_t)(((uint64_t)kp.lfactor * lf) >> 16);
        const uint32_t SF = (uint32_t)(((uint64_t)kp.sfactor * sf) >> 16);
        int32_t pL = 0, pS = 0, t = 0, score = 0;
        while (pL < nl && pS < ns) {
            const int32_t ls = window_large(nl - pL, LF);
            const int32_t ss = window_small(ns - pS, SF, ds.get(2u + (uint32_t)t), ls);
            int32_t kb, db;
            best_shift_lane(prof, ps, lane_base, target_large, pL, pS, ls, ss, kb, db);
            cells += (uint64_t)(ls - ss + 1) * (uint64_t)ss;
            score += db - shift_penalty(kp, t, kb);
            pL += kb + ss;
            pS += ss;
            ++t;
        }
        score -= kp.pgp * ((nl - pL) + (ns - pS));
        if (score > best) {
            best = score;
            best_round = r;
        }
    }
}

// One wavefront per group of 64 targets, four groups per workgroup sharing
// one LDS profile.  Writes the pair score and winning round by target index;
// with kCount it also adds the residue pairs scored on diagonals (the work
// measure of Section III.B.4) to *cells_total.
template <bool kCount>
__global__ __launch_bounds__(256) void k_score_lanes(DbView db, const uint8_t* __restrict__ qcodes,
                                                    int32_t qlen, int32_t ps, KParams kp,
                                                    KMatrix km, int32_t* __restrict__ scores,
                                                    int32_t* __restrict__ rounds,
                                                    unsigned long long* cells_total) {
    extern __shared__ int8_t prof[];
    build_profile(prof, ps, qcodes, qlen, km);
    __syncthreads();
    const int32_t g = blockIdx.x * (blockDim.x / kLanes) + threadIdx.x / kLanes;
    const int32_t lane = threadIdx.x & (kLanes - 1);
    if (g >= db.n_groups) return;
    const int32_t slot = g * kLanes + lane;
    const int32_t id = db.slot_id[slot];
    uint64_t cells = 0;
    if (id >= 0) {
        const int32_t tlen = db.slot_len[slot];
        const uint32_t* lane_base = db.words + db.group_base[g] + lane;
        int32_t best, best_round;
        score_pair_lane(kp, prof, ps, qlen, lane_base, tlen, (uint64_t)id, best, best_round, cells);
        scores[id] = best;
        if (rounds) rounds[id] = best_round;
    }
    if (kCount) {
        for (int off = kLanes / 2; off > 0; off >>= 1) cells += __shfl_xor(cells, off, kLanes);
        if (lane == 0) atomicAdd(cells_total, (unsigned long long)cells);
    }
}

}  // namespace hs
