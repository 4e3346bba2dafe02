// align_kernels.hpp -- the pairwise mode of Fig. 1: the small window slides
// across the large one from end to end (placements i = 0 .. ss + ls - 2,
// shift k = i - ss + 1, at least one letter of overlap), and the best of
// Rounds rounds is kept (the paper's alignment tests ran Rounds = 20).
//
// A placement gives up all ss letters of the small window -- those hanging
// over an end of the large window face gaps -- and the large window's
// letters through the last one facing small, min(k + ss, ls); the rest of
// the large window goes back to large (Section III.B.2).
//
// One workgroup per (pair, round) scores that round: its threads share each
// step's placements, four neighbouring ones to a thread (they share their
// letter reads), summing the letters that face each other from the two
// sequences staged in LDS.  The workgroup that finishes a pair's last round
// then replays the pair's best round (its sequences are still staged) and
// writes its run-length ops, so that a long pair's replay follows its own
// rounds rather than waiting for every pair's.
#pragma once

#include "device_common.hpp"
#include "traceback_kernels.hpp"   // run-length op codes

namespace hs {

constexpr int kAlThreads = 256;                  // threads per workgroup of the op packing
constexpr int kAlWaves = kAlThreads / kLanes;
constexpr int kAlThreadsShort = 128;             // threads per (pair, round) of short pairs
constexpr int kAlThreadsLong = 1024;             // of batches holding a long pair
constexpr int kAlWavesMax = kAlThreadsLong / kLanes;
constexpr int kAlLongPair = 4000;                // letters: a long pair
constexpr int kAlMaxLen = 5600;                  // longest sequence of the pairwise mode

// One pair of a pairwise batch: query codes at qoff, target codes at toff.
struct AlignPair {
    int64_t qoff, toff;
    int32_t qlen, tlen;
    int64_t ops_off;     // first op of the pair's output
};

// LDS of a workgroup (dynamic, sized by the launch to the batch's longest
// sequence, `cap` letters): a fixed head -- the substitution matrix
// transposed (row = the small sequence's letter), the wavefronts' best keys,
// the replay's round and flag -- then the large sequence as one 32-bit word
// per position holding that letter and the three after it (so that the four
// placements of a thread read their letters in one aligned read), then the
// small sequence.
struct AlignHead {
    int8_t matT[kNsym * kNsym];
    uint64_t wbest[kAlWavesMax];
    int32_t best_round, last;
};
__host__ __device__ constexpr size_t al_lds_bytes(int32_t cap) {
    return sizeof(AlignHead) + 5 * (size_t)((cap + 15) & ~15);
}
struct AlignLds {
    AlignHead* h;
    int8_t* matT;
    uint64_t* wbest;
    uint32_t* L4;
    uint8_t* S;
    __device__ AlignLds(uint8_t* base, int32_t cap) {
        h = (AlignHead*)base;
        matT = h->matT;
        wbest = h->wbest;
        L4 = (uint32_t*)(base + sizeof(AlignHead));
        S = (uint8_t*)(L4 + ((cap + 15) & ~15));
    }
};

// Largest 64-bit key over the wavefront (all lanes active), by two 32-bit
// maxima through DPP-free shuffles.
__device__ __forceinline__ uint64_t al_wave_max(uint64_t key) {
    for (int o = kLanes / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(key, o, kLanes);
        key = y > key ? y : key;
    }
    return key;
}

// Random draws of one (pair, round), one Philox block at a time.
struct AlDraws {
    int32_t blk;
    uint64_t w[4];
    __device__ __forceinline__ uint32_t get(uint64_t seed, int32_t id, int32_t round, uint32_t d) {
        const int32_t b = (int32_t)(d >> 4);
        if (b != blk) {
            philox_block(seed, (uint64_t)id, (uint32_t)round, (uint32_t)b, w);
            blk = b;
        }
        const uint32_t wi = (d >> 2) & 3;
        const uint64_t x = wi == 0 ? w[0] : wi == 1 ? w[1] : wi == 2 ? w[2] : w[3];
        return (uint32_t)(x >> (16 * (d & 3))) & 0xFFFFu;
    }
};

// Appends n columns of op to the run-length ops (one thread).
__device__ __forceinline__ void al_emit(uint32_t* ops, int32_t& n_ops, uint32_t op, int32_t n) {
    if (n <= 0) return;
    if (n_ops > 0 && (ops[n_ops - 1] & 3u) == op) ops[n_ops - 1] += (uint32_t)n << 2;
    else ops[n_ops++] = ((uint32_t)n << 2) | op;
}

// One round of pair `id` by the whole workgroup of kT threads: the round's
// score (SCORE of its aligned rows, streamed step by step) and, with kEmit,
// its ops written by thread 0.  Each thread takes four neighbouring
// placements at a time, which read their large letters as one word and
// share the small letter.  The large sequence (nl letters, as L4) and the
// small one (ns <= nl, as S) are in LDS; tl: the target is the large one.
template <int kT, bool kEmit>
__device__ int32_t al_round(AlignLds& A, int32_t nl, int32_t ns, bool tl, const KParams& kp,
                            int32_t id, int32_t round, uint32_t* ops, int32_t* n_ops_out) {
    const int32_t tid = threadIdx.x, lane = tid & (kLanes - 1), wave = tid / kLanes;
    AlDraws dr;
    dr.blk = -1;
    const uint32_t LF = round_factor(kp.lfactor, kp.minfactor, dr.get(kp.seed, id, round, 0));
    const uint32_t SF = round_factor(kp.sfactor, kp.minfactor, dr.get(kp.seed, id, round, 1));
    // ops: a large letter against a gap, a small letter against a gap
    const uint32_t opL = tl ? kOpD : kOpI, opS = tl ? kOpI : kOpD;
    int32_t n_ops = 0;
    int32_t pL = 0, pS = 0, score = 0;
    bool open_l = false;     // the last column was a gap of the large row, inside it
    for (int32_t t = 0; pL < nl && pS < ns; ++t) {
        const int32_t ls = window_large(nl - pL, LF);
        int32_t ss = (int32_t)(((uint64_t)(ns - pS) * SF * dr.get(kp.seed, id, round, 2u + (uint32_t)t)) >> 32);
        ss = ss < 1 ? 1 : ss;
        // every placement i: shift k = i - ss + 1; the letters facing each
        // other are small j in [max(0, -k), min(ss, ls - k))
        const int32_t np = ls + ss - 1;
        uint64_t best = 0;
        for (int32_t i0 = 4 * tid; i0 < np; i0 += 4 * kT) {
            // placements i0 .. i0 + 3 (those below np): placement i0 + m
            // faces small letters [j0_m, j1_m); both ends fall with m by at
            // most one per placement, so [j0_0, j1_3) is faced by all four
            // (the interior) and each has at most three letters outside it
            const int32_t k0 = i0 - ss + 1;
            const int32_t n4 = np - i0 < 4 ? np - i0 : 4;
            const int32_t J0 = k0 < 0 ? -k0 : 0;
            const int32_t J1 = ss < ls - k0 - 3 ? ss : ls - k0 - 3;
            const int32_t lb = pL + k0;              // L4[lb + j]: letters lb + j + m, m = 0..3
            const uint8_t* Sj = A.S + pS;
            int32_t D0 = 0, D1 = 0, D2 = 0, D3 = 0;
            if (n4 == 4) {
                for (int32_t j = J0; j < J1; ++j) {
                    const uint32_t w = A.L4[lb + j];
                    const int8_t* row = A.matT + Sj[j] * kNsym;
                    D0 += row[w & 0xFFu];
                    D1 += row[(w >> 8) & 0xFFu];
                    D2 += row[(w >> 16) & 0xFFu];
                    D3 += row[w >> 24];
                }
            }
            // the letters of each placement outside the interior: at most
            // three before it and three after it, read as independent
            // predicated loads (a loop here would chain their latencies);
            // without an interior (fewer than four placements left, or a
            // window of a few letters) each placement sums its own range
            const bool in = n4 == 4 && J0 < J1;
#define HS_AL_EDGE(m, D)                                                              \
            if (m < n4) {                                                             \
                const int32_t km = k0 + m;                                            \
                const int32_t a = km < 0 ? -km : 0;                                   \
                const int32_t b = ss < ls - km ? ss : ls - km;                        \
                if (in) {                                                             \
                    _Pragma("unroll") for (int e = 1; e <= 3; ++e) {                  \
                        const int32_t jh = J0 - e, jt = J1 - 1 + e;                   \
                        if (jh >= a) D += A.matT[Sj[jh] * kNsym + (A.L4[lb + jh + m] & 0xFFu)]; \
                        if (jt < b) D += A.matT[Sj[jt] * kNsym + (A.L4[lb + jt + m] & 0xFFu)];  \
                    }                                                                 \
                } else {                                                              \
                    for (int32_t j = a; j < b; ++j)                                   \
                        D += A.matT[Sj[j] * kNsym + (A.L4[lb + j + m] & 0xFFu)];      \
                }                                                                     \
                const uint64_t key = shift_key(D, i0 + m);                            \
                best = key > best ? key : best;                                       \
            }
            HS_AL_EDGE(0, D0) HS_AL_EDGE(1, D1) HS_AL_EDGE(2, D2) HS_AL_EDGE(3, D3)
#undef HS_AL_EDGE
        }
        best = al_wave_max(best);
        if (lane == 0) A.wbest[wave] = best;
        __syncthreads();
        uint64_t b = A.wbest[0];
        for (int w = 1; w < kT / kLanes; ++w) b = A.wbest[w] > b ? A.wbest[w] : b;
        __syncthreads();          // wbest is rewritten by the next step
        const int32_t k = key_shift(b) - ss + 1;
        const int32_t D = key_score(b);
        // gaps in front of the placement: large letters before a positive
        // shift (small row; before small's first letter when pS == 0), or
        // small letters before the large window (large row; before large's
        // first letter when pL == 0, else continuing an inner run left open
        // by the previous step's overhang)
        if (k > 0) {
            score -= pS == 0 ? kp.pgp * k : kp.gop + (k - 1) * kp.gep;
            if (kEmit && tid == 0) al_emit(ops, n_ops, opL, k);
        } else if (k < 0) {
            const int32_t g = -k;
            score -= pL == 0 ? kp.pgp * g : open_l ? kp.gep * g : kp.gop + (g - 1) * kp.gep;
            if (kEmit && tid == 0) al_emit(ops, n_ops, opS, g);
        }
        score += D;
        const int32_t face = (ss < ls - k ? ss : ls - k) - (k < 0 ? -k : 0);
        if (kEmit && tid == 0) al_emit(ops, n_ops, kOpM, face);
        const int32_t take = k + ss < ls ? k + ss : ls;
        const int32_t hang = k + ss - ls;         // small letters past the window's end
        pL += take;
        pS += ss;
        open_l = false;
        if (hang > 0) {
            // after large's last letter if large is used up, else an inner run
            if (pL == nl) {
                score -= kp.pgp * hang;
            } else {
                score -= kp.gop + (hang - 1) * kp.gep;
                open_l = true;
            }
            if (kEmit && tid == 0) al_emit(ops, n_ops, opS, hang);
        }
    }
    // what is left of either sequence faces gaps after the other's last letter
    score -= kp.pgp * ((nl - pL) + (ns - pS));
    if (kEmit && tid == 0) {
        al_emit(ops, n_ops, opL, nl - pL);
        al_emit(ops, n_ops, opS, ns - pS);
        *n_ops_out = n_ops;
    }
    return score;
}

// Stages pair p in LDS as (large, small) with kT threads; returns (nl, ns, tl).
template <int kT>
__device__ __forceinline__ void al_stage(AlignLds& A, const AlignPair& P, const uint8_t* codes,
                                         const KMatrix& km, int32_t& nl, int32_t& ns, bool& tl) {
    tl = P.tlen >= P.qlen;
    nl = tl ? P.tlen : P.qlen;
    ns = tl ? P.qlen : P.tlen;
    const uint8_t* src_l = codes + (tl ? P.toff : P.qoff);
    const uint8_t* src_s = codes + (tl ? P.qoff : P.toff);
    // codes above the alphabet's last (possible in device input) read as it
    auto code = [](uint8_t c) { return (uint32_t)(c < kNsym ? c : kNsym - 1); };
    for (int32_t i = threadIdx.x; i < nl; i += kT) {
        // letters i .. i + 3 (past the end: 0, never summed)
        uint32_t w = code(src_l[i]);
        if (i + 1 < nl) w |= code(src_l[i + 1]) << 8;
        if (i + 2 < nl) w |= code(src_l[i + 2]) << 16;
        if (i + 3 < nl) w |= code(src_l[i + 3]) << 24;
        A.L4[i] = w;
    }
    for (int32_t i = threadIdx.x; i < ns; i += kT) A.S[i] = (uint8_t)code(src_s[i]);
    // matT[s * kNsym + l] = score of small letter s against large letter l:
    // the matrix scores a query letter (its row) against a target letter (its
    // column), so this is the matrix itself when the query is the small
    // sequence and its transpose otherwise
    for (int32_t i = threadIdx.x; i < kNsym * kNsym; i += kT)
        A.matT[i] = tl ? km.m[i] : km.m[(i % kNsym) * kNsym + i / kNsym];
    __syncthreads();
}

// Workgroup b scores round b % rounds of pair order[b / rounds] (pairs
// in order of decreasing work, so that the longest chains start first) into
// round_scores[pair * rounds + round].  The workgroup that completes a
// pair's rounds (the pair's counter in `done`, zero at launch, reaching
// rounds) replays the best round (the first with the highest score) with
// its sequences still in LDS: score, round, op count and ops at
// ops + pairs[pair].ops_off (rounds may be NULL).  kT threads per
// workgroup; no sequence longer than cap letters; al_lds_bytes(cap) bytes of
// dynamic LDS.
template <int kT>
__global__ __launch_bounds__(kT) void k_align_pairs(const AlignPair* __restrict__ pairs,
                                                    const int32_t* __restrict__ order,
                                                    const uint8_t* __restrict__ codes, int32_t cap,
                                                    KParams kp, KMatrix km,
                                                    int32_t* __restrict__ round_scores,
                                                    uint32_t* __restrict__ done,
                                                    int32_t* __restrict__ scores,
                                                    int32_t* __restrict__ rounds,
                                                    int32_t* __restrict__ n_ops,
                                                    uint32_t* __restrict__ ops) {
    extern __shared__ __align__(16) uint8_t al_lds[];
    AlignLds A(al_lds, cap);
    const int32_t pair = order[blockIdx.x / kp.rounds], round = blockIdx.x % kp.rounds;
    const AlignPair P = pairs[pair];
    int32_t nl, ns;
    bool tl;
    al_stage<kT>(A, P, codes, km, nl, ns, tl);
    if (kp.rounds == 1) {
        // the only round is the best: scored and written in one pass
        const int32_t s1 = al_round<kT, true>(A, nl, ns, tl, kp, pair, 0, ops + P.ops_off, n_ops + pair);
        if (threadIdx.x == 0) {
            scores[pair] = s1;
            if (rounds) rounds[pair] = 0;
        }
        return;
    }
    const int32_t s = al_round<kT, false>(A, nl, ns, tl, kp, pair, round, nullptr, nullptr);
    int32_t* rs = round_scores + (int64_t)pair * kp.rounds;
    if (threadIdx.x == 0) {
        rs[round] = s;
        __threadfence();                               // the score before the count
        const uint32_t prev = atomicAdd(done + pair, 1u);
        A.h->last = prev == (uint32_t)kp.rounds - 1u;
        if (A.h->last) {
            __threadfence();                           // every round's score after the count
            int32_t best = INT32_MIN, best_r = 0;
            for (int32_t r = 0; r < kp.rounds; ++r) {
                const int32_t v = r == round ? s : __hip_atomic_load(rs + r, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
                if (v > best) {
                    best = v;
                    best_r = r;
                }
            }
            A.h->best_round = best_r;
        }
    }
    __syncthreads();
    if (!A.h->last) return;                            // the same for the whole workgroup
    const int32_t best_r = A.h->best_round;
    const int32_t s2 = al_round<kT, true>(A, nl, ns, tl, kp, pair, best_r, ops + P.ops_off, n_ops + pair);
    if (threadIdx.x == 0) {
        scores[pair] = s2;       // equal to the round's score: the replay is the same round
        if (rounds) rounds[pair] = best_r;
    }
}

// Zeroes the pairs' round counters before k_align_pairs (a kernel rather
// than a memset, so that work queued on a stream being captured into a
// graph holds no memset node).
__global__ __launch_bounds__(256) void k_align_reset(uint32_t* __restrict__ done, int32_t n) {
    const int32_t i = (int32_t)blockIdx.x * 256 + (int32_t)threadIdx.x;
    if (i < n) done[i] = 0;
}

// Exclusive prefix sums of the pairs' op counts, one workgroup: off[i] is
// the first packed op of pair i, off[n] the total.  Each thread sums a run of
// consecutive counts, the run totals are scanned in LDS, and each thread
// then writes its run's offsets.
constexpr int kAlScanThreads = 1024;
__global__ __launch_bounds__(kAlScanThreads) void k_align_ops_scan(const int32_t* __restrict__ cnt,
                                                                   int32_t n, int64_t* __restrict__ off) {
    __shared__ int64_t part[kAlScanThreads];
    const int32_t per = (n + kAlScanThreads - 1) / kAlScanThreads;
    const int32_t lo = (int32_t)threadIdx.x * per;
    const int32_t hi = lo + per < n ? lo + per : n;
    int64_t sum = 0;
    for (int32_t i = lo; i < hi; ++i) sum += cnt[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    for (int o = 1; o < kAlScanThreads; o <<= 1) {
        const int64_t y = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - sum;
    for (int32_t i = lo; i < hi; ++i) {
        off[i] = run;
        run += cnt[i];
    }
    if (threadIdx.x == kAlScanThreads - 1) off[n] = part[kAlScanThreads - 1];
}

// One wavefront per pair moves the pair's ops from its slot in `ops` to its
// packed place.
__global__ __launch_bounds__(kAlThreads) void k_align_ops_pack(const AlignPair* __restrict__ pairs,
                                                               int32_t n, const int32_t* __restrict__ cnt,
                                                               const int64_t* __restrict__ off,
                                                               const uint32_t* __restrict__ ops,
                                                               uint32_t* __restrict__ packed) {
    const int32_t pair = (int32_t)blockIdx.x * kAlWaves + (int32_t)(threadIdx.x / kLanes);
    if (pair >= n) return;
    const int64_t src = pairs[pair].ops_off, dst = off[pair];
    for (int32_t j = (int32_t)(threadIdx.x & (kLanes - 1)); j < cnt[pair]; j += kLanes)
        packed[dst + j] = ops[src + j];
}

}  // namespace hs
