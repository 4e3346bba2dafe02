// traceback_kernels.hpp -- alignments for the best hits only.  The scoring
// pass keeps no per-pair state beyond the score and the winning round (the
// constant auxiliary space of Section III.B.4); the aligned rows of the top
// hits are recovered by replaying that round, which is deterministic because
// every draw is keyed by (seed, target, round, draw index).  Every step's
// placements are scored in blocks of 8 diagonals by the scoring pass's own
// block scorer, so every step picks the placement the scoring pass picked,
// and each chosen placement becomes run-length ops.  Two replays:
//   * wave_trace_one (one query's hits): a wavefront replays one hit at a
//     time, all its lanes sharing the pair state and taking a step's blocks
//     side by side -- the fewest instructions per step, for hits that run
//     on an otherwise idle device;
//   * wave_trace_slots (a batch's hits): the scoring pass's slot scheduler
//     with several hits per wavefront, so that they share each phase's
//     fixed cost.
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

// One alignment being recovered (held by its lane in wave_trace_slots, by
// every lane of the wavefront in wave_trace_one): the winning round of a hit
// replayed step by step, each step's placement appended to the alignment's
// ops.  Plain scalars only, so that the whole state stays in registers.
struct TraceState {
    int32_t id;          // target index, -1 when the slot is empty
    int32_t a;           // alignment index (hits[a], alns[a])
    int32_t nl, ns;
    bool tl;             // target is the large sequence
    int32_t round, t;
    uint32_t LF, SF;
    int32_t pL, pS, score;
    int32_t ss, blk, nblk;
    bool stepping;
    int64_t tbase;
    int32_t dblk;                    // Philox block held in w0..w3 (-1: none)
    uint64_t w0, w1, w2, w3;
    uint32_t* out;                   // the alignment's ops
    int32_t n_ops;
    uint32_t op, len;                // run being merged
};

// random() draw d of the replayed round (same stream as the scoring pass).
__device__ __forceinline__ uint32_t trace_draw(TraceState& s, uint64_t seed, uint32_t d) {
    const int32_t b = (int32_t)(d >> 4);
    if (b != s.dblk) {
        uint64_t w[4];
        philox_block(seed, (uint64_t)s.id, (uint32_t)s.round, (uint32_t)b, w);
        s.w0 = w[0];
        s.w1 = w[1];
        s.w2 = w[2];
        s.w3 = w[3];
        s.dblk = b;
    }
    const uint32_t wi = (d >> 2) & 3;
    const uint64_t x = wi == 0 ? s.w0 : wi == 1 ? s.w1 : wi == 2 ? s.w2 : s.w3;
    return (uint32_t)(x >> (16 * (d & 3))) & 0xFFFFu;
}

// Appends a run of l ops o, merging it with the previous run of the same op
// (only the lane with `w` stores).
__device__ __forceinline__ void trace_emit(TraceState& s, uint32_t o, int32_t l, bool w) {
    if (l <= 0) return;
    if (s.len && o == s.op) {
        s.len += (uint32_t)l;
        return;
    }
    if (s.len) {
        if (w) s.out[s.n_ops] = (s.len << 2) | s.op;
        ++s.n_ops;
    }
    s.op = o;
    s.len = (uint32_t)l;
}

// Draws the next step of the alignment or, after the last one, writes the
// alignment: inside the chop-and-consume loop only the small sequence
// receives gaps (Section III.B.3) -- the k* skipped letters of large are
// target letters over gaps (D) when the target is large and query letters
// over gaps (I) otherwise -- and after the loop the rest of whichever
// sequence is left goes against gaps.
__device__ __forceinline__ void trace_advance(TraceState& s, const KParams& kp, SlotInfo* slot,
                                              DevAln* __restrict__ alns, int64_t ops_off) {
    if (s.id < 0 || s.stepping) return;
    if (s.pL < s.nl && s.pS < s.ns) {
        const int32_t ls = window_large(s.nl - s.pL, s.LF);
        const int32_t ss =
            window_small(s.ns - s.pS, s.SF, trace_draw(s, kp.seed, 2u + (uint32_t)s.t), ls);
        const int32_t nk = ls - ss + 1;
        s.ss = ss;
        s.blk = 0;
        s.nblk = (nk + kBlockDiags - 1) / kBlockDiags;
        s.stepping = true;
        SlotInfo si;
        si.pL = s.pL;
        si.pS = s.pS;
        si.ss_tl = ss | (s.tl ? (int32_t)0x80000000 : 0);
        si.nk = nk;
        si.tbase = s.tbase;
        si.key = 0;
        *slot = si;
        return;
    }
    s.score -= kp.pgp * ((s.nl - s.pL) + (s.ns - s.pS));
    trace_emit(s, s.tl ? kOpD : kOpI, s.nl - s.pL, true);
    trace_emit(s, s.tl ? kOpI : kOpD, s.ns - s.pS, true);
    if (s.len) s.out[s.n_ops++] = (s.len << 2) | s.op;
    DevAln out;
    out.target_id = s.id;
    out.score = s.score;
    out.n_ops = s.n_ops;
    out.ops_off = ops_off;
    alns[s.a] = out;
    s.id = -1;
}

// Slot-based replay (a batch's hits): one wavefront's share of the
// alignments of one query, hit indices below `hi` taken from the workgroup
// counter `ctr`, at most `cap` in flight, one per lane.  The winning round of
// each hit is replayed on the scoring pass's scheduler and block scorer (so
// every step picks the same placement) and alignment a is written to
// alns[a], its ops to ops[ops_base + a * ops_stride ...].
template <int kCopies>
__device__ __forceinline__ void wave_trace_slots(WaveLds& W, int32_t lane, int32_t cap,
                                                 const uint8_t* prof, int32_t ps, int32_t cpb,
                                                 int32_t bias, int32_t qlen, const KParams& kp,
                                                 const DbView& db, const DevHit* __restrict__ hits,
                                                 uint32_t hi, uint32_t* ctr, DevAln* __restrict__ alns,
                                                 uint32_t* __restrict__ ops, int64_t ops_base,
                                                 int64_t ops_stride) {
    TraceState s;
    s.id = -1;
    s.stepping = false;
    bool exhausted = false;
    for (;;) {
        // ---- phase A: apply last step's winner, advance, refill ----
        if (s.id >= 0 && s.stepping && s.blk >= s.nblk) {
            const uint64_t key = W.slots[lane].key;
            const int32_t kb = key_shift(key);
            s.score += key_score(key) - shift_penalty(kp, s.t, kb);
            trace_emit(s, s.tl ? kOpD : kOpI, kb, true);
            trace_emit(s, kOpM, s.ss, true);
            s.pL += kb + s.ss;
            s.pS += s.ss;
            ++s.t;
            s.stepping = false;
        }
        trace_advance(s, kp, &W.slots[lane], alns, ops_base + (int64_t)s.a * ops_stride);
        for (;;) {
            const bool need = s.id < 0 && !exhausted && lane < cap;
            const uint64_t mask = __ballot(need);
            if (!mask) break;
            const uint32_t cnt = (uint32_t)__popcll(mask);
            const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(ctr, cnt);
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
            const uint32_t a = base + rank;
            if (need) {
                if (a < hi) {
                    const DevHit h = hits[a];
                    const int32_t id = (int32_t)h.target_id;
                    if (id >= 0 && id < db.n && h.round >= 0 && h.round < kp.rounds) {
                        const int32_t tlen = db.lens[id];
                        s.id = id;
                        s.a = (int32_t)a;
                        s.tl = tlen >= qlen;
                        s.nl = s.tl ? tlen : qlen;
                        s.ns = s.tl ? qlen : tlen;
                        s.tbase = db.offsets[id];
                        s.round = h.round;
                        s.dblk = -1;
                        s.LF = round_factor(kp.lfactor, kp.minfactor, trace_draw(s, kp.seed, 0));
                        s.SF = round_factor(kp.sfactor, kp.minfactor, trace_draw(s, kp.seed, 1));
                        s.pL = s.pS = s.t = s.score = 0;
                        s.stepping = false;
                        s.out = ops + ops_base + (int64_t)a * ops_stride;
                        s.n_ops = 0;
                        s.op = 0;
                        s.len = 0;
                        trace_advance(s, kp, &W.slots[lane], alns, ops_base + (int64_t)a * ops_stride);
                    }
                } else {
                    exhausted = true;
                }
            }
            if (__ballot(s.id >= 0) != 0) break;
        }
        if (__ballot(s.id >= 0) == 0) break;
        // ---- phases B and C ----
        // a few hits run on an otherwise idle device: latency, not occupancy,
        // bounds the replay, so it takes the high-ILP letter loop
        score_pending<kCopies, true>(W, lane, s.id >= 0 && s.stepping, s.tl, s.ss, s.blk, s.nblk,
                                     prof, ps, cpb, bias, db.letters);
    }
}

// One wavefront's share of the alignments of one query: hit indices below
// `hi`, taken one at a time from the workgroup counter `ctr`; alignment a is
// written to alns[a], its ops to ops[ops_base + a * ops_stride ...].
//
// The winning round of each hit is replayed step by step.  Inside the
// chop-and-consume loop only the small sequence receives gaps (Section
// III.B.3) -- the k* skipped letters of large are target letters over gaps
// (D) when the target is large and query letters over gaps (I) otherwise --
// and after the loop the rest of whichever sequence is left goes against
// gaps.  A step's blocks of 8 placements go to lanes 0, 1, ... (64 at a
// time); the best block key over the wavefront is the step's placement.
template <int kCopies>
__device__ __forceinline__ void wave_trace_one(int32_t lane, const uint8_t* prof, int32_t ps,
                                           int32_t cpb, int32_t bias, int32_t qlen,
                                           const KParams& kp, const DbView& db,
                                           const DevHit* __restrict__ hits, uint32_t hi,
                                           uint32_t* ctr, DevAln* __restrict__ alns,
                                           uint32_t* __restrict__ ops, int64_t ops_base,
                                           int64_t ops_stride, uint8_t* stage, int32_t stage_bytes) {
    const bool w = lane == 0;     // the lane that stores
    for (;;) {
        uint32_t a = 0;
        if (w) a = atomicAdd(ctr, 1u);
        a = (uint32_t)__builtin_amdgcn_readlane((int)a, 0);
        if (a >= hi) return;
        const DevHit h = hits[a];
        const int32_t id = (int32_t)h.target_id;
        if (id < 0 || id >= db.n || h.round < 0 || h.round >= kp.rounds) continue;
        TraceState s;
        const int32_t tlen = db.lens[id];
        s.id = id;
        s.tl = tlen >= qlen;
        s.nl = s.tl ? tlen : qlen;
        s.ns = s.tl ? qlen : tlen;
        s.tbase = db.offsets[id];
        // the target's letters from LDS when they fit in the stage
        const bool staged = stage_target(lane, db.letters + s.tbase, tlen, stage, stage_bytes);
        const uint8_t* base = staged ? (const uint8_t*)stage : db.letters;
        if (staged) s.tbase = 0;
        s.round = h.round;
        s.dblk = -1;
        s.LF = round_factor(kp.lfactor, kp.minfactor, trace_draw(s, kp.seed, 0));
        s.SF = round_factor(kp.sfactor, kp.minfactor, trace_draw(s, kp.seed, 1));
        s.pL = s.pS = s.t = s.score = 0;
        s.out = ops + ops_base + (int64_t)a * ops_stride;
        s.n_ops = 0;
        s.op = 0;
        s.len = 0;
        while (s.pL < s.nl && s.pS < s.ns) {
            const int32_t ls = window_large(s.nl - s.pL, s.LF);
            const int32_t ss =
                window_small(s.ns - s.pS, s.SF, trace_draw(s, kp.seed, 2u + (uint32_t)s.t), ls);
            const int32_t nk = ls - ss + 1;
            const uint64_t best = wave_step_key<kCopies>(lane, prof, ps, cpb, bias, base, s.tbase,
                                                         s.tl, s.pL, s.pS, ss, nk);
            const int32_t kb = key_shift(best);
            s.score += key_score(best) - shift_penalty(kp, s.t, kb);
            trace_emit(s, s.tl ? kOpD : kOpI, kb, w);
            trace_emit(s, kOpM, ss, w);
            s.pL += kb + ss;
            s.pS += ss;
            ++s.t;
        }
        s.score -= kp.pgp * ((s.nl - s.pL) + (s.ns - s.pS));
        trace_emit(s, s.tl ? kOpD : kOpI, s.nl - s.pL, w);
        trace_emit(s, s.tl ? kOpI : kOpD, s.ns - s.pS, w);
        if (s.len) {
            if (w) s.out[s.n_ops] = (s.len << 2) | s.op;
            ++s.n_ops;
        }
        if (w) {
            DevAln out;
            out.target_id = s.id;
            out.score = s.score;
            out.n_ops = s.n_ops;
            out.ops_off = ops_base + (int64_t)a * ops_stride;
            alns[a] = out;
        }
    }
}

// LDS of a one-query replay workgroup of `waves` wavefronts: the profile
// region, the substitution rows staged by build_profile, then (when it fits)
// one target buffer of a wavefront record's size per wavefront.
__host__ __device__ inline int32_t trace_stage_offset(int32_t prof_bytes) {
    return prof_bytes + ((kProfRows * kNsym + 15) & ~15);
}
__host__ __device__ inline int32_t trace_lds_bytes(int32_t prof_bytes, int32_t waves) {
    return trace_stage_offset(prof_bytes) + waves * (int32_t)sizeof(WaveLds);
}

// Alignments of one query: workgroup g recovers hits [g * per_wg, (g + 1) *
// per_wg) below min(n_aln, n_hits), one per wavefront at a time; with
// stage_bytes > 0 each wavefront has a target buffer of that size.
template <int kCopies>
__global__ __launch_bounds__(kThreads) void k_trace_sched(
    DbView db, const uint8_t* __restrict__ qcodes, int32_t qlen, KParams kp, KMatrix km,
    int32_t bias, const DevHit* __restrict__ hits, const int32_t* __restrict__ n_hits,
    int32_t n_aln, int32_t per_wg, DevAln* __restrict__ alns, uint32_t* __restrict__ ops,
    int64_t ops_stride, int32_t stage_bytes) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_ctr;
    const int32_t nh = *n_hits < n_aln ? *n_hits : n_aln;
    const int32_t lo = blockIdx.x * per_wg;
    const int32_t hi = lo + per_wg < nh ? lo + per_wg : nh;
    if (lo >= hi) return;
    const int32_t ps = profile_stride(qlen);
    const int32_t cpb = profile_copy_bytes(ps);
    build_profile<kCopies>(lds, ps, qcodes, qlen, km.m, bias, lds + profile_region_bytes(qlen, kCopies),
                           threadIdx.x, blockDim.x);
    if (threadIdx.x == 0) s_ctr = (uint32_t)lo;
    __syncthreads();
    uint8_t* stage = stage_bytes > 0 ? lds + trace_stage_offset(profile_region_bytes(qlen, kCopies)) +
                                           (threadIdx.x / kLanes) * stage_bytes
                                     : nullptr;
    wave_trace_one<kCopies>(threadIdx.x & (kLanes - 1), lds, ps, cpb, bias, qlen, kp, db, hits,
                            (uint32_t)hi, &s_ctr, alns, ops, 0, ops_stride, stage, stage_bytes);
}

// Alignments of a batch, persistent: a workgroup takes work items (query q,
// hit range [lo, hi)) from the counter, builds the query's profile and
// recovers the item's hits below min(hi, n_hits[q]): with `one`, one hit per
// wavefront at a time (a small batch, whose items all run at once); else up
// to `cap` per wavefront in flight (slot-based replay: a wavefront's hits
// share each phase's fixed cost).  Query q's hits start at
// hits[q * k], its alignments at alns[q * n_aln], and the ops of alignment
// (q, a) at ops[(q * n_aln + a) * ops_stride].
template <int kCopies>
__global__ __launch_bounds__(kThreads) void k_trace_batch(
    DbView db, const BatchQuery* __restrict__ qs, const KMatrix* __restrict__ mats,
    const uint8_t* __restrict__ qcodes, const BatchItem* __restrict__ items, int32_t n_items,
    uint32_t* item_ctr, int32_t prof_bytes, int32_t cap, int32_t one, int32_t k,
    const DevHit* __restrict__ hits, const int32_t* __restrict__ n_hits, int32_t n_aln,
    DevAln* __restrict__ alns, uint32_t* __restrict__ ops, int64_t ops_stride) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_item, s_ctr;
    const int32_t lane = threadIdx.x & (kLanes - 1);
    WaveLds& W = ((WaveLds*)(lds + prof_bytes))[threadIdx.x / kLanes];
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t it = atomicAdd(item_ctr, 1u);
            s_item = it;
            if (it < (uint32_t)n_items) s_ctr = items[it].lo;
        }
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
        if (it >= (uint32_t)n_items) break;
        const BatchItem item = items[it];
        const int32_t q = item.q;
        const int32_t nh = n_hits[q] < n_aln ? n_hits[q] : n_aln;
        const uint32_t hi = item.hi < (uint32_t)nh ? item.hi : (uint32_t)nh;
        if (item.lo < hi) {
            const BatchQuery Q = qs[q];
            const int32_t ps = profile_stride(Q.qlen);
            const int32_t cpb = profile_copy_bytes(ps);
            build_profile<kCopies>(lds, ps, qcodes + Q.qoff, Q.qlen, mats[q].m, Q.bias, lds + prof_bytes,
                                   threadIdx.x, blockDim.x);
            __syncthreads();
            if (one)
                // the wavefront's record is unused here: it stages the targets
                wave_trace_one<kCopies>(lane, lds, ps, cpb, Q.bias, Q.qlen, Q.kp, db,
                                        hits + (int64_t)q * k, hi, &s_ctr, alns + (int64_t)q * n_aln,
                                        ops, (int64_t)q * n_aln * ops_stride, ops_stride, (uint8_t*)&W,
                                        (int32_t)sizeof(WaveLds));
            else
                wave_trace_slots<kCopies>(W, lane, cap, lds, ps, cpb, Q.bias, Q.qlen, Q.kp, db,
                                          hits + (int64_t)q * k, hi, &s_ctr, alns + (int64_t)q * n_aln,
                                          ops, (int64_t)q * n_aln * ops_stride, ops_stride);
        }
        __syncthreads();   // the profile and the counter are rewritten for the next item
    }
}

// Packing of a batch's alignments: pos[i] = where alignment slot
// i = q * n_aln + a starts in a packed ops buffer (slots past the query's
// hit count hold no ops), pos[nq * n_aln] = the total.  One workgroup.
__global__ __launch_bounds__(1024) void k_ops_scan(const DevAln* __restrict__ alns,
                                                   const int32_t* __restrict__ n_hits, int32_t nq,
                                                   int32_t n_aln, int64_t* __restrict__ pos) {
    __shared__ int64_t part[1024];
    const int32_t total = nq * n_aln;
    const int32_t tid = threadIdx.x;
    int64_t carry = 0;
    for (int32_t base = 0; base < total; base += 1024) {
        const int32_t i = base + tid;
        int64_t v = 0;
        if (i < total) {
            const int32_t q = i / n_aln, a = i - q * n_aln;
            if (a < n_hits[q]) v = alns[i].n_ops;
        }
        part[tid] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const int64_t y = tid >= o ? part[tid - o] : 0;
            __syncthreads();
            part[tid] += y;
            __syncthreads();
        }
        if (i < total) pos[i] = carry + part[tid] - v;
        carry += part[1023];
        __syncthreads();
    }
    if (tid == 0) pos[total] = carry;
}

// Copies the ops of alignment (q = blockIdx.y, a = blockIdx.x) to the packed
// buffer at pos[q * n_aln + a].
__global__ __launch_bounds__(64) void k_ops_gather(const DevAln* __restrict__ alns,
                                                   const int32_t* __restrict__ n_hits,
                                                   int32_t n_aln, const uint32_t* __restrict__ ops,
                                                   const int64_t* __restrict__ pos,
                                                   uint32_t* __restrict__ packed) {
    const int32_t a = blockIdx.x, q = blockIdx.y;
    if (a >= n_hits[q]) return;
    const int64_t i = (int64_t)q * n_aln + a;
    const DevAln al = alns[i];
    for (int32_t j = threadIdx.x; j < al.n_ops; j += blockDim.x) packed[pos[i] + j] = ops[al.ops_off + j];
}

}  // namespace hs
