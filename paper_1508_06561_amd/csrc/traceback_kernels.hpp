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

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    for (int o = kLanes / 2; o > 0; o >>= 1) {
        const uint64_t y = __shfl_xor(x, o, kLanes);
        x = y > x ? y : x;
    }
    return x;
}

// Replays the winning round of one hit with the query profile (one copy) in
// LDS, lanes splitting each step's placements, and writes the alignment as
// ops oriented (query, target).  Inside the chop-and-consume loop only the
// small sequence receives gaps (Section III.B.3): the k* skipped letters of
// large are target letters over gaps (D) when the target is large and query
// letters over gaps (I) otherwise; after the loop the rest of whichever
// sequence is left goes against gaps.
__device__ __forceinline__ void traceback_one(const DbView& db, const uint8_t* prof, int32_t ps,
                                              int32_t qlen, const KParams& kp, int32_t bias,
                                              const DevHit& hit, DevAln* out_aln, uint32_t* ops,
                                              int64_t ops_off) {
    const int32_t lane = threadIdx.x;
    const int32_t id = (int32_t)hit.target_id;
    const int32_t r = hit.round;
    if (id < 0 || id >= db.n || r < 0 || r >= kp.rounds) return;   // never for a valid hit
    const int32_t tlen = db.lens[id];
    const uint8_t* T = db.letters + db.offsets[id];

    const bool tl = tlen >= qlen;
    const int32_t nl = tl ? tlen : qlen;
    const int32_t ns = tl ? qlen : tlen;
    const uint32_t gap_in_small = tl ? kOpD : kOpI;   // large letter over a gap
    const uint32_t gap_in_large = tl ? kOpI : kOpD;   // small letter over a gap

    DrawStream ds;
    ds.init(kp.seed, (uint64_t)id, (uint32_t)r);
    const uint32_t LF = round_factor(kp.lfactor, kp.minfactor, ds.get(0));
    const uint32_t SF = round_factor(kp.sfactor, kp.minfactor, ds.get(1));
    OpWriter w;
    w.init(ops + ops_off);
    int32_t pL = 0, pS = 0, t = 0, score = 0;
    while (pL < nl && pS < ns) {
        const int32_t ls = window_large(nl - pL, LF);
        const int32_t ss = window_small(ns - pS, SF, ds.get(2u + (uint32_t)t), ls);
        const int32_t nk = ls - ss + 1;
        uint64_t best = 0;
        for (int32_t k = lane; k < nk; k += kLanes) {
            int32_t D = 0;
            if (tl) {
                const uint8_t* col = prof + pS + kPad;
                for (int32_t j = 0; j < ss; ++j) D += col[(int32_t)T[pL + k + j] * ps + j];
            } else {
                const uint8_t* col = prof + pL + k + kPad;
                for (int32_t j = 0; j < ss; ++j) D += col[(int32_t)T[pS + j] * ps + j];
            }
            const uint64_t key = shift_key(D - bias * ss, k);
            best = key > best ? key : best;
        }
        best = wave_max_u64(best);
        const int32_t kb = key_shift(best);
        score += key_score(best) - shift_penalty(kp, t, kb);
        if (lane == 0) {
            w.emit(gap_in_small, kb);
            w.emit(kOpM, ss);
        }
        pL += kb + ss;
        pS += ss;
        ++t;
    }
    score -= kp.pgp * ((nl - pL) + (ns - pS));
    if (lane == 0) {
        w.emit(gap_in_small, nl - pL);
        w.emit(gap_in_large, ns - pS);
        w.flush();
        DevAln out;
        out.target_id = id;
        out.score = score;
        out.n_ops = w.n;
        out.ops_off = ops_off;
        *out_aln = out;
    }
}

// One wavefront per alignment a < min(n_aln, n_hits) of one query.
__global__ __launch_bounds__(64) void k_traceback(DbView db, const uint8_t* __restrict__ qcodes,
                                                  int32_t qlen, KParams kp, KMatrix km,
                                                  int32_t bias, const DevHit* __restrict__ hits,
                                                  const int32_t* __restrict__ n_hits, int32_t n_aln,
                                                  DevAln* __restrict__ alns,
                                                  uint32_t* __restrict__ ops, int64_t ops_stride) {
    extern __shared__ __align__(16) uint8_t prof[];
    const int32_t ps = profile_stride(qlen);
    build_profile<1>(prof, ps, qcodes, qlen, km, bias);
    __syncthreads();
    const int32_t a = blockIdx.x;
    if (a >= n_aln || a >= *n_hits) return;
    traceback_one(db, prof, ps, qlen, kp, bias, hits[a], alns + a, ops, (int64_t)a * ops_stride);
}

// Batch form: alignment a = blockIdx.x of query q = blockIdx.y; query q's
// hits start at hits[q * k], its alignments at alns[q * n_aln], and the ops
// of alignment (q, a) at ops[(q * n_aln + a) * ops_stride].
__global__ __launch_bounds__(64) void k_traceback_batch(
    DbView db, const BatchQuery* __restrict__ qs, const KMatrix* __restrict__ mats,
    const uint8_t* __restrict__ qcodes, int32_t nq, int32_t k, const DevHit* __restrict__ hits,
    const int32_t* __restrict__ n_hits, int32_t n_aln, DevAln* __restrict__ alns,
    uint32_t* __restrict__ ops, int64_t ops_stride) {
    extern __shared__ __align__(16) uint8_t prof[];
    const int32_t a = blockIdx.x, q = blockIdx.y;
    if (q >= nq || a >= n_aln || a >= n_hits[q]) return;
    const BatchQuery Q = qs[q];
    const int32_t ps = profile_stride(Q.qlen);
    build_profile<1>(prof, ps, qcodes + Q.qoff, Q.qlen, mats[q], Q.bias);
    __syncthreads();
    const int64_t slot = (int64_t)q * n_aln + a;
    traceback_one(db, prof, ps, Q.qlen, Q.kp, Q.bias, hits[(int64_t)q * k + a], alns + slot, ops,
                  slot * ops_stride);
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
