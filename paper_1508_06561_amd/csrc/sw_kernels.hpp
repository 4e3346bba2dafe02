// Smith-Waterman search with affine gaps: the exact local-alignment optimum
// of one query against every target, the baseline the paper sets its
// heuristic against (Sections I and IV compare its speed and sensitivity
// with Smith-Waterman).  Smith & Waterman (1981) local alignment with
// Gotoh's (1982) three-state recurrence; a gap run of g columns costs
// GOP + (g - 1) * GEP, the gap convention of Section III.B.1.
//
// Layout: most targets take one lane each, longest first (the database's
// order array), so that the 64 targets of a wavefront have similar lengths;
// the longest targets take a whole wavefront each (sw_wave below), so that
// no single lane sets the launch's critical path.  A lane sweeps its target
// in passes of kSwRows query rows; the rows' H and horizontal-gap values
// live in registers and move along the target one column per iteration.  The substitution scores of a
// column for all kSwRows rows are one 16-byte LDS read from the query
// profile (kNsym rows of qp bytes: score of query position i against code
// c at c * qp + i).  Between passes the bottom row's H and vertical-gap
// values go to a per-letter workspace (8 bytes per target letter, written
// by one pass and read by the next), about one byte of traffic per cell.
#pragma once

#include "device_common.hpp"

namespace hs {

constexpr int kSwRows = 16;          // query rows per pass: one 16-byte profile read
constexpr int kSwThreads = 256;
constexpr int kSwWaveRows = kSwRows * kLanes;    // query rows per pass of the wavefront role
constexpr int32_t kSwNeg = -(1 << 29);   // minus infinity; one subtraction stays in range
constexpr int32_t kSwGroupMin = 1;       // shortest group-role target, in group lanes

// Query profile bytes in LDS for a query of qlen letters.
__host__ __device__ inline int32_t sw_profile_stride(int32_t qlen) {
    return (qlen + kSwRows - 1) / kSwRows * kSwRows;
}

__device__ __forceinline__ int32_t sw_byte(uint32_t w, int k) {
    return (int32_t)(int8_t)(uint8_t)(w >> (8 * k));
}

// One column of kSwRows rows: sv holds the rows' substitution scores, H and
// Fr the rows' values at the previous column, top_prev H[i0-1][j-1]; up and
// v enter as H[i0-1][j] and the vertical gap into row i0 and leave as the
// bottom row's.  Rows r >= valid are outside the query and not counted in
// best.
__device__ __forceinline__ void sw_column(const uint4& sv, int32_t (&H)[kSwRows],
                                          int32_t (&Fr)[kSwRows], int32_t& top_prev, int32_t& up,
                                          int32_t& v, int32_t& best, int32_t valid, int32_t gop,
                                          int32_t gep) {
    int32_t diag = top_prev;
    top_prev = up;
#pragma unroll
    for (int r = 0; r < kSwRows; ++r) {
        const uint32_t word = r < 4 ? sv.x : r < 8 ? sv.y : r < 12 ? sv.z : sv.w;
        const int32_t s = sw_byte(word, r & 3);
        v = max(up - gop, v - gep);                        // gap in the target, down column j
        const int32_t f = max(H[r] - gop, Fr[r] - gep);    // gap in the query, along row i
        Fr[r] = f;
        const int32_t h = max(max(diag + s, v), max(f, 0));
        diag = H[r];
        H[r] = h;
        up = h;
        if (r < valid) best = max(best, h);
    }
}

// Lane role: the whole target on one lane, in passes of kSwRows query rows;
// the bottom row of a pass goes to cb (one int2 per target letter) for the
// next.  Returns the best cell.
__device__ __forceinline__ int32_t sw_lane(const uint8_t* __restrict__ t, int32_t tlen,
                                           int2* __restrict__ cb, const uint8_t* prof,
                                           int32_t qlen, int32_t qp, int32_t gop, int32_t gep) {
    int32_t best = 0;
    for (int32_t i0 = 0; i0 < qlen; i0 += kSwRows) {
        const bool first = i0 == 0;
        const bool last = i0 + kSwRows >= qlen;
        const int32_t valid = qlen - i0;          // rows r < valid are query rows
        int32_t H[kSwRows], Fr[kSwRows];          // H[i][j-1] and the horizontal gap along row i
#pragma unroll
        for (int r = 0; r < kSwRows; ++r) {
            H[r] = 0;
            Fr[r] = kSwNeg;
        }
        int32_t top_prev = 0;                     // H[i0-1][j-1]
        // the next column's letter and boundary load one iteration ahead
        int32_t c_next = t[0];
        int2 b_next = first ? make_int2(0, kSwNeg) : cb[0];
        for (int32_t j = 0; j < tlen; ++j) {
            const int32_t c = c_next;
            int32_t up = b_next.x, v = b_next.y;  // H[i0-1][j] and the vertical gap entering row i0
            if (j + 1 < tlen) {
                c_next = t[j + 1];
                if (!first) b_next = cb[j + 1];
            }
            const uint4 sv = *(const uint4*)(prof + c * qp + i0);
            sw_column(sv, H, Fr, top_prev, up, v, best, valid, gop, gep);
            if (!last) cb[j] = make_int2(up, v);
        }
    }
    return best;
}

// Wavefront role: a target on a group of G consecutive lanes of a
// wavefront (G = 64 for queries longer than one pass of kSwWaveRows rows;
// otherwise G = ceil(qlen / kSwRows), so that 64 / G targets share the
// wavefront and the lanes past the query's rows are not left idle), in
// passes of G * kSwRows query rows.  Lane ll of a group holds rows
// [p0 + 16 ll, p0 + 16 ll + 16) and works one column behind lane ll - 1,
// whose bottom row it takes by a one-lane shift at each step, so that a
// pass takes tlen + G - 1 steps.  Lane 0 of the group reads the previous
// pass's bottom row from cb, lane G - 1 writes its own there.  `active`
// lanes belong to a group with a target.  Returns each lane's best cell; the
// group's best is the maximum over its lanes.
__device__ __forceinline__ int32_t sw_wave(int32_t lane, int32_t G, bool active,
                                           const uint8_t* __restrict__ t, int32_t tlen,
                                           int2* __restrict__ cb, const uint8_t* prof, int32_t qlen,
                                           int32_t qp, int32_t gop, int32_t gep) {
    const int32_t ll = lane % G;
    int32_t steps = active ? tlen + G - 1 : 0;     // the same for every lane: the longest group
    for (int o = kLanes / 2; o >= 1; o >>= 1) steps = max(steps, __shfl_xor(steps, o));
    const int32_t rows_pass = G * kSwRows;
    int32_t best = 0;
    for (int32_t p0 = 0; p0 < qlen; p0 += rows_pass) {
        const bool first = p0 == 0;
        const bool last = p0 + rows_pass >= qlen;
        const int32_t i0 = p0 + ll * kSwRows;
        const int32_t valid = qlen - i0;          // rows r < valid are query rows
        const bool has_rows = active && valid > 0;
        const int32_t i0c = has_rows ? i0 : 0;
        int32_t H[kSwRows], Fr[kSwRows];
#pragma unroll
        for (int r = 0; r < kSwRows; ++r) {
            H[r] = 0;
            Fr[r] = kSwNeg;
        }
        int32_t top_prev = 0;
        int32_t out_h = 0, out_v = kSwNeg;        // this lane's bottom row at its last column
        int32_t c_next = (ll == 0 && active) ? t[0] : 0;    // step 0 works on column -ll
        int2 b_next = (ll == 0 && active && !first) ? cb[0] : make_int2(0, kSwNeg);
        for (int32_t st = 0; st < steps; ++st) {
            const int32_t j = st - ll;
            int32_t up = __shfl_up(out_h, 1);
            int32_t v = __shfl_up(out_v, 1);
            if (ll == 0) {
                up = b_next.x;
                v = b_next.y;
            }
            const int32_t c = c_next;
            const int32_t jn = j + 1;
            if (active && jn >= 0 && jn < tlen) {
                c_next = t[jn];
                if (ll == 0 && !first) b_next = cb[jn];
            }
            if (j >= 0 && j < tlen && has_rows) {
                const uint4 sv = *(const uint4*)(prof + c * qp + i0c);
                sw_column(sv, H, Fr, top_prev, up, v, best, valid, gop, gep);
                out_h = up;
                out_v = v;
                if (ll == G - 1 && !last) cb[j] = make_int2(up, v);
            }
        }
        __threadfence_block();   // lane G - 1's boundary stores land before lane 0 reads them
    }
    return best;
}

// Lanes per wavefront-role target: one pass of up to kSwWaveRows rows on as
// few lanes as hold the query, or the whole wavefront for longer queries.
__host__ __device__ inline int32_t sw_group_lanes(int32_t qlen) {
    return qlen > kSwWaveRows ? kLanes : (qlen + kSwRows - 1) / kSwRows;
}

// scores[t] = optimal local score of the query against target t (index
// order).  The n_long longest targets (order[0 .. n_long - 1]) take the
// wavefront role, 64 / G to a wavefront (G = sw_group_lanes(qlen)), in the
// first workgroups; the others take the lane role, one per lane.  col:
// workspace of one int2 per database letter (index as the letters).  LDS:
// kNsym * qp bytes.
__global__ __launch_bounds__(kSwThreads) void k_sw_scores(
    DbView db, int32_t n_long, const uint8_t* __restrict__ q, int32_t qlen, int32_t qp, KMatrix km,
    int32_t gop, int32_t gep, int2* __restrict__ col, int32_t* __restrict__ scores) {
    extern __shared__ __align__(16) uint8_t sw_prof[];
    for (int32_t w = threadIdx.x; w < kNsym * qp; w += blockDim.x) {
        const int32_t c = w / qp, i = w - c * qp;
        // codes outside the alphabet read row kNsym - 1 (never outside the matrix)
        const int32_t qc = i < qlen ? min((int32_t)q[i], kNsym - 1) : 0;
        sw_prof[w] = i < qlen ? (uint8_t)km.m[qc * kNsym + c] : (uint8_t)0;
    }
    __syncthreads();
    constexpr int kWavesPerBlock = kSwThreads / kLanes;
    const int32_t G = sw_group_lanes(qlen), NG = kLanes / G;
    const int32_t per_block = kWavesPerBlock * NG;
    const int32_t wave_blocks = (n_long + per_block - 1) / per_block;
    if ((int32_t)blockIdx.x < wave_blocks) {
        const int32_t w = (int32_t)blockIdx.x * kWavesPerBlock + (int32_t)(threadIdx.x / kLanes);
        if (w * NG >= n_long) return;             // uniform over the wavefront
        const int32_t lane = threadIdx.x & (kLanes - 1);
        const int32_t g = lane / G, slot = w * NG + g;
        const bool active = g < NG && slot < n_long;
        const int32_t tgt = active ? db.order[slot] : 0;
        const int64_t off = active ? db.offsets[tgt] : 0;
        const int32_t tlen = active ? db.lens[tgt] : 0;
        const int32_t best = sw_wave(lane, G, active, db.letters + off, tlen, col + off, sw_prof, qlen,
                                     qp, gop, gep);
        // the group's best: lane 0 of the group takes the maximum over its lanes
        int32_t gb = best;
        for (int32_t k = 1; k < G; ++k) {
            const int32_t o = __shfl(best, lane + k < kLanes ? lane + k : lane);
            if (lane % G + k < G) gb = max(gb, o);
        }
        if (active && lane % G == 0) scores[tgt] = gb;
        return;
    }
    const int64_t g = (int64_t)(blockIdx.x - wave_blocks) * blockDim.x + threadIdx.x + n_long;
    if (g >= db.n) return;
    const int32_t tgt = db.order[g];
    const int64_t off = db.offsets[tgt];
    scores[tgt] = sw_lane(db.letters + off, db.lens[tgt], col + off, sw_prof, qlen, qp, gop, gep);
}

}  // namespace hs
