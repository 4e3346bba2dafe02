// Smith-Waterman search with affine gaps: the exact local-alignment optimum
// of one query against every target, the baseline the paper sets its
// heuristic against (Sections I and IV compare its speed and sensitivity
// with Smith-Waterman).  Smith & Waterman (1981) local alignment with
// Gotoh's (1982) three-state recurrence; a gap run of g columns costs
// GOP + (g - 1) * GEP, the gap convention of Section III.B.1.
//
// Layout: one lane per target, lanes taking the targets longest first (the
// database's order array) so that the 64 targets of a wavefront have
// similar lengths.  A lane sweeps its target in passes of kSwRows query
// rows; the rows' H and horizontal-gap values live in registers and move
// along the target one column per iteration.  The substitution scores of a
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
constexpr int32_t kSwNeg = -(1 << 29);   // minus infinity; one subtraction stays in range

// Query profile bytes in LDS for a query of qlen letters.
__host__ __device__ inline int32_t sw_profile_stride(int32_t qlen) {
    return (qlen + kSwRows - 1) / kSwRows * kSwRows;
}

__device__ __forceinline__ int32_t sw_byte(uint32_t w, int k) {
    return (int32_t)(int8_t)(uint8_t)(w >> (8 * k));
}

// scores[t] = optimal local score of the query against target t (index
// order).  col: workspace of one int2 per database letter (index as the
// letters).  LDS: kNsym * qp bytes.
__global__ __launch_bounds__(kSwThreads) void k_sw_scores(
    DbView db, const uint8_t* __restrict__ q, int32_t qlen, int32_t qp, KMatrix km, int32_t gop,
    int32_t gep, int2* __restrict__ col, int32_t* __restrict__ scores) {
    extern __shared__ __align__(16) uint8_t sw_prof[];
    for (int32_t w = threadIdx.x; w < kNsym * qp; w += blockDim.x) {
        const int32_t c = w / qp, i = w - c * qp;
        // codes outside the alphabet read row kNsym - 1 (never outside the matrix)
        const int32_t qc = i < qlen ? min((int32_t)q[i], kNsym - 1) : 0;
        sw_prof[w] = i < qlen ? (uint8_t)km.m[qc * kNsym + c] : (uint8_t)0;
    }
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= db.n) return;
    const int32_t tgt = db.order[g];
    const int32_t tlen = db.lens[tgt];
    const int64_t off = db.offsets[tgt];
    const uint8_t* __restrict__ t = db.letters + off;
    int2* __restrict__ cb = col + off;
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
            const uint4 sv = *(const uint4*)(sw_prof + c * qp + i0);
            int32_t diag = top_prev;
            top_prev = up;
#pragma unroll
            for (int r = 0; r < kSwRows; ++r) {
                const uint32_t word = r < 4 ? sv.x : r < 8 ? sv.y : r < 12 ? sv.z : sv.w;
                const int32_t s = sw_byte(word, r & 3);
                v = max(up - gop, v - gep);                 // gap in the target, down column j
                const int32_t f = max(H[r] - gop, Fr[r] - gep);   // gap in the query, along row i
                Fr[r] = f;
                const int32_t h = max(max(diag + s, v), max(f, 0));
                diag = H[r];
                H[r] = h;
                up = h;
                if (r < valid) best = max(best, h);
            }
            if (!last) cb[j] = make_int2(up, v);
        }
    }
    scores[tgt] = best;
}

}  // namespace hs
