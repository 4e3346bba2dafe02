// device_common.hpp -- shared device-side pieces of the search library:
// the keyed random stream behind random() of Fig. 1, parameters in kernel
// form, the database view and the window arithmetic of one step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

constexpr int kNsym = 24;         // BLOSUM62 alphabet ARNDCQEGHILKMFPSTWYVBZX*
constexpr int kLanes = 64;        // wavefront width
constexpr int kZeroRow = 24;      // profile row of zeros (no-op lookups)
constexpr int kProfRows = 25;
constexpr int kPad = 8;           // zero profile columns on each side of the query
constexpr int kLetterPad = 64;    // readable bytes after the last target letter

// Parameters of Section III.B.1 as the kernels use them.
struct KParams {
    int32_t gop, gep, pgp;
    uint32_t lfactor, sfactor, minfactor;   // Q16
    int32_t rounds;
    int32_t min_score;
    uint64_t seed;
};

// 24x24 substitution matrix passed by value in the kernel arguments.
struct KMatrix {
    int8_t m[kNsym * kNsym];
};

// One query of a batch as the batch kernels read it from device memory.
struct BatchQuery {
    KParams kp;
    int64_t qoff;       // first code of the query in the batch's code array
    int32_t qlen;
    int32_t bias;       // makes every entry of the query's matrix a byte in 0..15
    int32_t table;      // 1: the round-0 draw table was filled with kp.seed
    int32_t pad_;
};

// Work item of the batch scoring kernel: hand-out positions [lo, hi) of the
// database for query q.
struct BatchItem {
    int32_t q;
    uint32_t lo, hi;
    int32_t pad_;
};

// Device image of a database: one byte (alphabet code) per residue, targets
// concatenated in index order, followed by kLetterPad readable bytes.
// `order` lists target indices longest first: the order in which pairs are
// handed out, so that the longest pairs start early.
struct DbView {
    const uint8_t* letters;
    const int64_t* offsets;     // start of target i in letters
    const int32_t* lens;
    const int32_t* order;
    int32_t n;
};

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Each round multiplies
// words 0 and 2 by the two Philox constants (full 128-bit products), mixes the
// high halves into the other two words with the round key and swaps; the key
// is advanced by the two Weyl increments between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t& x0, uint64_t& x1, uint64_t& x2,
                                              uint64_t& x3, uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a_lo = kMulA * x0, a_hi = __umul64hi(kMulA, x0);
        const uint64_t b_lo = kMulB * x2, b_hi = __umul64hi(kMulB, x2);
        const uint64_t y0 = b_hi ^ x1 ^ k0;
        const uint64_t y2 = a_hi ^ x3 ^ k1;
        x0 = y0; x1 = b_lo; x2 = y2; x3 = a_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
}

// The random fractions of one (target, round): 16-bit values, sixteen per
// Philox block.  Draw d lives in block d / 16 (counter = (target, round,
// d / 16, 0), key = (seed, 0)), word (d / 4) % 4, bits 16 * (d % 4).
__device__ __forceinline__ void philox_block(uint64_t seed, uint64_t target, uint32_t round,
                                             uint32_t block, uint64_t w[4]) {
    w[0] = target; w[1] = round; w[2] = block; w[3] = 0;
    philox4x64_10(w[0], w[1], w[2], w[3], seed, 0);
}

// Per-round factor (Fig. 1, ALGORITHM AlignSequences): a random fraction
// raised to at least MinFactor, scaled by LFactor (or SFactor), Q16.
__device__ __forceinline__ uint32_t round_factor(uint32_t factor, uint32_t minf, uint32_t u) {
    return (uint32_t)(((uint64_t)factor * (u < minf ? minf : u)) >> 16);
}

// Window sizes of one step (Fig. 1, PROCEDURE Align), Q16 fixed point.
__device__ __forceinline__ int32_t window_large(int32_t rem_large, uint32_t LF) {
    const int32_t ls = (int32_t)(((uint64_t)rem_large * LF) >> 16);
    return ls < 1 ? 1 : ls;
}
__device__ __forceinline__ int32_t window_small(int32_t rem_small, uint32_t SF, uint32_t u,
                                                int32_t ls) {
    int32_t ss = (int32_t)(((uint64_t)rem_small * SF * u) >> 32);
    ss = ss < 1 ? 1 : ss;
    return ss > ls ? ls : ss;
}

// Gap cost of the shift chosen at step t (Section III.B.1): the first
// step's leading gap is periphery, later ones are internal runs.
__device__ __forceinline__ int32_t shift_penalty(const KParams& p, int32_t t, int32_t k) {
    if (t == 0) return p.pgp * k;
    return k > 0 ? p.gop + (k - 1) * p.gep : 0;
}

// Key of a placement for the first-best rule: larger score first, then the
// smaller shift; comparing keys as unsigned integers picks the winner.
__device__ __forceinline__ uint64_t shift_key(int32_t D, int32_t k) {
    return ((uint64_t)((uint32_t)D ^ 0x80000000u) << 32) | (uint64_t)(~(uint32_t)k);
}
__device__ __forceinline__ int32_t key_score(uint64_t key) {
    return (int32_t)((uint32_t)(key >> 32) ^ 0x80000000u);
}
__device__ __forceinline__ int32_t key_shift(uint64_t key) { return (int32_t)(~(uint32_t)key); }

}  // namespace hs
