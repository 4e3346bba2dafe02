// device_common.hpp -- shared device-side pieces of the search library:
// the keyed random stream behind random() of Fig. 1, parameters in kernel
// form, and the packed database view.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hs {

constexpr int kNsym = 24;         // BLOSUM62 alphabet ARNDCQEGHILKMFPSTWYVBZX*
constexpr int kLanes = 64;        // wavefront width; also the interleave width
constexpr int kResPerWord = 6;    // 5-bit residue codes per 32-bit word

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

// Device image of a database.  Targets are sorted by length (longest first)
// and dealt into groups of 64; group g occupies rows of 64 words starting at
// words[group_base[g]], lane l of the group reading word w at
// words[group_base[g] + w * 64 + l], so that a wavefront whose lanes walk
// their targets in step reads 256 contiguous bytes.
struct DbView {
    const uint32_t* words;
    const int64_t* group_base;
    const int32_t* slot_id;     // g * 64 + lane -> target index, -1 if empty
    const int32_t* slot_len;    // g * 64 + lane -> length
    const int32_t* loc;         // target index -> g * 64 + lane
    int32_t n_groups;
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
struct DrawStream {
    uint64_t seed, target;
    uint32_t round;
    int32_t block;
    uint64_t w0, w1, w2, w3;

    __device__ __forceinline__ void init(uint64_t s, uint64_t t, uint32_t r) {
        seed = s; target = t; round = r; block = -1;
    }
    __device__ __forceinline__ uint32_t get(uint32_t d) {
        const int32_t b = (int32_t)(d >> 4);
        if (b != block) {
            block = b;
            w0 = target; w1 = round; w2 = (uint64_t)b; w3 = 0;
            philox4x64_10(w0, w1, w2, w3, seed, 0);
        }
        const uint32_t wi = (d >> 2) & 3;
        const uint64_t w = wi == 0 ? w0 : wi == 1 ? w1 : wi == 2 ? w2 : w3;
        return (uint32_t)(w >> (16 * (d & 3))) & 0xFFFFu;
    }
};

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

// Sequential reader of one interleaved target: returns 5-bit codes from
// position p onwards.  Reads one word ahead, so the word array carries one
// spare row of padding after the last group.
struct TargetStream {
    const uint32_t* ptr;
    uint32_t w;
    int32_t ph;
    __device__ __forceinline__ void seek(const uint32_t* lane_base, int32_t p) {
        const int32_t q = p / kResPerWord;
        ph = p - q * kResPerWord;
        ptr = lane_base + (int64_t)q * kLanes;
        w = *ptr >> (5 * ph);
    }
    __device__ __forceinline__ uint32_t next() {
        const uint32_t r = w & 31u;
        if (++ph == kResPerWord) {
            ph = 0;
            ptr += kLanes;
            w = *ptr;
        } else {
            w >>= 5;
        }
        return r;
    }
};

}  // namespace hs
