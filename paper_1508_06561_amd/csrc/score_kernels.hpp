// score_kernels.hpp -- pair scoring: the search-mode heuristic of Fig. 1
// (Section III.B.3: contained shifts only) for every (query, target) pair.
//
// Work decomposition.  A pair is a chain of steps; step t slides an ss-letter
// window of the small sequence over an ls-letter window of the large one and
// keeps the first best of nk = ls - ss + 1 placements (diagonals).  Every
// wavefront of a persistent workgroup runs on its own: it keeps 64 pairs in
// flight (one slot per lane; pairs are pulled from a global queue, longest
// first) and advances them in phases: every phase applies the previous step's
// winner to each slot, draws the next windows, cuts each step into blocks of
// 8 consecutive diagonals, counting-sorts the blocks by (orientation, ss) so
// that the lanes get blocks of equal length, and lets every lane score blocks.
// The workgroup's wavefronts share only the query profile, so one
// wavefront's memory waits are covered by the others' arithmetic.
//
// Block kernel.  The query profile lives in LDS as biased bytes (B + bias in
// 0..15), four copies shifted by one column so that every 8-column read is
// dword aligned.  For a block, one 8-byte read of the profile row of a target
// letter yields the 8 cells of that letter with 8 consecutive query columns,
// which belong to the block's 8 diagonals; they are added with one 32-bit add
// per 4 cells into byte-packed accumulators, widened to 16 bits every 16
// letters.
//   * target is small: iterate over the ss window letters of the target; the
//     8 columns are the 8 diagonals' query letters; no masking.
//   * target is large: iterate over the ss + 7 target letters the block
//     touches; letter i meets query columns pS + i - 7 .. pS + i, so the
//     first and last 7 letters carry cells outside the window: those bytes
//     are masked with compile-time masks (entry and exit ramps).
#pragma once

#include "device_common.hpp"
#include "topk_kernels.hpp"

namespace hs {

constexpr int kBlockDiags = 8;
constexpr int kWaves = 8;            // wavefronts per workgroup
constexpr int kThreads = kWaves * kLanes;
constexpr int kItemCap = 512;        // blocks issued per wavefront and phase
constexpr int kBins = 128;           // (orientation, ss bucket)

// Profile layout: copy s (0..kCopies-1) holds column c of row r at byte
// s * cpb + r * ps + (c + kPad - s).  With four copies, column c is read from
// copy (c + kPad) & 3 at a 4-aligned offset; with one copy (queries too long
// for four copies in LDS) reads are assembled from aligned dwords.  Columns outside [0, qlen) and
// row kZeroRow are 0.
// The row stride is an odd number of dwords, so that the 25 rows start in
// 25 different LDS banks: lanes reading different rows at one column (the
// blocks of one step) then rarely conflict.
__host__ __device__ inline int32_t profile_stride(int32_t qlen) {
    const int32_t ps = (qlen + 2 * kPad + 8 + 3) & ~3;
    return ((ps >> 2) & 1) ? ps : ps + 4;
}
__host__ __device__ inline int32_t profile_copy_bytes(int32_t ps) { return kProfRows * ps; }

// LDS bytes of the profile copies, rounded up to 16 so that the 64-bit
// records placed after them stay aligned.
__host__ __device__ inline int32_t profile_region_bytes(int32_t qlen, int copies) {
    return (copies * profile_copy_bytes(profile_stride(qlen)) + 15) & ~15;
}

// Builds the profile with all threads tid = 0 .. nthreads - 1 of the
// workgroup (every thread must call it: it holds a workgroup barrier).  The
// biased substitution rows (row kZeroRow zero) go to `tmp` first, LDS outside
// the profile (at least kProfRows * kNsym bytes), so that each profile dword
// costs one memory round trip for its four query letters and four LDS
// lookups, instead of a dependent pair of global loads per byte.
template <int kCopies>
__device__ __forceinline__ void build_profile(uint8_t* prof, int32_t ps, const uint8_t* qcodes,
                                              int32_t qlen, const int8_t* mat, int32_t bias,
                                              uint8_t* tmp, int32_t tid, int32_t nthreads) {
    // row r of tmp: the scores of every query letter against target letter
    // r, i.e. column r of the matrix (it scores a query letter, its row,
    // against a target letter, its column)
    for (int32_t i = tid; i < kProfRows * kNsym; i += nthreads)
        tmp[i] = i < kNsym * kNsym ? (uint8_t)(mat[(i % kNsym) * kNsym + i / kNsym] + bias) : (uint8_t)0;
    __syncthreads();
    const int32_t cpb = profile_copy_bytes(ps);
    uint32_t* p32 = (uint32_t*)prof;
    const int32_t nw = kCopies * cpb / 4;
    for (int32_t w = tid; w < nw; w += nthreads) {
        const int32_t byte0 = w * 4;
        const int32_t s = byte0 / cpb;
        const int32_t rem = byte0 - s * cpb;
        const int32_t r = rem / ps;
        const int32_t c0 = rem - r * ps + s - kPad;     // column of byte 0
        uint32_t code[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int32_t c = c0 + b;
            code[b] = qcodes[(uint32_t)c < (uint32_t)qlen ? c : 0];   // qlen >= 1
        }
        const uint8_t* row = tmp + r * kNsym;              // r <= kZeroRow
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int32_t c = c0 + b;
            const uint32_t e = (uint32_t)c < (uint32_t)qlen ? (uint32_t)row[code[b]] : 0u;
            v |= e << (8 * b);
        }
        p32[w] = v;
    }
}

// Byte-packed accumulators of 8 diagonals: b0 holds bytes 0..3, b1 bytes
// 4..7 of each profile read; h0..h3 hold the widened 16-bit sums as pairs
// (h0 = bytes 0 and 2, h1 = 1 and 3, h2 = 4 and 6, h3 = 5 and 7); w[] holds
// 32-bit totals for windows longer than 4096 letters.
struct Acc8 {
    uint32_t b0, b1, h0, h1, h2, h3;
    uint32_t w[8];
    __device__ __forceinline__ void zero() {
        b0 = b1 = h0 = h1 = h2 = h3 = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) w[i] = 0;
    }
    __device__ __forceinline__ void flush() {
        // odd bytes 1 and 3 moved to 16-bit lanes in one byte permute
        h0 += b0 & 0x00FF00FFu;
        h1 += __builtin_amdgcn_perm(0u, b0, 0x0c030c01u);
        h2 += b1 & 0x00FF00FFu;
        h3 += __builtin_amdgcn_perm(0u, b1, 0x0c030c01u);
        b0 = b1 = 0;
    }
    // 16-bit lanes stay below 65536 for 4096 letters (4096 * 15)
    __device__ __forceinline__ void widen() {
        w[0] += h0 & 0xFFFFu; w[2] += h0 >> 16;
        w[1] += h1 & 0xFFFFu; w[3] += h1 >> 16;
        w[4] += h2 & 0xFFFFu; w[6] += h2 >> 16;
        w[5] += h3 & 0xFFFFu; w[7] += h3 >> 16;
        h0 = h1 = h2 = h3 = 0;
    }
};

// Per-block read bases: iteration i (0-based from a column e = c + kPad) reads
// copy (e + i) & 3 at offset e + i - ((e + i) & 3); with i = 4m + v that is
// base[v] + 4m, base[v] = ((e+v)&3) * cpb + e + v - ((e+v)&3).  With one copy
// base[v] = e + v.
template <int kCopies>
struct Bases {
    int32_t v0, v1, v2, v3;
    __device__ __forceinline__ void set(int32_t e, int32_t cpb) {
        if (kCopies == 4) {
            // s * cpb + e + v - s = s * (cpb - 1) + e + v; copy indices and
            // strides fit 24 bits, so the full-rate 24-bit multiply is exact
            const uint32_t cm = (uint32_t)cpb - 1u;
            v0 = (int32_t)__umul24((uint32_t)e & 3u, cm) + e;
            v1 = (int32_t)__umul24((uint32_t)(e + 1) & 3u, cm) + e + 1;
            v2 = (int32_t)__umul24((uint32_t)(e + 2) & 3u, cm) + e + 2;
            v3 = (int32_t)__umul24((uint32_t)(e + 3) & 3u, cm) + e + 3;
        } else {
            v0 = e; v1 = e + 1; v2 = e + 2; v3 = e + 3;
        }
    }
    __device__ __forceinline__ void advance(int32_t d) { v0 += d; v1 += d; v2 += d; v3 += d; }
};

// Eight profile bytes at byte address addr.  Four copies: the address is
// dword aligned.  One copy: three aligned dwords, funnel-shifted by the low
// two address bits (unaligned 8-byte LDS reads are several times slower).
template <int kCopies>
__device__ __forceinline__ uint2 lds8(const uint8_t* prof, int32_t addr) {
    if (kCopies == 4) {
        const uint32_t* p = (const uint32_t*)(prof + addr);
        return make_uint2(p[0], p[1]);
    }
    const uint32_t* p = (const uint32_t*)(prof + (addr & ~3));
    const uint32_t d0 = p[0], d1 = p[1], d2 = p[2];
    return make_uint2(__builtin_amdgcn_alignbyte(d1, d0, (uint32_t)addr),
                      __builtin_amdgcn_alignbyte(d2, d1, (uint32_t)addr));
}

__device__ __forceinline__ uint32_t load4(const uint8_t* p) {
    uint32_t w;
    __builtin_memcpy(&w, p, 4);
    return w;
}
__device__ __forceinline__ uint4 load16(const uint8_t* p) {
    uint4 w;
    __builtin_memcpy(&w, p, 16);
    return w;
}

__device__ __forceinline__ uint32_t letter_of(uint32_t w, int v) { return (w >> (8 * v)) & 0xFFu; }

// One letter: the profile row of `r` at 8 columns, optionally masked.
template <int kCopies, uint32_t kMaskLo = 0xFFFFFFFFu, uint32_t kMaskHi = 0xFFFFFFFFu>
__device__ __forceinline__ void step_letter(const uint8_t* prof, int32_t ps, int32_t base,
                                            uint32_t r, Acc8& a) {
    // rows < 25 and strides < 2^15: a 24-bit multiply-add forms the address
    const uint2 x = lds8<kCopies>(prof, (int32_t)(__umul24(r, (uint32_t)ps) + (uint32_t)base));
    if (kMaskLo) a.b0 += x.x & kMaskLo;
    if (kMaskHi) a.b1 += x.y & kMaskHi;
}

// Profile row r of one letter of the unmasked run: `o` is the aligned
// offset of this letter position's read in row 0, plus `m` bytes (one copy:
// the low bits of `sh` give the byte offset within the aligned read).
template <int kCopies>
__device__ __forceinline__ uint2 row8(const uint8_t* prof, uint32_t o, int32_t m, int32_t ps,
                                      uint32_t sh, uint32_t r) {
    const uint32_t* p = (const uint32_t*)(prof + __umul24(r, (uint32_t)ps) + o) + (m >> 2);
    if (kCopies == 4) return make_uint2(p[0], p[1]);
    const uint32_t d0 = p[0], d1 = p[1], d2 = p[2];
    return make_uint2(__builtin_amdgcn_alignbyte(d1, d0, sh), __builtin_amdgcn_alignbyte(d2, d1, sh));
}

__device__ __forceinline__ uint32_t pick4(const uint4& w, int32_t i) {
    return i == 0 ? w.x : i == 1 ? w.y : i == 2 ? w.z : w.w;
}

// Letters as the block scorers read them, 16 per "chunk" (a uint4), letter
// j of a chunk being at<j>.  kBits = 8: the byte image, a chunk is the 16
// bytes from letter p on.  kBits = 5: the 5-bit image (letter p at bits
// 5p .. 5p + 4 of a dense little-endian stream); a chunk is the 80 bits from
// letter p on, funnel-shifted so that letter j sits at bits 5j of (x, y, z).
template <int kBits>
struct Letters;

template <>
struct Letters<8> {
    static __device__ __forceinline__ uint4 load(const uint8_t* img, int64_t p) {
        return load16(img + p);
    }
    template <int j>
    static __device__ __forceinline__ uint32_t at(const uint4& w) {
        return letter_of(pick4(w, j >> 2), j & 3);
    }
    // letter 4g + v, g known at run time only
    template <int v>
    static __device__ __forceinline__ uint32_t at_rt(const uint4& w, int32_t g) {
        return letter_of(pick4(w, g), v);
    }
};

template <>
struct Letters<5> {
    static __device__ __forceinline__ uint4 load(const uint8_t* img, int64_t p) {
        const uint64_t b = (uint64_t)p * 5u;
        uint4 w;
        __builtin_memcpy(&w, img + ((b >> 5) << 2), 16);   // dword aligned
        const uint32_t s = (uint32_t)b & 31u;
        return make_uint4(__builtin_amdgcn_alignbit(w.y, w.x, s), __builtin_amdgcn_alignbit(w.z, w.y, s),
                          __builtin_amdgcn_alignbit(w.w, w.z, s), 0u);
    }
    template <int j>
    static __device__ __forceinline__ uint32_t at(const uint4& w) {
        constexpr int b = 5 * j, d = b >> 5, o = b & 31;
        if (o <= 27) return (pick4(w, d) >> o) & 31u;
        return __builtin_amdgcn_alignbit(pick4(w, d + 1), pick4(w, d), (uint32_t)o) & 31u;
    }
    template <int v>
    static __device__ __forceinline__ uint32_t at_rt(const uint4& w, int32_t g) {
        const uint32_t b = 5u * (4u * (uint32_t)g + (uint32_t)v);
        const int32_t d = (int32_t)(b >> 5);
        return __builtin_amdgcn_alignbit(pick4(w, d + 1), pick4(w, d), b & 31u) & 31u;
    }
};

// Unmasked run of `count` letters starting at T with read bases B.  Letters
// come 16 at a time, fetched one chunk ahead; `first` holds letters 0..15 and
// `tail` the 16 letters from count & ~15 on, both fetched by the caller.
// kIlp issues the sixteen profile reads of a chunk before summing them: more
// reads in flight for more registers (three wavefronts per SIMD instead of
// four), which pays for long blocks only.
template <int kCopies, bool kIlp = false, int kBits = 8>
__device__ __forceinline__ void run_letters(const uint8_t* prof, int32_t ps, const uint8_t* img,
                                            int64_t pos, int32_t count, uint4 first, uint4 tail,
                                            Bases<kCopies>& B, Acc8& a, int32_t& since_widen) {
    using LT = Letters<kBits>;
    const int32_t n16 = count >> 4;
    if (kIlp && n16 > 0) {
        // one LDS pointer per letter position mod 4 (aligned down with one
        // copy, the low address bits then select the bytes), so that a
        // letter's address is one multiply-add and the position within the
        // chunk folds into the read's offset
        const uint32_t am = kCopies == 4 ? ~0u : ~3u;
        uint32_t o0 = (uint32_t)B.v0 & am, o1 = (uint32_t)B.v1 & am;
        uint32_t o2 = (uint32_t)B.v2 & am, o3 = (uint32_t)B.v3 & am;
        const uint32_t s0 = (uint32_t)B.v0 & 3u, s1 = (uint32_t)B.v1 & 3u;
        const uint32_t s2 = (uint32_t)B.v2 & 3u, s3 = (uint32_t)B.v3 & 3u;
        uint4 wn = first;
        for (int32_t q = 0; q < n16; ++q) {
            const uint4 w = wn;
            pos += 16;
            wn = LT::load(img, pos);   // the letter image is padded, so this stays in range
            // the four letters of a group: reads first, then the sums
#define HS_ILP_GROUP(m)                                                                  \
            {                                                                            \
                const uint2 x0 = row8<kCopies>(prof, o0, 4 * m, ps, s0, LT::template at<4 * m>(w));     \
                const uint2 x1 = row8<kCopies>(prof, o1, 4 * m, ps, s1, LT::template at<4 * m + 1>(w)); \
                const uint2 x2 = row8<kCopies>(prof, o2, 4 * m, ps, s2, LT::template at<4 * m + 2>(w)); \
                const uint2 x3 = row8<kCopies>(prof, o3, 4 * m, ps, s3, LT::template at<4 * m + 3>(w)); \
                a.b0 += (x0.x + x1.x) + (x2.x + x3.x);                                   \
                a.b1 += (x0.y + x1.y) + (x2.y + x3.y);                                   \
            }
            HS_ILP_GROUP(0) HS_ILP_GROUP(1) HS_ILP_GROUP(2) HS_ILP_GROUP(3)
#undef HS_ILP_GROUP
            // advance the four offsets after this chunk's reads: as one
            // induction variable they would cost an extra add per letter
            asm volatile(
                "v_add_u32 %0, 16, %0\n\t"
                "v_add_u32 %1, 16, %1\n\t"
                "v_add_u32 %2, 16, %2\n\t"
                "v_add_u32 %3, 16, %3"
                : "+v"(o0), "+v"(o1), "+v"(o2), "+v"(o3));
            a.flush();
            if (++since_widen == 256) {
                a.widen();
                since_widen = 0;
            }
        }
        B.advance(16 * n16);
    } else {
        uint4 wn = first;
        for (int32_t q = 0; q < n16; ++q) {
            const uint4 w = wn;
            pos += 16;
            wn = LT::load(img, pos);     // the letter image is padded, so this stays in range
#define HS_GROUP(m)                                                                          \
            step_letter<kCopies>(prof, ps, B.v0 + 4 * m, LT::template at<4 * m>(w), a);     \
            step_letter<kCopies>(prof, ps, B.v1 + 4 * m, LT::template at<4 * m + 1>(w), a); \
            step_letter<kCopies>(prof, ps, B.v2 + 4 * m, LT::template at<4 * m + 2>(w), a); \
            step_letter<kCopies>(prof, ps, B.v3 + 4 * m, LT::template at<4 * m + 3>(w), a);
            HS_GROUP(0) HS_GROUP(1) HS_GROUP(2)
            HS_GROUP(3)
#undef HS_GROUP
            B.advance(16);
            a.flush();
            if (++since_widen == 256) {
                a.widen();
                since_widen = 0;
            }
        }
    }
    const int32_t n4 = (count >> 2) & 3;
#define HS_TAIL_GROUP(u)                                                       \
    if (u < n4) {                                                              \
        step_letter<kCopies>(prof, ps, B.v0, LT::template at<4 * u>(tail), a);     \
        step_letter<kCopies>(prof, ps, B.v1, LT::template at<4 * u + 1>(tail), a); \
        step_letter<kCopies>(prof, ps, B.v2, LT::template at<4 * u + 2>(tail), a); \
        step_letter<kCopies>(prof, ps, B.v3, LT::template at<4 * u + 3>(tail), a); \
        B.advance(4);                                                          \
    }
    HS_TAIL_GROUP(0) HS_TAIL_GROUP(1) HS_TAIL_GROUP(2)
#undef HS_TAIL_GROUP
    const int32_t rem = count & 3;
    if (rem) {
        step_letter<kCopies>(prof, ps, B.v0, LT::template at_rt<0>(tail, n4), a);
        step_letter<kCopies>(prof, ps, B.v1, rem > 1 ? LT::template at_rt<1>(tail, n4) : (uint32_t)kZeroRow, a);
        step_letter<kCopies>(prof, ps, B.v2, rem > 2 ? LT::template at_rt<2>(tail, n4) : (uint32_t)kZeroRow, a);
        B.advance(4);
    }
    a.flush();
}

// Diagonal sums (biased) of byte position b of the block's reads.
__device__ __forceinline__ void acc_values(const Acc8& a, uint32_t v[8]) {
    v[0] = a.w[0] + (a.h0 & 0xFFFFu);
    v[2] = a.w[2] + (a.h0 >> 16);
    v[1] = a.w[1] + (a.h1 & 0xFFFFu);
    v[3] = a.w[3] + (a.h1 >> 16);
    v[4] = a.w[4] + (a.h2 & 0xFFFFu);
    v[6] = a.w[6] + (a.h2 >> 16);
    v[5] = a.w[5] + (a.h3 & 0xFFFFu);
    v[7] = a.w[7] + (a.h3 >> 16);
}

// Best placement of a block: byte b holds the biased sum of diagonal
// k0 + b (ascending) or k0 + 7 - b; only diagonals below nk are real.  The
// largest sum wins, the smaller diagonal on ties: each real diagonal d gets
// the key (sum + 1) * 8 + 7 - d (padding diagonals 0), so the largest key
// names the winner.  Sums stay below 2^28 (at most 15 per letter, windows
// of at most HS_MAX_SEQ letters), so the keys fit 32 bits.
__device__ __forceinline__ uint64_t block_best_dir(const uint32_t v[8], int32_t k0, int32_t nk,
                                                   int32_t off, bool ascending) {
    const int32_t nreal = nk - k0;          // >= 1
    uint32_t key[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        // diagonal k0 + d: byte d, or byte 7 - d of a large target's reads
        // (indexing by diagonal keeps every constant a compile-time one)
        const uint32_t va = v[d], vd = v[7 - d];
        const uint32_t x = ascending ? va : vd;
        key[d] = d < nreal ? (x << 3) + (uint32_t)(15 - d) : 0u;
    }
    const uint32_t m01 = key[0] > key[1] ? key[0] : key[1];
    const uint32_t m23 = key[2] > key[3] ? key[2] : key[3];
    const uint32_t m45 = key[4] > key[5] ? key[4] : key[5];
    const uint32_t m67 = key[6] > key[7] ? key[6] : key[7];
    const uint32_t ma = m01 > m23 ? m01 : m23;
    const uint32_t mb = m45 > m67 ? m45 : m67;
    const uint32_t m = ma > mb ? ma : mb;
    const int32_t dbest = 7 - (int32_t)(m & 7u);
    return shift_key((int32_t)(m >> 3) - 1 - off, k0 + dbest);
}

// Letters of one block, fetched before it is scored: the run of letters that
// needs no masking starts at `run` and has `count` letters (first 16 and
// last count % 16 of them preloaded); blocks of a large target also preload
// their entry and exit ramps.
struct BlockFetch {
    int64_t run;        // letter position of the run's first letter
    int32_t count;
    uint4 first, tail, ramp_in, ramp_out;
};

// LDS slot record read by the block scorers.
struct SlotInfo {
    int32_t pL, pS;
    int32_t ss_tl;      // ss | (target_large << 31)
    int32_t nk;
    int64_t tbase;      // offset of the target's first letter
    uint64_t key;       // best placement of the current step so far
};

// Issues the letter loads of block k0 of slot `si` from the letter image
// (byte or 5-bit, kBits).
template <int kBits = 8>
__device__ __forceinline__ void fetch_block(const SlotInfo& si, int32_t k0,
                                            const uint8_t* __restrict__ letters, BlockFetch& f) {
    using LT = Letters<kBits>;
    const int32_t ss = si.ss_tl & 0x7FFFFFFF;
    if (si.ss_tl < 0) {
        const int64_t T = si.tbase + si.pL + k0;
        f.run = T + 7;
        f.count = ss - 7;
        // letters 0..15: the entry ramp, or all ss + 7 letters of a short window
        f.ramp_in = LT::load(letters, T);
        if (ss >= 7) {
            f.ramp_out = LT::load(letters, T + ss);
            f.first = LT::load(letters, f.run);
            f.tail = LT::load(letters, f.run + (f.count & ~15));
        }
    } else {
        f.run = si.tbase + si.pS;
        f.count = ss;
        f.first = LT::load(letters, f.run);
        f.tail = LT::load(letters, f.run + (ss & ~15));
    }
}

// Scores one block.  Both orientations share one pass over the unmasked run
// of letters, so that lanes holding blocks of either orientation run the same
// loop; blocks of a large target add their masked entry and exit ramps, and
// short windows of a large target (ss < 7) are summed cell by cell.
template <int kCopies, bool kIlp = false, int kBits = 8>
__device__ __forceinline__ uint64_t score_block(const uint8_t* prof, int32_t ps, int32_t cpb,
                                                int32_t bias, const SlotInfo& si, int32_t k0,
                                                const BlockFetch& f, const uint8_t* letters) {
    using LT = Letters<kBits>;
    const int32_t ss = si.ss_tl & 0x7FFFFFFF;
    const bool tl = si.ss_tl < 0;
    const int32_t off = (int32_t)__umul24((uint32_t)bias, (uint32_t)ss);
    uint32_t v[8];
    if (tl && ss < 7) {
        // short window of a large target: letters 0 .. ss + 6 (prefetched,
        // at most 12) all carry out-of-window cells.  Letter i meets query
        // columns pS + i - 7 + b; byte b is real when 7 - i <= b < ss + 7 - i.
        // Byte sums stay below 256 (at most 6 cells of at most 15 each).
        uint32_t b0 = 0, b1 = 0;
        Bases<kCopies> Bs;
        Bs.set(si.pS - 7 + kPad, cpb);
#define HS_SHORT_LETTER(i)                                                                 \
        {                                                                                  \
            const int32_t n = ss + 7 - i;          /* bytes below this one are real */     \
            if (n > 0) {                                                                   \
                const int32_t base = (i & 3) == 0 ? Bs.v0 : (i & 3) == 1 ? Bs.v1 : (i & 3) == 2 ? Bs.v2 : Bs.v3; \
                const uint32_t r = LT::template at<i>(f.ramp_in);                          \
                const uint2 x = lds8<kCopies>(prof, (int32_t)(__umul24(r, (uint32_t)ps) + (uint32_t)base) + 4 * (i >> 2)); \
                const uint64_t lo = i < 7 ? (~0ull << (8 * ((7 - i) & 7))) : ~0ull;        \
                const uint64_t hi = n >= 8 ? ~0ull : ((1ull << (8 * n)) - 1ull);           \
                const uint64_t m = lo & hi;                                                \
                b0 += x.x & (uint32_t)m;                                                   \
                b1 += x.y & (uint32_t)(m >> 32);                                           \
            }                                                                              \
        }
        HS_SHORT_LETTER(0) HS_SHORT_LETTER(1) HS_SHORT_LETTER(2) HS_SHORT_LETTER(3)
        HS_SHORT_LETTER(4) HS_SHORT_LETTER(5) HS_SHORT_LETTER(6) HS_SHORT_LETTER(7)
        HS_SHORT_LETTER(8) HS_SHORT_LETTER(9) HS_SHORT_LETTER(10) HS_SHORT_LETTER(11)
        HS_SHORT_LETTER(12)
#undef HS_SHORT_LETTER
        // byte b of the reads is diagonal k0 + 7 - b
        v[0] = b0 & 0xFFu; v[1] = (b0 >> 8) & 0xFFu; v[2] = (b0 >> 16) & 0xFFu; v[3] = b0 >> 24;
        v[4] = b1 & 0xFFu; v[5] = (b1 >> 8) & 0xFFu; v[6] = (b1 >> 16) & 0xFFu; v[7] = b1 >> 24;
        return block_best_dir(v, k0, si.nk, off, false);
    }
    Acc8 a;
    a.zero();
    Bases<kCopies> B;
    // large target: letter i of the block meets query columns pS + i - 7 + b
    const int32_t e = si.pS - 7 + kPad;
    if (tl) {
        // entry ramp: letters 0..6, letter i keeps bytes >= 7 - i
        B.set(e, cpb);
        const uint4& w = f.ramp_in;
        step_letter<kCopies, 0u, 0xFF000000u>(prof, ps, B.v0, LT::template at<0>(w), a);
        step_letter<kCopies, 0u, 0xFFFF0000u>(prof, ps, B.v1, LT::template at<1>(w), a);
        step_letter<kCopies, 0u, 0xFFFFFF00u>(prof, ps, B.v2, LT::template at<2>(w), a);
        step_letter<kCopies, 0u, 0xFFFFFFFFu>(prof, ps, B.v3, LT::template at<3>(w), a);
        step_letter<kCopies, 0xFF000000u, 0xFFFFFFFFu>(prof, ps, B.v0 + 4, LT::template at<4>(w), a);
        step_letter<kCopies, 0xFFFF0000u, 0xFFFFFFFFu>(prof, ps, B.v1 + 4, LT::template at<5>(w), a);
        step_letter<kCopies, 0xFFFFFF00u, 0xFFFFFFFFu>(prof, ps, B.v2 + 4, LT::template at<6>(w), a);
        a.flush();
    }
    // the unmasked run: letters 7 .. ss - 1 of a large target (columns from
    // pS), or the ss letters of a small target (columns from pL + k0)
    int32_t sw = 0;
    B.set(tl ? e + 7 : si.pL + k0 + kPad, cpb);
    run_letters<kCopies, kIlp, kBits>(prof, ps, letters, f.run, f.count, f.first, f.tail, B, a, sw);
    if (tl) {
        // exit ramp: letters ss .. ss + 6; letter ss + u keeps bytes < 7 - u
        B.set(e + ss, cpb);
        const uint4& w = f.ramp_out;
        step_letter<kCopies, 0xFFFFFFFFu, 0x00FFFFFFu>(prof, ps, B.v0, LT::template at<0>(w), a);
        step_letter<kCopies, 0xFFFFFFFFu, 0x0000FFFFu>(prof, ps, B.v1, LT::template at<1>(w), a);
        step_letter<kCopies, 0xFFFFFFFFu, 0x000000FFu>(prof, ps, B.v2, LT::template at<2>(w), a);
        step_letter<kCopies, 0xFFFFFFFFu, 0u>(prof, ps, B.v3, LT::template at<3>(w), a);
        step_letter<kCopies, 0x00FFFFFFu, 0u>(prof, ps, B.v0 + 4, LT::template at<4>(w), a);
        step_letter<kCopies, 0x0000FFFFu, 0u>(prof, ps, B.v1 + 4, LT::template at<5>(w), a);
        step_letter<kCopies, 0x000000FFu, 0u>(prof, ps, B.v2 + 4, LT::template at<6>(w), a);
        a.flush();
    }
    acc_values(a, v);
    // byte b is diagonal k0 + b of a small target, k0 + 7 - b of a large one
    return block_best_dir(v, k0, si.nk, off, !tl);
}

// A target as handed out by the queue (stored in hand-out order); 16 bytes,
// read as one vector.
struct PairRec {
    int32_t id, len;
    int64_t offset;
};
static_assert(sizeof(PairRec) == 16, "PairRec is read as one 16-byte vector");

// One pair's progress, held in the registers of the slot's lane.
struct PairState {
    int32_t id;          // target index, -1 when the slot is empty
    int32_t qi;          // hand-out position (indexes the precomputed draws)
    int32_t nl, ns;
    bool tl;             // target is the large sequence
    int32_t round, t;
    uint32_t LF, SF;
    int32_t pL, pS, score, best, best_round;
    int32_t ss, blk, nblk;
    bool stepping;
    int64_t tbase;
    uint32_t dw_i, pf_i;  // indices of the cached and the prefetched draw word
    uint64_t dw, pf;      // Philox words of round 0 (four draws each)
};

// random() draw d of the pair's current round: round 0's first 32 draws come
// from the table filled before the search, the rest from Philox directly.
// With kOptTable the table may be absent (NULL: a query whose seed differs
// from the table's), and every draw comes from Philox.
template <bool kOptTable>
__device__ __forceinline__ uint32_t pair_draw(PairState& s, const KParams& kp,
                                              const uint64_t* __restrict__ draws, uint32_t d) {
    if ((!kOptTable || draws != nullptr) && s.round == 0 && d < 32) {
        const uint32_t wi = d >> 2;
        if (wi != s.dw_i) {
            if (wi == s.pf_i) {
                s.dw = s.pf;
            } else {
                s.dw = draws[(int64_t)s.qi * 8 + wi];
            }
            s.dw_i = wi;
        }
        return (uint32_t)(s.dw >> (16 * (d & 3))) & 0xFFFFu;
    }
    uint64_t w[4];
    philox_block(kp.seed, (uint64_t)s.id, (uint32_t)s.round, d >> 4, w);
    const uint32_t wi = (d >> 2) & 3;
    const uint64_t x = wi == 0 ? w[0] : wi == 1 ? w[1] : wi == 2 ? w[2] : w[3];
    return (uint32_t)(x >> (16 * (d & 3))) & 0xFFFFu;
}

template <bool kOptTable>
__device__ __forceinline__ void start_round(PairState& s, const KParams& kp,
                                            const uint64_t* __restrict__ draws) {
    s.LF = round_factor(kp.lfactor, kp.minfactor, pair_draw<kOptTable>(s, kp, draws, 0));
    s.SF = round_factor(kp.sfactor, kp.minfactor, pair_draw<kOptTable>(s, kp, draws, 1));
    s.pL = s.pS = s.t = s.score = 0;
}

// Advances the pair until it has a step to score (or finishes).  Finished
// pairs write their best round's score.
template <bool kCount, bool kOptTable>
__device__ __forceinline__ void advance_pair(PairState& s, const KParams& kp,
                                             const uint64_t* __restrict__ draws, SlotInfo* slot,
                                             int32_t* scores, int32_t* rounds, uint64_t& cells,
                                             int32_t& best_seen) {
    while (s.id >= 0 && !s.stepping) {
        if (s.pL < s.nl && s.pS < s.ns) {
            const int32_t ls = window_large(s.nl - s.pL, s.LF);
            const int32_t ss =
                window_small(s.ns - s.pS, s.SF, pair_draw<kOptTable>(s, kp, draws, 2u + (uint32_t)s.t), ls);
            const int32_t nk = ls - ss + 1;
            s.ss = ss;
            s.blk = 0;
            s.nblk = (nk + kBlockDiags - 1) / kBlockDiags;
            s.stepping = true;
            // fetch the word of the next step's draw while this step is scored
            const uint32_t wn = (3u + (uint32_t)s.t) >> 2;
            if ((!kOptTable || draws != nullptr) && s.round == 0 && wn < 8 && wn != s.dw_i &&
                wn != s.pf_i) {
                s.pf = draws[(int64_t)s.qi * 8 + wn];
                s.pf_i = wn;
            }
            if (kCount) cells += (uint64_t)nk * (uint64_t)ss;
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
        if (s.score > s.best) {
            s.best = s.score;
            s.best_round = s.round;
        }
        if (++s.round < kp.rounds) {
            start_round<kOptTable>(s, kp, draws);
            continue;
        }
        scores[s.id] = s.best;
        if (rounds) rounds[s.id] = s.best_round;
        best_seen = s.best > best_seen ? s.best : best_seen;
        s.id = -1;
    }
}

// Wavefront-private LDS: slots, issued blocks, bin counters.
struct WaveLds {
    static constexpr int kItems = kItemCap;
    SlotInfo slots[kLanes];
    uint32_t items[kItemCap];
    uint32_t bins[kBins];
};
// Smaller records for batches whose profile leaves little LDS, so that more
// wavefronts share it, in workgroups of up to kBigWaves wavefronts: at most
// 16 pairs in flight and 256 blocks per phase (2 KB), or 64 pairs and 256
// blocks (3.6 KB).
constexpr int kBigWaves = 16;
template <int kSlots>
struct WaveLdsSmall {
    static constexpr int kItems = 256;
    SlotInfo slots[kSlots];
    uint32_t items[kItems];
    uint32_t bins[kBins];
};
using WaveLds16 = WaveLdsSmall<16>;
using WaveLds64 = WaveLdsSmall<kLanes>;
// Record kinds of the batch kernel: 0 WaveLds, 1 WaveLds16, 2 WaveLds64.
template <int kRec>
struct RecOf {
    using type = WaveLds;
};
template <>
struct RecOf<1> {
    using type = WaveLds16;
};
template <>
struct RecOf<2> {
    using type = WaveLds64;
};
__host__ __device__ constexpr int rec_slots(int rec) { return rec == 1 ? 16 : kLanes; }

// Queue positions are taken from the global counter 64 at a time per
// wavefront, so that the counter sees one atomic per 64 pairs.
constexpr uint32_t kGrab = 64;
constexpr int64_t kGrabSize = kGrab;

// Bin of a step: orientation, then ss exactly below 32, in steps of 4 up to
// 95 and of 16 up to 351, so that neighbouring blocks in the sorted order
// have close ss.
__device__ __forceinline__ int32_t ss_bin(bool tl, int32_t ss) {
    int32_t b;
    if (ss < 32) b = ss;
    else if (ss < 96) b = 32 + ((ss - 32) >> 2);
    else b = 48 + ((ss - 96) >> 4);
    return (tl ? 64 : 0) + (b < 63 ? b : 63);
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum across the wavefront (all 64 lanes active), in
// registers: sums within each row of 16 lanes by DPP row shifts of 1, 2, 4
// and 8 (lanes without a source add 0), then lane 15's row total is
// broadcast into rows 1 and 3 and lane 31's into rows 2 and 3.  A shuffle
// through LDS would take six dependent LDS round trips instead.
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Phases B and C of a wavefront: every slot with a step in progress
// (`stepping`, window size ss, orientation tl) issues its remaining blocks
// blk..nblk-1 (as many as fit), counting-sorted by (orientation, ss),
// longest first, so that neighbouring lanes get blocks of equal length;
// every lane then scores blocks, and the best placement of each step is
// folded into its slot's key in LDS.
template <int kCopies, bool kIlp = false, int kBits = 8, class WL = WaveLds>
__device__ __forceinline__ void score_pending(WL& W, int32_t lane, bool stepping, bool tl,
                                              int32_t ss, int32_t& blk, int32_t nblk,
                                              const uint8_t* prof, int32_t ps, int32_t cpb,
                                              int32_t bias, const uint8_t* __restrict__ letters) {
    // ---- phase B: issue blocks, sorted by (orientation, ss) descending ----
    const int32_t want = stepping ? nblk - blk : 0;
    const uint32_t winc = wave_inclusive_scan((uint32_t)want);
    const uint32_t nw = (uint32_t)__builtin_amdgcn_readlane((int)winc, kLanes - 1);  // all wants
    int32_t start;
    if (nw <= (uint32_t)kLanes) {
        // one round of 64 lanes holds every block: their order does not
        // matter, so they go in slot order without the counting sort
        start = (int32_t)(winc - (uint32_t)want);
    } else {
        W.bins[lane] = 0;
        W.bins[lane + kLanes] = 0;
        wave_sync();
        // descending bins: the last, partly filled round of 64 blocks then
        // holds the shortest blocks rather than the longest
        const int32_t bkey = (kBins - 1) - ss_bin(tl, ss);
        uint32_t off = 0;
        if (want > 0) off = atomicAdd(&W.bins[bkey], (uint32_t)want);
        wave_sync();
        {
            // exclusive scan over the 128 bins: lane l owns bins 2l, 2l + 1
            const uint32_t a0 = W.bins[2 * lane], a1 = W.bins[2 * lane + 1];
            const uint32_t inc = wave_inclusive_scan(a0 + a1);
            const uint32_t before = inc - (a0 + a1);
            wave_sync();
            W.bins[2 * lane] = before;
            W.bins[2 * lane + 1] = before + a0;
        }
        wave_sync();
        start = (int32_t)(W.bins[bkey] + off);
    }
    if (want > 0) {
        int32_t issue = WL::kItems - start;
        issue = issue < 0 ? 0 : (issue > want ? want : issue);
        for (int32_t b = 0; b < issue; ++b)
            W.items[start + b] = ((uint32_t)lane << 24) | (uint32_t)(blk + b);
        blk += issue;
    }
    // blocks issued = number of slots' wants, capped
    const int32_t n_items = (int32_t)(nw < (uint32_t)WL::kItems ? nw : (uint32_t)WL::kItems);
    wave_sync();

    // ---- phase C: score the blocks; each lane fetches the letters of its
    // next block before scoring the current one ----
    {
        int32_t i = lane;
        bool have = i < n_items;
        SlotInfo si;
        int32_t sl = 0, k0 = 0;
        BlockFetch f;
        if (have) {
            const uint32_t it = W.items[i];
            sl = (int32_t)(it >> 24);
            k0 = (int32_t)(it & 0xFFFFFFu) * kBlockDiags;
            si = W.slots[sl];
            fetch_block<kBits>(si, k0, letters, f);
        }
        while (have) {
            const int32_t in = i + kLanes;
            const bool have_n = in < n_items;
            SlotInfo si_n;
            int32_t sl_n = 0, k0_n = 0;
            BlockFetch f_n;
            if (have_n) {
                const uint32_t it = W.items[in];
                sl_n = (int32_t)(it >> 24);
                k0_n = (int32_t)(it & 0xFFFFFFu) * kBlockDiags;
                si_n = W.slots[sl_n];
                fetch_block<kBits>(si_n, k0_n, letters, f_n);
            }
            const uint64_t key = score_block<kCopies, kIlp, kBits>(prof, ps, cpb, bias, si, k0, f, letters);
            atomicMax((unsigned long long*)&W.slots[sl].key, (unsigned long long)key);
            si = si_n;
            sl = sl_n;
            k0 = k0_n;
            f = f_n;
            i = in;
            have = have_n;
        }
    }
    wave_sync();
}

// Hand-out position of length rank r (longest first): positions hold rank
// i * nb + b at kGrab * b + i (nb batches of kGrab positions).
__device__ __forceinline__ uint32_t rank_position(uint32_t r, uint32_t nb) {
    return (r % nb) * kGrab + r / nb;
}

// One wavefront's share of the pairs of one query: hand-out positions below
// `hi`, taken from the counter `ctr` (global, or a workgroup counter in LDS)
// at least `grab` at a time -- a large grab keeps atomics on a global
// counter rare, grab 0 takes exactly what the wavefront needs -- with at
// most `cap` pairs in flight (lanes 0..cap-1 hold them).
// With stride > 0 (the one-query kernel on a database of many short
// targets) the pairs go by length rank instead: wavefront gw of `stride`
// takes ranks gw, gw + stride, ... below r0 (the longest ones, the same mix
// of lengths for every wavefront, with no atomics), then ranks from r0 on
// from the counter, `grab` at a time, so that the wavefronts that run
// faster take more of the short tail and all finish together.
// Returns when no pair is left; scores go to scores[target], the best round
// to rounds[target].  kExact allows a missing draw table (see pair_draw).
template <int kCopies, bool kCount, bool kExact, bool kIlp, int kBits = 8, class WL = WaveLds>
__device__ __forceinline__ void wave_pairs(WL& W, int32_t lane, int32_t cap, uint32_t grab,
                                           uint32_t stride, uint32_t r0, uint32_t gw,
                                           const uint8_t* prof, int32_t ps, int32_t cpb,
                                           int32_t bias, int32_t qlen, const KParams& kp,
                                           const PairRec* __restrict__ recs, uint32_t hi,
                                           const uint8_t* __restrict__ letters,
                                           const uint64_t* __restrict__ draws, uint32_t* ctr,
                                           int32_t* __restrict__ scores,
                                           int32_t* __restrict__ rounds, uint64_t& cells,
                                           int32_t& best_seen) {
    PairState s;
    s.id = -1;
    s.stepping = false;
    bool exhausted = false;
    uint32_t q_next = 0, q_end = 0;   // held range of the counter (wavefront-uniform)
    uint32_t k_next = 0;              // ranks of the stripe handed out (stride > 0)
    const uint32_t nb = hi / kGrab;

    for (;;) {
        // ---- phase A: apply last step's winner, advance, refill ----
        if (s.id >= 0 && s.stepping && s.blk >= s.nblk) {
            const uint64_t key = W.slots[lane].key;
            const int32_t kb = key_shift(key);
            s.score += key_score(key) - shift_penalty(kp, s.t, kb);
            s.pL += kb + s.ss;
            s.pS += s.ss;
            ++s.t;
            s.stepping = false;
        }
        advance_pair<kCount, kExact>(s, kp, draws, &W.slots[lane], scores, rounds, cells, best_seen);
        // Refill empty slots.  A position may hold padding (id -1): its lane
        // stays empty and asks again; the refill repeats while no lane holds
        // a pair, so the wavefront leaves only once every lane that may take
        // pairs has seen the end of the range.
        for (;;) {
            const bool need = s.id < 0 && !exhausted && lane < cap;
            const uint64_t mask = __ballot(need);
            if (!mask) break;
            const uint32_t cnt = (uint32_t)__popcll(mask);
            const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lane) - 1));
            uint32_t qi = hi;
            // the first n_static lanes take the next ranks of the stripe
            uint32_t n_static = 0;
            if (stride) {
                const uint32_t k0 = r0 / stride;
                n_static = k_next < k0 ? (cnt < k0 - k_next ? cnt : k0 - k_next) : 0u;
                if (rank < n_static) qi = rank_position(gw + (k_next + rank) * stride, nb);
                k_next += n_static;
            }
            const uint32_t cnt_d = cnt - n_static;
            if (cnt_d) {
                // the others: from the range already held, then from one new range
                const uint32_t rank_d = rank - n_static;     // used where rank >= n_static
                const uint32_t take1 = cnt_d < q_end - q_next ? cnt_d : q_end - q_next;
                uint32_t d = q_next + rank_d;
                q_next += take1;
                if (take1 < cnt_d) {
                    const uint32_t g = cnt_d - take1 > grab ? cnt_d - take1 : grab;
                    uint32_t base = 0;
                    if (lane == 0) base = atomicAdd(ctr, g);
                    base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
                    if (rank_d >= take1) d = base + (rank_d - take1);
                    q_next = base + (cnt_d - take1);
                    q_end = base + g;
                }
                if (rank >= n_static) {
                    if (!stride) {
                        qi = d;
                    } else {
                        const uint32_t r = r0 + d;      // past the last rank: exhausted
                        qi = r >= r0 && r < hi ? rank_position(r, nb) : hi;
                    }
                }
            }
            if (need && qi < hi) {
                // Every field of the record and the first draw word are
                // consumed before the id is tested, so that all of them load
                // in one memory round trip (tested first, the id would be
                // fetched alone and the rest after it).  For a padding
                // position (id -1) they are read and ignored: the slot stays
                // empty.
                const uint4 rv = *(const uint4*)(recs + qi);
                s.dw = (!kExact || draws != nullptr) ? draws[(int64_t)qi * 8] : 0ull;
                const int32_t rid = (int32_t)rv.x, rlen = (int32_t)rv.y;
                s.tl = rlen >= qlen;
                s.nl = s.tl ? rlen : qlen;
                s.ns = s.tl ? qlen : rlen;
                s.tbase = (int64_t)(((uint64_t)rv.w << 32) | rv.z);
                if (rid >= 0) {
                    s.dw_i = 0;
                    s.pf_i = 0xFFFFFFFFu;
                    s.id = rid;
                    s.qi = (int32_t)qi;
                    s.round = 0;
                    s.best = INT32_MIN;
                    s.best_round = 0;
                    s.stepping = false;
                    start_round<kExact>(s, kp, draws);
                    advance_pair<kCount, kExact>(s, kp, draws, &W.slots[lane], scores, rounds,
                                                 cells, best_seen);
                }
            } else if (need) {
                exhausted = true;
            }
            if (__ballot(s.id >= 0) != 0) break;
        }
        if (__ballot(s.id >= 0) == 0) break;

        // ---- phases B and C ----
        score_pending<kCopies, kIlp, kBits>(W, lane, s.id >= 0 && s.stepping, s.tl, s.ss, s.blk, s.nblk,
                                     prof, ps, cpb, bias, letters);
    }
}

__device__ __forceinline__ int32_t wave_max_i32(int32_t x) {
    for (int o = kLanes / 2; o > 0; o >>= 1) {
        const int32_t y = __shfl_xor(x, o, kLanes);
        x = y > x ? y : x;
    }
    return x;
}


// Maximum over the wavefront (all 64 lanes active), in registers: DPP row
// shifts give every row's maximum in its lane 15, row broadcasts carry it
// to lane 63.  Lanes without a source contribute 0.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    uint32_t y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false); x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false); x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false); x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false); x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false); x = x > y ? x : y;
    y = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false); x = x > y ? x : y;
    return (uint32_t)__builtin_amdgcn_readlane((int)x, kLanes - 1);
}

// Largest 64-bit key over the wavefront: the largest high word, then the
// largest low word among the lanes holding it.
__device__ __forceinline__ uint64_t wave_max_key(uint64_t key) {
    const uint32_t h = (uint32_t)(key >> 32), l = (uint32_t)key;
    const uint32_t hm = wave_max_u32(h);
    const uint32_t lm = wave_max_u32(h == hm ? l : 0u);
    return ((uint64_t)hm << 32) | lm;
}

// Sum over aligned groups of P = 1 << lg lanes (lg <= 4, so that a group
// lies within a row of 16 lanes), valid in each group's last lane: DPP row
// shifts by 1, 2, .. P / 2 (adds only), after which lane L holds lanes
// L - P + 1 .. L.  (A subtraction with a DPP operand is avoided: folded into
// a reversed subtract, it returned the negated difference here.)
__device__ __forceinline__ uint32_t group_sum(uint32_t x, int32_t lg) {
    if (lg > 0) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
    if (lg > 1) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
    if (lg > 2) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
    if (lg > 3) x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
    return x;
}

// Best placement of one step, cell-parallel (the step's placements are
// few, or short): P = 1 << lg lanes per placement, lane l summing cells
// [(l % P) * per, ...) of placement d0 + l / P, 64 / P placements per round.
// Cell (k, j) pairs large letter pL + k + j with small letter pS + j; its
// biased score is the profile byte of the target letter's row at the query
// letter's column.  Returns the lane's best key over the rounds (0 in lanes
// that end no group).
__device__ __forceinline__ uint64_t step_best_cells(const uint8_t* prof, int32_t ps, int32_t bias,
                                                    const uint8_t* tletters,
                                                    bool tl, int32_t pL, int32_t pS, int32_t ss,
                                                    int32_t nk, int32_t lane, int32_t lg) {
    const int32_t P = 1 << lg;
    const int32_t per = (ss + P - 1) >> lg;
    const int32_t j0 = (lane & (P - 1)) * per;
    const int32_t j1 = j0 + per < ss ? j0 + per : ss;
    const bool last = (lane & (P - 1)) == P - 1;
    const int32_t off = bias * ss;
    uint64_t best = 0;
    for (int32_t d0 = 0; d0 < nk; d0 += kLanes >> lg) {
        const int32_t k = d0 + (lane >> lg);
        uint32_t sum = 0;
        if (k < nk) {
            // target letter at tpos + j, query column qcol + j (profile copy 0)
            const int32_t tpos = tl ? pL + k : pS;
            const int32_t qcol = (tl ? pS : pL + k) + kPad;
#pragma unroll 4
            for (int32_t j = j0; j < j1; ++j)
                sum += prof[__umul24((uint32_t)tletters[tpos + j], (uint32_t)ps) + (uint32_t)(qcol + j)];
        }
        sum = group_sum(sum, lg);
        if (last && k < nk) {
            const uint64_t key = shift_key((int32_t)sum - off, k);
            best = key > best ? key : best;
        }
    }
    return best;
}

// One step of a pair followed by every lane of a wavefront (all 64 lanes
// active): the wavefront's best placement key over the step's nk
// placements.  Whichever scorer has the shorter serial loop: the step's
// blocks of 8 diagonals side by side on the lanes (the scoring pass's block
// scorer, high-ILP loop: a lone wavefront is bound by latency), or every
// placement's cells spread over up to 16 lanes.
template <int kCopies>
__device__ __forceinline__ uint64_t wave_step_key(int32_t lane, const uint8_t* prof, int32_t ps,
                                                  int32_t cpb, int32_t bias,
                                                  const uint8_t* letters,
                                                  int64_t tbase, bool tl, int32_t pL, int32_t pS,
                                                  int32_t ss, int32_t nk) {
    const int32_t nblk = (nk + kBlockDiags - 1) / kBlockDiags;
    int32_t lg = 0;
    while (lg < 4 && (nk << (lg + 1)) <= kLanes && (1 << (lg + 1)) <= ss) ++lg;
    const int32_t cells_it = ((nk + (kLanes >> lg) - 1) / (kLanes >> lg)) * ((ss + (1 << lg) - 1) >> lg);
    const int32_t block_it = ((nblk + kLanes - 1) / kLanes) * (ss + (tl ? 14 : 0));
    uint64_t best = 0;       // below every placement's key
    if (2 * cells_it <= block_it + 64) {
        best = step_best_cells(prof, ps, bias, letters + tbase, tl, pL, pS, ss, nk, lane, lg);
    } else {
        SlotInfo si;
        si.pL = pL;
        si.pS = pS;
        si.ss_tl = ss | (tl ? (int32_t)0x80000000 : 0);
        si.nk = nk;
        si.tbase = tbase;
        si.key = 0;
        for (int32_t b0 = 0; b0 < nblk; b0 += kLanes) {
            const int32_t k0 = (b0 + lane) * kBlockDiags;
            if (k0 < nk) {
                BlockFetch f;
                fetch_block(si, k0, letters, f);
                const uint64_t key = score_block<kCopies, true>(prof, ps, cpb, bias, si, k0, f, letters);
                best = key > best ? key : best;
            }
        }
    }
    return wave_max_key(best);
}

// Copies a target's tlen letters from memory into the wavefront's LDS
// buffer `stage` (all 64 lanes, reading exactly the target's letters) and
// pads them with the zero-row code up to kLetterPad readable bytes past the
// end, as the database is; returns false, copying nothing, when they do not
// fit in stage_bytes.  The copy is complete when it returns true.  A lone
// wavefront then reads its letters from LDS instead of waiting on memory
// at every step.
__device__ __forceinline__ bool stage_target(int32_t lane, const uint8_t* __restrict__ src,
                                             int32_t tlen, uint8_t* stage, int32_t stage_bytes) {
    const int32_t nbytes = (tlen + kLetterPad + 15) & ~15;
    if (stage == nullptr || nbytes > stage_bytes) return false;
    for (int32_t i = lane * 16; i < nbytes; i += kLanes * 16) {
        uint4 v;
        if (i + 16 <= tlen) {
            v = load16(src + i);
        } else {
            uint32_t w[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int32_t j = i + 4 * q + b;
                    w[q] |= (j < tlen ? (uint32_t)src[j] : (uint32_t)kZeroRow) << (8 * b);
                }
            }
            v = make_uint4(w[0], w[1], w[2], w[3]);
        }
        *(uint4*)(stage + i) = v;
    }
    __builtin_amdgcn_s_waitcnt(0);
    wave_sync();
    return true;
}

// random() draws of one (target, round), computed one Philox block at a
// time and cached.
struct DrawCache {
    int32_t blk;                     // Philox block held in w (-1: none)
    uint64_t w[4];
};
__device__ __forceinline__ uint32_t cached_draw(DrawCache& c, uint64_t seed, int32_t id,
                                                int32_t round, uint32_t d) {
    const int32_t b = (int32_t)(d >> 4);
    if (b != c.blk) {
        philox_block(seed, (uint64_t)id, (uint32_t)round, (uint32_t)b, c.w);
        c.blk = b;
    }
    const uint32_t wi = (d >> 2) & 3;
    const uint64_t x = wi == 0 ? c.w[0] : wi == 1 ? c.w[1] : wi == 2 ? c.w[2] : c.w[3];
    return (uint32_t)(x >> (16 * (d & 3))) & 0xFFFFu;
}

// One pair per wavefront at a time (for searches with no more pairs than
// resident wavefronts, where each pair's chain of steps sets the time):
// hand-out positions below `hi` from the counter `ctr`, every lane following
// the pair, every round's steps by wave_step_key; the best round's score (the
// first best) goes to scores[target], the round to rounds[target].  Same
// arithmetic as wave_pairs, so the same scores.
template <int kCopies, bool kCount>
__device__ __forceinline__ void wave_score_one(int32_t lane, const uint8_t* prof, int32_t ps,
                                               int32_t cpb, int32_t bias, int32_t qlen,
                                               const KParams& kp, const PairRec* __restrict__ recs,
                                               uint32_t hi, const uint8_t* __restrict__ letters,
                                               uint32_t* ctr, int32_t* __restrict__ scores,
                                               int32_t* __restrict__ rounds, uint64_t& cells,
                                               int32_t& best_seen, uint8_t* stage,
                                               int32_t stage_bytes) {
    const bool w = lane == 0;     // the lane that stores (and counts)
    for (;;) {
        uint32_t qi = 0;
        if (w) qi = atomicAdd(ctr, 1u);
        qi = (uint32_t)__builtin_amdgcn_readlane((int)qi, 0);
        if (qi >= hi) return;
        const PairRec r = recs[qi];
        if (r.id < 0) continue;
        const bool tl = r.len >= qlen;
        const int32_t nl = tl ? r.len : qlen, ns = tl ? qlen : r.len;
        // the target's letters from LDS when they fit in the stage
        const bool staged = stage_target(lane, letters + r.offset, r.len, stage, stage_bytes);
        const uint8_t* base = staged ? (const uint8_t*)stage : letters;
        const int64_t tbase = staged ? 0 : r.offset;
        int32_t best = INT32_MIN, best_round = 0;
        for (int32_t round = 0; round < kp.rounds; ++round) {
            DrawCache dc;
            dc.blk = -1;
            const uint32_t LF = round_factor(kp.lfactor, kp.minfactor, cached_draw(dc, kp.seed, r.id, round, 0));
            const uint32_t SF = round_factor(kp.sfactor, kp.minfactor, cached_draw(dc, kp.seed, r.id, round, 1));
            int32_t pL = 0, pS = 0, score = 0;
            for (int32_t t = 0; pL < nl && pS < ns; ++t) {
                const int32_t ls = window_large(nl - pL, LF);
                const int32_t ss = window_small(ns - pS, SF, cached_draw(dc, kp.seed, r.id, round, 2u + (uint32_t)t), ls);
                const int32_t nk = ls - ss + 1;
                if (kCount && w) cells += (uint64_t)nk * (uint64_t)ss;
                const uint64_t key = wave_step_key<kCopies>(lane, prof, ps, cpb, bias, base, tbase,
                                                            tl, pL, pS, ss, nk);
                const int32_t kb = key_shift(key);
                score += key_score(key) - shift_penalty(kp, t, kb);
                pL += kb + ss;
                pS += ss;
            }
            score -= kp.pgp * ((nl - pL) + (ns - pS));
            if (score > best) {
                best = score;
                best_round = round;
            }
        }
        if (w) {
            scores[r.id] = best;
            if (rounds) rounds[r.id] = best_round;
        }
        best_seen = best > best_seen ? best : best_seen;
    }
}

// The default scoring kernels ask for four wavefronts per SIMD (at most 128
// VGPRs): below that occupancy the phases' latency is no longer hidden.  The
// high-ILP variants run where LDS already limits residency, and take the
// registers their reads in flight need.
//
// One query against the whole database: every workgroup holds the query
// profile, every wavefront pulls pairs from the global queue, `grab`
// positions at a time with at most `cap` in flight (small databases spread
// thin over all wavefronts, large ones in grabs of 64).
// kBits: the letter image read by the block scorers, 8 (bytes) or 5 (the
// packed image, a measured alternative).
template <int kCopies, bool kCount, bool kIlp, int kBits = 8>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kIlp ? 1 : 4)))
void k_score_sched(
    const PairRec* __restrict__ recs, int32_t n, const uint8_t* __restrict__ letters,
    const uint8_t* __restrict__ qcodes, int32_t qlen, KParams kp, KMatrix km, int32_t bias,
    int32_t cap, uint32_t grab, uint32_t stride, uint32_t r0,
    const uint64_t* __restrict__ draws, uint32_t* queue, int32_t* __restrict__ scores,
    int32_t* __restrict__ rounds, unsigned long long* cells_total, int32_t* max_score) {
    extern __shared__ __align__(16) uint8_t lds[];
    const int32_t ps = profile_stride(qlen);
    const int32_t cpb = profile_copy_bytes(ps);
    uint8_t* prof = lds;
    build_profile<kCopies>(prof, ps, qcodes, qlen, km.m, bias, lds + profile_region_bytes(qlen, kCopies),
                           threadIdx.x, blockDim.x);
    __syncthreads();   // the only workgroup barrier: wavefronts run independently from here

    const int32_t lane = threadIdx.x & (kLanes - 1);
    WaveLds& W = ((WaveLds*)(lds + profile_region_bytes(qlen, kCopies)))[threadIdx.x / kLanes];
    uint64_t cells = 0;
    int32_t best_seen = INT32_MIN;    // largest pair score written by this lane
    const uint32_t gw = blockIdx.x * (blockDim.x / kLanes) +
                        (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kLanes));
    wave_pairs<kCopies, kCount, false, kIlp, kBits>(W, lane, cap, grab, stride, r0, gw, prof, ps, cpb,
                                                    bias, qlen, kp,
                                             recs, (uint32_t)n, letters, draws, queue, scores,
                                             rounds, cells, best_seen);
    if (kCount) {
        for (int o = kLanes / 2; o > 0; o >>= 1) cells += __shfl_xor(cells, o, kLanes);
        if (lane == 0) atomicAdd(cells_total, (unsigned long long)cells);
    }
    if (max_score) {
        best_seen = wave_max_i32(best_seen);
        if (lane == 0 && best_seen != INT32_MIN) atomicMax(max_score, best_seen);
    }
}

// Many queries against the whole database in one persistent launch.  A
// workgroup takes work items (query, range of hand-out positions) from a
// global counter, longest queries first; for each it builds that query's
// profile, then its wavefronts pull the item's pairs from a counter in LDS,
// at most `cap` in flight per wavefront.  Query q's scores go to
// scores[q * stride + target], its maximum score to max_score[q * ms_stride].
// kRec: the wavefront records (RecOf); kinds 1 and 2 run workgroups of up
// to kBigWaves wavefronts, kind 1 at most 16 pairs in flight per wavefront.
template <int kCopies, bool kCount, bool kIlp, int kRec = 0>
__global__ __launch_bounds__(kRec ? kBigWaves * kLanes : kThreads)
__attribute__((amdgpu_waves_per_eu(kIlp && !kRec ? 1 : 4)))
void k_score_batch(
    const BatchQuery* __restrict__ qs, const KMatrix* __restrict__ mats,
    const uint8_t* __restrict__ qcodes, const BatchItem* __restrict__ items, int32_t n_items,
    uint32_t* item_ctr, int32_t prof_bytes, int32_t cap, const PairRec* __restrict__ recs,
    const uint8_t* __restrict__ letters, const uint64_t* __restrict__ draws,
    int32_t* __restrict__ scores, int32_t* __restrict__ rounds, int64_t stride,
    int32_t* max_score, int32_t ms_stride, unsigned long long* cells_total) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_item, s_ctr;
    const int32_t lane = threadIdx.x & (kLanes - 1);
    using WL = typename RecOf<kRec>::type;
    WL& W = ((WL*)(lds + prof_bytes))[threadIdx.x / kLanes];
    uint64_t cells = 0;
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
        const BatchQuery Q = qs[q];
        const int32_t ps = profile_stride(Q.qlen);
        const int32_t cpb = profile_copy_bytes(ps);
        build_profile<kCopies>(lds, ps, qcodes + Q.qoff, Q.qlen, mats[q].m, Q.bias, lds + prof_bytes,
                               threadIdx.x, blockDim.x);
        __syncthreads();
        int32_t best_seen = INT32_MIN;
        wave_pairs<kCopies, kCount, true, kIlp>(W, lane, cap > rec_slots(kRec) ? rec_slots(kRec) : cap,
                                                0u, 0u, 0u, 0u, lds, ps, cpb, Q.bias, Q.qlen,
                                                Q.kp, recs, item.hi, letters,
                                                Q.table ? draws : nullptr, &s_ctr,
                                                scores + (int64_t)q * stride,
                                                rounds ? rounds + (int64_t)q * stride : nullptr,
                                                cells, best_seen);
        best_seen = wave_max_i32(best_seen);
        if (lane == 0 && best_seen != INT32_MIN) atomicMax(max_score + (int64_t)q * ms_stride, best_seen);
        __syncthreads();   // the profile and the counter are rewritten for the next item
    }
    if (kCount) {
        for (int o = kLanes / 2; o > 0; o >>= 1) cells += __shfl_xor(cells, o, kLanes);
        if (lane == 0) atomicAdd(cells_total, (unsigned long long)cells);
    }
}

// A batch with no more pairs than resident wavefronts: as k_score_batch, but
// each wavefront takes the item's pairs one at a time and all its lanes
// follow the pair (wave_score_one), its record serving as the pair's target
// buffer.  A kernel of its own, so that its registers do not weigh on
// k_score_batch.  Query q's scores go to
// scores[q * stride + target], its maximum score to max_score[q * ms_stride].
template <int kCopies, bool kCount>
__global__ __launch_bounds__(kThreads) void k_score_one(
    const BatchQuery* __restrict__ qs, const KMatrix* __restrict__ mats,
    const uint8_t* __restrict__ qcodes, const BatchItem* __restrict__ items, int32_t n_items,
    uint32_t* item_ctr, int32_t prof_bytes, const PairRec* __restrict__ recs,
    const uint8_t* __restrict__ letters, const uint64_t* __restrict__ draws,
    int32_t* __restrict__ scores, int32_t* __restrict__ rounds, int64_t stride,
    int32_t* max_score, int32_t ms_stride, unsigned long long* cells_total) {
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t s_item, s_ctr;
    const int32_t lane = threadIdx.x & (kLanes - 1);
    WaveLds& W = ((WaveLds*)(lds + prof_bytes))[threadIdx.x / kLanes];
    uint64_t cells = 0;
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
        const BatchQuery Q = qs[q];
        const int32_t ps = profile_stride(Q.qlen);
        const int32_t cpb = profile_copy_bytes(ps);
        build_profile<kCopies>(lds, ps, qcodes + Q.qoff, Q.qlen, mats[q].m, Q.bias, lds + prof_bytes,
                               threadIdx.x, blockDim.x);
        __syncthreads();
        int32_t best_seen = INT32_MIN;
        // the wavefront's record is unused here: it stages the targets
        wave_score_one<kCopies, kCount>(lane, lds, ps, cpb, Q.bias, Q.qlen, Q.kp, recs, item.hi,
                                        letters, &s_ctr, scores + (int64_t)q * stride,
                                        rounds ? rounds + (int64_t)q * stride : nullptr, cells,
                                        best_seen, (uint8_t*)&W, (int32_t)sizeof(WaveLds));
        best_seen = wave_max_i32(best_seen);
        if (lane == 0 && best_seen != INT32_MIN) atomicMax(max_score + (int64_t)q * ms_stride, best_seen);
        __syncthreads();   // the profile and the counter are rewritten for the next item
    }
    if (kCount) {
        for (int o = kLanes / 2; o > 0; o >>= 1) cells += __shfl_xor(cells, o, kLanes);
        if (lane == 0) atomicAdd(cells_total, (unsigned long long)cells);
    }
}

// Random draws 0..31 of round 0 for every target in hand-out order (two
// Philox blocks each, one thread per block), and the queue counter reset:
// run before the scoring kernel with 2n threads.  With `reset`, the first
// workgroup also sets up the ranking state of query 0 (a one-query search).
__global__ __launch_bounds__(256) void k_draws(const PairRec* __restrict__ recs, int32_t n,
                                               uint64_t seed, uint64_t* __restrict__ out,
                                               uint32_t* queue, TopkWs tw, int32_t min_score,
                                               int32_t reset) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) *queue = 0;
    if (reset && blockIdx.x == 0) topk_state_init(tw, 0, min_score, threadIdx.x, blockDim.x);
    const int64_t i = t >> 1;
    const uint32_t half = (uint32_t)(t & 1);
    if (i >= n || recs[i].id < 0) return;
    uint64_t w[4];
    philox_block(seed, (uint64_t)recs[i].id, 0, half, w);
    uint64_t* o = out + i * 8 + half * 4;
    o[0] = w[0];
    o[1] = w[1];
    o[2] = w[2];
    o[3] = w[3];
}

}  // namespace hs
