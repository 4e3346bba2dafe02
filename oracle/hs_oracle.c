/*
 * hs_oracle.c -- reference oracle for the search-mode heuristic of
 * Nag & Karforma, "A Space-Efficient Approach towards Distantly Homologous
 * Protein Similarity Searches" (arXiv 1508.06561).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded CPU
 * implementation written to be checked by eye against the paper.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never links or calls it, and it shares no code,
 * header or table with the HIP path.
 *
 * Structure follows Fig. 1 of the paper.  Two slides are implemented: the
 * search mode of Section III.B.3 (contained shifts only; the database search
 * runs it with Rounds = 1) and the pairwise mode of Fig. 1 as written (the
 * small window slides across the large one from end to end, every placement
 * overlapping at least one letter; the paper's alignment tests used
 * Rounds = 20, Section V).
 *   orc_align_pair            -> ALGORITHM AlignSequences
 *   align_round               -> PROCEDURE Align
 *   best_subsequence_alignment-> PROCEDURE getBestSubsequenceAlignment
 *   virtual_alignment_score   -> getVirtualAlignmentScore (Section III.B.2)
 *   score_columns             -> SCORE, with the three gap penalties of
 *                                Section III.B.1
 *
 * Points the paper leaves open are settled as follows (each is one line of
 * the reading register in the design notes):
 *   - LFactor / SFactor scale the per-round random factors:
 *       LF = LFactor * max(MinFactor, u),  SF = SFactor * max(MinFactor, u)
 *     (Section III.B.1 names the factors; Fig. 1 draws lf, sf).
 *   - All fractions are Q16 fixed point (1.0 = 65536); lengths are floored.
 *   - ls = max(1, floor(len(large) * LF)); ss = max(1, floor(len(small) *
 *     SF * u)); in the search mode also ss = min(ss, ls), so that a
 *     contained shift exists.
 *   - A placement uses all ss letters of the small window (Fig. 1 removes
 *     them from small whatever the shift) and, of the large window, its
 *     letters up to the last one facing a small letter; the rest of the large
 *     window goes back to large (Section III.B.2).  Small letters hanging
 *     over either end of the large window face gaps (pairwise mode only).
 *   - random() is a 16-bit fraction taken from Philox4x64-10 (Salmon et al.,
 *     SC'11) keyed by (seed, 0) with counter (target_id, round, d/16, 0);
 *     draw d uses 16-bit chunk d%4 of output word (d/4)%4.  Draw 0 is lf,
 *     draw 1 is sf, draw 2+t is the per-step draw of step t.
 *   - "large" is the longer sequence; on equal length the target is large.
 *   - Ties: the first shift and the first round reaching the best score win
 *     (strict '>' in Fig. 1).
 *   - A gap run of g columns inside the gapped sequence costs GOP+(g-1)*GEP;
 *     every leading or trailing gap column costs PGP.
 *   - A substitution matrix scores a query letter (row) against a target
 *     letter (column), whichever of the two is the large sequence (the paper
 *     uses only the symmetric BLOSUM62, where the order does not matter).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* Alphabet and BLOSUM62 (Henikoff & Henikoff, PNAS 1992), NCBI order.     */
/* ---------------------------------------------------------------------- */
#define ORC_NSYM 24
#define ORC_GAP 0xFF

static const char orc_alphabet[ORC_NSYM + 1] = "ARNDCQEGHILKMFPSTWYVBZX*";

static const int8_t orc_blosum62[ORC_NSYM][ORC_NSYM] = {
    /*        A   R   N   D   C   Q   E   G   H   I   L   K   M   F   P   S   T   W   Y   V   B   Z   X   * */
    /* A */ { 4, -1, -2, -2,  0, -1, -1,  0, -2, -1, -1, -1, -1, -2, -1,  1,  0, -3, -2,  0, -2, -1,  0, -4},
    /* R */ {-1,  5,  0, -2, -3,  1,  0, -2,  0, -3, -2,  2, -1, -3, -2, -1, -1, -3, -2, -3, -1,  0, -1, -4},
    /* N */ {-2,  0,  6,  1, -3,  0,  0,  0,  1, -3, -3,  0, -2, -3, -2,  1,  0, -4, -2, -3,  3,  0, -1, -4},
    /* D */ {-2, -2,  1,  6, -3,  0,  2, -1, -1, -3, -4, -1, -3, -3, -1,  0, -1, -4, -3, -3,  4,  1, -1, -4},
    /* C */ { 0, -3, -3, -3,  9, -3, -4, -3, -3, -1, -1, -3, -1, -2, -3, -1, -1, -2, -2, -1, -3, -3, -2, -4},
    /* Q */ {-1,  1,  0,  0, -3,  5,  2, -2,  0, -3, -2,  1,  0, -3, -1,  0, -1, -2, -1, -2,  0,  3, -1, -4},
    /* E */ {-1,  0,  0,  2, -4,  2,  5, -2,  0, -3, -3,  1, -2, -3, -1,  0, -1, -3, -2, -2,  1,  4, -1, -4},
    /* G */ { 0, -2,  0, -1, -3, -2, -2,  6, -2, -4, -4, -2, -3, -3, -2,  0, -2, -2, -3, -3, -1, -2, -1, -4},
    /* H */ {-2,  0,  1, -1, -3,  0,  0, -2,  8, -3, -3, -1, -2, -1, -2, -1, -2, -2,  2, -3,  0,  0, -1, -4},
    /* I */ {-1, -3, -3, -3, -1, -3, -3, -4, -3,  4,  2, -3,  1,  0, -3, -2, -1, -3, -1,  3, -3, -3, -1, -4},
    /* L */ {-1, -2, -3, -4, -1, -2, -3, -4, -3,  2,  4, -2,  2,  0, -3, -2, -1, -2, -1,  1, -4, -3, -1, -4},
    /* K */ {-1,  2,  0, -1, -3,  1,  1, -2, -1, -3, -2,  5, -1, -3, -1,  0, -1, -3, -2, -2,  0,  1, -1, -4},
    /* M */ {-1, -1, -2, -3, -1,  0, -2, -3, -2,  1,  2, -1,  5,  0, -2, -1, -1, -1, -1,  1, -3, -1, -1, -4},
    /* F */ {-2, -3, -3, -3, -2, -3, -3, -3, -1,  0,  0, -3,  0,  6, -4, -2, -2,  1,  3, -1, -3, -3, -1, -4},
    /* P */ {-1, -2, -2, -1, -3, -1, -1, -2, -2, -3, -3, -1, -2, -4,  7, -1, -1, -4, -3, -2, -2, -1, -2, -4},
    /* S */ { 1, -1,  1,  0, -1,  0,  0,  0, -1, -2, -2,  0, -1, -2, -1,  4,  1, -3, -2, -2,  0,  0,  0, -4},
    /* T */ { 0, -1,  0, -1, -1, -1, -1, -2, -2, -1, -1, -1, -1, -2, -1,  1,  5, -2, -2,  0, -1, -1,  0, -4},
    /* W */ {-3, -3, -4, -4, -2, -2, -3, -2, -2, -3, -2, -3, -1,  1, -4, -3, -2, 11,  2, -3, -4, -3, -2, -4},
    /* Y */ {-2, -2, -2, -3, -2, -1, -2, -3,  2, -1, -1, -2, -1,  3, -3, -2, -2,  2,  7, -1, -3, -2, -1, -4},
    /* V */ { 0, -3, -3, -3, -1, -2, -2, -3, -3,  3,  1, -2,  1, -1, -2, -2,  0, -3, -1,  4, -3, -2, -1, -4},
    /* B */ {-2, -1,  3,  4, -3,  0,  1, -1,  0, -3, -4,  0, -3, -3, -2,  0, -1, -4, -3, -3,  4,  1, -1, -4},
    /* Z */ {-1,  0,  0,  1, -3,  3,  4, -2,  0, -3, -3,  1, -1, -3, -1,  0, -1, -3, -2, -2,  1,  4, -1, -4},
    /* X */ { 0, -1, -1, -1, -2, -1, -1, -1, -1, -1, -1, -1, -1, -1, -2,  0,  0, -2, -1, -1, -1, -1, -1, -4},
    /* * */ {-4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4, -4,  1},
};

/* Robinson & Robinson (PNAS 1991) amino-acid counts, the standard background
 * composition for BLOSUM62 statistics, in the order of the first 20 letters
 * of the alphabet above. */
static const int32_t orc_rr_counts[20] = {
    35155, 23105, 20212, 24161, 8669, 19208, 28354, 33229, 9906, 23161,
    40625, 25872, 10101, 17367, 23435, 32070, 26311, 5990, 14488, 29012};

const char* orc_alphabet_str(void) { return orc_alphabet; }

void orc_blosum62_copy(int8_t* out /* 24*24 */) {
    memcpy(out, orc_blosum62, sizeof(orc_blosum62));
}

void orc_background_counts(int32_t* out /* 20 */) {
    memcpy(out, orc_rr_counts, sizeof(orc_rr_counts));
}

/* Map one ASCII residue to its code.  Letters are case-insensitive; J, O and
 * U (not in BLOSUM62) read as X.  Returns -1 for anything else. */
int orc_code_of(int c) {
    if (c >= 'a' && c <= 'z') c = c - 'a' + 'A';
    if (c == 'J' || c == 'O' || c == 'U') c = 'X';
    for (int i = 0; i < ORC_NSYM; ++i)
        if (orc_alphabet[i] == c) return i;
    return -1;
}

int orc_encode(const char* ascii, int64_t n, uint8_t* codes) {
    for (int64_t i = 0; i < n; ++i) {
        int c = orc_code_of((unsigned char)ascii[i]);
        if (c < 0) return -1;
        codes[i] = (uint8_t)c;
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two    */
/* 64x64->128 multiplies with the round keys bumped by the Weyl constants.  */
/* ---------------------------------------------------------------------- */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL; /* golden ratio */
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1  */

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0;
        uint64_t y1 = lo1;
        uint64_t y2 = hi0 ^ x3 ^ k1;
        uint64_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* random() of Fig. 1: the d-th 16-bit fraction of (target, round). */
uint32_t orc_draw(uint64_t seed, uint64_t target_id, uint32_t round, uint32_t d) {
    uint64_t ctr[4] = {target_id, (uint64_t)round, (uint64_t)(d >> 4), 0};
    uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    orc_philox4x64_10(ctr, key, w);
    uint64_t word = w[(d >> 2) & 3];
    return (uint32_t)((word >> (16 * (d & 3))) & 0xFFFFu);
}

/* ---------------------------------------------------------------------- */
/* Parameters and trace records                                           */
/* ---------------------------------------------------------------------- */
typedef struct {
    int32_t gop, gep, pgp;                          /* Section III.B.1 */
    int32_t lfactor_q16, sfactor_q16, minfactor_q16; /* Q16, in [0, 65536] */
    int32_t rounds;                                 /* >= 1 */
    int32_t full_slide;     /* 0: search mode (Section III.B.3); 1: pairwise
                               mode, every overlapping placement (Fig. 1) */
    uint64_t seed;
} orc_params;

typedef struct {
    int32_t pL, pS;   /* letters of large / small already consumed */
    int32_t ls, ss;   /* window sizes of this step */
    int32_t kstar;    /* chosen shift */
    int32_t dscore;   /* virtual alignment score at kstar */
} orc_step;

typedef struct {
    const int8_t* B;            /* 24 x 24, looked up as [large letter][small letter] */
    const orc_params* p;
    uint64_t target_id;
    int64_t cells;              /* residue pairs scored on diagonals */
} orc_ctx;

/* ---------------------------------------------------------------------- */
/* getVirtualAlignmentScore: ungapped score of small placed at shift k of  */
/* large, summed over the overlapping letters (Section III.B.2).           */
/* ---------------------------------------------------------------------- */
static int64_t virtual_alignment_score(orc_ctx* cx, const uint8_t* large, int32_t nl,
                                       const uint8_t* small, int32_t ns, int32_t k) {
    int64_t s = 0;
    for (int32_t j = 0; j < ns; ++j) {
        int32_t i = k + j;
        if (i < 0 || i >= nl) continue;
        s += cx->B[large[i] * ORC_NSYM + small[j]];
        cx->cells += 1;
    }
    return s;
}

/* getBestSubsequenceAlignment: placement i puts small at shift
 * k = i - length(small) + 1 of large.  Pairwise mode grades every placement
 * with some overlap, i = 0 .. length(small) + length(large) - 2 (Fig. 1);
 * the search mode of Section III.B.3 grades only i = length(small) - 1 ..
 * length(large) - 1, where small lies wholly inside large.  The first
 * placement reaching the best score is kept. */
static void best_subsequence_alignment(orc_ctx* cx, const uint8_t* large, int32_t nl,
                                       const uint8_t* small, int32_t ns,
                                       int32_t* kbest, int64_t* sbest) {
    int32_t start = cx->p->full_slide ? 0 : ns - 1;
    int32_t end = cx->p->full_slide ? ns + nl - 2 : nl - 1;
    int64_t best = INT64_MIN;
    int32_t bk = 0;
    for (int32_t i = start; i <= end; ++i) {
        int32_t k = i - ns + 1;
        int64_t score = virtual_alignment_score(cx, large, nl, small, ns, k);
        if (score > best) { best = score; bk = k; }
    }
    *kbest = bk;
    *sbest = best;
}

/* SCORE of two aligned rows (Section III.B.1).  Columns holding two letters
 * score from the matrix.  In each row, a maximal run of g gap columns costs
 * PGP per column when it lies before that row's first letter or after its
 * last letter, and GOP + (g-1)*GEP otherwise. */
static int64_t score_row_gaps(const uint8_t* row, int32_t n, const orc_params* p) {
    int32_t first = -1, last = -1;
    for (int32_t c = 0; c < n; ++c)
        if (row[c] != ORC_GAP) { if (first < 0) first = c; last = c; }
    int64_t pen = 0;
    int32_t c = 0;
    while (c < n) {
        if (row[c] != ORC_GAP) { ++c; continue; }
        int32_t b = c;
        while (c < n && row[c] == ORC_GAP) ++c;
        int32_t g = c - b;                        /* run [b, c) */
        int periphery = (first < 0) || (c <= first) || (b > last);
        if (periphery) pen += (int64_t)p->pgp * g;
        else pen += (int64_t)p->gop + (int64_t)(g - 1) * p->gep;
    }
    return pen;
}

static int64_t score_columns(const int8_t* B, const uint8_t* aL, const uint8_t* aS, int32_t n,
                             const orc_params* p) {
    int64_t s = 0;
    for (int32_t c = 0; c < n; ++c)
        if (aL[c] != ORC_GAP && aS[c] != ORC_GAP) s += B[aL[c] * ORC_NSYM + aS[c]];
    s -= score_row_gaps(aL, n, p);
    s -= score_row_gaps(aS, n, p);
    return s;
}

/* PROCEDURE Align (Fig. 1): one round with factors LF and SF.  Each step
 * takes a window from the front of each sequence, finds the best placement
 * of the small window on the large one, moves the letters that placement
 * used into the aligned rows and leaves the rest; when one sequence runs out,
 * the other's remaining letters are set against gaps and the rows are scored
 * with SCORE.  aL / aS receive the aligned rows (capacity nl + ns). */
static int64_t align_round(orc_ctx* cx, const uint8_t* large, int32_t nl, const uint8_t* small,
                           int32_t ns, uint32_t round, uint32_t LF, uint32_t SF,
                           uint8_t* aL, uint8_t* aS, int32_t* alen,
                           orc_step* trace, int32_t trace_cap, int32_t* n_steps) {
    const orc_params* p = cx->p;
    int32_t len = 0, t = 0;
    int32_t doneL = 0, doneS = 0;
    while (nl > 0 && ns > 0) {
        /* window sizes: the fraction LF of what is left of large, and the
         * fraction SF times this step's random draw of what is left of
         * small, both floored and at least one letter */
        int64_t ls = (int64_t)(((uint64_t)nl * LF) >> 16);
        if (ls < 1) ls = 1;
        uint32_t u = orc_draw(p->seed, cx->target_id, round, 2u + (uint32_t)t);
        int64_t ss = (int64_t)(((uint64_t)ns * SF * u) >> 32);
        if (ss < 1) ss = 1;
        if (!p->full_slide && ss > ls) ss = ls;   /* search mode: a contained shift exists */

        int32_t kstar;
        int64_t dbest;
        best_subsequence_alignment(cx, large, (int32_t)ls, small, (int32_t)ss, &kstar, &dbest);

        if (trace && t < trace_cap) {
            trace[t].pL = doneL; trace[t].pS = doneS;
            trace[t].ls = (int32_t)ls; trace[t].ss = (int32_t)ss;
            trace[t].kstar = kstar; trace[t].dscore = (int32_t)dbest;
        }
        /* columns of the step, left to right: large letters skipped before a
         * positive shift face gaps; then every small letter of the window,
         * facing the large letter at its place or, hanging over an end of the
         * large window, a gap */
        for (int32_t i = 0; i < kstar; ++i) { aL[len] = large[i]; aS[len] = ORC_GAP; ++len; }
        for (int32_t j = 0; j < (int32_t)ss; ++j) {
            int32_t i = kstar + j;
            aL[len] = (i >= 0 && i < (int32_t)ls) ? large[i] : ORC_GAP;
            aS[len] = small[j];
            ++len;
        }
        /* large gives up its window up to the last letter facing small; small
         * gives up the whole window */
        int32_t takeL = kstar + (int32_t)ss < (int32_t)ls ? kstar + (int32_t)ss : (int32_t)ls;
        large += takeL; nl -= takeL; doneL += takeL;
        small += ss;    ns -= (int32_t)ss; doneS += (int32_t)ss;
        ++t;
    }
    /* whichever sequence is left over faces gaps */
    for (int32_t i = 0; i < nl; ++i) { aL[len] = large[i]; aS[len] = ORC_GAP; ++len; }
    for (int32_t i = 0; i < ns; ++i) { aL[len] = ORC_GAP; aS[len] = small[i]; ++len; }
    *alen = len;
    if (n_steps) *n_steps = t;
    return score_columns(cx->B, aL, aS, len, p);
}

/* ALGORITHM AlignSequences (Fig. 1): Rounds independent runs of Align, each
 * with two fresh random fractions raised to at least MinFactor (and scaled
 * by LFactor and SFactor); the first round with the highest score is kept.
 *
 * Roles: the longer of query and target is "large" (the target on a tie).
 * The aligned rows of the best round are returned oriented as (query row,
 * target row) with code ORC_GAP for gaps. */
int orc_align_pair(const uint8_t* q, int32_t qlen, const uint8_t* tg, int32_t tlen,
                   uint64_t target_id, const orc_params* p, const int8_t* matrix,
                   int32_t* score_out, int32_t* round_out,
                   uint8_t* qrow, uint8_t* trow, int32_t row_cap, int32_t* row_len,
                   orc_step* trace, int32_t trace_cap, int32_t* n_steps,
                   int64_t* cells) {
    if (qlen <= 0 || tlen <= 0 || p->rounds < 1) return -1;
    /* The matrix scores a query letter (row) against a target letter
     * (column).  The rounds look it up as [large letter][small letter], so
     * it is transposed when the target is the large sequence. */
    const int8_t* M = matrix ? matrix : &orc_blosum62[0][0];
    int target_is_large = tlen >= qlen;
    int8_t MT[ORC_NSYM * ORC_NSYM];
    if (target_is_large) {
        for (int a = 0; a < ORC_NSYM; ++a)
            for (int b = 0; b < ORC_NSYM; ++b) MT[b * ORC_NSYM + a] = M[a * ORC_NSYM + b];
        M = MT;
    }
    orc_ctx cx = {M, p, target_id, 0};
    const uint8_t* large = target_is_large ? tg : q;
    const uint8_t* small = target_is_large ? q : tg;
    int32_t nl = target_is_large ? tlen : qlen;
    int32_t ns = target_is_large ? qlen : tlen;

    int32_t cap = nl + ns;
    uint8_t* aL = (uint8_t*)malloc((size_t)cap);
    uint8_t* aS = (uint8_t*)malloc((size_t)cap);
    uint8_t* bL = (uint8_t*)malloc((size_t)cap);
    uint8_t* bS = (uint8_t*)malloc((size_t)cap);
    orc_step* tr = trace ? (orc_step*)malloc(sizeof(orc_step) * (size_t)(ns + 1)) : NULL;
    if (!aL || !aS || !bL || !bS || (trace && !tr)) {
        free(aL); free(aS); free(bL); free(bS); free(tr);
        return -2;
    }

    int64_t best = INT64_MIN;
    int32_t best_round = 0, best_len = 0, best_steps = 0;
    for (int32_t r = 0; r < p->rounds; ++r) {
        uint32_t lf = orc_draw(p->seed, target_id, (uint32_t)r, 0);
        uint32_t sf = orc_draw(p->seed, target_id, (uint32_t)r, 1);
        if (lf < (uint32_t)p->minfactor_q16) lf = (uint32_t)p->minfactor_q16;
        if (sf < (uint32_t)p->minfactor_q16) sf = (uint32_t)p->minfactor_q16;
        uint32_t LF = (uint32_t)(((uint64_t)(uint32_t)p->lfactor_q16 * lf) >> 16);
        uint32_t SF = (uint32_t)(((uint64_t)(uint32_t)p->sfactor_q16 * sf) >> 16);
        int32_t len = 0, steps = 0;
        int64_t s = align_round(&cx, large, nl, small, ns, (uint32_t)r, LF, SF, aL, aS, &len,
                                tr, ns + 1, &steps);
        if (s > best) {
            best = s; best_round = r; best_len = len; best_steps = steps;
            memcpy(bL, aL, (size_t)len);
            memcpy(bS, aS, (size_t)len);
            if (trace) {
                int32_t n = steps < trace_cap ? steps : trace_cap;
                memcpy(trace, tr, sizeof(orc_step) * (size_t)n);
            }
        }
    }
    if (score_out) *score_out = (int32_t)best;
    if (round_out) *round_out = best_round;
    if (n_steps) *n_steps = best_steps;
    if (cells) *cells = cx.cells;
    int rc = 0;
    if (row_len) *row_len = best_len;
    if (qrow && trow) {
        if (best_len > row_cap) rc = -3;
        else {
            memcpy(qrow, target_is_large ? bS : bL, (size_t)best_len);
            memcpy(trow, target_is_large ? bL : bS, (size_t)best_len);
        }
    }
    free(aL); free(aS); free(bL); free(bS); free(tr);
    return rc;
}

/* Database search (Sections I and III.B.3): the query against every target.
 * Writes the pair score and the winning round of each target; ranking is done
 * by the caller with a sort on (score descending, target index ascending). */
int orc_search(const uint8_t* db, const int64_t* offsets, int64_t n_targets,
               const uint8_t* q, int32_t qlen, const orc_params* p, const int8_t* matrix,
               int32_t* scores, int32_t* rounds, int64_t* cells_total) {
    int64_t cells = 0;
    for (int64_t i = 0; i < n_targets; ++i) {
        int64_t c = 0;
        int rc = orc_align_pair(q, qlen, db + offsets[i], (int32_t)(offsets[i + 1] - offsets[i]),
                                (uint64_t)i, p, matrix, &scores[i], rounds ? &rounds[i] : NULL,
                                NULL, NULL, 0, NULL, NULL, 0, NULL, &c);
        if (rc) return rc;
        cells += c;
    }
    if (cells_total) *cells_total = cells;
    return 0;
}

/* Same as orc_search over a subset of target indices (used to time a bounded
 * sample of a large database). */
int orc_search_subset(const uint8_t* db, const int64_t* offsets, const int64_t* ids, int64_t n_ids,
                      const uint8_t* q, int32_t qlen, const orc_params* p, const int8_t* matrix,
                      int32_t* scores, int64_t* cells_total) {
    int64_t cells = 0;
    for (int64_t n = 0; n < n_ids; ++n) {
        int64_t i = ids[n], c = 0;
        int rc = orc_align_pair(q, qlen, db + offsets[i], (int32_t)(offsets[i + 1] - offsets[i]),
                                (uint64_t)i, p, matrix, &scores[n], NULL,
                                NULL, NULL, 0, NULL, NULL, 0, NULL, &c);
        if (rc) return rc;
        cells += c;
    }
    if (cells_total) *cells_total = cells;
    return 0;
}

/* Score of two given aligned rows (codes, ORC_GAP for gaps) under SCORE;
 * the matrix is looked up as [row_a letter][row_b letter] (query row first). */
int64_t orc_score_rows(const uint8_t* row_a, const uint8_t* row_b, int32_t n,
                       const orc_params* p, const int8_t* matrix) {
    return score_columns(matrix ? matrix : &orc_blosum62[0][0], row_a, row_b, n, p);
}
