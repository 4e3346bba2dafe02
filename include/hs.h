/*
 * hs.h -- C ABI of an MI355X (gfx950) library for the constant-auxiliary-space
 * heuristic protein database search of Nag & Karforma, "A Space-Efficient
 * Approach towards Distantly Homologous Protein Similarity Searches"
 * (arXiv 1508.06561).
 *
 * The search compares one query (or a batch) against every database sequence
 * with the search-mode heuristic (Fig. 1, Section III.B.3), ranks the targets
 * by score (ties by lower target index) and returns alignments for the best
 * hits.  All arithmetic is integer, so results are exact and reproducible.
 *
 * Conventions shared by every call:
 *   - Return value: HS_OK (0) or a negative HS_E* code.  On error no output
 *     is written and hs_last_error() describes the failure.
 *   - Residues are ASCII letters of the 24-letter BLOSUM62 alphabet
 *     "ARNDCQEGHILKMFPSTWYVBZX*" (case-insensitive; J, O and U read as X).
 *     Any other byte is HS_EINVAL.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     ordered on that stream; calls taking host output pointers return after
 *     the results are on the host, calls ending in _dev return as soon as the
 *     work is queued.
 *   - A database handle is immutable after hs_db_load; concurrent searches on
 *     one database from different streams are allowed as long as each uses
 *     its own workspace.
 *   - Run-length alignment ops are uint32 values (len << 2 | op) with
 *     op = HS_OP_M (letter over letter), HS_OP_I (query letter over a gap) or
 *     HS_OP_D (target letter over a gap); they cover both whole sequences
 *     from position 0, oriented (query, target).
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HS_OK 0
#define HS_EINVAL (-1)   /* bad argument or residue */
#define HS_ENOMEM (-2)   /* device or host allocation failed, or over a size limit */
#define HS_ENOSPC (-3)   /* caller buffer too small; the needed size is reported */
#define HS_EDEVICE (-4)  /* a HIP runtime error */

#define HS_NSYM 24
#define HS_OP_M 0
#define HS_OP_I 1
#define HS_OP_D 2

#define HS_MAX_K 4096          /* most ranked hits per query */
#define HS_MAX_SEQ 1000000     /* longest target */
#define HS_MAX_QUERY 5600      /* longest query: its score profile lives in LDS */
#define HS_MAX_PENALTY 1000    /* largest GOP, GEP or PGP */

/* Parameters of Section III.B.1.  Factors are Q16 fixed point (65536 = 1.0)
 * and lie in [0, 65536]; penalties lie in [0, HS_MAX_PENALTY].
 *   LF = LFactor * max(MinFactor, u) and SF = SFactor * max(MinFactor, u) per
 *   round; per step ls = max(1, floor(len(large) * LF)) and
 *   ss = min(ls, max(1, floor(len(small) * SF * u))).
 * `rounds` is the Rounds parameter (1 in search mode, Section III.B.3).
 * `min_score` is the reporting threshold of Section IV (hits below it are
 * not reported).  `seed` keys the random stream: draws depend only on
 * (seed, target index, round, draw index), never on batching or order.
 * `matrix` is a host pointer to a 24x24 row-major int8 substitution matrix in
 * alphabet order, or NULL for the built-in BLOSUM62; its largest and smallest
 * entries may differ by at most 15 (BLOSUM62: -4..11). */
typedef struct hs_params {
    int32_t gop;            /* gap opening penalty */
    int32_t gep;            /* gap extension penalty */
    int32_t pgp;            /* periphery (leading / trailing) gap penalty */
    int32_t lfactor_q16;
    int32_t sfactor_q16;
    int32_t minfactor_q16;
    int32_t rounds;
    int32_t min_score;
    uint64_t seed;
    const int8_t* matrix;
} hs_params;

/* One ranked hit.  `round` is the round whose alignment scored best. */
typedef struct hs_hit {
    int64_t target_id;
    int32_t score;
    int32_t round;
} hs_hit;

/* One alignment: ops[ops_off .. ops_off + n_ops) in the caller's ops buffer. */
typedef struct hs_aln {
    int64_t target_id;
    int32_t score;
    int32_t n_ops;
    int64_t ops_off;
} hs_aln;

typedef struct hs_db hs_db;

/* Fills *p with the search setting of Section IV of the paper: PGP 0,
 * GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, Rounds 1 (Section
 * III.B.3); seed 0, no threshold, built-in BLOSUM62. */
void hs_params_default(hs_params* p);

/* Copies the built-in BLOSUM62 (Section III.A; 24x24 int8, alphabet order)
 * into out[576]. */
void hs_builtin_matrix(int8_t* out);

/* Encodes n ASCII residues (host) into alphabet codes 0..23 (host).
 * HS_EINVAL on a byte outside the alphabet. */
int hs_encode(const char* ascii, int64_t n, uint8_t* codes);

/* Loads a database (Section III.B.5: a flat collection of protein
 * sequences).  `residues` (host) holds the targets' letters concatenated;
 * target i is residues[offsets[i] .. offsets[i+1]).  Target i's index in
 * every result is i.  The library copies the letters to the device and
 * encodes them there (one alphabet code per byte, targets back to back, a
 * length-sorted hand-out order alongside); the returned handle owns that
 * device image until hs_db_free.  Every target needs 1..HS_MAX_SEQ letters. */
int hs_db_load(const char* residues, const int64_t* offsets, int64_t n_targets,
               void* stream, hs_db** out);

/* Releases a database and its device memory.  NULL is allowed. */
int hs_db_free(hs_db* db);

/* Size facts about a loaded database (any pointer may be NULL). */
int hs_db_info(const hs_db* db, int64_t* n_targets, int64_t* n_residues,
               int64_t* device_bytes);

/* One query against the whole database: search-mode heuristic alignment of
 * the query with every target (Fig. 1 with Section III.B.3), ranking by
 * (score descending, target index ascending) over the targets scoring at
 * least params->min_score, and alignments for the first n_aln ranks.
 *   query, qlen      host ASCII query, 1..HS_MAX_QUERY letters
 *   k                ranks to return, 1..HS_MAX_K
 *   n_aln            alignments to return, 0..k
 *   hits             host array of k entries; *n_hits receives how many
 *                    were filled (min(k, targets at or above min_score))
 *   alns             host array of n_aln entries; *n_alns receives the count
 *                    (min(n_aln, *n_hits)); alns[i] belongs to hits[i]
 *   ops, ops_cap     host buffer for the alignments' ops; HS_ENOSPC if too
 *                    small, with *ops_used set to the size needed
 * Host-side temporaries and device workspace are allocated per call. */
int hs_search(const hs_db* db, const char* query, int32_t qlen, const hs_params* params,
              int32_t k, int32_t n_aln, void* stream,
              hs_hit* hits, int32_t* n_hits, hs_aln* alns, int32_t* n_alns,
              uint32_t* ops, int64_t ops_cap, int64_t* ops_used);

/* Device-resident form of hs_search for callers that keep everything in
 * device memory (benchmarks, serving loops).  Queues the whole search on
 * `stream` and returns without waiting.
 *   d_qcodes         device query codes (from hs_encode), qlen of them
 *   d_ws, ws_bytes   device workspace of at least hs_workspace_bytes(db, 1,
 *                    qlen, k, n_aln) bytes, owned by the caller; one search
 *                    at a time may use it
 *   d_hits, d_n_hits device outputs: k hits, one int32 count
 *   d_alns, d_ops    device outputs: n_aln alignments; alignment i's ops
 *                    start at d_ops + i * ops_stride, and its ops_off holds
 *                    that offset; ops_stride >= 2 * qlen + 2 always suffices */
size_t hs_workspace_bytes(const hs_db* db, int32_t nq, int32_t max_qlen, int32_t k, int32_t n_aln);
int hs_search_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                  int32_t k, int32_t n_aln, void* stream, void* d_ws, size_t ws_bytes,
                  hs_hit* d_hits, int32_t* d_n_hits, hs_aln* d_alns, uint32_t* d_ops,
                  int64_t ops_stride);

/* Pair scores only: the search-mode heuristic score of the query against
 * every target (Fig. 1 with Section III.B.3), written by target index into
 * d_scores (int32) and the winning round into d_rounds (int32; may be NULL),
 * both device arrays of n_targets entries.  No ranking, no alignments; the
 * caller may threshold or rank the scores itself.  d_ws is a device
 * workspace of at least hs_workspace_bytes(db, 1, qlen, 1, 0) bytes.  If
 * d_cells (one device uint64) is not NULL, the number of residue pairs scored
 * on diagonals -- the sum over all steps of (ls - ss + 1) * ss, the work
 * measure of Section III.B.4 -- is added to it.  Queued on `stream`. */
int hs_score_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                 void* stream, void* d_ws, size_t ws_bytes, int32_t* d_scores, int32_t* d_rounds,
                 uint64_t* d_cells);

/* Thread-local description of the last failing call on this thread. */
const char* hs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
