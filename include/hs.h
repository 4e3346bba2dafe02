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
#define HS_MAX_BATCH 4096      /* most queries in one batch */
#define HS_MAX_SERVER_WORKERS 8 /* most batches a server keeps in flight */

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
 * alphabet order, or NULL for the built-in BLOSUM62; entry [a][b] scores
 * query letter a against target letter b (whichever sequence is the longer);
 * its largest and smallest entries may differ by at most 15 (BLOSUM62:
 * -4..11). */
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
typedef struct hs_batch hs_batch;

/* Fills *p with the search setting of Section IV of the paper: PGP 0,
 * GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, Rounds 1 (Section
 * III.B.3); seed 0, no threshold, built-in BLOSUM62. */
void hs_params_default(hs_params* p);

/* HS_OK if *p is a valid parameter set (ranges above), else HS_EINVAL with
 * the reason in hs_last_error(). */
int hs_params_check(const hs_params* p);

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

/* Letter image that the one-query scoring kernel reads (Section III.B.5's
 * database, stored two ways): bits = 8, the default, one alphabet code per
 * byte; bits = 5, a dense 5-bit image (5/8 of the bytes), built on the device
 * on first request and kept until hs_db_free.  Results are identical either
 * way; only speed and memory traffic differ, so that the two layouts can be
 * measured against each other.  The 5-bit image serves queries whose four
 * profile copies fit in LDS beside a full workgroup (up to about 1,100
 * letters); longer queries, batches, alignments and Smith-Waterman read the
 * byte image.
 * Not thread-safe against searches running on the same database.
 * Errors: HS_EINVAL (bits not 8 or 5), HS_ENOMEM, HS_EDEVICE. */
int hs_db_set_letters(hs_db* db, int32_t bits, void* stream);

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

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): hs_search_dev
 * without the workspace argument.  The workspace is a static device array of
 * HS_NOALLOC_SCRATCH_BYTES that comes with the library's code object; each
 * device holds its own copy from the library's first kernel launch there until
 * the process ends.  The call allocates nothing (no hipMalloc, hipFree or
 * other allocating routine); the caller still passes the query and the
 * outputs, with the meaning, layout and ownership of hs_search_dev.
 *   HS_ENOMEM   the database needs more workspace than the scratch holds:
 *               hs_workspace_bytes(db, 1, qlen, k, n_aln) above
 *               HS_NOALLOC_SCRATCH_BYTES (about 72 bytes per target, so
 *               databases of up to roughly 900,000 targets fit)
 *   HS_EINVAL   as hs_search_dev
 * Every call on one device shares that device's scratch and keeps the last
 * call's contents there (each search resets what it needs): calls that
 * overlap on one device -- queued on different streams, or from different
 * threads, without ordering -- race and give undefined results. */
#define HS_NOALLOC_SCRATCH_BYTES (64u << 20)
int hs_search_dev_noalloc(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen,
                          const hs_params* params, int32_t k, int32_t n_aln, void* stream,
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

/* ---------------------------------------------------------------------------
 * Threshold reporting.  Section IV reports the database sequences whose
 * score reaches a threshold, ranked.  These calls return every target
 * scoring at least params->min_score, in rank order (score descending,
 * target index ascending), with no cap on the count (hs_search keeps at most
 * HS_MAX_K ranks), and alignments for the first n_aln of them.  The ranking
 * is a stable radix sort on the device; scores are those of hs_search.
 * ------------------------------------------------------------------------- */

/* Device workspace bytes of hs_search_threshold_dev for `db` (0 for NULL):
 * the search's workspace plus 16 bytes per target and a histogram. */
size_t hs_threshold_workspace_bytes(const hs_db* db);

/* Device form, queued on `stream`:
 *   d_qcodes, qlen   device query codes (hs_encode), 1..HS_MAX_QUERY
 *   cap              ranks the caller has room for (>= 0)
 *   n_aln            alignments wanted, 0..min(cap, HS_MAX_K)
 *   d_ws, ws_bytes   device workspace of at least hs_threshold_workspace_bytes
 *   d_hits           device array of cap hits: the first min(n, cap) ranks
 *   d_n              one device int64: n, the number of targets at or above
 *                    the threshold (written also when n > cap)
 *   d_alns, d_ops    as hs_search_dev: alignment i (i < min(n_aln, n)) belongs
 *                    to rank i, its ops at d_ops + i * ops_stride
 * Errors: HS_EINVAL (arguments), HS_ENOSPC (workspace too small), HS_EDEVICE. */
int hs_search_threshold_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen,
                            const hs_params* params, int64_t cap, int32_t n_aln, void* stream,
                            void* d_ws, size_t ws_bytes, hs_hit* d_hits, int64_t* d_n,
                            hs_aln* d_alns, uint32_t* d_ops, int64_t ops_stride);

/* Host form (host query in, host results out; returns when they are there):
 *   hits, cap        host array of cap entries; *n_hits receives n.  When
 *                    n > cap the call returns HS_ENOSPC with *n_hits set and
 *                    writes nothing else, so that the caller can retry with
 *                    cap >= *n_hits
 *   n_aln, alns, n_alns, ops, ops_cap, ops_used
 *                    as hs_search, for the first min(n_aln, n) ranks
 * Device memory is allocated per call. */
int hs_search_threshold(const hs_db* db, const char* query, int32_t qlen, const hs_params* params,
                        int64_t cap, int32_t n_aln, void* stream, hs_hit* hits, int64_t* n_hits,
                        hs_aln* alns, int32_t* n_alns, uint32_t* ops, int64_t ops_cap,
                        int64_t* ops_used);

/* ---------------------------------------------------------------------------
 * Pairwise alignment mode.  Fig. 1 as printed: getBestSubsequenceAlignment
 * slides the small window across the large one from one end to the other
 * (start = 0, end = length(small) + length(large) - 2: every placement with
 * at least one overlapping letter, Section III.B.2), and AlignSequences keeps
 * the best of params->rounds rounds (Section III.B.1; the paper's alignment
 * tests used Rounds = 20, Section V).  The database search uses the search
 * mode of Section III.B.3 instead (contained shifts only).
 *
 * A placement at shift k gives up all ss letters of the small window -- those
 * hanging over an end of the large window are set against gaps -- and the
 * large window's letters through the last one facing small, min(k + ss, ls);
 * the rest of the large window goes back to large.  Ties go to the first
 * placement (most negative shift) and the first round.  The score is SCORE
 * of the aligned rows, with the penalties of Section III.B.1.
 * ------------------------------------------------------------------------- */
#define HS_MAX_ALIGN 5600           /* longest sequence of a pairwise alignment */
#define HS_MAX_ALIGN_PAIRS 1000000  /* most pairs in one call */

/* Aligns n pairs (query i = qres[qoff[i] .. qoff[i+1]), target i =
 * tres[toff[i] .. toff[i+1]), host ASCII, each 1..HS_MAX_ALIGN letters).
 * Pair i's random draws are keyed by i in place of a target index.
 *   scores[n]       host: each pair's score
 *   rounds[n]       host: the round that scored best (may be NULL)
 *   ops, ops_cap    host buffer for the run-length ops of every pair, back
 *                   to back, oriented (query, target) as in hs_search;
 *                   HS_ENOSPC when too small (*ops_used = size needed)
 *   ops_off[n + 1]  host: pair i's ops are ops[ops_off[i] .. ops_off[i+1])
 * Returns when the results are on the host; device memory is allocated per
 * call.  Errors: HS_EINVAL (arguments, residues), HS_ENOSPC, HS_ENOMEM,
 * HS_EDEVICE. */
int hs_align_batch(int32_t n, const char* qres, const int64_t* qoff, const char* tres,
                   const int64_t* toff, const hs_params* params, void* stream, int32_t* scores,
                   int32_t* rounds, uint32_t* ops, int64_t ops_cap, int64_t* ops_off,
                   int64_t* ops_used);

/* Device workspace bytes of hs_align_batch_dev for n pairs at `rounds`
 * rounds (about 16 + 4 * rounds bytes per pair); 0 when n or rounds is out
 * of range. */
int64_t hs_align_workspace_bytes(int32_t n, int32_t rounds);

/* Device form of hs_align_batch (the pairwise mode of Fig. 1, best of
 * Rounds; Section III.B.2, Section V): the letters are already in device
 * memory and the results stay there.  Queues the work on `stream` and
 * returns; only the pair table (32 bytes per pair, built from the host
 * offsets) is copied from the host.
 *   d_codes          device letter codes (as hs_encode writes them, 0..23;
 *                    larger values read as 23)
 *   qoff, toff       host offsets into d_codes, n + 1 each: pair i's query is
 *                    d_codes[qoff[i] .. qoff[i+1]), its target
 *                    d_codes[toff[i] .. toff[i+1]), each 1..HS_MAX_ALIGN
 *                    letters; pair i's draws are keyed by i
 *   d_ws, ws_bytes   device workspace of at least
 *                    hs_align_workspace_bytes(n, params->rounds) bytes
 *   d_scores         device int32[n]: each pair's score
 *   d_rounds         device int32[n]: the best round (may be NULL)
 *   d_ops            device uint32 array of sum(qlen + tlen) entries: pair
 *                    i's run-length ops, oriented (query, target), from entry
 *                    (qoff[i] - qoff[0]) + (toff[i] - toff[0]) on, in a slot
 *                    of its qlen + tlen entries
 *   d_n_ops          device int32[n]: each pair's op count
 * Pair i's results equal hs_align_batch's.  Errors: HS_EINVAL (arguments),
 * HS_ENOSPC (workspace too small), HS_EDEVICE. */
int hs_align_batch_dev(int32_t n, const uint8_t* d_codes, const int64_t* qoff, const int64_t* toff,
                       const hs_params* params, void* stream, void* d_ws, size_t ws_bytes,
                       int32_t* d_scores, int32_t* d_rounds, uint32_t* d_ops, int32_t* d_n_ops);

/* One pair: hs_align_batch with n = 1; *n_ops receives the op count (also on
 * HS_ENOSPC). */
int hs_align(const char* query, int32_t qlen, const char* target, int32_t tlen,
             const hs_params* params, void* stream, int32_t* score, int32_t* round, uint32_t* ops,
             int64_t ops_cap, int64_t* n_ops);

/* ---------------------------------------------------------------------------
 * Smith-Waterman baseline.  The exact optimum that the paper measures its
 * heuristic against (Sections I and IV compare the two for speed and
 * sensitivity): Smith & Waterman (1981) local alignment with Gotoh's (1982)
 * affine gaps, a gap run of g columns costing gop + (g - 1) * gep, the
 * convention of Section III.B.1.  Scores only, no alignments.
 * ------------------------------------------------------------------------- */

/* Device workspace bytes hs_sw_scores_dev needs for `db`: 8 bytes per
 * database letter (a boundary row of H and gap values per target letter,
 * written by one pass over 16 query rows and read by the next).  Returns
 * HS_EINVAL for a NULL db. */
int64_t hs_sw_workspace_bytes(const hs_db* db);

/* Optimal local alignment score of one query against every target of `db`,
 * queued on `stream`:
 *   d_qcodes, qlen   device query codes from hs_encode (each < HS_NSYM),
 *                    1..HS_MAX_QUERY of them; the query profile lives in LDS
 *   params           gop, gep and matrix are used (checked as for hs_search);
 *                    the heuristic's factors, rounds and seed are ignored
 *   d_ws, ws_bytes   device workspace, at least hs_sw_workspace_bytes(db);
 *                    contents on entry are ignored, on return unspecified
 *   d_scores         device int32[n_targets] in target index order; 0 when no
 *                    positive-scoring local alignment exists
 * Errors: HS_EINVAL (NULL pointer, qlen out of range, bad params), HS_ENOSPC
 * (workspace too small), HS_EDEVICE (launch failed).  All buffers stay owned
 * by the caller and must stay valid until the stream has run the launch. */
int hs_sw_scores_dev(const hs_db* db, const uint8_t* d_qcodes, int32_t qlen, const hs_params* params,
                     void* stream, void* d_ws, size_t ws_bytes, int32_t* d_scores);

/* ---------------------------------------------------------------------------
 * Batches.  The query-against-database comparison of Section II, done for
 * many queries at once: every (query, target) pair is scored by the same
 * search-mode heuristic (Fig. 1 with Section III.B.3) and every query is
 * ranked and aligned exactly as hs_search would, so the results of a batch
 * are identical, bit for bit, to separate hs_search calls with the same
 * parameters -- whatever the batch size, query order or schedule.  Scoring
 * runs as one persistent launch over (query, range of targets) work items,
 * longest queries first; a workgroup builds one query's score profile in
 * LDS per item.
 *
 * A batch handle (hs_batch) owns one device allocation sized at creation and
 * reuses it for every batch of queries set on it; it borrows the database,
 * which must outlive it.  One handle runs one search at a time.
 * ------------------------------------------------------------------------- */

/* Creates a batch handle for up to max_nq (1..HS_MAX_BATCH) queries of at
 * most max_qlen (1..HS_MAX_QUERY) letters and max_residues letters in all,
 * returning k (1..HS_MAX_K) ranks and n_aln (0..k) alignments per query.
 * Device memory: about max_nq * n_targets * 8 bytes of scores plus
 * max_nq * n_aln * (2 * max_qlen + 2) * 8 bytes of alignment ops. */
int hs_batch_create(const hs_db* db, int32_t max_nq, int32_t max_qlen, int64_t max_residues,
                    int32_t k, int32_t n_aln, hs_batch** out);

/* Releases a batch handle and its device memory.  NULL is allowed. */
int hs_batch_free(hs_batch* b);

/* Sets the queries of the next searches: query q is the host ASCII letters
 * residues[offsets[q] .. offsets[q+1]) and uses params[q] (n_params == nq)
 * or params[0] (n_params == 1).  Encodes and uploads the queries on `stream`
 * and returns when the upload is complete; the host inputs may be reused
 * afterwards.  Also lays out the work items under the current schedule. */
int hs_batch_set(hs_batch* b, int32_t nq, const char* residues, const int64_t* offsets,
                 const hs_params* params, int32_t n_params, void* stream);

/* Fixes the schedule of the scoring launch (results do not depend on it):
 *   copies   score-profile copies in LDS, 1 or 4 (4: aligned reads; needs
 *            more LDS), 0 = 4 whenever it fits
 *   cap      pairs in flight per wavefront, 1..64, 0 = an item's positions
 *            shared by the workgroup's wavefronts (at most 64), and at most
 *            24,576 letters / the database's median target length (at least 1)
 *   chunk    target positions per work item, a multiple of 64, 0 = sized
 *            so that every workgroup gets about four items
 * With cap and chunk both 0, a batch whose pairs each get a resident
 * wavefront is instead scored one pair per wavefront (reported as cap 1,
 * chunk = wavefronts per workgroup).
 * Applies to the current queries at once and to every later hs_batch_set. */
int hs_batch_schedule(hs_batch* b, int32_t copies, int32_t cap, int32_t chunk, void* stream);

/* The schedule in use, the workgroup count and the number of work items
 * (any pointer may be NULL). */
int hs_batch_get_schedule(const hs_batch* b, int32_t* copies, int32_t* cap, int32_t* chunk,
                          int32_t* grid, int32_t* n_items);

/* The scoring launch that the schedule in use selects (Section III.B.4's
 * work, distributed over the device; any pointer may be NULL):
 *   record   per-wavefront LDS record: 0 = 64 pairs in flight and 512
 *            blocks per phase, 1 = 16 pairs and 256 blocks, 2 = 64 pairs
 *            and 256 blocks (1 and 2 in workgroups of up to 16 wavefronts,
 *            chosen when they fit more wavefronts on a compute unit)
 *   waves    wavefronts per workgroup of the scoring launch
 *   ilp      1 when the letter loop issues a chunk's profile reads before
 *            summing them
 *   one_pair 1 when the batch is scored one pair per wavefront (all lanes of
 *            a wavefront on one pair; record is then 0)
 * Valid after hs_batch_set; HS_EINVAL before it. */
int hs_batch_get_launch(const hs_batch* b, int32_t* record, int32_t* waves, int32_t* ilp,
                        int32_t* one_pair);

/* Autotuner: times the scoring pass of the current queries under every
 * candidate schedule (copies x cap in {4, 8, 16, 32, 64} x chunk halvings), `reps`
 * timed passes each on `stream`, keeps the fastest as the fixed schedule and
 * reports its mean time in *best_ms (may be NULL).  Synchronizes `stream`. */
int hs_batch_tune(hs_batch* b, void* stream, int32_t reps, float* best_ms);

/* Queues the whole search of the current queries on `stream` (scoring,
 * ranking, alignments) and returns.  Only kernel launches are queued, so the
 * call may be captured into a graph.  hs_batch_run_graph does the same
 * through a graph captured on its first use after hs_batch_set or
 * hs_batch_schedule and replayed on `stream` afterwards. */
int hs_batch_run(hs_batch* b, void* stream);
int hs_batch_run_graph(hs_batch* b, void* stream);

/* Queues the scoring pass alone (no ranking, no alignments); if d_cells (one
 * device uint64) is not NULL, the residue pairs scored on diagonals are
 * added to it, as in hs_score_dev. */
int hs_batch_score(hs_batch* b, void* stream, uint64_t* d_cells);

/* Results of the last run on the host, after the work queued on `stream`:
 *   hits    nq * k entries, query q's ranks at hits[q * k], n_hits[q] filled
 *   alns    nq * n_aln entries, query q's at alns[q * n_aln], n_alns[q]
 *           filled; ops_off indexes the caller's ops buffer, which receives
 *           every alignment's ops back to back (HS_ENOSPC if ops_cap is too
 *           small, with *ops_used set to the size needed; the results stay
 *           on the device and the call may be repeated)
 * Synchronizes `stream`. */
int hs_batch_results(hs_batch* b, void* stream, hs_hit* hits, int32_t* n_hits, hs_aln* alns,
                     int32_t* n_alns, uint32_t* ops, int64_t ops_cap, int64_t* ops_used);

/* Pair scores of the last run on the host: scores[q * n_targets + i] and,
 * if rounds is not NULL, the winning rounds likewise.  Synchronizes `stream`. */
int hs_batch_scores(hs_batch* b, void* stream, int32_t* scores, int32_t* rounds);

/* Device addresses of the batch's outputs, for callers that keep results on
 * the device: hits [max_nq][k], n_hits [max_nq], alns [max_nq][n_aln] (ops_off
 * indexes d_ops), d_ops with alignment (q, a) at (q * n_aln + a) * ops_stride,
 * scores and rounds [max_nq][n_targets].  Any pointer may be NULL.  Valid until
 * hs_batch_free. */
int hs_batch_outputs(const hs_batch* b, hs_hit** d_hits, int32_t** d_n_hits, hs_aln** d_alns,
                     uint32_t** d_ops, int64_t* ops_stride, int32_t** d_scores,
                     int32_t** d_rounds);

/* One-shot batch search: create, set, run, results, free.  Arguments as in
 * hs_batch_set and hs_batch_results; query lengths 1..HS_MAX_QUERY. */
int hs_search_batch(const hs_db* db, int32_t nq, const char* residues, const int64_t* offsets,
                    const hs_params* params, int32_t n_params, int32_t k, int32_t n_aln,
                    void* stream, hs_hit* hits, int32_t* n_hits, hs_aln* alns, int32_t* n_alns,
                    uint32_t* ops, int64_t ops_cap, int64_t* ops_used);

/* ---------------------------------------------------------------------------
 * Serving.  A server owns a few workers, each a batch handle, a stream and a
 * thread, that run continuous batching: queries are submitted one at a time
 * (from any thread) and queue up; whenever a worker is free it takes the
 * waiting queries, first come first served, while they fit the batch's
 * footprint: device memory -- at most max_batch queries and max_residues
 * letters in all, the capacity of the worker's buffers, each query at most
 * max_qlen letters -- and LDS: a query whose score profile needs the one-copy
 * layout (too long for four copies beside a full workgroup) is not batched
 * with queries that keep four copies, so that it does not slow their launch;
 * it starts the next batch.  The worker searches them as one batch on its
 * stream and publishes each query's results.  With more than one worker, queries that arrive while a batch is
 * on the device start beside it.  Results are identical to a separate
 * hs_search of the same query and parameters.
 * ------------------------------------------------------------------------- */
typedef struct hs_server hs_server;

/* Per-query timing (milliseconds, host steady clock unless noted).  batch_ms
 * is split into set_ms (encoding and upload of the batch's queries), run_ms
 * (queueing its kernels) and results_ms (waiting for the device and copying
 * the results back); gpu_ms is the device time of its kernels (HIP events on
 * the worker's stream). */
typedef struct hs_server_timing {
    double submit_ms;       /* submission time since the server was created */
    double queue_ms;        /* submission to the start of its batch */
    double batch_ms;        /* duration of its batch (upload, search, results) */
    double total_ms;        /* submission to results available */
    double set_ms, run_ms, results_ms;
    double gpu_ms;
    int32_t batch_size;     /* queries in its batch */
    int32_t pad_;
} hs_server_timing;

/* Creates a server with two workers on the current device for searches
 * returning k ranks and n_aln alignments per query (limits as in
 * hs_batch_create, and max_residues >= max_qlen so that every acceptable
 * query can be admitted: HS_EINVAL otherwise).  The database must outlive
 * the server. */
int hs_server_create(const hs_db* db, int32_t max_batch, int32_t max_qlen, int64_t max_residues,
                     int32_t k, int32_t n_aln, hs_server** out);

/* As hs_server_create with n_workers (1..HS_MAX_SERVER_WORKERS) workers, i.e.
 * at most that many batches in flight; each holds its own device buffers. */
int hs_server_create_workers(const hs_db* db, int32_t max_batch, int32_t max_qlen,
                             int64_t max_residues, int32_t k, int32_t n_aln, int32_t n_workers,
                             hs_server** out);

/* Stops the workers after their current batches and releases the server; queries
 * still waiting are dropped, unclaimed results discarded.  NULL is allowed. */
int hs_server_free(hs_server* s);

/* Queues one query (host ASCII, 1..max_qlen letters) with its parameters
 * (copied, matrix included) under a caller-chosen tag that is not pending
 * (queued or being searched) or unclaimed: HS_EINVAL otherwise.  Validates
 * the letters; returns at once. */
int hs_server_submit(hs_server* s, const char* query, int32_t qlen, const hs_params* params,
                     uint64_t tag);

/* Tags of finished queries, oldest first: up to max_tags into tags,
 * *n_tags set to the count; waits up to timeout_ms for the first one when
 * none is ready (0: do not wait).  Each finished tag is reported once. */
int hs_server_poll(hs_server* s, uint64_t* tags, int32_t max_tags, int32_t* n_tags,
                   int32_t timeout_ms);

/* Results of a finished query, as hs_search reports them (hits: k entries,
 * alns: n_aln entries, ops_off into ops), and its timing (may be NULL).
 * Claims the result, except on HS_ENOSPC (*ops_used = size needed).  If the
 * query's batch failed, returns that error. */
int hs_server_result(hs_server* s, uint64_t tag, hs_hit* hits, int32_t* n_hits, hs_aln* alns,
                     int32_t* n_alns, uint32_t* ops, int64_t ops_cap, int64_t* ops_used,
                     hs_server_timing* timing);

/* Queries waiting, batches run and queries served so far (any pointer may be
 * NULL). */
int hs_server_stats(hs_server* s, int64_t* pending, int64_t* batches, int64_t* served);

/* Thread-local description of the last failing call on this thread. */
const char* hs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HS_H */
