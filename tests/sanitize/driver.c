/* Host-sanitizer driver (built with AddressSanitizer and UndefinedBehavior-
 * Sanitizer by tests/test_sanitize_cpu.py; needs no GPU).
 *
 * Part 1 runs the oracle (linked in from oracle/*.c) on random pairs in both
 * modes, a small search, the Smith-Waterman checker and the encoder, and
 * checks that every alignment rescored from its rows gives its score.
 * Part 2 calls the host-only paths of the library's C ABI (defaults, checks,
 * encoding, matrix copy, and the argument errors every entry point returns
 * before it touches the device).  Exit status 0 when everything held. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hs.h"

/* oracle entry points (oracle/hs_oracle.c, oracle/sw_check.c) */
typedef struct {
    int32_t gop, gep, pgp, lfactor_q16, sfactor_q16, minfactor_q16, rounds, full_slide;
    uint64_t seed;
} orc_params;
typedef struct { int32_t pL, pS, ls, ss, kstar, dscore; } orc_step;
int orc_align_pair(const uint8_t* q, int32_t qlen, const uint8_t* tg, int32_t tlen,
                   uint64_t target_id, const orc_params* p, const int8_t* matrix,
                   int32_t* score_out, int32_t* round_out, uint8_t* qrow, uint8_t* trow,
                   int32_t row_cap, int32_t* row_len, orc_step* trace, int32_t trace_cap,
                   int32_t* n_steps, int64_t* cells);
int orc_search(const uint8_t* db, const int64_t* offsets, int64_t n_targets, const uint8_t* q,
               int32_t qlen, const orc_params* p, const int8_t* matrix, int32_t* scores,
               int32_t* rounds, int64_t* cells_total);
int64_t orc_score_rows(const uint8_t* a, const uint8_t* b, int32_t n, const orc_params* p,
                       const int8_t* matrix);
int orc_encode(const char* ascii, int64_t n, uint8_t* codes);
int64_t sw_gotoh_local(const uint8_t* a, int32_t na, const uint8_t* b, int32_t nb,
                       const int8_t* B, int32_t gop, int32_t gep);
void orc_blosum62_copy(int8_t* out);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) {           /* splitmix64 */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int32_t below(int32_t n) { return (int32_t)(next() % (uint64_t)n); }

static int failures = 0;
#define CHECK(cond, ...)                                   \
    do {                                                   \
        if (!(cond)) {                                     \
            fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            fprintf(stderr, __VA_ARGS__);                  \
            fprintf(stderr, "\n");                         \
            ++failures;                                    \
        }                                                  \
    } while (0)

static void oracle_part(void) {
    int8_t B[24 * 24];
    orc_blosum62_copy(B);
    for (int it = 0; it < 400; ++it) {
        int32_t qlen = 1 + below(150), tlen = 1 + below(220);
        uint8_t* q = malloc((size_t)qlen);
        uint8_t* t = malloc((size_t)tlen);
        for (int32_t i = 0; i < qlen; ++i) q[i] = (uint8_t)below(24);
        for (int32_t i = 0; i < tlen; ++i) t[i] = (uint8_t)below(24);
        orc_params p = {below(15), below(8), below(4), below(65537), below(65537), below(65537),
                        1 + below(4), it & 1, next()};
        int32_t cap = qlen + tlen, len = 0, score = 0, round = 0, steps = 0;
        int32_t tcap = (qlen < tlen ? qlen : tlen) + 1;
        uint8_t* qr = malloc((size_t)cap);
        uint8_t* tr = malloc((size_t)cap);
        orc_step* trace = malloc(sizeof(orc_step) * (size_t)tcap);
        int64_t cells = 0;
        int rc = orc_align_pair(q, qlen, t, tlen, (uint64_t)it, &p, NULL, &score, &round, qr, tr,
                                cap, &len, trace, tcap, &steps, &cells);
        CHECK(rc == 0, "align_pair rc %d", rc);
        CHECK(orc_score_rows(qr, tr, len, &p, NULL) == score, "rescore differs (case %d)", it);
        CHECK(score <= sw_gotoh_local(q, qlen, t, tlen, B, p.gop, p.gep),
              "above the Smith-Waterman optimum (case %d)", it);
        free(q); free(t); free(qr); free(tr); free(trace);
    }
    /* a small search */
    const int32_t n = 50;
    int64_t off[51];
    off[0] = 0;
    for (int i = 0; i < n; ++i) off[i + 1] = off[i] + 1 + below(120);
    uint8_t* db = malloc((size_t)off[n]);
    for (int64_t i = 0; i < off[n]; ++i) db[i] = (uint8_t)below(20);
    uint8_t q[40];
    for (int i = 0; i < 40; ++i) q[i] = (uint8_t)below(20);
    int32_t scores[50], rounds[50];
    int64_t cells = 0;
    orc_params p = {10, 5, 0, 32768, 65536, 32768, 2, 0, 7};
    CHECK(orc_search(db, off, n, q, 40, &p, NULL, scores, rounds, &cells) == 0, "search");
    free(db);
    uint8_t codes[8];
    CHECK(orc_encode("ACDJOU*x", 8, codes) == 0, "encode");
    CHECK(orc_encode("AC-D", 4, codes) != 0, "encode accepted a dash");
}

static void abi_part(void) {
    hs_params p;
    hs_params_default(&p);
    CHECK(p.gop == 10 && p.gep == 5 && p.pgp == 0 && p.rounds == 1, "defaults");
    CHECK(hs_params_check(&p) == HS_OK, "default params rejected");
    hs_params bad = p;
    bad.rounds = 0;
    CHECK(hs_params_check(&bad) == HS_EINVAL && strlen(hs_last_error()) > 0, "rounds 0 accepted");
    bad = p;
    bad.lfactor_q16 = 70000;
    CHECK(hs_params_check(&bad) == HS_EINVAL, "factor above 1 accepted");
    bad = p;
    bad.gop = -1;
    CHECK(hs_params_check(&bad) == HS_EINVAL, "negative penalty accepted");
    int8_t m[24 * 24];
    hs_builtin_matrix(m);
    CHECK(m[0] == 4 && m[17 * 24 + 17] == 11, "matrix");
    int8_t wide[24 * 24];
    memset(wide, 0, sizeof(wide));
    wide[5] = 16;
    bad = p;
    bad.matrix = wide;
    CHECK(hs_params_check(&bad) == HS_EINVAL, "matrix spanning 16 accepted");
    uint8_t codes[16];
    CHECK(hs_encode("ARNDjou*", 8, codes) == HS_OK && codes[7] == 23 && codes[4] == 22, "encode");
    CHECK(hs_encode("AR ND", 5, codes) == HS_EINVAL, "encode accepted a space");
    /* argument errors returned before any device work */
    hs_hit hits[4];
    int32_t nh = 0;
    int64_t used = 0, n64 = 0;
    CHECK(hs_search(NULL, "ACD", 3, &p, 4, 0, NULL, hits, &nh, NULL, NULL, NULL, 0, &used) == HS_EINVAL,
          "search without a database");
    CHECK(hs_db_load(NULL, NULL, 1, NULL, NULL) != HS_OK, "db_load without inputs");
    CHECK(hs_db_free(NULL) == HS_OK, "db_free(NULL)");
    CHECK(hs_batch_create(NULL, 1, 10, 10, 1, 0, NULL) == HS_EINVAL, "batch without a database");
    CHECK(hs_batch_free(NULL) == HS_OK, "batch_free(NULL)");
    CHECK(hs_server_create(NULL, 1, 10, 10, 1, 0, NULL) == HS_EINVAL, "server without a database");
    CHECK(hs_server_free(NULL) == HS_OK, "server_free(NULL)");
    CHECK(hs_search_threshold(NULL, "ACD", 3, &p, 4, 0, NULL, hits, &n64, NULL, NULL, NULL, 0, &used)
              == HS_EINVAL, "threshold search without a database");
    int32_t score = 0, round = 0;
    uint32_t ops[8];
    CHECK(hs_align("", 0, "ACD", 3, &p, NULL, &score, &round, ops, 8, &used) == HS_EINVAL,
          "empty query aligned");
    CHECK(hs_align("ACD", 3, "A1D", 3, &p, NULL, &score, &round, ops, 8, &used) == HS_EINVAL,
          "bad residue aligned");
    CHECK(hs_workspace_bytes(NULL, 1, 10, 1, 0) == 0, "workspace of no database");
    CHECK(hs_threshold_workspace_bytes(NULL) == 0, "threshold workspace of no database");
}

int main(void) {
    oracle_part();
    abi_part();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("sanitized oracle and host ABI paths: all checks held\n");
    return 0;
}
