/*
 * sw_check.c -- TEST INFRASTRUCTURE ONLY: an upper-bound checker for the
 * oracle, not part of the method.
 *
 * Optimal local alignment score with affine gaps (Smith & Waterman 1981 with
 * Gotoh's 1982 three-state recurrence), in two rows of memory.  A gap run of g
 * columns costs GOP + (g-1)*GEP, the convention of Section III.B.1 of the
 * paper, so that every alignment the heuristic reports, with its leading and
 * trailing gap columns removed, is one of the alignments maximised here.
 */
#include <stdint.h>
#include <stdlib.h>

#define SW_NSYM 24
#define SW_NEG (INT64_MIN / 4)

int64_t sw_gotoh_local(const uint8_t* a, int32_t n, const uint8_t* b, int32_t m,
                       const int8_t* B, int32_t gop, int32_t gep) {
    /* H: best alignment ending at (i, j); E: ending with a gap in a (b[j]
     * against nothing); F: ending with a gap in b. */
    int64_t* H = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    int64_t* E = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!H || !E) { free(H); free(E); return SW_NEG; }
    int64_t best = 0;
    for (int32_t j = 0; j <= m; ++j) { H[j] = 0; E[j] = SW_NEG; }
    for (int32_t i = 1; i <= n; ++i) {
        int64_t diag = H[0];       /* H[i-1][j-1] */
        int64_t Hleft = 0;         /* H[i][j-1] */
        int64_t F = SW_NEG;        /* F[i][j-1] along row i */
        H[0] = 0;
        for (int32_t j = 1; j <= m; ++j) {
            int64_t up = H[j];     /* H[i-1][j] */
            /* vertical gap (a[i] against nothing), run continues down column j */
            int64_t e = up - gop;
            if (E[j] - gep > e) e = E[j] - gep;
            E[j] = e;
            /* horizontal gap (b[j] against nothing) */
            int64_t f = Hleft - gop;
            if (F - gep > f) f = F - gep;
            F = f;
            int64_t h = diag + B[a[i - 1] * SW_NSYM + b[j - 1]];
            if (e > h) h = e;
            if (f > h) h = f;
            if (h < 0) h = 0;
            diag = up;
            H[j] = h;
            Hleft = h;
            if (h > best) best = h;
        }
    }
    free(H);
    free(E);
    return best;
}
