"""Pins on the Smith-Waterman upper-bound checker used by the oracle pins:
exhaustive enumeration of every local alignment on tiny inputs, and a second,
full-matrix implementation on larger ones."""
import functools

import numpy as np
import pytest

import oracle as O

B = O.blosum62().astype(np.int64)
NEG = -10**9


def brute_local(a, b, gop, gep):
    """Best score over every alignment of every pair of non-empty substrings
    (and 0 for the empty alignment), with each gap run of g columns costing
    gop + (g - 1) * gep.  Pure enumeration, no dynamic programming."""
    def aligns(x, y):
        # all global alignments of x and y as op strings over M, I, D
        if not x and not y:
            yield ""
            return
        if x and y:
            for r in aligns(x[1:], y[1:]):
                yield "M" + r
        if x:
            for r in aligns(x[1:], y):
                yield "I" + r
        if y:
            for r in aligns(x, y[1:]):
                yield "D" + r

    def score(x, y, ops):
        s, i, j, prev = 0, 0, 0, None
        for o in ops:
            if o == "M":
                s += int(B[x[i], y[j]]); i += 1; j += 1
            else:
                s -= gep if o == prev else gop
                if o == "I":
                    i += 1
                else:
                    j += 1
            prev = o
        return s

    best = 0
    for i1 in range(len(a)):
        for i2 in range(i1 + 1, len(a) + 1):
            for j1 in range(len(b)):
                for j2 in range(j1 + 1, len(b) + 1):
                    x, y = tuple(a[i1:i2]), tuple(b[j1:j2])
                    for ops in aligns(x, y):
                        best = max(best, score(x, y, ops))
    return best


def full_matrix_local(a, b, gop, gep):
    """Textbook three-matrix Gotoh recurrences over the full (n+1)x(m+1) grid."""
    n, m = len(a), len(b)
    H = np.zeros((n + 1, m + 1), dtype=np.int64)
    E = np.full((n + 1, m + 1), NEG, dtype=np.int64)   # gap in b (a letter vs nothing)
    F = np.full((n + 1, m + 1), NEG, dtype=np.int64)   # gap in a
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            E[i, j] = max(H[i - 1, j] - gop, E[i - 1, j] - gep)
            F[i, j] = max(H[i, j - 1] - gop, F[i, j - 1] - gep)
            H[i, j] = max(0, H[i - 1, j - 1] + B[a[i - 1], b[j - 1]], E[i, j], F[i, j])
    return int(H.max())


@pytest.mark.parametrize("case", range(40))
def test_sw_vs_enumeration(case):
    rng = np.random.default_rng(700 + case)
    n, m = int(rng.integers(1, 5)), int(rng.integers(1, 5))
    letters = 4 if case % 2 else 20       # small alphabets make gaps pay off
    a = rng.integers(0, letters, n).astype(np.uint8)
    b = rng.integers(0, letters, m).astype(np.uint8)
    gop, gep = int(rng.integers(0, 6)), int(rng.integers(0, 4))
    assert O.sw_score(a, b, gop, gep) == brute_local(a, b, gop, gep)


def test_sw_gap_case():
    # W..W against W W: bridging the two W's needs a gap run of 3 in b
    a = O.encode("WAAAW")
    b = O.encode("WW")
    assert O.sw_score(a, b, 2, 1) == 22 - (2 + 2 * 1)
    assert brute_local(a, b, 2, 1) == 18


@pytest.mark.parametrize("case", range(12))
def test_sw_vs_full_matrix(case):
    rng = np.random.default_rng(800 + case)
    a = rng.integers(0, 20, int(rng.integers(1, 60))).astype(np.uint8)
    b = rng.integers(0, 20, int(rng.integers(1, 60))).astype(np.uint8)
    if case % 3 == 0:
        b = np.concatenate([a[5:], b[:10], a[:20]])
    gop, gep = int(rng.integers(0, 15)), int(rng.integers(0, 6))
    assert O.sw_score(a, b, gop, gep) == full_matrix_local(a, b, gop, gep)
