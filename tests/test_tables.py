"""Pins on the substitution table and background composition (BLOSUM62,
Section III.A/B.5 of the paper; Henikoff & Henikoff 1992)."""
import os

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _stats():
    d = {}
    for line in open(os.path.join(GOLD, "blosum62_stats.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        d[k] = float(v)
    return d


def test_alphabet():
    assert O.alphabet() == "ARNDCQEGHILKMFPSTWYVBZX*"


def test_symmetric():
    B = O.blosum62().astype(int)
    assert (B == B.T).all()


def test_diagonal_dominates_column_on_20_letters():
    # needed by the identity-prefix pin: B[y][y] > B[x][y] for every x != y
    B = O.blosum62().astype(int)[:20, :20]
    for y in range(20):
        col = B[:, y]
        assert col[y] == col.max() and (col == col[y]).sum() == 1


def test_range_and_star():
    B = O.blosum62().astype(int)
    assert B.min() == -4 and B.max() == 11 and B[17, 17] == 11  # W/W
    assert (B[23, :23] == -4).all() and B[23, 23] == 1


def test_background_and_lambda():
    """lambda solves sum p_a p_b exp(lambda s_ab) = 1; it and H agree with the
    published BLOSUM62 statistics to the printed digits, which a wrong entry or
    a wrong frequency would break."""
    counts = O.background_counts().astype(float)
    p = counts / counts.sum()
    assert counts.sum() == 450431
    assert abs(p.sum() - 1) < 1e-12
    S = O.blosum62().astype(float)[:20, :20]
    PP = np.outer(p, p)
    assert (PP * S).sum() < 0  # negative expected score (local alignment regime)
    lam = brentq(lambda l: (PP * np.exp(l * S)).sum() - 1, 1e-3, 5)
    H = lam * (PP * S * np.exp(lam * S)).sum()
    st = _stats()
    assert round(lam, 4) == st["lambda"]
    assert round(H, 4) == st["H"]


def test_generator_tables_match_oracle():
    alpha, M = synth.matrix_table()
    assert alpha == O.alphabet()
    assert (M == O.blosum62().astype(int)).all()
    counts = O.background_counts().astype(float)
    assert np.allclose(synth.background_probs(), counts / counts.sum())
