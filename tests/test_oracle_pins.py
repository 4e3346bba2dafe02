"""Pins on the oracle's heuristic, in the search mode (Fig. 1 with Section
III.B.3) and the pairwise mode (Fig. 1 as written), each checked against
something other than the oracle itself: hand-worked examples, closed forms
that hold for any random stream, brute-force re-derivation of every step, an
independent rescoring of every alignment, and the Smith-Waterman upper
bound."""
import os
import re

import numpy as np
import pytest

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
B = O.blosum62().astype(np.int64)
M64 = 2**64 - 1


# ----------------------------------------------------------------------------
# helpers written independently of the oracle
# ----------------------------------------------------------------------------
def rescore(qrow, trow, gop, gep, pgp):
    """SCORE of two aligned ASCII rows, from the wording of Section III.B.1:
    letter pairs from BLOSUM62; in each row, leading/trailing gap columns cost
    PGP each, any other maximal gap run costs GOP + (len - 1) * GEP."""
    al = O.alphabet()
    s = 0
    for a, b in zip(qrow, trow):
        if a != "-" and b != "-":
            s += int(B[al.index(a), al.index(b)])
    for row in (qrow, trow):
        core = row.strip("-")
        lead = len(row) - len(row.lstrip("-"))
        trail = len(row) - len(row.rstrip("-"))
        s -= pgp * (lead + trail) if core else pgp * len(row)
        for m in re.finditer(r"-+", core):
            s -= gop + (len(m.group()) - 1) * gep
    return s


def ungap(row):
    return row.replace("-", "")


def rand_seq(rng, n, letters=20):
    return rng.integers(0, letters, size=n).astype(np.uint8)


def rand_params(rng, pgp=None):
    return O.Params(gop=int(rng.integers(0, 15)), gep=int(rng.integers(0, 8)),
                    pgp=int(rng.integers(0, 4)) if pgp is None else pgp,
                    lfactor_q16=int(rng.integers(0, 65537)),
                    sfactor_q16=int(rng.integers(0, 65537)),
                    minfactor_q16=int(rng.integers(0, 65537)),
                    rounds=int(rng.integers(1, 4)), seed=int(rng.integers(0, 2**63)))


def numpy_draw(seed, tid, rnd, d):
    """random() of (target, round), from numpy's own Philox4x64-10 (which
    steps its 256-bit counter by one before each block, so start one below)."""
    c = [tid, rnd, d // 16, 0]
    for i in range(4):          # 256-bit decrement with borrow
        c[i] = (c[i] - 1) & M64
        if c[i] != M64:
            break
    g = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                         key=np.array([seed, 0], dtype=np.uint64))
    w = g.random_raw(4)
    return (int(w[(d // 4) % 4]) >> (16 * (d % 4))) & 0xFFFF


# ----------------------------------------------------------------------------
# hand-worked examples
# ----------------------------------------------------------------------------
def _examples():
    ex, cur = [], None
    for line in open(os.path.join(GOLD, "worked_examples.txt")):
        line = line.rstrip("\n")
        if line.startswith("#") or not line.strip():
            continue
        key, _, val = line.partition(" ")
        if key == "example":
            cur = {}
        elif key == "end":
            ex.append(cur)
        else:
            cur[key] = val
    return ex


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["query"])
def test_worked_examples(ex):
    gop, gep, pgp = map(int, ex["penalties"].split())
    lf, mf, sf = map(int, ex["factors"].split())
    p = O.Params(gop=gop, gep=gep, pgp=pgp, lfactor_q16=lf, minfactor_q16=mf, sfactor_q16=sf,
                 rounds=1, seed=int(ex["seed"]), full_slide=ex.get("mode") == "full")
    r = O.align_pair(O.encode(ex["query"]), O.encode(ex["target"]), int(ex["target_id"]), p,
                     trace=True)
    steps = [tuple(map(int, s.split())) for s in ex["steps"].split("|")]
    assert r["trace"] == steps
    assert O.decode(r["qrow"]) == ex["qrow"]
    assert O.decode(r["trow"]) == ex["trow"]
    assert r["score"] == int(ex["score"])


# ----------------------------------------------------------------------------
# P1: identity prefix -- closed form for any parameters, seed and rounds
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(60))
def test_identity_prefix(case):
    rng = np.random.default_rng(100 + case)
    p = rand_params(rng)
    n = int(rng.integers(1, 120))
    x = int(rng.integers(0, 80))
    a = rand_seq(rng, n)
    tail = rand_seq(rng, x)
    expect = int(sum(B[c, c] for c in a)) - p.pgp * x
    # target = query + tail: the target is large
    r = O.align_pair(a, np.concatenate([a, tail]), int(rng.integers(0, 10**6)), p)
    assert r["score"] == expect
    assert r["ops"] == ([n << 2 | O.OP_M] + ([x << 2 | O.OP_D] if x else []))
    # query = target + tail: the query is large
    r = O.align_pair(np.concatenate([a, tail]), a, int(rng.integers(0, 10**6)), p)
    assert r["score"] == expect
    assert r["ops"] == ([n << 2 | O.OP_M] + ([x << 2 | O.OP_I] if x else []))


# ----------------------------------------------------------------------------
# P2: one-letter small sequence with LF = 1: first best letter, closed form
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(40))
def test_single_letter(case):
    rng = np.random.default_rng(200 + case)
    p = rand_params(rng)
    p.lfactor_q16 = 65536
    p.minfactor_q16 = 65536
    L = rand_seq(rng, int(rng.integers(2, 60)))
    s = rand_seq(rng, 1)
    col = B[L, s[0]]
    kbest = int(np.argmax(col))          # first maximum
    expect = int(col.max()) - p.pgp * (len(L) - 1)
    r = O.align_pair(s, L, 7, p)         # target large
    assert r["score"] == expect
    ops = ([kbest << 2 | O.OP_D] if kbest else []) + [4 | O.OP_M]
    rest = len(L) - kbest - 1
    ops += [rest << 2 | O.OP_D] if rest else []
    assert r["ops"] == ops
    r = O.align_pair(L, s, 8, p)         # query large
    assert r["score"] == expect


# ----------------------------------------------------------------------------
# P3 + P4: every step re-derived by brute force, draws from numpy
# ----------------------------------------------------------------------------
def check_trace(q, t, tid, p, r, matrix=None):
    target_large = len(t) >= len(q)
    L, S = (t, q) if target_large else (q, t)
    # the matrix scores a query letter (row) against a target letter
    # (column): seen from (large, small) it is transposed when the target is
    # the large one
    M = B if matrix is None else matrix.astype(np.int64)
    BLS = M.T if target_large else M
    tr = r["trace"]
    # round actually reported: recompute its factors from numpy draws
    rnd = r["round"]
    lf = max(p.minfactor_q16, numpy_draw(p.seed, tid, rnd, 0))
    sf = max(p.minfactor_q16, numpy_draw(p.seed, tid, rnd, 1))
    LF = (p.lfactor_q16 * lf) >> 16
    SF = (p.sfactor_q16 * sf) >> 16
    pL = pS = 0
    total = 0
    cols_q, cols_t = [], []
    for step, (tpL, tpS, ls, ss, k, D) in enumerate(tr):
        assert (tpL, tpS) == (pL, pS)
        nL, nS = len(L) - pL, len(S) - pS
        assert nL > 0 and nS > 0
        u = numpy_draw(p.seed, tid, rnd, 2 + step)
        assert ls == max(1, (nL * LF) >> 16)
        assert ss == min(ls, max(1, (nS * SF * u) >> 32))
        assert 1 <= ss <= ls <= nL and ss <= nS
        Ds = [int(BLS[L[pL + kk:pL + kk + ss], S[pS:pS + ss]].sum()) for kk in range(ls - ss + 1)]
        assert D == max(Ds) and k == Ds.index(max(Ds))
        total += D
        if step == 0:
            total -= p.pgp * k
        elif k > 0:
            total -= p.gop + (k - 1) * p.gep
        pL += k + ss
        pS += ss
    assert pL >= len(L) or pS >= len(S)
    total -= p.pgp * ((len(L) - pL) + (len(S) - pS))
    assert total == r["score"]


@pytest.mark.parametrize("case", range(40))
def test_steps_brute_force(case):
    rng = np.random.default_rng(300 + case)
    p = rand_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 90)), 24)
    t = rand_seq(rng, int(rng.integers(1, 140)), 24)
    tid = int(rng.integers(0, 2**40))
    r = O.align_pair(q, t, tid, p, trace=True)
    check_trace(q, t, tid, p, r)


@pytest.mark.parametrize("case", range(10))
def test_steps_equal_length(case):
    """Equal lengths: the target plays "large" (the paper leaves the choice
    open); every gap column before the tail is then a target letter (D)."""
    rng = np.random.default_rng(350 + case)
    p = rand_params(rng)
    n = int(rng.integers(2, 80))
    q, t = rand_seq(rng, n), rand_seq(rng, n)
    r = O.align_pair(q, t, case, p, trace=True)
    check_trace(q, t, case, p, r)
    assert all((o & 3) != O.OP_I for o in r["ops"][:-1])


def test_steps_full_factors():
    """LFactor = MinFactor = 1 makes ls exactly the rest of large."""
    rng = np.random.default_rng(7)
    for i in range(20):
        p = O.Params(lfactor_q16=65536, minfactor_q16=65536, sfactor_q16=65536,
                     seed=int(rng.integers(0, 2**62)))
        q, t = rand_seq(rng, 40), rand_seq(rng, 70)
        r = O.align_pair(q, t, i, p, trace=True)
        for (pL, pS, ls, ss, k, D) in r["trace"]:
            assert ls == len(t) - pL
        check_trace(q, t, i, p, r)


# ----------------------------------------------------------------------------
# P4b: a matrix that is not symmetric scores query letters (rows) against
# target letters (columns), whichever sequence is the large one
# ----------------------------------------------------------------------------
def asym_matrix(rng):
    m = rng.integers(-5, 11, size=(24, 24)).astype(np.int8)    # span 15
    assert (m != m.T).any()
    return m


@pytest.mark.parametrize("case", range(20))
def test_asymmetric_single_letter(case):
    """One-letter small sequence, LF = 1: the first best letter of the
    matrix column (target large) or row (query large), in closed form."""
    rng = np.random.default_rng(560 + case)
    m = asym_matrix(rng)
    p = rand_params(rng)
    p.lfactor_q16 = p.minfactor_q16 = 65536
    L = rand_seq(rng, int(rng.integers(2, 40)), 24)
    s = rand_seq(rng, 1, 24)
    col = m[s[0], L].astype(np.int64)        # query s, targets L[k]
    r = O.align_pair(s, L, 3, p, matrix=m)
    assert r["score"] == int(col.max()) - p.pgp * (len(L) - 1)
    row = m[L, s[0]].astype(np.int64)        # query letters L[k], target s
    r = O.align_pair(L, s, 4, p, matrix=m)
    assert r["score"] == int(row.max()) - p.pgp * (len(L) - 1)


@pytest.mark.parametrize("case", range(20))
def test_asymmetric_swap(case):
    """Swapping query and target and transposing the matrix leaves every
    letter pair's score, and so the alignment's score, unchanged (unequal
    lengths, so that the large sequence is the same one)."""
    rng = np.random.default_rng(600 + case)
    m = asym_matrix(rng)
    p = rand_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 80)), 24)
    t = rand_seq(rng, int(rng.integers(1, 120)), 24)
    if len(q) == len(t):
        t = np.concatenate([t, rand_seq(rng, 1, 24)])
    a = O.align_pair(q, t, case, p, matrix=m)
    b = O.align_pair(t, q, case, p, matrix=np.ascontiguousarray(m.T))
    assert (a["score"], a["round"]) == (b["score"], b["round"])


@pytest.mark.parametrize("case", range(20))
def test_asymmetric_steps_brute_force(case):
    rng = np.random.default_rng(640 + case)
    m = asym_matrix(rng)
    p = rand_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 90)), 24)
    t = rand_seq(rng, int(rng.integers(1, 140)), 24)
    r = O.align_pair(q, t, case, p, matrix=m, trace=True)
    check_trace(q, t, case, p, r, matrix=m)


# ----------------------------------------------------------------------------
# P5: independent rescoring and validity of every alignment
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(60))
def test_rescore(case):
    rng = np.random.default_rng(400 + case)
    p = rand_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 200)), 24)
    t = rand_seq(rng, int(rng.integers(1, 300)), 24)
    r = O.align_pair(q, t, case, p)
    qr, tr = O.decode(r["qrow"]), O.decode(r["trow"])
    assert ungap(qr) == O.decode(q) and ungap(tr) == O.decode(t)
    assert all(not (a == "-" and b == "-") for a, b in zip(qr, tr))
    assert rescore(qr, tr, p.gop, p.gep, p.pgp) == r["score"]
    # ops cover both sequences from position 0
    nq = sum(o >> 2 for o in r["ops"] if (o & 3) in (O.OP_M, O.OP_I))
    nt = sum(o >> 2 for o in r["ops"] if (o & 3) in (O.OP_M, O.OP_D))
    assert (nq, nt) == (len(q), len(t))


# ----------------------------------------------------------------------------
# P6: no heuristic score exceeds the affine Smith-Waterman optimum
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(40))
def test_below_smith_waterman(case):
    rng = np.random.default_rng(500 + case)
    p = rand_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 150)))
    if case % 2:   # related pair: mutated copy with an insertion
        t = q.copy()
        t[rng.random(len(t)) < 0.3] = rng.integers(0, 20)
        t = np.concatenate([rand_seq(rng, 5), t[: len(t) // 2], rand_seq(rng, 7), t[len(t) // 2:]])
    else:
        t = rand_seq(rng, int(rng.integers(1, 200)))
    r = O.align_pair(q, t, case, p)
    assert r["score"] <= O.sw_score(q, t, p.gop, p.gep)


# ----------------------------------------------------------------------------
# P9: more rounds never lower the score (round r's draws depend only on r)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("case", range(15))
def test_rounds_monotone(case):
    rng = np.random.default_rng(600 + case)
    p = rand_params(rng)
    q, t = rand_seq(rng, int(rng.integers(5, 100))), rand_seq(rng, int(rng.integers(5, 150)))
    prev = None
    for R in range(1, 7):
        p.rounds = R
        r = O.align_pair(q, t, case, p)
        if prev is not None:
            assert r["score"] >= prev[0]
            if r["score"] == prev[0]:
                assert r["round"] == prev[1]    # first round kept on ties
        prev = (r["score"], r["round"])


# ----------------------------------------------------------------------------
# search: ranking rule and agreement with pairwise runs
# ----------------------------------------------------------------------------
def test_search_rank_and_planted():
    import synth
    q, res, off, planted = synth.tiny_db(seed=11, n_bg=300, qlen=40, n_hom=8)
    codes = O.encode_db(res, off)
    qc = O.encode(bytes(q))
    out = O.search(codes, off, qc, O.Params(), k=60, n_aln=10)
    sc = out["all_scores"]
    ids = out["ids"]
    keys = [(-int(sc[i]), int(i)) for i in ids]
    assert keys == sorted(keys)
    rest = np.setdiff1d(np.arange(len(sc)), ids)
    assert (sc[rest] <= sc[ids[-1]]).all()
    for i in (0, 5, 77):
        a = O.align_pair(qc, codes[off[i]:off[i + 1]], i, O.Params())
        assert a["score"] == sc[i]


# ----------------------------------------------------------------------------
# Pairwise mode (Fig. 1 as written): every placement with some overlap
# ----------------------------------------------------------------------------
def full_params(rng, rounds=None):
    p = rand_params(rng)
    p.full_slide = True
    if rounds is not None:
        p.rounds = rounds
    return p


def full_slide_reference(q, t, tid, p):
    """Independent re-derivation of one pair in the pairwise mode, from the
    wording of Fig. 1 and Section III.B.2.  Per round: draws from numpy's
    Philox; per step, windows of ls and ss letters (no contained-shift clamp)
    and every placement i = 0 .. ss + ls - 2 (shift k = i - ss + 1) scored
    over the letters that face each other, the first best kept; small gives
    up its whole window, large its letters through the last one facing small;
    the rows are built column by column and scored by rescore().  Returns
    (score, round, query row, target row, trace of that round)."""
    al = O.alphabet()
    target_large = len(t) >= len(q)
    L, S = (t, q) if target_large else (q, t)
    best = None
    for rnd in range(p.rounds):
        lf = max(p.minfactor_q16, numpy_draw(p.seed, tid, rnd, 0))
        sf = max(p.minfactor_q16, numpy_draw(p.seed, tid, rnd, 1))
        LF, SF = (p.lfactor_q16 * lf) >> 16, (p.sfactor_q16 * sf) >> 16
        pL = pS = 0
        rowL, rowS, trace = [], [], []
        step = 0
        while pL < len(L) and pS < len(S):
            nL, nS = len(L) - pL, len(S) - pS
            u = numpy_draw(p.seed, tid, rnd, 2 + step)
            ls = max(1, (nL * LF) >> 16)
            ss = max(1, (nS * SF * u) >> 32)
            Lw, Sw = L[pL:pL + ls], S[pS:pS + ss]
            Ds = []
            for i in range(ss + ls - 1):
                k = i - ss + 1
                Ds.append(sum(int(B[Lw[k + j], Sw[j]]) for j in range(ss) if 0 <= k + j < ls))
            i_best = Ds.index(max(Ds))
            k = i_best - ss + 1
            trace.append((pL, pS, ls, ss, k, max(Ds)))
            for i in range(k):
                rowL.append(al[Lw[i]])
                rowS.append("-")
            for j in range(ss):
                rowL.append(al[Lw[k + j]] if 0 <= k + j < ls else "-")
                rowS.append(al[Sw[j]])
            pL += min(k + ss, ls)
            pS += ss
            step += 1
        rowL += [al[c] for c in L[pL:]] + ["-"] * (len(S) - pS)
        rowS += ["-"] * (len(L) - pL) + [al[c] for c in S[pS:]]
        qrow, trow = ("".join(rowS), "".join(rowL)) if target_large else ("".join(rowL), "".join(rowS))
        score = rescore(qrow, trow, p.gop, p.gep, p.pgp)
        if best is None or score > best[0]:
            best = (score, rnd, qrow, trow, trace)
    return best


@pytest.mark.parametrize("case", range(50))
def test_full_slide_brute_force(case):
    rng = np.random.default_rng(700 + case)
    p = full_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 40)), 24)
    t = rand_seq(rng, int(rng.integers(1, 60)), 24)
    tid = int(rng.integers(0, 2**40))
    r = O.align_pair(q, t, tid, p, trace=True)
    score, rnd, qrow, trow, trace = full_slide_reference(q, t, tid, p)
    assert (r["score"], r["round"]) == (score, rnd)
    assert O.decode(r["qrow"]) == qrow and O.decode(r["trow"]) == trow
    assert r["trace"] == trace


def test_full_slide_differs_from_search():
    """Some pairs do take shifts outside the contained range (the pins above
    therefore exercise both kinds of overhang)."""
    rng = np.random.default_rng(790)
    neg = over = 0
    for case in range(60):
        p = full_params(rng)
        q = rand_seq(rng, int(rng.integers(2, 40)))
        t = rand_seq(rng, int(rng.integers(2, 60)))
        r = O.align_pair(q, t, case, p, trace=True)
        neg += any(k < 0 for (_, _, ls, ss, k, _) in r["trace"])
        over += any(k + ss > ls for (_, _, ls, ss, k, _) in r["trace"])
    assert neg > 5 and over > 5


@pytest.mark.parametrize("case", range(40))
def test_full_slide_identity_prefix(case):
    """With LF = 1 (LFactor = MinFactor = 1) the large window is all that is
    left of large, never shorter than the small window, and the identity
    placement beats every other one term by term (each BLOSUM62 diagonal entry
    is its column's maximum and positive), so the pair aligns ungapped at
    offset 0 for any SF, seed and rounds."""
    rng = np.random.default_rng(800 + case)
    p = full_params(rng)
    p.lfactor_q16 = p.minfactor_q16 = 65536
    n, x = int(rng.integers(1, 100)), int(rng.integers(0, 60))
    a, tail = rand_seq(rng, n), rand_seq(rng, x)
    expect = int(sum(B[c, c] for c in a)) - p.pgp * x
    r = O.align_pair(a, np.concatenate([a, tail]), int(rng.integers(0, 10**6)), p)
    assert r["score"] == expect
    assert r["ops"] == ([n << 2 | O.OP_M] + ([x << 2 | O.OP_D] if x else []))
    r = O.align_pair(np.concatenate([a, tail]), a, int(rng.integers(0, 10**6)), p)
    assert r["score"] == expect
    assert r["ops"] == ([n << 2 | O.OP_M] + ([x << 2 | O.OP_I] if x else []))


def _ss_sequence(p, tid, rnd, nL0, nS0, LF, SF, take_large):
    """Window sizes of a round from numpy draws, given how many large letters
    each step gives up (take_large(ls, ss))."""
    out = []
    nL, nS, step = nL0, nS0, 0
    while nL > 0 and nS > 0:
        u = numpy_draw(p.seed, tid, rnd, 2 + step)
        ls = max(1, (nL * LF) >> 16)
        ss = max(1, (nS * SF * u) >> 32)
        out.append((ls, ss))
        nL -= take_large(ls, ss)
        nS -= ss
        step += 1
    return out, nL, nS


@pytest.mark.parametrize("case", range(30))
def test_full_slide_least_overlap(case):
    """Every letter pair scores -3 (query all A, target all W): the best
    placement overlaps one letter, and the first such is the one with small's
    last window letter on large's first, so each step gives up one large
    letter and ss small letters, ss - 1 of them against gaps in front.
    Closed form of the score from the window sizes (numpy draws)."""
    rng = np.random.default_rng(850 + case)
    p = full_params(rng, rounds=1)
    tid = int(rng.integers(0, 10**6))
    nq, nt = int(rng.integers(1, 60)), int(rng.integers(1, 60))
    q = O.encode("A" * nq)
    t = O.encode("W" * nt)
    L, S = (t, q) if nt >= nq else (q, t)
    lf = max(p.minfactor_q16, numpy_draw(p.seed, tid, 0, 0))
    sf = max(p.minfactor_q16, numpy_draw(p.seed, tid, 0, 1))
    LF, SF = (p.lfactor_q16 * lf) >> 16, (p.sfactor_q16 * sf) >> 16
    steps, nL, nS = _ss_sequence(p, tid, 0, len(L), len(S), LF, SF, lambda ls, ss: 1)
    expect = -3 * len(steps)
    for i, (ls, ss) in enumerate(steps):
        g = ss - 1
        if g:
            expect -= p.pgp * g if i == 0 else p.gop + (g - 1) * p.gep
    expect -= p.pgp * (nL + nS)
    r = O.align_pair(q, t, tid, p, trace=True)
    assert r["score"] == expect
    assert [(ls, ss, k) for (_, _, ls, ss, k, _) in r["trace"]] == [(ls, ss, 1 - ss) for ls, ss in steps]


@pytest.mark.parametrize("case", range(30))
def test_full_slide_most_overlap(case):
    """Every letter pair scores 11 (both sequences all W): the best placement
    has the most overlap, min(ss, ls) letters, first reached at shift 0 when
    the small window fits (ss <= ls) and at shift ls - ss < 0 otherwise, where
    the first ss - ls small letters hang in front against gaps.  Closed form
    of the score from the window sizes (numpy draws)."""
    rng = np.random.default_rng(900 + case)
    p = full_params(rng, rounds=1)
    tid = int(rng.integers(0, 10**6))
    nq, nt = int(rng.integers(1, 60)), int(rng.integers(1, 60))
    q, t = O.encode("W" * nq), O.encode("W" * nt)
    L, S = (t, q) if nt >= nq else (q, t)
    lf = max(p.minfactor_q16, numpy_draw(p.seed, tid, 0, 0))
    sf = max(p.minfactor_q16, numpy_draw(p.seed, tid, 0, 1))
    LF, SF = (p.lfactor_q16 * lf) >> 16, (p.sfactor_q16 * sf) >> 16
    steps, nL, nS = _ss_sequence(p, tid, 0, len(L), len(S), LF, SF, lambda ls, ss: min(ss, ls))
    expect = 0
    for i, (ls, ss) in enumerate(steps):
        expect += 11 * min(ss, ls)
        g = max(0, ss - ls)
        if g:
            expect -= p.pgp * g if i == 0 else p.gop + (g - 1) * p.gep
    expect -= p.pgp * (nL + nS)
    r = O.align_pair(q, t, tid, p, trace=True)
    assert r["score"] == expect
    assert [k for (_, _, _, _, k, _) in r["trace"]] == [min(0, ls - ss) for ls, ss in steps]


@pytest.mark.parametrize("case", range(40))
def test_full_slide_rescore(case):
    rng = np.random.default_rng(950 + case)
    p = full_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 150)), 24)
    t = rand_seq(rng, int(rng.integers(1, 200)), 24)
    r = O.align_pair(q, t, case, p)
    qr, tr = O.decode(r["qrow"]), O.decode(r["trow"])
    assert ungap(qr) == O.decode(q) and ungap(tr) == O.decode(t)
    assert all(not (a == "-" and b == "-") for a, b in zip(qr, tr))
    assert rescore(qr, tr, p.gop, p.gep, p.pgp) == r["score"]


@pytest.mark.parametrize("case", range(30))
def test_full_slide_below_smith_waterman(case):
    rng = np.random.default_rng(1000 + case)
    p = full_params(rng)
    q = rand_seq(rng, int(rng.integers(1, 120)))
    if case % 2:
        t = q.copy()
        t[rng.random(len(t)) < 0.3] = rng.integers(0, 20)
        t = np.concatenate([rand_seq(rng, 4), t, rand_seq(rng, 9)])
    else:
        t = rand_seq(rng, int(rng.integers(1, 160)))
    r = O.align_pair(q, t, case, p)
    assert r["score"] <= O.sw_score(q, t, p.gop, p.gep)


@pytest.mark.parametrize("case", range(8))
def test_full_slide_rounds_monotone(case):
    """Up to the Rounds = 20 of the paper's alignment tests (Section V)."""
    rng = np.random.default_rng(1050 + case)
    p = full_params(rng)
    q, t = rand_seq(rng, int(rng.integers(5, 80))), rand_seq(rng, int(rng.integers(5, 120)))
    prev = None
    for R in (1, 2, 5, 10, 20):
        p.rounds = R
        r = O.align_pair(q, t, case, p)
        if prev is not None:
            assert r["score"] >= prev[0]
            if r["score"] == prev[0]:
                assert r["round"] == prev[1]
        prev = (r["score"], r["round"])
