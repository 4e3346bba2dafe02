"""GPU parity: the HIP path against the oracle, bit for bit (all arithmetic is
integer, so the tolerance is zero): every pair score, the winning round, the
work count, the ranked list and every returned alignment, on seeded synthetic
databases from tiny edge cases to the full 500,200-target workload."""
import concurrent.futures as cf
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def H():
    import paper_1508_06561_amd as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_scores(codes, off, q, params, threads=None):
    """All pair scores from the oracle, in parallel over target chunks (the C
    oracle releases the GIL)."""
    n = len(off) - 1
    threads = threads or min(16, os.cpu_count() or 1)
    chunks = np.array_split(np.arange(n, dtype=np.int64), max(1, threads * 4))
    out = np.zeros(n, dtype=np.int32)
    cells = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {ex.submit(O.score_all, codes, off, q, params, None, ids): ids for ids in chunks
                if len(ids)}
        for f, ids in futs.items():
            s, _, c = f.result()
            out[ids] = s
            cells += c
    return out, cells


def to_oparams(p):
    return O.Params(gop=p.gop, gep=p.gep, pgp=p.pgp, lfactor_q16=p.lfactor_q16,
                    sfactor_q16=p.sfactor_q16, minfactor_q16=p.minfactor_q16, rounds=p.rounds,
                    seed=p.seed)


def check_search(db, codes, off, query, p, k, n_aln, matrix=None):
    """hs_search against the oracle: ranked hits and every alignment."""
    r = db.search(bytes(query), p, k=k, n_aln=n_aln)
    ref = O.search(codes, off, O.encode(bytes(query)), to_oparams(p), k=k, n_aln=n_aln,
                   min_score=p.min_score, matrix=matrix)
    assert list(r.hits["target_id"]) == [int(i) for i in ref["ids"]]
    assert list(r.hits["score"]) == [int(s) for s in ref["scores"]]
    assert list(r.hits["round"]) == [int(ref["rounds"][i]) for i in ref["ids"]]
    assert len(r.alns) == len(ref["alns"])
    for i, (tid, score, ops) in enumerate(ref["alns"]):
        assert int(r.alns[i]["target_id"]) == tid
        assert int(r.alns[i]["score"]) == score
        assert [int(x) for x in r.ops_of(i)] == ops, f"alignment of rank {i} (target {tid})"
    return r, ref


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny():
    w = synth.config_tiny()
    codes = O.encode_db(w.residues, w.offsets)
    say(f"tiny workload: {w.n_targets} targets, {w.db_residues} residues")
    db = H().Database(w.residues, w.offsets)
    yield w, codes, db
    db.close()


def test_tiny_every_score(tiny):
    w, codes, db = tiny
    q = w.queries[0]
    s, rounds, cells = db.scores(bytes(q))
    ref, ref_cells = oracle_scores(codes, w.offsets, O.encode(bytes(q)), O.Params())
    assert (s == ref).all(), f"{(s != ref).sum()} scores differ"
    assert (rounds == 0).all()
    assert cells == ref_cells


def test_tiny_search_full_ranking(tiny):
    w, codes, db = tiny
    # k = every target: the whole ranked list, plus 50 alignments
    check_search(db, codes, w.offsets, w.queries[0], H().Params(), k=w.n_targets, n_aln=50)


def test_tiny_repeat_identical(tiny):
    w, codes, db = tiny
    a = db.search(bytes(w.queries[0]), H().Params(), k=50, n_aln=50)
    b = db.search(bytes(w.queries[0]), H().Params(), k=50, n_aln=50)
    assert (a.hits == b.hits).all() and (a.alns == b.alns).all() and (a.ops == b.ops).all()


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small():
    q, res, off, planted = synth.tiny_db(seed=5, n_bg=400, qlen=70, n_hom=10)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    yield q, res, off, codes, db
    db.close()


VARIANTS = {
    "periphery": dict(pgp=3),
    "rounds4": dict(rounds=4, seed=12345),
    "full_factors": dict(lfactor_q16=65536, sfactor_q16=65536, minfactor_q16=65536),
    "section_b1_factors": dict(lfactor_q16=65536, sfactor_q16=32768),
    "zero_factors": dict(lfactor_q16=0, sfactor_q16=0, minfactor_q16=0),
    "cheap_gaps": dict(gop=1, gep=0, pgp=1, seed=99),
    "big_penalties": dict(gop=1000, gep=1000, pgp=1000, rounds=2, seed=2**63 + 5),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_parameter_variants(small, name):
    q, res, off, codes, db = small
    p = H().Params(**VARIANTS[name])
    say(f"variant {name}")
    s, rounds, cells = db.scores(bytes(q), p)
    oc = O.encode(bytes(q))
    ref = O.score_all(codes, off, oc, to_oparams(p))
    assert (s == ref[0]).all(), f"{(s != ref[0]).sum()} scores differ"
    assert (rounds == ref[1]).all()
    assert cells == ref[2]
    check_search(db, codes, off, q, p, k=120, n_aln=40)


def test_custom_matrix(small):
    q, res, off, codes, db = small
    m = np.full((24, 24), -2, dtype=np.int8)
    np.fill_diagonal(m, 7)
    m[0, 1] = m[1, 0] = 13       # span 15, the widest allowed
    p = H().Params(matrix=m, pgp=1)
    s, _, _ = db.scores(bytes(q), p)
    ref = O.score_all(codes, off, O.encode(bytes(q)), to_oparams(p), matrix=m)[0]
    assert (s == ref).all()
    check_search(db, codes, off, q, p, k=60, n_aln=20, matrix=m)


@pytest.mark.parametrize("qlen", [70, 300])
def test_asymmetric_matrix(small, qlen):
    """A matrix that is not symmetric scores query letters (rows) against
    target letters (columns): every pair score, the ranking and the
    alignments equal the oracle's, for targets shorter and longer than the
    query; the transposed matrix gives other scores."""
    q0, res, off, codes, db = small
    rng = np.random.default_rng(71 + qlen)
    q = q0 if qlen == len(q0) else synth.random_protein(rng, qlen)
    m = rng.integers(-5, 11, size=(24, 24)).astype(np.int8)     # span 15
    p = H().Params(matrix=m, pgp=1, seed=4)
    lens = np.diff(off)
    say(f"asymmetric matrix, query {len(q)}: {(lens < len(q)).sum()} shorter targets, "
        f"{(lens >= len(q)).sum()} longer")
    assert (lens < len(q)).sum() >= 20 and (lens >= len(q)).sum() >= 20
    s, _, _ = db.scores(bytes(q), p)
    ref = O.score_all(codes, off, O.encode(bytes(q)), to_oparams(p), matrix=m)[0]
    assert (s == ref).all(), f"{(s != ref).sum()} pair scores differ"
    check_search(db, codes, off, q, p, k=60, n_aln=30, matrix=m)
    st, _, _ = db.scores(bytes(q), H().Params(matrix=np.ascontiguousarray(m.T), pgp=1, seed=4))
    assert (st != s).any()


def test_threshold_and_counts(small):
    q, res, off, codes, db = small
    ref = O.score_all(codes, off, O.encode(bytes(q)), O.Params())[0]
    thr = int(np.sort(ref)[-17])           # exactly the top 17 (or more on ties)
    p = H().Params(min_score=thr)
    r, rr = check_search(db, codes, off, q, p, k=100, n_aln=30)
    assert len(r.hits) == (ref >= thr).sum() and (r.hits["score"] >= thr).all()
    # nothing above the threshold
    p = H().Params(min_score=int(ref.max()) + 1)
    r = db.search(bytes(q), p, k=10, n_aln=5)
    assert len(r.hits) == 0 and len(r.alns) == 0
    # k larger than the database, no alignments
    r, _ = check_search(db, codes, off, q, H().Params(), k=4096, n_aln=0)
    assert len(r.hits) == len(off) - 1


# ---------------------------------------------------------------------------
def edge_db(rng, qlen):
    L = [1, 2, 3, 5, 6, 7, 12, qlen - 1, qlen, qlen + 1, 2 * qlen, 300, 1000, 2500]
    L = [x for x in L if x >= 1] + list(rng.integers(1, 40, size=60))
    seqs = [synth.random_protein(rng, int(n)) for n in L]
    # every letter of the alphabet, lower case, and the J/O/U aliases
    seqs.append(np.frombuffer(b"ARNDCQEGHILKMFPSTWYVBZX*arndcJOU", dtype=np.uint8).copy())
    return synth.pack(seqs)


@pytest.mark.parametrize("qlen", [1, 2, 7, 33, 64, 65, 300])
def test_edge_lengths(qlen):
    rng = np.random.default_rng(1000 + qlen)
    res, off = edge_db(rng, qlen)
    q = synth.random_protein(rng, qlen)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        say(f"edge lengths, qlen {qlen}, {len(off) - 1} targets")
        for p in [H().Params(), H().Params(pgp=2, rounds=3, seed=7)]:
            s, rounds, cells = db.scores(bytes(q), p)
            ref = O.score_all(codes, off, O.encode(bytes(q)), to_oparams(p))
            assert (s == ref[0]).all() and (rounds == ref[1]).all() and cells == ref[2]
            check_search(db, codes, off, q, p, k=len(off) - 1, n_aln=len(off) - 1)
    finally:
        db.close()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 129])
def test_group_boundaries(n):
    rng = np.random.default_rng(2000 + n)
    res, off = synth.random_db(rng, rng.integers(1, 200, size=n))
    q = synth.random_protein(rng, 50)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        check_search(db, codes, off, q, H().Params(), k=n, n_aln=min(n, 20))
    finally:
        db.close()


@pytest.mark.parametrize("n", [258_049, 300_007])
def test_striped_schedule_sizes(n):
    """Databases just large enough for the one-query kernel to put a pair on
    every lane of every resident wavefront (so it stripes length ranks over
    the wavefronts and takes the short tail from the counter), at a size that
    leaves a smaller grid and one with padding positions: every score and
    the work count, then the ranked list and alignments."""
    rng = np.random.default_rng(4000 + n)
    res, off = synth.random_db(rng, rng.integers(10, 121, size=n))
    q = synth.random_protein(rng, 40)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        say(f"striped schedule: {n} targets")
        s, _, cells = db.scores(bytes(q))
        ref, ref_cells = oracle_scores(codes, off, O.encode(bytes(q)), O.Params())
        assert (s == ref).all(), f"{(s != ref).sum()} scores differ"
        assert cells == ref_cells
        check_search(db, codes, off, q, H().Params(), k=100, n_aln=10)
    finally:
        db.close()


def test_identical_targets_tie_on_index():
    """Equal scores are ranked by target index (every target identical)."""
    rng = np.random.default_rng(3)
    t = synth.random_protein(rng, 120)
    res, off = synth.pack([t] * 300)
    q = synth.random_protein(rng, 40)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        p = H().Params(lfactor_q16=65536, minfactor_q16=65536, sfactor_q16=0)
        r, ref = check_search(db, codes, off, q, p, k=100, n_aln=10)
    finally:
        db.close()


def test_identity_prefix_on_gpu():
    """Closed form (identity prefix): a target that starts with the query
    scores sum B[q][q] and aligns ungapped at offset 0, for any parameters."""
    rng = np.random.default_rng(4)
    B = O.blosum62().astype(int)
    q = synth.random_protein(rng, 90)
    seqs = [np.concatenate([q, synth.random_protein(rng, int(x))]) for x in rng.integers(0, 200, 30)]
    res, off = synth.pack(seqs)
    db = H().Database(res, off)
    try:
        for p in [H().Params(), H().Params(pgp=2, rounds=3, seed=11, lfactor_q16=1000)]:
            s, _, _ = db.scores(bytes(q), p)
            qc = O.encode(bytes(q))
            expect = np.array([B[qc, qc].sum() - p.pgp * (len(x) - len(q)) for x in seqs])
            assert (s == expect).all()
    finally:
        db.close()


def test_errors():
    Hm = H()
    res, off = synth.pack([np.frombuffer(b"ACDEFG1HIK", dtype=np.uint8).copy()])
    with pytest.raises(Hm.HSError) as e:
        Hm.Database(res, off)
    assert e.value.code == -1
    res, off = synth.pack([np.frombuffer(b"ACDEFGHIK", dtype=np.uint8).copy()] * 3)
    db = Hm.Database(res, off)
    try:
        with pytest.raises(Hm.HSError):
            db.search(b"ACD-", Hm.Params(), k=3, n_aln=1)
        with pytest.raises(Hm.HSError):
            db.search(b"ACD", Hm.Params(), k=0, n_aln=0)
        with pytest.raises(Hm.HSError):
            db.search(b"A" * 5601, Hm.Params(), k=3, n_aln=1)
        # ops buffer too small: reported, nothing written
        import ctypes
        L = Hm.lib()
        p = Hm.Params().c()
        hits = np.zeros(3, dtype=Hm.hs.HIT_DTYPE)
        alns = np.zeros(3, dtype=Hm.hs.ALN_DTYPE)
        ops = np.zeros(1, dtype=np.uint32)
        nh, na, used = ctypes.c_int32(-7), ctypes.c_int32(-7), ctypes.c_int64()
        rc = L.hs_search(db._h, b"ACDKLM", 6, ctypes.byref(p), 3, 3, None, hits.ctypes.data,
                         ctypes.byref(nh), alns.ctypes.data, ctypes.byref(na), ops.ctypes.data, 1,
                         ctypes.byref(used))
        assert rc == Hm.hs.HS_ENOSPC and used.value > 1 and nh.value == -7
    finally:
        db.close()
    # empty database
    res, off = synth.pack([])
    db = Hm.Database(res, off)
    try:
        r = db.search(b"ACD", Hm.Params(), k=5, n_aln=5)
        assert len(r.hits) == 0
    finally:
        db.close()


# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_full_size_every_score():
    """The full 500,200-target, 300-residue-query workload, in the launch
    configuration the benchmark times: every score, the top 500 and the top-50
    alignments."""
    w = synth.config_full()
    say(f"full workload: {w.n_targets} targets, {w.db_residues} residues")
    db = H().Database(w.residues, w.offsets)
    try:
        q = w.queries[0]
        s, rounds, cells = db.scores(bytes(q))
        say("gpu scores done")
        codes = O.encode_db(w.residues, w.offsets)
        ref, ref_cells = oracle_scores(codes, w.offsets, O.encode(bytes(q)), O.Params())
        say("oracle scores done")
        assert (s == ref).all(), f"{(s != ref).sum()} scores differ"
        assert cells == ref_cells
        r = db.search(bytes(q), H().Params(), k=w.k, n_aln=w.n_aln)
        top = O.rank(ref, w.k)
        assert list(r.hits["target_id"]) == [int(i) for i in top]
        assert list(r.hits["score"]) == [int(ref[i]) for i in top]
        for i in range(w.n_aln):
            tid = int(top[i])
            a = O.align_pair(O.encode(bytes(q)), codes[w.offsets[tid]:w.offsets[tid + 1]], tid,
                             O.Params())
            assert int(r.alns[i]["score"]) == a["score"]
            assert [int(x) for x in r.ops_of(i)] == a["ops"]
    finally:
        db.close()


def test_ranking_fallback_wide_scores():
    """Scores spread wider than the ranking histogram window: 50 exact copies
    of a long query score far above 200 unrelated targets, and k = 100 needs
    ranks below the window (exact radix-select path)."""
    rng = np.random.default_rng(9)
    q = synth.random_protein(rng, 900)
    seqs = [q.copy() for _ in range(50)] + [synth.random_protein(rng, int(n))
                                            for n in rng.integers(100, 400, 200)]
    order = rng.permutation(len(seqs))
    seqs = [seqs[i] for i in order]
    res, off = synth.pack(seqs)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        check_search(db, codes, off, q, H().Params(), k=100, n_aln=60)
        check_search(db, codes, off, q, H().Params(min_score=-500), k=100, n_aln=10)
    finally:
        db.close()


def test_ranking_fallback_many_ties():
    """More tied keys at the k-th score than one workgroup sorts (10,000
    identical targets): exact radix-select path, ties by index."""
    rng = np.random.default_rng(10)
    t = synth.random_protein(rng, 12)
    res, off = synth.pack([t] * 10000)
    q = synth.random_protein(rng, 8)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        p = H().Params(lfactor_q16=65536, minfactor_q16=65536, sfactor_q16=0)
        check_search(db, codes, off, q, p, k=300, n_aln=5)
    finally:
        db.close()
