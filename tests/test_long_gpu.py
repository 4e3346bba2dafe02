"""GPU parity for long sequences: queries of thousands of residues (one
profile copy, fewer wavefronts per workgroup when LDS is short) and targets of
10,000-35,000 residues.  At the full long-sequence workload the oracle cannot
score every pair within a test, so it checks sampled outputs one by one:
pair scores of planted, long, short and top-ranked targets, the alignments of
the best hits, and the ranking against the device's own scores."""
import concurrent.futures as cf
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


def op_params(p):
    return O.Params(gop=p.gop, gep=p.gep, pgp=p.pgp, lfactor_q16=p.lfactor_q16,
                    sfactor_q16=p.sfactor_q16, minfactor_q16=p.minfactor_q16, rounds=p.rounds,
                    seed=p.seed)


def check_full(r, codes, off, q, p, k, n_aln):
    ref = O.search(codes, off, O.encode(bytes(q)), op_params(p), k=k, n_aln=n_aln,
                   min_score=p.min_score)
    assert list(r.hits["target_id"]) == [int(i) for i in ref["ids"]]
    assert list(r.hits["score"]) == [int(s) for s in ref["scores"]]
    assert len(r.alns) == len(ref["alns"])
    for i, (tid, score, ops) in enumerate(ref["alns"]):
        assert int(r.alns[i]["target_id"]) == tid
        assert int(r.alns[i]["score"]) == score
        assert [int(x) for x in r.ops_of(i)] == ops, f"alignment of rank {i}"


@pytest.fixture(scope="module")
def small():
    q, res, off, planted = synth.tiny_db(seed=21, n_bg=150, qlen=64, n_hom=4)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    yield res, off, codes, db
    db.close()


@pytest.mark.parametrize("qlen", [1300, 4000, 5600])
def test_long_query_full_parity(small, qlen):
    """One long query (5,600 = the longest accepted) against a small
    database: every rank and alignment equals the oracle."""
    res, off, codes, db = small
    rng = np.random.default_rng(qlen)
    q = synth.random_protein(rng, qlen)
    say(f"query of {qlen}")
    r = db.search(bytes(q), H().Params(), k=40, n_aln=10)
    check_full(r, codes, off, q, H().Params(), 40, 10)


@pytest.mark.parametrize("qlen", [500, 1000, 1200])
def test_four_copy_one_workgroup_parity(small, qlen):
    """Queries of 450-1,200 letters keep four profile copies but leave LDS
    for one workgroup per compute unit, so the launch takes the high-ILP
    letter loop: every rank and alignment equals the oracle."""
    res, off, codes, db = small
    rng = np.random.default_rng(1000 + qlen)
    q = synth.random_protein(rng, qlen)
    say(f"query of {qlen}")
    r = db.search(bytes(q), H().Params(), k=40, n_aln=10)
    check_full(r, codes, off, q, H().Params(), 40, 10)


def test_four_copy_batch_parity(small):
    """A batch of 460-1,200-letter queries with four profile copies
    requested: one workgroup fits per compute unit, the batch kernel takes
    the high-ILP letter loop, and every query equals the oracle."""
    res, off, codes, db = small
    rng = np.random.default_rng(4242)
    qs = [synth.random_protein(rng, n) for n in (460, 700, 1000, 1200, 512)]
    b = H().Batch(db, len(qs), 1200, sum(map(len, qs)), k=30, n_aln=8)
    b.set([bytes(q) for q in qs])
    b.schedule(4, 0, 0)
    say(f"schedule {b.get_schedule()}")
    assert b.get_schedule()["copies"] == 4
    b.run(graph=True)
    for q, r in zip(qs, b.results()):
        check_full(r, codes, off, q, H().Params(), 30, 8)
    b.close()


def test_mixed_lengths_batch(small):
    """One batch holding the longest and shortest queries: the launch is laid
    out for the longest, every query still equals the oracle."""
    res, off, codes, db = small
    rng = np.random.default_rng(77)
    qs = [synth.random_protein(rng, n) for n in (5600, 30, 1000, 2, 4999, 300)]
    b = H().Batch(db, len(qs), 5600, sum(map(len, qs)), k=30, n_aln=8)
    b.set([bytes(q) for q in qs])
    say(f"schedule {b.get_schedule()}")
    b.run(graph=True)
    for q, r in zip(qs, b.results()):
        check_full(r, codes, off, q, H().Params(), 30, 8)
    b.close()


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def long_run():
    w = synth.config_long()
    codes = O.encode_db(w.residues, w.offsets)
    say(f"long workload: {len(w.queries)} queries, {w.n_targets} targets, {w.db_residues} residues")
    db = H().Database(w.residues, w.offsets)
    qs = [bytes(q) for q in w.queries]
    b = H().Batch(db, len(qs), max(map(len, qs)), sum(map(len, qs)), k=w.k, n_aln=w.n_aln)
    b.set(qs)
    say(f"schedule {b.get_schedule()}")
    b.run()
    res = b.results()
    sc, rd = b.scores()
    say("batch done")
    yield w, codes, db, res, sc, rd
    b.close()
    db.close()


def test_long_ranking_consistent(long_run):
    """Every query's ranked list is the exact (score desc, index asc) order of
    the device's pair scores, and every hit's round is the stored one."""
    w, codes, db, res, sc, rd = long_run
    for qi, r in enumerate(res):
        ref = O.rank(sc[qi], w.k)
        assert list(r.hits["target_id"]) == [int(i) for i in ref]
        assert list(r.hits["score"]) == [int(sc[qi][i]) for i in ref]
        assert (r.hits["round"] == 0).all()


def test_long_sampled_pair_scores(long_run):
    """Pair scores against the oracle for each query's planted homologs, its
    best hits and random long and short targets."""
    w, codes, db, res, sc, rd = long_run
    rng = np.random.default_rng(5)
    n_short = 2020
    jobs = []
    for qi, q in enumerate(w.queries):
        ids = set(int(x) for x in w.planted[2 * qi:2 * qi + 2])
        ids |= set(int(x) for x in res[qi].hits["target_id"][:3])
        ids |= set(int(x) for x in rng.integers(n_short, w.n_targets, size=3))
        ids |= set(int(x) for x in rng.integers(0, n_short, size=3))
        jobs.append((qi, np.array(sorted(ids), dtype=np.int64)))

    def run(job):
        qi, ids = job
        s, _, _ = O.score_all(codes, w.offsets, O.encode(bytes(w.queries[qi])), O.Params(), ids=ids)
        return qi, ids, s

    with cf.ThreadPoolExecutor(16) as ex:
        for qi, ids, s in ex.map(run, jobs):
            assert (sc[qi][ids] == s).all(), f"query {qi}: targets {ids[sc[qi][ids] != s]}"
    say(f"{sum(len(j[1]) for j in jobs)} sampled pairs equal the oracle")


def test_long_alignments(long_run):
    """The first alignments of every query equal the oracle's replay of the
    same (query, target) pair."""
    w, codes, db, res, sc, rd = long_run

    def run(qi):
        q = O.encode(bytes(w.queries[qi]))
        out = []
        for i in range(2):
            tid = int(res[qi].alns[i]["target_id"])
            t = codes[w.offsets[tid]:w.offsets[tid + 1]]
            out.append((i, tid, O.align_pair(q, t, target_id=tid)))
        return qi, out

    with cf.ThreadPoolExecutor(16) as ex:
        for qi, out in ex.map(run, range(len(w.queries))):
            r = res[qi]
            for i, tid, ref in out:
                assert int(r.alns[i]["score"]) == ref["score"], f"query {qi} rank {i}"
                assert [int(x) for x in r.ops_of(i)] == ref["ops"], f"query {qi} rank {i}"
    # planted homologs of the longest queries rank first
    top = sum(int(res[qi].hits["target_id"][0]) in set(int(x) for x in w.planted[2 * qi:2 * qi + 2])
              for qi in range(len(w.queries)))
    say(f"planted homolog ranked first for {top} of {len(w.queries)} queries")


def test_long_batch_equals_single_search(long_run):
    """Two long queries searched alone give the batch's results."""
    w, codes, db, res, sc, rd = long_run
    for qi in (0, 4):
        r = db.search(bytes(w.queries[qi]), H().Params(), k=w.k, n_aln=w.n_aln)
        assert (r.hits == res[qi].hits).all()
        assert (r.ops == res[qi].ops).all()
        assert (r.alns["score"] == res[qi].alns["score"]).all()
