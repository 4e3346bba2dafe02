"""GPU parity for long sequences: queries of thousands of residues (one
profile copy, fewer wavefronts per workgroup when LDS is short) and targets of
10,000-35,000 residues, and targets of 100,000 to 1,000,000 residues (the
longest accepted).  At the full long-sequence workload the oracle's results
(every pair score, each query's ranking and all its alignments) were stored
by tests/golden/make_golden.py, which calls only the oracle; sampled pairs
are also rescored by the oracle inside the test."""
import concurrent.futures as cf
import hashlib
import json
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
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
long_run_batch = []      # the long workload's batch handle while its fixture lives


def sha_i32(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def sha_u32(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


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
    long_run_batch[:] = [b]
    yield w, codes, db, res, sc, rd
    long_run_batch.clear()
    b.close()
    db.close()


def golden_long():
    return json.load(open(os.path.join(GOLDEN, "long_oracle.json")))


def test_long_every_score_and_ranking(long_run):
    """Every one of the 226,688 pair scores of the long-sequence workload
    against the oracle's (stored by tests/golden/make_golden.py long: a
    SHA-256 of each query's 7,084 scores), and every query's 50 ranks
    (score desc, index asc) against the oracle's ranking."""
    w, codes, db, res, sc, rd = long_run
    gold = golden_long()
    assert gold["n_targets"] == w.n_targets and len(gold["queries"]) == len(w.queries)
    for qi, r in enumerate(res):
        g = gold["queries"][qi]
        assert g["qlen"] == len(w.queries[qi])
        assert sha_i32(sc[qi]) == g["scores_sha256"], f"query {qi}: pair scores differ"
        assert [int(x) for x in r.hits["target_id"]] == g["top_ids"], f"query {qi}: ranking"
        assert [int(x) for x in r.hits["score"]] == g["top_scores"], f"query {qi}: ranked scores"
        assert (r.hits["round"] == 0).all()
    say(f"all {len(res)} x {w.n_targets} pair scores and rankings equal the oracle")


def test_long_cell_count(long_run):
    """The batch kernel's own count of scored residue pairs equals the sum of
    the oracle's counts over every pair."""
    w, codes, db, res, sc, rd = long_run
    import torch
    b = long_run_batch[0]
    cells = torch.zeros(1, dtype=torch.int64, device="cuda")
    b.score(cells)
    torch.cuda.synchronize()
    assert int(cells.cpu()[0]) == sum(q["cells"] for q in golden_long()["queries"])


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
    """All 50 alignments of every query equal the oracle's (stored: target,
    score, op count and a SHA-256 of the run-length ops); the first two of
    every query are also replayed by the oracle here, op by op."""
    w, codes, db, res, sc, rd = long_run
    gold = golden_long()
    for qi, r in enumerate(res):
        g = gold["queries"][qi]["alns"]
        assert len(r.alns) == len(g) == w.n_aln
        for i, (tid, score, n_ops, ops_sha) in enumerate(g):
            a = r.alns[i]
            assert (int(a["target_id"]), int(a["score"]), int(a["n_ops"])) == (tid, score, n_ops), \
                f"query {qi} rank {i}"
            assert sha_u32(r.ops_of(i))[:len(ops_sha)] == ops_sha, f"query {qi} rank {i}: ops"

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


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def very_long():
    """Targets of 100,000 to 1,000,000 letters (HS_MAX_SEQ, the longest
    accepted) beside short ones, with a copy of a query planted in a
    300,000-letter target: windows of hundreds of thousands of letters,
    tens of thousands of blocks per step, 32-bit totals."""
    rng = np.random.default_rng(31337)
    lens = [1_000_000, 500_000, 250_000, 100_000, 300_000, 40, 700, 3]
    seqs = [synth.random_protein(rng, n) for n in lens]
    q1200 = synth.random_protein(rng, 1200)
    seqs[4] = synth.embed(rng, synth.mutate(rng, q1200, 0.8), 300_000)
    res, off = synth.pack(seqs)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    say(f"very long targets: {list(np.diff(off))}")
    yield res, off, codes, db, q1200
    db.close()


def oracle_search_threads(codes, off, q, p, k, n_aln):
    """O.search with the pair scores computed one target per thread."""
    n = len(off) - 1
    with cf.ThreadPoolExecutor(min(16, n)) as ex:
        parts = list(ex.map(lambda i: O.score_all(codes, off, q, p, ids=np.array([i]))[0][0],
                            range(n)))
    scores = np.array(parts, dtype=np.int32)
    top = O.rank(scores, k)

    def aln(tid):
        return O.align_pair(q, codes[off[tid]:off[tid + 1]], int(tid), p)

    with cf.ThreadPoolExecutor(min(16, n)) as ex:
        alns = list(ex.map(aln, [int(t) for t in top[:n_aln]]))
    return scores, top, alns


@pytest.mark.parametrize("qlen", [300, 1200, 5600])
def test_very_long_targets(very_long, qlen):
    """Targets of up to 1,000,000 letters: every pair score, the ranking and
    every alignment equal the oracle, in a one-query search and a batch."""
    res, off, codes, db, q1200 = very_long
    q = q1200 if qlen == 1200 else synth.random_protein(np.random.default_rng(qlen), qlen)
    n = len(off) - 1
    p = H().Params()
    say(f"very long targets, query of {qlen}: oracle")
    scores, top, alns = oracle_search_threads(codes, off, O.encode(bytes(q)), op_params(p), n, n)
    say("device")
    dev, _, cells = db.scores(bytes(q), p)
    assert (dev == scores).all(), list(zip(dev, scores))
    r = db.search(bytes(q), p, k=n, n_aln=n)
    assert [int(x) for x in r.hits["target_id"]] == [int(t) for t in top]
    assert [int(x) for x in r.hits["score"]] == [int(scores[t]) for t in top]
    for i, a in enumerate(alns):
        assert int(r.alns[i]["score"]) == a["score"], f"rank {i}"
        assert [int(x) for x in r.ops_of(i)] == a["ops"], f"rank {i}"
    b = H().Batch(db, 2, qlen, qlen + 7, k=n, n_aln=n)
    b.set([bytes(q), b"MKVLAAG"])
    b.run(graph=True)
    rb = b.results()[0]
    assert (rb.hits == r.hits).all() and (rb.ops == r.ops).all()
    b.close()
