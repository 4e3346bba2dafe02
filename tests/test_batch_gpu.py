"""GPU parity of batches: a batch of queries scored in one persistent launch
must give, for every query, exactly what a separate search gives -- and both
must equal the oracle -- whatever the schedule, the batch composition, the
per-query parameters, or whether the run is replayed from a captured graph."""
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


def to_oparams(p):
    return O.Params(gop=p.gop, gep=p.gep, pgp=p.pgp, lfactor_q16=p.lfactor_q16,
                    sfactor_q16=p.sfactor_q16, minfactor_q16=p.minfactor_q16, rounds=p.rounds,
                    seed=p.seed)


def oracle_search(codes, off, q, p, k, n_aln, matrix=None):
    return O.search(codes, off, O.encode(bytes(q)), to_oparams(p), k=k, n_aln=n_aln,
                    min_score=p.min_score, matrix=matrix)


def same_result(r, ref, what):
    """A Result against an oracle search dict, bit for bit."""
    assert list(r.hits["target_id"]) == [int(i) for i in ref["ids"]], what
    assert list(r.hits["score"]) == [int(s) for s in ref["scores"]], what
    assert list(r.hits["round"]) == [int(ref["rounds"][i]) for i in ref["ids"]], what
    assert len(r.alns) == len(ref["alns"]), what
    for i, (tid, score, ops) in enumerate(ref["alns"]):
        assert int(r.alns[i]["target_id"]) == tid, what
        assert int(r.alns[i]["score"]) == score, what
        assert [int(x) for x in r.ops_of(i)] == ops, f"{what}: alignment of rank {i}"


def same_results(a, b, what):
    """Two Results, bit for bit."""
    assert (a.hits == b.hits).all(), what
    assert len(a.alns) == len(b.alns), what
    for i in range(len(a.alns)):
        assert a.alns[i]["target_id"] == b.alns[i]["target_id"], what
        assert a.alns[i]["score"] == b.alns[i]["score"], what
        assert (a.ops_of(i) == b.ops_of(i)).all(), f"{what}: alignment {i}"


def oracle_all(codes, off, queries, params, k, n_aln, threads=16):
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = [ex.submit(oracle_search, codes, off, q, p, k, n_aln)
                for q, p in zip(queries, params)]
        return [f.result() for f in futs]


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def batched():
    w = synth.config_batched()
    codes = O.encode_db(w.residues, w.offsets)
    say(f"batched workload: {len(w.queries)} queries, {w.n_targets} targets")
    db = H().Database(w.residues, w.offsets)
    yield w, codes, db
    db.close()


@pytest.fixture(scope="module")
def batched_oracle(batched):
    w, codes, db = batched
    p = H().Params()
    ref = oracle_all(codes, w.offsets, w.queries, [p] * len(w.queries), w.k, w.n_aln)
    say("oracle done for the batched workload")
    return ref


def test_batched_workload_equals_oracle(batched, batched_oracle):
    """All 256 queries in one batch: ranking and alignments of every query,
    and every pair score, equal the oracle."""
    w, codes, db = batched
    b = H().Batch(db, len(w.queries), 1000, sum(len(q) for q in w.queries), k=w.k, n_aln=w.n_aln)
    b.set([bytes(q) for q in w.queries])
    say(f"schedule {b.get_schedule()}")
    b.run()
    res = b.results()
    for qi, (r, ref) in enumerate(zip(res, batched_oracle)):
        same_result(r, ref, f"query {qi} (length {len(w.queries[qi])})")
    sc, rd = b.scores()
    for qi, ref in enumerate(batched_oracle):
        assert (sc[qi] == ref["all_scores"]).all(), f"query {qi}: {(sc[qi] != ref['all_scores']).sum()} scores"
        assert (rd[qi] == 0).all()
    b.close()


def test_batch_equals_separate_searches(batched):
    w, codes, db = batched
    qs = [bytes(q) for q in w.queries[:24]]
    res = H().search_batch(db, qs, H().Params(), k=w.k, n_aln=w.n_aln)
    for qi, q in enumerate(qs):
        same_results(res[qi], db.search(q, H().Params(), k=w.k, n_aln=w.n_aln), f"query {qi}")


SCHEDULES = [(1, 64, 0), (4, 64, 0), (4, 16, 64), (1, 32, 128), (4, 64, 2048), (4, 1, 64)]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[f"c{a}_cap{b}_chunk{c}" for a, b, c in SCHEDULES])
def test_schedule_invariance(batched, batched_oracle, sched):
    w, codes, db = batched
    sel = list(range(0, len(w.queries), 8))          # 32 queries of every length
    qs = [bytes(w.queries[i]) for i in sel]
    b = H().Batch(db, len(qs), 1000, sum(map(len, qs)), k=w.k, n_aln=w.n_aln)
    b.schedule(*sched)
    b.set(qs)
    got = b.get_schedule()
    say(f"schedule {got}")
    assert got["copies"] == sched[0] and got["cap"] == sched[1]
    b.run()
    for r, i in zip(b.results(), sel):
        same_result(r, batched_oracle[i], f"query {i} under {sched}")
    b.close()


# (queries, schedule, expected LDS record kind): beside the four-copy
# profile of the 32 queries of every length (up to 1,000 letters, about
# 100 KB) one workgroup of eight full records fits per compute unit, so
# they run the smaller records (sixteen wavefronts), of 64 slots at 64
# pairs in flight and of 16 slots at 16; with one copy (25 KB), or with
# queries of at most 300 letters, two full workgroups fit and the full
# records stay.
RECORD_CASES = [("every length", (4, 64, 0), 2), ("every length", (4, 16, 64), 1),
                ("every length", (1, 64, 0), 0), ("at most 300", (4, 64, 0), 0),
                ("at most 300", (4, 8, 128), 0)]


@pytest.mark.parametrize("case", RECORD_CASES,
                         ids=[f"{q.split()[-1]}_c{s[0]}_cap{s[1]}_rec{r}" for q, s, r in RECORD_CASES])
def test_record_kinds(batched, batched_oracle, case):
    """Each per-wavefront LDS record kind of the batch kernel runs in one of
    these launches, and every query still equals the oracle."""
    which, sched, rec = case
    w, codes, db = batched
    if which == "every length":
        sel = list(range(0, len(w.queries), 8))
    else:
        sel = [i for i in range(len(w.queries)) if len(w.queries[i]) <= 300][:32]
    qs = [bytes(w.queries[i]) for i in sel]
    b = H().Batch(db, len(qs), 1000, sum(map(len, qs)), k=w.k, n_aln=w.n_aln)
    b.schedule(*sched)
    b.set(qs)
    launch = b.get_launch()
    say(f"{which} {sched}: schedule {b.get_schedule()}, launch {launch}")
    assert launch["record"] == rec and launch["one_pair"] == 0
    b.run()
    for r, i in zip(b.results(), sel):
        same_result(r, batched_oracle[i], f"query {i} under {sched}, record {rec}")
    b.close()


def test_graph_replays(batched, batched_oracle):
    """The captured graph, replayed several times with other work on the
    stream in between, gives the eager result every time."""
    import torch
    w, codes, db = batched
    sel = list(range(3, len(w.queries), 16))
    qs = [bytes(w.queries[i]) for i in sel]
    b = H().Batch(db, len(qs), 1000, sum(map(len, qs)), k=w.k, n_aln=w.n_aln)
    b.set(qs)
    b.run()
    eager = b.results()
    x = torch.zeros(1 << 20, device="cuda")
    for rep in range(4):
        b.run(graph=True)
        x.add_(1.0)                      # unrelated eager work between replays
        got = b.results()
        for j, (r, e) in enumerate(zip(got, eager)):
            same_results(r, e, f"replay {rep}, query {sel[j]}")
    torch.cuda.synchronize()
    assert float(x[0]) == 4.0
    for r, i in zip(eager, sel):
        same_result(r, batched_oracle[i], f"query {i}")
    # a new query set invalidates the graph; the next replay uses it
    b.set(qs[:3])
    b.run(graph=True)
    for r, i in zip(b.results(), sel[:3]):
        same_result(r, batched_oracle[i], f"query {i} after a new set")
    b.close()


def test_tuner_keeps_results(batched, batched_oracle):
    w, codes, db = batched
    sel = list(range(5, len(w.queries), 4))
    qs = [bytes(w.queries[i]) for i in sel]
    b = H().Batch(db, len(qs), 1000, sum(map(len, qs)), k=w.k, n_aln=w.n_aln)
    b.set(qs)
    ms = b.tune(reps=1)
    say(f"tuned schedule {b.get_schedule()} at {ms:.3f} ms")
    assert ms > 0
    b.run()
    for r, i in zip(b.results(), sel):
        same_result(r, batched_oracle[i], f"query {i} after tuning")
    b.close()


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small():
    q, res, off, planted = synth.tiny_db(seed=11, n_bg=300, qlen=90, n_hom=8)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    yield q, res, off, codes, db
    db.close()


def test_per_query_parameters(small):
    """Each query of one batch with its own parameters: seeds (with and
    without the shared draw table), rounds, penalties, factors, matrix and
    threshold; each equals the oracle with those parameters."""
    q0, res, off, codes, db = small
    rng = np.random.default_rng(3)
    m = O.blosum62().astype(np.int16)
    m2 = np.clip(m + rng.integers(-1, 2, size=m.shape), -4, 11).astype(np.int8)
    m2 = ((m2.astype(np.int16) + m2.T) // 2).astype(np.int8)
    P = H().Params
    plist = [P(), P(seed=7), P(rounds=3, seed=7), P(pgp=2, gop=3, gep=1, seed=0),
             P(lfactor_q16=65536, sfactor_q16=32768), P(matrix=m2, seed=5),
             P(min_score=40), P(rounds=2, seed=2**63 + 1)]
    queries = [bytes(q0)] + [bytes(synth.random_protein(rng, int(n)))
                             for n in rng.integers(1, 400, size=len(plist) - 1)]
    queries[3] = bytes(synth.mutate(rng, q0, 0.6))
    res_b = H().search_batch(db, queries, plist, k=40, n_aln=20)
    for i, (q, p) in enumerate(zip(queries, plist)):
        ref = O.search(codes, off, O.encode(q), to_oparams(p), k=40, n_aln=20,
                       min_score=p.min_score, matrix=p.matrix)
        same_result(res_b[i], ref, f"query {i} with {p}")


def test_asymmetric_matrix_in_batch(small):
    """Queries of one batch with a matrix that is not symmetric (and its
    transpose, and the built-in one) equal the oracle."""
    q0, res, off, codes, db = small
    rng = np.random.default_rng(38)
    m = rng.integers(-5, 11, size=(24, 24)).astype(np.int8)
    qs = [bytes(synth.random_protein(rng, int(n))) for n in (40, 120, 260, 480)]
    ps = [H().Params(matrix=m), H().Params(matrix=np.ascontiguousarray(m.T)),
          H().Params(matrix=m, seed=3), H().Params()]
    got = H().search_batch(db, qs, ps, k=50, n_aln=10)
    for i, (q, p) in enumerate(zip(qs, ps)):
        ref = oracle_search(codes, off, q, p, k=50, n_aln=10, matrix=p.matrix)
        same_result(got[i], ref, f"query {i}")


def test_edge_batches(small):
    q0, res, off, codes, db = small
    rng = np.random.default_rng(8)
    P = H().Params()
    # single queries of edge lengths, and a batch of them with duplicates
    qs = [bytes(synth.random_protein(rng, n)) for n in (1, 2, 7, 8, 9, 63, 64, 65)]
    qs += [qs[3], bytes(q0), qs[0]]
    for q in (qs[0], qs[4]):
        r = H().search_batch(db, [q], P, k=10, n_aln=10)[0]
        same_result(r, O.search(codes, off, O.encode(q), to_oparams(P), k=10, n_aln=10), "single")
    rb = H().search_batch(db, qs, P, k=25, n_aln=25)
    for i, q in enumerate(qs):
        same_result(rb[i], O.search(codes, off, O.encode(q), to_oparams(P), k=25, n_aln=25),
                    f"query {i} (length {len(q)})")
    # nothing eligible: a threshold above every score
    r = H().search_batch(db, qs[:3], H().Params(min_score=10**6), k=5, n_aln=5)
    assert all(len(x.hits) == 0 and len(x.alns) == 0 for x in r)
    # no alignments asked for
    r = H().search_batch(db, qs[:3], P, k=5, n_aln=0)
    for i in range(3):
        ref = O.search(codes, off, O.encode(qs[i]), to_oparams(P), k=5, n_aln=0)
        assert list(r[i].hits["target_id"]) == [int(x) for x in ref["ids"]]


def test_handle_reuse_and_errors(small):
    q0, res, off, codes, db = small
    rng = np.random.default_rng(9)
    P = H().Params()
    b = H().Batch(db, 6, 200, 600, k=10, n_aln=4)
    with pytest.raises(H().HSError):
        b.run()                                   # no queries yet
    with pytest.raises(H().HSError):
        b.set([b"A" * 201])                       # longer than max_qlen
    with pytest.raises(H().HSError):
        b.set([b"ACD"] * 7)                       # more than max_nq
    with pytest.raises(H().HSError):
        b.set([b"A" * 200] * 4)                   # more than max_residues
    with pytest.raises(H().HSError):
        b.set([b"AC-D"])                          # outside the alphabet
    with pytest.raises(H().HSError):
        b.schedule(copies=2)
    with pytest.raises(H().HSError):
        b.schedule(chunk=100)
    for rep, n in enumerate((6, 2, 5)):
        qs = [bytes(synth.random_protein(rng, int(L))) for L in rng.integers(5, 120, size=n)]
        b.set(qs, P)
        b.run(graph=rep == 2)
        got = b.results()
        assert len(got) == n
        for i, q in enumerate(qs):
            same_result(got[i], O.search(codes, off, O.encode(q), to_oparams(P), k=10, n_aln=4),
                        f"set {rep}, query {i}")
    b.close()


def test_one_pair_paths_equal_oracle_and_slots(small):
    """A one-query batch on a small database is scored one pair per
    wavefront (k_score_one) and aligned one hit per wavefront; with every
    parameter family it equals the oracle, and a fixed schedule (the slot
    paths) gives the same results."""
    q0, res, off, codes, db = small
    rng = np.random.default_rng(21)
    P = H().Params
    m = O.blosum62().astype(np.int16)
    m2 = np.clip(m + rng.integers(-1, 2, size=m.shape), -4, 11).astype(np.int8)
    m2 = ((m2.astype(np.int16) + m2.T) // 2).astype(np.int8)
    plist = [P(), P(rounds=3, seed=9), P(pgp=2, gop=3, gep=1), P(matrix=m2), P(min_score=30)]
    queries = [bytes(q0), bytes(synth.mutate(rng, q0, 0.5)), bytes(synth.random_protein(rng, 250))]
    for qi, q in enumerate(queries):
        for p in plist:
            b = H().Batch(db, 1, 400, 400, k=30, n_aln=15)
            b.set([q], p)
            sched = b.get_schedule()
            assert sched["cap"] == 1, f"one-pair mode not chosen: {sched}"
            b.run()
            got = b.results()[0]
            ref = O.search(codes, off, O.encode(q), to_oparams(p), k=30, n_aln=15,
                           min_score=p.min_score, matrix=p.matrix)
            same_result(got, ref, f"query {qi} with {p}")
            b.schedule(4, 64, 64)
            b.run()
            same_results(b.results()[0], got, f"query {qi} with {p}, slot paths")
            b.close()
