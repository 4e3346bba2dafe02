"""GPU tests of the serving loop: queries submitted one at a time, at random
moments and with their own parameters, are searched in continuous batches;
every result equals a separate search of the same query (and the oracle),
whatever batch it landed in."""
import time

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def H():
    import paper_1508_06561_amd as mod
    return mod


def op_params(p):
    return O.Params(gop=p.gop, gep=p.gep, pgp=p.pgp, lfactor_q16=p.lfactor_q16,
                    sfactor_q16=p.sfactor_q16, minfactor_q16=p.minfactor_q16, rounds=p.rounds,
                    seed=p.seed)


@pytest.fixture(scope="module")
def served():
    w = synth.config_serving(200, duration_s=0.25)
    codes = O.encode_db(w.residues, w.offsets)
    db = H().Database(w.residues, w.offsets)
    yield w, codes, db
    db.close()


def drain(srv, n, timeout_s=60):
    got, t0 = [], time.time()
    while len(got) < n and time.time() - t0 < timeout_s:
        got += srv.poll(timeout_ms=100)
    return got


def test_served_results_equal_alone_and_oracle(served):
    w, codes, db = served
    rng = np.random.default_rng(4)
    P = H().Params
    plist = [P(), P(seed=3), P(rounds=2, seed=9), P(pgp=1, gop=4, gep=2), P(min_score=30)]
    srv = H().Server(db, max_batch=16, max_qlen=2000, max_residues=8000, k=w.k, n_aln=w.n_aln)
    queries = [bytes(q) for q in w.queries[:40]]
    params = [plist[i % len(plist)] for i in range(len(queries))]
    for i, (q, p) in enumerate(zip(queries, params)):
        srv.submit(q, tag=1000 + i, params=p)
        time.sleep(float(rng.exponential(0.002)))
    tags = drain(srv, len(queries))
    assert sorted(tags) == [1000 + i for i in range(len(queries))]
    st = srv.stats()
    print(f"served {st}", flush=True)
    assert st["served"] == len(queries) and st["batches"] <= len(queries)
    for tag in tags:
        i = tag - 1000
        r, t = srv.result(tag)
        assert 1 <= t["batch_size"] <= 16 and t["total_ms"] >= t["batch_ms"] > 0
        alone = db.search(queries[i], params[i], k=w.k, n_aln=w.n_aln)
        assert (r.hits == alone.hits).all(), f"query {i}"
        assert (r.alns["score"] == alone.alns["score"]).all() and (r.ops == alone.ops).all()
        if i % 8 == 0:
            ref = O.search(codes, w.offsets, O.encode(queries[i]), op_params(params[i]), k=w.k,
                           n_aln=w.n_aln, min_score=params[i].min_score)
            assert list(r.hits["target_id"]) == [int(x) for x in ref["ids"]]
            for a, (tid, score, ops) in enumerate(ref["alns"]):
                assert [int(x) for x in r.ops_of(a)] == ops
    srv.close()


def test_burst_is_batched_and_admission_bounds(served):
    """A burst submitted at once is served in few batches, each within the
    footprint (count and total letters)."""
    w, codes, db = served
    srv = H().Server(db, max_batch=8, max_qlen=2000, max_residues=3000, k=20, n_aln=5)
    qs = [bytes(q) for q in w.queries[:30]]
    for i, q in enumerate(qs):
        srv.submit(q, tag=i)
    tags = drain(srv, len(qs))
    assert sorted(tags) == list(range(len(qs)))
    sizes = []
    for tag in tags:
        r, t = srv.result(tag)
        sizes.append(t["batch_size"])
        alone = db.search(qs[tag], H().Params(), k=20, n_aln=5)
        assert (r.hits == alone.hits).all() and (r.ops == alone.ops).all()
    assert max(sizes) <= 8
    assert srv.stats()["batches"] < len(qs)
    srv.close()


def test_server_errors_and_shutdown(served):
    w, codes, db = served
    srv = H().Server(db, max_batch=4, max_qlen=100, k=5, n_aln=2)
    with pytest.raises(H().HSError):
        srv.submit(b"A" * 101, tag=1)
    with pytest.raises(H().HSError):
        srv.submit(b"AC-D", tag=1)
    with pytest.raises(H().HSError):
        srv.submit(b"ACD", tag=1, params=H().Params(gop=-3))
    srv.submit(b"ACDEFGHIK", tag=7)
    with pytest.raises(H().HSError):
        srv.submit(b"ACD", tag=7)                 # tag pending or unclaimed
    assert drain(srv, 1) == [7]
    r, _ = srv.result(7)
    assert (r.hits == db.search(b"ACDEFGHIK", H().Params(), k=5, n_aln=2).hits).all()
    with pytest.raises(H().HSError):
        srv.result(7)                             # already claimed
    # shutting down with work still queued returns promptly
    for i in range(50):
        srv.submit(bytes(w.queries[i % len(w.queries)][:100]), tag=100 + i)
    t0 = time.time()
    srv.close()
    assert time.time() - t0 < 30


def test_two_workers_overlap_on_device(served):
    """With two workers, a query submitted while another one's batch is on the
    device starts beside it: of six long queries submitted at once (one query
    per batch), some batches overlap in time, and every result still equals
    a separate search."""
    w, codes, db = served
    rng = np.random.default_rng(11)
    qs = [bytes(synth.random_protein(rng, 1500)) for _ in range(6)]
    srv = H().Server(db, max_batch=1, max_qlen=1500, k=20, n_aln=3, workers=2)
    for i, q in enumerate(qs):
        srv.submit(q, tag=i)
    tags = drain(srv, len(qs))
    assert sorted(tags) == list(range(len(qs)))
    spans = []
    for tag in tags:
        r, t = srv.result(tag)
        assert t["batch_size"] == 1
        start = t["submit_ms"] + t["queue_ms"]
        spans.append((start, start + t["batch_ms"]))
        alone = db.search(qs[tag], H().Params(), k=20, n_aln=3)
        assert (r.hits == alone.hits).all() and (r.ops == alone.ops).all()
    spans.sort()
    overlaps = sum(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    print(f"batch spans (ms): {[(round(a, 2), round(b, 2)) for a, b in spans]}", flush=True)
    assert overlaps >= 1
    assert srv.stats()["batches"] == len(qs)
    srv.close()


def test_lds_class_admission(served):
    """A query too long for four profile copies is not batched with queries
    that keep them: with one worker and a burst short, long, short, the long
    query runs in a batch of its own class; every result still equals a
    separate search."""
    w, codes, db = served
    rng = np.random.default_rng(12)
    short = [bytes(synth.random_protein(rng, int(n))) for n in rng.integers(30, 200, 6)]
    longq = [bytes(synth.random_protein(rng, 1800)), bytes(synth.random_protein(rng, 1900))]
    order = short[:3] + longq + short[3:]
    srv = H().Server(db, max_batch=16, max_qlen=5600, max_residues=30000, k=20, n_aln=5,
                     workers=1)
    # hold the worker on a long first query so that the rest queue up as one burst
    srv.submit(bytes(synth.random_protein(rng, 5600)), tag=99)
    for i, q in enumerate(order):
        srv.submit(q, tag=200 + i)
    tags = drain(srv, len(order) + 1)
    assert len(tags) == len(order) + 1
    sizes = {}
    for tag in tags:
        r, t = srv.result(tag)
        sizes[tag] = t["batch_size"]
        if tag == 99:
            continue
        q = order[tag - 200]
        alone = db.search(q, H().Params(), k=20, n_aln=5)
        assert (r.hits == alone.hits).all() and (r.ops == alone.ops).all()
    # the two long queries were served together, apart from the short ones
    assert sizes[203] == sizes[204] == 2
    assert all(sizes[200 + i] <= 3 for i in (0, 1, 2, 5, 6, 7))
    srv.close()
