"""Threshold reporting (Section IV: the database sequences scoring above a
threshold, ranked) on the GPU against the oracle, bit for bit: every target
at or above min_score in (score descending, index ascending) order with no
cap on the count, the winning rounds, and the alignments of the first ranks.
Cases: thresholds admitting every target, some, none, and more than the
4,096 ranks hs_search can return; score ranges needing one to three radix
passes; ties; the too-small buffer; the device form."""
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


def oracle_scores(codes, off, q, params):
    """(scores, rounds) of every target from the oracle, over a thread pool
    (the C oracle releases the GIL)."""
    n = len(off) - 1
    threads = min(16, os.cpu_count() or 1)
    chunks = np.array_split(np.arange(n, dtype=np.int64), max(1, threads * 4))
    out = np.zeros(n, dtype=np.int32)
    rounds = np.zeros(n, dtype=np.int32)
    single = params.rounds == 1
    with cf.ThreadPoolExecutor(threads) as ex:
        futs = {ex.submit(O.score_all, codes, off, q, params, None, ids): ids for ids in chunks
                if len(ids)}
        for f, ids in futs.items():
            out[ids] = f.result()[0]
    if not single:
        rounds = O.score_all(codes, off, q, params)[1]
    return out, rounds


def check_threshold(db, codes, off, query, p, n_aln=0, ref=None):
    """hs_search_threshold against oracle.rank with k unbounded."""
    q = O.encode(bytes(query))
    if ref is None:
        ref = oracle_scores(codes, off, q, to_oparams(p))
    scores, rounds = ref
    order = O.rank(scores, len(scores), p.min_score)
    r = db.search_threshold(bytes(query), p, n_aln=n_aln)
    assert len(r.hits) == len(order), f"{len(r.hits)} hits, oracle {len(order)}"
    assert np.array_equal(r.hits["target_id"], order.astype(np.int64))
    assert np.array_equal(r.hits["score"], scores[order])
    assert np.array_equal(r.hits["round"], rounds[order])
    na = min(n_aln, len(order))
    assert len(r.alns) == na
    for i in range(na):
        tid = int(order[i])
        a = O.align_pair(q, codes[off[tid]:off[tid + 1]], tid, to_oparams(p))
        assert int(r.alns[i]["target_id"]) == tid and int(r.alns[i]["score"]) == a["score"]
        assert [int(x) for x in r.ops_of(i)] == a["ops"], f"alignment of rank {i}"
    return r, order


@pytest.fixture(scope="module")
def tiny():
    w = synth.config_tiny()
    codes = O.encode_db(w.residues, w.offsets)
    db = H().Database(w.residues, w.offsets)
    q = w.queries[0]
    ref = oracle_scores(codes, w.offsets, O.encode(bytes(q)), O.Params())
    yield w, codes, db, ref
    db.close()


def test_every_target(tiny):
    w, codes, db, ref = tiny
    say("threshold: every target")
    r, order = check_threshold(db, codes, w.offsets, w.queries[0], H().Params(), n_aln=30, ref=ref)
    assert len(order) == w.n_targets


@pytest.mark.parametrize("quantile", [0.0, 0.5, 0.9, 0.999])
def test_thresholds(tiny, quantile):
    w, codes, db, ref = tiny
    thr = int(np.quantile(ref[0], quantile))
    say(f"threshold {thr} (quantile {quantile})")
    check_threshold(db, codes, w.offsets, w.queries[0], H().Params(min_score=thr), n_aln=10,
                    ref=ref)


def test_nothing_reaches(tiny):
    w, codes, db, ref = tiny
    p = H().Params(min_score=int(ref[0].max()) + 1)
    r = db.search_threshold(bytes(w.queries[0]), p, n_aln=5)
    assert len(r.hits) == 0 and len(r.alns) == 0


def test_buffer_too_small(tiny):
    w, codes, db, ref = tiny
    thr = int(np.quantile(ref[0], 0.5))
    n = int((ref[0] >= thr).sum())
    with pytest.raises(H().HSError) as e:
        db.search_threshold(bytes(w.queries[0]), H().Params(min_score=thr), cap=n - 1)
    assert e.value.code == H().hs.HS_ENOSPC
    r = db.search_threshold(bytes(w.queries[0]), H().Params(min_score=thr), cap=n)
    assert len(r.hits) == n


@pytest.mark.parametrize("name,kw", [
    ("wide_range", dict(gop=1000, gep=1000, pgp=1000)),          # scores span > 2^16: 3 passes
    ("rounds3", dict(rounds=3, seed=77, pgp=2)),
    ("narrow", dict(gop=0, gep=0, lfactor_q16=65536, minfactor_q16=65536)),
])
def test_parameter_ranges(tiny, name, kw):
    w, codes, db, _ = tiny
    p = H().Params(**kw)
    say(f"threshold variant {name}")
    r, order = check_threshold(db, codes, w.offsets, w.queries[0], p, n_aln=8)
    if name == "wide_range":
        s = r.hits["score"]
        assert int(s.max()) - int(s.min()) >= 1 << 16


def test_ties_by_index():
    rng = np.random.default_rng(21)
    t = synth.random_protein(rng, 12)
    res, off = synth.pack([t] * 5000 + [synth.random_protein(rng, 30) for _ in range(100)])
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        q = synth.random_protein(rng, 8)
        p = H().Params(lfactor_q16=65536, minfactor_q16=65536, sfactor_q16=0)
        check_threshold(db, codes, off, q, p, n_aln=4)
    finally:
        db.close()


def test_device_form(tiny):
    import torch
    w, codes, db, ref = tiny
    q = bytes(w.queries[0])
    thr = int(np.quantile(ref[0], 0.8))
    p = H().Params(min_score=thr)
    n_ref = int((ref[0] >= thr).sum())
    codes_d = torch.from_numpy(H().encode(q)).cuda()
    ws = torch.empty(db.threshold_workspace_bytes(), dtype=torch.uint8, device="cuda")
    cap = n_ref // 2          # short buffer: the count is still reported
    hits = torch.zeros(cap * 16, dtype=torch.uint8, device="cuda")
    n = torch.zeros(1, dtype=torch.int64, device="cuda")
    db.search_threshold_dev(codes_d, len(q), p, cap, 0, ws, hits, n)
    torch.cuda.synchronize()
    assert int(n.cpu()[0]) == n_ref
    h = np.frombuffer(hits.cpu().numpy().tobytes(), dtype=H().hs.HIT_DTYPE)
    order = O.rank(ref[0], n_ref, thr)
    assert np.array_equal(h["target_id"], order[:cap].astype(np.int64))
    assert np.array_equal(h["score"], ref[0][order[:cap]])


def test_full_size_beyond_max_k():
    """The full 500,200-target workload with thresholds admitting about
    100,000 targets and every target: far beyond hs_search's 4,096 ranks."""
    w = synth.config_full()
    say(f"full workload: {w.n_targets} targets")
    codes = O.encode_db(w.residues, w.offsets)
    db = H().Database(w.residues, w.offsets)
    try:
        q = w.queries[0]
        ref = oracle_scores(codes, w.offsets, O.encode(bytes(q)), O.Params())
        say("oracle scores done")
        thr = int(np.sort(ref[0])[::-1][100_000])
        r, order = check_threshold(db, codes, w.offsets, q, H().Params(min_score=thr), n_aln=20,
                                   ref=ref)
        assert len(order) > 4096
        r, order = check_threshold(db, codes, w.offsets, q, H().Params(), n_aln=0, ref=ref)
        assert len(order) == w.n_targets
    finally:
        db.close()
