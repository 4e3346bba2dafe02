"""GPU parity of the Smith-Waterman-Gotoh baseline (hs_sw_scores_dev): every
score against the oracle's Gotoh checker (itself pinned by exhaustive
enumeration of alignments on tiny inputs), bit for bit, on the tiny database
over ragged query lengths and gap parameters, an asymmetric matrix, the
longest query against long targets (sampled), and the full 500,200-target
database (every score against the oracle's stored score vector, plus the
bound that no heuristic pair score exceeds the optimum, for every target)."""
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

ALPHA = b"ARNDCQEGHILKMFPSTWYVBZX*"
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def H():
    import paper_1508_06561_amd as mod
    return mod


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sw_ref(codes, off, q, ids, gop=10, gep=5, matrix=None):
    """Oracle scores of the query against targets `ids` (C checker, threads)."""
    threads = min(16, os.cpu_count() or 1)
    out = np.zeros(len(ids), dtype=np.int64)

    def one(k):
        t = ids[k]
        out[k] = O.sw_score(q, codes[off[t]:off[t + 1]], gop, gep, matrix)

    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(one, range(len(ids))))
    return out


def query(rng, n, alphabet=ALPHA[:20]):
    return bytes(alphabet[i] for i in rng.integers(0, len(alphabet), size=n))


@pytest.fixture(scope="module")
def tiny():
    w = synth.config_tiny()
    codes = O.encode_db(w.residues, w.offsets)
    db = H().Database(w.residues, w.offsets)
    yield w, codes, db
    db.close()


@pytest.mark.parametrize("qlen", [1, 2, 15, 16, 17, 31, 33, 64, 300, 700, 1000, 1024, 1025, 1100])
def test_tiny_every_score(tiny, qlen):
    """Every target, query lengths around the 16-row pass (ragged last
    pass), lane groups of 1 to 64 lanes sharing a wavefront, and around the
    1,024-row wavefront pass (one pass of 63 or 64 lanes, then two passes)."""
    w, codes, db = tiny
    rng = np.random.default_rng(100 + qlen)
    q = query(rng, qlen, ALPHA)
    say(f"sw tiny qlen {qlen}")
    s = db.sw_scores(q)
    ref = sw_ref(codes, w.offsets, O.encode(q), np.arange(w.n_targets))
    assert (s == ref).all(), f"{(s != ref).sum()} scores differ"


@pytest.mark.parametrize("gop,gep", [(0, 0), (1, 1), (11, 1), (3, 7), (1000, 1000)])
def test_gap_parameters(tiny, gop, gep):
    w, codes, db = tiny
    rng = np.random.default_rng(7 * gop + gep)
    q = query(rng, 120)
    say(f"sw gaps {gop} {gep}")
    s = db.sw_scores(q, H().Params(gop=gop, gep=gep))
    ref = sw_ref(codes, w.offsets, O.encode(q), np.arange(w.n_targets), gop, gep)
    assert (s == ref).all(), f"{(s != ref).sum()} scores differ"


def test_asymmetric_matrix(tiny):
    """A matrix that is not symmetric: the query indexes rows, the target columns."""
    w, codes, db = tiny
    rng = np.random.default_rng(31)
    m = rng.integers(-6, 10, size=(24, 24)).astype(np.int8)
    q = query(rng, 90, ALPHA)
    s = db.sw_scores(q, H().Params(matrix=m))
    ref = sw_ref(codes, w.offsets, O.encode(q), np.arange(w.n_targets), matrix=m)
    assert (s == ref).all(), f"{(s != ref).sum()} scores differ"
    mt = np.ascontiguousarray(m.T)
    assert not (db.sw_scores(q, H().Params(matrix=mt)) == s).all()


def test_longest_query_long_targets():
    """The longest accepted query (5,600 letters: a 134 KB profile in LDS)
    against the long-sequence database; sampled targets, among them the
    longest and the shortest."""
    w = synth.config_long()
    codes = O.encode_db(w.residues, w.offsets)
    lens = np.diff(w.offsets)
    order = np.argsort(-lens, kind="stable")
    rng = np.random.default_rng(5)
    ids = np.unique(np.concatenate([order[:3], order[-3:], rng.choice(w.n_targets, 6, replace=False)]))
    q = bytes(synth.random_protein(rng, 5600))
    db = H().Database(w.residues, w.offsets)
    try:
        say("sw longest query")
        s = db.sw_scores(q)
        ref = sw_ref(codes, w.offsets, O.encode(q), ids)
        assert (s[ids] == ref).all(), list(zip(ids, s[ids], ref))
        # a planted homolog of query 0 scores far above random long targets
        s0 = db.sw_scores(bytes(w.queries[0]))
        planted = [t for t in w.planted if t >= 0][:2]
        say(f"planted {planted}: {s0[planted]}, median {np.median(s0)}")
        ref0 = sw_ref(codes, w.offsets, O.encode(bytes(w.queries[0])), np.array(planted))
        assert (s0[planted] == ref0).all()
    finally:
        db.close()


def test_full_size_every_score_and_bound():
    """The full 500,200-target database with the 300-residue query: every
    one of the 500,200 scores against the oracle's (stored by
    tests/golden/make_golden.py sw_full: SHA-256 of the whole score vector,
    its sum and the 500 best), a sample rescored by the oracle here, and for
    every target the bound that the heuristic's pair score never exceeds the
    local optimum (its alignment, with end gaps removed, is one of the
    alignments the optimum ranges over)."""
    gold = json.load(open(os.path.join(GOLDEN, "sw_full_oracle.json")))
    w = synth.config_full()
    assert w.n_targets == gold["n_targets"]
    db = H().Database(w.residues, w.offsets)
    try:
        q = bytes(w.queries[0])
        sw = db.sw_scores(q)
        say("gpu sw scores done")
        top = O.rank(sw, len(gold["top_ids"]))
        assert [int(i) for i in top] == gold["top_ids"]
        assert [int(sw[i]) for i in top] == gold["top_scores"]
        assert int(sw.astype(np.int64).sum()) == gold["score_sum"]
        assert hashlib.sha256(np.ascontiguousarray(sw, dtype="<i4").tobytes()).hexdigest() == \
            gold["scores_sha256"], "the score vector differs from the oracle's"
        heur, _, _ = db.scores(q)
        assert (sw >= heur).all(), f"{(sw < heur).sum()} targets above the optimum"
        assert (sw >= 0).all()
        codes = O.encode_db(w.residues, w.offsets)
        lens = np.diff(w.offsets)
        rng = np.random.default_rng(11)
        ids = np.unique(np.concatenate([np.argsort(-lens, kind="stable")[:8],
                                        np.asarray(w.planted[:40]),
                                        rng.choice(w.n_targets, 100, replace=False)]))
        ref = sw_ref(codes, w.offsets, O.encode(q), ids)
        say("oracle sample done")
        assert (sw[ids] == ref).all(), f"{(sw[ids] != ref).sum()} sampled scores differ"
    finally:
        db.close()


def test_errors(tiny):
    w, codes, db = tiny
    import torch
    lib = H()
    codes_d = torch.zeros(8, dtype=torch.uint8, device="cuda")
    out = torch.zeros(w.n_targets, dtype=torch.int32, device="cuda")
    ws = torch.empty(db.sw_workspace_bytes(), dtype=torch.uint8, device="cuda")
    p = lib.Params()
    with pytest.raises(lib.HSError):
        db.sw_scores_dev(codes_d, 0, p, ws, out)
    with pytest.raises(lib.HSError):
        db.sw_scores_dev(codes_d, 5601, p, ws, out)
    with pytest.raises(lib.HSError):
        db.sw_scores_dev(codes_d, 8, p, ws[:16], out)
    with pytest.raises(lib.HSError):
        db.sw_scores_dev(codes_d, 8, lib.Params(gop=-1), ws, out)
    # all-A query of 8 letters (code 0): the same as the oracle
    db.sw_scores_dev(codes_d, 8, p, ws, out)
    ref = sw_ref(codes, w.offsets, np.zeros(8, dtype=np.uint8), np.arange(w.n_targets))
    assert (out.cpu().numpy() == ref).all()
