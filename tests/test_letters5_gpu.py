"""The 5-bit letter image (hs_db_set_letters(db, 5)), a measured alternative
to the byte image for the one-query scoring kernel: every pair score, the
work count, the ranking and the alignments equal those of the byte image and
the oracle, on the 2,020-target database, a database of edge lengths (1 to
2,500 letters: short windows of a large target, ragged chunk tails) and the
full 500,200-target workload."""
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


def both_images(db, q, p):
    db.set_letters(8)
    s8, r8, c8 = db.scores(bytes(q), p)
    db.set_letters(5)
    s5, r5, c5 = db.scores(bytes(q), p)
    db.set_letters(8)
    return (s8, r8, c8), (s5, r5, c5)


def test_tiny_database():
    w = synth.config_tiny()
    db = H().Database(w.residues, w.offsets)
    try:
        q = w.queries[0]
        codes = O.encode_db(w.residues, w.offsets)
        for p in (H().Params(), H().Params(pgp=3, rounds=3, seed=77)):
            (s8, r8, c8), (s5, r5, c5) = both_images(db, q, p)
            ref = O.score_all(codes, w.offsets, O.encode(bytes(q)), O.Params(
                gop=p.gop, gep=p.gep, pgp=p.pgp, rounds=p.rounds, seed=p.seed))
            assert (s5 == ref[0]).all() and (r5 == ref[1]).all() and c5 == ref[2]
            assert (s5 == s8).all() and c5 == c8
        db.set_letters(5)
        a = db.search(bytes(q), H().Params(), k=100, n_aln=30)
        db.set_letters(8)
        b = db.search(bytes(q), H().Params(), k=100, n_aln=30)
        assert (a.hits == b.hits).all() and (a.alns == b.alns).all() and (a.ops == b.ops).all()
    finally:
        db.close()


@pytest.mark.parametrize("qlen", [1, 7, 64, 300, 1000])
def test_edge_lengths(qlen):
    rng = np.random.default_rng(500 + qlen)
    lens = list(range(1, 40)) + [63, 64, 65, 127, 128, 129, 300, 1000, 2500]
    seqs = [synth.random_protein(rng, n) for n in lens]
    res, off = synth.pack(seqs)
    codes = O.encode_db(res, off)
    db = H().Database(res, off)
    try:
        q = synth.random_protein(rng, qlen)
        (s8, _, c8), (s5, _, c5) = both_images(db, q, H().Params())
        ref = O.score_all(codes, off, O.encode(bytes(q)), O.Params())
        assert (s5 == ref[0]).all() and c5 == ref[2]
        assert (s8 == s5).all()
    finally:
        db.close()


def test_full_workload():
    w = synth.config_full()
    say(f"full workload, 5-bit letters: {w.n_targets} targets")
    db = H().Database(w.residues, w.offsets)
    try:
        (s8, _, c8), (s5, _, c5) = both_images(db, w.queries[0], H().Params())
        assert c5 == c8
        assert (s5 == s8).all(), f"{(s5 != s8).sum()} scores differ"
    finally:
        db.close()
