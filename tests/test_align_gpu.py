"""Pairwise alignment mode (Fig. 1 as written: every placement of the small
window with at least one overlapping letter, best of Rounds rounds) on the
GPU against the oracle, bit for bit: score, winning round and every
run-length op, at Rounds = 20 (the setting of the paper's alignment tests,
Section V) and other parameter sets, on pairs from one letter up to the
longest accepted length (5,600 letters each)."""
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


def oparams(p):
    return O.Params(gop=p.gop, gep=p.gep, pgp=p.pgp, lfactor_q16=p.lfactor_q16,
                    sfactor_q16=p.sfactor_q16, minfactor_q16=p.minfactor_q16, rounds=p.rounds,
                    seed=p.seed, full_slide=True)


def oracle_pairs(pairs, p):
    """Oracle results of every pair (pair i keyed by i), over a thread pool."""
    op = oparams(p)

    def one(i):
        q, t = pairs[i]
        return O.align_pair(O.encode(bytes(q)), O.encode(bytes(t)), i, op)

    with cf.ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, range(len(pairs))))


def check_pairs(pairs, p):
    got = H().align_batch(pairs, p)
    ref = oracle_pairs(pairs, p)
    assert len(got) == len(pairs)
    for i, (g, r) in enumerate(zip(got, ref)):
        assert (g.score, g.round) == (r["score"], r["round"]), f"pair {i} ({len(pairs[i][0])} x {len(pairs[i][1])})"
        assert [int(x) for x in g.ops] == r["ops"], f"ops of pair {i}"
    return got


def rand_pairs(rng, n, lo, hi):
    return [(synth.random_protein(rng, int(rng.integers(lo, hi + 1))),
             synth.random_protein(rng, int(rng.integers(lo, hi + 1)))) for _ in range(n)]


VARIANTS = {
    "defaults": dict(),
    "section_b1_factors": dict(lfactor_q16=65536, sfactor_q16=32768),
    "periphery": dict(pgp=3, seed=5),
    "cheap_gaps": dict(gop=1, gep=0, pgp=1, seed=99),
    "big_penalties": dict(gop=1000, gep=1000, pgp=1000, seed=2**63 + 5),
    "small_windows": dict(lfactor_q16=8192, minfactor_q16=65536, sfactor_q16=65536, seed=3),
    "zero_factors": dict(lfactor_q16=0, sfactor_q16=0, minfactor_q16=0),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_random_pairs_rounds20(name):
    rng = np.random.default_rng(40 + list(VARIANTS).index(name))
    p = H().Params(rounds=20, **VARIANTS[name])
    pairs = rand_pairs(rng, 60, 1, 300)
    say(f"pairwise {name}: {len(pairs)} pairs, Rounds 20")
    check_pairs(pairs, p)


@pytest.mark.parametrize("rounds", [1, 2])
def test_few_rounds(rounds):
    """Rounds = 1 (each round's workgroup writes its ops in the same pass)
    and Rounds = 2 (the second finisher replays the better round)."""
    rng = np.random.default_rng(50 + rounds)
    pairs = rand_pairs(rng, 80, 1, 400)
    for _ in range(20):
        q = synth.random_protein(rng, int(rng.integers(50, 400)))
        pairs.append((q, synth.embed(rng, synth.mutate(rng, q, rng.uniform(0.3, 0.9)),
                                     int(rng.integers(len(q), 600)))))
    say(f"pairwise: {len(pairs)} pairs, Rounds {rounds}")
    check_pairs(pairs, H().Params(rounds=rounds, seed=rounds))
    L = H().hs.MAX_ALIGN
    check_pairs([(synth.random_protein(rng, L), synth.random_protein(rng, L - 7))],
                H().Params(rounds=rounds, seed=9))


def test_asymmetric_matrix():
    """A matrix that is not symmetric scores query letters (rows) against
    target letters (columns), whichever sequence is the large one."""
    rng = np.random.default_rng(37)
    m = rng.integers(-5, 11, size=(24, 24)).astype(np.int8)
    pairs = rand_pairs(rng, 60, 1, 300)
    p = H().Params(rounds=20, matrix=m, seed=2)
    got = H().align_batch(pairs, p)
    op = oparams(p)
    for i, ((q, t), g) in enumerate(zip(pairs, got)):
        r = O.align_pair(O.encode(bytes(q)), O.encode(bytes(t)), i, op, matrix=m)
        assert (g.score, g.round) == (r["score"], r["round"]), f"pair {i} ({len(q)} x {len(t)})"
        assert [int(x) for x in g.ops] == r["ops"], f"ops of pair {i}"


def test_homologs_rounds20():
    """Mutated copies with indels (the paper's distant-homology use)."""
    rng = np.random.default_rng(31)
    pairs = []
    for _ in range(40):
        q = synth.random_protein(rng, int(rng.integers(50, 400)))
        t = synth.embed(rng, synth.mutate(rng, q, rng.uniform(0.2, 0.9)), int(rng.integers(len(q), 600)))
        pairs.append((q, t))
    check_pairs(pairs, H().Params(rounds=20))


def test_edge_lengths():
    rng = np.random.default_rng(32)
    lens = [(1, 1), (1, 2), (2, 1), (1, 300), (300, 1), (7, 7), (64, 64), (65, 63), (255, 257)]
    pairs = [(synth.random_protein(rng, a), synth.random_protein(rng, b)) for a, b in lens]
    pairs.append((np.frombuffer(b"JOUBZX*ACD", np.uint8), np.frombuffer(b"XXBZUOJ*", np.uint8)))
    check_pairs(pairs, H().Params(rounds=20, seed=11))
    check_pairs(pairs, H().Params(rounds=3, pgp=2, seed=12))


def test_longest_pairs():
    """Both sequences at the longest accepted length, and the most lopsided
    pairs it allows, at Rounds = 20."""
    rng = np.random.default_rng(33)
    L = H().hs.MAX_ALIGN
    q = synth.random_protein(rng, L)
    pairs = [(q, synth.random_protein(rng, L)),
             (q, synth.embed(rng, synth.mutate(rng, q[:3000], 0.5), L)),
             (synth.random_protein(rng, 1), synth.random_protein(rng, L)),
             (synth.random_protein(rng, L), synth.random_protein(rng, 2))]
    say("pairwise: longest pairs")
    check_pairs(pairs, H().Params(rounds=20))


def test_thousand_pairs_of_mixed_lengths():
    """1,000 pairs of log-normal lengths (median 300, up to 2,000), the
    pairwise benchmark's mix: many pairs in flight, their rounds finishing in
    any order, each pair replayed by the workgroup of its last round."""
    rng = np.random.default_rng(35)
    pairs = []
    for L in synth.lognormal_lengths(rng, 1000, 300, 0.6, 20, 2000):
        q = synth.random_protein(rng, int(L))
        tl = int(synth.lognormal_lengths(rng, 1, 300, 0.6, 20, 2000)[0])
        pairs.append((q, synth.embed(rng, synth.mutate(rng, q, rng.uniform(0.2, 0.9)), tl)))
    say("pairwise: 1,000 pairs of mixed lengths, Rounds 20")
    got = check_pairs(pairs, H().Params(rounds=20, seed=21))
    assert len({g.round for g in got}) > 10        # the best round varies over the pairs


def test_device_form_equals_host_form():
    """hs_align_batch_dev (letters and results in device memory) gives what
    hs_align_batch gives, pair by pair, at Rounds 20 and 1 (rounds output
    omitted), on short pairs and on a batch holding a longest pair; codes
    above the alphabet's last read as it; a short workspace is refused."""
    import torch
    Hm = H()
    rng = np.random.default_rng(36)
    short = rand_pairs(rng, 200, 1, 500)
    longp = short[:20] + [(synth.random_protein(rng, Hm.hs.MAX_ALIGN), synth.random_protein(rng, 4500))]
    for pairs, rounds in ((short, 20), (short, 1), (longp, 20)):
        p = Hm.Params(rounds=rounds, seed=17)
        host = Hm.align_batch(pairs, p)
        qs = [Hm.encode(bytes(q)) for q, _ in pairs]
        ts = [Hm.encode(bytes(t)) for _, t in pairs]
        # targets first, queries after them, to check that offsets are honoured
        tl = np.cumsum([0] + [len(t) for t in ts])
        ql = np.cumsum([0] + [len(q) for q in qs]) + tl[-1]
        codes = torch.from_numpy(np.concatenate(ts + qs)).cuda()
        n = len(pairs)
        ws = torch.empty(Hm.align_workspace_bytes(n, rounds), dtype=torch.uint8, device="cuda")
        sc = torch.empty(n, dtype=torch.int32, device="cuda")
        rd = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        total = int(tl[-1] + ql[-1] - ql[0])
        ops = torch.zeros(total, dtype=torch.int32, device="cuda")
        nops = torch.empty(n, dtype=torch.int32, device="cuda")
        Hm.align_batch_dev(codes, ql, tl, p, ws, sc, rd if rounds > 1 else None, ops, nops)
        torch.cuda.synchronize()
        sc, rd, ops, nops = sc.cpu().numpy(), rd.cpu().numpy(), ops.cpu().numpy().view(np.uint32), nops.cpu().numpy()
        for i, h in enumerate(host):
            slot = int(ql[i] - ql[0] + tl[i] - tl[0])
            assert sc[i] == h.score, f"pair {i}"
            assert rd[i] == (h.round if rounds > 1 else -7), f"pair {i}"
            assert np.array_equal(ops[slot:slot + nops[i]], h.ops), f"ops of pair {i}"
    # a code above 23 reads as 23 ('*')
    q, t = Hm.encode(b"ACDW*"), Hm.encode(b"WACD*")
    bad = torch.from_numpy(np.concatenate([q[:4], np.array([200], np.uint8), t])).cuda()
    assert bad.dtype == torch.uint8
    ref = Hm.align(b"ACDW*", b"WACD*", Hm.Params(rounds=3))
    ws = torch.empty(Hm.align_workspace_bytes(1, 3), dtype=torch.uint8, device="cuda")
    sc = torch.empty(1, dtype=torch.int32, device="cuda")
    ops = torch.zeros(10, dtype=torch.int32, device="cuda")
    nops = torch.empty(1, dtype=torch.int32, device="cuda")
    Hm.align_batch_dev(bad, [0, 5], [5, 10], Hm.Params(rounds=3), ws, sc, None, ops, nops)
    torch.cuda.synchronize()
    assert int(sc.cpu()[0]) == ref.score
    assert np.array_equal(ops.cpu().numpy().view(np.uint32)[:int(nops.cpu()[0])], ref.ops)
    with pytest.raises(Hm.HSError):
        Hm.align_batch_dev(bad, [0, 5], [5, 10], Hm.Params(rounds=3), ws[:8], sc, None, ops, nops)
    with pytest.raises(Hm.HSError):
        Hm.align_batch_dev(bad, [0, 5], [5, 5], Hm.Params(rounds=3), ws, sc, None, ops, nops)


def test_single_equals_batch():
    rng = np.random.default_rng(34)
    q, t = synth.random_protein(rng, 120), synth.random_protein(rng, 90)
    p = H().Params(rounds=20, seed=8)
    a = H().align(bytes(q), bytes(t), p)
    b = H().align_batch([(q, t)], p)[0]
    assert (a.score, a.round) == (b.score, b.round)
    assert np.array_equal(a.ops, b.ops)
    r = O.align_pair(O.encode(bytes(q)), O.encode(bytes(t)), 0, oparams(p))
    assert (a.score, a.round, [int(x) for x in a.ops]) == (r["score"], r["round"], r["ops"])


def test_errors():
    Hm = H()
    with pytest.raises(Hm.HSError):
        Hm.align(b"", b"ACD")
    with pytest.raises(Hm.HSError):
        Hm.align(b"A" * 5601, b"ACD")
    with pytest.raises(Hm.HSError):
        Hm.align(b"AC1", b"ACD")
    with pytest.raises(Hm.HSError):
        Hm.align(b"ACD", b"ACD", Hm.Params(rounds=0))
