"""hs_search_dev_noalloc, the search entry point that allocates nothing (its
workspace is the library's static device scratch array), against
hs_search_dev with a caller workspace and against the oracle, bit for bit:
two calls in a row on one device, the second with a smaller database and a
shorter query, so that the second runs over the first one's leftovers."""
import ctypes
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_both(H, torch, db, query, params, k, n_aln):
    """(noalloc result, workspace result) of one query on `db`."""
    out = []
    for noalloc in (True, False):
        ds = H.DeviceSearch(db, len(query), k, n_aln)
        ds.set_query(bytes(query))
        # poison the outputs, so that anything left unwritten shows
        ds.hits.fill_(0xA5)
        ds.alns.fill_(0xA5)
        ds.ops.fill_(-1)
        ds.run(params, noalloc=noalloc)
        torch.cuda.synchronize()
        out.append(ds.fetch())
    return out


def check_equal(a, b):
    assert len(a.hits) == len(b.hits)
    assert (a.hits == b.hits).all()
    assert len(a.alns) == len(b.alns)
    assert (a.alns == b.alns).all()
    assert np.array_equal(a.ops, b.ops)


def check_oracle(r, res, off, query, k, n_aln):
    codes = O.encode_db(res, off)
    ref = O.search(codes, off, O.encode(bytes(query)), O.Params(), k=k, n_aln=n_aln)
    assert [int(i) for i in r.hits["target_id"]] == [int(i) for i in ref["ids"]]
    assert [int(s) for s in r.hits["score"]] == [int(s) for s in ref["scores"]]
    assert len(r.alns) == len(ref["alns"])
    for i, (tid, score, ops) in enumerate(ref["alns"]):
        assert int(r.alns[i]["target_id"]) == tid and int(r.alns[i]["score"]) == score
        assert [int(x) for x in r.ops_of(i)] == [int(x) for x in ops]


def test_noalloc_two_calls_then_smaller():
    import torch
    import paper_1508_06561_amd as H
    torch.cuda.set_device(0)
    p = H.Params()
    # call 1: the full workload (500,200 targets, 300-letter query), which
    # fills about 36 MB of the scratch
    w = synth.config_full()
    say(f"noalloc call 1: {w.n_targets} targets, query {len(w.queries[0])}")
    db = H.Database(w.residues, w.offsets)
    a, b = run_both(H, torch, db, w.queries[0], p, w.k, w.n_aln)
    check_equal(a, b)
    check_oracle(a, w.residues, w.offsets, w.queries[0], w.k, w.n_aln)
    db.close()
    # call 2: a smaller database (2,020 targets) and a shorter query (64)
    q, res, off, _ = synth.tiny_db(seed=synth.BASE_SEED)
    say(f"noalloc call 2: {len(off) - 1} targets, query {len(q)}")
    db = H.Database(res, off)
    a, b = run_both(H, torch, db, q, p, 50, 50)
    check_equal(a, b)
    check_oracle(a, res, off, q, 50, 50)
    db.close()


def test_noalloc_rejects_oversize_database():
    import torch
    import paper_1508_06561_amd as H
    torch.cuda.set_device(0)
    n = 1_000_000     # needs about 72 MB of workspace, above the 64 MiB scratch
    res = np.full(n, ord("A"), dtype=np.uint8)
    off = np.arange(n + 1, dtype=np.int64)
    say(f"noalloc oversize: {n} targets")
    db = H.Database(res, off)
    need = db.workspace_bytes(1, 8, 10, 0)
    assert need > (64 << 20)
    ds = H.DeviceSearch(db, 8, 10, 0)
    ds.set_query(b"ACDEFGHI")
    with pytest.raises(H.HSError) as e:
        ds.run(H.Params(), noalloc=True)
    assert e.value.code == H.hs.HS_ENOMEM and "scratch" in str(e.value)
    # the workspace form of the same search still runs
    ds.run(H.Params())
    torch.cuda.synchronize()
    assert len(ds.fetch().hits) == 10
    db.close()
