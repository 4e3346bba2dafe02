"""Writes the stored oracle results of the two workloads too large for the
oracle to rerun inside a GPU test.  Calls only the oracle (``oracle/``) and
the seeded input generators (``synth/``); nothing here comes from the HIP
path.

    python tests/golden/make_golden.py long     -> tests/golden/long_oracle.json
    python tests/golden/make_golden.py sw_full  -> tests/golden/sw_full_oracle.json

long: the long-sequence workload (32 queries of 2,000-5,000 letters against
the 2,020-target database plus 5,064 targets of 10,000-35,000 letters, search
setting of Section IV).  For every query: a SHA-256 of all 7,084 pair scores
(int32 little endian, target order), the cells scored (the work measure of
Section III.B.4), the first 50 ranks (score descending, index ascending) and,
for each of them, the oracle's alignment (Fig. 1 replay) as its score, op
count and the first 24 hex digits of a SHA-256 of its run-length ops.

sw_full: the Smith-Waterman-Gotoh optimum (gap run of g columns costs
GOP + (g - 1) * GEP, Section III.B.1) of the 300-letter query of the full
workload against all 500,200 targets: SHA-256 of the score vector, the 500
best (score, index) and the score sum.

The oracle is single-threaded C that releases the GIL, so the pairs are
spread over a thread pool of every host core.
"""
import concurrent.futures as cf
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
LONG_PATH = os.path.join(HERE, "long_oracle.json")
SW_PATH = os.path.join(HERE, "sw_full_oracle.json")


def sha_i32(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<i4").tobytes()).hexdigest()


def sha_u32(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def _pool():
    return cf.ThreadPoolExecutor(os.cpu_count() or 1)


def make_long(k=50, n_aln=50):
    w = synth.config_long()
    codes = O.encode_db(w.residues, w.offsets)
    n = w.n_targets
    p = O.Params()
    # longest targets first, in small chunks, so that the pool stays balanced
    lens = np.diff(w.offsets)
    order = np.argsort(-lens, kind="stable")
    chunks = [order[i:i + 16] for i in range(0, n, 16)]
    t0 = time.time()
    out = []
    for qi, q in enumerate(w.queries):
        qc = O.encode(bytes(q))
        scores = np.zeros(n, dtype=np.int32)
        cells = 0
        with _pool() as ex:
            futs = {ex.submit(O.score_all, codes, w.offsets, qc, p, None,
                              np.sort(c).astype(np.int64)): np.sort(c) for c in chunks}
            for f, ids in futs.items():
                s, _, c = f.result()
                scores[ids] = s
                cells += c
        top = O.rank(scores, k)

        def aln(tid):
            t = codes[w.offsets[tid]:w.offsets[tid + 1]]
            return O.align_pair(qc, t, int(tid), p)

        with _pool() as ex:
            alns = list(ex.map(aln, [int(t) for t in top[:n_aln]]))
        rec = dict(query=qi, qlen=len(q), scores_sha256=sha_i32(scores), cells=int(cells),
                   top_ids=[int(t) for t in top], top_scores=[int(scores[t]) for t in top],
                   alns=[])
        for tid, a in zip(top[:n_aln], alns):
            assert a["score"] == scores[tid]
            rec["alns"].append([int(tid), int(a["score"]), len(a["ops"]), sha_u32(a["ops"])[:24]])
        out.append(rec)
        print(f"query {qi} ({len(q)} letters): {cells} cells, best {rec['top_scores'][0]}, "
              f"{time.time() - t0:.0f}s", flush=True)
    doc = dict(workload=w.name, n_targets=n, db_residues=w.db_residues, k=k, n_aln=n_aln,
               params="PGP 0, GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, Rounds 1, "
                      "seed 0", writer="tests/golden/make_golden.py long",
               aln_fields="target_id, score, n_ops, first 24 hex digits of the SHA-256 of the "
                          "ops (uint32 little endian)")
    with open(LONG_PATH, "w") as f:     # one line per query
        f.write("{\n")
        for k, v in doc.items():
            f.write(f" {json.dumps(k)}: {json.dumps(v)},\n")
        f.write(' "queries": [\n')
        f.write(",\n".join("  " + json.dumps(q, separators=(",", ":")) for q in out))
        f.write("\n ]\n}\n")
    print(f"wrote {LONG_PATH}")


def make_sw_full(top=500):
    w = synth.config_full()
    codes = O.encode_db(w.residues, w.offsets)
    q = O.encode(bytes(w.queries[0]))
    n = w.n_targets
    off = w.offsets
    m = O.blosum62()
    t0 = time.time()

    def run(ids):
        return ids, [O.sw_score(q, codes[off[i]:off[i + 1]], 10, 5, m) for i in ids]

    scores = np.zeros(n, dtype=np.int32)
    with _pool() as ex:
        for ids, s in ex.map(run, np.array_split(np.arange(n), 4096)):
            scores[ids] = s
    best = O.rank(scores, top)
    doc = dict(workload=w.name, n_targets=n, query_len=len(q), gop=10, gep=5,
               scores_sha256=sha_i32(scores), score_sum=int(scores.astype(np.int64).sum()),
               top_ids=[int(i) for i in best], top_scores=[int(scores[i]) for i in best],
               writer="tests/golden/make_golden.py sw_full")
    with open(SW_PATH, "w") as f:
        json.dump(doc, f)
        f.write("\n")
    print(f"wrote {SW_PATH} in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "long"
    {"long": make_long, "sw_full": make_sw_full}[what]()
