"""Reference oracle for the search-mode heuristic of Nag & Karforma
(arXiv 1508.06561): a plain, slow, single-threaded CPU implementation.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
CPU-baseline leg are the only callers; the product library never imports it.
The heavy lifting is plain C (``hs_oracle.c``, following Fig. 1 of the paper
procedure by procedure); this module marshals arguments through ctypes and does
the final ranking with a library sort, which the paper leaves to the caller
("ranked against a database", Abstract and Section IV).
"""
import ctypes
import dataclasses
import os

import numpy as np

from . import build as _build

GAP = 0xFF
OP_M, OP_I, OP_D = 0, 1, 2

_lib = None


def lib():
    """Load the compiled oracle, compiling it with gcc if it is not built."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIB", _build.LIB)   # a planted-mistake build in tests
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        L.orc_alphabet_str.restype = ctypes.c_char_p
        L.orc_draw.restype = ctypes.c_uint32
        L.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_encode.argtypes = [ctypes.c_char_p, ctypes.c_int64, u8p]
        L.orc_score_rows.restype = ctypes.c_int64
        L.sw_gotoh_local.restype = ctypes.c_int64
        L.sw_gotoh_local.argtypes = [u8p, ctypes.c_int32, u8p, ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int8), ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


class _Params(ctypes.Structure):
    _fields_ = [("gop", ctypes.c_int32), ("gep", ctypes.c_int32), ("pgp", ctypes.c_int32),
                ("lfactor_q16", ctypes.c_int32), ("sfactor_q16", ctypes.c_int32),
                ("minfactor_q16", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("full_slide", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class _Step(ctypes.Structure):
    _fields_ = [("pL", ctypes.c_int32), ("pS", ctypes.c_int32), ("ls", ctypes.c_int32),
                ("ss", ctypes.c_int32), ("kstar", ctypes.c_int32), ("dscore", ctypes.c_int32)]


@dataclasses.dataclass
class Params:
    """Parameters of Section III.B.1; defaults are the search setting of
    Section IV (PGP 0, GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5)
    with Rounds = 1 (Section III.B.3).  Factors are Q16 (65536 = 1.0).
    full_slide selects the pairwise mode of Fig. 1 (every overlapping
    placement) instead of the search mode's contained shifts."""
    gop: int = 10
    gep: int = 5
    pgp: int = 0
    lfactor_q16: int = 32768
    sfactor_q16: int = 65536
    minfactor_q16: int = 32768
    rounds: int = 1
    seed: int = 0
    full_slide: bool = False

    def c(self):
        return _Params(self.gop, self.gep, self.pgp, self.lfactor_q16, self.sfactor_q16,
                       self.minfactor_q16, self.rounds, 1 if self.full_slide else 0,
                       self.seed & (2**64 - 1))


def alphabet():
    return lib().orc_alphabet_str().decode()


def blosum62():
    out = np.zeros((24, 24), dtype=np.int8)
    lib().orc_blosum62_copy(out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return out


def background_counts():
    out = np.zeros(20, dtype=np.int32)
    lib().orc_background_counts(out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)) if a is not None else None


def encode(seq):
    """ASCII residues -> uint8 codes in alphabet order (ValueError if invalid)."""
    if isinstance(seq, str):
        seq = seq.encode()
    b = bytes(seq)
    out = np.empty(len(b), dtype=np.uint8)
    if lib().orc_encode(b, len(b), _u8(out)) != 0:
        raise ValueError("residue outside the alphabet")
    return out


def decode(codes):
    al = alphabet()
    return "".join("-" if c == GAP else al[c] for c in codes)


def philox4x64_10(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (ctypes.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [int(x) for x in o]


def draw(seed, target_id, rnd, d):
    return int(lib().orc_draw(seed & (2**64 - 1), target_id, rnd, d))


def _matrix(matrix):
    if matrix is None:
        return None
    m = np.ascontiguousarray(matrix, dtype=np.int8)
    assert m.shape == (24, 24)
    return m


def rows_to_ops(qrow, trow):
    """Aligned (query row, target row) -> run-length ops (len << 2 | op) with
    M = letter over letter, I = query letter over a gap, D = target letter
    over a gap."""
    ops = []
    for a, b in zip(qrow, trow):
        op = OP_M if (a != GAP and b != GAP) else (OP_I if a != GAP else OP_D)
        if ops and (ops[-1] & 3) == op:
            ops[-1] += 4
        else:
            ops.append(4 | op)
    return ops


def align_pair(q, t, target_id=0, params=None, matrix=None, trace=False):
    """Search-mode heuristic alignment of query q against target t (codes);
    `matrix` (24 x 24, default BLOSUM62) scores a query letter (row) against a
    target letter (column).

    Returns dict(score, round, qrow, trow (codes, GAP for gaps), ops, cells,
    trace) where trace lists (pL, pS, ls, ss, kstar, dscore) per step of the
    best round when requested."""
    p = params or Params()
    q = np.ascontiguousarray(q, dtype=np.uint8)
    t = np.ascontiguousarray(t, dtype=np.uint8)
    cap = len(q) + len(t)
    qrow = np.zeros(cap, dtype=np.uint8)
    trow = np.zeros(cap, dtype=np.uint8)
    m = _matrix(matrix)
    score, rnd, rowlen, nsteps, cells = (ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(),
                                         ctypes.c_int32(), ctypes.c_int64())
    tcap = min(len(q), len(t)) + 1
    tr = (_Step * tcap)() if trace else None
    rc = lib().orc_align_pair(_u8(q), len(q), _u8(t), len(t), ctypes.c_uint64(target_id),
                              ctypes.byref(p.c()), _i8(m), ctypes.byref(score), ctypes.byref(rnd),
                              _u8(qrow), _u8(trow), cap, ctypes.byref(rowlen),
                              tr, tcap if trace else 0, ctypes.byref(nsteps), ctypes.byref(cells))
    if rc != 0:
        raise ValueError(f"oracle align_pair failed ({rc})")
    n = rowlen.value
    out = dict(score=score.value, round=rnd.value, qrow=qrow[:n].copy(), trow=trow[:n].copy(),
               cells=cells.value, steps=nsteps.value)
    out["ops"] = rows_to_ops(out["qrow"], out["trow"])
    if trace:
        out["trace"] = [(s.pL, s.pS, s.ls, s.ss, s.kstar, s.dscore) for s in tr[:nsteps.value]]
    return out


def score_rows(row_a, row_b, params=None, matrix=None):
    """SCORE of two aligned rows of codes (GAP = gap); the matrix scores a
    row_a letter (row) against a row_b letter (column)."""
    p = params or Params()
    a = np.ascontiguousarray(row_a, dtype=np.uint8)
    b = np.ascontiguousarray(row_b, dtype=np.uint8)
    L = lib()
    L.orc_score_rows.argtypes = [ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint8),
                                 ctypes.c_int32, ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_int8)]
    return int(L.orc_score_rows(_u8(a), _u8(b), len(a), ctypes.byref(p.c()), _i8(_matrix(matrix))))


def encode_db(residues, offsets):
    """Concatenated ASCII residues (uint8 array) -> codes (same layout)."""
    res = np.ascontiguousarray(residues, dtype=np.uint8)
    out = np.empty(len(res), dtype=np.uint8)
    if lib().orc_encode(res.ctypes.data_as(ctypes.c_char_p), len(res), _u8(out)) != 0:
        raise ValueError("residue outside the alphabet")
    return out


def score_all(db_codes, offsets, q, params=None, matrix=None, ids=None):
    """Pair score of the query against every target (or the targets in ids).
    Returns (scores int32, rounds int32 or None, cells)."""
    p = params or Params()
    db = np.ascontiguousarray(db_codes, dtype=np.uint8)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    q = np.ascontiguousarray(q, dtype=np.uint8)
    m = _matrix(matrix)
    cells = ctypes.c_int64()
    L = lib()
    if ids is None:
        n = len(off) - 1
        scores = np.zeros(n, dtype=np.int32)
        rounds = np.zeros(n, dtype=np.int32)
        rc = L.orc_search(_u8(db), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          ctypes.c_int64(n), _u8(q), len(q), ctypes.byref(p.c()), _i8(m),
                          scores.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          rounds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.byref(cells))
    else:
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        scores = np.zeros(len(ids), dtype=np.int32)
        rounds = None
        rc = L.orc_search_subset(_u8(db), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ctypes.c_int64(len(ids)), _u8(q), len(q), ctypes.byref(p.c()),
                                 _i8(m), scores.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 ctypes.byref(cells))
    if rc != 0:
        raise ValueError(f"oracle search failed ({rc})")
    return scores, rounds, cells.value


def rank(scores, k, min_score=-(2**31)):
    """Ranking of the database search: targets with score >= min_score sorted
    by (score descending, target index ascending), first k kept."""
    scores = np.asarray(scores)
    ids = np.arange(len(scores), dtype=np.int64)
    order = np.lexsort((ids, -scores.astype(np.int64)))
    order = order[scores[order] >= min_score]
    return order[:k]


def search(db_codes, offsets, q, params=None, k=50, n_aln=50, min_score=-(2**31), matrix=None):
    """One query against the whole database: ranked hits plus alignments of
    the first n_aln ranks.  Returns dict(ids, scores (ranked), all_scores,
    rounds, alns=[(id, score, ops)], cells)."""
    p = params or Params()
    scores, rounds, cells = score_all(db_codes, offsets, q, p, matrix)
    top = rank(scores, k, min_score)
    alns = []
    off = np.asarray(offsets, dtype=np.int64)
    for tid in top[:n_aln]:
        t = np.asarray(db_codes[off[tid]:off[tid + 1]])
        a = align_pair(q, t, int(tid), p, matrix)
        assert a["score"] == scores[tid]
        alns.append((int(tid), a["score"], a["ops"]))
    return dict(ids=top, scores=scores[top], all_scores=scores, rounds=rounds, alns=alns,
                cells=cells)


def sw_score(a, b, gop=10, gep=5, matrix=None):
    """Gotoh affine local-alignment optimum (upper-bound checker)."""
    a = np.ascontiguousarray(a, dtype=np.uint8)
    b = np.ascontiguousarray(b, dtype=np.uint8)
    m = _matrix(matrix) if matrix is not None else blosum62()
    return int(lib().sw_gotoh_local(_u8(a), len(a), _u8(b), len(b), _i8(m), gop, gep))
