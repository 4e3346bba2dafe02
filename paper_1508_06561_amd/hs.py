"""Python binding of the C ABI in include/hs.h (argument marshalling only).

Every step of a search runs in the HIP kernels of ``libhs.so``; this module
passes pointers and sizes through ctypes, takes device buffers from torch and
the stream from ``torch.cuda.current_stream()``.  It fails loudly when the
library is missing: there is no other path.
"""
import ctypes
import dataclasses
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhs.so")

HS_OK, HS_EINVAL, HS_ENOMEM, HS_ENOSPC, HS_EDEVICE = 0, -1, -2, -3, -4
OP_M, OP_I, OP_D = 0, 1, 2
MAX_K = 4096
MAX_QUERY = 5600
MAX_BATCH = 4096
MAX_SERVER_WORKERS = 8
MAX_ALIGN = 5600
ALPHABET = "ARNDCQEGHILKMFPSTWYVBZX*"


class HSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hs error {code}: {msg}")
        self.code = code


class _CParams(ctypes.Structure):
    _fields_ = [("gop", ctypes.c_int32), ("gep", ctypes.c_int32), ("pgp", ctypes.c_int32),
                ("lfactor_q16", ctypes.c_int32), ("sfactor_q16", ctypes.c_int32),
                ("minfactor_q16", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("min_score", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("matrix", ctypes.POINTER(ctypes.c_int8))]


class Hit(ctypes.Structure):
    _fields_ = [("target_id", ctypes.c_int64), ("score", ctypes.c_int32), ("round", ctypes.c_int32)]


class Aln(ctypes.Structure):
    _fields_ = [("target_id", ctypes.c_int64), ("score", ctypes.c_int32), ("n_ops", ctypes.c_int32),
                ("ops_off", ctypes.c_int64)]


class ServerTiming(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("queue_ms", ctypes.c_double),
                ("batch_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("set_ms", ctypes.c_double), ("run_ms", ctypes.c_double),
                ("results_ms", ctypes.c_double), ("gpu_ms", ctypes.c_double),
                ("batch_size", ctypes.c_int32), ("pad_", ctypes.c_int32)]


HIT_DTYPE = np.dtype([("target_id", np.int64), ("score", np.int32), ("round", np.int32)])
ALN_DTYPE = np.dtype([("target_id", np.int64), ("score", np.int32), ("n_ops", np.int32),
                      ("ops_off", np.int64)])

_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        # torch brings its own HIP runtime (same soname); loading it first
        # makes libhs.so bind to that one instead of a second runtime that
        # would contend for the device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.hs_params_default.argtypes = [P(_CParams)]
        L.hs_builtin_matrix.argtypes = [P(ctypes.c_int8)]
        L.hs_encode.argtypes = [ctypes.c_char_p, ctypes.c_int64, P(ctypes.c_uint8)]
        L.hs_db_load.argtypes = [vp, P(ctypes.c_int64), ctypes.c_int64, vp, P(vp)]
        L.hs_db_free.argtypes = [vp]
        L.hs_db_set_letters.argtypes = [vp, ctypes.c_int32, vp]
        L.hs_db_info.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
        L.hs_workspace_bytes.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32]
        L.hs_workspace_bytes.restype = ctypes.c_size_t
        L.hs_search.argtypes = [vp, ctypes.c_char_p, ctypes.c_int32, P(_CParams), ctypes.c_int32,
                                ctypes.c_int32, vp, vp, P(ctypes.c_int32), vp, P(ctypes.c_int32),
                                vp, ctypes.c_int64, P(ctypes.c_int64)]
        L.hs_search_dev.argtypes = [vp, vp, ctypes.c_int32, P(_CParams), ctypes.c_int32,
                                    ctypes.c_int32, vp, vp, ctypes.c_size_t, vp, vp, vp, vp,
                                    ctypes.c_int64]
        L.hs_search_dev_noalloc.argtypes = [vp, vp, ctypes.c_int32, P(_CParams), ctypes.c_int32,
                                            ctypes.c_int32, vp, vp, vp, vp, vp, ctypes.c_int64]
        L.hs_score_dev.argtypes = [vp, vp, ctypes.c_int32, P(_CParams), vp, vp, ctypes.c_size_t,
                                   vp, vp, vp]
        L.hs_threshold_workspace_bytes.argtypes = [vp]
        L.hs_threshold_workspace_bytes.restype = ctypes.c_size_t
        L.hs_search_threshold_dev.argtypes = [vp, vp, ctypes.c_int32, P(_CParams), ctypes.c_int64,
                                              ctypes.c_int32, vp, vp, ctypes.c_size_t, vp, vp, vp,
                                              vp, ctypes.c_int64]
        L.hs_search_threshold.argtypes = [vp, ctypes.c_char_p, ctypes.c_int32, P(_CParams),
                                          ctypes.c_int64, ctypes.c_int32, vp, vp,
                                          P(ctypes.c_int64), vp, P(ctypes.c_int32), vp,
                                          ctypes.c_int64, P(ctypes.c_int64)]
        i32, i64, pi32 = ctypes.c_int32, ctypes.c_int64, P(ctypes.c_int32)
        L.hs_sw_workspace_bytes.argtypes = [vp]
        L.hs_sw_workspace_bytes.restype = ctypes.c_int64
        L.hs_sw_scores_dev.argtypes = [vp, vp, ctypes.c_int32, P(_CParams), vp, vp, ctypes.c_size_t, vp]
        L.hs_batch_create.argtypes = [vp, i32, i32, i64, i32, i32, P(vp)]
        L.hs_batch_free.argtypes = [vp]
        L.hs_batch_set.argtypes = [vp, i32, vp, P(ctypes.c_int64), P(_CParams), i32, vp]
        L.hs_batch_schedule.argtypes = [vp, i32, i32, i32, vp]
        L.hs_batch_get_schedule.argtypes = [vp, pi32, pi32, pi32, pi32, pi32]
        L.hs_batch_get_launch.argtypes = [vp, pi32, pi32, pi32, pi32]
        L.hs_batch_tune.argtypes = [vp, vp, i32, P(ctypes.c_float)]
        L.hs_batch_run.argtypes = [vp, vp]
        L.hs_batch_run_graph.argtypes = [vp, vp]
        L.hs_batch_score.argtypes = [vp, vp, vp]
        L.hs_batch_results.argtypes = [vp, vp, vp, pi32, vp, pi32, vp, i64, P(ctypes.c_int64)]
        L.hs_batch_scores.argtypes = [vp, vp, vp, vp]
        L.hs_batch_outputs.argtypes = [vp, P(vp), P(vp), P(vp), P(vp), P(ctypes.c_int64), P(vp),
                                       P(vp)]
        L.hs_search_batch.argtypes = [vp, i32, vp, P(ctypes.c_int64), P(_CParams), i32, i32, i32,
                                      vp, vp, pi32, vp, pi32, vp, i64, P(ctypes.c_int64)]
        L.hs_params_check.argtypes = [P(_CParams)]
        L.hs_align_batch.argtypes = [i32, vp, P(ctypes.c_int64), vp, P(ctypes.c_int64), P(_CParams),
                                     vp, pi32, pi32, vp, i64, P(ctypes.c_int64), P(ctypes.c_int64)]
        L.hs_align.argtypes = [ctypes.c_char_p, i32, ctypes.c_char_p, i32, P(_CParams), vp, pi32,
                               pi32, vp, i64, P(ctypes.c_int64)]
        L.hs_align_workspace_bytes.argtypes = [i32, i32]
        L.hs_align_workspace_bytes.restype = ctypes.c_int64
        L.hs_align_batch_dev.argtypes = [i32, vp, P(ctypes.c_int64), P(ctypes.c_int64), P(_CParams), vp,
                                         vp, ctypes.c_size_t, vp, vp, vp, vp]
        L.hs_server_create.argtypes = [vp, i32, i32, i64, i32, i32, P(vp)]
        L.hs_server_create_workers.argtypes = [vp, i32, i32, i64, i32, i32, i32, P(vp)]
        L.hs_server_free.argtypes = [vp]
        L.hs_server_submit.argtypes = [vp, ctypes.c_char_p, i32, P(_CParams), ctypes.c_uint64]
        L.hs_server_poll.argtypes = [vp, P(ctypes.c_uint64), i32, pi32, i32]
        L.hs_server_result.argtypes = [vp, ctypes.c_uint64, vp, pi32, vp, pi32, vp, i64,
                                       P(ctypes.c_int64), P(ServerTiming)]
        L.hs_server_stats.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64)]
        L.hs_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc):
    if rc != HS_OK:
        raise HSError(rc, lib().hs_last_error().decode())
    return rc


@dataclasses.dataclass
class Params:
    """hs_params; defaults are the search setting of Section IV of the paper
    (PGP 0, GOP 10, GEP 5, LFactor 0.5, SFactor 1, MinFactor 0.5, Rounds 1)."""
    gop: int = 10
    gep: int = 5
    pgp: int = 0
    lfactor_q16: int = 32768
    sfactor_q16: int = 65536
    minfactor_q16: int = 32768
    rounds: int = 1
    min_score: int = -(2**31)
    seed: int = 0
    matrix: np.ndarray = None

    def c(self):
        p = _CParams(self.gop, self.gep, self.pgp, self.lfactor_q16, self.sfactor_q16,
                     self.minfactor_q16, self.rounds, self.min_score, self.seed & (2**64 - 1), None)
        if self.matrix is not None:
            self._m = np.ascontiguousarray(self.matrix, dtype=np.int8).reshape(24, 24)
            p.matrix = self._m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
        return p


def params_default():
    p = _CParams()
    lib().hs_params_default(ctypes.byref(p))
    return Params(p.gop, p.gep, p.pgp, p.lfactor_q16, p.sfactor_q16, p.minfactor_q16, p.rounds,
                  p.min_score, p.seed)


def builtin_matrix():
    m = np.zeros((24, 24), dtype=np.int8)
    lib().hs_builtin_matrix(m.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return m


def encode(seq):
    """ASCII -> alphabet codes (host)."""
    b = seq.encode() if isinstance(seq, str) else bytes(seq)
    out = np.empty(len(b), dtype=np.uint8)
    _check(lib().hs_encode(b, len(b), out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclasses.dataclass
class Result:
    hits: np.ndarray          # HIT_DTYPE, ranked
    alns: np.ndarray          # ALN_DTYPE, alns[i] belongs to hits[i]
    ops: np.ndarray           # uint32 run-length ops, alns index into it

    def ops_of(self, i):
        a = self.alns[i]
        return self.ops[a["ops_off"]:a["ops_off"] + a["n_ops"]]


class Database:
    """A database loaded on the device (hs_db_load).  `residues` is a uint8
    array of concatenated ASCII letters, `offsets` int64 with n + 1 bounds."""

    def __init__(self, residues, offsets, stream=None):
        res = np.ascontiguousarray(residues, dtype=np.uint8)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        h = ctypes.c_void_p()
        _check(lib().hs_db_load(res.ctypes.data_as(ctypes.c_void_p),
                                off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                len(off) - 1, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n_targets = len(off) - 1

    def close(self):
        if getattr(self, "_h", None):
            lib().hs_db_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_letters(self, bits, stream=None):
        """hs_db_set_letters: the letter image (8 = bytes, 5 = packed) that
        the one-query scoring kernel reads."""
        _check(lib().hs_db_set_letters(self._h, bits, _stream(stream)))

    def info(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hs_db_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(n_targets=a.value, n_residues=b.value, device_bytes=c.value)

    def search(self, query, params=None, k=50, n_aln=50, stream=None):
        """hs_search: host query in, host results out."""
        p = (params or Params()).c()
        q = query.encode() if isinstance(query, str) else bytes(query)
        hits = np.zeros(k, dtype=HIT_DTYPE)
        alns = np.zeros(max(n_aln, 1), dtype=ALN_DTYPE)
        cap = max(1, n_aln * (2 * len(q) + 2))
        ops = np.zeros(cap, dtype=np.uint32)
        nh, na, used = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().hs_search(self._h, q, len(q), ctypes.byref(p), k, n_aln, _stream(stream),
                               hits.ctypes.data, ctypes.byref(nh), alns.ctypes.data,
                               ctypes.byref(na), ops.ctypes.data, cap, ctypes.byref(used)))
        n_a = na.value if n_aln > 0 else 0
        return Result(hits[:nh.value].copy(), alns[:n_a].copy(), ops[:used.value].copy())

    def search_threshold(self, query, params=None, cap=None, n_aln=0, stream=None):
        """hs_search_threshold: every target scoring at least params.min_score,
        ranked (no cap on the count), with alignments for the first n_aln.
        cap defaults to the number of targets, which always suffices."""
        p = (params or Params()).c()
        q = query.encode() if isinstance(query, str) else bytes(query)
        cap = self.n_targets if cap is None else cap
        hits = np.zeros(max(cap, 1), dtype=HIT_DTYPE)
        alns = np.zeros(max(n_aln, 1), dtype=ALN_DTYPE)
        ocap = max(1, n_aln * (2 * len(q) + 2))
        ops = np.zeros(ocap, dtype=np.uint32)
        n, na, used = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().hs_search_threshold(self._h, q, len(q), ctypes.byref(p), cap, n_aln,
                                         _stream(stream), hits.ctypes.data, ctypes.byref(n),
                                         alns.ctypes.data, ctypes.byref(na), ops.ctypes.data,
                                         ocap, ctypes.byref(used)))
        n_a = na.value if n_aln > 0 else 0
        return Result(hits[:n.value].copy(), alns[:n_a].copy(), ops[:used.value].copy())

    def threshold_workspace_bytes(self):
        return int(lib().hs_threshold_workspace_bytes(self._h))

    def search_threshold_dev(self, d_qcodes, qlen, params, cap, n_aln, d_ws, d_hits, d_n,
                             d_alns=None, d_ops=None, ops_stride=0, stream=None):
        """Queues hs_search_threshold_dev; buffers are torch CUDA tensors."""
        p = params.c()
        _check(lib().hs_search_threshold_dev(
            self._h, d_qcodes.data_ptr(), qlen, ctypes.byref(p), cap, n_aln, _stream(stream),
            d_ws.data_ptr(), d_ws.numel() * d_ws.element_size(),
            d_hits.data_ptr() if d_hits is not None else None, d_n.data_ptr(),
            d_alns.data_ptr() if d_alns is not None else None,
            d_ops.data_ptr() if d_ops is not None else None, ops_stride))

    # ---- device-resident form (hs_search_dev) ----
    def workspace_bytes(self, nq, max_qlen, k, n_aln):
        return int(lib().hs_workspace_bytes(self._h, nq, max_qlen, k, n_aln))

    def search_dev(self, d_qcodes, qlen, params, k, n_aln, d_ws, d_hits, d_n_hits, d_alns, d_ops,
                   ops_stride, stream=None):
        """Queues one search; every buffer argument is a torch CUDA tensor."""
        p = params.c()
        _check(lib().hs_search_dev(self._h, d_qcodes.data_ptr(), qlen, ctypes.byref(p), k, n_aln,
                                   _stream(stream), d_ws.data_ptr(), d_ws.numel() * d_ws.element_size(),
                                   d_hits.data_ptr(), d_n_hits.data_ptr(),
                                   d_alns.data_ptr() if d_alns is not None else None,
                                   d_ops.data_ptr() if d_ops is not None else None, ops_stride))

    def search_dev_noalloc(self, d_qcodes, qlen, params, k, n_aln, d_hits, d_n_hits, d_alns,
                           d_ops, ops_stride, stream=None):
        """hs_search_dev_noalloc: search_dev with the library's static device
        scratch as its workspace (allocates nothing)."""
        p = params.c()
        _check(lib().hs_search_dev_noalloc(self._h, d_qcodes.data_ptr(), qlen, ctypes.byref(p), k,
                                           n_aln, _stream(stream), d_hits.data_ptr(),
                                           d_n_hits.data_ptr(),
                                           d_alns.data_ptr() if d_alns is not None else None,
                                           d_ops.data_ptr() if d_ops is not None else None,
                                           ops_stride))

    def score_dev(self, d_qcodes, qlen, params, d_ws, d_scores, d_rounds=None, d_cells=None,
                  stream=None):
        """Queues hs_score_dev: every target's pair score into d_scores (int32
        torch CUDA tensor of n_targets), winning rounds into d_rounds, and
        the scored residue pairs added to d_cells (one int64)."""
        p = params.c()
        _check(lib().hs_score_dev(self._h, d_qcodes.data_ptr(), qlen, ctypes.byref(p),
                                  _stream(stream), d_ws.data_ptr(),
                                  d_ws.numel() * d_ws.element_size(), d_scores.data_ptr(),
                                  d_rounds.data_ptr() if d_rounds is not None else None,
                                  d_cells.data_ptr() if d_cells is not None else None))

    def sw_workspace_bytes(self):
        """Device workspace bytes of sw_scores_dev (hs_sw_workspace_bytes)."""
        n = lib().hs_sw_workspace_bytes(self._h)
        if n < 0:
            _check(int(n))
        return int(n)

    def sw_scores_dev(self, d_qcodes, qlen, params, d_ws, d_scores, stream=None):
        """Queues hs_sw_scores_dev: every target's Smith-Waterman-Gotoh local
        score into d_scores (int32 torch CUDA tensor of n_targets)."""
        p = params.c()
        _check(lib().hs_sw_scores_dev(self._h, d_qcodes.data_ptr(), qlen, ctypes.byref(p),
                                      _stream(stream), d_ws.data_ptr(),
                                      d_ws.numel() * d_ws.element_size(), d_scores.data_ptr()))

    def sw_scores(self, query, params=None):
        """Every target's Smith-Waterman-Gotoh local score (host int32 array)."""
        import torch
        codes = torch.from_numpy(encode(query)).cuda()
        out = torch.empty(max(self.n_targets, 1), dtype=torch.int32, device="cuda")
        ws = torch.empty(self.sw_workspace_bytes(), dtype=torch.uint8, device="cuda")
        self.sw_scores_dev(codes, len(codes), params or Params(), ws, out)
        return out.cpu().numpy()[:self.n_targets]

    def scores(self, query, params=None):
        """(scores, rounds, cells): every target's pair score and winning
        round (host int32 arrays) and the total scored residue pairs."""
        import torch
        codes = torch.from_numpy(encode(query)).cuda()
        out = torch.empty(max(self.n_targets, 1), dtype=torch.int32, device="cuda")
        rounds = torch.empty(max(self.n_targets, 1), dtype=torch.int32, device="cuda")
        cells = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws = torch.empty(self.workspace_bytes(1, len(codes), 1, 0), dtype=torch.uint8, device="cuda")
        self.score_dev(codes, len(codes), params or Params(), ws, out, rounds, cells)
        return (out.cpu().numpy()[:self.n_targets], rounds.cpu().numpy()[:self.n_targets],
                int(cells.cpu()[0]))


class DeviceSearch:
    """Preallocated torch device buffers for repeated hs_search_dev calls on
    one database (benchmarks, serving)."""

    def __init__(self, db, max_qlen, k, n_aln, device="cuda"):
        import torch
        self.db, self.k, self.n_aln = db, k, n_aln
        self.stride = 2 * max_qlen + 2
        ws = db.workspace_bytes(1, max_qlen, k, n_aln)
        self.ws = torch.empty(ws, dtype=torch.uint8, device=device)
        self.q = torch.empty(max_qlen, dtype=torch.uint8, device=device)
        self.hits = torch.empty(k * HIT_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.n_hits = torch.empty(1, dtype=torch.int32, device=device)
        self.alns = torch.empty(max(n_aln, 1) * ALN_DTYPE.itemsize, dtype=torch.uint8, device=device)
        self.ops = torch.empty(max(n_aln, 1) * self.stride, dtype=torch.int32, device=device)

    def set_query(self, query):
        import torch
        codes = encode(query)
        self.qlen = len(codes)
        self.q[:self.qlen].copy_(torch.from_numpy(codes))

    def run(self, params, stream=None, noalloc=False):
        """Queues the search; noalloc: through hs_search_dev_noalloc."""
        if noalloc:
            self.db.search_dev_noalloc(self.q, self.qlen, params, self.k, self.n_aln, self.hits,
                                       self.n_hits, self.alns, self.ops, self.stride, stream)
        else:
            self.db.search_dev(self.q, self.qlen, params, self.k, self.n_aln, self.ws, self.hits,
                               self.n_hits, self.alns, self.ops, self.stride, stream)

    def fetch(self):
        """Copies the last results to the host (synchronises)."""
        nh = int(self.n_hits.cpu()[0])
        hits = np.frombuffer(self.hits.cpu().numpy().tobytes(), dtype=HIT_DTYPE)[:nh].copy()
        na = min(self.n_aln, nh)
        alns = np.frombuffer(self.alns.cpu().numpy().tobytes(), dtype=ALN_DTYPE)[:na].copy()
        ops = self.ops.cpu().numpy().view(np.uint32)
        chunks, off = [], 0
        for i in range(na):
            a = alns[i]
            chunks.append(ops[a["ops_off"]:a["ops_off"] + a["n_ops"]])
            alns[i]["ops_off"] = off
            off += a["n_ops"]
        return Result(hits, alns, np.concatenate(chunks) if chunks else np.zeros(0, np.uint32))


def _as_bytes(q):
    return q if type(q) is bytes else q.encode() if isinstance(q, str) else bytes(q)


def _pack_queries(queries):
    """(concatenated ASCII bytes as a read-only uint8 array, int64 offsets) of
    a list of queries."""
    bs = list(map(_as_bytes, queries))
    off = np.zeros(len(bs) + 1, dtype=np.int64)
    np.cumsum(np.fromiter(map(len, bs), dtype=np.int64, count=len(bs)), out=off[1:])
    return np.frombuffer(b"".join(bs), dtype=np.uint8), off


def _params_array(params, nq):
    """ctypes array of hs_params: one shared entry or one per query."""
    if params is None or isinstance(params, Params):
        plist = [params or Params()]
    else:
        plist = list(params)
        if len(plist) not in (1, nq):
            raise ValueError("params must be one Params or one per query")
    arr = (_CParams * len(plist))(*[p.c() for p in plist])
    return arr, len(plist), plist


def _split_batch(nq, k, n_aln, hits, n_hits, alns, n_alns, ops):
    out = []
    for q in range(nq):
        h = hits[q * k:q * k + n_hits[q]].copy()
        if n_aln > 0:
            a = alns[q * n_aln:q * n_aln + n_alns[q]].copy()
            o0 = int(a["ops_off"][0]) if len(a) else 0
            o1 = int(a["ops_off"][-1] + a["n_ops"][-1]) if len(a) else 0
            a["ops_off"] -= o0
            out.append(Result(h, a, ops[o0:o1].copy()))
        else:
            out.append(Result(h, np.zeros(0, ALN_DTYPE), np.zeros(0, np.uint32)))
    return out


class Batch:
    """A batch handle (hs_batch_*): many queries scored in one persistent
    launch, ranked and aligned per query; results equal separate searches."""

    def __init__(self, db, max_nq, max_qlen, max_residues=None, k=50, n_aln=50):
        self.db, self.k, self.n_aln = db, k, n_aln
        self.max_nq, self.max_qlen = max_nq, max_qlen
        h = ctypes.c_void_p()
        _check(lib().hs_batch_create(db._h, max_nq, max_qlen,
                                     max_residues or max_nq * max_qlen, k, n_aln, ctypes.byref(h)))
        self._h = h
        self.nq = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().hs_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set(self, queries, params=None, stream=None):
        res, off = _pack_queries(queries)
        arr, n_p, _ = _params_array(params, len(queries))
        _check(lib().hs_batch_set(self._h, len(queries), res.ctypes.data_as(ctypes.c_void_p),
                                  off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr, n_p,
                                  _stream(stream)))
        self.nq = len(queries)
        self.qlens = np.diff(off)

    def schedule(self, copies=0, cap=0, chunk=0, stream=None):
        _check(lib().hs_batch_schedule(self._h, copies, cap, chunk, _stream(stream)))

    def get_schedule(self):
        v = [ctypes.c_int32() for _ in range(5)]
        _check(lib().hs_batch_get_schedule(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("copies", "cap", "chunk", "grid", "n_items"), [x.value for x in v]))

    def get_launch(self):
        """The scoring launch the schedule selects: LDS record kind, wavefronts
        per workgroup, high-ILP letter loop, one pair per wavefront."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(lib().hs_batch_get_launch(self._h, *[ctypes.byref(x) for x in v]))
        return dict(zip(("record", "waves", "ilp", "one_pair"), [x.value for x in v]))

    def tune(self, reps=2, stream=None):
        ms = ctypes.c_float()
        _check(lib().hs_batch_tune(self._h, _stream(stream), reps, ctypes.byref(ms)))
        return ms.value

    def run(self, stream=None, graph=False):
        fn = lib().hs_batch_run_graph if graph else lib().hs_batch_run
        _check(fn(self._h, _stream(stream)))

    def score(self, d_cells=None, stream=None):
        _check(lib().hs_batch_score(self._h, _stream(stream),
                                    d_cells.data_ptr() if d_cells is not None else None))

    def results(self, stream=None):
        """Per-query Result list of the last run (synchronises)."""
        nq, k, na = self.nq, self.k, self.n_aln
        hits = np.zeros(nq * k, dtype=HIT_DTYPE)
        n_hits = np.zeros(nq, dtype=np.int32)
        alns = np.zeros(max(nq * na, 1), dtype=ALN_DTYPE)
        n_alns = np.zeros(nq, dtype=np.int32)
        cap = max(1, int(sum(na * (2 * int(L) + 2) for L in self.qlens)))
        ops = np.zeros(cap, dtype=np.uint32)
        used = ctypes.c_int64()
        P = ctypes.POINTER(ctypes.c_int32)
        _check(lib().hs_batch_results(self._h, _stream(stream), hits.ctypes.data,
                                      n_hits.ctypes.data_as(P), alns.ctypes.data,
                                      n_alns.ctypes.data_as(P), ops.ctypes.data, cap,
                                      ctypes.byref(used)))
        return _split_batch(nq, k, na, hits, n_hits, alns, n_alns, ops)

    def scores(self, stream=None):
        """(scores, rounds): host int32 arrays of shape (nq, n_targets)."""
        n = self.db.n_targets
        sc = np.zeros((self.nq, max(n, 1)), dtype=np.int32)
        rd = np.zeros((self.nq, max(n, 1)), dtype=np.int32)
        _check(lib().hs_batch_scores(self._h, _stream(stream), sc.ctypes.data, rd.ctypes.data))
        return sc[:, :n], rd[:, :n]


def search_batch(db, queries, params=None, k=50, n_aln=50, stream=None):
    """hs_search_batch: one-shot batch search, per-query Result list."""
    nq = len(queries)
    res, off = _pack_queries(queries)
    arr, n_p, _ = _params_array(params, nq)
    hits = np.zeros(nq * k, dtype=HIT_DTYPE)
    n_hits = np.zeros(nq, dtype=np.int32)
    alns = np.zeros(max(nq * n_aln, 1), dtype=ALN_DTYPE)
    n_alns = np.zeros(nq, dtype=np.int32)
    cap = max(1, int(n_aln * (2 * np.diff(off) + 2).sum()))
    ops = np.zeros(cap, dtype=np.uint32)
    used = ctypes.c_int64()
    P = ctypes.POINTER(ctypes.c_int32)
    _check(lib().hs_search_batch(db._h, nq, res.ctypes.data_as(ctypes.c_void_p),
                                 off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), arr, n_p, k,
                                 n_aln, _stream(stream), hits.ctypes.data, n_hits.ctypes.data_as(P),
                                 alns.ctypes.data, n_alns.ctypes.data_as(P), ops.ctypes.data, cap,
                                 ctypes.byref(used)))
    return _split_batch(nq, k, n_aln, hits, n_hits, alns, n_alns, ops)


@dataclasses.dataclass(slots=True)
class Alignment:
    score: int
    round: int
    ops: np.ndarray           # uint32 run-length ops, oriented (query, target)


def align_batch(pairs, params=None, stream=None):
    """hs_align_batch: the pairwise mode of Fig. 1 (every overlapping
    placement, best of params.rounds rounds) for a list of (query, target)
    pairs; pair i's draws are keyed by i.  Returns a list of Alignment."""
    n = len(pairs)
    qres, qoff = _pack_queries([q for q, _ in pairs])
    tres, toff = _pack_queries([t for _, t in pairs])
    p = (params or Params()).c()
    scores = np.zeros(n, dtype=np.int32)
    rounds = np.zeros(n, dtype=np.int32)
    cap = max(1, int(np.diff(qoff).sum() + np.diff(toff).sum()))
    ops = np.zeros(cap, dtype=np.uint32)
    ops_off = np.zeros(n + 1, dtype=np.int64)
    used = ctypes.c_int64()
    P = ctypes.POINTER(ctypes.c_int32)
    P64 = ctypes.POINTER(ctypes.c_int64)
    _check(lib().hs_align_batch(n, qres.ctypes.data_as(ctypes.c_void_p), qoff.ctypes.data_as(P64),
                                tres.ctypes.data_as(ctypes.c_void_p), toff.ctypes.data_as(P64),
                                ctypes.byref(p), _stream(stream), scores.ctypes.data_as(P),
                                rounds.ctypes.data_as(P), ops.ctypes.data, cap,
                                ops_off.ctypes.data_as(P64), ctypes.byref(used)))
    # one buffer holds every pair's ops; each Alignment keeps a view of its run
    o = ops_off.tolist()
    return list(map(Alignment, scores.tolist(), rounds.tolist(),
                    [ops[a:b] for a, b in zip(o[:-1], o[1:])]))


def align_workspace_bytes(n, rounds):
    """Device workspace bytes of align_batch_dev (hs_align_workspace_bytes)."""
    b = lib().hs_align_workspace_bytes(n, rounds)
    if b <= 0:
        raise HSError(HS_EINVAL, "n or rounds out of range")
    return int(b)


def align_batch_dev(d_codes, qoff, toff, params, d_ws, d_scores, d_rounds, d_ops, d_n_ops,
                    stream=None):
    """Queues hs_align_batch_dev: pair i's query d_codes[qoff[i]:qoff[i+1]]
    against its target d_codes[toff[i]:toff[i+1]] (device uint8 codes, host
    int64 offsets); results into the device tensors (d_rounds may be None),
    pair i's ops from (qoff[i] - qoff[0]) + (toff[i] - toff[0]) on."""
    qoff = np.ascontiguousarray(qoff, dtype=np.int64)
    toff = np.ascontiguousarray(toff, dtype=np.int64)
    p = (params or Params()).c()
    P64 = ctypes.POINTER(ctypes.c_int64)
    _check(lib().hs_align_batch_dev(len(qoff) - 1, d_codes.data_ptr(), qoff.ctypes.data_as(P64),
                                    toff.ctypes.data_as(P64), ctypes.byref(p), _stream(stream),
                                    d_ws.data_ptr(), d_ws.numel() * d_ws.element_size(),
                                    d_scores.data_ptr(),
                                    d_rounds.data_ptr() if d_rounds is not None else None,
                                    d_ops.data_ptr(), d_n_ops.data_ptr()))


def align(query, target, params=None, stream=None):
    """hs_align: one pair in the pairwise mode (draws keyed by index 0)."""
    q = query.encode() if isinstance(query, str) else bytes(query)
    t = target.encode() if isinstance(target, str) else bytes(target)
    p = (params or Params()).c()
    cap = max(1, len(q) + len(t))
    ops = np.zeros(cap, dtype=np.uint32)
    sc, rd, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().hs_align(q, len(q), t, len(t), ctypes.byref(p), _stream(stream), ctypes.byref(sc),
                          ctypes.byref(rd), ops.ctypes.data, cap, ctypes.byref(n)))
    return Alignment(sc.value, rd.value, ops[:n.value].copy())


class Server:
    """A serving loop (hs_server_*): queries submitted one at a time are
    searched in continuous batches by native worker threads, up to `workers`
    batches in flight."""

    def __init__(self, db, max_batch=64, max_qlen=2000, max_residues=None, k=500, n_aln=50,
                 workers=2):
        self.db, self.k, self.n_aln, self.max_qlen = db, k, n_aln, max_qlen
        h = ctypes.c_void_p()
        _check(lib().hs_server_create_workers(db._h, max_batch, max_qlen,
                                              max_residues or max_batch * max_qlen, k, n_aln,
                                              workers, ctypes.byref(h)))
        self._h = h
        self._qlen = {}
        self._params = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().hs_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, query, tag, params=None):
        q = query.encode() if isinstance(query, str) else bytes(query)
        p = (params or Params()).c()
        _check(lib().hs_server_submit(self._h, q, len(q), ctypes.byref(p), tag))
        self._qlen[tag] = len(q)

    def poll(self, max_tags=1024, timeout_ms=0):
        tags = (ctypes.c_uint64 * max_tags)()
        n = ctypes.c_int32()
        _check(lib().hs_server_poll(self._h, tags, max_tags, ctypes.byref(n), timeout_ms))
        return [int(tags[i]) for i in range(n.value)]

    def result(self, tag):
        """(Result, timing dict) of a finished query; claims it."""
        k, na = self.k, self.n_aln
        hits = np.zeros(k, dtype=HIT_DTYPE)
        alns = np.zeros(max(na, 1), dtype=ALN_DTYPE)
        cap = max(1, na * (2 * self._qlen.pop(tag, self.max_qlen) + 2))
        ops = np.zeros(cap, dtype=np.uint32)
        nh, nal, used = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        t = ServerTiming()
        _check(lib().hs_server_result(self._h, tag, hits.ctypes.data, ctypes.byref(nh),
                                      alns.ctypes.data, ctypes.byref(nal), ops.ctypes.data, cap,
                                      ctypes.byref(used), ctypes.byref(t)))
        n_a = nal.value if na > 0 else 0
        timing = {f: getattr(t, f) for f, _ in ServerTiming._fields_ if f != "pad_"}
        return Result(hits[:nh.value].copy(), alns[:n_a].copy(), ops[:used.value].copy()), timing

    def stats(self):
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().hs_server_stats(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(pending=a.value, batches=b.value, served=c.value)
