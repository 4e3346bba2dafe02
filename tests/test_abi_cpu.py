"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/hs.h declares, and its host-only calls behave."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hs.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(hs_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["hs_params_default", "hs_db_load", "hs_db_free", "hs_search", "hs_search_dev",
              "hs_score_dev", "hs_last_error", "hs_encode", "hs_workspace_bytes",
              "hs_search_batch", "hs_batch_create", "hs_batch_set", "hs_batch_run",
              "hs_batch_run_graph", "hs_batch_tune", "hs_batch_results", "hs_batch_free"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1508_06561_amd as H
    L = H.lib()
    for n in declared_functions():
        assert hasattr(L, n), f"libhs.so does not export {n}"


def test_defaults_are_the_papers_search_setting():
    import paper_1508_06561_amd as H
    p = H.params_default()
    assert (p.gop, p.gep, p.pgp) == (10, 5, 0)
    assert (p.lfactor_q16, p.sfactor_q16, p.minfactor_q16) == (32768, 65536, 32768)
    assert p.rounds == 1 and p.min_score == -(2**31) and p.seed == 0


def test_builtin_matrix_equals_oracle_table():
    import paper_1508_06561_amd as H
    assert (H.builtin_matrix() == O.blosum62()).all()


def test_encode_matches_oracle_and_rejects():
    import paper_1508_06561_amd as H
    s = "ARNDCQEGHILKMFPSTWYVBZX*arndjou"
    assert (H.encode(s) == O.encode(s)).all()
    for bad in ["AC-D", "A1", "A C", "\x00"]:
        with pytest.raises(H.HSError) as e:
            H.encode(bad)
        assert e.value.code == -1


def test_argument_errors_before_device_use():
    import paper_1508_06561_amd as H
    L = H.lib()
    p = H.Params().c()
    hits = np.zeros(4, dtype=H.hs.HIT_DTYPE)
    nh = ctypes.c_int32()
    rc = L.hs_search(None, b"ACD", 3, ctypes.byref(p), 4, 0, None, hits.ctypes.data,
                     ctypes.byref(nh), None, None, None, 0, None)
    assert rc == H.hs.HS_EINVAL and b"db" in L.hs_last_error()
    bad = H.Params(gop=-1).c()
    rc = L.hs_score_dev(ctypes.c_void_p(1), ctypes.c_void_p(1), 3, ctypes.byref(bad), None,
                        ctypes.c_void_p(1), 1 << 30, ctypes.c_void_p(1), None, None)
    assert rc == H.hs.HS_EINVAL
    bad = H.Params(lfactor_q16=70000).c()
    rc = L.hs_score_dev(ctypes.c_void_p(1), ctypes.c_void_p(1), 3, ctypes.byref(bad), None,
                        ctypes.c_void_p(1), 1 << 30, ctypes.c_void_p(1), None, None)
    assert rc == H.hs.HS_EINVAL
    wide = np.zeros((24, 24), np.int8)
    wide[0, 0] = 20
    bad = H.Params(matrix=wide)
    rc = L.hs_score_dev(ctypes.c_void_p(1), ctypes.c_void_p(1), 3, ctypes.byref(bad.c()), None,
                        ctypes.c_void_p(1), 1 << 30, ctypes.c_void_p(1), None, None)
    assert rc == H.hs.HS_EINVAL
    rc = L.hs_score_dev(ctypes.c_void_p(1), ctypes.c_void_p(1), 0, ctypes.byref(p), None,
                        ctypes.c_void_p(1), 1 << 30, ctypes.c_void_p(1), None, None)
    assert rc == H.hs.HS_EINVAL
    assert L.hs_workspace_bytes(None, 1, 10, 10, 1) == 0


def test_batch_argument_errors_before_device_use():
    import paper_1508_06561_amd as H
    L = H.lib()
    E = H.hs.HS_EINVAL
    h = ctypes.c_void_p()
    assert L.hs_batch_create(None, 4, 100, 400, 10, 5, ctypes.byref(h)) == E
    assert b"db" in L.hs_last_error()
    fake = ctypes.c_void_p(1)
    # sizes are checked before the database is touched
    assert L.hs_batch_create(fake, 0, 100, 400, 10, 5, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, H.hs.MAX_BATCH + 1, 100, 400, 10, 5, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, 0, 400, 10, 5, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, H.hs.MAX_QUERY + 1, 400, 10, 5, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, 100, 401, 10, 5, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, 100, 400, 0, 0, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, 100, 400, 10, 11, ctypes.byref(h)) == E
    assert L.hs_batch_create(fake, 4, 100, 400, 10, 5, None) == E
    for fn in (L.hs_batch_run, L.hs_batch_run_graph):
        assert fn(None, None) == E
    assert L.hs_batch_score(None, None, None) == E
    assert L.hs_batch_set(None, 1, None, None, None, 1, None) == E
    assert L.hs_batch_schedule(None, 0, 0, 0, None) == E
    assert L.hs_batch_free(None) == 0
    p = H.Params().c()
    off = np.array([0, 3], np.int64)
    assert L.hs_search_batch(None, 1, b"ACD", off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             ctypes.byref(p), 1, 4, 0, None, None, None, None, None, None, 0,
                             None) == E


def test_server_argument_errors_before_device_use():
    import paper_1508_06561_amd as H
    L = H.lib()
    E = H.hs.HS_EINVAL
    h = ctypes.c_void_p()
    assert L.hs_server_create(None, 4, 100, 400, 10, 5, ctypes.byref(h)) == E
    assert L.hs_server_create(ctypes.c_void_p(1), 4, 100, 400, 10, 5, None) == E
    assert L.hs_server_create(ctypes.c_void_p(1), 0, 100, 400, 10, 5, ctypes.byref(h)) == E
    for n_workers in (0, H.hs.MAX_SERVER_WORKERS + 1):
        assert L.hs_server_create_workers(ctypes.c_void_p(1), 4, 100, 400, 10, 5, n_workers,
                                          ctypes.byref(h)) == E
    p = H.Params().c()
    assert L.hs_server_submit(None, b"ACD", 3, ctypes.byref(p), 1) == E
    n = ctypes.c_int32()
    tags = (ctypes.c_uint64 * 4)()
    assert L.hs_server_poll(None, tags, 4, ctypes.byref(n), 0) == E
    assert L.hs_server_stats(None, None, None, None) == E
    assert L.hs_server_free(None) == 0
    assert L.hs_params_check(ctypes.byref(p)) == 0
    assert L.hs_params_check(ctypes.byref(H.Params(gep=-1).c())) == E
    assert L.hs_params_check(ctypes.byref(H.Params(rounds=0).c())) == E


def test_server_rejects_a_footprint_that_cannot_admit_its_longest_query():
    """A query longer than max_residues could never be admitted and would
    block the queue behind it, so such a server is refused at creation
    (checked before any device work)."""
    import paper_1508_06561_amd as H
    L = H.lib()
    h = ctypes.c_void_p()
    rc = L.hs_server_create_workers(ctypes.c_void_p(1), 4, 100, 99, 10, 5, 2, ctypes.byref(h))
    assert rc == H.hs.HS_EINVAL and b"max_residues" in L.hs_last_error()
    rc = L.hs_server_create(ctypes.c_void_p(1), 4, 100, 50, 10, 5, ctypes.byref(h))
    assert rc == H.hs.HS_EINVAL
