"""Pins on the counter-based generator behind random() of Fig. 1:
Philox4x64-10 (Salmon et al., SC'11) against its published known answers and
against numpy's independent implementation, and the draw indexing."""
import os

import numpy as np

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")
M64 = 2**64 - 1


def test_philox_known_answers():
    n = 0
    for line in open(os.path.join(GOLD, "philox4x64_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        assert O.philox4x64_10(w[0:4], w[4:6]) == w[6:10]
        n += 1
    assert n == 3


def _numpy_block(ctr, key):
    # numpy's Philox steps its 256-bit counter by one before each block
    c = list(ctr)
    for i in range(4):
        c[i] = (c[i] - 1) & M64
        if c[i] != M64:
            break
    g = np.random.Philox(counter=np.array(c, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def test_philox_vs_numpy():
    rng = np.random.default_rng(1)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(1, 2**63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert O.philox4x64_10(ctr, key) == _numpy_block(ctr, key)


def test_draw_indexing_vs_numpy():
    """Draw d of (target, round) is 16-bit chunk d%4 of word (d/4)%4 of the
    block with counter (target, round, d/16, 0) and key (seed, 0)."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        seed = int(rng.integers(0, 2**63))
        tid = int(rng.integers(0, 10**6)) if _ else 0
        rnd = int(rng.integers(0, 30))
        for d in list(range(40)) + [int(rng.integers(0, 5000))]:
            words = _numpy_block([tid, rnd, d // 16, 0], [seed, 0])
            chunk = (words[(d // 4) % 4] >> (16 * (d % 4))) & 0xFFFF
            assert O.draw(seed, tid, rnd, d) == chunk


def test_draws_roughly_uniform():
    u = np.array([O.draw(7, t, 0, d) for t in range(200) for d in range(20)]) / 65536.0
    assert abs(u.mean() - 0.5) < 0.02 and abs(u.var() - 1 / 12) < 0.01
