"""Seeded synthetic protein databases and queries.

Serves both the oracle and the HIP path (tests and benchmark) with the same
inputs, and holds none of the method's arithmetic.  The paper measured on
UniProt/Swiss-Prot (547,085 sequences) with short queries; none of that data
is used here.  Every input is drawn from seeded generators with the shape of
that workload instead:

* residues i.i.d. from the Robinson & Robinson background composition
  (20 standard letters);
* target lengths uniform or log-normal, as each workload states;
* planted homologs: a copy of a query with exactly ceil((1 - id) * |Q|)
  substituted positions, each replacement b != a drawn with probability
  proportional to p_b * 2^(B62[a][b] / 2) (the inverse of BLOSUM's half-bit
  log-odds definition), then a number of insertions/deletions (50/50) of short
  lengths (inserted letters from the background), then embedded at a random
  offset in a background flank whose total length is drawn from the database
  length distribution.

Databases are returned as (residues, offsets): residues is a uint8 array of
concatenated ASCII letters, offsets an int64 array of n + 1 boundaries.
"""
import dataclasses
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LETTERS20 = "ARNDCQEGHILKMFPSTWYV"
BASE_SEED = 150806561


def _read_counts():
    counts = {}
    with open(os.path.join(HERE, "rr_counts.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            a, c = line.split()
            counts[a] = int(c)
    return np.array([counts[a] for a in LETTERS20], dtype=np.float64)


def _read_matrix():
    rows = [l for l in open(os.path.join(HERE, "blosum62.txt")) if not l.startswith("#")]
    hdr = rows[0].split()
    m = np.zeros((24, 24), dtype=np.int64)
    for i, l in enumerate(rows[1:25]):
        parts = l.split()
        assert parts[0] == hdr[i]
        m[i] = [int(x) for x in parts[1:]]
    return "".join(hdr), m


_COUNTS = _read_counts()
BACKGROUND = _COUNTS / _COUNTS.sum()
_ALPHA24, _B62 = _read_matrix()
_ASCII20 = np.frombuffer(LETTERS20.encode(), dtype=np.uint8)

# substitution distribution p(b | a), b != a, proportional to p_b 2^(B[a][b]/2)
_SUB = np.zeros((20, 20))
for _a in range(20):
    w = BACKGROUND * np.power(2.0, _B62[:20, :20][_a] / 2.0)
    w[_a] = 0.0
    _SUB[_a] = w / w.sum()
_SUB_CDF = np.cumsum(_SUB, axis=1)


def background_probs():
    return BACKGROUND.copy()


def matrix_table():
    """(alphabet string, 24x24 int matrix) as read from the data file."""
    return _ALPHA24, _B62.copy()


def random_idx(rng, n):
    """n residue indices (0..19 over LETTERS20) drawn from the background."""
    return np.searchsorted(np.cumsum(BACKGROUND), rng.random(n), side="right").clip(0, 19).astype(np.uint8)


def random_protein(rng, n):
    """n ASCII residues drawn i.i.d. from the background composition."""
    return _ASCII20[random_idx(rng, n)]


def to_idx(ascii_seq):
    lut = np.full(256, 255, dtype=np.uint8)
    lut[_ASCII20] = np.arange(20, dtype=np.uint8)
    return lut[np.asarray(ascii_seq, dtype=np.uint8)]


def mutate(rng, query, identity, n_indels=(1, 5), indel_len=(1, 4)):
    """Homolog of `query` (ASCII uint8) at the given identity with indels."""
    idx = to_idx(query).copy()
    n = len(idx)
    n_sub = int(math.ceil((1.0 - identity) * n - 1e-9))
    pos = rng.choice(n, size=min(n_sub, n), replace=False)
    for p in pos:
        a = idx[p]
        b = int(np.searchsorted(_SUB_CDF[a], rng.random(), side="right"))
        idx[p] = min(b, 19)
    seq = list(idx)
    k = int(rng.integers(n_indels[0], n_indels[1] + 1))
    for _ in range(k):
        ln = int(rng.integers(indel_len[0], indel_len[1] + 1))
        at = int(rng.integers(0, max(1, len(seq))))
        if rng.random() < 0.5 or len(seq) <= ln + 1:
            seq[at:at] = list(random_idx(rng, ln))
        else:
            del seq[at:at + ln]
    return _ASCII20[np.array(seq, dtype=np.uint8)]


def embed(rng, core, total_len):
    """Place `core` at a random offset in a background flank of total_len."""
    if total_len <= len(core):
        return core
    off = int(rng.integers(0, total_len - len(core) + 1))
    return np.concatenate([random_protein(rng, off), core,
                           random_protein(rng, total_len - len(core) - off)])


def pack(seqs):
    """List of ASCII uint8 arrays -> (residues, offsets)."""
    lens = np.array([len(s) for s in seqs], dtype=np.int64)
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    return np.concatenate(seqs).astype(np.uint8) if seqs else np.zeros(0, np.uint8), offsets


def random_db(rng, lengths):
    """Background-only database with the given target lengths (vectorised)."""
    lengths = np.asarray(lengths, dtype=np.int64)
    offsets = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    return random_protein(rng, int(offsets[-1])), offsets


def lognormal_lengths(rng, n, median, sigma, lo, hi):
    return np.clip(np.rint(median * np.exp(sigma * rng.standard_normal(n))), lo, hi).astype(np.int64)


def plant(rng, residues, offsets, homologs):
    """Insert homolog sequences at random target indices.  Returns (residues,
    offsets, planted_ids)."""
    n_bg = len(offsets) - 1
    n = n_bg + len(homologs)
    slots = np.sort(rng.choice(n, size=len(homologs), replace=False))
    is_hom = np.zeros(n, dtype=bool)
    is_hom[slots] = True
    lens = np.empty(n, dtype=np.int64)
    lens[~is_hom] = np.diff(offsets)
    lens[is_hom] = [len(h) for h in homologs]
    new_off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=new_off[1:])
    out = np.empty(int(new_off[-1]), dtype=np.uint8)
    # background targets keep their order, in the non-homolog slots
    bg_slots = np.nonzero(~is_hom)[0]
    src_starts, dst_starts = offsets[:-1], new_off[bg_slots]
    if len(bg_slots):
        # vectorised segment copy
        seg_len = np.diff(offsets)
        rep = np.repeat(dst_starts - src_starts, seg_len)
        out[np.arange(len(residues)) + rep] = residues
    for s, h in zip(slots, homologs):
        out[new_off[s]:new_off[s + 1]] = h
    return out, new_off, slots


@dataclasses.dataclass
class Workload:
    name: str
    residues: np.ndarray          # concatenated ASCII database
    offsets: np.ndarray           # n + 1 boundaries
    queries: list                 # ASCII uint8 arrays
    planted: np.ndarray           # target ids holding planted homologs
    k: int                        # ranked hits reported per query
    n_aln: int                    # alignments reported per query
    seed: int
    arrivals: np.ndarray = None   # serving: arrival times (s), one per query

    @property
    def n_targets(self):
        return len(self.offsets) - 1

    @property
    def db_residues(self):
        return int(self.offsets[-1])


def tiny_db(seed=BASE_SEED, n_bg=2000, qlen=64, n_hom=20):
    """One 64-residue query vs 2,000 targets of length U[50, 500] plus 20
    homologs of the query at 30-90% identity with 1-5 indels of length 1-4."""
    rng = np.random.default_rng(seed)
    q = random_protein(rng, qlen)
    res, off = random_db(rng, rng.integers(50, 501, size=n_bg))
    homs = [embed(rng, mutate(rng, q, rng.uniform(0.3, 0.9)), int(rng.integers(50, 501)))
            for _ in range(n_hom)]
    res, off, planted = plant(rng, res, off, homs)
    return q, res, off, planted


def config_tiny():
    q, res, off, planted = tiny_db(BASE_SEED + 0)
    return Workload("tiny: 64-aa query vs 2,020 targets U[50,500]", res, off, [q], planted,
                    k=50, n_aln=50, seed=BASE_SEED + 0)


def config_full(n_bg=500_000, n_hom=200, seed=BASE_SEED + 1):
    """A 300-residue query vs 500,000 log-normal targets (median 300,
    sigma 0.6, clipped to 10-35,000) plus 200 planted homologs at 20-90%
    identity with indels; top 500 ranked, top 50 aligned."""
    rng = np.random.default_rng(seed)
    q = random_protein(rng, 300)
    res, off = random_db(rng, lognormal_lengths(rng, n_bg, 300, 0.6, 10, 35_000))
    homs = []
    for _ in range(n_hom):
        tl = int(lognormal_lengths(rng, 1, 300, 0.6, 10, 35_000)[0])
        homs.append(embed(rng, mutate(rng, q, rng.uniform(0.2, 0.9)), tl))
    res, off, planted = plant(rng, res, off, homs)
    return Workload("full: 300-aa query vs 500,200 log-normal targets", res, off, [q], planted,
                    k=500, n_aln=50, seed=seed)


def config_batched(nq=256, seed=BASE_SEED + 2):
    """256 queries of length U[30, 1000] against the tiny database."""
    q0, res, off, planted = tiny_db(BASE_SEED + 0)
    rng = np.random.default_rng(seed)
    qs = [random_protein(rng, int(n)) for n in rng.integers(30, 1001, size=nq)]
    return Workload("batched: 256 queries U[30,1000] vs the tiny database", res, off, qs, planted,
                    k=50, n_aln=50, seed=seed)


def config_long(nq=32, n_long=5000, n_hom_per_query=2, seed=BASE_SEED + 3):
    """32 queries of 2,000-5,000 residues vs the tiny database plus 5,000
    targets of 10,000-35,000 residues, with mutated copies of the queries
    planted in some of the long targets."""
    q0, res, off, _ = tiny_db(BASE_SEED + 0)
    rng = np.random.default_rng(seed)
    qs = [random_protein(rng, int(n)) for n in rng.integers(2000, 5001, size=nq)]
    lres, loff = random_db(rng, rng.integers(10_000, 35_001, size=n_long))
    homs = []
    for q in qs:
        for _ in range(n_hom_per_query):
            homs.append(embed(rng, mutate(rng, q, rng.uniform(0.3, 0.9), n_indels=(1, 10)),
                              int(rng.integers(10_000, 35_001))))
    lres, loff, lplanted = plant(rng, lres, loff, homs)
    allres = np.concatenate([res, lres])
    alloff = np.concatenate([off, loff[1:] + off[-1]])
    planted = lplanted + (len(off) - 1)
    return Workload("long: 32 queries U[2000,5000] vs tiny database + 5,064 targets U[10k,35k]",
                    allres, alloff, qs, planted, k=50, n_aln=50, seed=seed)


def config_serving(rate, duration_s=2.0, seed=BASE_SEED + 4):
    """Poisson arrivals at `rate` queries/s with log-normal query lengths
    (median 250, sigma 0.6, clipped to 20-2,000) against the tiny database;
    top 500 hits plus top-50 alignments per query."""
    q0, res, off, planted = tiny_db(BASE_SEED + 0)
    rng = np.random.default_rng(seed + int(rate))
    n = max(1, int(rng.poisson(rate * duration_s)))
    arrivals = np.sort(rng.uniform(0.0, duration_s, size=n))
    lens = lognormal_lengths(rng, n, 250, 0.6, 20, 2000)
    qs = [random_protein(rng, int(L)) for L in lens]
    return Workload(f"serving: Poisson {rate} q/s, |Q| log-normal median 250", res, off, qs,
                    planted, k=500, n_aln=50, seed=seed, arrivals=arrivals)
