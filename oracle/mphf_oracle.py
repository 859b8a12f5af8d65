"""CPU oracle for the cascading-bit-array minimal perfect hash function of
Limasset, Rizk, Chikhi and Peterlongo, "Fast and scalable minimal perfect
hashing for massive key sets" (arXiv 1702.03154).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only the tests, the smoke check of ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constant tables); the only module both
sides use is the seeded input generator, which holds none of the method's
arithmetic.

It is the plain sequential method written from the paper's definitions, in
numpy, with no blocking or reordering:

* level d hashes every key of F_d into a bit array of m_d = ceil(gamma*|F_d|)
  positions (Section 2.2, "Faster query and construction times (parameter
  gamma)"); A_d[i] = 1 iff exactly one key lands on i and C_d[i] = 1 iff two
  or more do (Section 2.2, "Collision detection"; Algorithm 2);
* F_{d+1} holds the keys of F_d whose bit in A_d is 0 (Section 2.1;
  Algorithm 1); the loop stops when F_{d+1} is empty or after D levels, and
  the keys left over go to a table H with labels N-|L|+1 .. N (Section 3,
  "Termination"; the footnote of Algorithm 1);
* the label of a key is the number of ones of the concatenated array A before
  its bit, plus one (Section 2.1, the query paragraph and Figure 1; Section
  2.2, "Minimality"; Algorithm 3);
* the rank table keeps a 64-bit count of the ones before every 512th
  position (Section 3.1, "Rank structure").

Readings where the paper is silent or garbled (each also listed in the design
notes of the repository):

* Hash family.  The paper only says "xor-shift based" (Section 3.3).  Here the
  level-d hash is h_d(x) = fmix64(x XOR s_d), where fmix64 is the 64-bit
  finalizer of MurmurHash3 and s_d is output d of a SplitMix64 stream seeded
  with the build seed; the position is h_d(x) mod m_d, the paper's ``mod``
  (Algorithms 1-3).  These values are a project definition: parity unpinned
  by the paper (only the structural pins of the tests apply to them).
* m_d = ceil(gamma * n_d) evaluated in IEEE double (the paper does not say
  how gamma*|F_d| is rounded).
* Algorithm 2's three ``if``s are read as ``if / else if`` so that the final
  state matches the formal rules of Section 2.2.
* The minimal value: Section 2.2 writes the sum with a misplaced bracket and
  Algorithm 3 sums |A_j| (a size, not a weight).  Read as
  sum_{i<d} weight(A_i) + rank, with the rank 1-based (inclusive), which is
  what Figure 1 prints (labels in [1, N]).
* A is the concatenation of the levels, each starting on a 64-bit boundary
  with zero padding (Section 2.1 only says "concatenating").
* Leftover keys get the labels N-|L|+1 .. N in ascending key order; equal
  leftover keys mean duplicate input keys, which is an error.
* A non-member key gets whatever the level walk reaches, else its H label if
  present, else 0 (the footnote of Algorithm 3 allows any value).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
DEFAULT_MAX_LEVELS = 25      # Section 3, "Termination": D = 25
DEFAULT_RANK_SAMPLE = 512    # Section 3.1: one counter every 512 positions


class DuplicateKeysError(ValueError):
    """Two equal keys were given; they collide at every level (Section 4 assumes unique keys)."""


# ---------------------------------------------------------------- hash family

def level_seeds(seed: int, count: int) -> list[int]:
    """s_0 .. s_{count-1}: the outputs of a SplitMix64 stream whose state starts at ``seed``."""
    out = []
    state = seed & MASK64
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        out.append(z ^ (z >> 31))
    return out


def fmix64(x: np.ndarray) -> np.ndarray:
    """MurmurHash3's 64-bit finalizer on a uint64 array (wrapping arithmetic)."""
    x = x.astype(np.uint64, copy=True)
    x ^= x >> np.uint64(33)
    x *= np.uint64(0xFF51AFD7ED558CCD)
    x ^= x >> np.uint64(33)
    x *= np.uint64(0xC4CEB9FE1A85EC53)
    x ^= x >> np.uint64(33)
    return x


def level_positions(keys: np.ndarray, level_seed: int, m: int) -> np.ndarray:
    """pos_d(x) = fmix64(x XOR s_d) mod m_d (Algorithms 1-3 reduce the hash with ``mod``)."""
    with np.errstate(over="ignore"):
        h = fmix64(np.asarray(keys, dtype=np.uint64) ^ np.uint64(level_seed))
    return h % np.uint64(m)


def level_size(gamma: float, n: int) -> int:
    """m_d = ceil(gamma * n_d), the product taken in IEEE double (Section 2.2, parameter gamma)."""
    return int(math.ceil(float(gamma) * float(n)))


# ---------------------------------------------------------------- the structure

@dataclass
class Level:
    n: int                 # |F_d|
    m: int                 # |A_d| = |C_d|
    seed: int              # s_d
    offset: int            # bit offset of A_d inside the concatenated A
    A: np.ndarray          # bool[m]
    C: np.ndarray          # bool[m]

    @property
    def weight(self) -> int:
        return int(self.A.sum())


@dataclass
class Structure:
    N: int
    gamma: float
    seed: int
    max_levels: int
    rank_sample: int
    levels: list[Level] = field(default_factory=list)
    total_bits: int = 0                 # M: bits of the concatenated A, padding included
    words: np.ndarray = None            # uint64[M/64]: the concatenated A
    ones_before: np.ndarray = None      # int64[M+1]: ones of A strictly before each position
    rank: np.ndarray = None             # uint64[ceil(M/rank_sample)]
    fallback_keys: np.ndarray = None    # uint64[|L|], ascending
    fallback_labels: np.ndarray = None  # uint64[|L|]: N-|L|+1 .. N

    @property
    def num_levels(self) -> int:
        return len(self.levels)

    @property
    def bits_per_key(self) -> float:
        """Size of A plus the rank counters plus H (two 64-bit words per leftover) per key."""
        if self.N == 0:
            return 0.0
        bits = self.total_bits + 64 * len(self.rank) + 128 * len(self.fallback_keys)
        return bits / self.N


def _default_positions(seeds):
    def pos(keys, d, m):
        return level_positions(keys, seeds[d], m)
    return pos


def build(keys, gamma: float, seed: int = 0, max_levels: int = DEFAULT_MAX_LEVELS,
          rank_sample: int = DEFAULT_RANK_SAMPLE, positions=None) -> Structure:
    """Build the structure for ``keys`` (distinct uint64) following Algorithms 1 and 2.

    ``positions(keys, d, m) -> uint64 array`` replaces the level hash; only the
    tests use it, to replay the worked example of Figure 1 with positions that
    the caption fixes.
    """
    keys = np.ascontiguousarray(np.asarray(keys, dtype=np.uint64))
    if not (gamma >= 1.0):          # also rejects NaN
        raise ValueError("gamma must be a number >= 1 (Section 2.2)")
    if max_levels < 1 or rank_sample not in (512, 1024):
        raise ValueError("max_levels >= 1 and rank_sample in {512, 1024}")
    N = len(keys)
    seeds = level_seeds(seed, max_levels)
    pos_fn = positions if positions is not None else _default_positions(seeds)
    st = Structure(N=N, gamma=float(gamma), seed=seed, max_levels=max_levels,
                   rank_sample=rank_sample)

    # Algorithm 1: cascade of levels.
    F = keys
    offset = 0
    for d in range(max_levels):
        if len(F) == 0:
            break
        n = len(F)
        m = level_size(gamma, n)
        p = np.asarray(pos_fn(F, d, m), dtype=np.uint64)
        # Algorithm 2 (ArrayFill): the final state is A = [exactly one key], C = [two or more].
        hits = np.bincount(p.astype(np.int64), minlength=m)
        A = hits == 1
        C = hits >= 2
        st.levels.append(Level(n=n, m=m, seed=seeds[d], offset=offset, A=A, C=C))
        offset += 64 * ((m + 63) // 64)
        # Algorithm 1, filter: keys whose bit in A_d is 0 go on to F_{d+1}.
        F = F[~A[p]]

    # Termination (Section 3): leftovers go to H, labelled N-|L|+1 .. N in key order.
    L = np.sort(F)
    if len(L) > 1 and bool(np.any(L[1:] == L[:-1])):
        raise DuplicateKeysError("duplicate keys in the input")
    st.fallback_keys = L
    st.fallback_labels = np.arange(N - len(L) + 1, N + 1, dtype=np.uint64)

    # The concatenated A, each level on a 64-bit boundary.
    st.total_bits = offset
    bits = np.zeros(offset, dtype=bool)
    for lev in st.levels:
        bits[lev.offset:lev.offset + lev.m] = lev.A
    st.words = np.packbits(bits, bitorder="little").view(np.uint64) if offset else np.zeros(0, np.uint64)
    st.ones_before = np.concatenate([[0], np.cumsum(bits, dtype=np.int64)])

    # Rank table (Section 3.1): ones before every rank_sample-th position.
    nb = -(-offset // rank_sample)
    st.rank = st.ones_before[np.arange(nb, dtype=np.int64) * rank_sample].astype(np.uint64)
    return st


def lookup(st: Structure, queries, positions=None) -> np.ndarray:
    """Algorithm 3 for every query: the first level whose bit is set gives
    label = (ones of A before that bit) + 1; otherwise H, otherwise 0."""
    q = np.ascontiguousarray(np.asarray(queries, dtype=np.uint64))
    out = np.zeros(len(q), dtype=np.uint64)
    seeds = [lev.seed for lev in st.levels]
    pos_fn = positions if positions is not None else _default_positions(seeds)
    todo = np.arange(len(q), dtype=np.int64)
    for d, lev in enumerate(st.levels):
        if len(todo) == 0:
            break
        p = np.asarray(pos_fn(q[todo], d, lev.m), dtype=np.uint64).astype(np.int64)
        hit = lev.A[p]
        g = lev.offset + p[hit]
        out[todo[hit]] = (st.ones_before[g] + 1).astype(np.uint64)
        todo = todo[~hit]
    if len(todo) and len(st.fallback_keys):
        i = np.searchsorted(st.fallback_keys, q[todo])
        i = np.minimum(i, len(st.fallback_keys) - 1)
        found = st.fallback_keys[i] == q[todo]
        out[todo[found]] = st.fallback_labels[i[found]]
    return out


def level_of(st: Structure, queries) -> np.ndarray:
    """The level at which each query stops (0-based); num_levels for H or fall-through."""
    q = np.asarray(queries, dtype=np.uint64)
    lvl = np.full(len(q), st.num_levels, dtype=np.int64)
    todo = np.arange(len(q), dtype=np.int64)
    for d, lev in enumerate(st.levels):
        p = level_positions(q[todo], lev.seed, lev.m).astype(np.int64)
        hit = lev.A[p]
        lvl[todo[hit]] = d
        todo = todo[~hit]
    return lvl


def collision_words(st: Structure, d: int) -> np.ndarray:
    """C_d packed like A_d (bit i of word j = position 64j+i), for parity of the debug export."""
    lev = st.levels[d]
    bits = np.zeros(64 * ((lev.m + 63) // 64), dtype=bool)
    bits[:lev.m] = lev.C
    return np.packbits(bits, bitorder="little").view(np.uint64)


def level_words(st: Structure, d: int) -> np.ndarray:
    """The words of A_d inside the concatenated A."""
    lev = st.levels[d]
    w0 = lev.offset // 64
    return st.words[w0:w0 + (lev.m + 63) // 64]
