"""Oracle for the k-mer workload: test infrastructure only (never imported by the product).

Written from the definitions with strings, not bit arithmetic:
* a 2-bit packed sequence decodes to a string over ACGT, 32 bases per 64-bit word, the first
  base of a word in its two most significant bits (A=0, C=1, G=2, T=3);
* the k-mer at p is the substring of length k at p; its reverse complement is the reversed
  string with A<->T and C<->G swapped; a k-mer encodes as the base-4 number of its letters,
  first letter most significant; the canonical k-mer is the smaller encoding of the two
  (de Bruijn graph nodes of the bioinformatics use in Section 1);
* the first occurrences of a key sequence keep each distinct key at its first position, in
  order, up to a target count.

Pure Python loops: small inputs only.
"""
from __future__ import annotations

import numpy as np

LETTERS = "ACGT"
_COMPLEMENT = str.maketrans("ACGT", "TGCA")


def decode(seq_words, nbases: int) -> str:
    out = []
    for i in range(nbases):
        w = int(seq_words[i // 32])
        shift = 62 - 2 * (i % 32)
        out.append(LETTERS[(w >> shift) & 3])
    return "".join(out)


def encode(s: str) -> int:
    v = 0
    for c in s:
        v = 4 * v + LETTERS.index(c)
    return v


def reverse_complement(s: str) -> str:
    return s[::-1].translate(_COMPLEMENT)


def canonical(s: str) -> int:
    return min(encode(s), encode(reverse_complement(s)))


def canonical_kmers(seq_words, nbases: int, k: int) -> np.ndarray:
    text = decode(seq_words, nbases)
    return np.array([canonical(text[p:p + k]) for p in range(nbases - k + 1)], dtype=np.uint64)


def first_occurrences(keys, target: int) -> np.ndarray:
    seen, out = set(), []
    for x in keys:
        x = int(x)
        if x in seen:
            continue
        seen.add(x)
        out.append(x)
        if len(out) == target:
            break
    return np.array(out, dtype=np.uint64)
