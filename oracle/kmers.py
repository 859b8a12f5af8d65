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

Pure Python: a few million positions at most.
"""
from __future__ import annotations

import numpy as np

LETTERS = "ACGT"
_COMPLEMENT = str.maketrans("ACGT", "TGCA")
_TO_DIGITS = str.maketrans("ACGT", "0123")
_TO_LETTERS = str.maketrans("0123", "ACGT")


def decode(seq_words, nbases: int) -> str:
    """Each word written as its 32 base-4 digits, first digit most significant, then the digits
    0..3 read as A, C, G, T."""
    digits = "".join(np.base_repr(int(w), 4).rjust(32, "0") for w in seq_words[:(nbases + 31) // 32])
    return digits[:nbases].translate(_TO_LETTERS)


def encode(s: str) -> int:
    """The base-4 number whose digits are the letters of s (A=0, C=1, G=2, T=3), first letter most
    significant."""
    return int(s.translate(_TO_DIGITS), 4) if s else 0


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
