"""Pins of the k-mer oracle against textbook facts of DNA k-mers (no GPU).

The k-mer keys are the nodes of the de Bruijn graphs the method was built for (Section 1).
These pins fix the encoding and the reverse complement by hand-worked values and by identities
a wrong implementation would break (complement pairs, involution, strand symmetry)."""
import numpy as np

from oracle import kmers as K


def pack(text: str) -> np.ndarray:
    """2-bit packing written independently of the oracle's decoder: 32 bases per word, first base
    in the top two bits."""
    words = np.zeros((len(text) + 31) // 32, dtype=np.uint64)
    for i, c in enumerate(text):
        words[i // 32] |= np.uint64("ACGT".index(c)) << np.uint64(62 - 2 * (i % 32))
    return words


def test_encoding_first_base_most_significant():
    # C=1, G=2, T=3: CGT = 1*16 + 2*4 + 3 = 27, ACG = 0*16 + 1*4 + 2 = 6
    assert K.encode("CGT") == 27
    assert K.encode("ACG") == 6
    assert K.encode("A" * 31) == 0
    assert K.encode("T" * 31) == 4 ** 31 - 1


def test_reverse_complement_textbook_values():
    # the reverse complement of CGT is ACG (reverse TGC, complement ACG)
    assert K.reverse_complement("CGT") == "ACG"
    assert K.canonical("CGT") == 6
    assert K.reverse_complement("AACCGGTT") == "AACCGGTT"   # a reverse-complement palindrome
    assert K.reverse_complement("GATTACA") == "TGTAATC"


def test_reverse_complement_is_an_involution_and_strand_symmetric():
    rng = np.random.default_rng(1)
    for _ in range(200):
        k = int(rng.integers(1, 33))
        s = "".join("ACGT"[v] for v in rng.integers(0, 4, size=k))
        rc = K.reverse_complement(s)
        assert K.reverse_complement(rc) == s
        assert K.canonical(s) == K.canonical(rc)
        # complement pairs: A-T and C-G sum to 3 position by position
        assert all("ACGT".index(a) + "ACGT".index(b) == 3 for a, b in zip(s, rc[::-1]))
        if k % 2:
            assert rc != s   # odd k: no reverse-complement palindromes (the middle base would be its own complement)


def test_decode_inverts_the_packing_across_word_boundaries():
    rng = np.random.default_rng(2)
    text = "".join("ACGT"[v] for v in rng.integers(0, 4, size=150))
    assert K.decode(pack(text), len(text)) == text


def test_canonical_kmers_of_a_worked_sequence():
    text = "ACGTTGCAAGT"
    got = K.canonical_kmers(pack(text), len(text), 4)
    want = []
    for p in range(len(text) - 3):
        s = text[p:p + 4]
        comp = "".join({"A": "T", "C": "G", "G": "C", "T": "A"}[c] for c in reversed(s))
        want.append(min(K.encode(s), K.encode(comp)))
    assert got.tolist() == want
    # ACGT is its own reverse complement; CGTT vs AACG: AACG = 0*64 + 0*16 + 1*4 + 2 = 6
    assert got[0] == K.encode("ACGT")
    assert got[1] == 6


def test_first_occurrences_keep_order_and_stop_at_target():
    keys = [5, 3, 5, 9, 3, 3, 7, 9, 1]
    assert K.first_occurrences(keys, 100).tolist() == [5, 3, 9, 7, 1]
    assert K.first_occurrences(keys, 3).tolist() == [5, 3, 9]
    assert K.first_occurrences([], 3).tolist() == []
