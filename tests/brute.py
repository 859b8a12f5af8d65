"""Brute-force restatement of the method for tiny key sets (N <= 64).

It is written independently of the oracle and in a different form: a
sequential state machine over (A, C) per Algorithm 2 read with ``else if``
(Section 2.2, "Collision detection"), Python integers for the hash, a dict for
the level of each key, and labels counted bit by bit over the concatenated
array (Section 2.1 and Figure 1).  Used only to pin the oracle.
"""
M64 = (1 << 64) - 1


def sm64_stream(seed, count):
    s, out = seed & M64, []
    for _ in range(count):
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def fmix(x):
    x ^= x >> 33
    x = (x * 0xFF51AFD7ED558CCD) & M64
    x ^= x >> 33
    x = (x * 0xC4CEB9FE1A85EC53) & M64
    return x ^ (x >> 33)


def brute(keys, gamma, seed, max_levels=25, pos=None):
    """Returns (levels, leftovers, labels) with levels = [(m, A list, C list, set F_d)]."""
    import math
    seeds = sm64_stream(seed, max_levels)
    if pos is None:
        def pos(x, d, m):
            return fmix(x ^ seeds[d]) % m
    F = list(keys)
    levels = []
    level_of = {}
    for d in range(max_levels):
        if not F:
            break
        m = int(math.ceil(gamma * len(F)))
        A = [0] * m
        C = [0] * m
        for x in F:                      # Algorithm 2, one key at a time
            h = pos(x, d, m)
            if A[h] == 0 and C[h] == 0:
                A[h] = 1
            elif A[h] == 1 and C[h] == 0:
                A[h] = 0
                C[h] = 1
            else:                        # A == 0 and C == 1: skip
                assert A[h] == 0 and C[h] == 1
        nxt = []
        for x in F:                      # Algorithm 1, filter
            if A[pos(x, d, m)] == 0:
                nxt.append(x)
            else:
                level_of[x] = d
        levels.append((m, A, C, set(F)))
        F = nxt
    # concatenated A, each level padded to a multiple of 64 bits
    concat = []
    starts = []
    for m, A, _, _ in levels:
        starts.append(len(concat))
        concat += A + [0] * ((-m) % 64)
    N = len(keys)
    labels = {}
    for x, d in level_of.items():
        m = levels[d][0]
        g = starts[d] + pos(x, d, m)
        labels[x] = sum(concat[:g]) + 1
    left = sorted(F)
    for i, x in enumerate(left):
        labels[x] = N - len(left) + 1 + i
    return levels, left, labels, concat
