"""Philox4x32-10 counter-based uniforms for the oracle (test infrastructure only).

The paper only needs i.i.d. uniforms U_n that feed both the exact and the approximate
inverse CDF (Section 3, the coupling paragraph); it does not name a generator.  The
generator used here is Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter, a 2x32-bit
key, ten rounds, each round two 32x32->64 multiplications by fixed odd constants whose
high halves are xor-ed with the other two counter words and the round key; the key is
bumped by two Weyl constants between rounds.

Counter layout (the build's reading, fixed for every implementation):
    key     = (seed mod 2^32, seed >> 32)
    levels >= 2:  counter = (n >> 2, path, (stream << 16) | level, pset), word n & 3
    levels 0, 1:  a path has S = 2^level < 4 steps, and one call serves G = 4 / S
                  consecutive paths: counter = (0, path div G, (stream << 16) | level, pset),
                  word (path mod G) S + n
so that no output word is drawn and left unused.  The mapping depends only on (seed,
stream, level, pset, path, n) -- never on how work is scheduled.

Pinned by ``tests/test_oracle_philox.py`` against rocRAND's Philox4x32-10 engine (a
library implementation of the same published generator) compiled for the host.
"""

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
# multipliers and Weyl key increments of Philox4x32 (Salmon et al., SC'11, Table 2)
_MUL0 = np.uint64(0xD2511F53)
_MUL1 = np.uint64(0xCD9E8D57)
_WEYL0 = np.uint64(0x9E3779B9)
_WEYL1 = np.uint64(0xBB67AE85)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on (broadcastable) arrays of 32-bit counter words.

    Every argument is converted to uint64 holding a 32-bit value; the result is a tuple of
    four uint64 arrays, each holding one 32-bit output word.
    """
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & MASK32
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    for _round in range(10):
        p0 = _MUL0 * c0  # < 2^64: exact in uint64
        p1 = _MUL1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _WEYL0) & MASK32
        k1 = (k1 + _WEYL1) & MASK32
    return c0, c1, c2, c3


def words(seed, stream, level, pset, paths, n_steps):
    """All uniform words of ``n_steps`` fine steps for each path in ``paths``.

    Returns a uint32 array of shape (len(paths), n_steps); entry [i, n] is the word that
    fine step n of path ``paths[i]`` consumes.  At levels 0 and 1 n_steps is at most 2^level.
    """
    paths = np.asarray(paths, dtype=np.uint64)
    seed = int(seed)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    c2 = np.uint64(((int(stream) & 0xFFFF) << 16) | (int(level) & 0xFFFF))
    c3 = np.uint64(int(pset) & 0xFFFFFFFF)
    if int(level) < 2:
        S = 1 << int(level)
        G = 4 // S
        if int(n_steps) > S:
            raise ValueError("levels 0 and 1 have at most 2^level steps")
        r = philox4x32_10(np.uint64(0), paths // np.uint64(G), c2, c3, k0, k1)
        r = np.stack(r, axis=1).astype(np.uint32)                  # (paths, 4)
        first = (paths % np.uint64(G)).astype(np.int64) * S        # word of step 0
        out = np.empty((paths.size, int(n_steps)), dtype=np.uint32)
        for n in range(int(n_steps)):
            out[:, n] = r[np.arange(paths.size), first + n]
        return out
    n_calls = (int(n_steps) + 3) // 4
    out = np.empty((paths.size, 4 * n_calls), dtype=np.uint32)
    for q in range(n_calls):
        r = philox4x32_10(np.uint64(q), paths, c2, c3, k0, k1)
        for i in range(4):
            out[:, 4 * q + i] = r[i].astype(np.uint32)
    return out[:, :n_steps]


def word(seed, stream, level, pset, path, n):
    """The single word that fine step ``n`` of ``path`` consumes (scalar helper)."""
    if level < 2:
        S = 1 << level
        G = 4 // S
        r = philox4x32_10(np.uint64(0), np.uint64(path // G),
                          np.uint64(((stream & 0xFFFF) << 16) | (level & 0xFFFF)),
                          np.uint64(pset), np.uint64(seed & 0xFFFFFFFF),
                          np.uint64((seed >> 32) & 0xFFFFFFFF))
        return int(r[(path % G) * S + n])
    r = philox4x32_10(np.uint64(n >> 2), np.uint64(path),
                      np.uint64(((stream & 0xFFFF) << 16) | (level & 0xFFFF)),
                      np.uint64(pset), np.uint64(seed & 0xFFFFFFFF),
                      np.uint64((seed >> 32) & 0xFFFFFFFF))
    return int(r[n & 3])


def uniform(x):
    """U = (x + 1/2) 2^-32 in float64: exact, never 0 or 1, and x -> 2^32-1-x maps U to 1-U."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32
